// walk_inst_direct_pw2.hip -- instantiates the walk kernel of every shape for the
// direct scoring variant with 2 visited-table probes in flight.

#include "walk_impl.hpp"

namespace liblabs {

WalkKernel pick_walk_kernel_direct_pw2(int shape)
{
    switch (shape) {
    case 0: return k_walk<0, true, 2>;
    case 1: return k_walk<1, true, 2>;
    case 2: return k_walk<2, true, 2>;
    case 3: return k_walk<3, true, 2>;
    case 4: return k_walk<4, true, 2>;
    case 5: return k_walk<5, true, 2>;
    case 6: return k_walk<6, true, 2>;
    case 7: return k_walk<7, true, 2>;
    default: return k_walk<-1, true, 2>;
    }
}

} // namespace liblabs
