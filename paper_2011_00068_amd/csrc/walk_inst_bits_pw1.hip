// walk_inst_bits_pw1.hip -- instantiates the walk kernel of every shape for the
// bit-sliced scoring variant with 1 visited-table probe in flight.

#include "walk_impl.hpp"

namespace liblabs {

WalkKernel pick_walk_kernel_bits_pw1(int shape)
{
    switch (shape) {
    case 0: return k_walk<0, false, 1>;
    case 1: return k_walk<1, false, 1>;
    case 2: return k_walk<2, false, 1>;
    case 3: return k_walk<3, false, 1>;
    case 4: return k_walk<4, false, 1>;
    case 5: return k_walk<5, false, 1>;
    case 6: return k_walk<6, false, 1>;
    case 7: return k_walk<7, false, 1>;
    default: return k_walk<-1, false, 1>;
    }
}

} // namespace liblabs
