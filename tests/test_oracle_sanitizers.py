"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc): a small C
driver includes the oracle source and runs every entry point the tests use on small inputs (the
definitions, the one-flip scores, the walk with its bounded table, exact set, brute-force scoring
and general sequences, the best-first search with and without the second table, the
first-improvement search with its perturbation draw, the enumerations);
any out-of-bounds access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "labs_oracle.c")

DRIVER = r"""
#include <stdio.h>
#include "%s"

static int check(int ok, const char *what)
{
    if (!ok)
        fprintf(stderr, "FAILED: %%s\n", what);
    return ok ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    const int8_t barker[13] = {1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1};
    bad += check(ref_isl(13, barker) == 6, "Barker 13 ISL");
    bad += check(ref_psl(13, barker) == 1, "Barker 13 PSL");
    bad += check(ref_is_skew(13, barker), "Barker 13 skew");
    char hex[64];
    int8_t back[13];
    bad += check(ref_hex_encode(13, barker, hex, (int32_t)sizeof hex) >= 0, "hex encode");
    bad += check(ref_hex_decode(hex, 13, back) == 0 && memcmp(back, barker, 13) == 0, "hex round trip");

    uint64_t x[ORACLE_MAX_WORDS] = {0};
    int64_t scores[512], brute[512];
    for (int32_t L = 3; L <= 303; L += 50) {
        ref_start_bits(L, 7, 1, 0, x, ORACLE_MAX_WORDS);
        ref_flip_scores(L, x, scores, 0);
        ref_flip_scores(L, x, brute, 1);
        bad += check(memcmp(scores, brute, sizeof(int64_t) * (size_t)((L + 1) / 2)) == 0, "flip scores");
    }

    ref_walk_cfg c;
    ref_walk_result r;
    static int32_t trace[2 * 3000], stra[3000 * 192];
    const uint32_t flags[4] = {0u, ORACLE_IDEAL, ORACLE_BRUTE, ORACLE_GENERAL};
    for (int f = 0; f < 4; f++) {
        memset(&c, 0, sizeof c);
        c.L = flags[f] == ORACLE_GENERAL ? 40 : 31;
        c.table_log2 = 10;
        c.seed = 11;
        c.walk_id = 2;
        c.flags = flags[f];
        c.steps = 300;
        c.restart_period = 97;
        c.target_isl = -1;
        c.watch_isl = 200;
        bad += check(ref_walk(&c, &r, trace, stra) == 0 && r.steps_done == 300, "walk");
    }
    memset(&c, 0, sizeof c);
    c.L = 61;
    c.table_log2 = 6;
    c.seed = 3;
    c.steps = 200;
    c.target_isl = -1;
    c.watch_isl = -1;
    bad += check(ref_pq_walk(&c, 16, 0, &r, trace, stra) == 0, "best-first search");
    bad += check(ref_pq_walk(&c, 16, 5, &r, trace, stra) == 0, "best-first search, second table");
    c.restart_period = 70;
    bad += check(ref_fi_walk(&c, 3, &r, trace, stra) == 0 && r.traps > 0, "first-improvement search");
    c.flags = ORACLE_BRUTE;
    bad += check(ref_fi_walk(&c, 31, &r, trace, stra) == 0, "first-improvement search, all symbols");
    int32_t picks[32];
    ref_perturb_indices(191, 5, 9, 123, 32, picks);

    static int64_t all[1 << 8];
    bad += check(ref_enum_skew(15, all) == 0, "skew enumeration");
    int64_t mn = 0;
    uint64_t cnt = 0, first = 0;
    bad += check(ref_enum_skew_min(21, 0, 1u << 9, &mn, &cnt, &first) == 0 && mn > 0, "skew minimum");
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER % ORACLE_C)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", str(src), "-o", str(exe), "-lm"]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0 and "asan" in out.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed: " + out.stderr[-300:])
    assert out.returncode == 0, out.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("another preloaded library keeps the AddressSanitizer runtime from loading first")
    assert run.returncode == 0, run.stderr[-3000:]
    assert "runtime error" not in run.stderr, run.stderr[-3000:]
