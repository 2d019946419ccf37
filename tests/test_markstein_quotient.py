"""Host check of the arithmetic identity the OC kernel relies on: with
y = 1 / b correctly rounded, q = a y, r = fma(-q, b, a) and q' = fma(r, y, q),
q' equals the correctly rounded quotient a / b (the final step of
Markstein's division).  The OC candidates use it in place of a division per
element, so their values, and hence the bisection decisions, must be the
division's.  Sampled over the ranges of ocP (a) and the multiplier (b), with
C's fma (the same IEEE fused multiply-add the GPU executes)."""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t nx(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u01(void) { return (double)(nx() >> 11) * (1.0 / 9007199254740992.0); }
int main(int argc, char** argv) {
    long n = atol(argv[1]), bad = 0;
    for (long i = 0; i < n; ++i) {
        double a = exp(-30.0 + 37.0 * u01());     /* ocP: 1e-13 .. 1e3 */
        double b = exp(-25.0 + 35.0 * u01());     /* multiplier: 1e-11 .. 2e4 */
        if (i % 3 == 1) a = nextafter(a, 0.0);
        if (i % 5 == 2) b = nextafter(b, 1e300);
        double y = 1.0 / b, q = a * y, r = fma(-q, b, a), q2 = fma(r, y, q);
        if (q2 != a / b) ++bad;
    }
    printf("%ld\n", bad);
    return 0;
}
"""


def test_fma_corrected_reciprocal_quotient_is_correctly_rounded(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "q.c"
    src.write_text("#include <stdlib.h>\n" + SRC)
    exe = tmp_path / "q"
    # -ffp-contract=off: the products and sums are the ones written, fma only where called
    subprocess.run([cc, "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    out = subprocess.run([str(exe), "20000000"], check=True, capture_output=True, text=True).stdout
    assert int(out.strip()) == 0
