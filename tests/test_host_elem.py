"""Host check of the compact FP64 elementary functions of the F/D update
(fd_elem.hpp): the header is compiled for the host, with the hardware
reciprocal and reciprocal-square-root estimates replaced by correctly
rounded ones (the correction steps that follow them are the device code's)
and a wave ballot by the one lane's predicate, and compared with long-double
libm over the argument ranges the update uses.  The bound, a few ulp, is far
below the 1e-10 agreement with the oracle."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_04232_amd", "csrc")

PROGRAM = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#define __device__
#define __forceinline__ inline
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / sqrt(x))
#define __ballot(p) ((unsigned long long)((p) ? 1 : 0))
#include "fd_elem.hpp"
using namespace sdpd;
static uint64_t s = 0x9E3779B97F4A7C15ull;
static double u01() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (double)(s >> 11) * 0x1p-53; }
static double ulps(double got, long double want) {
    if (want == 0.0L) return got == 0.0 ? 0.0 : 1e300;
    const double w = (double)want;
    return (double)fabsl((long double)got - want) / (nextafter(fabs(w), INFINITY) - fabs(w));
}
int main() {
    double m_expm1 = 0, m_log = 0, m_log1p = 0, m_sin = 0, m_cos = 0, m_sqrt = 0, m_small = 0;
    double m_pair = 0;
    for (int k = 0; k < 2000000; ++k) {
        const double a = u01();
        // expm1 over the friction exponents: -c kappa in (-50, 0], tiny to large
        double x = -pow(10.0, -12.0 + 13.7 * a);
        if (k % 7 == 0) x = -50.0 * a;
        if (k % 11 == 0) x = 0.7 * (a - 0.5);
        double e = ulps(fd_expm1(x), expm1l((long double)x));
        if (e > m_expm1) m_expm1 = e;
        // the short form on |x| <= 2^-5 (as fd_expm1_wave takes it) and the
        // wave form over the whole range
        const double xs = (a - 0.5) * 0x1p-4;
        e = ulps(fd_expm1_small(xs), expm1l((long double)xs));
        if (e > m_small) m_small = e;
        e = ulps(fd_expm1_wave(x), expm1l((long double)x));
        if (e > m_small) m_small = e;
        // log over (0, 4]: uniforms, ratios of noise amplitudes
        const double y = k % 3 ? a + 0x1p-40 : 4.0 * a + 1e-300;
        e = ulps(fd_log(y), logl((long double)y));
        if (e > m_log) m_log = e;
        const double w = k % 2 ? (a - 0.5) * 1e-6 : 3.0 * a - 0.999;
        e = ulps(fd_log1p(w), log1pl((long double)w));
        if (e > m_log1p) m_log1p = e;
        double sn, cs;
        const double t = 2.0 * a;
        fd_sincospi(t, sn, cs);
        const long double pl = 3.14159265358979323846264338327950288L;
        // absolute error in units of 2^-53 (sin/cos of pi t pass through zero)
        const double as = (double)fabsl((long double)sn - sinl(pl * (long double)t)) / 0x1p-53;
        const double ac = (double)fabsl((long double)cs - cosl(pl * (long double)t)) / 0x1p-53;
        if (as > m_sin) m_sin = as;
        if (ac > m_cos) m_cos = ac;
        const double z = pow(10.0, -20.0 + 22.0 * a);
        e = ulps(fd_sqrt(z), sqrtl((long double)z));
        if (e > m_sqrt) m_sqrt = e;
        e = ulps(fd_sqrt_pair(z), sqrtl((long double)z));
        if (e > m_pair) m_pair = e;
    }
    printf("%g %g %g %g %g %g %g %g\n", m_expm1, m_log, m_log1p, m_sin, m_cos, m_sqrt, m_small,
           m_pair);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_elementary_functions_within_a_few_ulp():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "elem.cpp")
        exe = os.path.join(d, "elem")
        with open(src, "w") as f:
            f.write(PROGRAM)
        subprocess.run(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-I", CSRC, src, "-o",
                        exe, "-lm"], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    e_expm1, e_log, e_log1p, e_sin, e_cos, e_sqrt, e_small, e_pair = map(float, out)
    print("max ulp: expm1", e_expm1, "log", e_log, "log1p", e_log1p, "sin/cos (abs, 2^-53)",
          e_sin, e_cos, "sqrt", e_sqrt, "short expm1", e_small, "pair sqrt", e_pair)
    assert e_expm1 <= 4.0
    assert e_log <= 4.0
    assert e_log1p <= 4.0
    assert e_sin <= 8.0 and e_cos <= 8.0
    assert e_sqrt <= 2.0
    assert e_small <= 4.0
    assert e_pair <= 3.0
