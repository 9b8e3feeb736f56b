"""Host check of the multiply-shift division used for the task numbering of
the F/D schedule (Granlund & Montgomery 1994, Thm. 4.2): the header is
compiled for the host with a plain 32x32 -> high 32 product and compared with
integer division over edge cases and random numerators for divisors across
the whole supported range 1 <= d <= 2^31."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_04232_amd", "csrc")

PROGRAM = r"""
#include <stdint.h>
#include <stdio.h>
#define __device__
#define __forceinline__ inline
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
#include "fastdiv.hpp"
using namespace sdpd;
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint32_t rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)(s >> 16); }
static int check(uint32_t d) {
    const FastDiv f = make_fastdiv(d);
    uint32_t edge[] = {0u, 1u, d - 1u, d, d + 1u, 2u * d - 1u, 0x7FFFFFFFu, 0x80000000u,
                       0xFFFFFFFEu, 0xFFFFFFFFu, (0xFFFFFFFFu / d) * d, (0xFFFFFFFFu / d) * d - 1u};
    for (uint32_t n : edge)
        if (fast_div(f, n) != n / d) { printf("FAIL d=%u n=%u\n", d, n); return 1; }
    for (int k = 0; k < 2000; ++k) {
        const uint32_t n = rnd() ^ (rnd() << 16);
        if (fast_div(f, n) != n / d) { printf("FAIL d=%u n=%u\n", d, n); return 1; }
    }
    return 0;
}
int main() {
    int bad = 0;
    for (uint32_t d = 1; d <= 4096; ++d) bad |= check(d);
    for (int k = 0; k < 2000 && !bad; ++k) bad |= check(1u + (rnd() ^ (rnd() << 15)) % 0x80000000u);
    for (int sh = 12; sh <= 31 && !bad; ++sh) {
        bad |= check(1u << sh);
        bad |= check((1u << sh) - 1u);
        if (sh < 31) bad |= check((1u << sh) + 1u);
    }
    bad |= check(0x80000000u);
    if (!bad) printf("ok\n");
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_fastdiv_exact():
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "fastdiv_check.cpp")
        exe = os.path.join(tmp, "fastdiv_check")
        with open(src, "w") as f:
            f.write(PROGRAM)
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
