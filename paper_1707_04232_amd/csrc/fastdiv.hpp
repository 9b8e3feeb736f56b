// Exact division by a 32-bit divisor that is fixed per context, as a
// multiply-high and a shift.
#pragma once

#include <stdint.h>

namespace sdpd {

// Division by a divisor fixed per context, 1 <= d <= 2^31: with sh = ceil(log2 d)
// and 2^32 + mul = ceil(2^(32 + sh) / d), floor(n / d) equals
// (n + mulhi(mul, n)) >> sh for every 32-bit n (Granlund & Montgomery,
// "Division by invariant integers using multiplication", 1994, Thm. 4.2)
struct FastDiv {
    uint32_t d, mul;
    int sh;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.sh = 0;
    while ((1ull << f.sh) < d) ++f.sh;
    const uint64_t m = ((1ull << (32 + f.sh)) + d - 1) / d;   // < 2^33
    f.mul = (uint32_t)(m - (1ull << 32));
    return f;
}

__device__ __forceinline__ uint32_t fast_div(const FastDiv &f, uint32_t n)
{
    return (uint32_t)(((uint64_t)__umulhi(f.mul, n) + n) >> f.sh);
}

}  // namespace sdpd
