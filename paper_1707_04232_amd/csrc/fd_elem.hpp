// Compact FP64 elementary functions for the fluctuation/dissipation update
// and the particle passes (pair distances).
//
// Their arguments are always positive, finite and well ranged (uniform draws
// in (0, 1), energies, ratios of friction amplitudes, squared distances
// below h^2; a zero distance is handled by the caller), so the special-case
// handling of a general math library is not needed.  Accuracy: a few ulp,
// far below the 1e-10 agreement required with the FP64 oracle.
//   * log: x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(f),
//     f = (m - 1)/(m + 1), |f| <= 0.1716, atanh series to f^23;
//     e ln 2 added with a two-part ln 2 (32-bit head, so e * head is exact).
//   * log1p: log(1 + x) plus the exact rounding error of 1 + x divided by
//     1 + x (the error is recovered with the Fast2Sum step).
//   * sin(pi t), cos(pi t): t reduced by multiples of 1/2 to |r| <= 1/4,
//     Taylor polynomials of sin(pi r) and cos(pi r) to degree 19 / 18, then a
//     quarter-turn rotation.
//   * reciprocal and reciprocal square root: the hardware estimate (relative
//     error below 6e-8) and one second-order correction; sqrt: the
//     reciprocal square root and one Newton correction of the product.
//   * expm1: x = k ln 2 + r with |r| <= ln 2 / 2 (two-part ln 2), the Taylor
//     polynomial of expm1(r) to degree 13 (its tail is below 2^-53 |r|), and
//     expm1(x) = 2^k expm1(r) + (2^k - 1) in one fused step; for |x| <= ln 2 / 2
//     k = 0 and the polynomial alone is the result.  When no active lane of
//     a wave has |x| > 2^-5 the wave takes the Taylor polynomial of expm1(x)
//     to degree 8 instead.
#pragma once

namespace sdpd {

// reciprocal to about one ulp: the hardware estimate r (relative error
// below 5e-8 on gfx950) and one second-order step, r (1 + e + e^2) with
// e = 1 - x r, whose own error is e^3 (three dependent operations where two
// Newton steps take four)
__device__ __forceinline__ double fast_rcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// reciprocal square root to about one ulp: the hardware estimate y and one
// second-order step, y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2 (error of order
// e^3)
__device__ __forceinline__ double fast_rsq(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// sqrt(x) as x / sqrt(x) from the reciprocal square root alone (within
// about two ulp): the pair distances of the particle passes, whose kernel
// values tolerate it
__device__ __forceinline__ double fd_sqrt_pair(double x) { return x * fast_rsq(x); }

__device__ __forceinline__ double fd_sqrt(double x)
{
    const double y = fast_rsq(x);
    const double s = x * y;
    return fma(0.5 * y, fma(-s, s, x), s);
}

// expm1(x) for finite x with |x| < 700
__device__ __forceinline__ double fd_expm1(double x)
{
    const double k = rint(x * 1.4426950408889634);
    const double r = fma(-k, 1.9082149292705877e-10, fma(-k, 0.6931471803691238, x));
    double p = 1.6059043836821613e-10;   // 1/13!
    p = fma(p, r, 2.08767569878681e-09);   // 1/12!
    p = fma(p, r, 2.505210838544172e-08);  // 1/11!
    p = fma(p, r, 2.755731922398589e-07);  // 1/10!
    p = fma(p, r, 2.7557319223985893e-06); // 1/9!
    p = fma(p, r, 2.48015873015873e-05);   // 1/8!
    p = fma(p, r, 0.0001984126984126984);  // 1/7!
    p = fma(p, r, 0.001388888888888889);   // 1/6!
    p = fma(p, r, 0.008333333333333333);   // 1/5!
    p = fma(p, r, 0.041666666666666664);   // 1/4!
    p = fma(p, r, 0.16666666666666666);    // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p * r, r, r);                  // r + r^2 (1/2 + r/6 + ...)
    const double t = ldexp(1.0, (int)k);
    return fma(t, p, t - 1.0);
}

// expm1(x) for |x| <= 2^-5: its Taylor polynomial to x^8 (the first term
// left out, x^9/9!, is below 2^-58 |x| there)
__device__ __forceinline__ double fd_expm1_small(double x)
{
    double p = 2.48015873015873e-05;      // 1/8!
    p = fma(p, x, 0.0001984126984126984);  // 1/7!
    p = fma(p, x, 0.001388888888888889);   // 1/6!
    p = fma(p, x, 0.008333333333333333);   // 1/5!
    p = fma(p, x, 0.041666666666666664);   // 1/4!
    p = fma(p, x, 0.16666666666666666);    // 1/3!
    p = fma(p, x, 0.5);
    return fma(p * x, x, x);               // x + x^2 (1/2 + x/6 + ...)
}

// expm1 with the short form when no active lane of the wave has |x| > 2^-5
// (the friction exponents of a step of ordinary size), else fd_expm1
__device__ __forceinline__ double fd_expm1_wave(double x)
{
    if (__ballot(fabs(x) > 0x1p-5) == 0ull) return fd_expm1_small(x);
    return fd_expm1(x);
}

__device__ __forceinline__ double fd_log(double x)
{
    int e;
    double m = frexp(x, &e);   // m in [0.5, 1)
    const bool low = m < 0.7071067811865476;
    m = low ? 2.0 * m : m;
    e = low ? e - 1 : e;
    const double f = (m - 1.0) * fast_rcp(m + 1.0);
    const double s = f * f;
    // 2 atanh(f) = 2 f + f s (2/3 + 2/5 s + 2/7 s^2 + ... + 2/23 s^10)
    double p = 0.08695652173913043;
    p = fma(p, s, 0.09523809523809523);
    p = fma(p, s, 0.10526315789473684);
    p = fma(p, s, 0.11764705882352941);
    p = fma(p, s, 0.13333333333333333);
    p = fma(p, s, 0.15384615384615385);
    p = fma(p, s, 0.18181818181818182);
    p = fma(p, s, 0.2222222222222222);
    p = fma(p, s, 0.2857142857142857);
    p = fma(p, s, 0.4);
    p = fma(p, s, 0.6666666666666666);
    const double lm = fma(f * s, p, 2.0 * f);
    const double de = (double)e;
    return fma(de, 0.6931471803691238, fma(de, 1.9082149292705877e-10, lm));
}

// log(1 + x) for x > -1
__device__ __forceinline__ double fd_log1p(double x)
{
    const double y = 1.0 + x;
    const double c = fabs(x) < 1.0 ? x - (y - 1.0) : 1.0 - (y - x);
    return fd_log(y) + c * fast_rcp(y);
}

__device__ __forceinline__ void fd_sincospi_reduced(double r, double &s, double &c)
{
    const double z = r * r;
    double ps = -2.2948428997269873e-08;
    ps = fma(ps, z, 7.952054001475513e-07);
    ps = fma(ps, z, -2.1915353447830217e-05);
    ps = fma(ps, z, 0.00046630280576761255);
    ps = fma(ps, z, -0.0073704309457143504);
    ps = fma(ps, z, 0.08214588661112823);
    ps = fma(ps, z, -0.5992645293207921);
    ps = fma(ps, z, 2.5501640398773455);
    ps = fma(ps, z, -5.16771278004997);
    ps = fma(ps, z, 3.141592653589793);
    double pc = -1.3878952462213771e-07;
    pc = fma(pc, z, 4.303069587032947e-06);
    pc = fma(pc, z, -0.0001046381049248457);
    pc = fma(pc, z, 0.0019295743094039231);
    pc = fma(pc, z, -0.02580689139001406);
    pc = fma(pc, z, 0.2353306303588932);
    pc = fma(pc, z, -1.3352627688545895);
    pc = fma(pc, z, 4.0587121264167685);
    pc = fma(pc, z, -4.934802200544679);
    pc = fma(pc, z, 1.0);
    s = r * ps;
    c = pc;
}

// sin(pi t), cos(pi t) for 0 <= t <= 2
__device__ __forceinline__ void fd_sincospi(double t, double &s, double &c)
{
    const double k = rint(2.0 * t);   // quarter turns, 0..4
    const double r = t - 0.5 * k;     // exact, |r| <= 1/4
    double sr, cr;
    fd_sincospi_reduced(r, sr, cr);
    // quarter-turn rotation as selects (no branches): odd q swaps sin and
    // cos; sin changes sign for q = 2, 3 and cos for q = 1, 2
    const int q = ((int)k) & 3;
    const bool sw = (q & 1) != 0;
    const double a = sw ? cr : sr, b = sw ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

}  // namespace sdpd
