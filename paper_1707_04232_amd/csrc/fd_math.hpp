// Device math of one fluctuation/dissipation pair update (Sec. 3.2-3.3 of
// Faure & Stoltz): Philox4x32-10 draws, the Ornstein-Uhlenbeck proposal in
// the relative velocity, the energy bound and the Metropolis log-ratio.
#pragma once

#include "sdpd_internal.hpp"
#include "fd_elem.hpp"

namespace sdpd {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products with multipliers 0xD2511F53 and 0xCD9E8D57, key
// advanced by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                              uint32_t &x3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * x0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double open_unit(uint32_t w)
{
    return ((double)w + 0.5) * 2.3283064365386962890625e-10;  // (w + 1/2) 2^-32
}

// Gaussian vector (Box-Muller on the first block) and uniform of one pair
__device__ __forceinline__ void pair_draws(const DevParams &P, uint32_t step, uint32_t id_i,
                                           uint32_t id_j, double G[3], double &U)
{
#pragma clang fp contract(fast)
    uint32_t a0 = step, a1 = id_i, a2 = id_j, a3 = P.replica * 2u;
    uint32_t b0 = step, b1 = id_i, b2 = id_j, b3 = P.replica * 2u + 1u;
    philox4x32_10(a0, a1, a2, a3, P.seed_lo, P.seed_hi);
    philox4x32_10(b0, b1, b2, b3, P.seed_lo, P.seed_hi);
    const double R1 = fd_sqrt(-2.0 * fd_log(open_unit(a0)));
    const double R2 = fd_sqrt(-2.0 * fd_log(open_unit(a2)));
    double s1, c1, s3, c3;
    fd_sincospi(2.0 * open_unit(a1), s1, c1);
    fd_sincospi(2.0 * open_unit(a3), s3, c3);
    G[0] = R1 * c1;
    G[1] = R1 * s1;
    G[2] = R2 * c3;
    U = open_unit(b0);
}

// Mixed precision: the Gaussian vector from the same Philox words through
// Box-Muller in FP32.  The radius sqrt(-2 ln u) takes ln u as log1p(-(1 - u))
// for u > 1/2, with 1 - u formed from the complement word, so that u near 1
// keeps its relative precision (log1p(x) = ln(1 + x) x / ((1 + x) - 1)
// compensates the rounding of 1 + x); the angles 2 pi t go to the hardware
// sine and cosine, whose argument is in turns.  U stays the FP64 uniform.
__device__ __forceinline__ float radius_f32(uint32_t w)
{
    const bool hi = w >= 0x80000000u;
    const float v = ((float)(hi ? ~w : w) + 0.5f) * 2.3283064365386963e-10f;   // u or 1 - u
    const float y = 1.0f - v;
    const float l1 = y == 1.0f ? -v : __logf(y) * (-v / (y - 1.0f));
    const float l = hi ? l1 : __logf(v);
    return sqrtf(-2.0f * l);
}
__device__ __forceinline__ float turns_f32(uint32_t w)
{
    return ((float)w + 0.5f) * 2.3283064365386963e-10f;
}
__device__ __forceinline__ void gauss3_f32(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                                           double G[3])
{
    const float R1 = radius_f32(a0), R2 = radius_f32(a2);
    const float t1 = turns_f32(a1), t3 = turns_f32(a3);
    G[0] = (double)(R1 * __builtin_amdgcn_cosf(t1));
    G[1] = (double)(R1 * __builtin_amdgcn_sinf(t1));
    G[2] = (double)(R2 * __builtin_amdgcn_cosf(t3));
}
__device__ __forceinline__ void pair_draws_f32(const DevParams &P, uint32_t step, uint32_t id_i,
                                               uint32_t id_j, double out[4])
{
    uint32_t a0 = step, a1 = id_i, a2 = id_j, a3 = P.replica * 2u;
    uint32_t b0 = step, b1 = id_i, b2 = id_j, b3 = P.replica * 2u + 1u;
    philox4x32_10(a0, a1, a2, a3, P.seed_lo, P.seed_hi);
    philox4x32_10(b0, b1, b2, b3, P.seed_lo, P.seed_hi);
    gauss3_f32(a0, a1, a2, a3, out);
    out[3] = open_unit(b0);
}

// ---------------------------------------------------------------- coefficients
// alpha^theta and the squared relative-velocity noise amplitude
// b^theta^2 = ((2/m) zeta^theta)^2 at energies (ei, ej).  With
// gamma = kappa (1 - d) and sigma^2 = 4 kappa kB T_i T_j/(T_i + T_j) of
// eq. (sdpd-gamma-sigma), zeta^2 = sigma^2 m (1 - alpha^2)/(4 gamma) reduces
// to m kB T_red (1 - alpha^2)/(1 - d) with T_red = T_i T_j/(T_i + T_j), so
// b^2 = (4 kB/m) T_red (1 - alpha^2)/(1 - d).  With e = expm1(-2 gamma dt/m):
// alpha = 1 + e and 1 - alpha^2 = -e (2 + e), both without cancellation.
struct Coef {
    double al_par, al_perp, b2_par, b2_perp;
    double b_par, b_perp;   // square roots of b2 (set by fd_coef_f32 only)
};

// When zeta = 0 the parallel friction is exactly twice the perpendicular one,
// and expm1(2y) = e (2 + e) with e = expm1(y) saves one exponential.
// FAST = the common case fixed at compile time: EMS, Lucy kernel, zeta = 0
template <bool FAST, class R>
__device__ __forceinline__ Coef fd_coef(const DevParams &P, const R &pr, double kpar, double kperp,
                                        double ei, double ej, double dt)
{
#pragma clang fp contract(fast)
    const double Ti = ei * pr.inv_Cv, Tj = ej * pr.inv_Cv;
    const double inv_Ts = fast_rcp(Ti + Tj);
    const double Tred = Ti * Tj * inv_Ts;
    const double d = pr.kB * Tred * inv_Ts * pr.two_over_Cv;
    const double omd = 1.0 - d;
    const double c = -2.0 * dt * pr.inv_m * omd;
    const double e_perp = fd_expm1_wave(c * kperp);
    const double e_par =
        (FAST || P.par_twice_perp) ? e_perp * (2.0 + e_perp) : fd_expm1_wave(c * kpar);
    const double s = pr.b2_c * Tred * fast_rcp(omd);
    Coef r;
    r.al_par = 1.0 + e_par;
    r.al_perp = 1.0 + e_perp;
    r.b2_par = -s * e_par * (2.0 + e_par);
    r.b2_perp = -s * e_perp * (2.0 + e_perp);
    return r;
}

// ---------------------------------------------------------------- FP32 proposal
// Mixed precision: the geometry and the proposal coefficients e = alpha - 1
// and b of eq. (proposal) in FP32 (hardware reciprocal, square root and
// exponential), for the forward and the reverse move alike.  The proposal
// v' = alpha v + b G, the energies, Delta and the Metropolis log-ratio of
// eq. (metropolis-ratio) stay FP64 and use exactly these coefficients: alpha
// = 1 + e and b are FP32 values promoted, b^2 is formed in FP64 from b (an
// exact square), so the ratio is the exact one of the FP32-defined proposal.

// expm1(x): Taylor polynomial to x^8 for |x| < 1/2 (its tail is below
// 2^-26 |x| there), exp(x) - 1 otherwise (no cancellation for |x| >= 1/2)
__device__ __forceinline__ float expm1_f32(float x)
{
    float p = 2.4801587e-05f;        // 1/8!
    p = fmaf(p, x, 1.9841270e-04f);  // 1/7!
    p = fmaf(p, x, 1.3888889e-03f);  // 1/6!
    p = fmaf(p, x, 8.3333333e-03f);  // 1/5!
    p = fmaf(p, x, 4.1666668e-02f);  // 1/4!
    p = fmaf(p, x, 1.6666667e-01f);  // 1/3!
    p = fmaf(p, x, 0.5f);
    const float small = fmaf(p * x, x, x);
    const float big = __expf(x) - 1.0f;
    return fabsf(x) < 0.5f ? small : big;
}

// the coefficients at energies (ei, ej), EMS with Lucy's kernel and zeta = 0
// (kpar = 2 kperp, so e_par = e_perp (2 + e_perp)); kperp in FP32
__device__ __forceinline__ Coef fd_coef_f32(const DevParams &P, float kperp, double ei, double ej,
                                            float dt)
{
    const float Ti = (float)ei * P.inv_Cv_f, Tj = (float)ej * P.inv_Cv_f;
    const float inv_Ts = __builtin_amdgcn_rcpf(Ti + Tj);
    const float Tred = Ti * Tj * inv_Ts;
    const float d = P.d_c_f * Tred * inv_Ts;
    const float omd = 1.0f - d;
    const float c = -2.0f * dt * P.inv_m_f * omd;
    const float e_perp = expm1_f32(c * kperp);
    const float e_par = e_perp * (2.0f + e_perp);
    const float s = P.b2_c_f * Tred * __builtin_amdgcn_rcpf(omd);
    const float bp = __builtin_amdgcn_sqrtf(-s * e_par * (2.0f + e_par));
    const float bq = __builtin_amdgcn_sqrtf(-s * e_perp * (2.0f + e_perp));
    Coef r;
    r.al_par = 1.0 + (double)e_par;
    r.al_perp = 1.0 + (double)e_perp;
    r.b_par = (double)bp;
    r.b_perp = (double)bq;
    r.b2_par = r.b_par * r.b_par;
    r.b2_perp = r.b_perp * r.b_perp;
    return r;
}

struct FdCount {
    uint32_t proposed, rej_energy, rej_ratio, marginal, negeps;
};

// Read-only data of one oriented pair (i = smaller id): positions,
// densities and its random draws (Gaussian vector and uniform), gathered
// from global memory one level step ahead of its use.
struct PairGeo {
    double xi, yi, zi, xj, yj, zj, rho_i, rho_j;
    double G0, G1, G2, U;
};

// The draws of the pair (id_i < id_j) as stored for the sweep: G1, G2, G3, U
__device__ __forceinline__ void pair_draws_stored(const DevParams &P, uint32_t step,
                                                  uint32_t id_i, uint32_t id_j, double out[4])
{
    double G[3], U;
    pair_draws(P, step, id_i, id_j, G, U);
    out[0] = G[0];
    out[1] = G[1];
    out[2] = G[2];
    out[3] = U;
}

// x - x^2/2 + x^3/3.  For |x| <= 1/2 the alternating series of log(1 + x)
// puts log(1 + x) within x^4/2 of it (the tail after the cubic term is at
// most |x|^4 / (4 (1 - |x|))).
__device__ __forceinline__ double log1p_cubic(double x)
{
    return x * (1.0 + x * (-0.5 + x * 0.3333333333333333));
}

// Brackets closer than this are decided with the logarithms evaluated: it
// covers the 1e-9 window in which a decision counts as marginal plus the
// rounding of both evaluations (below 1e-13 for the values that occur).
constexpr double kLazyMargin = 2e-9;

// The parameters the pair update reads in its dependent chain (the box for
// the minimum image, the constants of the coefficients), by the names of
// DevParams: the update takes either DevParams itself or this copy, which
// the level loop holds in vector registers (read once per batch), so that
// no scalar load waits inside the loop.
struct PairRegs {
    double box[3], half_box[3];
    double inv_Cv, kB, two_over_Cv, inv_m, b2_c, kperp_c, cF;
};

// One pair update; li has the smaller id.  Momenta (x, y, z planes at
// stride ps) and energies are LDS-resident.  MIX (with FAST only): the
// geometry and the proposal coefficients in FP32 (fd_coef_f32).
template <bool FAST, bool MIX = false, class R = DevParams>
__device__ __forceinline__ void fd_pair(const DevParams &P, const R &bx, double dt, int li,
                                        int lj, const PairGeo &pg, double *s_p, int ps,
                                        double *s_eps, FdCount &cnt, bool &negeps)
{
#pragma clang fp contract(fast)
    static_assert(!MIX || FAST, "the FP32 proposal covers EMS, Lucy's kernel, zeta = 0");
    // geometry (Sec. 2.1.1): r_ij, e_ij, F_ij
    const double dx = min_image(pg.xi - pg.xj, bx.box[0], bx.half_box[0]);
    const double dy = min_image(pg.yi - pg.yj, bx.box[1], bx.half_box[1]);
    const double dz = min_image(pg.zi - pg.zj, bx.box[2], bx.half_box[2]);
    double ex, ey, ez, kpar = 0.0, kperp = 0.0;
    float kperp_f = 0.0f;
    if (MIX) {
        const float xf = (float)dx, yf = (float)dy, zf = (float)dz;
        const float r2 = xf * xf + yf * yf + zf * zf;
        const float inv_r = __builtin_amdgcn_rsqf(r2);
        const float t = 1.0f - r2 * inv_r * P.inv_h_f;
        ex = (double)(xf * inv_r);
        ey = (double)(yf * inv_r);
        ez = (double)(zf * inv_r);
        // kappa_perp of Sec. 2.2.2 with Lucy's F
        kperp_f = P.kperp_c_f * (P.cF_f * (t * t)) *
                  __builtin_amdgcn_rcpf((float)(pg.rho_i * pg.rho_j));
    } else {
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv_r = fast_rsq(r2);
        const double r = r2 * inv_r;
        ex = dx * inv_r;
        ey = dy * inv_r;
        ez = dz * inv_r;
        const double x = r * P.inv_h, t = 1.0 - x;
        double F;
        if (FAST || P.kernel == SDPD_KERNEL_LUCY) F = bx.cF * (t * t);
        else F = x <= 0.5 ? bx.cF * (2.0 - 3.0 * x) : bx.cF * P.h * (t * t) * inv_r;
        // kappa^theta of Sec. 2.2.2
        const double kfac = F * fast_rcp(pg.rho_i * pg.rho_j);
        kpar = P.kpar_c * kfac;
        kperp = bx.kperp_c * kfac;
    }

    const double ei = s_eps[li], ej = s_eps[lj];
    const double vx = (s_p[li] - s_p[lj]) * P.inv_m;
    const double vy = (s_p[ps + li] - s_p[ps + lj]) * P.inv_m;
    const double vz = (s_p[2 * ps + li] - s_p[2 * ps + lj]) * P.inv_m;

    const double G[3] = {pg.G0, pg.G1, pg.G2};

    // proposal, eq. (proposal): v' = A(v) v + B(v) G, B = (2/m) zeta^theta P^theta
    const Coef f = MIX ? fd_coef_f32(P, kperp_f, ei, ej, (float)dt)
                       : fd_coef<FAST>(P, bx, kpar, kperp, ei, ej, dt);
    const double b_par = MIX ? f.b_par : fd_sqrt(f.b2_par);
    const double b_perp = MIX ? f.b_perp : fd_sqrt(f.b2_perp);
    const double vpar = vx * ex + vy * ey + vz * ez;
    const double Gpar = G[0] * ex + G[1] * ey + G[2] * ez;
    const double vqx = vx - vpar * ex, vqy = vy - vpar * ey, vqz = vz - vpar * ez;
    const double Gqx = G[0] - Gpar * ex, Gqy = G[1] - Gpar * ey, Gqz = G[2] - Gpar * ez;
    const double npar = f.al_par * vpar + b_par * Gpar;
    const double nqx = f.al_perp * vqx + b_perp * Gqx;
    const double nqy = f.al_perp * vqy + b_perp * Gqy;
    const double nqz = f.al_perp * vqz + b_perp * Gqz;
    const double nvx = npar * ex + nqx, nvy = npar * ey + nqy, nvz = npar * ez + nqz;
    // energy change, eq. (proposal-update)
    const double delta = P.m_over_8 * ((nvx * nvx + nvy * nvy + nvz * nvz)
                                       - (vx * vx + vy * vy + vz * vz));
    const double emin = fmin(ei, ej);
    bool accept = true;
    cnt.proposed += 1;
    if (!FAST && P.fd == SDPD_FD_SSA) {
        if (!(ei - delta > 0.0 && ej - delta > 0.0)) {
            cnt.negeps += 1;
            negeps = true;
        }
    } else {
        if (fabs(emin - delta) <= 1e-12 * fmax(fabs(emin), fabs(delta))) cnt.marginal += 1;
        if (!(emin > delta)) {                       // eq. (energy-bound)
            accept = false;
            cnt.rej_energy += 1;
        } else if (FAST || P.fd == SDPD_FD_EMS) {
            // reverse move from v' at the proposed energies, eq. (metropolis-ratio)
            const double ei2 = ei - delta, ej2 = ej - delta;
            const Coef g = MIX ? fd_coef_f32(P, kperp_f, ei2, ej2, (float)dt)
                               : fd_coef<FAST>(P, bx, kpar, kperp, ei2, ej2, dt);
            const double wpar = vpar - g.al_par * npar;
            const double wqx = vqx - g.al_perp * nqx;
            const double wqy = vqy - g.al_perp * nqy;
            const double wqz = vqz - g.al_perp * nqz;
            // one reciprocal serves both inverse variances and the determinant
            // ratio: inv = 1/(b'_par^2 b'_perp^2)
            const double inv = fast_rcp(g.b2_par * g.b2_perp);
            const double quad = wpar * wpar * (g.b2_perp * inv)
                                + (wqx * wqx + wqy * wqy + wqz * wqz) * (g.b2_par * inv);
            const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
            const double A = 0.5 * G2 - 0.5 * quad;
            // log|B(v)| - log|B(v')| = (1/2) log Dr, Dr = b_par^2 b_perp^4 / (b'_par^2 b'_perp^4)
            const double Dr = (f.b2_par * f.b2_perp * f.b2_perp) * (g.b2_par * (inv * inv));
            // ideal gas: sum_k (S(eps'_k) - S(eps_k))/kB - log T(eps'_k) + log T(eps_k)
            //          = (Cv/kB - 1) log(1 + w), 1 + w = (1 - delta/ei)(1 - delta/ej)
            const double inv_eiej = fast_rcp(ei * ej);
            const double ui = -delta * ej * inv_eiej, uj = -delta * ei * inv_eiej;
            const double w = ui + uj + ui * uj;
            const double U = pg.U;
            // a = A + logdet + ent is compared with log U (reject iff U > exp(a)).
            // Both are first bracketed with the cubic bounds of log1p_cubic;
            // the logarithms are evaluated only when the brackets come within
            // kLazyMargin of each other, which keeps every decision and the
            // marginal count equal to those of the evaluated comparison.
            bool evaluate = true;
            const double xd = Dr - 1.0, xu = U - 1.0;
            if (fabs(xd) <= 0.5 && fabs(w) <= 0.5) {
                const double xd2 = xd * xd, w2 = w * w;
                const double am = A + 0.5 * log1p_cubic(xd) + P.ent_c * log1p_cubic(w);
                const double ar = 0.25 * xd2 * xd2 + 0.5 * fabs(P.ent_c) * w2 * w2;
                double lu_lo, lu_hi;
                if (xu >= -0.5) {
                    const double xu2 = xu * xu;
                    const double um = log1p_cubic(xu);
                    lu_lo = um - 0.5 * xu2 * xu2;
                    lu_hi = um + 0.5 * xu2 * xu2;
                } else {   // U < 1/2: log U < log(1/2) < -0.69
                    lu_lo = -INFINITY;
                    lu_hi = -0.69;
                }
                if (lu_hi < am - ar - kLazyMargin) {
                    evaluate = false;                // log U < a: accept
                } else if (lu_lo > am + ar + kLazyMargin) {
                    evaluate = false;                // log U > a: reject
                    accept = false;
                    cnt.rej_ratio += 1;
                }
            }
            if (evaluate) {
                const double logdet = 0.5 * fd_log(Dr);
                const double ent = P.ent_c * fd_log1p(w);
                const double a = A + logdet + ent;
                const double lnU = fd_log(U);
                if (fabs(a - lnU) <= 1e-9) cnt.marginal += 1;
                if (!(lnU <= a)) {
                    accept = false;
                    cnt.rej_ratio += 1;
                }
            }
        }
    }
    if (accept) {
        const double hm = P.m_over_2;
        const double dpx = hm * (nvx - vx), dpy = hm * (nvy - vy), dpz = hm * (nvz - vz);
        s_p[li] += dpx;
        s_p[ps + li] += dpy;
        s_p[2 * ps + li] += dpz;
        s_p[lj] -= dpx;
        s_p[ps + lj] -= dpy;
        s_p[2 * ps + lj] -= dpz;
        s_eps[li] = ei - delta;
        s_eps[lj] = ej - delta;
    }
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint64_t xor_permute_bits(uint64_t m, uint32_t x)
{
    // bit b of m moves to bit b ^ x
    const uint64_t M[6] = {0x5555555555555555ull, 0x3333333333333333ull,
                           0x0F0F0F0F0F0F0F0Full, 0x00FF00FF00FF00FFull,
                           0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sh = 1 << k;
        const uint64_t sw = ((m & M[k]) << sh) | ((m >> sh) & M[k]);
        m = ((x >> k) & 1u) ? sw : m;
    }
    return m;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, off);
        hi |= (uint32_t)__shfl_xor((int)hi, off);
    }
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
    return v;
}

}  // namespace sdpd
