// Pairwise fluctuation/dissipation sweep with the Metropolis correction of
// Faure & Stoltz: the proposal of eq. (proposal) (the Ornstein-Uhlenbeck
// step of eq. ssa-ou written in the relative velocity), the energy update of
// eq. (proposal-update), the energy bound of eq. (energy-bound) and the
// log-ratio of eq. (metropolis-ratio) (Sec. 3.3.2); AMS and SSA as modes.
//
// Order of the pair updates.  Every active pair (r < h) has the key
// (phase, round): phase 0 = pairs inside one cell, phase 1 + 8 o + pi =
// pairs between a cell A of coordinate parity pi and A + delta_o (o-th of
// the 13 forward offsets); round = slot_A XOR slot_B.  The sweep is the
// sequential application in ascending key.  Inside one phase the tasks
// (one cell, or one cell pair) share no particle, and inside a task two
// pairs of one round share no particle, so any schedule that keeps the key
// order between pairs sharing a particle gives the same result.
//
// GPU schedule.  One launch per phase.  A workgroup of one wave takes a
// batch of tasks, stages their particles in LDS, and for each task walks
// the rounds that have an active pair: lane x holds slot x of A and of B,
// the partner of slot x in round s is x ^ s (a lane shuffle), and each pair
// gets the level 1 + max(level of the previous pair of either particle).
// Pairs of one level share no particle, so the wave then applies the
// pending pairs of all its tasks level by level, 64 at a time.
#include "sdpd_internal.hpp"

namespace sdpd {

constexpr int FD_MAXP = 256;       // particles staged per batch
constexpr int FD_MAXPAIRS = 1024;  // pending pairs per flush
constexpr int FD_MAXTASKS = 64;    // tasks per batch
constexpr int FD_NLVL = 64;        // levels are 1..64 between flushes

struct FdPhase {
    int phase;          // 0..104
    int mslot;          // mask slot of the B cell (0 = own cell)
    int d[3];           // offset of B relative to A
    int par[3];         // coordinate parity of A
    int hx, hy;         // tasks per axis (x, y) of a parity class
    int64_t ntasks;
    int64_t tasks_per_wg;
};

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
    uint32_t a0 = step, a1 = id_i, a2 = id_j, a3 = P.replica * 2u;
    uint32_t b0 = step, b1 = id_i, b2 = id_j, b3 = P.replica * 2u + 1u;
    philox4x32_10(a0, a1, a2, a3, P.seed_lo, P.seed_hi);
    philox4x32_10(b0, b1, b2, b3, P.seed_lo, P.seed_hi);
    const double R1 = sqrt(-2.0 * log(open_unit(a0)));
    const double R2 = sqrt(-2.0 * log(open_unit(a2)));
    double s1, c1;
    sincospi(2.0 * open_unit(a1), &s1, &c1);
    G[0] = R1 * c1;
    G[1] = R1 * s1;
    G[2] = R2 * cospi(2.0 * open_unit(a3));
    U = open_unit(b0);
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
};

__device__ __forceinline__ Coef fd_coef(const DevParams &P, double kpar, double kperp, double ei,
                                        double ej, double dt)
{
    const double Ti = ei * P.inv_Cv, Tj = ej * P.inv_Cv;
    const double inv_Ts = 1.0 / (Ti + Tj);
    const double Tred = Ti * Tj * inv_Ts;
    const double d = P.kB * Tred * inv_Ts * P.two_over_Cv;
    const double omd = 1.0 - d;
    const double c = -2.0 * dt * P.inv_m * omd;
    const double e_par = expm1(c * kpar), e_perp = expm1(c * kperp);
    const double s = P.b2_c * Tred / omd;
    Coef r;
    r.al_par = 1.0 + e_par;
    r.al_perp = 1.0 + e_perp;
    r.b2_par = -s * e_par * (2.0 + e_par);
    r.b2_perp = -s * e_perp * (2.0 + e_perp);
    return r;
}

struct FdCount {
    uint32_t proposed, rej_energy, rej_ratio, marginal, negeps;
};

// One pair update on LDS-resident state; li has the smaller id.
__device__ __forceinline__ void fd_pair(const DevParams &P, uint32_t step, double dt, int li,
                                        int lj, double (*s_q)[FD_MAXP], double (*s_p)[FD_MAXP],
                                        double *s_eps, const double *s_rho,
                                        const uint32_t *s_id, FdCount &cnt, bool &negeps)
{
    // geometry (Sec. 2.1.1): r_ij, e_ij, F_ij
    const double dx = min_image(s_q[0][li] - s_q[0][lj], P.box[0], P.half_box[0]);
    const double dy = min_image(s_q[1][li] - s_q[1][lj], P.box[1], P.half_box[1]);
    const double dz = min_image(s_q[2][li] - s_q[2][lj], P.box[2], P.half_box[2]);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double inv_r = 1.0 / r;
    const double ex = dx * inv_r, ey = dy * inv_r, ez = dz * inv_r;
    const double x = r * P.inv_h, t = 1.0 - x;
    double F;
    if (P.kernel == SDPD_KERNEL_LUCY) F = P.cF * (t * t);
    else F = x <= 0.5 ? P.cF * (2.0 - 3.0 * x) : P.cF * P.h * (t * t) * inv_r;
    // kappa^theta of Sec. 2.2.2
    const double kfac = F / (s_rho[li] * s_rho[lj]);
    const double kpar = P.kpar_c * kfac, kperp = P.kperp_c * kfac;

    const double ei = s_eps[li], ej = s_eps[lj];
    const double vx = (s_p[0][li] - s_p[0][lj]) * P.inv_m;
    const double vy = (s_p[1][li] - s_p[1][lj]) * P.inv_m;
    const double vz = (s_p[2][li] - s_p[2][lj]) * P.inv_m;

    double G[3], U;
    pair_draws(P, step, s_id[li], s_id[lj], G, U);

    // proposal, eq. (proposal): v' = A(v) v + B(v) G, B = (2/m) zeta^theta P^theta
    const Coef f = fd_coef(P, kpar, kperp, ei, ej, dt);
    const double b_par = sqrt(f.b2_par), b_perp = sqrt(f.b2_perp);
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
    if (P.fd == SDPD_FD_SSA) {
        if (!(ei - delta > 0.0 && ej - delta > 0.0)) {
            cnt.negeps += 1;
            negeps = true;
        }
    } else {
        if (fabs(emin - delta) <= 1e-12 * fmax(fabs(emin), fabs(delta))) cnt.marginal += 1;
        if (!(emin > delta)) {                       // eq. (energy-bound)
            accept = false;
            cnt.rej_energy += 1;
        } else if (P.fd == SDPD_FD_EMS) {
            // reverse move from v' at the proposed energies, eq. (metropolis-ratio)
            const double ei2 = ei - delta, ej2 = ej - delta;
            const Coef g = fd_coef(P, kpar, kperp, ei2, ej2, dt);
            const double wpar = vpar - g.al_par * npar;
            const double wqx = vqx - g.al_perp * nqx;
            const double wqy = vqy - g.al_perp * nqy;
            const double wqz = vqz - g.al_perp * nqz;
            const double quad = wpar * wpar / g.b2_par + (wqx * wqx + wqy * wqy + wqz * wqz) / g.b2_perp;
            const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
            // log|B(v)| - log|B(v')| = (1/2) log(b_par^2 b_perp^4 / (b'_par^2 b'_perp^4))
            const double logdet = 0.5 * log((f.b2_par * f.b2_perp * f.b2_perp)
                                            / (g.b2_par * g.b2_perp * g.b2_perp));
            // ideal gas: sum_k (S(eps'_k) - S(eps_k))/kB - log T(eps'_k) + log T(eps_k)
            //          = (Cv/kB - 1) log((1 - delta/ei)(1 - delta/ej))
            const double ui = -delta / ei, uj = -delta / ej;
            const double ent = P.ent_c * log1p(ui + uj + ui * uj);
            const double a = 0.5 * G2 - 0.5 * quad + logdet + ent;
            const double lnU = log(U);
            if (fabs(a - lnU) <= 1e-9) cnt.marginal += 1;
            if (!(lnU <= a)) {                       // reject iff U > exp(a)
                accept = false;
                cnt.rej_ratio += 1;
            }
        }
    }
    if (accept) {
        const double hm = P.m_over_2;
        const double dpx = hm * (nvx - vx), dpy = hm * (nvy - vy), dpz = hm * (nvz - vz);
        s_p[0][li] += dpx;
        s_p[1][li] += dpy;
        s_p[2][li] += dpz;
        s_p[0][lj] -= dpx;
        s_p[1][lj] -= dpy;
        s_p[2][lj] -= dpz;
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

// ---------------------------------------------------------------- the phase kernel
struct FdShared {
    double q[3][FD_MAXP];
    double p[3][FD_MAXP];
    double eps[FD_MAXP];
    double rho[FD_MAXP];
    uint32_t id[FD_MAXP];
    uint32_t gidx[FD_MAXP];
    uint32_t pair[FD_MAXPAIRS];
    uint32_t sorted[FD_MAXPAIRS];
    uint8_t lvl[FD_MAXPAIRS];
    uint32_t hist[FD_NLVL + 1];
    uint32_t off[FD_NLVL + 2];
    uint32_t cursor[FD_NLVL + 1];
    int tA[FD_MAXTASKS], tnA[FD_MAXTASKS], tbA[FD_MAXTASKS];
    int tB[FD_MAXTASKS], tnB[FD_MAXTASKS], tbB[FD_MAXTASKS];
};

// Apply all pending pairs level by level, then clear the pending list.
__device__ void fd_flush(const DevParams &P, FdShared &S, int &npairs, int &maxlvl,
                         uint32_t step, double dt, FdCount &cnt, bool &negeps)
{
    const int lane = threadIdx.x;
    __syncthreads();
    if (npairs > 0) {
        // exclusive prefix over levels 1..64: lane x holds level x + 1
        const uint32_t h = S.hist[lane + 1];
        uint32_t incl = h;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = (uint32_t)__shfl_up((int)incl, off);
            if (lane >= off) incl += v;
        }
        S.off[lane + 1] = incl - h;
        S.cursor[lane + 1] = incl - h;
        __syncthreads();
        for (int k = lane; k < npairs; k += 64) {
            const uint32_t pos = atomicAdd(&S.cursor[S.lvl[k]], 1u);
            S.sorted[pos] = S.pair[k];
        }
        __syncthreads();
        for (int l = 1; l <= maxlvl; ++l) {
            const int beg = (int)S.off[l], end = beg + (int)S.hist[l];
            for (int base = beg; base < end; base += 64) {
                const int k = base + lane;
                if (k < end) {
                    const uint32_t pr = S.sorted[k];
                    int li = (int)(pr & 0xFFFFu), lj = (int)(pr >> 16);
                    if (S.id[li] > S.id[lj]) {
                        const int tt = li;
                        li = lj;
                        lj = tt;
                    }
                    fd_pair(P, step, dt, li, lj, S.q, S.p, S.eps, S.rho, S.id, cnt, negeps);
                }
            }
            __syncthreads();
        }
    }
    S.hist[lane + 1] = 0u;
    npairs = 0;
    maxlvl = 0;
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_fd_phase(DevParams P, FdPhase ph,
                                                 const double *__restrict__ q, double *p,
                                                 double *eps, const double *__restrict__ rho,
                                                 const uint32_t *__restrict__ id,
                                                 const uint32_t *__restrict__ cell_start,
                                                 const uint64_t *__restrict__ masks,
                                                 uint32_t step, double dt,
                                                 unsigned long long *counters, uint32_t *err)
{
    __shared__ FdShared S;
    const int lane = threadIdx.x;
    const int64_t n = P.n;
    const bool intra = ph.phase == 0;
    int64_t t = (int64_t)blockIdx.x * ph.tasks_per_wg;
    const int64_t t_end = t + ph.tasks_per_wg < ph.ntasks ? t + ph.tasks_per_wg : ph.ntasks;
    FdCount cnt = {0u, 0u, 0u, 0u, 0u};
    bool negeps = false, capbad = false;
    if (lane == 0) S.hist[0] = 0u;
    S.hist[lane + 1] = 0u;
    __syncthreads();

    while (t < t_end) {
        // ---- batch of tasks whose particles fit in LDS (uniform control flow)
        int nt = 0, np = 0;
        while (t < t_end && nt < FD_MAXTASKS) {
            int64_t A, B;
            if (intra) {
                A = B = t;
            } else {
                const int tx = (int)(t % ph.hx), ty = (int)((t / ph.hx) % ph.hy);
                const int tz = (int)(t / ((int64_t)ph.hx * ph.hy));
                const int ax = 2 * tx + ph.par[0], ay = 2 * ty + ph.par[1], az = 2 * tz + ph.par[2];
                int bx = ax + ph.d[0], by = ay + ph.d[1], bz = az + ph.d[2];
                bx += bx >= P.nc[0] ? -P.nc[0] : (bx < 0 ? P.nc[0] : 0);
                by += by >= P.nc[1] ? -P.nc[1] : (by < 0 ? P.nc[1] : 0);
                bz += bz >= P.nc[2] ? -P.nc[2] : (bz < 0 ? P.nc[2] : 0);
                A = ax + (int64_t)P.nc[0] * (ay + (int64_t)P.nc[1] * az);
                B = bx + (int64_t)P.nc[0] * (by + (int64_t)P.nc[1] * bz);
            }
            const int sA = (int)cell_start[A], nA = (int)cell_start[A + 1] - sA;
            const int sB = (int)cell_start[B], nB = (int)cell_start[B + 1] - sB;
            if (nA > P.cap || nB > P.cap) {   // cell overflow: skip, report
                capbad = true;
                ++t;
                continue;
            }
            const int need = intra ? nA : nA + nB;
            if (np + need > FD_MAXP) break;
            if (lane == 0) {
                S.tA[nt] = sA;
                S.tnA[nt] = nA;
                S.tbA[nt] = np;
                S.tB[nt] = sB;
                S.tnB[nt] = nB;
                S.tbB[nt] = intra ? np : np + nA;
            }
            np += need;
            ++nt;
            ++t;
        }
        __syncthreads();
        // ---- stage particles
        for (int k = 0; k < nt; ++k) {
            const int cells = intra ? 1 : 2;
            for (int h = 0; h < cells; ++h) {
                const int g0 = h ? S.tB[k] : S.tA[k];
                const int cnt_h = h ? S.tnB[k] : S.tnA[k];
                const int b0 = h ? S.tbB[k] : S.tbA[k];
                if (lane < cnt_h) {
                    const int g = g0 + lane, l = b0 + lane;
                    S.q[0][l] = q[g];
                    S.q[1][l] = q[n + g];
                    S.q[2][l] = q[2 * n + g];
                    S.p[0][l] = p[g];
                    S.p[1][l] = p[n + g];
                    S.p[2][l] = p[2 * n + g];
                    S.eps[l] = eps[g];
                    S.rho[l] = rho[g];
                    S.id[l] = id[g];
                    S.gidx[l] = (uint32_t)g;
                }
            }
        }
        __syncthreads();
        // ---- levels of every task, flushing when the pending list is full
        int npairs = 0, maxlvl = 0;
        for (int k = 0; k < nt; ++k) {
            const int nA = S.tnA[k], bA = S.tbA[k], bB = S.tbB[k];
            const uint64_t mask = lane < nA ? masks[(int64_t)ph.mslot * n + S.tA[k] + lane] : 0ull;
            const uint64_t rm = xor_permute_bits(mask, (uint32_t)lane);
            uint64_t rounds = wave_or64(rm);
            int LA = 0, LB = 0, rcount = 0;
            while (rounds) {
                const int s = __builtin_ctzll(rounds);
                rounds &= rounds - 1;
                const int partner = lane ^ s;
                const bool actA = (rm >> s) & 1ull;
                int la = __shfl(LA, partner), lb = __shfl(LB, partner);
                const bool actB = __shfl((int)actA, partner) != 0;
                const bool own = intra ? (actA && lane < partner) : actA;
                const uint64_t bal = __ballot(own);
                const int c = __popcll(bal);
                if (npairs + c > FD_MAXPAIRS) {
                    fd_flush(P, S, npairs, maxlvl, step, dt, cnt, negeps);
                    LA = LB = 0;
                    la = lb = 0;
                    rcount = 0;
                }
                ++rcount;
                int lvl = 0;
                if (intra) {
                    if (actA) LA = (LA > la ? LA : la) + 1;
                    lvl = LA;
                } else {
                    if (actA) LA = (LA > lb ? LA : lb) + 1;
                    if (actB) LB = (LB > la ? LB : la) + 1;
                    lvl = LA;
                }
                if (own) {
                    const int pos = npairs + __popcll(bal & ((1ull << lane) - 1ull));
                    S.pair[pos] = (uint32_t)(bA + lane) | ((uint32_t)(bB + partner) << 16);
                    S.lvl[pos] = (uint8_t)lvl;
                    atomicAdd(&S.hist[lvl], 1u);
                }
                npairs += c;
                maxlvl = maxlvl > rcount ? maxlvl : rcount;
            }
        }
        fd_flush(P, S, npairs, maxlvl, step, dt, cnt, negeps);
        // ---- write back momenta and energies
        for (int k = 0; k < nt; ++k) {
            const int cells = intra ? 1 : 2;
            for (int h = 0; h < cells; ++h) {
                const int cnt_h = h ? S.tnB[k] : S.tnA[k];
                const int b0 = h ? S.tbB[k] : S.tbA[k];
                if (lane < cnt_h) {
                    const int l = b0 + lane, g = (int)S.gidx[l];
                    p[g] = S.p[0][l];
                    p[n + g] = S.p[1][l];
                    p[2 * n + g] = S.p[2][l];
                    eps[g] = S.eps[l];
                }
            }
        }
        __syncthreads();
    }
    // ---- counters: one atomic per counter per workgroup
    const uint32_t v0 = wave_sum_u32(cnt.proposed), v1 = wave_sum_u32(cnt.rej_energy);
    const uint32_t v2 = wave_sum_u32(cnt.rej_ratio), v3 = wave_sum_u32(cnt.marginal);
    const uint32_t v4 = wave_sum_u32(cnt.negeps);
    const bool any_neg = __ballot(negeps) != 0ull;
    if (lane == 0) {
        if (v0) atomicAdd(&counters[CNT_PROPOSED], (unsigned long long)v0);
        if (v1) atomicAdd(&counters[CNT_REJ_ENERGY], (unsigned long long)v1);
        if (v2) atomicAdd(&counters[CNT_REJ_RATIO], (unsigned long long)v2);
        if (v3) atomicAdd(&counters[CNT_MARGINAL], (unsigned long long)v3);
        if (v4) atomicAdd(&counters[CNT_NEGEPS], (unsigned long long)v4);
        if (any_neg) atomicOr(err, ERR_NEGEPS);
        if (capbad) atomicOr(err, ERR_CELLCAP);
    }
}

int run_fd_sweep(sdpd_ctx *c, const sdpd_state *s, uint64_t step, double dt_fd)
{
    if (c->prm.fd == SDPD_FD_NONE || c->n == 0) return SDPD_OK;
    const int *nc = c->dp.nc;
    for (int phase = 0; phase <= 104; ++phase) {
        FdPhase ph;
        ph.phase = phase;
        if (phase == 0) {
            ph.mslot = 0;
            ph.d[0] = ph.d[1] = ph.d[2] = 0;
            ph.par[0] = ph.par[1] = ph.par[2] = 0;
            ph.hx = ph.hy = 0;
            ph.ntasks = c->ncell;
            ph.tasks_per_wg = c->fd_tasks_intra;
        } else {
            const int o = (phase - 1) / 8, pi = (phase - 1) % 8, k = 14 + o;
            ph.mslot = o + 1;
            ph.d[0] = k % 3 - 1;
            ph.d[1] = (k / 3) % 3 - 1;
            ph.d[2] = k / 9 - 1;
            ph.par[0] = pi & 1;
            ph.par[1] = (pi >> 1) & 1;
            ph.par[2] = (pi >> 2) & 1;
            ph.hx = nc[0] / 2;
            ph.hy = nc[1] / 2;
            ph.ntasks = c->ncell / 8;
            ph.tasks_per_wg = c->fd_tasks_inter;
        }
        const int64_t grid = (ph.ntasks + ph.tasks_per_wg - 1) / ph.tasks_per_wg;
        timer_begin(c, TK_FD);
        hipLaunchKernelGGL(k_fd_phase, dim3((unsigned)grid), dim3(64), 0, c->stream, c->dp, ph,
                           s->q, s->p, s->eps, s->rho, s->id, c->cell_start, c->masks,
                           (uint32_t)step, dt_fd, c->counters, c->err);
        timer_end(c, TK_FD);
        int rc = check_hip(hipGetLastError());
        if (rc) return rc;
    }
    return SDPD_OK;
}

}  // namespace sdpd
