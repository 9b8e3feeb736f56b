// Conservative pressure forces, eq. (cons-forces), fused with the second
// half kick of eq. (sdpd-verlet); observables (Sec. 2.2.1).
#include "sdpd_internal.hpp"
#include "fd_elem.hpp"

#include <float.h>

#include <algorithm>

namespace sdpd {

// F(r) with grad W(r) = -F(|r|) r, for 0 < r < h (Sec. 2.1.1; the cubic
// spline's second branch is 48/(pi h^4 r)(1 - r/h)^2)
__device__ __forceinline__ double kernel_f(const DevParams &P, double r)
{
    double x = r * P.inv_h;
    double t = 1.0 - x;
    if (P.kernel == SDPD_KERNEL_LUCY) return P.cF * (t * t);
    if (x <= 0.5) return P.cF * (2.0 - 3.0 * x);
    return P.cF * P.h * (t * t) / r;
}

// P_i / rho_i^2 from the ideal-gas closure: A kB rho eps / (m Cv) / rho^2
// Pi_i = P_i / rho_i^2, stored with the position as (x, y, z, Pi) so that
// the force pass reads one 32-byte record per partner
struct PressureArgs {
    DevParams P;
    const double *q, *eps, *rho;
    double *q4;
};
__device__ __forceinline__ void pressure_term_body(const PressureArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const double *q = a.q, *eps = a.eps, *rho = a.rho;
    double *q4 = a.q4;
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const double v = P.cPi * eps[i] / rho[i];
    double4 r;
    r.x = q[i];
    r.y = q[P.n + i];
    r.z = q[2 * P.n + i];
    r.w = v;
    reinterpret_cast<double4 *>(q4)[i] = r;
}
__global__ void k_pressure_term(PressureArgs a) { pressure_term_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_pressure_term_multi, PressureArgs, pressure_term_body, 256)

// f_i = sum_{j != i, r < h} m^2 (Pi_i + Pi_j) F_ij r_ij over the partners
// recorded in the 27 active-pair masks of the density pass (same positions),
// in the fixed order (offset index, then slot); optionally p_i += dt/2 f_i.
// Only the set bits of each mask are visited.
struct ForcesArgs {
    DevParams P;
    const double *q4;
    const uint32_t *cell_sorted, *cell_start;
    const uint64_t *masks;
    double *f, *p;
    int half_kick;
};

// One loop over a lane's partners in that order: the trip count is the
// lane's partner count, and a lane moves on to its next non-empty neighbour
// cell inside the loop body, whose cell start and mask are loaded one cell
// ahead.  A wave then runs as many iterations as its busiest lane has
// partners, instead of the sum over the 27 cells of the busiest lane in
// each.  EDGE: some lane of the wave sits in a first or last cell of an
// axis, where neighbour steps wrap and carry a periodic shift; elsewhere
// cell k is c + o_x + o_y n_x + o_z n_x n_y - (1 + n_x + n_x n_y) for the
// offset digits o of k, with no shift.
template <bool EDGE>
__device__ __forceinline__ void forces_flat_loop(const DevParams &P, const double *__restrict__ q4,
                                                 const uint32_t *__restrict__ cell_start,
                                                 const uint64_t *__restrict__ masks, int64_t i,
                                                 uint32_t c, const NbSteps &nb, uint32_t todo,
                                                 int total, double4 qi, double &fx, double &fy,
                                                 double &fz)
{
    const int64_t n = P.n;
    const uint32_t nx = (uint32_t)P.nc[0], nxy = nx * (uint32_t)P.nc[1];
    const uint32_t c0 = c - 1u - nx - nxy;
    const double xi = qi.x, yi = qi.y, zi = qi.z, pii = qi.w;
    const double m2 = P.m * P.m;
    // cell k: start and mask requested, shift set
    auto cell = [&](int k, uint32_t &start, uint64_t &m, double &hx, double &hy, double &hz) {
        uint32_t cn;
        if (EDGE) {
            const NbCell r = nb.get(P, k);
            cn = (uint32_t)r.c;
            hx = r.sx;
            hy = r.sy;
            hz = r.sz;
        } else {
            const uint32_t q3 = ((uint32_t)k * 11u) >> 5;   // k / 3 for k < 27
            const uint32_t o0 = (uint32_t)k - 3u * q3, o2 = (q3 * 11u) >> 5, o1 = q3 - 3u * o2;
            cn = c0 + o0 + o1 * nx + o2 * nxy;
        }
        start = cell_start[cn];
        m = masks[(int64_t)k * n + i];
    };
    uint64_t mask = 0ull, mn = 0ull;
    uint32_t s = 0u, sn = 0u;
    double sx = 0.0, sy = 0.0, sz = 0.0, shx = 0.0, shy = 0.0, shz = 0.0;
    if (todo) {
        cell(__builtin_ctz(todo), sn, mn, shx, shy, shz);
        todo &= todo - 1u;
    }
    for (int t = 0; t < total; ++t) {
        if (mask == 0ull) {   // the prefetched cell becomes current
            s = sn;
            mask = mn;
            if (EDGE) {
                sx = shx;
                sy = shy;
                sz = shz;
            }
            if (todo) {
                cell(__builtin_ctz(todo), sn, mn, shx, shy, shz);
                todo &= todo - 1u;
            }
        }
        const uint32_t j = s + (uint32_t)__builtin_ctzll(mask);
        mask &= mask - 1ull;
        const double4 qj = reinterpret_cast<const double4 *>(q4)[j];
        // without a shift x_i - x_j is never -0, so adding +0 changes no bit
        const double dx = EDGE ? (xi - qj.x) + sx : xi - qj.x;
        const double dy = EDGE ? (yi - qj.y) + sy : yi - qj.y;
        const double dz = EDGE ? (zi - qj.z) + sz : zi - qj.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        // coincident particles (r = 0): F(sqrt(DBL_MIN)) = F(0) and dx = 0
        const double sc = m2 * (pii + qj.w) * kernel_f(P, fd_sqrt_pair(fmax(r2, DBL_MIN)));
        fx += sc * dx;
        fy += sc * dy;
        fz += sc * dz;
    }
}

template <int G>
__device__ __forceinline__ void forces_body(const ForcesArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = a.cell_sorted[i];
    const uint32_t nx = (uint32_t)P.nc[0], ny = (uint32_t)P.nc[1];
    const NbSteps nb(P, (int)(c % nx), (int)((c / nx) % ny), (int)(c / (nx * ny)));
    const double4 qi = reinterpret_cast<const double4 *>(a.q4)[i];
    const bool edge = __ballot((nb.lo | nb.hi) != 0u) != 0ull;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    // G = 3: one loop per layer of nine neighbour cells (offsets 9l .. 9l + 8,
    // equal z offset), so that the lanes of a wave read the records of nearby
    // cells at about the same time; G = 1: one loop over all 27 (the same
    // sums in the same order either way)
    constexpr int kGroups = G, kPer = 27 / kGroups;
    for (int g = 0; g < kGroups; ++g) {
        // non-empty neighbour cells (bit k) and the number of partners
        uint32_t todo = 0u;
        int total = 0;
        for (int k = g * kPer; k < (g + 1) * kPer; ++k) {
            const uint64_t m = a.masks[(int64_t)k * n + i];
            todo |= (m != 0ull ? 1u : 0u) << k;
            total += __popcll(m);
        }
        if (edge)
            forces_flat_loop<true>(P, a.q4, a.cell_start, a.masks, i, c, nb, todo, total, qi, fx,
                                   fy, fz);
        else
            forces_flat_loop<false>(P, a.q4, a.cell_start, a.masks, i, c, nb, todo, total, qi, fx,
                                    fy, fz);
    }
    double *f = a.f, *p = a.p;
    f[i] = fx;
    f[n + i] = fy;
    f[2 * n + i] = fz;
    if (a.half_kick) {
        const double hd = 0.5 * P.dt;
        p[i] += hd * fx;
        p[n + i] += hd * fy;
        p[2 * n + i] += hd * fz;
    }
}
template <int G>
__global__ __launch_bounds__(256) void k_forces(ForcesArgs a)
{
    forces_body<G>(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_forces_multi, ForcesArgs, forces_body<1>, 256)

// Boxes above 2^17 particles take one partner loop per layer of neighbour
// cells; smaller boxes, whose few workgroups leave the pass latency-bound,
// and the multi-box launches of batches one loop over all 27.
constexpr int64_t kLayerMinParticles = (int64_t)1 << 17;

int run_forces(sdpd_ctx *c, const sdpd_state *s, int half_kick)
{
    if (c->n == 0) return SDPD_OK;
    if (c->dp.mixed) return run_forces_f32(c, s, half_kick);
    const unsigned g = (unsigned)((c->n + 255) / 256);
    timer_begin(c, TK_FORCE);
    int rc = launch_or_record(c, k_pressure_term, k_pressure_term_multi, g, 256, 0,
                              PressureArgs{c->dp, s->q, s->eps, s->rho, c->q4});
    if (!rc)
        rc = launch_or_record(c, c->n > kLayerMinParticles ? k_forces<3> : k_forces<1>,
                              k_forces_multi, g, 256, 0,
                              ForcesArgs{c->dp, c->q4, c->cell_sorted, c->cell_start, c->masks,
                                         s->f, s->p, half_kick});
    timer_end(c, TK_FORCE);
    return rc;
}

// --- observables: E_int, KE, P (3), min eps; deterministic two-level sums
constexpr int OBS_THREADS = 256;
constexpr int OBS_FIELDS = 6;

__global__ __launch_bounds__(OBS_THREADS) void k_observe_partial(DevParams P, const double *p,
                                                                 const double *eps,
                                                                 double *partial)
{
    __shared__ double s[OBS_FIELDS][OBS_THREADS];
    const int64_t n = P.n;
    double v[OBS_FIELDS] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * OBS_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * OBS_THREADS) {
        double px = p[i], py = p[n + i], pz = p[2 * n + i];
        v[0] += eps[i];
        v[1] += (px * px + py * py + pz * pz) / (2.0 * P.m);
        v[2] += px;
        v[3] += py;
        v[4] += pz;
        v[5] = fmin(v[5], eps[i]);
    }
    for (int k = 0; k < OBS_FIELDS; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = OBS_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int k = 0; k < 5; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + off];
            s[5][threadIdx.x] = fmin(s[5][threadIdx.x], s[5][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x < OBS_FIELDS) partial[blockIdx.x * OBS_FIELDS + threadIdx.x] = s[threadIdx.x][0];
}


// one workgroup: partials summed in a fixed tree order (deterministic)
__global__ __launch_bounds__(OBS_THREADS) void k_observe_final(const double *partial,
                                                               int64_t nblocks,
                                                               const unsigned long long *counters,
                                                               double *rec)
{
    __shared__ double s[OBS_FIELDS][OBS_THREADS];
    double v[OBS_FIELDS] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    for (int64_t b = threadIdx.x; b < nblocks; b += OBS_THREADS) {
        for (int k = 0; k < 5; ++k) v[k] += partial[b * OBS_FIELDS + k];
        v[5] = fmin(v[5], partial[b * OBS_FIELDS + 5]);
    }
    for (int k = 0; k < OBS_FIELDS; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = OBS_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int k = 0; k < 5; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + off];
            s[5][threadIdx.x] = fmin(s[5][threadIdx.x], s[5][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    rec[0] = s[0][0] + s[1][0];
    rec[1] = s[0][0];
    rec[2] = s[1][0];
    rec[3] = s[2][0];
    rec[4] = s[3][0];
    rec[5] = s[4][0];
    rec[6] = s[5][0];
    if (!counters) return;   // a record without the F/D counters (7 doubles)
    unsigned long long *ci = reinterpret_cast<unsigned long long *>(rec + 7);
    for (int k = 0; k < CNT_N; ++k) ci[k] = counters[k];
}

int observe_blocks(int64_t n) { return n > 0 ? (int)std::min<int64_t>(OBS_MAX_BLOCKS, (n + 255) / 256) : 0; }

int launch_observe(const DevParams &dp, const double *p, const double *eps, double *partial,
                   const unsigned long long *counters, double *dst_record, hipStream_t stream)
{
    const int nb = observe_blocks(dp.n);
    if (nb > 0)
        hipLaunchKernelGGL(k_observe_partial, dim3((unsigned)nb), dim3(OBS_THREADS), 0, stream,
                           dp, p, eps, partial);
    hipLaunchKernelGGL(k_observe_final, dim3(1), dim3(OBS_THREADS), 0, stream, partial,
                       (int64_t)nb, counters, dst_record);
    return check_hip(hipGetLastError());
}

int run_observe(sdpd_ctx *c, const sdpd_state *s, double *dst_record)
{
    return launch_observe(c->dp, s->p, s->eps, c->obs_partial, c->counters, dst_record,
                          c->stream);
}

}  // namespace sdpd
