// Mixed-precision particle passes: SPH density (eq. sdpd-rho-v) with the
// active-pair masks, and the conservative pressure forces (eq. cons-forces),
// from FP32 positions relative to each particle's cell.  The separation of
// particle i (cell c) and particle j found in the neighbour cell c + dk
// (before the periodic wrap) is (xr_i - xr_j) - dk * cell_edge: no periodic
// case analysis and no loss of digits to the box size.  Kernel values and the
// per-particle sums are FP32; rho, f, eps and everything downstream (the
// equation of state, the F/D update, the observables) stay FP64.
#include "sdpd_internal.hpp"

namespace sdpd {

__device__ __forceinline__ float kernel_w_f32(const DevParams &P, float r)
{
    const float x = r * P.inv_h_f, t = 1.0f - x;
    if (P.kernel == SDPD_KERNEL_LUCY) return P.cW_f * (1.0f + 3.0f * x) * (t * t * t);
    if (x <= 0.5f) return P.cW_f * (1.0f - 6.0f * x * x + 6.0f * x * x * x);
    return 2.0f * P.cW_f * (t * t * t);
}

__device__ __forceinline__ float kernel_f_f32(const DevParams &P, float r)
{
    const float x = r * P.inv_h_f, t = 1.0f - x;
    if (P.kernel == SDPD_KERNEL_LUCY) return P.cF_f * (t * t);
    if (x <= 0.5f) return P.cF_f * (2.0f - 3.0f * x);
    return P.cF_f * P.h_f * (t * t) / r;
}

struct NbCellF {
    int64_t c;
    float sx, sy, sz;   // -dk * cell edge
};

__device__ __forceinline__ NbCellF neighbour_cell_f32(const DevParams &P, int cx, int cy, int cz,
                                                      int k)
{
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
    NbCellF r;
    r.sx = -(float)dx * P.cell_f[0];
    r.sy = -(float)dy * P.cell_f[1];
    r.sz = -(float)dz * P.cell_f[2];
    int x2 = cx + dx, y2 = cy + dy, z2 = cz + dz;
    x2 += x2 < 0 ? P.nc[0] : (x2 >= P.nc[0] ? -P.nc[0] : 0);
    y2 += y2 < 0 ? P.nc[1] : (y2 >= P.nc[1] ? -P.nc[1] : 0);
    z2 += z2 < 0 ? P.nc[2] : (z2 >= P.nc[2] ? -P.nc[2] : 0);
    r.c = x2 + (int64_t)P.nc[0] * (y2 + (int64_t)P.nc[1] * z2);
    return r;
}

// One thread per particle; candidates of the 27 cells in the fixed order;
// masks[k * n + i] as in the FP64 pass (bit = slot of an active partner).
struct DensityF32Args {
    DevParams P;
    const float *q4f;
    const uint32_t *cell_sorted, *cell_start;
    double *rho, *eps;
    int update_eps;
    uint64_t *masks;
    uint32_t *err;
};
__device__ __forceinline__ void density_f32_body(const DensityF32Args &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const float4 *__restrict__ qf = reinterpret_cast<const float4 *>(a.q4f);
    const uint32_t *__restrict__ cell_sorted = a.cell_sorted;
    const uint32_t *__restrict__ cell_start = a.cell_start;
    double *rho = a.rho, *eps = a.eps;
    const int update_eps = a.update_eps;
    uint64_t *__restrict__ masks = a.masks;
    uint32_t *err = a.err;
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = cell_sorted[i];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const float4 qi = qf[i];
    const float xi = qi.x, yi = qi.y, zi = qi.z;
    float acc = 0.0f;
    for (int k = 0; k < 27; ++k) {
        const NbCellF nb = neighbour_cell_f32(P, cx, cy, cz, k);
        const uint32_t s = cell_start[nb.c], e = cell_start[nb.c + 1];
        uint64_t mask = 0;
        if (e - s > (uint32_t)P.cap) {   // overflowing cell: reported, not visited
            atomicOr(err, ERR_CELLCAP);
            masks[(int64_t)k * n + i] = 0ull;
            continue;
        }
        for (uint32_t j = s; j < e; ++j) {
            const float4 qj = qf[j];
            const float dx = (xi - qj.x) + nb.sx;
            const float dy = (yi - qj.y) + nb.sy;
            const float dz = (zi - qj.z) + nb.sz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < P.h2_f) {
                acc += P.m_f * kernel_w_f32(P, sqrtf(r2));
                if (j != (uint32_t)i) mask |= 1ull << (j - s);
            }
        }
        masks[(int64_t)k * n + i] = mask;
    }
    const double rho_new = (double)acc;
    const double rho_old = rho[i];
    rho[i] = rho_new;
    if (update_eps) {
        double e_new = eps[i] * pow(rho_new / rho_old, P.eps_exp);
        if (!(e_new > 0.0) || !isfinite(e_new)) atomicOr(err, ERR_NONFINITE);
        eps[i] = e_new;
    }
}
__global__ __launch_bounds__(256) void k_density_f32(DensityF32Args a)
{
    density_f32_body(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_density_f32_multi, DensityF32Args, density_f32_body, 256)

// P_i / rho_i^2 into the w slot of the particle's FP32 record
struct PressureF32Args {
    DevParams P;
    const double *eps, *rho;
    float *q4f;
};
__device__ __forceinline__ void pressure_term_f32_body(const PressureF32Args &a, uint32_t blk)
{
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i < a.P.n) a.q4f[4 * i + 3] = (float)(a.P.cPi * a.eps[i] / a.rho[i]);
}
__global__ void k_pressure_term_f32(PressureF32Args a) { pressure_term_f32_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_pressure_term_f32_multi, PressureF32Args, pressure_term_f32_body, 256)

// f_i over the partners recorded by the density pass, FP32 terms and sums
struct ForcesF32Args {
    DevParams P;
    const float *q4f;
    const uint32_t *cell_sorted, *cell_start;
    const uint64_t *masks;
    double *f, *p;
    int half_kick;
};
// One loop over the lane's partners in the fixed order, moving on to the
// next non-empty neighbour cell inside the loop body (that cell's start and
// mask loaded one cell ahead), as in the FP64 force pass.  EDGE: some lane of
// the wave sits in a first or last cell of an axis, where the neighbour index
// wraps; elsewhere cell k is c + o_x + o_y n_x + o_z n_x n_y - (1 + n_x +
// n_x n_y) for the offset digits o of k.  The shift -(o - 1) * cell edge is
// the same in both cases (positions are relative to the cell).
template <bool EDGE>
__device__ __forceinline__ void forces_f32_loop(const DevParams &P, const float4 *__restrict__ qf,
                                                const uint32_t *__restrict__ cell_start,
                                                const uint64_t *__restrict__ masks, int64_t i,
                                                uint32_t c, int cx, int cy, int cz, uint32_t todo,
                                                int total, float4 qi, float &fx, float &fy,
                                                float &fz)
{
    const int64_t n = P.n;
    const uint32_t nx = (uint32_t)P.nc[0], nxy = nx * (uint32_t)P.nc[1];
    const uint32_t c0 = c - 1u - nx - nxy;
    const float xi = qi.x, yi = qi.y, zi = qi.z, pii = qi.w;
    const float m2 = P.m_f * P.m_f;
    auto cell = [&](int k, uint32_t &start, uint64_t &m, float &hx, float &hy, float &hz) {
        uint32_t cn;
        if (EDGE) {
            const NbCellF nb = neighbour_cell_f32(P, cx, cy, cz, k);
            cn = (uint32_t)nb.c;
            hx = nb.sx;
            hy = nb.sy;
            hz = nb.sz;
        } else {
            const uint32_t q3 = ((uint32_t)k * 11u) >> 5;   // k / 3 for k < 27
            const uint32_t o0 = (uint32_t)k - 3u * q3, o2 = (q3 * 11u) >> 5, o1 = q3 - 3u * o2;
            cn = c0 + o0 + o1 * nx + o2 * nxy;
            hx = -(float)((int)o0 - 1) * P.cell_f[0];
            hy = -(float)((int)o1 - 1) * P.cell_f[1];
            hz = -(float)((int)o2 - 1) * P.cell_f[2];
        }
        start = cell_start[cn];
        m = masks[(int64_t)k * n + i];
    };
    uint64_t mask = 0ull, mn = 0ull;
    uint32_t s = 0u, sn = 0u;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f, shx = 0.0f, shy = 0.0f, shz = 0.0f;
    if (todo) {
        cell(__builtin_ctz(todo), sn, mn, shx, shy, shz);
        todo &= todo - 1u;
    }
    for (int t = 0; t < total; ++t) {
        if (mask == 0ull) {   // the prefetched cell becomes current
            s = sn;
            mask = mn;
            sx = shx;
            sy = shy;
            sz = shz;
            if (todo) {
                cell(__builtin_ctz(todo), sn, mn, shx, shy, shz);
                todo &= todo - 1u;
            }
        }
        const uint32_t j = s + (uint32_t)__builtin_ctzll(mask);
        mask &= mask - 1ull;
        const float4 qj = qf[j];
        const float dx = (xi - qj.x) + sx;
        const float dy = (yi - qj.y) + sy;
        const float dz = (zi - qj.z) + sz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float sc = m2 * (pii + qj.w) * kernel_f_f32(P, sqrtf(r2));
        fx += sc * dx;
        fy += sc * dy;
        fz += sc * dz;
    }
}

template <int G>
__device__ __forceinline__ void forces_f32_body(const ForcesF32Args &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const float4 *__restrict__ qf = reinterpret_cast<const float4 *>(a.q4f);
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = a.cell_sorted[i];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const float4 qi = qf[i];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    const bool edge = __ballot(cx == 0 || cy == 0 || cz == 0 || cx == P.nc[0] - 1 ||
                               cy == P.nc[1] - 1 || cz == P.nc[2] - 1) != 0ull;
    // G loops over the neighbour cells, as in the FP64 force pass
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
            forces_f32_loop<true>(P, qf, a.cell_start, a.masks, i, c, cx, cy, cz, todo, total, qi,
                                  fx, fy, fz);
        else
            forces_f32_loop<false>(P, qf, a.cell_start, a.masks, i, c, cx, cy, cz, todo, total, qi,
                                   fx, fy, fz);
    }
    const double gx = fx, gy = fy, gz = fz;
    double *f = a.f, *p = a.p;
    f[i] = gx;
    f[n + i] = gy;
    f[2 * n + i] = gz;
    if (a.half_kick) {
        const double hd = 0.5 * P.dt;
        p[i] += hd * gx;
        p[n + i] += hd * gy;
        p[2 * n + i] += hd * gz;
    }
}
template <int G>
__global__ __launch_bounds__(256) void k_forces_f32(ForcesF32Args a)
{
    forces_f32_body<G>(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_forces_f32_multi, ForcesF32Args, forces_f32_body<1>, 256)

int run_density_f32(sdpd_ctx *c, const sdpd_state *s, int update_eps)
{
    timer_begin(c, TK_DENSITY);
    const int rc = launch_or_record(c, k_density_f32, k_density_f32_multi,
                                    (unsigned)((c->n + 255) / 256), 256, 0,
                                    DensityF32Args{c->dp, c->q4f, c->cell_sorted, c->cell_start,
                                                   s->rho, s->eps, update_eps, c->masks, c->err});
    timer_end(c, TK_DENSITY);
    return rc;
}

// boxes above 2^17 particles: one partner loop per layer of neighbour cells
constexpr int64_t kLayerMinParticlesF32 = (int64_t)1 << 17;

int run_forces_f32(sdpd_ctx *c, const sdpd_state *s, int half_kick)
{
    const unsigned g = (unsigned)((c->n + 255) / 256);
    timer_begin(c, TK_FORCE);
    int rc = launch_or_record(c, k_pressure_term_f32, k_pressure_term_f32_multi, g, 256, 0,
                              PressureF32Args{c->dp, s->eps, s->rho, c->q4f});
    if (!rc)
        rc = launch_or_record(c, c->n > kLayerMinParticlesF32 ? k_forces_f32<3> : k_forces_f32<1>,
                              k_forces_f32_multi, g, 256, 0,
                              ForcesF32Args{c->dp, c->q4f, c->cell_sorted, c->cell_start,
                                            c->masks, s->f, s->p, half_kick});
    timer_end(c, TK_FORCE);
    return rc;
}

}  // namespace sdpd
