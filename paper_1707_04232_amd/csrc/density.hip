// SPH density, eq. (sdpd-rho-v), the entropy-conserving energy update of
// Sec. 3.1, and the active-pair masks of the fluctuation/dissipation sweep.
#include "sdpd_internal.hpp"
#include "fd_elem.hpp"

#include <float.h>

namespace sdpd {

// W(r) for r < h (Sec. 2.1.1; Lucy's kernel or the cubic spline of
// eq. sdpd-cubic-w)
__device__ __forceinline__ double kernel_w(const DevParams &P, double r)
{
    double x = r * P.inv_h;
    double t = 1.0 - x;
    if (P.kernel == SDPD_KERNEL_LUCY) return P.cW * (1.0 + 3.0 * x) * (t * t * t);
    if (x <= 0.5) return P.cW * (1.0 - 6.0 * x * x + 6.0 * x * x * x);
    return 2.0 * P.cW * (t * t * t);
}

// Candidates of one neighbour cell [s, e): adds m W(r) to acc and returns
// the slot bits of the partners with r < h.
template <bool SHIFT>
__device__ __forceinline__ uint64_t density_cell(const DevParams &P, const double *__restrict__ q4,
                                                 uint32_t s, uint32_t e, double xi, double yi,
                                                 double zi, const NbCell &nb, double &acc)
{
    uint64_t mask = 0, bit = 1ull;   // slot bit of candidate j
    for (uint32_t j = s; j < e; ++j, bit <<= 1) {
        const double2 xy = *reinterpret_cast<const double2 *>(q4 + 4 * (int64_t)j);
        double dx = xi - xy.x, dy = yi - xy.y, dz = zi - q4[4 * (int64_t)j + 2];
        if (SHIFT) {
            dx += nb.sx;
            dy += nb.sy;
            dz += nb.sz;
        }
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < P.h2) {
            // r = 0 (i itself): sqrt(DBL_MIN) gives the same W as r = 0, exactly
            acc += P.m * kernel_w(P, fd_sqrt_pair(fmax(r2, DBL_MIN)));
            mask |= bit;
        }
    }
    return mask;
}

// One thread per particle in cell order, positions read from the packed
// (x, y, z, .) records the cell pass writes.  Candidates are the particles of
// the 27 cells around the particle's cell, visited in the fixed order
// (offset index k = 0..26 with z slowest, then slot), so the sum is
// deterministic.  The periodic image is chosen per neighbour cell: a cell
// reached across the box boundary contributes (x_i - x_j) + shift with
// shift = +-L, which is exactly the minimum-image difference for every pair
// closer than h (L >= 4 h), in the same rounding as the plain form.  For all
// 27 cells the bit of every active partner's slot is stored in
// masks[k * n + i] (the own cell, k = 13, without i itself).
struct DensityArgs {
    DevParams P;
    const double *q4;
    const uint32_t *cell_sorted, *cell_start;
    double *rho, *eps;
    int update_eps;
    uint64_t *masks;
    uint32_t *err;
    double *rho_w;
};

__device__ __forceinline__ void density_body(const DensityArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const double *__restrict__ q4 = a.q4;
    const uint32_t *__restrict__ cell_sorted = a.cell_sorted;
    const uint32_t *__restrict__ cell_start = a.cell_start;
    double *rho = a.rho, *eps = a.eps;
    const int update_eps = a.update_eps;
    uint64_t *__restrict__ masks = a.masks;
    uint32_t *err = a.err;
    double *rho_w = a.rho_w;
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = cell_sorted[i];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const double xi = q4[4 * i], yi = q4[4 * i + 1], zi = q4[4 * i + 2];
    double acc = 0.0;
    const NbSteps steps(P, cx, cy, cz);
    for (int k = 0; k < 27; ++k) {
        const NbCell nb = steps.get(P, k);
        const uint32_t s = cell_start[nb.c], e = cell_start[nb.c + 1];
        uint64_t mask = 0;
        if (e - s > (uint32_t)P.cap) {   // overflowing cell: reported, not visited
            atomicOr(err, ERR_CELLCAP);
            masks[(int64_t)k * n + i] = 0ull;
            continue;
        }
        // the shift adds only where a lane of the wave crosses the boundary
        // (x + 0.0 == x, so the results do not depend on the choice)
        const bool shifted = nb.sx != 0.0 || nb.sy != 0.0 || nb.sz != 0.0;
        mask = __any(shifted) ? density_cell<true>(P, q4, s, e, xi, yi, zi, nb, acc)
                              : density_cell<false>(P, q4, s, e, xi, yi, zi, nb, acc);
        if (k == OWN_NB) mask &= ~(1ull << (i - (int64_t)s));   // i itself is no partner
        masks[(int64_t)k * n + i] = mask;
    }
    const double rho_old = rho[i];
    rho[i] = acc;
    // also into the w slot of the particle's packed record (never read in
    // this pass), where the fluctuation/dissipation sweep reads it
    if (rho_w) rho_w[4 * i + 3] = acc;
    if (update_eps) {
        double e_new = eps[i] * pow(acc / rho_old, P.eps_exp);
        if (!(e_new > 0.0) || !isfinite(e_new)) atomicOr(err, ERR_NONFINITE);
        eps[i] = e_new;
    }
}
__global__ __launch_bounds__(256) void k_density(DensityArgs a)
{
    density_body(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_density_multi, DensityArgs, density_body, 256)

// The same pass with four lanes per particle, for boxes too small to fill
// the GPU with a thread per particle (the pass is then bound by the length
// of one thread's candidate loop): lane q of a particle's group of four
// takes candidates s + q, s + q + 4, ... of each neighbour cell and forms
// m W(r), 0 out of range; the four lanes then add the four values in
// candidate order.  Adding +0 leaves the sum unchanged, so rho is
// bit-identical to k_density's.
constexpr int64_t kQuadMaxParticles = 1 << 17;

template <bool SHIFT>
__device__ __forceinline__ uint64_t density_cell_quad(const DevParams &P,
                                                      const double *__restrict__ q4, uint32_t s,
                                                      uint32_t e, double xi, double yi, double zi,
                                                      const NbCell &nb, double &acc, int q,
                                                      int base)
{
    uint64_t mask = 0;
    const uint32_t cnt = e - s;   // the same for the four lanes
    for (uint32_t c0 = 0; c0 < cnt; c0 += 4) {
        const uint32_t jj = c0 + (uint32_t)q;
        double w = 0.0;
        if (jj < cnt) {
            const int64_t j = (int64_t)s + jj;
            const double2 xy = *reinterpret_cast<const double2 *>(q4 + 4 * j);
            double dx = xi - xy.x, dy = yi - xy.y, dz = zi - q4[4 * j + 2];
            if (SHIFT) {
                dx += nb.sx;
                dy += nb.sy;
                dz += nb.sz;
            }
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < P.h2) {
                w = P.m * kernel_w(P, fd_sqrt_pair(fmax(r2, DBL_MIN)));
                mask |= 1ull << jj;
            }
        }
        const double w0 = __shfl(w, base), w1 = __shfl(w, base + 1);
        const double w2 = __shfl(w, base + 2), w3 = __shfl(w, base + 3);
        acc += w0;
        acc += w1;
        acc += w2;
        acc += w3;
    }
    return mask;
}

__device__ __forceinline__ void density_quad_body(const DensityArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const double *__restrict__ q4 = a.q4;
    const uint32_t *__restrict__ cell_sorted = a.cell_sorted;
    const uint32_t *__restrict__ cell_start = a.cell_start;
    double *rho = a.rho, *eps = a.eps;
    const int update_eps = a.update_eps;
    uint64_t *__restrict__ masks = a.masks;
    uint32_t *err = a.err;
    double *rho_w = a.rho_w;
    const int64_t t = (int64_t)blk * blockDim.x + threadIdx.x;
    const int64_t n = P.n;
    const int64_t i = t >> 2;
    const int q = (int)(threadIdx.x & 3u), base = (int)(threadIdx.x & 63u) & ~3;
    // a group past the last particle runs the loops of the last one (its
    // lanes must take part in the shuffles of their own group only) and
    // stores nothing
    const bool live = i < n;
    const int64_t ii = live ? i : n - 1;
    const uint32_t c = cell_sorted[ii];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const double xi = q4[4 * ii], yi = q4[4 * ii + 1], zi = q4[4 * ii + 2];
    double acc = 0.0;
    const NbSteps steps(P, cx, cy, cz);
    for (int k = 0; k < 27; ++k) {
        const NbCell nb = steps.get(P, k);
        const uint32_t s = cell_start[nb.c], e = cell_start[nb.c + 1];
        if (e - s > (uint32_t)P.cap) {   // overflowing cell: reported, not visited
            if (live && q == 0) {
                atomicOr(err, ERR_CELLCAP);
                masks[(int64_t)k * n + i] = 0ull;
            }
            continue;
        }
        const bool shifted = nb.sx != 0.0 || nb.sy != 0.0 || nb.sz != 0.0;
        uint64_t mask = __any(shifted)
                            ? density_cell_quad<true>(P, q4, s, e, xi, yi, zi, nb, acc, q, base)
                            : density_cell_quad<false>(P, q4, s, e, xi, yi, zi, nb, acc, q, base);
        uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
        lo |= (uint32_t)__shfl_xor((int)lo, 1);
        hi |= (uint32_t)__shfl_xor((int)hi, 1);
        lo |= (uint32_t)__shfl_xor((int)lo, 2);
        hi |= (uint32_t)__shfl_xor((int)hi, 2);
        mask = ((uint64_t)hi << 32) | lo;
        if (k == OWN_NB) mask &= ~(1ull << (ii - (int64_t)s));   // i itself is no partner
        if (live && q == 0) masks[(int64_t)k * n + i] = mask;
    }
    if (!live || q != 0) return;
    const double rho_old = rho[i];
    rho[i] = acc;
    if (rho_w) rho_w[4 * i + 3] = acc;
    if (update_eps) {
        double e_new = eps[i] * pow(acc / rho_old, P.eps_exp);
        if (!(e_new > 0.0) || !isfinite(e_new)) atomicOr(err, ERR_NONFINITE);
        eps[i] = e_new;
    }
}
__global__ __launch_bounds__(256) void k_density_quad(DensityArgs a)
{
    density_quad_body(a, blockIdx.x);
}
SDPD_MULTI_KERNEL(k_density_quad_multi, DensityArgs, density_quad_body, 256)

int run_density(sdpd_ctx *c, const sdpd_state *s, int update_eps, bool pack_rho)
{
    if (c->n == 0) {
        c->masks_valid = 1;
        return SDPD_OK;
    }
    if (c->dp.mixed) {
        const int rc = run_density_f32(c, s, update_eps);
        if (!rc) c->masks_valid = 1;
        return rc;
    }
    timer_begin(c, TK_DENSITY);
    const DensityArgs args{c->dp, c->q4, c->cell_sorted, c->cell_start, s->rho, s->eps,
                           update_eps, c->masks, c->err, pack_rho ? c->q4 : nullptr};
    // four lanes per particle only where one lane per particle cannot fill
    // the GPU: a small box on its own (not a box whose launches are recorded
    // for a batch, where all boxes share each launch)
    const int rc = c->n <= kQuadMaxParticles && !c->rec
                       ? launch_or_record(c, k_density_quad, k_density_quad_multi,
                                          (unsigned)((4 * c->n + 255) / 256), 256, 0, args)
                       : launch_or_record(c, k_density, k_density_multi,
                                          (unsigned)((c->n + 255) / 256), 256, 0, args);
    timer_end(c, TK_DENSITY);
    if (!rc) c->masks_valid = 1;
    return rc;
}

}  // namespace sdpd
