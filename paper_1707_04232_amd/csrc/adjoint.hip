// Adjoint (reverse-mode gradient) of the conservative SDPD dynamics: the
// Velocity-Verlet steps of eq. (sdpd-verlet) with the SPH density of
// eq. (sdpd-rho-v), the constant-entropy energy update of Sec. 3.1 and the
// pressure force of eq. (cons-forces); the F/D sweep is off.
//
// With the entropies fixed by the initial state, eps_k = c_k rho_k^g with
// g = A kB / Cv and c_k = eps0_k rho0_k^-g, so P_k / rho_k^2 = Pi_k =
// kap c_k rho_k^(g-1), kap = A kB / (m Cv).  One step maps (q, p) to
//   p' = p + h f(q),  q'' = q + dt p'/m,  p'' = p' + h f(q''),  h = dt/2,
// so the cotangents go back as
//   lq += h Jf(q'')^T lp,  lp += (dt/m) lq,  lq += h Jf(q)^T lp,
// and the product Jf(q^n)^T (h lp^n) serves the second half kick of step
// n - 1 and the first of step n: one product per configuration.  With
// v = h lp, for the pairs (i, j) within h (r = q_i - q_j, u = v_i - v_j):
//   pibar_k  = m^2 sum_j F(r_kj) (r_kj . u_kj)              cotangent of Pi_k
//   rhobar_k = pibar_k (g - 1) Pi_k / rho_k                 through Pi(rho)
//   qbar_i   = sum_j m^2 (Pi_i + Pi_j) [F u + (F'/r)(r . u) r]
//              - m (rhobar_i + rhobar_j) F r                through rho(q)
// (grad W = -F r).  The products accumulate G_k = sum pibar_k Pi_k and
// H_k = sum pibar_k Pi_k ln rho_k, which give the initial-state path
// (rho0bar = -g G / rho0 through the density of q0, eps0bar = G / eps0)
// and dJ/dA = sum_k G_k / A + (kB/Cv)(H_k - G_k ln rho0_k).  The reference
// density rho0 cancels (eps depends on eps0 and rho / rho0_k only).
//
// Cotangents of the final energies and densities (J may read eps_K, rho_K,
// e.g. the mean pressure of the closure of Sec. 2.1.2): since
// eps_K = c rho_K^g, epsbar_K adds g epsbar eps_K / rho_K to rhobar_K, which
// together with the caller's rhobar_K enters the density term of the final
// configuration's q product, and epsbar eps_K to the cotangent of ln c
// (Ge), which joins G on the initial-state path; its A part is
// (kB/Cv)(He - Ge ln rho0) with He = Ge ln rho_K (no 1/A term: eps has no
// A prefactor).  The conservative dynamics depends on A and Cv only through
// A/Cv (g = A kB/Cv, kap = A kB/(m Cv)), so at fixed A
// dJ/dCv = -(A/Cv) dJ/dA for a J without an explicit Cv dependence.
//
// Forward: checkpoints of the full state every `every` steps; backward:
// each segment is recomputed from its checkpoint (bit-identical: the same
// kernels on the same data), its configurations kept, and processed in
// reverse.  Cotangents live in id order (ids must be 0..n-1).
#include <math.h>

#include <algorithm>

#include <new>
#include <utility>
#include <vector>

#include "sdpd_internal.hpp"

namespace sdpd {

struct StateBuf {
    double *q = nullptr, *p = nullptr, *eps = nullptr, *rho = nullptr, *f = nullptr;
    uint32_t *id = nullptr;
    sdpd_state view() const { return sdpd_state{q, p, eps, rho, f, id}; }
};

struct AdjointWork {
    int K = 0, every = 0, nck = 0;
    std::vector<StateBuf> ckpt, seg;
    StateBuf w;
    double *lq = nullptr, *lp = nullptr, *G = nullptr, *H = nullptr;   // id order
    double *Ge = nullptr, *He = nullptr;   // final-energy path (id order)
    double *eps0 = nullptr, *rho0 = nullptr;                             // id order
    double *vc = nullptr, *wc = nullptr, *pibar = nullptr, *rhobar = nullptr;   // cell order
    uint32_t *idcount = nullptr;
    std::vector<void *> owned;
};

static int walloc(AdjointWork *a, void **p, size_t bytes)
{
    *p = nullptr;
    if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) return SDPD_ENOMEM;
    a->owned.push_back(*p);
    return SDPD_OK;
}

static int state_alloc(AdjointWork *a, StateBuf &s, size_t n)
{
    int rc = SDPD_OK;
    rc = rc ? rc : walloc(a, (void **)&s.q, sizeof(double) * 3 * n);
    rc = rc ? rc : walloc(a, (void **)&s.p, sizeof(double) * 3 * n);
    rc = rc ? rc : walloc(a, (void **)&s.f, sizeof(double) * 3 * n);
    rc = rc ? rc : walloc(a, (void **)&s.eps, sizeof(double) * n);
    rc = rc ? rc : walloc(a, (void **)&s.rho, sizeof(double) * n);
    rc = rc ? rc : walloc(a, (void **)&s.id, sizeof(uint32_t) * n);
    return rc;
}

void adjoint_free(AdjointWork *a)
{
    if (!a) return;
    for (void *p : a->owned) (void)hipFree(p);
    delete a;
}

static int copy_state(sdpd_ctx *c, const StateBuf &dst, const sdpd_state &src)
{
    const size_t n = (size_t)c->n;
    const size_t d3 = sizeof(double) * 3 * n, d1 = sizeof(double) * n;
    int rc = SDPD_OK;
    auto cp = [&](void *d, const void *s, size_t b) {
        if (!rc) rc = check_hip(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, c->stream));
    };
    cp(dst.q, src.q, d3);
    cp(dst.p, src.p, d3);
    cp(dst.f, src.f, d3);
    cp(dst.eps, src.eps, d1);
    cp(dst.rho, src.rho, d1);
    cp(dst.id, src.id, sizeof(uint32_t) * n);
    return rc;
}

// ---------------------------------------------------------------- kernels

__global__ void k_count_ids(int64_t n, const uint32_t *id, uint32_t *count, uint32_t *err)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = id[k];
    if (i >= (uint64_t)n) {
        atomicOr(err, ERR_IDS);
        return;
    }
    if (atomicAdd(&count[i], 1u) != 0u) atomicOr(err, ERR_IDS);
}

// dst (cell order) = scale * src (id order), ncomp planes
__global__ void k_gather_id(int64_t n, int ncomp, const uint32_t *id, double scale,
                            const double *src, double *dst)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = id[k];
    for (int c = 0; c < ncomp; ++c) dst[c * n + k] = scale * src[c * n + i];
}

// dst (id order) += weight * src (cell order); each id appears once
__global__ void k_scatter_add_id(int64_t n, int ncomp, const uint32_t *id, double weight,
                                 const double *src, double *dst)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = id[k];
    for (int c = 0; c < ncomp; ++c) dst[c * n + i] += weight * src[c * n + k];
}

__global__ void k_axpy(int64_t len, double a, const double *x, double *y)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) y[k] += a * x[k];
}

// state value (cell order) -> id order
__global__ void k_to_id(int64_t n, const uint32_t *id, const double *src, double *dst)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[id[k]] = src[k];
}

__device__ __forceinline__ double kernel_F(const DevParams &P, double r)
{
    const double x = r * P.inv_h, t = 1.0 - x;
    if (P.kernel == SDPD_KERNEL_LUCY) return P.cF * (t * t);
    if (x <= 0.5) return P.cF * (2.0 - 3.0 * x);
    return P.cF * P.h * (t * t) / r;
}

// dF/dr
__device__ __forceinline__ double kernel_dF(const DevParams &P, double r)
{
    const double x = r * P.inv_h;
    if (P.kernel == SDPD_KERNEL_LUCY) return -2.0 * P.cF * (1.0 - x) * P.inv_h;
    if (x <= 0.5) return -3.0 * P.cF * P.inv_h;
    return -P.cF * P.h * (1.0 - x * x) / (r * r);
}

// pibar, rhobar (cell order); G, H accumulate (id order) with the weight
__global__ __launch_bounds__(256) void k_vjp_pi(DevParams P, const double *__restrict__ q,
                                                const double *__restrict__ v,
                                                const double *__restrict__ eps,
                                                const double *__restrict__ rho,
                                                const uint32_t *__restrict__ id,
                                                const uint32_t *__restrict__ cell_sorted,
                                                const uint32_t *__restrict__ cell_start,
                                                const uint64_t *__restrict__ masks,
                                                double weight, double *pibar, double *rhobar,
                                                double *G, double *H)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = cell_sorted[i];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const double xi = q[i], yi = q[n + i], zi = q[2 * n + i];
    const double vx = v[i], vy = v[n + i], vz = v[2 * n + i];
    double acc = 0.0;
    for (int k = 0; k < 27; ++k) {
        uint64_t mask = masks[(int64_t)k * n + i];
        if (!mask) continue;
        const NbCell nb = neighbour_cell(P, cx, cy, cz, k);
        const uint32_t s = cell_start[nb.c];
        while (mask) {
            const uint32_t j = s + (uint32_t)__builtin_ctzll(mask);
            mask &= mask - 1ull;
            const double dx = (xi - q[j]) + nb.sx;
            const double dy = (yi - q[n + j]) + nb.sy;
            const double dz = (zi - q[2 * n + j]) + nb.sz;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double ru = dx * (vx - v[j]) + dy * (vy - v[n + j]) + dz * (vz - v[2 * n + j]);
            acc += kernel_F(P, r) * ru;
        }
    }
    const double pb = P.m * P.m * acc;
    const double Pi = P.cPi * eps[i] / rho[i];
    pibar[i] = pb;
    rhobar[i] = pb * (P.eps_exp - 1.0) * Pi / rho[i];
    const int64_t g = id[i];
    G[g] += weight * pb * Pi;
    H[g] += weight * pb * Pi * log(rho[i]);
}

// qbar (cell order): the force term (with_force) and the density term
__global__ __launch_bounds__(256) void k_vjp_q(DevParams P, const double *__restrict__ q,
                                               const double *__restrict__ v,
                                               const double *__restrict__ eps,
                                               const double *__restrict__ rho,
                                               const double *__restrict__ rhobar,
                                               const uint32_t *__restrict__ cell_sorted,
                                               const uint32_t *__restrict__ cell_start,
                                               const uint64_t *__restrict__ masks,
                                               int with_force, double *w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const uint32_t c = cell_sorted[i];
    const int cx = (int)(c % (uint32_t)P.nc[0]);
    const int cy = (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]);
    const int cz = (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]));
    const double xi = q[i], yi = q[n + i], zi = q[2 * n + i];
    const double vx = with_force ? v[i] : 0.0, vy = with_force ? v[n + i] : 0.0,
                 vz = with_force ? v[2 * n + i] : 0.0;
    const double Pii = P.cPi * eps[i] / rho[i];
    const double rbi = rhobar[i];
    const double m2 = P.m * P.m;
    double wx = 0.0, wy = 0.0, wz = 0.0;
    for (int k = 0; k < 27; ++k) {
        uint64_t mask = masks[(int64_t)k * n + i];
        if (!mask) continue;
        const NbCell nb = neighbour_cell(P, cx, cy, cz, k);
        const uint32_t s = cell_start[nb.c];
        while (mask) {
            const uint32_t j = s + (uint32_t)__builtin_ctzll(mask);
            mask &= mask - 1ull;
            const double dx = (xi - q[j]) + nb.sx;
            const double dy = (yi - q[n + j]) + nb.sy;
            const double dz = (zi - q[2 * n + j]) + nb.sz;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double F = kernel_F(P, r);
            // density term: -m (rhobar_i + rhobar_j) F r
            double sx = -P.m * (rbi + rhobar[j]) * F;
            double tx = sx * dx, ty = sx * dy, tz = sx * dz;
            if (with_force) {
                const double ux = vx - v[j], uy = vy - v[n + j], uz = vz - v[2 * n + j];
                const double Pij = m2 * (Pii + P.cPi * eps[j] / rho[j]);
                const double dFr = kernel_dF(P, r) / r;
                const double ru = dx * ux + dy * uy + dz * uz;
                tx += Pij * (F * ux + dFr * ru * dx);
                ty += Pij * (F * uy + dFr * ru * dy);
                tz += Pij * (F * uz + dFr * ru * dz);
            }
            wx += tx;
            wy += ty;
            wz += tz;
        }
    }
    w[i] = wx;
    w[n + i] = wy;
    w[2 * n + i] = wz;
}

// cotangents of the final energies and densities (id order, either may be
// NULL) at the final configuration (cell order): rhobar += drho + g deps
// eps / rho, Ge = deps eps, He = Ge ln rho
__global__ void k_final_cotangent(int64_t n, double g, const uint32_t *id, const double *deps,
                                  const double *drho, const double *eps, const double *rho,
                                  double *rhobar, double *Ge, double *He)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = id[k];
    const double de = deps ? deps[i] : 0.0;
    const double dr = drho ? drho[i] : 0.0;
    rhobar[k] += dr + g * de * eps[k] / rho[k];
    const double ge = de * eps[k];
    Ge[i] = ge;
    He[i] = ge * log(rho[k]);
}

// (G + Ge) -> eps0bar = (G + Ge) / eps0 and rho0bar = -g (G + Ge) / rho0
// (id order, into the given outputs)
__global__ void k_initial_path(int64_t n, double g, const double *G, const double *Ge,
                               const double *eps0, const double *rho0, double *eps0bar,
                               double *rho0bar)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double gt = G[k] + Ge[k];
    if (eps0bar) eps0bar[k] = gt / eps0[k];
    rho0bar[k] = -g * gt / rho0[k];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// one vector-Jacobian product of the force at configuration X (already in
// W): lq += weight * Jf(q)^T (h lp), G and H accumulate.  At the final
// configuration (weight 1) the cotangents of the final energies and
// densities (deps, drho: id order, may be NULL) join the density term.
static int vjp_config(sdpd_ctx *c, AdjointWork *a, const sdpd_state &Ws, double weight,
                      const double *deps = nullptr, const double *drho = nullptr)
{
    const int64_t n = c->n;
    int rc;
    if ((rc = run_build_cells(c, &Ws, 0))) return rc;
    if ((rc = run_density(c, &Ws, 0))) return rc;
    const double h = 0.5 * c->prm.dt;
    hipLaunchKernelGGL(k_gather_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, 3, Ws.id, h, a->lp,
                       a->vc);
    hipLaunchKernelGGL(k_vjp_pi, dim3(nblk(n)), dim3(256), 0, c->stream, c->dp, Ws.q, a->vc,
                       Ws.eps, Ws.rho, Ws.id, c->cell_sorted, c->cell_start, c->masks, weight,
                       a->pibar, a->rhobar, a->G, a->H);
    if (deps || drho)
        hipLaunchKernelGGL(k_final_cotangent, dim3(nblk(n)), dim3(256), 0, c->stream, n,
                           c->dp.eps_exp, Ws.id, deps, drho, Ws.eps, Ws.rho, a->rhobar, a->Ge,
                           a->He);
    hipLaunchKernelGGL(k_vjp_q, dim3(nblk(n)), dim3(256), 0, c->stream, c->dp, Ws.q, a->vc,
                       Ws.eps, Ws.rho, a->rhobar, c->cell_sorted, c->cell_start, c->masks, 1,
                       a->wc);
    hipLaunchKernelGGL(k_scatter_add_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, 3, Ws.id,
                       weight, a->wc, a->lq);
    return check_hip(hipGetLastError());
}

}  // namespace sdpd

using namespace sdpd;

extern "C" {

int sdpd_adjoint_forward(sdpd_ctx *c, sdpd_state *s, int nsteps, int every)
{
    if (!c || !s || nsteps < 1 || every < 1 || !c->cells_valid) return SDPD_EINVAL;
    if (c->prm.fd != SDPD_FD_NONE || c->prm.prec != SDPD_FP64 || c->n == 0) return SDPD_EINVAL;
    if (!s->q || !s->p || !s->eps || !s->rho || !s->f || !s->id) return SDPD_EINVAL;
    const int64_t n = c->n;
    adjoint_free(c->adj);
    c->adj = nullptr;
    AdjointWork *a = new (std::nothrow) AdjointWork();
    if (!a) return SDPD_ENOMEM;
    a->K = nsteps;
    a->every = every;
    a->nck = (nsteps + every - 1) / every;
    a->ckpt.resize(a->nck);
    a->seg.resize(every + 1);
    int rc = SDPD_OK;
    for (auto &b : a->ckpt)
        if (!rc) rc = state_alloc(a, b, n);
    for (auto &b : a->seg)
        if (!rc) rc = state_alloc(a, b, n);
    if (!rc) rc = state_alloc(a, a->w, n);
    for (double **p : {&a->lq, &a->lp, &a->vc, &a->wc})
        if (!rc) rc = walloc(a, (void **)p, sizeof(double) * 3 * n);
    for (double **p : {&a->G, &a->H, &a->Ge, &a->He, &a->eps0, &a->rho0, &a->pibar,
                       &a->rhobar})
        if (!rc) rc = walloc(a, (void **)p, sizeof(double) * n);
    if (!rc) rc = walloc(a, (void **)&a->idcount, sizeof(uint32_t) * n);
    if (rc) {
        adjoint_free(a);
        return rc;
    }
    c->adj = a;
    // ids must be a permutation of 0..n-1 (cotangents are indexed by id)
    if ((rc = launch_fill_u32(c, a->idcount, 0u, n))) return rc;
    hipLaunchKernelGGL(k_count_ids, dim3(nblk(n)), dim3(256), 0, c->stream, n, s->id, a->idcount,
                       c->err);
    hipLaunchKernelGGL(k_to_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, s->id, s->eps,
                       a->eps0);
    hipLaunchKernelGGL(k_to_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, s->id, s->rho,
                       a->rho0);
    if ((rc = check_hip(hipGetLastError()))) return rc;
    for (int k = 0; k < nsteps; ++k) {
        if (k % every == 0 && (rc = copy_state(c, a->ckpt[k / every], *s))) return rc;
        if ((rc = enqueue_step(c, s, (uint64_t)k, true))) return rc;
    }
    return SDPD_OK;
}

}  // extern "C"

namespace sdpd {

// reverse pass from the cotangents of the final state (q, p: 3 x n; eps,
// rho: n; id order; q, p required, eps, rho may be NULL); dA and dCv (host,
// may be NULL) synchronise
static int adjoint_backward(sdpd_ctx *c, const double *dJ_dq, const double *dJ_dp,
                            const double *dJ_deps, const double *dJ_drho, double *dJ_dq0,
                            double *dJ_dp0, double *dJ_deps0, double *dJ_dA, double *dJ_dCv)
{
    AdjointWork *a = c->adj;
    const int64_t n = c->n;
    const size_t d3 = sizeof(double) * 3 * (size_t)n;
    int rc = SDPD_OK;
    if ((rc = check_hip(hipMemcpyAsync(a->lq, dJ_dq, d3, hipMemcpyDeviceToDevice, c->stream))))
        return rc;
    if ((rc = check_hip(hipMemcpyAsync(a->lp, dJ_dp, d3, hipMemcpyDeviceToDevice, c->stream))))
        return rc;
    for (double *z : {a->G, a->H, a->Ge, a->He})
        if ((rc = launch_fill_u64(c, (unsigned long long *)z, 0ull, n))) return rc;
    const sdpd_state Ws = a->w.view();
    const double dt_m = c->prm.dt / c->prm.m;
    for (int sg = a->nck - 1; sg >= 0; --sg) {
        const int start = sg * a->every, end = std::min(start + a->every, a->K);
        // recompute the segment's configurations start .. end
        if ((rc = copy_state(c, a->seg[0], a->ckpt[sg].view()))) return rc;
        for (int k = 1; k <= end - start; ++k) {
            const sdpd_state cur = a->seg[k - 1].view();
            if ((rc = copy_state(c, a->seg[k], cur))) return rc;
            const sdpd_state nxt = a->seg[k].view();
            if ((rc = enqueue_step(c, &nxt, (uint64_t)(start + k - 1), true))) return rc;
        }
        if (sg == a->nck - 1) {   // the final configuration: second half kick of step K-1
            if ((rc = copy_state(c, a->w, a->seg[end - start].view()))) return rc;
            if ((rc = vjp_config(c, a, Ws, 1.0, dJ_deps, dJ_drho))) return rc;
        }
        for (int N = end - 1; N >= start; --N) {
            hipLaunchKernelGGL(k_axpy, dim3(nblk(3 * n)), dim3(256), 0, c->stream, 3 * n, dt_m,
                               a->lq, a->lp);
            if ((rc = copy_state(c, a->w, a->seg[N - start].view()))) return rc;
            if ((rc = vjp_config(c, a, Ws, N > 0 ? 2.0 : 1.0))) return rc;
        }
    }
    // initial-state path: the entropies come from eps0 and rho(q0)
    const double g = c->dp.eps_exp;
    double *eps0bar = dJ_deps0;
    hipLaunchKernelGGL(k_initial_path, dim3(nblk(n)), dim3(256), 0, c->stream, n, g, a->G, a->Ge,
                       a->eps0, a->rho0, eps0bar, a->rhobar);   // rhobar: id order here
    // W holds configuration 0 with its cells and masks (last vjp_config)
    hipLaunchKernelGGL(k_gather_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, 1, Ws.id, 1.0,
                       a->rhobar, a->pibar);                    // pibar: rho0bar in cell order
    hipLaunchKernelGGL(k_vjp_q, dim3(nblk(n)), dim3(256), 0, c->stream, c->dp, Ws.q, a->vc,
                       Ws.eps, Ws.rho, a->pibar, c->cell_sorted, c->cell_start, c->masks, 0,
                       a->wc);
    hipLaunchKernelGGL(k_scatter_add_id, dim3(nblk(n)), dim3(256), 0, c->stream, n, 3, Ws.id,
                       1.0, a->wc, a->lq);
    if ((rc = check_hip(hipGetLastError()))) return rc;
    if ((rc = check_hip(hipMemcpyAsync(dJ_dq0, a->lq, d3, hipMemcpyDeviceToDevice, c->stream))))
        return rc;
    if ((rc = check_hip(hipMemcpyAsync(dJ_dp0, a->lp, d3, hipMemcpyDeviceToDevice, c->stream))))
        return rc;
    if (dJ_dA || dJ_dCv) {
        std::vector<double> G(n), H(n), Ge(n), He(n), r0(n);
        const std::pair<double *, const double *> cp[] = {
            {G.data(), a->G}, {H.data(), a->H}, {Ge.data(), a->Ge}, {He.data(), a->He},
            {r0.data(), a->rho0}};
        for (const auto &x : cp)
            if (!rc)
                rc = check_hip(hipMemcpyAsync(x.first, x.second, sizeof(double) * n,
                                              hipMemcpyDeviceToHost, c->stream));
        if (!rc) rc = check_hip(hipStreamSynchronize(c->stream));
        if (rc) return rc;
        const double kc = c->prm.kB / c->prm.Cv;
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double lr0 = log(r0[k]);
            acc += G[k] / c->dp.A + kc * (H[k] - G[k] * lr0) + kc * (He[k] - Ge[k] * lr0);
        }
        if (dJ_dA) *dJ_dA = acc;
        if (dJ_dCv) *dJ_dCv = -(c->dp.A / c->prm.Cv) * acc;
    }
    return SDPD_OK;
}

}  // namespace sdpd

extern "C" {

int sdpd_adjoint_backward(sdpd_ctx *c, const double *dJ_dq, const double *dJ_dp, double *dJ_dq0,
                          double *dJ_dp0, double *dJ_deps0, double *dJ_dA)
{
    if (!c || !c->adj || !dJ_dq || !dJ_dp || !dJ_dq0 || !dJ_dp0) return SDPD_EINVAL;
    return adjoint_backward(c, dJ_dq, dJ_dp, nullptr, nullptr, dJ_dq0, dJ_dp0, dJ_deps0, dJ_dA,
                            nullptr);
}

int sdpd_adjoint_vjp(sdpd_ctx *c, const sdpd_cotangent *ct, sdpd_gradient *gr)
{
    if (!c || !c->adj || !ct || !gr || !ct->dq || !ct->dp || !gr->dq0 || !gr->dp0)
        return SDPD_EINVAL;
    gr->dA = gr->dCv = gr->drho0 = 0.0;
    int rc = adjoint_backward(c, ct->dq, ct->dp, ct->deps, ct->drho, gr->dq0, gr->dp0, gr->deps0,
                              &gr->dA, &gr->dCv);
    if (!rc) rc = check_hip(hipStreamSynchronize(c->stream));
    gr->drho0 = 0.0;   // rho0 cancels from the dynamics (eps depends on rho/rho0_k only)
    return rc;
}

}  // extern "C"
