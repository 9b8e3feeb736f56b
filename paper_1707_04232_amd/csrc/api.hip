// C ABI of libsdpd: parameter checks, workspace, launch order, errors.
#include <math.h>
#include <algorithm>
#include <cmath>
#include <string.h>

#include <mutex>
#include <new>

#include "sdpd_internal.hpp"

namespace sdpd {

int check_hip(hipError_t e) { return e == hipSuccess ? SDPD_OK : SDPD_EHIP; }

// c->timing: bit k set = the launches of timing class k are bracketed by
// events

void timer_begin(sdpd_ctx *c, int k)
{
    if (!((c->timing >> k) & 1)) return;
    Timer &T = c->timer;
    if (T.used + 2 > T.pool.size()) {
        size_t old = T.pool.size();
        T.pool.resize(old + 4096);
        for (size_t i = old; i < T.pool.size(); ++i) (void)hipEventCreate(&T.pool[i]);
        T.cls.resize(T.pool.size() / 2);
    }
    T.cls[T.used / 2] = k;
    (void)hipEventRecord(T.pool[T.used], c->stream);
}

void timer_end(sdpd_ctx *c, int k)
{
    if (!((c->timing >> k) & 1)) return;
    Timer &T = c->timer;
    (void)hipEventRecord(T.pool[T.used + 1], c->stream);
    T.used += 2;
}

static bool valid_positive(double x) { return isfinite(x) && x > 0.0; }

// number of cells per axis (the requested value or the largest even
// integer <= box/h), or -1 when the grid would not cover the cutoff
static int grid_axis(double box, double h, int req)
{
    int c = req;
    if (c <= 0) {
        c = (int)floor(box / h);
        if (c % 2) c -= 1;
    }
    if (c < 4 || c % 2 || box / c < h) return -1;
    return c;
}

// The closure coefficient A of eq. (pg-eos): A = 0 selects the default
// A = Cv / (3 kB), the paper's ideal-gas entropy with kB restored in its
// density term (a parameter so that the textbook value 2 Cv / 3 can be used)
static double resolved_A(const sdpd_params *P)
{
    return P->A == 0.0 ? P->Cv / (3.0 * P->kB) : P->A;
}

static int check_params(const sdpd_params *P, int nc[3])
{
    if (!P) return SDPD_EINVAL;
    if (P->n < 0 || P->n > 0x7fffffffLL) return SDPD_EINVAL;
    if (!valid_positive(P->m) || !valid_positive(P->h) || !valid_positive(P->kB) ||
        !valid_positive(P->Cv) || !valid_positive(P->rho0) ||
        !valid_positive(P->dt) || !valid_positive(P->eta))
        return SDPD_EINVAL;
    if (!valid_positive(resolved_A(P))) return SDPD_EINVAL;
    if (!(P->Cv > 0.5 * P->kB)) return SDPD_EINVAL;           // d_ij < 1
    if (!(isfinite(P->zeta) && P->zeta >= 0.0 && P->zeta < 5.0 * P->eta / 3.0))
        return SDPD_EINVAL;                                   // kappa_perp > 0
    if (P->kernel != SDPD_KERNEL_LUCY && P->kernel != SDPD_KERNEL_CUBIC) return SDPD_EINVAL;
    if (P->fd < SDPD_FD_EMS || P->fd > SDPD_FD_NONE) return SDPD_EINVAL;
    if (P->prec != SDPD_FP64 && P->prec != SDPD_MIXED) return SDPD_EINVAL;
    if (P->cell_cap < 1 || P->cell_cap > MAX_CAP) return SDPD_EINVAL;
    if (P->fd_every < 1) return SDPD_EINVAL;
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        if (!valid_positive(P->box[k])) return SDPD_EINVAL;
        nc[k] = grid_axis(P->box[k], P->h, P->ncell[k]);
        if (nc[k] < 0) return SDPD_EINVAL;
        ncell *= nc[k];
    }
    if ((int64_t)NMASK * ncell > 0xffffffffLL) return SDPD_EINVAL;   // 32-bit task indices
    return SDPD_OK;
}

static void derive(const sdpd_params *P, const int nc[3], DevParams &d)
{
    const double pi = 3.14159265358979323846;
    memset(&d, 0, sizeof d);
    d.n = P->n;
    d.ncell = 1;
    for (int k = 0; k < 3; ++k) {
        d.box[k] = P->box[k];
        d.half_box[k] = 0.5 * P->box[k];
        d.nc[k] = nc[k];
        d.inv_cell[k] = (double)nc[k] / P->box[k];
        d.ncell *= nc[k];
    }
    d.m = P->m;
    d.inv_m = 1.0 / P->m;
    d.h = P->h;
    d.h2 = P->h * P->h;
    d.inv_h = 1.0 / P->h;
    d.kB = P->kB;
    d.Cv = P->Cv;
    d.inv_Cv = 1.0 / P->Cv;
    d.A = P->A;
    d.dt = P->dt;
    d.kernel = P->kernel;
    d.fd = P->fd;
    d.cap = P->cell_cap;
    d.seed_lo = (uint32_t)P->seed;
    d.seed_hi = (uint32_t)(P->seed >> 32);
    d.replica = P->replica;
    const double h = P->h;
    if (P->kernel == SDPD_KERNEL_LUCY) {
        d.cW = 105.0 / (16.0 * pi * h * h * h);
        d.cF = 315.0 / (4.0 * pi * pow(h, 5));
    } else {
        d.cW = 8.0 / (pi * h * h * h);
        d.cF = 48.0 / (pi * pow(h, 5));
    }
    d.cPi = P->A * P->kB / (P->m * P->Cv);
    d.eps_exp = P->A * P->kB / P->Cv;
    d.kpar_c = (10.0 / 3.0 * P->eta + 4.0 * P->zeta) * P->m * P->m;
    d.kperp_c = (5.0 / 3.0 * P->eta - P->zeta) * P->m * P->m;
    d.two_over_Cv = 2.0 / P->Cv;
    d.b2_c = 4.0 * P->kB / P->m;
    d.ent_c = P->Cv / P->kB - 1.0;
    d.m_over_8 = P->m / 8.0;
    d.m_over_2 = P->m / 2.0;
    d.par_twice_perp = d.kpar_c == 2.0 * d.kperp_c;
    d.mixed = P->prec == SDPD_MIXED;
    for (int k = 0; k < 3; ++k) d.cell_f[k] = (float)(P->box[k] / nc[k]);
    d.h_f = (float)h;
    d.h2_f = (float)(h * h);
    d.inv_h_f = (float)(1.0 / h);
    d.m_f = (float)P->m;
    d.cW_f = (float)d.cW;
    d.cF_f = (float)d.cF;
    d.inv_Cv_f = (float)d.inv_Cv;
    d.d_c_f = (float)(d.kB * d.two_over_Cv);
    d.inv_m_f = (float)d.inv_m;
    d.b2_c_f = (float)d.b2_c;
    d.kperp_c_f = (float)d.kperp_c;
    d.div_per = make_fastdiv((uint32_t)std::max<int64_t>(d.ncell / 8, 1));
    d.div_hx = make_fastdiv((uint32_t)std::max(nc[0] / 2, 1));
    d.div_hy = make_fastdiv((uint32_t)std::max(nc[1] / 2, 1));
}

template <typename T>
static int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * count) == hipSuccess ? SDPD_OK : SDPD_ENOMEM;
}

static void free_ctx(sdpd_ctx *c)
{
    void *bufs[] = {c->cell_of, c->count, c->cursor, c->cell_start, c->block_sums, c->tmp_idx,
                    c->perm, c->cell_sorted, c->tq, c->tp, c->teps, c->trho, c->tf, c->tid,
                    c->masks, c->counters, c->err, c->obs_partial, c->obs_out,
                    c->dparams, c->task_count, c->task_np, c->pair_off, c->part_off,
                    c->part_list, c->pairs, c->draws, c->q4f, c->dstep, c->q4,
                    c->sweep, c->epoch, c->sweep_order};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : c->timer.pool) (void)hipEventDestroy(e);
    adjoint_free(c->adj);
    delete c;
}

static bool state_ok(const sdpd_ctx *c, const sdpd_state *s)
{
    if (!s) return false;
    if (c->n == 0) return true;
    return s->q && s->p && s->eps && s->rho && s->f && s->id;
}

static int take_error(sdpd_ctx *c)
{
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, c->err, sizeof e, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SDPD_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SDPD_EHIP;
    if (e) {
        uint32_t z = 0;
        if (hipMemcpy(c->err, &z, sizeof z, hipMemcpyHostToDevice) != hipSuccess) return SDPD_EHIP;
    }
    if (e & ERR_STALL) return SDPD_EHIP;   // a sweep range gave up waiting (not expected)
    if (e & ERR_IDS) return SDPD_EINVAL;
    if (e & ERR_CELLCAP) return SDPD_ECELLCAP;
    if (e & ERR_NONFINITE) return SDPD_ENONFINITE;
    if (e & ERR_PAIRCAP) return SDPD_ECAPACITY;
    if (e & ERR_NEGEPS) return SDPD_ENEGEPS;
    return SDPD_OK;
}

static void record_to_stats(const double *rec, sdpd_stats *st)
{
    st->E = rec[0];
    st->Eint = rec[1];
    st->KE = rec[2];
    st->P[0] = rec[3];
    st->P[1] = rec[4];
    st->P[2] = rec[5];
    st->min_eps = rec[6];
    uint64_t cnt[CNT_N];
    memcpy(cnt, rec + 7, sizeof cnt);
    st->proposed = cnt[CNT_PROPOSED];
    st->rej_energy = cnt[CNT_REJ_ENERGY];
    st->rej_ratio = cnt[CNT_REJ_RATIO];
    st->marginal = cnt[CNT_MARGINAL];
    st->negeps = cnt[CNT_NEGEPS];
}

// per-step observable records kept on the device by sdpd_step (allocated
// once, at context creation)
static const int64_t STEP_RECORDS = 64;

static int alloc_records(sdpd_ctx *c)
{
    int rc = dalloc(&c->obs_out, (size_t)(STEP_RECORDS * REC));
    if (!rc) c->obs_cap = STEP_RECORDS;
    return rc;
}

}  // namespace sdpd

using namespace sdpd;

extern "C" {

int sdpd_abi_version(void) { return SDPD_ABI_VERSION; }

const char *sdpd_strerror(int s)
{
    switch (s) {
    case SDPD_OK: return "success";
    case SDPD_EINVAL: return "invalid argument or parameter";
    case SDPD_EHIP: return "HIP runtime error";
    case SDPD_ENOMEM: return "out of device memory";
    case SDPD_ECELLCAP: return "a cell holds more particles than cell_cap";
    case SDPD_ENEGEPS: return "non-positive internal energy (SSA)";
    case SDPD_ENONFINITE: return "non-finite or non-positive state value";
    case SDPD_ECAPACITY: return "pair schedule capacity exceeded";
    default: return "unknown status";
    }
}

int sdpd_create(const sdpd_params *params, void *hip_stream, sdpd_ctx **out)
{
    if (!out) return SDPD_EINVAL;
    *out = nullptr;
    int nc[3];
    int rc = check_params(params, nc);
    if (rc) return rc;
    sdpd_ctx *c = new (std::nothrow) sdpd_ctx();
    if (!c) return SDPD_ENOMEM;
    c->prm = *params;
    c->prm.A = resolved_A(params);
    derive(&c->prm, nc, c->dp);
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return SDPD_EHIP;
    }
    c->n = params->n;
    c->ncell = c->dp.ncell;
    const size_t n = (size_t)c->n, nce = (size_t)c->ncell;
    c->nscan_blocks = (int64_t)(((size_t)NMASK * nce + 1023) / 1024) + 1;
    c->obs_blocks = std::max(observe_blocks(c->n), 1);
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
            hipSuccess || lds <= 0)
            lds = 65536;
        c->max_lds = lds;
        // the LDS share of one sweep workgroup when the CU holds two waves
        // per SIMD (eight waves per CU); the default capacities stay within it
        int per_cu = 0;
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  c->device) != hipSuccess || per_cu <= 0)
            per_cu = 65536;
        c->lds_share = std::max(per_cu / 8 * FD_WAVES, 4096);
    }
    fd_default_tuning(c);
    // schedule capacity: 64 pairs per particle (a jittered lattice has ~39),
    // and at most 27 list entries per particle (1 own-cell + 2 x 13 tasks)
    c->pair_cap = std::max<int64_t>(64 * c->n, 1024);
    c->part_cap = std::max<int64_t>(27 * c->n, 1024);
    rc = SDPD_OK;
    rc = rc ? rc : dalloc(&c->cell_of, n);
    rc = rc ? rc : dalloc(&c->count, nce);
    rc = rc ? rc : dalloc(&c->cursor, nce);
    rc = rc ? rc : dalloc(&c->cell_start, nce + 1);
    rc = rc ? rc : dalloc(&c->block_sums, (size_t)c->nscan_blocks);
    rc = rc ? rc : dalloc(&c->tmp_idx, n);
    rc = rc ? rc : dalloc(&c->perm, n);
    rc = rc ? rc : dalloc(&c->cell_sorted, n);
    rc = rc ? rc : dalloc(&c->tq, 3 * n);
    rc = rc ? rc : dalloc(&c->tp, 3 * n);
    rc = rc ? rc : dalloc(&c->tf, 3 * n);
    rc = rc ? rc : dalloc(&c->teps, n);
    rc = rc ? rc : dalloc(&c->trho, n);
    rc = rc ? rc : dalloc(&c->tid, n);
    rc = rc ? rc : dalloc(&c->q4, 4 * n);
    if (c->dp.mixed) rc = rc ? rc : dalloc(&c->q4f, 4 * n);
    rc = rc ? rc : dalloc(&c->masks, (size_t)NNB * n);
    rc = rc ? rc : dalloc(&c->counters, (size_t)CNT_N);
    rc = rc ? rc : dalloc(&c->err, 1);
    rc = rc ? rc : dalloc(&c->obs_partial, (size_t)c->obs_blocks * 6);
    rc = rc ? rc : alloc_records(c);
    rc = rc ? rc : dalloc(&c->dparams, 1);
    rc = rc ? rc : dalloc(&c->task_count, (size_t)NMASK * nce);
    rc = rc ? rc : dalloc(&c->task_np, (size_t)NMASK * nce);
    rc = rc ? rc : dalloc(&c->pair_off, (size_t)NMASK * nce + 1);
    rc = rc ? rc : dalloc(&c->part_off, (size_t)NMASK * nce + 1);
    rc = rc ? rc : dalloc(&c->pairs, (size_t)c->pair_cap);
    rc = rc ? rc : dalloc(&c->draws, (size_t)4 * c->pair_cap);
    rc = rc ? rc : dalloc(&c->epoch, (size_t)c->ncell + 1);
    rc = rc ? rc : dalloc(&c->dstep, 1);
    rc = rc ? rc : dalloc(&c->part_list, (size_t)c->part_cap);
    if (!rc)
        rc = check_hip(hipMemcpyAsync(c->dparams, &c->dp, sizeof c->dp, hipMemcpyHostToDevice,
                                      c->stream));
    if (!rc) rc = launch_fill_u32(c, c->err, 0u, 1);
    if (!rc) rc = launch_fill_u64(c, c->counters, 0ull, CNT_N);
    if (!rc) rc = check_hip(hipStreamSynchronize(c->stream));
    if (!rc) rc = fd_prepare_sweep(c);
    if (rc) {
        free_ctx(c);
        return rc;
    }
    *out = c;
    return SDPD_OK;
}

int sdpd_destroy(sdpd_ctx *c)
{
    if (!c) return SDPD_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return SDPD_OK;
}

int sdpd_build_cells(sdpd_ctx *c, const sdpd_state *s)
{
    if (!c || !state_ok(c, s)) return SDPD_EINVAL;
    return run_build_cells(c, s, 0);
}

int sdpd_cell_info(sdpd_ctx *c, int32_t ncell[3], const uint32_t **cell_start)
{
    if (!c || !ncell || !cell_start) return SDPD_EINVAL;
    for (int k = 0; k < 3; ++k) ncell[k] = c->dp.nc[k];
    *cell_start = c->cell_start;
    return SDPD_OK;
}

int sdpd_copy_cell_start(sdpd_ctx *c, uint32_t *dst, int64_t capacity)
{
    if (!c || !dst || capacity < c->ncell + 1) return SDPD_EINVAL;
    int rc = check_hip(hipMemcpyAsync(dst, c->cell_start, sizeof(uint32_t) * (size_t)(c->ncell + 1),
                                      hipMemcpyDeviceToHost, c->stream));
    if (rc) return rc;
    return check_hip(hipStreamSynchronize(c->stream));
}

int sdpd_density(sdpd_ctx *c, const sdpd_state *s, int update_eps_const_S)
{
    if (!c || !state_ok(c, s) || !c->cells_valid) return SDPD_EINVAL;
    return run_density(c, s, update_eps_const_S != 0);
}

int sdpd_forces(sdpd_ctx *c, const sdpd_state *s)
{
    if (!c || !state_ok(c, s) || !c->cells_valid || !c->masks_valid) return SDPD_EINVAL;
    return run_forces(c, s, 0);
}

int sdpd_fd_metropolis(sdpd_ctx *c, const sdpd_state *s, uint64_t step, sdpd_stats *out)
{
    if (!c || !state_ok(c, s) || !c->cells_valid || !c->masks_valid) return SDPD_EINVAL;
    int rc = launch_fill_u64(c, c->counters, 0ull, CNT_N);
    if (!rc) rc = launch_fill_u64(c, (unsigned long long *)c->dstep, step, 1);
    if (!rc) rc = run_fd_sweep(c, s, c->prm.dt * c->prm.fd_every);
    if (rc) return rc;
    if (out) {
        if ((rc = run_observe(c, s, c->obs_out))) return rc;
        double rec[REC];
        if ((rc = check_hip(hipMemcpyAsync(rec, c->obs_out, sizeof rec, hipMemcpyDeviceToHost,
                                           c->stream))))
            return rc;
        rc = take_error(c);
        record_to_stats(rec, out);
        return rc;
    }
    return SDPD_OK;
}

}  // extern "C"

namespace sdpd {

// One full step (order B) enqueued on the context's stream, without any host
// synchronisation.  With set_step the device step index is written first;
// otherwise (a captured graph) it is taken as it is and advanced at the end.
int enqueue_step(sdpd_ctx *c, const sdpd_state *s, uint64_t step, bool set_step)
{
    int rc;
    const uint64_t theta = (uint64_t)c->prm.fd_every;
    if ((rc = run_build_cells(c, s, 1))) return rc;
    // FP64: the density pass leaves (x, y, z, rho) packed for the sweep
    const bool packed = !c->dp.mixed;
    if ((rc = run_density(c, s, 1, packed))) return rc;
    if ((rc = launch_fill_u64(c, c->counters, 0ull, CNT_N))) return rc;
    if (step % theta == 0) {
        if (set_step &&
            (rc = launch_fill_u64(c, (unsigned long long *)c->dstep, step, 1)))
            return rc;
        if ((rc = run_fd_sweep(c, s, c->prm.dt * (double)theta, packed))) return rc;
    }
    if ((rc = run_forces(c, s, 1))) return rc;
    if (!set_step && (rc = launch_incr_u64(c, (unsigned long long *)c->dstep))) return rc;
    return SDPD_OK;
}

}  // namespace sdpd

extern "C" {

int sdpd_step(sdpd_ctx *c, const sdpd_state *s, uint64_t step0, int nsteps, sdpd_stats *per_step)
{
    if (!c || !state_ok(c, s) || nsteps < 0 || !c->cells_valid) return SDPD_EINVAL;
    int rc;
    if (!per_step) {
        for (int k = 0; k < nsteps; ++k)
            if ((rc = enqueue_step(c, s, step0 + (uint64_t)k, true))) return rc;
        return SDPD_OK;
    }
    if (nsteps == 0) return SDPD_OK;
    double *host = new (std::nothrow) double[(size_t)nsteps * REC];
    if (!host) return SDPD_ENOMEM;
    // the context's record buffer holds obs_cap steps: records go to the
    // host in chunks of that many steps (the copy of a chunk is ordered on
    // the stream before the next chunk overwrites the buffer)
    rc = SDPD_OK;
    for (int k0 = 0; k0 < nsteps && !rc; k0 += (int)c->obs_cap) {
        const int kn = std::min((int)c->obs_cap, nsteps - k0);
        for (int k = 0; k < kn && !rc; ++k) {
            rc = enqueue_step(c, s, step0 + (uint64_t)(k0 + k), true);
            if (rc) break;
            timer_begin(c, TK_OBSERVE);
            rc = run_observe(c, s, c->obs_out + (size_t)k * REC);
            timer_end(c, TK_OBSERVE);
        }
        if (!rc)
            rc = check_hip(hipMemcpyAsync(host + (size_t)k0 * REC, c->obs_out,
                                          sizeof(double) * REC * (size_t)kn,
                                          hipMemcpyDeviceToHost, c->stream));
    }
    const int rc2 = take_error(c);
    if (!rc)
        for (int k = 0; k < nsteps; ++k) record_to_stats(host + (size_t)k * REC, &per_step[k]);
    delete[] host;
    return rc ? rc : rc2;
}

int sdpd_observe(sdpd_ctx *c, const sdpd_state *s, sdpd_stats *out)
{
    if (!c || !state_ok(c, s) || !out) return SDPD_EINVAL;
    int rc = run_observe(c, s, c->obs_out);
    if (rc) return rc;
    double rec[REC];
    if ((rc = check_hip(hipMemcpyAsync(rec, c->obs_out, sizeof rec, hipMemcpyDeviceToHost,
                                       c->stream))))
        return rc;
    rc = take_error(c);
    record_to_stats(rec, out);
    return rc;
}

}  // extern "C"

namespace {

// Scratch of sdpd_observe_noalloc: the per-block partial sums (6 doubles per
// block, at most OBS_MAX_BLOCKS blocks: 48 KiB).  Each device holds its own
// copy until the process ends.  In host code `scratch` only names the
// symbol: kernels and copies use the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) double scratch[(size_t)sdpd::OBS_MAX_BLOCKS * 6];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];

// the current device's address of `scratch` (looked up on the first call on
// that device)
int scratch_address(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SDPD_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SDPD_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SDPD_EHIP;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SDPD_OK;
}

}  // namespace

extern "C" {

int sdpd_observe_noalloc(const sdpd_params *params, const sdpd_state *s, void *hip_stream,
                         double *out)
{
    int nc[3];
    int rc = check_params(params, nc);
    if (rc) return rc;
    if (!s || !out || (params->n > 0 && (!s->p || !s->eps))) return SDPD_EINVAL;
    if (params->n > SDPD_OBSERVE_NOALLOC_MAX_N) return SDPD_EINVAL;
    if ((int64_t)observe_blocks(params->n) * 6 > (int64_t)(sizeof(scratch) / sizeof(double)))
        return SDPD_EINVAL;
    double *partial = nullptr;
    if ((rc = scratch_address(&partial))) return rc;
    sdpd_params prm = *params;
    prm.A = resolved_A(params);
    DevParams dp;
    derive(&prm, nc, dp);
    return launch_observe(dp, s->p, s->eps, partial, nullptr, out, (hipStream_t)hip_stream);
}

int sdpd_sync(sdpd_ctx *c)
{
    if (!c) return SDPD_EINVAL;
    return take_error(c);
}

int sdpd_set_timing(sdpd_ctx *c, int enable)
{
    return sdpd_set_timing_mask(c, enable ? (1u << TK_N) - 1u : 0u);
}

int sdpd_set_timing_mask(sdpd_ctx *c, uint32_t mask)
{
    if (!c || (mask >> TK_N) != 0u) return SDPD_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SDPD_EHIP;
    c->timing = (int)mask;
    c->timer.used = 0;
    return SDPD_OK;
}

int sdpd_timing(sdpd_ctx *c, double ms[6], int64_t launches[6])
{
    if (!c || !ms || !launches) return SDPD_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SDPD_EHIP;
    for (int k = 0; k < TK_N; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    Timer &T = c->timer;
    for (size_t i = 0; i < T.used; i += 2) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, T.pool[i], T.pool[i + 1]) != hipSuccess) return SDPD_EHIP;
        ms[T.cls[i / 2]] += t;
        launches[T.cls[i / 2]] += 1;
    }
    T.used = 0;
    return SDPD_OK;
}

int sdpd_tune(sdpd_ctx *c, const sdpd_tuning *t)
{
    if (!c || !t) return SDPD_EINVAL;
    sdpd_tuning u = c->tuning;
    for (int k = 0; k < 4; ++k) {
        if (t->fd_tasks[k]) u.fd_tasks[k] = t->fd_tasks[k];
        if (t->fd_lds_particles[k] < 0 || t->fd_lds_pairs[k] < 0) {
            // the capacities the defaults give this many tasks
            if (u.fd_tasks[k] < 1 || u.fd_tasks[k] > FD_MAXTASKS) return SDPD_EINVAL;
            fd_class_caps(c, k, u.fd_tasks[k], u.fd_lds_particles[k], u.fd_lds_pairs[k]);
            continue;
        }
        if (t->fd_lds_particles[k]) u.fd_lds_particles[k] = t->fd_lds_particles[k];
        if (t->fd_lds_pairs[k]) u.fd_lds_pairs[k] = t->fd_lds_pairs[k];
    }
    const int rc = fd_check_tuning(c, &u);
    if (rc) return rc;
    c->tuning = u;
    ++c->tune_gen;   // graphs captured before keep the old launch size
    return fd_prepare_sweep(c);
}

int sdpd_fd_schedule_size(sdpd_ctx *c, int64_t *pairs, int64_t *staged)
{
    if (!c || !pairs || !staged) return SDPD_EINVAL;
    *pairs = *staged = 0;
    if (!c->fd_swept) return SDPD_OK;
    const int64_t ntask = (int64_t)NMASK * c->ncell;
    uint32_t v[2] = {0u, 0u};
    int rc = check_hip(hipMemcpyAsync(&v[0], c->pair_off + ntask, sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, c->stream));
    if (!rc)
        rc = check_hip(hipMemcpyAsync(&v[1], c->part_off + ntask, sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, c->stream));
    if (!rc) rc = check_hip(hipStreamSynchronize(c->stream));
    if (rc) return rc;
    *pairs = v[0];
    *staged = v[1];
    return SDPD_OK;
}

int sdpd_get_tuning(sdpd_ctx *c, sdpd_tuning *out)
{
    if (!c || !out) return SDPD_EINVAL;
    *out = c->tuning;
    return SDPD_OK;
}

int sdpd_set_sweep_mode(sdpd_ctx *c, int mode)
{
    if (!c || mode < SDPD_SWEEP_AUTO || mode > SDPD_SWEEP_PER_GROUP) return SDPD_EINVAL;
    c->sweep_mode = mode;
    return SDPD_OK;
}

int sdpd_sweep_mode(sdpd_ctx *c, int *in_use)
{
    if (!c) return SDPD_EINVAL;
    if (in_use) *in_use = fd_one_launch(c) ? SDPD_SWEEP_ONE : SDPD_SWEEP_PER_GROUP;
    return c->sweep_mode;
}

}  // extern "C"

namespace {

// Fastest of `trials` sweeps (ms) with the context's current tuning and
// layout.  The schedule is in place; each trial starts from the momenta and
// energies of s, copied into the scratch state w.
int time_sweeps(sdpd_ctx *c, const sdpd_state *s, const sdpd_state *w, int trials,
                hipEvent_t e0, hipEvent_t e1, double &best)
{
    const size_t n = (size_t)c->n;
    const double dt_fd = c->prm.dt * c->prm.fd_every;
    best = 1e300;
    for (int t = 0; t < trials; ++t) {
        int rc = check_hip(hipMemcpyAsync(w->p, s->p, sizeof(double) * 3 * n,
                                          hipMemcpyDeviceToDevice, c->stream));
        if (!rc) rc = check_hip(hipMemcpyAsync(w->eps, s->eps, sizeof(double) * n,
                                               hipMemcpyDeviceToDevice, c->stream));
        if (!rc) rc = launch_fill_u64(c, c->counters, 0ull, CNT_N);
        if (!rc) rc = check_hip(hipEventRecord(e0, c->stream));
        if (!rc) rc = fd_launch_sweep(c, w, dt_fd);
        if (!rc) rc = check_hip(hipEventRecord(e1, c->stream));
        if (!rc) rc = check_hip(hipEventSynchronize(e1));
        float ms = 0.0f;
        if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1));
        if (rc) return rc;
        best = std::min(best, (double)ms);
    }
    return SDPD_OK;
}

int autotune(sdpd_ctx *c, const sdpd_state *s, int trials, const sdpd_state *w, hipEvent_t e0,
             hipEvent_t e1)
{
    int rc = launch_fill_u64(c, (unsigned long long *)c->dstep, 0ull, 1);
    if (!rc) rc = fd_sweep_prepare(c, w, false);
    if (rc) return rc;
    const int mode0 = c->sweep_mode;
    sdpd_tuning best = c->tuning;
    double tbest;
    if ((rc = time_sweeps(c, s, w, trials, e0, e1, tbest))) return rc;
    // coordinate descent over the tasks per workgroup of each phase class,
    // with the LDS capacities the defaults give that many tasks; a candidate
    // must be 1 % faster to replace the current choice
    static const double kFactor[4] = {0.5, 0.75, 1.5, 2.0};
    for (int k = 0; k < 4; ++k) {
        const int t0 = best.fd_tasks[k];
        int tried[4] = {0, 0, 0, 0};
        for (int f = 0; f < 4; ++f) {
            const int t = std::min(std::max((int)std::lround(t0 * kFactor[f]), 1), FD_MAXTASKS);
            bool seen = t == t0;
            for (int q = 0; q < f; ++q) seen = seen || tried[q] == t;
            tried[f] = t;
            if (seen) continue;
            sdpd_tuning u = best;
            u.fd_tasks[k] = t;
            fd_class_caps(c, k, t, u.fd_lds_particles[k], u.fd_lds_pairs[k]);
            if (fd_check_tuning(c, &u)) continue;
            c->tuning = u;
            double tm;
            if ((rc = fd_prepare_sweep(c)) || (rc = time_sweeps(c, s, w, trials, e0, e1, tm)))
                return rc;
            if (tm < 0.99 * tbest) {
                best = u;
                tbest = tm;
            }
        }
    }
    c->tuning = best;
    if ((rc = fd_prepare_sweep(c))) return rc;
    if (mode0 == SDPD_SWEEP_AUTO) {   // the layout too, unless the caller fixed it
        int win = SDPD_SWEEP_AUTO;
        for (int m = SDPD_SWEEP_ONE; m <= SDPD_SWEEP_PER_GROUP; ++m) {
            c->sweep_mode = m;
            double tm;
            if ((rc = time_sweeps(c, s, w, trials, e0, e1, tm))) return rc;
            if (tm < 0.99 * tbest) {
                win = m;
                tbest = tm;
            }
        }
        c->sweep_mode = mode0;
        if (win != SDPD_SWEEP_AUTO) {
            // keep the automatic choice when it is the faster layout
            c->sweep_mode = SDPD_SWEEP_AUTO;
            const int autom = fd_one_launch(c) ? SDPD_SWEEP_ONE : SDPD_SWEEP_PER_GROUP;
            c->sweep_mode = win == autom ? SDPD_SWEEP_AUTO : win;
        }
    }
    return SDPD_OK;
}

}  // namespace

extern "C" {

int sdpd_autotune(sdpd_ctx *c, const sdpd_state *s, int trials, sdpd_tuning *chosen)
{
    if (!c || !state_ok(c, s) || !c->cells_valid || !c->masks_valid || trials < 1 || trials > 64)
        return SDPD_EINVAL;
    if (c->prm.fd == SDPD_FD_NONE || c->n == 0) {
        if (chosen) *chosen = c->tuning;
        return SDPD_OK;
    }
    // scratch momenta and energies: the caller's state is not touched
    sdpd_state w = *s;
    double *wp = nullptr, *weps = nullptr;
    int rc = dalloc(&wp, 3 * (size_t)c->n);
    if (!rc) rc = dalloc(&weps, (size_t)c->n);
    w.p = wp;
    w.eps = weps;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) rc = check_hip(hipEventCreate(&e0));
    if (!rc) rc = check_hip(hipEventCreate(&e1));
    const sdpd_tuning before = c->tuning;
    const int mode_before = c->sweep_mode;
    if (!rc) {
        const int tt = c->timing;
        c->timing = 0;   // the context's own event timer stays out of the trials
        rc = check_hip(hipStreamSynchronize(c->stream));
        if (!rc) {
            ++c->tune_gen;   // graphs captured before keep the old launch size
            rc = autotune(c, s, trials, &w, e0, e1);
        }
        c->timing = tt;
        if (!rc) rc = take_error(c);
        if (rc) {   // back to where the call started
            c->tuning = before;
            c->sweep_mode = mode_before;
            (void)fd_prepare_sweep(c);
        }
    }
    (void)hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (wp) (void)hipFree(wp);
    if (weps) (void)hipFree(weps);
    if (!rc && chosen) *chosen = c->tuning;
    return rc;
}

}  // extern "C"
