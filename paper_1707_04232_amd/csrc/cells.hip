// Cell list: (optional half kick + drift), cell assignment, counting sort by
// cell, deterministic order by id inside each cell, gather of the state.
//
// The cell list is not part of the paper; it fixes the neighbour search and
// the order of the pairwise fluctuation/dissipation updates.
#include "sdpd_internal.hpp"

namespace sdpd {

struct FillU32Args {
    uint32_t *p;
    uint32_t v;
    int64_t n;
};
__device__ __forceinline__ void fill_u32_body(const FillU32Args &a, uint32_t blk)
{
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i < a.n) a.p[i] = a.v;
}
__global__ void k_fill_u32(FillU32Args a) { fill_u32_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_fill_u32_multi, FillU32Args, fill_u32_body, 256)

struct FillU64Args {
    unsigned long long *p;
    unsigned long long v;
    int64_t n;
};
__device__ __forceinline__ void fill_u64_body(const FillU64Args &a, uint32_t blk)
{
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i < a.n) a.p[i] = a.v;
}
__global__ void k_fill_u64(FillU64Args a) { fill_u64_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_fill_u64_multi, FillU64Args, fill_u64_body, 256)

// Half kick and drift of the Velocity-Verlet scheme, eq. (sdpd-verlet),
// fused with the cell assignment:  p += dt/2 f;  q += dt p / m wrapped once
// into [0, box);  cell = cx + nx (cy + ny cz).
// ctr[key] += 1 for every active lane with one atomic per distinct key of
// the wave (the state arrives nearly in cell order, so a wave holds a few
// cells); returns the lane's position among the increments of its key
__device__ __forceinline__ uint32_t wave_counted_inc(uint32_t *ctr, uint32_t key)
{
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(1);
    uint32_t pos = 0;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const uint32_t lkey = (uint32_t)__shfl((int)key, leader);
        const uint64_t peers = __ballot(key == lkey) & todo;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[lkey], (uint32_t)__popcll(peers));
        base = (uint32_t)__shfl((int)base, leader);
        if ((peers >> lane) & 1ull)
            pos = base + (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
        todo &= ~peers;
    }
    return pos;
}

struct KickDriftArgs {
    DevParams P;
    double *q, *p;
    const double *f;
    int kick_drift;
    uint32_t *cell_of, *count, *err;
};
__device__ __forceinline__ void kick_drift_assign_body(const KickDriftArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    double *q = a.q, *p = a.p;
    const double *f = a.f;
    const int kick_drift = a.kick_drift;
    uint32_t *cell_of = a.cell_of, *count = a.count, *err = a.err;
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    int cc[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x = q[k * n + i];
        if (kick_drift) {
            double pk = p[k * n + i] + (0.5 * P.dt) * f[k * n + i];
            p[k * n + i] = pk;
            x = x + P.dt * pk / P.m;
            if (x >= P.box[k]) x -= P.box[k];
            else if (x < 0.0) x += P.box[k];
            q[k * n + i] = x;
        }
        finite = finite && isfinite(x);
        cc[k] = cell_coord(finite ? x : 0.0, P.inv_cell[k], P.nc[k]);
    }
    if (!finite) atomicOr(err, ERR_NONFINITE);
    uint32_t c = (uint32_t)(cc[0] + P.nc[0] * (cc[1] + P.nc[1] * cc[2]));
    cell_of[i] = c;
    (void)wave_counted_inc(count, c);
}
__global__ void k_kick_drift_assign(KickDriftArgs a) { kick_drift_assign_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_kick_drift_assign_multi, KickDriftArgs, kick_drift_assign_body, 256)

// --- exclusive scan of the cell counts into cell_start (3 passes) ---------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;

__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s, uint32_t *total)
{
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        uint32_t add = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    uint32_t incl = s[t];
    *total = s[SCAN_THREADS - 1];
    __syncthreads();
    return incl - v;
}

struct ScanLocalArgs {
    const uint32_t *count;
    int64_t ncell;
    int cap;
    uint32_t *out, *block_sums, *err;
};
__device__ __forceinline__ void scan_local_body(const ScanLocalArgs &a, uint32_t blk)
{
    const uint32_t *count = a.count;
    const int64_t ncell = a.ncell;
    const int cap = a.cap;
    uint32_t *out = a.out, *block_sums = a.block_sums, *err = a.err;
    __shared__ uint32_t s[SCAN_THREADS];
    int64_t base = (int64_t)blk * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD], sum = 0;
    bool over = false;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = base + k < ncell ? count[base + k] : 0u;
        over = over || (cap >= 0 && v[k] > (uint32_t)cap);
        sum += v[k];
    }
    if (over) atomicOr(err, ERR_CELLCAP);
    uint32_t total;
    uint32_t ex = block_exclusive_scan(sum, s, &total);
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        if (base + k < ncell) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) block_sums[blk] = total;
}
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_local(ScanLocalArgs a)
{
    scan_local_body(a, blockIdx.x);
}
SDPD_MULTI_KERNEL(k_scan_local_multi, ScanLocalArgs, scan_local_body, SCAN_THREADS)

// one workgroup: exclusive scan of the block sums, in place; the grand
// total goes to block_sums[nblocks]
struct ScanSumsArgs {
    uint32_t *block_sums;
    int64_t nblocks;
};
__device__ __forceinline__ void scan_sums_body(const ScanSumsArgs &a, uint32_t)
{
    uint32_t *block_sums = a.block_sums;
    const int64_t nblocks = a.nblocks;
    __shared__ uint32_t s[SCAN_THREADS];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nblocks; base += SCAN_THREADS) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nblocks ? block_sums[i] : 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(v, s, &total);
        if (i < nblocks) block_sums[i] = ex + carry;
        carry += total;
    }
    if (threadIdx.x == 0) block_sums[nblocks] = carry;
}
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(ScanSumsArgs a)
{
    scan_sums_body(a, 0u);
}
SDPD_MULTI_KERNEL(k_scan_sums_multi, ScanSumsArgs, scan_sums_body, SCAN_THREADS)

struct ScanAddArgs {
    uint32_t *out;
    const uint32_t *block_sums;
    int64_t count, nblocks;
};
__device__ __forceinline__ void scan_add_body(const ScanAddArgs &a, uint32_t blk)
{
    int64_t base = (int64_t)blk * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
    uint32_t add = a.block_sums[blk];
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k)
        if (base + k < a.count) a.out[base + k] += add;
    if (blk == 0 && threadIdx.x == 0) a.out[a.count] = a.block_sums[a.nblocks];
}
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(ScanAddArgs a)
{
    scan_add_body(a, blockIdx.x);
}
SDPD_MULTI_KERNEL(k_scan_add_multi, ScanAddArgs, scan_add_body, SCAN_THREADS)

// out[0..count] = exclusive prefix sums of in[0..count), out[count] = total.
// block_sums needs ceil(count / 1024) + 1 entries.  A value above cap sets
// ERR_CELLCAP (cap < 0: no check).
int run_scan(sdpd_ctx *c, const uint32_t *in, uint32_t *out, int64_t count, uint32_t *block_sums,
             int cap)
{
    const int64_t nb = (count + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb == 0) return launch_fill_u32(c, out, 0u, 1);
    int rc = launch_or_record(c, k_scan_local, k_scan_local_multi, (unsigned)nb, SCAN_THREADS, 0,
                              ScanLocalArgs{in, count, cap, out, block_sums, c->err});
    if (!rc)
        rc = launch_or_record(c, k_scan_sums, k_scan_sums_multi, 1u, SCAN_THREADS, 0,
                              ScanSumsArgs{block_sums, nb});
    if (!rc)
        rc = launch_or_record(c, k_scan_add, k_scan_add_multi, (unsigned)nb, SCAN_THREADS, 0,
                              ScanAddArgs{out, block_sums, count, nb});
    return rc;
}

// particle i goes to an arbitrary free position of its cell
struct ScatterArgs {
    const uint32_t *cell_of, *cell_start;
    uint32_t *cursor, *tmp_idx;
    int64_t n;
};
__device__ __forceinline__ void scatter_body(const ScatterArgs &a, uint32_t blk)
{
    int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t c = a.cell_of[i];
    uint32_t pos = a.cell_start[c] + wave_counted_inc(a.cursor, c);
    a.tmp_idx[pos] = (uint32_t)i;
}
__global__ void k_scatter(ScatterArgs a) { scatter_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_scatter_multi, ScatterArgs, scatter_body, 256)

// final position = cell start + rank of the id inside the cell (ties, which
// only invalid input with repeated ids has, broken by the scatter position so
// that every slot is written once); cells above the capacity keep the
// scatter order (the overflow is reported by the scan)
struct RankArgs {
    const uint32_t *tmp_idx, *cell_of, *cell_start, *id;
    uint32_t *perm;
    int64_t n;
    int cap;
};
__device__ __forceinline__ void rank_body(const RankArgs &a, uint32_t blk)
{
    const uint32_t *tmp_idx = a.tmp_idx, *cell_of = a.cell_of, *cell_start = a.cell_start,
                   *id = a.id;
    uint32_t *perm = a.perm;
    const int cap = a.cap;
    int64_t k = (int64_t)blk * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    uint32_t i = tmp_idx[k];
    uint32_t c = cell_of[i];
    uint32_t s = cell_start[c], e = cell_start[c + 1];
    if (e - s > (uint32_t)cap) {
        perm[k] = i;
        return;
    }
    uint32_t my = id[i], rank = 0;
    for (uint32_t t = s; t < e; ++t) {
        const uint32_t o = id[tmp_idx[t]];
        rank += (o < my || (o == my && t < (uint32_t)k)) ? 1u : 0u;
    }
    perm[s + rank] = i;
}
__global__ void k_rank(RankArgs a) { rank_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_rank_multi, RankArgs, rank_body, 256)

// gather into (cell, id) order; with q4f (mixed precision) also the FP32
// position relative to the particle's cell origin, in the x, y, z slots of
// the particle's 16-byte record (the w slot takes P/rho^2 later)
struct GatherArgs {
    DevParams P;
    int64_t n;
    const uint32_t *perm, *cell_of;
    const double *q, *p, *eps, *rho, *f;
    const uint32_t *id;
    double *tq, *tp, *teps, *trho, *tf;
    uint32_t *tid, *cell_sorted;
    float *q4f;
    double *q4;
};
__device__ __forceinline__ void gather_body(const GatherArgs &a, uint32_t blk)
{
    const DevParams &P = a.P;
    const int64_t n = a.n;
    const uint32_t *perm = a.perm, *cell_of = a.cell_of;
    const double *q = a.q, *p = a.p, *eps = a.eps, *rho = a.rho, *f = a.f;
    const uint32_t *id = a.id;
    double *tq = a.tq, *tp = a.tp, *teps = a.teps, *trho = a.trho, *tf = a.tf;
    uint32_t *tid = a.tid, *cell_sorted = a.cell_sorted;
    float *q4f = a.q4f;
    double *q4 = a.q4;
    int64_t k = (int64_t)blk * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
    if (q4f) {
        const uint32_t c = cell_of[i];
        const int cc[3] = {(int)(c % (uint32_t)P.nc[0]), (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]),
                           (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]))};
#pragma unroll
        for (int d = 0; d < 3; ++d)
            q4f[4 * k + d] = (float)(q[d * n + i] - (double)cc[d] * (P.box[d] / P.nc[d]));
    }
    q4[4 * k] = q[i];
    q4[4 * k + 1] = q[n + i];
    q4[4 * k + 2] = q[2 * n + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        tq[c * n + k] = q[c * n + i];
        tp[c * n + k] = p[c * n + i];
        if (tf) tf[c * n + k] = f[c * n + i];
    }
    teps[k] = eps[i];
    trho[k] = rho[i];
    tid[k] = id[i];
    cell_sorted[k] = cell_of[i];
}
__global__ void k_gather(GatherArgs a) { gather_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_gather_multi, GatherArgs, gather_body, 256)

// the sorted arrays back into the caller's state, one launch (f only when
// it was gathered)
struct CopyBackArgs {
    int64_t n;
    const double *tq, *tp, *tf, *teps, *trho;
    const uint32_t *tid;
    double *q, *p, *f, *eps, *rho;
    uint32_t *id;
};
__device__ __forceinline__ void copy_back_body(const CopyBackArgs &a, uint32_t blk)
{
    const int64_t n = a.n;
    const double *tq = a.tq, *tp = a.tp, *tf = a.tf, *teps = a.teps, *trho = a.trho;
    const uint32_t *tid = a.tid;
    double *q = a.q, *p = a.p, *f = a.f, *eps = a.eps, *rho = a.rho;
    uint32_t *id = a.id;
    const int64_t k = (int64_t)blk * blockDim.x + threadIdx.x;
    if (k >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        q[c * n + k] = tq[c * n + k];
        p[c * n + k] = tp[c * n + k];
        if (tf) f[c * n + k] = tf[c * n + k];
    }
    eps[k] = teps[k];
    rho[k] = trho[k];
    id[k] = tid[k];
}
__global__ void k_copy_back(CopyBackArgs a) { copy_back_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_copy_back_multi, CopyBackArgs, copy_back_body, 256)

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

struct IncrArgs {
    unsigned long long *p;
};
__device__ __forceinline__ void incr_u64_body(const IncrArgs &a, uint32_t)
{
    if (threadIdx.x == 0) *a.p += 1ull;
}
__global__ void k_incr_u64(IncrArgs a) { incr_u64_body(a, 0u); }
SDPD_MULTI_KERNEL(k_incr_u64_multi, IncrArgs, incr_u64_body, 64)

int launch_incr_u64(sdpd_ctx *c, unsigned long long *p)
{
    return launch_or_record(c, k_incr_u64, k_incr_u64_multi, 1u, 64, 0, IncrArgs{p});
}

int launch_fill_u32(sdpd_ctx *c, uint32_t *p, uint32_t v, int64_t n)
{
    if (n <= 0) return SDPD_OK;
    return launch_or_record(c, k_fill_u32, k_fill_u32_multi, blocks_for(n, 256), 256, 0,
                            FillU32Args{p, v, n});
}

int launch_fill_u64(sdpd_ctx *c, unsigned long long *p, unsigned long long v, int64_t n)
{
    if (n <= 0) return SDPD_OK;
    return launch_or_record(c, k_fill_u64, k_fill_u64_multi, blocks_for(n, 256), 256, 0,
                            FillU64Args{p, v, n});
}

// Sort the state by (cell, id).  With kick_drift the first half kick and the
// drift of the step are applied first.
int run_build_cells(sdpd_ctx *c, const sdpd_state *s, int kick_drift)
{
    const int64_t n = c->n, nc = c->ncell;
    int rc;
    timer_begin(c, TK_CELLS);
    if ((rc = launch_fill_u32(c, c->count, 0u, nc))) return rc;
    if ((rc = launch_fill_u32(c, c->cursor, 0u, nc))) return rc;
    if (n > 0 &&
        (rc = launch_or_record(c, k_kick_drift_assign, k_kick_drift_assign_multi,
                               blocks_for(n, 256), 256, 0,
                               KickDriftArgs{c->dp, s->q, s->p, s->f, kick_drift, c->cell_of,
                                             c->count, c->err})))
        return rc;
    if ((rc = run_scan(c, c->count, c->cell_start, nc, c->block_sums, c->prm.cell_cap))) return rc;
    if (n > 0) {
        unsigned g = blocks_for(n, 256);
        // inside a step (kick_drift) the forces are recomputed before
        // anything reads them, so they are not carried through the sort
        double *tf = kick_drift ? nullptr : c->tf;
        rc = launch_or_record(c, k_scatter, k_scatter_multi, g, 256, 0,
                              ScatterArgs{c->cell_of, c->cell_start, c->cursor, c->tmp_idx, n});
        if (!rc)
            rc = launch_or_record(c, k_rank, k_rank_multi, g, 256, 0,
                                  RankArgs{c->tmp_idx, c->cell_of, c->cell_start, s->id, c->perm,
                                           n, c->prm.cell_cap});
        if (!rc)
            rc = launch_or_record(c, k_gather, k_gather_multi, g, 256, 0,
                                  GatherArgs{c->dp, n, c->perm, c->cell_of, s->q, s->p, s->eps,
                                             s->rho, s->f, s->id, c->tq, c->tp, c->teps, c->trho,
                                             tf, c->tid, c->cell_sorted, c->q4f, c->q4});
        if (!rc)
            rc = launch_or_record(c, k_copy_back, k_copy_back_multi, g, 256, 0,
                                  CopyBackArgs{n, c->tq, c->tp, tf, c->teps, c->trho, c->tid, s->q,
                                               s->p, s->f, s->eps, s->rho, s->id});
        if (rc) return rc;
    }
    timer_end(c, TK_CELLS);
    c->cells_valid = 1;
    c->masks_valid = 0;
    return SDPD_OK;
}

}  // namespace sdpd
