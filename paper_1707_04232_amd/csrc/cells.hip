// Cell list: (optional half kick + drift), cell assignment, counting sort by
// cell, deterministic order by id inside each cell, gather of the state.
//
// The cell list is not part of the paper; it fixes the neighbour search and
// the order of the pairwise fluctuation/dissipation updates.
#include "sdpd_internal.hpp"

namespace sdpd {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

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

__global__ void k_kick_drift_assign(DevParams P, double *q, double *p, const double *f,
                                    int kick_drift, uint32_t *cell_of, uint32_t *count,
                                    uint32_t *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_scan_local(const uint32_t *count, int64_t ncell, int cap, uint32_t *out,
                             uint32_t *block_sums, uint32_t *err)
{
    __shared__ uint32_t s[SCAN_THREADS];
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
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
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the block sums, in place; the grand
// total goes to block_sums[nblocks]
__global__ void k_scan_sums(uint32_t *block_sums, int64_t nblocks)
{
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

__global__ void k_scan_add(uint32_t *out, const uint32_t *block_sums, int64_t count,
                           int64_t nblocks)
{
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
    uint32_t add = block_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k)
        if (base + k < count) out[base + k] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[count] = block_sums[nblocks];
}

// out[0..count] = exclusive prefix sums of in[0..count), out[count] = total.
// block_sums needs ceil(count / 1024) + 1 entries.  A value above cap sets
// ERR_CELLCAP (cap < 0: no check).
int run_scan(sdpd_ctx *c, const uint32_t *in, uint32_t *out, int64_t count, uint32_t *block_sums,
             int cap)
{
    const int64_t nb = (count + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb == 0) return launch_fill_u32(c, out, 0u, 1);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, c->stream, in,
                       count, cap, out, block_sums, c->err);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, c->stream, block_sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, c->stream, out,
                       block_sums, count, nb);
    return check_hip(hipGetLastError());
}

// particle i goes to an arbitrary free position of its cell
__global__ void k_scatter(const uint32_t *cell_of, const uint32_t *cell_start, uint32_t *cursor,
                          uint32_t *tmp_idx, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = cell_of[i];
    uint32_t pos = cell_start[c] + wave_counted_inc(cursor, c);
    tmp_idx[pos] = (uint32_t)i;
}

// final position = cell start + rank of the id inside the cell (ties, which
// only invalid input with repeated ids has, broken by the scatter position so
// that every slot is written once); cells above the capacity keep the
// scatter order (the overflow is reported by the scan)
__global__ void k_rank(const uint32_t *tmp_idx, const uint32_t *cell_of,
                       const uint32_t *cell_start, const uint32_t *id, uint32_t *perm, int64_t n,
                       int cap)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
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

// gather into (cell, id) order; with qr (mixed precision) also the FP32
// position relative to the particle's cell origin
__global__ void k_gather(DevParams P, int64_t n, const uint32_t *perm, const uint32_t *cell_of,
                         const double *q, const double *p, const double *eps, const double *rho,
                         const double *f, const uint32_t *id, double *tq, double *tp,
                         double *teps, double *trho, double *tf, uint32_t *tid,
                         uint32_t *cell_sorted, float *qr, double *q4)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
    if (qr) {
        const uint32_t c = cell_of[i];
        const int cc[3] = {(int)(c % (uint32_t)P.nc[0]), (int)((c / (uint32_t)P.nc[0]) % (uint32_t)P.nc[1]),
                           (int)(c / ((uint32_t)P.nc[0] * (uint32_t)P.nc[1]))};
#pragma unroll
        for (int d = 0; d < 3; ++d)
            qr[d * n + k] = (float)(q[d * n + i] - (double)cc[d] * (P.box[d] / P.nc[d]));
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

// the sorted arrays back into the caller's state, one launch (f only when
// it was gathered)
__global__ void k_copy_back(int64_t n, const double *tq, const double *tp, const double *tf,
                            const double *teps, const double *trho, const uint32_t *tid,
                            double *q, double *p, double *f, double *eps, double *rho,
                            uint32_t *id)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ void k_incr_u64(unsigned long long *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1ull;
}

int launch_incr_u64(sdpd_ctx *c, unsigned long long *p)
{
    hipLaunchKernelGGL(k_incr_u64, dim3(1), dim3(64), 0, c->stream, p);
    return check_hip(hipGetLastError());
}

int launch_fill_u32(sdpd_ctx *c, uint32_t *p, uint32_t v, int64_t n)
{
    if (n <= 0) return SDPD_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, p, v, n);
    return check_hip(hipGetLastError());
}

int launch_fill_u64(sdpd_ctx *c, unsigned long long *p, unsigned long long v, int64_t n)
{
    if (n <= 0) return SDPD_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, p, v, n);
    return check_hip(hipGetLastError());
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
    if (n > 0) {
        hipLaunchKernelGGL(k_kick_drift_assign, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                           c->dp, s->q, s->p, s->f, kick_drift, c->cell_of, c->count, c->err);
        if ((rc = check_hip(hipGetLastError()))) return rc;
    }
    if ((rc = run_scan(c, c->count, c->cell_start, nc, c->block_sums, c->prm.cell_cap))) return rc;
    if (n > 0) {
        unsigned g = blocks_for(n, 256);
        hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, c->stream, c->cell_of, c->cell_start,
                           c->cursor, c->tmp_idx, n);
        hipLaunchKernelGGL(k_rank, dim3(g), dim3(256), 0, c->stream, c->tmp_idx, c->cell_of,
                           c->cell_start, s->id, c->perm, n, c->prm.cell_cap);
        // inside a step (kick_drift) the forces are recomputed before
        // anything reads them, so they are not carried through the sort
        double *tf = kick_drift ? nullptr : c->tf;
        hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, c->stream, c->dp, n, c->perm,
                           c->cell_of, s->q, s->p, s->eps, s->rho, s->f, s->id, c->tq, c->tp,
                           c->teps, c->trho, tf, c->tid, c->cell_sorted, c->qr, c->q4);
        hipLaunchKernelGGL(k_copy_back, dim3(g), dim3(256), 0, c->stream, n, c->tq, c->tp, tf,
                           c->teps, c->trho, c->tid, s->q, s->p, s->f, s->eps, s->rho, s->id);
        if ((rc = check_hip(hipGetLastError()))) return rc;
    }
    timer_end(c, TK_CELLS);
    c->cells_valid = 1;
    c->masks_valid = 0;
    return SDPD_OK;
}

}  // namespace sdpd
