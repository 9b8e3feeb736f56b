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
// GPU schedule.  The scheduling pass (schedule.hip) has stored, for every
// task, its active pairs with their conflict level.  One launch per phase:
// a workgroup of one wave takes a batch of consecutive tasks of the phase,
// stages in LDS only the particles that take part in a pair, sorts the
// batch's pairs by level and applies the pairs of one level (which share no
// particle) as parallel steps of 64 lanes.
#include "fd_math.hpp"

namespace sdpd {

constexpr int FD_MAXTASKS = 64;    // tasks per batch
constexpr int FD_NLVL = 64;        // levels of a task are 1..64

struct FdPhase {
    int phase;          // 0..104
    int mslot;          // mask / task slot of the phase (0 = own cell)
    int d[3];           // offset of B relative to A
    int par[3];         // coordinate parity of A
    int hx, hy;         // tasks per axis (x, y) of a parity class
    int64_t ntasks;
    int64_t tasks_per_wg;
    int64_t task_base;  // index of the phase's first task in sweep order
};

template <int MAXP, int MAXPAIRS>
struct FdShared {
    double q[3][MAXP];
    double p[3][MAXP];
    double eps[MAXP];
    double rho[MAXP];
    uint32_t id[MAXP];
    uint32_t gidx[MAXP];
    uint32_t sorted[MAXPAIRS];       // batch particle index of the A side | B side << 16
    uint32_t hist[FD_NLVL + 2];
    uint32_t off[FD_NLVL + 2];
    uint32_t cur[FD_NLVL + 2];
    uint32_t eoff[FD_MAXTASKS + 1];  // pair-entry offsets of the workgroup's tasks
    uint32_t poff[FD_MAXTASKS + 1];  // particle-list offsets of the workgroup's tasks
    int maxlv;
};

constexpr uint64_t POS_MASK = (1ull << 25) - 1ull;

// One launch per phase; one wave per workgroup; the workgroup's tasks are
// [blockIdx * tpw, +tpw) (tpw <= 64), applied in batches that fit in LDS
// (normally one).  A batch's particles and pair entries are contiguous in
// the schedule written by the scheduling pass.
template <int MAXP, int MAXPAIRS>
__global__ __launch_bounds__(64) void k_fd_phase(const DevParams *__restrict__ Pp, FdPhase ph,
                                                 const double *__restrict__ q, double *p,
                                                 double *eps, const double *__restrict__ rho,
                                                 const uint32_t *__restrict__ id,
                                                 const uint32_t *__restrict__ pair_off,
                                                 const uint32_t *__restrict__ part_off,
                                                 const uint64_t *__restrict__ pairs,
                                                 const uint32_t *__restrict__ part_list,
                                                 uint32_t pair_cap, uint32_t part_cap,
                                                 uint32_t step, double dt,
                                                 unsigned long long *counters, uint32_t *err)
{
    __shared__ FdShared<MAXP, MAXPAIRS> S;
    constexpr int EPL = MAXPAIRS / 64;   // pair entries per lane in one load pass
    const DevParams &P = *Pp;
    const int lane = threadIdx.x;
    const int64_t n = P.n;
    const int64_t t0 = (int64_t)blockIdx.x * ph.tasks_per_wg;
    const int R = (int)(t0 + ph.tasks_per_wg < ph.ntasks ? ph.tasks_per_wg : ph.ntasks - t0);
    const int64_t T0 = ph.task_base + t0;
    FdCount cnt = {0u, 0u, 0u, 0u, 0u};
    bool negeps = false;

    // offsets of the range's tasks (R + 1 values) and of the phase
    if (lane < R) {
        S.eoff[lane] = pair_off[T0 + lane];
        S.poff[lane] = part_off[T0 + lane];
    }
    if (lane == 0) {   // end of the range (R may be 64)
        S.eoff[R] = pair_off[T0 + R];
        S.poff[R] = part_off[T0 + R];
    }
    const uint32_t phase_p0 = part_off[ph.task_base];
    __syncthreads();
    if (S.eoff[R] > pair_cap || S.poff[R] > part_cap) {   // schedule incomplete
        if (lane == 0) atomicOr(err, ERR_PAIRCAP);
        return;
    }

    int k = 0;
    while (k < R) {
        // ---- a batch of consecutive tasks that fits (LDS reads only)
        const int k0 = k;
        bool oversized = false;
        while (k < R) {
            const int c = (int)(S.eoff[k + 1] - S.eoff[k]);
            const int np_new = (int)(S.poff[k + 1] - S.poff[k0]);
            const int npr_new = (int)(S.eoff[k + 1] - S.eoff[k0]);
            if (k > k0 && c > 0 && (np_new > MAXP || npr_new > MAXPAIRS)) break;
            oversized = c > MAXPAIRS;   // only possible as the first task of a batch
            ++k;
            if (oversized) break;
        }
        const uint32_t e_begin = S.eoff[k0], p_begin = S.poff[k0];
        const int npr = (int)(S.eoff[k] - e_begin), np = (int)(S.poff[k] - p_begin);
        if (npr == 0) continue;
        const uint32_t rel0 = p_begin - phase_p0;   // list position of batch particle 0
        // ---- stage the particles that take part in a pair: list entries
        //      first (one round-trip), then all state loads
        {
            constexpr int PPL = (MAXP + 63) / 64;
            uint32_t gl[PPL];
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                const int l = r * 64 + lane;
                gl[r] = l < np ? part_list[p_begin + l] : 0u;
            }
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                const int l = r * 64 + lane;
                if (l < np) {
                    const int64_t g = gl[r];
                    S.gidx[l] = (uint32_t)g;
                    S.q[0][l] = q[g];
                    S.q[1][l] = q[n + g];
                    S.q[2][l] = q[2 * n + g];
                    S.p[0][l] = p[g];
                    S.p[1][l] = p[n + g];
                    S.p[2][l] = p[2 * n + g];
                    S.eps[l] = eps[g];
                    S.rho[l] = rho[g];
                    S.id[l] = id[g];
                }
            }
        }
        // ---- windows of levels (one window unless a single task overflows
        //      the LDS pair list; then consecutive level ranges that fit)
        int lo = 1;
        while (lo <= FD_NLVL) {
            int hi = FD_NLVL;
            S.hist[lane + 1] = 0u;
            if (lane == 0) S.maxlv = 0;
            __syncthreads();
            if (oversized) {
                for (int e = lane; e < npr; e += 64) {
                    const int lv = (int)(pairs[e_begin + e] >> 50);
                    if (lv >= 1 && lv <= FD_NLVL) atomicAdd(&S.hist[lv], 1u);
                }
                __syncthreads();
                int acc = 0;
                for (hi = lo; hi <= FD_NLVL; ++hi) {
                    if (acc + (int)S.hist[hi] > MAXPAIRS) break;
                    acc += (int)S.hist[hi];
                }
                --hi;
                hi = hi < lo ? lo : hi;   // one level (<= 64 pairs) always fits
                __syncthreads();
                S.hist[lane + 1] = 0u;
                __syncthreads();
            }
            // counting sort of the batch's entries by level: histogram pass,
            // prefix, scatter pass.  Entries stay in registers (EPL per lane)
            // between the passes unless the batch needs several load passes.
            uint64_t ebuf[EPL];
            const bool one_pass = npr <= MAXPAIRS;
            for (int base = 0; base < npr; base += MAXPAIRS) {
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    const int x = base + r * 64 + lane;
                    ebuf[r] = x < npr ? pairs[e_begin + x] : 0ull;
                }
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    const int lv = (int)(ebuf[r] >> 50);
                    if (lv >= lo && lv <= hi && lv <= FD_NLVL) atomicAdd(&S.hist[lv], 1u);
                }
            }
            __syncthreads();
            {   // exclusive prefix over levels: lane x holds level x + 1
                const uint32_t h = S.hist[lane + 1];
                uint32_t incl = h;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t v = (uint32_t)__shfl_up((int)incl, off);
                    if (lane >= off) incl += v;
                }
                S.off[lane + 1] = incl - h;
                S.cur[lane + 1] = incl - h;
                const uint64_t nz = __ballot(h != 0u);
                if (lane == 0) S.maxlv = nz ? 64 - __clzll(nz) : 0;
            }
            __syncthreads();
            for (int base = 0; base < npr; base += MAXPAIRS) {
                if (!one_pass) {
#pragma unroll
                    for (int r = 0; r < EPL; ++r) {
                        const int x = base + r * 64 + lane;
                        ebuf[r] = x < npr ? pairs[e_begin + x] : 0ull;
                    }
                }
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    const uint64_t e = ebuf[r];
                    const int lv = (int)(e >> 50);
                    const int li = (int)((uint32_t)(e & POS_MASK) - rel0);
                    const int lj = (int)((uint32_t)((e >> 25) & POS_MASK) - rel0);
                    if (lv >= lo && lv <= hi && lv <= FD_NLVL && li >= 0 && li < np && lj >= 0 &&
                        lj < np) {
                        const uint32_t pos = atomicAdd(&S.cur[lv], 1u);
                        if (pos < (uint32_t)MAXPAIRS) S.sorted[pos] = (uint32_t)li | ((uint32_t)lj << 16);
                    }
                }
            }
            __syncthreads();
            const int top = S.maxlv;
            for (int l = lo; l <= top; ++l) {
                const int beg = (int)S.off[l], end = beg + (int)S.hist[l];
                for (int b0 = beg; b0 < end; b0 += 64) {
                    const int e = b0 + lane;
                    if (e < end) {
                        const uint32_t pr = S.sorted[e];
                        int li = (int)(pr & 0xFFFFu), lj = (int)(pr >> 16);
                        if (S.id[li] > S.id[lj]) {
                            const int tt = li;
                            li = lj;
                            lj = tt;
                        }
                        fd_pair<MAXP>(P, step, dt, li, lj, S.q, S.p, S.eps, S.rho, S.id, cnt,
                                      negeps);
                    }
                }
                __syncthreads();
            }
            lo = hi + 1;
            if (!oversized) break;
        }
        // ---- write back momenta and energies
        for (int l = lane; l < np; l += 64) {
            const int64_t g = S.gidx[l];
            p[g] = S.p[0][l];
            p[n + g] = S.p[1][l];
            p[2 * n + g] = S.p[2][l];
            eps[g] = S.eps[l];
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
    }
}

// LDS sizes.  Phase 0: ~17 particles and ~150 pairs per cell, so about seven
// cells fill a batch; inter-cell phases: up to 2 x 64 particles per task and
// fewer pairs.  Any single task fits the particle arrays (<= 128).
constexpr int FD_INTRA_P = 192, FD_INTRA_PAIRS = 2048;
constexpr int FD_INTER_P = 384, FD_INTER_PAIRS = 1536;

int run_fd_sweep(sdpd_ctx *c, const sdpd_state *s, uint64_t step, double dt_fd)
{
    if (c->prm.fd == SDPD_FD_NONE || c->n == 0) return SDPD_OK;
    int rc = run_schedule(c);
    if (rc) return rc;
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
            ph.tasks_per_wg = c->fd_tasks[0];
            ph.task_base = 0;
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
            const int cls = (ph.d[0] != 0) + (ph.d[1] != 0) + (ph.d[2] != 0);   // 1, 2, 3
            ph.tasks_per_wg = c->fd_tasks[cls];
            ph.task_base = c->ncell + (int64_t)(phase - 1) * (c->ncell / 8);
        }
        const int64_t grid = (ph.ntasks + ph.tasks_per_wg - 1) / ph.tasks_per_wg;
        timer_begin(c, TK_FD);
        if (phase == 0)
            hipLaunchKernelGGL((k_fd_phase<FD_INTRA_P, FD_INTRA_PAIRS>), dim3((unsigned)grid),
                               dim3(64), 0, c->stream, c->dparams, ph, s->q, s->p, s->eps, s->rho,
                               s->id, c->pair_off, c->part_off, c->pairs, c->part_list,
                               (uint32_t)c->pair_cap, (uint32_t)c->part_cap, (uint32_t)step,
                               dt_fd, c->counters, c->err);
        else
            hipLaunchKernelGGL((k_fd_phase<FD_INTER_P, FD_INTER_PAIRS>), dim3((unsigned)grid),
                               dim3(64), 0, c->stream, c->dparams, ph, s->q, s->p, s->eps, s->rho,
                               s->id, c->pair_off, c->part_off, c->pairs, c->part_list,
                               (uint32_t)c->pair_cap, (uint32_t)c->part_cap, (uint32_t)step,
                               dt_fd, c->counters, c->err);
        timer_end(c, TK_FD);
        if ((rc = check_hip(hipGetLastError()))) return rc;
    }
    return SDPD_OK;
}

}  // namespace sdpd
