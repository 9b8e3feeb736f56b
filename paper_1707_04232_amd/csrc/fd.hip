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
// task, its active pairs with their conflict level.  A workgroup (FD_WAVES
// waves) takes a range of consecutive tasks of one phase, stages in LDS the
// momenta and energies of the particles that take part in a pair, sorts the
// range's pairs by level and applies the pairs of one level (which share no
// particle) as parallel steps over its lanes.  The number of level steps of
// a batch is set by its deepest task (the longest chain of pairs that share
// a particle, in round order), not by its size.  Positions, densities and ids do
// not change during the sweep: positions and densities are packed once per
// sweep into one (x, y, z, rho) record per particle and read from global
// memory two level steps ahead of their use, which keeps the LDS footprint
// at 36 B per particle and leaves room for more resident waves.  The random
// draws of a pair depend only on (step, ids): after the level sort they are
// computed for all of the batch's pairs at full lane occupancy (which also
// orients every pair, i = smaller id) and stored in sorted order in a global
// buffer, from which the level steps prefetch them with the positions.
//
// Phases that touch disjoint cells commute.  Phase 1 + 8 o + pi touches the
// cells of parity pi (as A) and pi ^ b_o (as B = A + delta_o, b_o the parity
// bits that delta_o flips; the number of cells per axis is even, so this
// holds across the periodic boundary).  Each phase is given the level
// 1 + the largest level of the earlier phases whose parity sets intersect
// its own; the phases of one level form a group.  For the 13 forward offsets
// this gives 26 groups of 4 phases, each touching every cell exactly once;
// with phase 0, 27 groups.  The whole sweep is one persistent launch: the
// task ranges of all groups, in group order, are handed out by an atomic
// counter, and a range of group g waits only until every cell it touches
// has been released by group g - 1 (per-cell epochs), so the groups overlap
// instead of draining one launch before the next.  Every pair of phases
// whose order is exchanged touches disjoint particles, so the result equals
// the sweep in key order bit for bit.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fd_math.hpp"
#include "tasks.hpp"

namespace sdpd {

constexpr int FD_NLVL = 64;        // levels of a task are 1..64
constexpr int FD_EPL = 16;         // pair entries per lane held in registers
constexpr int FD_PPL = 8;          // particle-list entries per lane per staging pass
constexpr int FD_MAXPH = 4;        // phases per launch

struct FdLaunch {
    int nph;
    int cap_p, cap_e;                // LDS capacity: particles, pair entries
    int64_t task_base[FD_MAXPH];     // index of the phase's first task in sweep order
    int64_t ntasks[FD_MAXPH];
    int64_t tpw[FD_MAXPH];           // tasks per workgroup
    int64_t wg_end[FD_MAXPH];        // cumulative workgroup counts
};

// dynamic LDS layout: p[3][cap_p], eps[cap_p] (doubles), then gidx[cap_p],
// sorted[cap_e] and the small tables (32-bit)
__host__ __device__ inline size_t fd_lds_bytes(int cap_p, int cap_e)
{
    return (size_t)36 * cap_p + (size_t)4 * cap_e + 4 * (3 * (FD_NLVL + 2) + 2 * (FD_MAXTASKS + 1) + 2);
}

constexpr uint64_t POS_MASK = (1ull << 25) - 1ull;   // list position field of a pair entry

// read-only data of the (oriented) pair at sorted position e: batch particle
// indices from the LDS list, then the (x, y, z, rho) records of both
// particles and the stored draws; loads are issued, not waited for
__device__ __forceinline__ void fd_gather(const uint32_t *s_sorted, const uint32_t *s_gidx,
                                          const double4 *__restrict__ qrho,
                                          const double *__restrict__ draws, int e,
                                          int &li, int &lj, PairGeo &g)
{
    const uint32_t pr = s_sorted[e];
    li = (int)(pr & 0xFFFFu);
    lj = (int)(pr >> 16);
    const double4 a = qrho[s_gidx[li]], b = qrho[s_gidx[lj]];
    g.xi = a.x;
    g.yi = a.y;
    g.zi = a.z;
    g.rho_i = a.w;
    g.xj = b.x;
    g.yj = b.y;
    g.zj = b.z;
    g.rho_j = b.w;
    const double2 *d = reinterpret_cast<const double2 *>(draws) + 2 * (int64_t)e;
    const double2 d01 = d[0], d23 = d[1];
    g.G0 = d01.x;
    g.G1 = d01.y;
    g.G2 = d23.x;
    g.U = d23.y;
}

// Momenta and energies are the state that workgroups hand on to each other.
// COHERENT (the one-launch sweep): another workgroup of the same kernel, on
// any XCD, may have written them, so they are read and written with
// agent-scope atomic loads and stores (coherent across the XCDs' L2 caches,
// with no cache flush); otherwise (one launch per group) plain accesses.
template <bool COHERENT>
__device__ __forceinline__ double state_load(const double *ptr)
{
    if (COHERENT) return __hip_atomic_load(ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *ptr;
}

template <bool COHERENT>
__device__ __forceinline__ void state_store(double *ptr, double v)
{
    if (COHERENT) __hip_atomic_store(ptr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *ptr = v;
}

// Arguments every range of the sweep reads or writes.
struct FdArgs {
    const double4 *qrho;
    double *p, *eps;
    const uint32_t *id, *pair_off, *part_off;
    const uint64_t *pairs;
    const uint32_t *part_list;
    uint32_t pair_cap, part_cap;
    const uint64_t *dstep;
    double dt;
    double *draws;
    uint32_t *err;
};

// One task range: workgroup-range index b of the launch L (a range of
// consecutive tasks of one of its phases), staged, sorted, drawn and applied
// level by level.  K: 0 = general, 1 = the common case (EMS, Lucy kernel,
// zeta = 0) fixed at compile time, 2 = that case with the FP32 proposal of
// mixed precision.
// wait() is called once, before the first access to momenta and energies:
// everything before it (entries, lists, ids, positions, the draws) is fixed
// during the sweep, so the level sort and the draws of a range overlap the
// wait for its predecessors.
template <int K, bool COHERENT, bool VREG, int SPL, class Wait>
__device__ __forceinline__ void fd_range(const DevParams &P, const FdLaunch &L, int64_t b,
                                         unsigned char *lds, const FdArgs &A, FdCount &cnt,
                                         bool &negeps, Wait &wait)
{
    const double4 *__restrict__ qrho = A.qrho;
    double *p = A.p, *eps = A.eps;
    const uint32_t *__restrict__ id = A.id;
    const uint32_t *__restrict__ pair_off = A.pair_off;
    const uint32_t *__restrict__ part_off = A.part_off;
    const uint64_t *__restrict__ pairs = A.pairs;
    const uint32_t *__restrict__ part_list = A.part_list;
    const uint32_t pair_cap = A.pair_cap, part_cap = A.part_cap;
    const uint64_t *__restrict__ dstep = A.dstep;
    const double dt = A.dt;
    double *draws = A.draws;
    uint32_t *err = A.err;
    const int CP = L.cap_p, CE = L.cap_e;
    double *s_p = (double *)lds;
    double *s_eps = s_p + 3 * CP;
    uint32_t *s_gidx = (uint32_t *)(s_eps + CP);
    uint32_t *s_sorted = s_gidx + CP;                 // A-side | B-side << 16
    uint32_t *s_hist = s_sorted + CE;
    uint32_t *s_off = s_hist + (FD_NLVL + 2);
    uint32_t *s_cur = s_off + (FD_NLVL + 2);
    uint32_t *s_eoff = s_cur + (FD_NLVL + 2);        // pair-entry offsets of the range's tasks
    uint32_t *s_poff = s_eoff + (FD_MAXTASKS + 1);   // particle-list offsets
    int *s_maxlv = (int *)(s_poff + (FD_MAXTASKS + 1));
    int *s_ntot = s_maxlv + 1;                        // sorted entries of the window

    const int tid = threadIdx.x;
    const int64_t n = P.n;
    // phase of this range and its tasks
    int k_ph = 0;
    while (k_ph + 1 < L.nph && b >= L.wg_end[k_ph]) ++k_ph;
    if (k_ph > 0) b -= L.wg_end[k_ph - 1];
    const int64_t tpw = L.tpw[k_ph], ntasks = L.ntasks[k_ph], task_base = L.task_base[k_ph];
    const int64_t t0 = b * tpw;
    const int R = (int)(t0 + tpw < ntasks ? tpw : ntasks - t0);
    const int64_t T0 = task_base + t0;

    // offsets of the range's tasks (R + 1 values) and of the phase
    if (tid < R) {
        s_eoff[tid] = pair_off[T0 + tid];
        s_poff[tid] = part_off[T0 + tid];
    }
    if (tid == 0) {   // end of the range (R may be FD_THREADS)
        s_eoff[R] = pair_off[T0 + R];
        s_poff[R] = part_off[T0 + R];
    }
    const uint32_t phase_p0 = part_off[task_base];
    __syncthreads();
    if (s_eoff[R] > pair_cap || s_poff[R] > part_cap) {   // schedule incomplete
        if (tid == 0) atomicOr(err, ERR_PAIRCAP);
        return;
    }

    int k = 0;
    while (k < R) {
        // ---- a batch of consecutive tasks that fits (LDS reads only)
        const int k0 = k;
        bool oversized = false;
        while (k < R) {
            const int c = (int)(s_eoff[k + 1] - s_eoff[k]);
            const int np_new = (int)(s_poff[k + 1] - s_poff[k0]);
            const int npr_new = (int)(s_eoff[k + 1] - s_eoff[k0]);
            if (k > k0 && c > 0 && (np_new > CP || npr_new > CE)) break;
            oversized = c > CE;   // only possible as the first task of a batch
            ++k;
            if (oversized) break;
        }
        const uint32_t e_begin = s_eoff[k0], p_begin = s_poff[k0];
        const int npr = (int)(s_eoff[k] - e_begin), np = (int)(s_poff[k] - p_begin);
        if (npr == 0) continue;
        const uint32_t rel0 = p_begin - phase_p0;   // list position of batch particle 0
        // ---- global indices of the particles that take part in a pair
        for (int base = 0; base < np; base += FD_PPL * FD_THREADS) {
            uint32_t gl[FD_PPL];
#pragma unroll
            for (int r = 0; r < FD_PPL; ++r) {
                const int l = base + r * FD_THREADS + tid;
                gl[r] = l < np ? part_list[p_begin + l] : 0u;
            }
#pragma unroll
            for (int r = 0; r < FD_PPL; ++r) {
                const int l = base + r * FD_THREADS + tid;
                if (l < np) s_gidx[l] = gl[r];
            }
        }
        __syncthreads();
        bool staged = false;   // momenta and energies of the batch in LDS
        // ---- windows of levels (one window unless a single task overflows
        //      the LDS pair list; then consecutive level ranges that fit)
        int lo = 1;
        while (lo <= FD_NLVL) {
            int hi = FD_NLVL;
            if (tid < FD_NLVL) s_hist[tid + 1] = 0u;
            if (tid == 0) *s_maxlv = 0;
            __syncthreads();
            if (oversized) {
                for (int e = tid; e < npr; e += FD_THREADS) {
                    const int lv = (int)(pairs[e_begin + e] >> 50);
                    if (lv >= 1 && lv <= FD_NLVL) atomicAdd(&s_hist[lv], 1u);
                }
                __syncthreads();
                int acc = 0;
                for (hi = lo; hi <= FD_NLVL; ++hi) {
                    if (acc + (int)s_hist[hi] > CE) break;
                    acc += (int)s_hist[hi];
                }
                --hi;
                hi = hi < lo ? lo : hi;   // one level (<= 64 pairs) always fits
                __syncthreads();
                if (tid < FD_NLVL) s_hist[tid + 1] = 0u;
                __syncthreads();
            }
            // counting sort of the batch's entries by level: histogram pass,
            // prefix, scatter pass.  Entries stay in registers (FD_EPL per
            // lane) between the passes unless the batch needs several passes.
            constexpr int EP = FD_EPL * FD_THREADS;
            uint64_t ebuf[FD_EPL];
            const bool one_pass = npr <= EP;
            for (int base = 0; base < npr; base += EP) {
#pragma unroll
                for (int r = 0; r < FD_EPL; ++r) {
                    const int x = base + r * FD_THREADS + tid;
                    ebuf[r] = x < npr ? pairs[e_begin + x] : 0ull;
                }
#pragma unroll
                for (int r = 0; r < FD_EPL; ++r) {
                    const uint64_t e = ebuf[r];
                    const int lv = (int)(e >> 50);
                    const int li = (int)((uint32_t)(e & POS_MASK) - rel0);
                    const int lj = (int)((uint32_t)((e >> 25) & POS_MASK) - rel0);
                    if (lv >= lo && lv <= hi && lv <= FD_NLVL && li >= 0 && li < np && lj >= 0 &&
                        lj < np)
                        atomicAdd(&s_hist[lv], 1u);
                }
            }
            __syncthreads();
            if (tid < 64) {   // exclusive prefix over levels (first wave): lane x holds level x + 1
                const uint32_t h = s_hist[tid + 1];
                uint32_t incl = h;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t v = (uint32_t)__shfl_up((int)incl, off);
                    if (tid >= off) incl += v;
                }
                s_off[tid + 1] = incl - h;
                s_cur[tid + 1] = incl - h;
                const uint64_t nz = __ballot(h != 0u);
                if (tid == 0) *s_maxlv = nz ? 64 - __clzll(nz) : 0;
                if (tid == 63) *s_ntot = (int)incl;
            }
            __syncthreads();
            for (int base = 0; base < npr; base += EP) {
                if (!one_pass) {
#pragma unroll
                    for (int r = 0; r < FD_EPL; ++r) {
                        const int x = base + r * FD_THREADS + tid;
                        ebuf[r] = x < npr ? pairs[e_begin + x] : 0ull;
                    }
                }
#pragma unroll
                for (int r = 0; r < FD_EPL; ++r) {
                    const uint64_t e = ebuf[r];
                    const int lv = (int)(e >> 50);
                    const int li = (int)((uint32_t)(e & POS_MASK) - rel0);
                    const int lj = (int)((uint32_t)((e >> 25) & POS_MASK) - rel0);
                    if (lv >= lo && lv <= hi && lv <= FD_NLVL && li >= 0 && li < np && lj >= 0 &&
                        lj < np) {
                        const uint32_t pos = atomicAdd(&s_cur[lv], 1u);
                        if (pos < (uint32_t)CE) s_sorted[pos] = (uint32_t)li | ((uint32_t)lj << 16);
                    }
                }
            }
            __syncthreads();
            // draws of the window's pairs in sorted order, all lanes busy; the
            // ids also orient each entry (A side = smaller id)
            {
                const uint32_t step = (uint32_t)*dstep;   // step index of the Philox counter
                const int ntot = min(*s_ntot, CE);
                double *wdraws = draws + 4 * (int64_t)e_begin;
                constexpr int DPL = 4;   // entries per lane per pass: id loads in flight
                for (int base = 0; base < ntot; base += DPL * FD_THREADS) {
                    uint32_t pr[DPL], ida[DPL], idb[DPL];
#pragma unroll
                    for (int r = 0; r < DPL; ++r) {
                        const int e = base + r * FD_THREADS + tid;
                        pr[r] = e < ntot ? s_sorted[e] : 0u;
                        ida[r] = e < ntot ? id[s_gidx[pr[r] & 0xFFFFu]] : 0u;
                        idb[r] = e < ntot ? id[s_gidx[pr[r] >> 16]] : 0u;
                    }
#pragma unroll
                    for (int r = 0; r < DPL; ++r) {
                        const int e = base + r * FD_THREADS + tid;
                        if (e < ntot) {
                            uint32_t i0 = ida[r], i1 = idb[r];
                            if (i0 > i1) {
                                s_sorted[e] = (pr[r] >> 16) | (pr[r] << 16);
                                const uint32_t t = i0;
                                i0 = i1;
                                i1 = t;
                            }
                            double d[4];
                            if (K == 2)   // mixed precision: FP32 Box-Muller
                                pair_draws_f32(P, step, i0, i1, d);
                            else
                                pair_draws_stored(P, step, i0, i1, d);
                            double2 *dst = reinterpret_cast<double2 *>(wdraws) + 2 * (int64_t)e;
                            dst[0] = make_double2(d[0], d[1]);
                            dst[1] = make_double2(d[2], d[3]);
                        }
                    }
                }
            }
            __syncthreads();
            if (!staged) {
                // ---- stage momenta and energies (after the wait for the
                //      range's predecessors, on the first batch)
                wait();
                for (int base = 0; base < np; base += FD_PPL * FD_THREADS) {
                    // SPL > 0: the loads of SPL particles issued before their
                    // LDS writes (an LDS write between two atomic loads makes
                    // the second wait for the first; plain loads the
                    // compiler reorders by itself, SPL = 0)
                    constexpr int SPB = SPL > 0 ? SPL : 1;
#pragma unroll
                    for (int r0 = 0; r0 < FD_PPL; r0 += SPB) {
                        if (SPL == 0) {
                            const int l = base + r0 * FD_THREADS + tid;
                            if (l < np) {
                                const int64_t g = s_gidx[l];
                                s_p[l] = state_load<COHERENT>(p + g);
                                s_p[CP + l] = state_load<COHERENT>(p + n + g);
                                s_p[2 * CP + l] = state_load<COHERENT>(p + 2 * n + g);
                                s_eps[l] = state_load<COHERENT>(eps + g);
                            }
                            continue;
                        }
                        double v[SPB][4];
#pragma unroll
                        for (int r = 0; r < SPB; ++r) {
                            const int l = base + (r0 + r) * FD_THREADS + tid;
                            if (l < np) {
                                const int64_t g = s_gidx[l];
                                v[r][0] = state_load<COHERENT>(p + g);
                                v[r][1] = state_load<COHERENT>(p + n + g);
                                v[r][2] = state_load<COHERENT>(p + 2 * n + g);
                                v[r][3] = state_load<COHERENT>(eps + g);
                            }
                        }
#pragma unroll
                        for (int r = 0; r < SPB; ++r) {
                            const int l = base + (r0 + r) * FD_THREADS + tid;
                            if (l < np) {
                                s_p[l] = v[r][0];
                                s_p[CP + l] = v[r][1];
                                s_p[2 * CP + l] = v[r][2];
                                s_eps[l] = v[r][3];
                            }
                        }
                    }
                }
                staged = true;
                __syncthreads();
            }
            // level steps: (level, first sorted position) in ascending order;
            // the read-only data of steps k + 1 and k + 2 is in flight while
            // step k runs (the gathers only read LDS entries fixed above)
            const int top = *s_maxlv;
            const double *wdr = draws + 4 * (int64_t)e_begin;
            // the step after (l, b): next FD_THREADS entries of level l, else
            // the first entry of the next non-empty level (l > top: none)
            auto advance = [&](int &l, int &b) {
                b += FD_THREADS;
                while (l <= top && b >= (int)(s_off[l] + s_hist[l])) {
                    ++l;
                    if (l <= top) b = (int)s_off[l];
                }
            };
            auto fetch = [&](int l, int b, int &li, int &lj, PairGeo &g) {
                bool v = false;
                if (l <= top) {
                    const int e = b + tid;
                    v = e < (int)(s_off[l] + s_hist[l]);
                    if (v) fd_gather(s_sorted, s_gidx, qrho, wdr, e, li, lj, g);
                }
                return v;
            };
            // the constants the pair update reads are held in vector registers
            // for the level loop where they fit (VREG: the one-box kernels of
            // the common case); otherwise they stay scalar loads from P
            PairRegs pr;
            if (VREG) {
                for (int a = 0; a < 3; ++a) {
                    pr.box[a] = P.box[a];
                    pr.half_box[a] = P.half_box[a];
                    __asm__ volatile("" : "+v"(pr.box[a]), "+v"(pr.half_box[a]));
                }
                pr.inv_Cv = P.inv_Cv;
                pr.kB = P.kB;
                pr.two_over_Cv = P.two_over_Cv;
                pr.inv_m = P.inv_m;
                pr.b2_c = P.b2_c;
                pr.kperp_c = P.kperp_c;
                pr.cF = P.cF;
                __asm__ volatile("" : "+v"(pr.inv_Cv), "+v"(pr.kB), "+v"(pr.two_over_Cv),
                                 "+v"(pr.inv_m), "+v"(pr.b2_c), "+v"(pr.kperp_c), "+v"(pr.cF));
            }
            int l0 = lo, b0 = (int)s_off[lo] - FD_THREADS;
            advance(l0, b0);
            int l1 = l0, b1 = b0;
            advance(l1, b1);
            PairGeo g0 = {}, g1 = {};
            int li0 = 0, lj0 = 0, li1 = 0, lj1 = 0;
            bool v0 = fetch(l0, b0, li0, lj0, g0);
            bool v1 = fetch(l1, b1, li1, lj1, g1);
            while (l0 <= top) {
                int l2 = l1, b2 = b1;
                advance(l2, b2);
                PairGeo g2 = {};
                int li2 = 0, lj2 = 0;
                const bool v2 = fetch(l2, b2, li2, lj2, g2);
                if (v0) {
                    if (VREG)
                        fd_pair<K != 0, K == 2>(P, pr, dt, li0, lj0, g0, s_p, CP, s_eps, cnt, negeps);
                    else
                        fd_pair<K != 0, K == 2>(P, P, dt, li0, lj0, g0, s_p, CP, s_eps, cnt, negeps);
                }
                __syncthreads();
                g0 = g1;
                li0 = li1;
                lj0 = lj1;
                v0 = v1;
                l0 = l1;
                g1 = g2;
                li1 = li2;
                lj1 = lj2;
                v1 = v2;
                l1 = l2;
                b1 = b2;
            }
            lo = hi + 1;
            if (!oversized) break;
        }
        // ---- write back momenta and energies
        for (int l = tid; staged && l < np; l += FD_THREADS) {
            const int64_t g = s_gidx[l];
            state_store<COHERENT>(p + g, s_p[l]);
            state_store<COHERENT>(p + n + g, s_p[CP + l]);
            state_store<COHERENT>(p + 2 * n + g, s_p[2 * CP + l]);
            state_store<COHERENT>(eps + g, s_eps[l]);
        }
        __syncthreads();
    }
}

// counters of a workgroup: one atomic per counter
__device__ __forceinline__ void fd_flush_counters(const FdCount &cnt, bool negeps,
                                                  unsigned long long *counters, uint32_t *err)
{
    const int lane = threadIdx.x & 63;   // one flush per wave
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

// one launch per group: workgroup b applies range b of L
struct FdPhaseArgs {
    const DevParams *Pp;
    FdLaunch L;
    FdArgs A;
    unsigned long long *counters;
};
template <int K>
__device__ __forceinline__ void fd_phase_body(const FdPhaseArgs &a, uint32_t blk)
{
    extern __shared__ __align__(16) unsigned char lds[];
    FdCount cnt = {0u, 0u, 0u, 0u, 0u};
    bool negeps = false;
    auto no_wait = [] {};
    fd_range<K, false, K != 0, 0>(*a.Pp, a.L, (int64_t)blk, lds, a.A, cnt, negeps, no_wait);
    fd_flush_counters(cnt, negeps, a.counters, a.A.err);
}
template <int K>
__global__ __launch_bounds__(FD_THREADS) void k_fd_phase(FdPhaseArgs a)
{
    fd_phase_body<K>(a, blockIdx.x);
}
SDPD_MULTI_KERNEL(k_fd_phase_gen_multi, FdPhaseArgs, fd_phase_body<0>, FD_THREADS)
SDPD_MULTI_KERNEL(k_fd_phase_fast_multi, FdPhaseArgs, fd_phase_body<1>, FD_THREADS)
SDPD_MULTI_KERNEL(k_fd_phase_mix_multi, FdPhaseArgs, fd_phase_body<2>, FD_THREADS)

// The whole sweep in one launch.  Its ranges, group by group (group 0 =
// phase 0, then the groups of mutually disjoint phases; inside a group in
// the order of `order`), are handed out by an atomic counter, so a range is
// only taken by a running workgroup and every range it waits for was taken
// before it.  Every group touches every
// cell exactly once, so epoch[c] = the number of groups done on cell c: a
// range of group g waits until its cells have epoch g, and sets them to
// g + 1 once its momenta and energies are written (stores completed first).
// A wait normally lasts microseconds, but when many queues share the GPU a
// workgroup holding a needed range can be descheduled for a long time (tens
// of milliseconds were measured with 32 queues), so the wait is bounded in
// time, not in polls: after kWaitTicks of the constant 100 MHz clock it
// reports ERR_STALL and goes on, so every workgroup ends.
constexpr int FD_MAXGROUPS = 32;
struct FdSweep {
    int ngroups;
    uint32_t nitems;
    uint32_t group_end[FD_MAXGROUPS];   // cumulative ranges per group
    FdLaunch launch[FD_MAXGROUPS];
};
constexpr uint64_t kWaitTicks = 20ull * 100000000ull;   // 20 s

// One range of the one-launch sweep: range b of group g, waiting until the
// cells of its tasks have epoch g and setting them to g + 1 afterwards.
template <int K, bool VREG, int SPL>
__device__ __forceinline__ void fd_flow_range(const DevParams &P, const FdLaunch &L, int g,
                                              int64_t b, const FdArgs &A, uint32_t *epoch,
                                              unsigned char *lds, FdCount &cnt, bool &negeps)
{
    const int tid = threadIdx.x;
    // the range's tasks (as fd_range finds them)
    int k_ph = 0;
    while (k_ph + 1 < L.nph && b >= L.wg_end[k_ph]) ++k_ph;
    const int64_t bl = k_ph > 0 ? b - L.wg_end[k_ph - 1] : b;
    const int64_t tpw = L.tpw[k_ph], ntasks = L.ntasks[k_ph];
    const int64_t t0 = bl * tpw;
    const int R = (int)(t0 + tpw < ntasks ? tpw : ntasks - t0);
    const int64_t T0 = L.task_base[k_ph] + t0;
    int64_t cA = -1, cB = -1;
    if (tid < R) {
        const TaskCells tc = task_cells(P, T0 + tid);
        cA = tc.A;
        cB = tc.slot == 0 ? -1 : tc.B;
    }
    bool waited = false;
    auto wait = [&] {
        if (waited) return;
        waited = true;
        if (g > 0) {   // each wave polls the cells of its lanes' tasks
            bool ready = tid >= R;
            const uint64_t t_wait = wall_clock64();
            for (;;) {
                if (!ready) {
                    const uint32_t ea = __hip_atomic_load(epoch + cA, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t eb =
                        cB < 0 ? (uint32_t)g
                               : __hip_atomic_load(epoch + cB, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    ready = ea >= (uint32_t)g && eb >= (uint32_t)g;
                }
                if (__ballot(!ready) == 0ull) break;
                if (wall_clock64() - t_wait > kWaitTicks) {
                    if ((tid & 63) == 0) atomicOr(A.err, ERR_STALL);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        // every wave has seen its cells released; no state access of the
        // range moves above the wait (the state loads are themselves
        // coherent, so no cache invalidation is needed)
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    fd_range<K, true, VREG, SPL>(P, L, b, lds, A, cnt, negeps, wait);
    // a range without pairs still orders its cells behind the predecessors
    wait();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);   // this wave's state stores have completed
    __syncthreads();                 // ... and those of the other waves
    if (tid < R) {
        __hip_atomic_store(epoch + cA, (uint32_t)g + 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (cB >= 0)
            __hip_atomic_store(epoch + cB, (uint32_t)g + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int K>
__global__ __launch_bounds__(FD_THREADS) void k_fd_sweep(const DevParams *__restrict__ Pp,
                                                 const FdSweep *__restrict__ SW,
                                                 const uint32_t *__restrict__ order, FdArgs A,
                                                 uint32_t *work, uint32_t *epoch,
                                                 unsigned long long *counters)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ uint32_t s_item;
    const DevParams &P = *Pp;
    const int tid = threadIdx.x;
    FdCount cnt = {0u, 0u, 0u, 0u, 0u};
    bool negeps = false;
    const uint32_t nitems = SW->nitems;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(work, 1u);
        __syncthreads();
        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        if (it >= nitems) break;
        int g = 0;
        while (it >= SW->group_end[g]) ++g;
        // range index within group g
        // batched state loads; the constants held in vector registers too
        // where both fit in 256 VGPRs (the FP32-proposal kernel, K = 2)
        fd_flow_range<K, K == 2, 2>(P, SW->launch[g], g, order[it], A, epoch, lds, cnt, negeps);
    }
    fd_flush_counters(cnt, negeps, counters, A.err);
}

// The one-launch sweep of many boxes (batched replicas, fused layout): the
// ranges of every box, group by group (all boxes' ranges of group 0, then of
// group 1, ...; a box's ranges of one group in its own order), handed out by
// one counter.  A range waits only on ranges of the previous group of its own
// box, all handed out before it, so the argument of the one-box sweep holds.
// While one box waits on its chain of groups the other boxes' ranges run.
struct FdBoxDesc {
    const DevParams *Pp;
    const FdSweep *SW;
    const uint32_t *order;
    FdArgs A;
    uint32_t *epoch;
    unsigned long long *counters;
};

// item_off[g * (nbox + 1) + b]: the first item of box b in group g; entry
// nbox of a row is the first item of the next group (nitems for the last)
template <int K>
__global__ __launch_bounds__(FD_THREADS) void k_fd_sweep_boxes(const FdBoxDesc *__restrict__ boxes,
                                                       const uint32_t *__restrict__ item_off,
                                                       int nbox, int ngroups, uint32_t nitems,
                                                       uint32_t *work)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(work, 1u);
        __syncthreads();
        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        if (it >= nitems) break;
        int g = 0;
        while (g + 1 < ngroups && it >= item_off[(int64_t)(g + 1) * (nbox + 1)]) ++g;
        const uint32_t *row = item_off + (int64_t)g * (nbox + 1);
        int lo = 0, hi = nbox;   // row[lo] <= it < row[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (it >= row[mid]) lo = mid;
            else hi = mid;
        }
        // box and group are the same in every lane: say so, so that the
        // descriptor and the box's parameters are read as scalars
        lo = __builtin_amdgcn_readfirstlane(lo);
        g = __builtin_amdgcn_readfirstlane(g);
        const FdBoxDesc &D = boxes[lo];
        const uint32_t gbeg = g > 0 ? D.SW->group_end[g - 1] : 0u;
        FdCount cnt = {0u, 0u, 0u, 0u, 0u};
        bool negeps = false;
        fd_flow_range<K, false, 0>(*D.Pp, D.SW->launch[g], g, D.order[gbeg + (it - row[lo])], D.A, D.epoch,
                         lds, cnt, negeps);
        fd_flush_counters(cnt, negeps, D.counters, D.A.err);
    }
}

// ---------------------------------------------------------------- host side

namespace {

// class of a phase: 0 = own cell, else the number of non-zero components of
// its offset; parity set: the cell parities the phase touches
struct PhaseGeom {
    int cls;
    unsigned parity_set;
};

PhaseGeom phase_geom(int phase)
{
    PhaseGeom g;
    if (phase == 0) {
        g.cls = 0;
        g.parity_set = 0xFFu;
        return g;
    }
    const int o = (phase - 1) / 8, pi = (phase - 1) % 8, k = 14 + o;
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
    const int b = (dx & 1) | ((dy & 1) << 1) | ((dz & 1) << 2);
    g.cls = (dx != 0) + (dy != 0) + (dz != 0);
    g.parity_set = (1u << pi) | (1u << (pi ^ b));
    return g;
}

// per-task staging allowance at 17.5 particles per cell: mean participants
// and pair entries per task, and their spread (standard deviation per task),
// measured on jittered lattices; then a headroom factor on both capacities.
// The own-cell phase gains from room for the heavy ranges (lattice cells of
// 27 particles) while it stays under the LDS share of a workgroup at two
// waves per SIMD (20 KB on a 160 KB CU).
struct Allow {
    double mp, sp, me, se, room;
};
constexpr Allow kAllow[4] = {
    {17.5, 5.5, 143.0, 50.0, 1.25},   // own cell
    {26.2, 10.0, 102.0, 59.0, 1.0},   // face
    {14.7, 10.0, 25.2, 20.0, 1.0},    // edge
    {6.7, 5.0, 5.4, 4.5, 1.0},        // corner
};
constexpr int kDefaultTasks[4] = {8 * FD_WAVES, 8 * FD_WAVES, 16 * FD_WAVES, 24 * FD_WAVES};

int round_up(double x, int q)
{
    return (int)((std::ceil(x) + q - 1) / q) * q;
}

}  // namespace

void fd_class_caps(const sdpd_ctx *c, int k, int t, int &cp, int &ce)
{
    const double s = c->ncell > 0 ? ((double)c->n / (double)c->ncell) / 17.5 : 1.0;
    // within the LDS share of two waves per SIMD: boxes with dense cells
    // (small boxes have up to ~34 particles per cell) would otherwise take
    // tens of KB per workgroup and leave the CU a few workgroups
    const int lim = std::min(std::min(c->max_lds, 65536), c->lds_share);
    const double st = std::sqrt((double)t);
    const double room = kAllow[k].room;
    cp = round_up((t * kAllow[k].mp + 4.0 * st * kAllow[k].sp) * s * room, 16);
    ce = round_up((t * kAllow[k].me + 4.0 * st * kAllow[k].se) * s * s * room, 64);
    cp = std::min(std::max(cp, 128), 65535);
    ce = std::max(ce, 64);
    // shrink to the LDS limit, keeping the particle / pair proportion
    while (fd_lds_bytes(cp, ce) > (size_t)lim && (cp > 128 || ce > 64)) {
        cp = std::max(128, cp * 7 / 8);
        ce = std::max(64, ce * 7 / 8);
    }
}

void fd_default_tuning(sdpd_ctx *c)
{
    for (int k = 0; k < 4; ++k) {
        int cp, ce;
        fd_class_caps(c, k, kDefaultTasks[k], cp, ce);
        c->tuning.fd_tasks[k] = kDefaultTasks[k];
        c->tuning.fd_lds_particles[k] = cp;
        c->tuning.fd_lds_pairs[k] = ce;
    }
    if (c->max_lds > 65536) {
        // allow dynamic LDS beyond 64 KiB where the device has it
        const void *kerns[] = {(const void *)k_fd_phase<0>, (const void *)k_fd_phase<1>,
                               (const void *)k_fd_phase<2>, (const void *)k_fd_sweep<0>,
                               (const void *)k_fd_sweep<1>, (const void *)k_fd_sweep<2>,
                               (const void *)k_fd_phase_gen_multi,
                               (const void *)k_fd_phase_fast_multi,
                               (const void *)k_fd_phase_mix_multi};
        bool ok = true;
        for (const void *k : kerns)
            ok = ok && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           c->max_lds) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            c->max_lds = 65536;
        }
    }
}

int fd_check_tuning(const sdpd_ctx *c, const sdpd_tuning *t)
{
    for (int k = 0; k < 4; ++k) {
        if (t->fd_tasks[k] < 1 || t->fd_tasks[k] > FD_MAXTASKS) return SDPD_EINVAL;
        if (t->fd_lds_particles[k] < 128 || t->fd_lds_particles[k] > 65535) return SDPD_EINVAL;
        if (t->fd_lds_pairs[k] < 64 || t->fd_lds_pairs[k] > (1 << 24)) return SDPD_EINVAL;
        if (fd_lds_bytes(t->fd_lds_particles[k], t->fd_lds_pairs[k]) > (size_t)c->max_lds)
            return SDPD_EINVAL;
    }
    return SDPD_OK;
}

// the launches of a sweep: phase 0, then each phase gets the level 1 + the
// largest level of the earlier phases whose parity sets intersect its own,
// and the phases of one level run together (at most FD_MAXPH per launch)
static std::vector<std::vector<int>> fd_groups()
{
    std::vector<std::vector<int>> groups(1, std::vector<int>(1, 0));
    int lvl[105];
    unsigned set[105];
    int maxl = 0;
    for (int p = 1; p <= 104; ++p) {
        set[p] = phase_geom(p).parity_set;
        lvl[p] = 1;
        for (int r = 1; r < p; ++r)
            if ((set[r] & set[p]) && lvl[r] + 1 > lvl[p]) lvl[p] = lvl[r] + 1;
        maxl = std::max(maxl, lvl[p]);
    }
    for (int l = 1; l <= maxl; ++l) {
        std::vector<int> g;
        for (int p = 1; p <= 104; ++p) {
            if (lvl[p] != l) continue;
            g.push_back(p);
            if ((int)g.size() == FD_MAXPH) {
                groups.push_back(g);
                g.clear();
            }
        }
        if (!g.empty()) groups.push_back(g);
    }
    return groups;
}

// workgroup ranges of one launch over the tasks of up to FD_MAXPH mutually
// disjoint phases; returns the number of ranges
static int64_t fd_launch_geometry(const sdpd_ctx *c, const int *phases, int nph, FdLaunch &L)
{
    L.nph = nph;
    L.cap_p = 0;
    L.cap_e = 0;
    int64_t wg = 0;
    for (int k = 0; k < FD_MAXPH; ++k) {
        L.task_base[k] = L.ntasks[k] = L.wg_end[k] = 0;
        L.tpw[k] = 1;
    }
    for (int k = 0; k < nph; ++k) {
        const int ph = phases[k];
        const int cls = phase_geom(ph).cls;
        L.task_base[k] = ph == 0 ? 0 : c->ncell + (int64_t)(ph - 1) * (c->ncell / 8);
        L.ntasks[k] = ph == 0 ? c->ncell : c->ncell / 8;
        L.tpw[k] = c->tuning.fd_tasks[cls];
        wg += (L.ntasks[k] + L.tpw[k] - 1) / L.tpw[k];
        L.wg_end[k] = wg;
        L.cap_p = std::max(L.cap_p, (int)c->tuning.fd_lds_particles[cls]);
        L.cap_e = std::max(L.cap_e, (int)c->tuning.fd_lds_pairs[cls]);
    }
    return wg;
}

static bool fd_fast(const sdpd_ctx *c)
{
    return c->dp.fd == SDPD_FD_EMS && c->dp.kernel == SDPD_KERNEL_LUCY && c->dp.par_twice_perp;
}

// kernel variant: 0 general, 1 the common case, 2 the common case with the
// FP32 proposal (mixed precision; other schemes keep the FP64 update)
static int fd_kind(const sdpd_ctx *c)
{
    return fd_fast(c) ? (c->dp.mixed ? 2 : 1) : 0;
}

static FdArgs fd_args(const sdpd_ctx *c, const sdpd_state *s, double dt_fd)
{
    FdArgs A;
    A.qrho = reinterpret_cast<const double4 *>(c->q4);
    A.p = s->p;
    A.eps = s->eps;
    A.id = s->id;
    A.pair_off = c->pair_off;
    A.part_off = c->part_off;
    A.pairs = c->pairs;
    A.part_list = c->part_list;
    A.pair_cap = (uint32_t)c->pair_cap;
    A.part_cap = (uint32_t)c->part_cap;
    A.dstep = c->dstep;
    A.dt = dt_fd;
    A.draws = c->draws;
    A.err = c->err;
    return A;
}

// Table of the sweep kernel (ranges of every group, in sweep order) and its
// launch size, rebuilt whenever the tuning changes.  The epochs need every
// group to touch every cell exactly once: its phases' parity sets partition
// the 8 parities (true of the 26 groups of the 13 forward offsets; checked).
bool fd_one_launch(const sdpd_ctx *c)
{
    if (c->fd_per_group || c->sweep_mode == SDPD_SWEEP_PER_GROUP) return false;
    return c->sweep_mode == SDPD_SWEEP_ONE || c->fd_dataflow;
}

// one launch per group
static int launch_phases(sdpd_ctx *c, const sdpd_state *s, const int *phases, int nph,
                         double dt_fd)
{
    FdLaunch L;
    const int64_t wg = fd_launch_geometry(c, phases, nph, L);
    if (wg == 0) return SDPD_OK;
    if (wg > 0x7fffffffLL) return SDPD_EINVAL;
    const size_t lds = fd_lds_bytes(L.cap_p, L.cap_e);
    if (lds > (size_t)c->max_lds) return SDPD_EINVAL;
    timer_begin(c, TK_FD);
    const FdPhaseArgs args{c->dparams, L, fd_args(c, s, dt_fd), c->counters};
    const int kind = fd_kind(c);
    const int rc =
        kind == 2 ? launch_or_record(c, k_fd_phase<2>, k_fd_phase_mix_multi, (unsigned)wg,
                                     FD_THREADS, lds, args)
        : kind == 1 ? launch_or_record(c, k_fd_phase<1>, k_fd_phase_fast_multi, (unsigned)wg,
                                       FD_THREADS, lds, args)
                    : launch_or_record(c, k_fd_phase<0>, k_fd_phase_gen_multi, (unsigned)wg,
                                       FD_THREADS, lds, args);
    timer_end(c, TK_FD);
    return rc;
}

// cells of task T (the host form of task_cells); B = -1 for a phase-0 task
static void task_cells_host(const sdpd_ctx *c, int64_t T, int64_t &A, int64_t &B)
{
    const int64_t ncell = c->ncell;
    const int nx = c->dp.nc[0], ny = c->dp.nc[1], nz = c->dp.nc[2];
    if (T < ncell) {
        A = T;
        B = -1;
        return;
    }
    const int64_t per = ncell / 8, u = T - ncell;
    const int p = 1 + (int)(u / per);
    const int64_t t = u % per;
    const int o = (p - 1) / 8, pi = (p - 1) % 8, k = 14 + o;
    const int64_t hx = nx / 2, hy = ny / 2;
    const int tx = (int)(t % hx), ty = (int)((t / hx) % hy), tz = (int)(t / (hx * hy));
    const int ax = 2 * tx + (pi & 1), ay = 2 * ty + ((pi >> 1) & 1), az = 2 * tz + (pi >> 2);
    const int bx = (ax + k % 3 - 1 + nx) % nx, by = (ay + (k / 3) % 3 - 1 + ny) % ny,
              bz = (az + k / 9 - 1 + nz) % nz;
    A = ax + (int64_t)nx * (ay + (int64_t)ny * az);
    B = bx + (int64_t)nx * (by + (int64_t)ny * bz);
}

// Order of the ranges inside each group: by the latest position, in the
// hand-out order, of the ranges of the previous group they wait for (ties in
// task order), so that ranges whose cells are released first are taken first.
static std::vector<uint32_t> fd_range_order(const sdpd_ctx *c, const FdSweep &h)
{
    std::vector<uint32_t> order(h.nitems);
    std::vector<int64_t> last(c->ncell, -1);   // hand-out position of the range that last touched c
    std::vector<std::pair<int64_t, uint32_t>> keyed;
    std::vector<std::vector<int64_t>> cells;
    uint32_t begin = 0;
    for (int g = 0; g < h.ngroups; ++g) {
        const FdLaunch &L = h.launch[g];
        const uint32_t nb = h.group_end[g] - begin;
        keyed.assign(nb, std::make_pair((int64_t)-1, 0u));
        cells.assign(nb, std::vector<int64_t>());
        for (uint32_t b = 0; b < nb; ++b) {
            int k_ph = 0;
            while (k_ph + 1 < L.nph && (int64_t)b >= L.wg_end[k_ph]) ++k_ph;
            const int64_t bl = k_ph > 0 ? (int64_t)b - L.wg_end[k_ph - 1] : (int64_t)b;
            const int64_t t0 = bl * L.tpw[k_ph];
            const int64_t t1 = std::min(t0 + L.tpw[k_ph], L.ntasks[k_ph]);
            int64_t key = -1;
            for (int64_t t = t0; t < t1; ++t) {
                int64_t A, B;
                task_cells_host(c, L.task_base[k_ph] + t, A, B);
                cells[b].push_back(A);
                key = std::max(key, last[A]);
                if (B >= 0) {
                    cells[b].push_back(B);
                    key = std::max(key, last[B]);
                }
            }
            keyed[b] = std::make_pair(key, b);
        }
        std::stable_sort(keyed.begin(), keyed.end(),
                         [](const std::pair<int64_t, uint32_t> &x,
                            const std::pair<int64_t, uint32_t> &y) { return x.first < y.first; });
        for (uint32_t r = 0; r < nb; ++r) {
            const uint32_t b = keyed[r].second;
            order[begin + r] = b;
            for (int64_t cc : cells[b]) last[cc] = begin + r;
        }
        begin = h.group_end[g];
    }
    return order;
}

int fd_prepare_sweep(sdpd_ctx *c)
{
    // the table and the order are rewritten in place: no sweep may be running
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SDPD_EHIP;
    c->sweep_ok = 0;
    const std::vector<std::vector<int>> groups = fd_groups();
    if ((int)groups.size() > FD_MAXGROUPS) return SDPD_EINVAL;
    FdSweep h;
    memset(&h, 0, sizeof h);
    h.ngroups = (int)groups.size();
    int64_t total = 0;
    size_t lds = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        unsigned cover = 0;
        for (int ph : groups[g]) {
            const unsigned ps = phase_geom(ph).parity_set;
            if (cover & ps) return SDPD_EINVAL;
            cover |= ps;
        }
        if (cover != 0xFFu) return SDPD_EINVAL;
        total += fd_launch_geometry(c, groups[g].data(), (int)groups[g].size(), h.launch[g]);
        if (total > 0x7fffffffLL) return SDPD_EINVAL;
        h.group_end[g] = (uint32_t)total;
        lds = std::max(lds, fd_lds_bytes(h.launch[g].cap_p, h.launch[g].cap_e));
    }
    h.nitems = (uint32_t)total;
    if (lds > (size_t)c->max_lds) return SDPD_EINVAL;
    c->sweep_ngroups = h.ngroups;
    memcpy(c->sweep_group_end, h.group_end, sizeof h.group_end);
    if (!c->sweep && hipMalloc(&c->sweep, sizeof(FdSweep)) != hipSuccess) {
        c->sweep = nullptr;
        return SDPD_ENOMEM;
    }
    int rc = check_hip(hipMemcpy(c->sweep, &h, sizeof h, hipMemcpyHostToDevice));
    if (rc) return rc;
    const std::vector<uint32_t> order = fd_range_order(c, h);
    // one range per task at most: the buffer is sized once and never moves
    const size_t order_cap = (size_t)NMASK * (size_t)c->ncell + 1;
    if (order.size() > order_cap) return SDPD_EINVAL;
    if (!c->sweep_order &&
        hipMalloc((void **)&c->sweep_order, sizeof(uint32_t) * order_cap) != hipSuccess) {
        c->sweep_order = nullptr;
        return SDPD_ENOMEM;
    }
    if (!order.empty() &&
        (rc = check_hip(hipMemcpy(c->sweep_order, order.data(), sizeof(uint32_t) * order.size(),
                                  hipMemcpyHostToDevice))))
        return rc;
    int per_cu = 0, cus = 0;
    const int kind = fd_kind(c);
    const void *kern = kind == 2 ? (const void *)k_fd_sweep<2>
                       : kind == 1 ? (const void *)k_fd_sweep<1> : (const void *)k_fd_sweep<0>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, FD_THREADS, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess || per_cu < 1 || cus < 1) {
        (void)hipGetLastError();
        return SDPD_EHIP;
    }
    c->sweep_lds = lds;
    c->sweep_grid = (int)std::min<int64_t>((int64_t)per_cu * cus, std::max<int64_t>(total, 1));
    // one launch when the sweep holds several GPU-fulls of ranges; a small box
    // would mostly wait on its chain of 27 groups, and one launch per group
    // then wastes no workgroup slots on waiting
    c->fd_dataflow = total >= 4 * (int64_t)per_cu * cus;
    c->sweep_ok = 1;
    return SDPD_OK;
}

// (x, y, z, rho) record of every particle for the pair gathers of the sweep
struct PackArgs {
    int64_t n;
    const double *q, *rho;
    double4 *qrho;
};
__device__ __forceinline__ void pack_qrho_body(const PackArgs &a, uint32_t blk)
{
    const int64_t n = a.n;
    const double *__restrict__ q = a.q;
    const double *__restrict__ rho = a.rho;
    double4 *qrho = a.qrho;
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 r;
    r.x = q[i];
    r.y = q[n + i];
    r.z = q[2 * n + i];
    r.w = rho[i];
    qrho[i] = r;
}
__global__ void k_pack_qrho(PackArgs a) { pack_qrho_body(a, blockIdx.x); }
SDPD_MULTI_KERNEL(k_pack_qrho_multi, PackArgs, pack_qrho_body, 256)

// Schedule and packed records of a sweep (independent of the tuning), then
// its launches.
int fd_sweep_prepare(sdpd_ctx *c, const sdpd_state *s, bool packed)
{
    int rc = run_schedule(c);
    if (rc) return rc;
    if (!packed) {
        timer_begin(c, TK_SCHED);   // sweep preparation, with the schedule
        rc = launch_or_record(c, k_pack_qrho, k_pack_qrho_multi, (unsigned)((c->n + 255) / 256),
                              256, 0,
                              PackArgs{c->n, s->q, s->rho, reinterpret_cast<double4 *>(c->q4)});
        timer_end(c, TK_SCHED);
        if (rc) return rc;
    }
    c->fd_swept = 1;
    return SDPD_OK;
}

int fd_launch_sweep(sdpd_ctx *c, const sdpd_state *s, double dt_fd)
{
    if (!c->sweep_ok) return SDPD_EINVAL;
    int rc;
    if (c->rec && c->fd_record_flow) {
        // fused batch: the epochs start at zero, then the sweep is recorded
        // as this box's part of one multi-box launch
        if ((rc = launch_fill_u32(c, c->epoch, 0u, c->ncell))) return rc;
        FdBoxDesc d;
        d.Pp = c->dparams;
        d.SW = (const FdSweep *)c->sweep;
        d.order = c->sweep_order;
        d.A = fd_args(c, s, dt_fd);
        d.epoch = c->epoch;
        d.counters = c->counters;
        RecordedLaunch r;
        r.multi = nullptr;
        r.grid = 1;
        r.block = FD_THREADS;
        r.lds = c->sweep_lds;
        r.flow_kind = fd_kind(c);
        r.args.resize(sizeof d);
        memcpy(r.args.data(), &d, sizeof d);
        c->rec->push_back(std::move(r));
        return SDPD_OK;
    }
    if (!fd_one_launch(c)) {
        for (const std::vector<int> &g : fd_groups())
            if ((rc = launch_phases(c, s, g.data(), (int)g.size(), dt_fd))) return rc;
        return SDPD_OK;
    }
    // epochs of the cells and the range counter start at zero
    if ((rc = launch_fill_u32(c, c->epoch, 0u, c->ncell + 1))) return rc;
    timer_begin(c, TK_FD);
    const int kind = fd_kind(c);
    auto kern = kind == 2 ? k_fd_sweep<2> : kind == 1 ? k_fd_sweep<1> : k_fd_sweep<0>;
    hipLaunchKernelGGL(kern, dim3((unsigned)c->sweep_grid), dim3(FD_THREADS), c->sweep_lds, c->stream,
                       c->dparams, (const FdSweep *)c->sweep, c->sweep_order, fd_args(c, s, dt_fd),
                       c->epoch + c->ncell, c->epoch, c->counters);
    timer_end(c, TK_FD);
    return check_hip(hipGetLastError());
}

int fd_flow_build(const std::vector<sdpd_ctx *> &ctxs,
                  const std::vector<const RecordedLaunch *> &recs, FlowSweep &out)
{
    const int nbox = (int)ctxs.size();
    if (nbox < 1 || recs.size() != ctxs.size()) return SDPD_EINVAL;
    out.kind = recs[0]->flow_kind;
    out.nbox = nbox;
    out.ngroups = ctxs[0]->sweep_ngroups;
    std::vector<FdBoxDesc> desc(nbox);
    out.lds = 0;
    for (int b = 0; b < nbox; ++b) {
        if (recs[b]->flow_kind != out.kind || ctxs[b]->sweep_ngroups != out.ngroups ||
            recs[b]->args.size() != sizeof(FdBoxDesc))
            return SDPD_EINVAL;
        memcpy(&desc[b], recs[b]->args.data(), sizeof(FdBoxDesc));
        out.lds = std::max(out.lds, recs[b]->lds);
    }
    // group-major item numbering: all boxes' ranges of group 0, then group 1, ...
    std::vector<uint32_t> off((size_t)out.ngroups * (nbox + 1));
    uint64_t item = 0;
    for (int g = 0; g < out.ngroups; ++g)
        for (int b = 0; b <= nbox; ++b) {
            off[(size_t)g * (nbox + 1) + b] = (uint32_t)item;
            if (b < nbox) {
                const uint32_t *ge = ctxs[b]->sweep_group_end;
                item += ge[g] - (g > 0 ? ge[g - 1] : 0u);
                if (item > 0x7fffffffull) return SDPD_EINVAL;
            }
        }
    out.nitems = (uint32_t)item;
    int per_cu = 0, cus = 0;
    const void *kern = out.kind == 2 ? (const void *)k_fd_sweep_boxes<2>
                       : out.kind == 1 ? (const void *)k_fd_sweep_boxes<1>
                                       : (const void *)k_fd_sweep_boxes<0>;
    if (out.lds > 65536 &&
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)out.lds) !=
            hipSuccess)
        return SDPD_EINVAL;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, FD_THREADS, out.lds) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctxs[0]->device) !=
            hipSuccess || per_cu < 1 || cus < 1) {
        (void)hipGetLastError();
        return SDPD_EHIP;
    }
    out.grid = (unsigned)std::min<int64_t>((int64_t)per_cu * cus, std::max<int64_t>(item, 1));
    if (hipMalloc(&out.boxes, sizeof(FdBoxDesc) * nbox) != hipSuccess ||
        hipMalloc((void **)&out.item_off, sizeof(uint32_t) * off.size()) != hipSuccess ||
        hipMalloc((void **)&out.work, sizeof(uint32_t)) != hipSuccess)
        return SDPD_ENOMEM;
    int rc = check_hip(hipMemcpy(out.boxes, desc.data(), sizeof(FdBoxDesc) * nbox,
                                 hipMemcpyHostToDevice));
    if (!rc)
        rc = check_hip(hipMemcpy(out.item_off, off.data(), sizeof(uint32_t) * off.size(),
                                 hipMemcpyHostToDevice));
    return rc;
}

// counter of the multi-box sweep back to zero (a kernel, so that a captured
// graph holds no memset node)
__global__ void k_flow_reset(uint32_t *work)
{
    if (threadIdx.x == 0) *work = 0u;
}

int fd_flow_launch(const FlowSweep &f, hipStream_t stream)
{
    if (f.nitems == 0) return SDPD_OK;
    hipLaunchKernelGGL(k_flow_reset, dim3(1), dim3(64), 0, stream, f.work);
    const FdBoxDesc *boxes = (const FdBoxDesc *)f.boxes;
    if (f.kind == 2)
        hipLaunchKernelGGL(k_fd_sweep_boxes<2>, dim3(f.grid), dim3(FD_THREADS), f.lds, stream,
                           boxes, f.item_off, f.nbox, f.ngroups, f.nitems, f.work);
    else if (f.kind == 1)
        hipLaunchKernelGGL(k_fd_sweep_boxes<1>, dim3(f.grid), dim3(FD_THREADS), f.lds, stream,
                           boxes, f.item_off, f.nbox, f.ngroups, f.nitems, f.work);
    else
        hipLaunchKernelGGL(k_fd_sweep_boxes<0>, dim3(f.grid), dim3(FD_THREADS), f.lds, stream,
                           boxes, f.item_off, f.nbox, f.ngroups, f.nitems, f.work);
    return check_hip(hipGetLastError());
}

void fd_flow_free(FlowSweep &f)
{
    if (f.boxes) (void)hipFree(f.boxes);
    if (f.item_off) (void)hipFree(f.item_off);
    if (f.work) (void)hipFree(f.work);
    f.boxes = nullptr;
    f.item_off = nullptr;
    f.work = nullptr;
}

// The step index of the draws is read from c->dstep on the device (set by
// the caller, or advanced inside a captured graph).
int run_fd_sweep(sdpd_ctx *c, const sdpd_state *s, double dt_fd, bool packed)
{
    if (c->prm.fd == SDPD_FD_NONE || c->n == 0) return SDPD_OK;
    const int rc = fd_sweep_prepare(c, s, packed);
    return rc ? rc : fd_launch_sweep(c, s, dt_fd);
}

}  // namespace sdpd
