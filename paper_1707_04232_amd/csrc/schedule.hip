// Pair schedule of the fluctuation/dissipation sweep, built once per sweep
// from the active-pair masks of the density pass.
//
// Tasks are numbered in sweep order: phase 0 holds one task per cell A
// (pairs inside A); phase 1 + 8 o + pi holds one task per cell A of
// coordinate parity pi (pairs between A and A + delta_o), in the order
// tx + hx (ty + hy tz) of A = 2 (tx, ty, tz) + parity bits.  For every task
// this pass writes, contiguously in task order,
//   * the list of particles that take part in one of its pairs: the A-cell
//     ones by slot, then (inter-cell tasks) the B-cell ones by slot;
//   * its active pairs in round order (round = slot_A XOR slot_B, the
//     order that defines the sweep), each with its level: 1 + the largest
//     level among the earlier pairs of the task that share a particle.
//     Pairs of equal level in one task share no particle.
// Pair entry (64 bits): the phase-relative list positions of its two
// particles (25 bits each) and the level (bits 50..56).
#include <type_traits>

#include "fd_math.hpp"
#include "tasks.hpp"

namespace sdpd {

// pairs and participating particles of every task: one 16-lane quarter-wave
// per task (a cell holds 16 particles on average), lane x reading the masks
// of slots x, x + 16, ... of cell A, then sums and ORs over the quarter
// (all mask loads of a task in flight at once)
constexpr int COUNT_WAVES = 4;     // waves per workgroup
constexpr int COUNT_LANES = 16;    // lanes per task: four tasks per wave

struct TaskCountArgs {
    const DevParams *Pp;
    const uint32_t *cell_start;
    const uint64_t *masks;
    uint32_t *tcount, *tnp;
};
__device__ __forceinline__ void task_count_body(const TaskCountArgs &a, uint32_t blk)
{
    const DevParams &P = *a.Pp;
    const uint32_t *__restrict__ cell_start = a.cell_start;
    const uint64_t *__restrict__ masks = a.masks;
    uint32_t *tcount = a.tcount, *tnp = a.tnp;
    const int lane = threadIdx.x & 63, x = lane & (COUNT_LANES - 1);
    const int64_t T = ((int64_t)blk * COUNT_WAVES + (threadIdx.x >> 6)) * (64 / COUNT_LANES) +
                      lane / COUNT_LANES;
    const bool ok = T < (int64_t)NMASK * P.ncell;
    uint32_t c = 0, na = 0;
    uint64_t orb = 0;
    int slot = 0;
    if (ok) {
        const TaskCells tc = task_cells(P, T);
        slot = tc.slot;
        const uint32_t sA = cell_start[tc.A], nA = cell_start[tc.A + 1] - sA;
        const uint32_t nB = cell_start[tc.B + 1] - cell_start[tc.B];
        if (nA <= (uint32_t)P.cap && nB <= (uint32_t)P.cap) {
            for (uint32_t a = (uint32_t)x; a < nA; a += COUNT_LANES) {
                const uint64_t m = masks[(int64_t)(OWN_NB + tc.slot) * P.n + sA + a];
                na += m != 0ull;
                orb |= m;
                c += (uint32_t)__popcll(tc.slot == 0 ? (m & ~((2ull << a) - 1ull)) : m);
            }
        }
    }
#pragma unroll
    for (int off = COUNT_LANES / 2; off > 0; off >>= 1) {   // stays inside the quarter
        c += (uint32_t)__shfl_xor((int)c, off);
        na += (uint32_t)__shfl_xor((int)na, off);
        orb |= (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)orb, off) |
               ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(orb >> 32), off) << 32);
    }
    if (ok && x == 0) {
        tcount[T] = c;
        tnp[T] = na + (slot == 0 ? 0u : (uint32_t)__popcll(orb));
    }
}
__global__ __launch_bounds__(64 * COUNT_WAVES) void k_task_count(TaskCountArgs a)
{
    task_count_body(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_task_count_multi, TaskCountArgs, task_count_body, 64 * COUNT_WAVES)

struct TaskSpan {
    TaskCells tc;
    uint32_t sA, nA, sB, nB, e0, e1, q0, q1, rel;
};

__device__ __forceinline__ TaskSpan task_span(const DevParams &P, const uint32_t *cell_start,
                                              const uint32_t *pair_off, const uint32_t *part_off,
                                              int64_t T)
{
    TaskSpan t;
    t.tc = task_cells(P, T);
    t.sA = cell_start[t.tc.A];
    t.nA = cell_start[t.tc.A + 1] - t.sA;
    t.sB = cell_start[t.tc.B];
    t.nB = cell_start[t.tc.B + 1] - t.sB;
    t.e0 = pair_off[T];
    t.e1 = pair_off[T + 1];
    t.q0 = part_off[T];
    t.q1 = part_off[T + 1];
    t.rel = t.q0 - part_off[phase_base(P.ncell, t.tc.phase)];
    return t;
}

// OR over the lanes of one W-lane segment
template <int W>
__device__ __forceinline__ uint64_t seg_or64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, off);
        hi |= (uint32_t)__shfl_xor((int)hi, off);
    }
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// One task on a W-lane segment of the wave (W = 64: the whole wave; W = 32:
// one half, for cells of at most 32 particles, so that every slot and every
// round partner x ^ s lies in the half).  Lane x of the segment is slot x of
// cell A and of cell B.  Writes the task's particle list and its pairs in
// round order with their levels.  `ok` = this segment has a task to do;
// INTRA (a phase-0 task) is the same for the whole wave (tasks of one pair
// never mix phase 0 with the others, since ncell is even).
template <int W, bool INTRA>
__device__ __forceinline__ void schedule_segment(const DevParams &P, const TaskSpan &t, bool ok,
                                                 const uint64_t *__restrict__ masks,
                                                 uint64_t *pairs, uint32_t *part_list)
{
    constexpr bool intra = INTRA;
    using M = typename std::conditional<W == 32, uint32_t, uint64_t>::type;
    const int lane = threadIdx.x & 63;
    const int base = lane & ~(W - 1), x = lane & (W - 1);
    const bool hi = base != 0;
    const M below = (M)(((uint64_t)1 << x) - 1u);   // x < W <= 64
    const uint64_t mask64 = ok && (uint32_t)x < t.nA
                                ? masks[(int64_t)(OWN_NB + t.tc.slot) * P.n + t.sA + x] : 0ull;
    const M mask = (M)mask64;   // W = 32: partner slots < 32
    const uint64_t bact = __ballot(mask != 0);
    const M actA = (M)(hi ? (bact >> 32) : bact);
    const M actB = intra ? actA : (M)seg_or64<W>(mask);
    const uint32_t nactA = (uint32_t)__popcll(actA);
    // particle list: A-side participants by slot, then (inter-cell) B-side
    if ((actA >> x) & 1u) part_list[t.q0 + __popcll(actA & below)] = t.sA + (uint32_t)x;
    if (!intra && ((actB >> x) & 1u))
        part_list[t.q0 + nactA + __popcll(actB & below)] = t.sB + (uint32_t)x;
    // phase-relative list positions of this lane as A-side and as B-side particle
    const uint32_t posA = t.rel + (uint32_t)__popcll(actA & below);
    const uint32_t posB = intra ? posA : t.rel + nactA + (uint32_t)__popcll(actB & below);
    const M rm = (M)xor_permute_bits(mask, (uint32_t)x);   // bit s: partner x ^ s active
    uint64_t r = seg_or64<W>(rm);
    if (W == 32) r |= (uint32_t)__shfl_xor((int)(uint32_t)r, 32);   // union of the halves
    uint64_t rounds = uniform64(r);
    int LA = 0, LB = 0;
    uint32_t pos = t.e0;
    while (rounds) {
        const int s = __builtin_ctzll(rounds);   // uniform
        rounds &= rounds - 1;
        const int partner = x ^ s;                // < W
        const int addr = (base + partner) << 2;   // byte address of the partner lane
        const bool act = (rm >> s) & 1u;
        const int la = __builtin_amdgcn_ds_bpermute(addr, LA);
        const uint32_t pB = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)posB);
        bool own;
        if (INTRA) {   // one role per particle; the pair's two lanes agree on act
            own = act && x < partner;
            LA = act ? max(LA, la) + 1 : LA;
        } else {       // lane x is slot x of cell A and slot x of cell B
            const int lb = __builtin_amdgcn_ds_bpermute(addr, LB);
            const bool actB_here = __builtin_amdgcn_ds_bpermute(addr, (int)act) != 0;
            own = act;
            const int nLA = act ? max(LA, lb) + 1 : LA;
            LB = actB_here ? max(LB, la) + 1 : LB;
            LA = nLA;
        }
        const uint64_t bal = __ballot(own);
        const uint32_t blo = (uint32_t)bal, bhi = (uint32_t)(bal >> 32);
        if (own) {
            // rank among the owning lanes of this segment
            uint32_t k = __builtin_amdgcn_mbcnt_hi(bhi, __builtin_amdgcn_mbcnt_lo(blo, 0u));
            if (W == 32 && hi) k -= (uint32_t)__popc(blo);
            const uint64_t e = (uint64_t)posA | ((uint64_t)pB << 25) | ((uint64_t)LA << 50);
            pairs[pos + k] = e;
        }
        pos += W == 32 ? (uint32_t)__popc(hi ? bhi : blo) : (uint32_t)__popcll(bal);
    }
}

// levels, particle lists and pair entries (grid-stride over pairs of
// consecutive tasks; 14 * ncell is even).  Both tasks of a pair run side by
// side in the two halves of the wave when all their cells hold at most 32
// particles, otherwise one after the other on the whole wave.
constexpr int SCHED_WAVES = 4;   // waves per workgroup, each on its own task pairs

struct ScheduleArgs {
    const DevParams *Pp;
    const uint32_t *cell_start;
    const uint64_t *masks;
    const uint32_t *pair_off, *part_off;
    uint64_t *pairs;
    uint32_t *part_list;
    uint32_t pair_cap, part_cap;
    uint32_t *err;
    uint32_t nblk;   // workgroups of the box's grid-stride loop
};
__device__ __forceinline__ void schedule_body(const ScheduleArgs &a, uint32_t blk)
{
    const DevParams &P = *a.Pp;
    const uint32_t *__restrict__ cell_start = a.cell_start;
    const uint64_t *__restrict__ masks = a.masks;
    const uint32_t *__restrict__ pair_off = a.pair_off;
    const uint32_t *__restrict__ part_off = a.part_off;
    uint64_t *pairs = a.pairs;
    uint32_t *part_list = a.part_list;
    const uint32_t pair_cap = a.pair_cap, part_cap = a.part_cap;
    uint32_t *err = a.err;
    const int64_t ntask = (int64_t)NMASK * P.ncell;
    // wave index made explicitly uniform: the task arithmetic below then runs
    // on the scalar unit once per wave
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (int64_t Wp = (int64_t)blk * SCHED_WAVES + wave; 2 * Wp < ntask;
         Wp += (int64_t)a.nblk * SCHED_WAVES) {
        const TaskSpan ta = task_span(P, cell_start, pair_off, part_off, 2 * Wp);
        const TaskSpan tb = task_span(P, cell_start, pair_off, part_off, 2 * Wp + 1);
        bool oka = ta.e1 > ta.e0, okb = tb.e1 > tb.e0;
        const bool bada = oka && (ta.nA > (uint32_t)P.cap || ta.nB > (uint32_t)P.cap ||
                                  ta.e1 > pair_cap || ta.q1 > part_cap);
        const bool badb = okb && (tb.nA > (uint32_t)P.cap || tb.nB > (uint32_t)P.cap ||
                                  tb.e1 > pair_cap || tb.q1 > part_cap);
        if (bada || badb) {
            if (lane == 0) atomicOr(err, ERR_PAIRCAP);
            oka = oka && !bada;
            okb = okb && !badb;
        }
        if (!oka && !okb) continue;
        uint32_t widest = 0;
        if (oka) widest = max(ta.nA, ta.nB);
        if (okb) widest = max(widest, max(tb.nA, tb.nB));
        if (widest <= 32) {
            const bool hi = lane >= 32;
            const TaskSpan t = hi ? tb : ta;   // field-wise select
            if (ta.tc.slot == 0)   // both tasks of the pair are of one kind
                schedule_segment<32, true>(P, t, hi ? okb : oka, masks, pairs, part_list);
            else
                schedule_segment<32, false>(P, t, hi ? okb : oka, masks, pairs, part_list);
        } else {
            if (oka) {
                if (ta.tc.slot == 0) schedule_segment<64, true>(P, ta, true, masks, pairs, part_list);
                else schedule_segment<64, false>(P, ta, true, masks, pairs, part_list);
            }
            if (okb) {
                if (tb.tc.slot == 0) schedule_segment<64, true>(P, tb, true, masks, pairs, part_list);
                else schedule_segment<64, false>(P, tb, true, masks, pairs, part_list);
            }
        }
    }
}

__global__ __launch_bounds__(64 * SCHED_WAVES) void k_schedule(ScheduleArgs a)
{
    schedule_body(a, xcd_block(blockIdx.x, gridDim.x));
}
SDPD_MULTI_KERNEL(k_schedule_multi, ScheduleArgs, schedule_body, 64 * SCHED_WAVES)

int run_schedule(sdpd_ctx *c)
{
    const int64_t ntask = (int64_t)NMASK * c->ncell;
    timer_begin(c, TK_SCHED);
    const int64_t per_block = (int64_t)COUNT_WAVES * (64 / COUNT_LANES);
    const int64_t count_blocks = (ntask + per_block - 1) / per_block;
    int rc = launch_or_record(c, k_task_count, k_task_count_multi, (unsigned)count_blocks,
                              64 * COUNT_WAVES, 0,
                              TaskCountArgs{c->dparams, c->cell_start, c->masks, c->task_count,
                                            c->task_np});
    if (rc) return rc;
    if ((rc = run_scan(c, c->task_count, c->pair_off, ntask, c->block_sums, -1))) return rc;
    if ((rc = run_scan(c, c->task_np, c->part_off, ntask, c->block_sums, -1))) return rc;
    // one workgroup per pair of tasks: many independent short waves hide the
    // load latency
    const int64_t grid = std::min<int64_t>((ntask / 2 + SCHED_WAVES - 1) / SCHED_WAVES, 0x7fffffffLL);
    rc = launch_or_record(c, k_schedule, k_schedule_multi, (unsigned)grid, 64 * SCHED_WAVES, 0,
                          ScheduleArgs{c->dparams, c->cell_start, c->masks, c->pair_off,
                                       c->part_off, c->pairs, c->part_list, (uint32_t)c->pair_cap,
                                       (uint32_t)c->part_cap, c->err, (uint32_t)grid});
    timer_end(c, TK_SCHED);
    return rc;
}

}  // namespace sdpd
