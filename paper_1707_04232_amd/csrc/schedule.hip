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
#include "fd_math.hpp"

namespace sdpd {

struct TaskCells {
    int64_t A, B;
    int slot;       // 0 = own cell, o + 1 = forward offset o
    int phase;
};

// first task of every phase: 0, ncell, ncell + ncell/8, ...
__device__ __host__ __forceinline__ int64_t phase_base(int64_t ncell, int p)
{
    return p == 0 ? 0 : ncell + (int64_t)(p - 1) * (ncell / 8);
}

__device__ __forceinline__ TaskCells task_cells(const DevParams &P, int64_t T)
{
    TaskCells r;
    if (T < P.ncell) {
        r.A = r.B = T;
        r.slot = 0;
        r.phase = 0;
        return r;
    }
    const int64_t per = P.ncell / 8;
    const int p = 1 + (int)((T - P.ncell) / per);
    const int64_t t = (T - P.ncell) % per;
    const int o = (p - 1) / 8, pi = (p - 1) % 8, k = 14 + o;
    const int hx = P.nc[0] / 2, hy = P.nc[1] / 2;
    const int tx = (int)(t % hx), ty = (int)((t / hx) % hy), tz = (int)(t / ((int64_t)hx * hy));
    const int ax = 2 * tx + (pi & 1), ay = 2 * ty + ((pi >> 1) & 1), az = 2 * tz + (pi >> 2);
    int bx = ax + k % 3 - 1, by = ay + (k / 3) % 3 - 1, bz = az + k / 9 - 1;
    bx += bx >= P.nc[0] ? -P.nc[0] : (bx < 0 ? P.nc[0] : 0);
    by += by >= P.nc[1] ? -P.nc[1] : (by < 0 ? P.nc[1] : 0);
    bz += bz >= P.nc[2] ? -P.nc[2] : (bz < 0 ? P.nc[2] : 0);
    r.A = ax + (int64_t)P.nc[0] * (ay + (int64_t)P.nc[1] * az);
    r.B = bx + (int64_t)P.nc[0] * (by + (int64_t)P.nc[1] * bz);
    r.slot = o + 1;
    r.phase = p;
    return r;
}

// pairs and participating particles of every task (one thread per task)
__global__ void k_task_count(const DevParams *__restrict__ Pp,
                             const uint32_t *__restrict__ cell_start,
                             const uint64_t *__restrict__ masks, uint32_t *tcount, uint32_t *tnp)
{
    const DevParams &P = *Pp;
    const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= (int64_t)NMASK * P.ncell) return;
    const TaskCells tc = task_cells(P, T);
    const uint32_t sA = cell_start[tc.A], nA = cell_start[tc.A + 1] - sA;
    const uint32_t nB = cell_start[tc.B + 1] - cell_start[tc.B];
    uint32_t c = 0, na = 0;
    uint64_t orb = 0;
    if (nA <= (uint32_t)P.cap && nB <= (uint32_t)P.cap) {
        for (uint32_t a = 0; a < nA; ++a) {
            const uint64_t m = masks[(int64_t)(OWN_NB + tc.slot) * P.n + sA + a];
            na += m != 0ull;
            orb |= m;
            c += (uint32_t)__popcll(tc.slot == 0 ? (m & ~((2ull << a) - 1ull)) : m);
        }
    }
    tcount[T] = c;
    tnp[T] = na + (tc.slot == 0 ? 0u : (uint32_t)__popcll(orb));
}

// levels, particle lists and pair entries: one wave per task (grid-stride)
__global__ __launch_bounds__(64) void k_schedule(const DevParams *__restrict__ Pp,
                                                 const uint32_t *__restrict__ cell_start,
                                                 const uint64_t *__restrict__ masks,
                                                 const uint32_t *__restrict__ pair_off,
                                                 const uint32_t *__restrict__ part_off,
                                                 uint64_t *pairs, uint32_t *part_list,
                                                 uint32_t pair_cap, uint32_t part_cap,
                                                 uint32_t *err)
{
    const DevParams &P = *Pp;
    const int lane = threadIdx.x;
    const int64_t ntask = (int64_t)NMASK * P.ncell;
    for (int64_t T = blockIdx.x; T < ntask; T += gridDim.x) {
        const TaskCells tc = task_cells(P, T);
        const bool intra = tc.slot == 0;
        const uint32_t sA = cell_start[tc.A], nA = cell_start[tc.A + 1] - sA;
        const uint32_t sB = cell_start[tc.B], nB = cell_start[tc.B + 1] - sB;
        const uint32_t e0 = pair_off[T], e1 = pair_off[T + 1];
        const uint32_t q0 = part_off[T], q1 = part_off[T + 1];
        if (e1 == e0) continue;
        if (nA > (uint32_t)P.cap || nB > (uint32_t)P.cap || e1 > pair_cap || q1 > part_cap) {
            if (lane == 0) atomicOr(err, ERR_PAIRCAP);
            continue;
        }
        const uint64_t mask =
            (uint32_t)lane < nA ? masks[(int64_t)(OWN_NB + tc.slot) * P.n + sA + lane] : 0ull;
        const uint64_t actA = __ballot(mask != 0ull);
        const uint64_t actB = intra ? actA : wave_or64(mask);
        const uint32_t nactA = (uint32_t)__popcll(actA);
        const uint32_t rel = q0 - part_off[phase_base(P.ncell, tc.phase)];
        // particle list
        if ((actA >> lane) & 1ull)
            part_list[q0 + __popcll(actA & ((1ull << lane) - 1ull))] = sA + (uint32_t)lane;
        if (!intra && ((actB >> lane) & 1ull))
            part_list[q0 + nactA + __popcll(actB & ((1ull << lane) - 1ull))] = sB + (uint32_t)lane;
        // list positions of this lane as A-side and as B-side particle
        const uint64_t posA = rel + (uint32_t)__popcll(actA & ((1ull << lane) - 1ull));
        const uint64_t posB = intra ? posA
                                    : rel + nactA + (uint32_t)__popcll(actB & ((1ull << lane) - 1ull));
        const uint64_t rm = xor_permute_bits(mask, (uint32_t)lane);
        uint64_t rounds = wave_or64(rm);
        int LA = 0, LB = 0;
        uint32_t pos = e0;
        while (rounds) {
            const int s = __builtin_ctzll(rounds);
            rounds &= rounds - 1;
            const int partner = lane ^ s;
            const bool act = (rm >> s) & 1ull;
            const int la = __shfl(LA, partner), lb = __shfl(LB, partner);
            const bool actB_here = __shfl((int)act, partner) != 0;
            const uint64_t pB = (uint64_t)(uint32_t)__shfl((int)(uint32_t)posB, partner);
            const bool own = intra ? (act && lane < partner) : act;
            if (intra) {
                if (act) LA = (LA > la ? LA : la) + 1;
            } else {
                if (act) LA = (LA > lb ? LA : lb) + 1;
                if (actB_here) LB = (LB > la ? LB : la) + 1;
            }
            const uint64_t bal = __ballot(own);
            if (own) {
                const uint32_t k = pos + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                pairs[k] = posA | (pB << 25) | ((uint64_t)LA << 50);
            }
            pos += (uint32_t)__popcll(bal);
        }
    }
}

int run_schedule(sdpd_ctx *c)
{
    const int64_t ntask = (int64_t)NMASK * c->ncell;
    hipLaunchKernelGGL(k_task_count, dim3((unsigned)((ntask + 255) / 256)), dim3(256), 0, c->stream,
                       c->dparams, c->cell_start, c->masks, c->task_count, c->task_np);
    int rc = check_hip(hipGetLastError());
    if (rc) return rc;
    if ((rc = run_scan(c, c->task_count, c->pair_off, ntask, c->block_sums, -1))) return rc;
    if ((rc = run_scan(c, c->task_np, c->part_off, ntask, c->block_sums, -1))) return rc;
    // one workgroup per task: many independent short tasks hide the load latency
    const int64_t grid = std::min<int64_t>(ntask, 0x7fffffffLL);
    hipLaunchKernelGGL(k_schedule, dim3((unsigned)grid), dim3(64), 0, c->stream, c->dparams,
                       c->cell_start, c->masks, c->pair_off, c->part_off, c->pairs, c->part_list,
                       (uint32_t)c->pair_cap, (uint32_t)c->part_cap, c->err);
    return check_hip(hipGetLastError());
}

}  // namespace sdpd
