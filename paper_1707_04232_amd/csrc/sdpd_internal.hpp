// Internal declarations of libsdpd (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <vector>

#include "sdpd.h"
#include "fastdiv.hpp"

namespace sdpd {

// sticky device error bits
enum : uint32_t {
    ERR_CELLCAP = 1u, ERR_NEGEPS = 2u, ERR_NONFINITE = 4u, ERR_PAIRCAP = 8u, ERR_IDS = 16u,
    ERR_STALL = 32u
};
struct AdjointWork;   // adjoint.hip

// F/D counters, in this order in the device counter array
enum { CNT_PROPOSED = 0, CNT_REJ_ENERGY, CNT_REJ_RATIO, CNT_MARGINAL, CNT_NEGEPS, CNT_N };

// tasks per cell of the F/D schedule: slot 0 = own cell, slots 1..13 = the
// 13 forward neighbour cells
constexpr int NMASK = 14;
// active-pair masks per particle: one per neighbour cell, offset index
// k = 0..26 (z slowest); k = 13 is the own cell, 14..26 the forward cells
constexpr int NNB = 27;
constexpr int OWN_NB = 13;
constexpr int MAX_CAP = 64;
// F/D sweep workgroups: FD_WAVES waves share one batch of tasks (the pairs
// of a level are split over their lanes); at most one task per lane
constexpr int FD_WAVES = 1;
constexpr int FD_THREADS = 64 * FD_WAVES;
constexpr int FD_MAXTASKS = FD_THREADS;   // tasks per workgroup range of the F/D sweep

// Everything a kernel needs, by value.  Derived constants are computed once
// on the host.
struct DevParams {
    int64_t n;
    double box[3], half_box[3], inv_cell[3];
    int nc[3];
    int64_t ncell;
    double m, inv_m, h, h2, inv_h, kB, Cv, inv_Cv, A;
    double dt;
    int kernel, fd, cap;
    uint32_t seed_lo, seed_hi, replica;
    double cW;          // W prefactor: Lucy 105/(16 pi h^3), cubic 8/(pi h^3)
    double cF;          // F prefactor: Lucy 315/(4 pi h^5), cubic 48/(pi h^5)
    double cPi;         // P/rho^2 = cPi * eps / rho, cPi = A kB / (m Cv)
    double eps_exp;     // A kB / Cv (constant-entropy exponent)
    double kpar_c;      // (10/3 eta + 4 zeta) m^2
    double kperp_c;     // (5/3 eta - zeta) m^2
    double two_over_Cv; // 1/C_i + 1/C_j
    double b2_c;        // 4 kB / m
    double ent_c;       // Cv/kB - 1
    double m_over_8, m_over_2;
    int par_twice_perp;     // kpar_c == 2 kperp_c exactly (zeta = 0)
    // mixed precision (prec == SDPD_MIXED): FP32 copies of the constants
    int mixed;
    float cell_f[3];        // cell edge lengths box / nc
    float h_f, h2_f, inv_h_f, m_f, cW_f, cF_f;
    // ... and of the F/D proposal coefficients (FP32 proposal, EMS with
    // Lucy's kernel and zeta = 0)
    float inv_Cv_f, d_c_f, inv_m_f, b2_c_f, kperp_c_f;
    // task numbering of the F/D schedule: tasks per inter-cell phase
    // (ncell / 8) and the half extents nc[0] / 2, nc[1] / 2
    FastDiv div_per, div_hx, div_hy;
};

// observable record (doubles): E, Eint, KE, P0, P1, P2, min_eps, then the
// five F/D counters stored as 64-bit integers
constexpr int REC = 12;

// kernel timing classes
enum { TK_CELLS = 0, TK_DENSITY, TK_FD, TK_FORCE, TK_OBSERVE, TK_SCHED, TK_N };

struct Timer {
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;
    size_t used = 0;
};

// ---------------------------------------------------------------- multi-box launches
// Every kernel of a step has an argument struct A, a body
// `body(const A &a, uint32_t blk)` (blk in place of blockIdx.x), a
// single-box kernel `k(A a)` and a multi-box kernel that runs, in one launch,
// workgroup blk of box w.x for every (w.x, w.y = blk) of a table: the boxes'
// argument structs are an array in device memory.  A context in recording
// mode appends its launches to a LaunchRecord instead of issuing them; the
// batch of many boxes (batch.hip) merges the boxes' records into multi-box
// launches, one per kernel and position of the step.
using MultiKernel = void (*)(const void *, const uint2 *);

struct RecordedLaunch {
    MultiKernel multi;
    unsigned grid, block;
    int flow_kind = -1;   // >= 0: a one-launch F/D sweep (args: the box's descriptor)
    size_t lds;
    std::vector<unsigned char> args;
};
using LaunchRecord = std::vector<RecordedLaunch>;

// (the table is read-only for the whole launch: restrict lets the compiler
// keep argument fields across the body's stores, as it does for kernel
// arguments)
// The chip deals workgroups to its 8 XCDs in turn (workgroup b to XCD
// b mod 8), each XCD with an L2 of its own.  xcd_block(b, n) renumbers the n
// workgroups of a grid so that each XCD takes runs of kRun consecutive
// workgroups (of every 8 kRun, the x-th run to XCD x): in cell order, the
// cells a particle pass reads around its own are then more often in the L2
// of the XCD that reads them, while the eight XCDs still work on nearby
// parts of the grid (one contiguous eighth per XCD helped a 2^20-particle box
// and hurt an 8M one, whose eight fronts no longer shared the last-level
// cache).  The trailing n mod 8 kRun workgroups keep their numbers.  A
// bijection onto [0, n) for any n (on a chip with another XCD count only the
// locality differs).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n)
{
    constexpr uint32_t kXcd = 8, kRun = 32;
    const uint32_t span = kXcd * kRun, full = n / span * span;
    if (b >= full) return b;
    const uint32_t base = b / span * span, o = b - base;
    return base + (o % kXcd) * kRun + o / kXcd;
}

#define SDPD_MULTI_KERNEL(NAME, ARGS, BODY, THREADS)                                          \
    __global__ __launch_bounds__(THREADS) void NAME(const void *__restrict__ tab,              \
                                                    const uint2 *__restrict__ wg)              \
    {                                                                                          \
        const uint2 w = wg[blockIdx.x];                                                        \
        const ARGS *__restrict__ t = static_cast<const ARGS *>(tab);                           \
        BODY(t[w.x], w.y);                                                                     \
    }

}  // namespace sdpd

struct sdpd_ctx {
    sdpd_params prm;
    sdpd::DevParams dp;
    sdpd::DevParams *dparams;    // device copy of dp (read by kernels through a pointer)
    hipStream_t stream;
    int device;
    int64_t n, ncell;
    // cell list
    uint32_t *cell_of, *count, *cursor, *cell_start, *block_sums, *tmp_idx, *perm, *cell_sorted;
    int64_t nscan_blocks;
    // gather targets of the sort (same shapes as the state)
    double *tq, *tp, *teps, *trho, *tf;
    uint32_t *tid;
    double *q4;                  // (x, y, z, P/rho^2) per particle in cell order, 32 B
    float *q4f;                  // mixed precision: (x, y, z) relative to the cell, P/rho^2
    uint64_t *masks;             // NNB * n
    unsigned long long *counters;
    uint32_t *err;
    double *obs_partial;         // per-block observable partials
    int64_t obs_blocks;
    double *obs_out;             // device stats records
    int64_t obs_cap;
    int cells_valid, masks_valid;
    int fd_swept;                // a schedule has been built (sdpd_fd_schedule_size)
    sdpd_tuning tuning;          // F/D workgroup sizes and LDS capacities per phase class
    int max_lds;                 // LDS bytes one workgroup may use
    int lds_share;               // LDS bytes of one sweep workgroup at two waves per SIMD
    // pair schedule (rebuilt before every sweep)
    uint32_t *task_count, *task_np, *pair_off, *part_off, *part_list;
    uint64_t *pairs;
    double *draws;               // 4 per pair entry: the sweep's random draws in sorted order
    void *sweep = nullptr;       // device table of the sweep kernel (fd.hip)
    uint32_t *sweep_order = nullptr;   // hand-out order of the ranges inside each group
    int tune_gen = 0;            // counts sdpd_tune calls (captured batches check it)
    int fd_dataflow = 0;         // SDPD_SWEEP_AUTO chooses one launch (large boxes)
    int fd_per_group = 0;        // force one launch per group (set while a batch captures)
    int fd_record_flow = 0;      // recording: the sweep as one multi-box launch (fused batch)
    int sweep_ngroups = 0;       // host copy of the sweep table's group ends
    uint32_t sweep_group_end[32] = {};
    int sweep_mode = 0;          // SDPD_SWEEP_*
    size_t sweep_lds = 0;
    int sweep_grid = 0, sweep_ok = 0;
    uint32_t *epoch = nullptr;   // ncell + 1: per-cell group epochs, then the range counter
    uint64_t *dstep;             // step index of the draws, on the device
    sdpd::AdjointWork *adj;      // checkpoints and cotangents of the adjoint (lazily)
    int64_t pair_cap, part_cap;
    sdpd::Timer timer;
    sdpd::LaunchRecord *rec = nullptr;   // recording mode: launches are appended here
    int timing;
    double last_fd_ms;
    int64_t last_fd_launches;
};

namespace sdpd {

int check_hip(hipError_t e);

// host launchers (each returns an sdpd_status)
int launch_fill_u32(sdpd_ctx *c, uint32_t *p, uint32_t v, int64_t n);
int launch_fill_u64(sdpd_ctx *c, unsigned long long *p, unsigned long long v, int64_t n);
int launch_incr_u64(sdpd_ctx *c, unsigned long long *p);
int run_scan(sdpd_ctx *c, const uint32_t *in, uint32_t *out, int64_t count, uint32_t *block_sums,
             int cap);
int run_schedule(sdpd_ctx *c);
int run_build_cells(sdpd_ctx *c, const sdpd_state *s, int kick_drift);
// pack_rho: also write rho into the w slot of the packed position records,
// where a sweep that follows in the same step reads it (FP64 path)
int run_density(sdpd_ctx *c, const sdpd_state *s, int update_eps, bool pack_rho = false);
int run_forces(sdpd_ctx *c, const sdpd_state *s, int half_kick);
int run_density_f32(sdpd_ctx *c, const sdpd_state *s, int update_eps);
int run_forces_f32(sdpd_ctx *c, const sdpd_state *s, int half_kick);
// packed: the (x, y, z, rho) records are already in place (a density pass
// with pack_rho ran since the cells were built)
int run_fd_sweep(sdpd_ctx *c, const sdpd_state *s, double dt_fd, bool packed = false);
// the two parts of run_fd_sweep: schedule (+ packing), then the launches
int fd_sweep_prepare(sdpd_ctx *c, const sdpd_state *s, bool packed);
int fd_launch_sweep(sdpd_ctx *c, const sdpd_state *s, double dt_fd);
int enqueue_step(sdpd_ctx *c, const sdpd_state *s, uint64_t step, bool set_step);
void fd_default_tuning(sdpd_ctx *c);
// LDS capacities (particles, pair entries) the defaults give phase class k
// at t tasks per workgroup
void fd_class_caps(const sdpd_ctx *c, int k, int t, int &cp, int &ce);
int fd_check_tuning(const sdpd_ctx *c, const sdpd_tuning *t);
int fd_prepare_sweep(sdpd_ctx *c);   // after any change of the tuning
bool fd_one_launch(const sdpd_ctx *c);   // the sweep runs as one launch
// The one-launch sweep of many boxes (fused batch): built from the boxes'
// flow records of one position, launched (with its counter reset) on a stream.
struct FlowSweep {
    int kind = 0, nbox = 0, ngroups = 0;
    uint32_t nitems = 0;
    size_t lds = 0;
    unsigned grid = 0;
    void *boxes = nullptr;          // device: the boxes' descriptors
    uint32_t *item_off = nullptr;   // device: ngroups x (nbox + 1) first items
    uint32_t *work = nullptr;       // device: the range counter
};
int fd_flow_build(const std::vector<sdpd_ctx *> &ctxs,
                  const std::vector<const RecordedLaunch *> &recs, FlowSweep &out);
int fd_flow_launch(const FlowSweep &f, hipStream_t stream);
void fd_flow_free(FlowSweep &f);
int run_observe(sdpd_ctx *c, const sdpd_state *s, double *dst_record);
// observables of n = dp.n particles into dst_record (REC doubles, or the
// first 7 when counters is NULL); partial holds 6 doubles per block of
// observe_blocks(n) <= OBS_MAX_BLOCKS blocks
constexpr int OBS_MAX_BLOCKS = 1024;
int observe_blocks(int64_t n);
int launch_observe(const DevParams &dp, const double *p, const double *eps, double *partial,
                   const unsigned long long *counters, double *dst_record, hipStream_t stream);
void adjoint_free(AdjointWork *a);

// event timing around one launch of class k (no-op unless c->timing)
void timer_begin(sdpd_ctx *c, int k);
void timer_end(sdpd_ctx *c, int k);

// Issue kernel `single` with `args` on the context's stream, or (recording
// mode) append the launch with its multi-box form.  grid 0 launches nothing.
template <class A>
int launch_or_record(sdpd_ctx *c, void (*single)(A), MultiKernel multi, unsigned grid,
                     unsigned block, size_t lds, const A &args)
{
    if (grid == 0) return SDPD_OK;
    if (c->rec) {
        RecordedLaunch r;
        r.multi = multi;
        r.grid = grid;
        r.block = block;
        r.lds = lds;
        r.args.resize(sizeof(A));
        memcpy(r.args.data(), &args, sizeof(A));
        c->rec->push_back(std::move(r));
        return SDPD_OK;
    }
    hipLaunchKernelGGL(single, dim3(grid), dim3(block), lds, c->stream, args);
    return check_hip(hipGetLastError());
}

}  // namespace sdpd

// --------------------------------------------------------------- device helpers
namespace sdpd {

// minimum-image component (pairs within h never straddle half a box since
// every box length is at least 4 h)
__device__ __forceinline__ double min_image(double d, double box, double half)
{
    if (d > half) return d - box;
    if (d < -half) return d + box;
    return d;
}

// neighbour cell k (offset index 0..26, z slowest) of cell (cx, cy, cz) and
// the periodic shift that turns x_i - x_j into the minimum image for it
struct NbCell {
    int64_t c;
    double sx, sy, sz;
};

__device__ __forceinline__ NbCell neighbour_cell(const DevParams &P, int cx, int cy, int cz, int k)
{
    NbCell r;
    int x2 = cx + (k % 3) - 1, y2 = cy + (k / 3) % 3 - 1, z2 = cz + k / 9 - 1;
    r.sx = x2 < 0 ? P.box[0] : (x2 >= P.nc[0] ? -P.box[0] : 0.0);
    r.sy = y2 < 0 ? P.box[1] : (y2 >= P.nc[1] ? -P.box[1] : 0.0);
    r.sz = z2 < 0 ? P.box[2] : (z2 >= P.nc[2] ? -P.box[2] : 0.0);
    x2 += x2 < 0 ? P.nc[0] : (x2 >= P.nc[0] ? -P.nc[0] : 0);
    y2 += y2 < 0 ? P.nc[1] : (y2 >= P.nc[1] ? -P.nc[1] : 0);
    z2 += z2 < 0 ? P.nc[2] : (z2 >= P.nc[2] ? -P.nc[2] : 0);
    r.c = x2 + (int64_t)P.nc[0] * (y2 + (int64_t)P.nc[1] * z2);
    return r;
}

// The same 27 neighbour cells of one cell, with the boundary tests done
// once: bit a of lo (hi) says the cell is the first (last) of axis a, where
// an offset of -1 (+1) wraps and carries the shift +L (-L).  Cell indices fit
// in 32 bits (14 ncell < 2^32).  get(k) equals neighbour_cell(P, cx, cy, cz, k).
struct NbSteps {
    uint32_t c, lo, hi;
    __device__ __forceinline__ NbSteps(const DevParams &P, int cx, int cy, int cz)
    {
        c = (uint32_t)cx + (uint32_t)P.nc[0] * ((uint32_t)cy + (uint32_t)P.nc[1] * (uint32_t)cz);
        lo = (cx == 0 ? 1u : 0u) | (cy == 0 ? 2u : 0u) | (cz == 0 ? 4u : 0u);
        hi = (cx == P.nc[0] - 1 ? 1u : 0u) | (cy == P.nc[1] - 1 ? 2u : 0u) |
             (cz == P.nc[2] - 1 ? 4u : 0u);
    }
    __device__ __forceinline__ NbCell get(const DevParams &P, int k) const
    {
        const int o[3] = {k % 3, (k / 3) % 3, k / 9};
        uint32_t d = 0, stride = 1;
        double sh[3];
        for (int a = 0; a < 3; ++a) {
            const bool wrap_lo = (lo >> a) & 1u, wrap_hi = (hi >> a) & 1u;
            const uint32_t n = (uint32_t)P.nc[a];
            if (o[a] == 0) {
                d += wrap_lo ? (n - 1u) * stride : 0u - stride;
                sh[a] = wrap_lo ? P.box[a] : 0.0;
            } else if (o[a] == 2) {
                d += wrap_hi ? 0u - (n - 1u) * stride : stride;
                sh[a] = wrap_hi ? -P.box[a] : 0.0;
            } else {
                sh[a] = 0.0;
            }
            stride *= n;
        }
        NbCell r;
        r.c = (int64_t)(uint32_t)(c + d);
        r.sx = sh[0];
        r.sy = sh[1];
        r.sz = sh[2];
        return r;
    }
};

__device__ __forceinline__ int cell_coord(double x, double inv_cell, int nc)
{
    int c = (int)floor(x * inv_cell);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

}  // namespace sdpd
