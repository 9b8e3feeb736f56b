/*
 * sdpd.h -- C ABI of libsdpd, Smoothed Dissipative Particle Dynamics with the
 * Metropolized fluctuation/dissipation scheme of Faure & Stoltz, "Stable and
 * accurate schemes for Smoothed Dissipative Particle Dynamics"
 * (arXiv:1707.04232), on AMD Instinct MI355X (gfx950).
 *
 * Conventions
 *  - All floating point is IEEE binary64.
 *  - State arrays are DEVICE pointers owned by the caller, structure of
 *    arrays: a 3-vector field of n particles is 3*n doubles, x[0..n) then
 *    y[0..n) then z[0..n).  Every array must be 8-byte aligned and hold n
 *    (or 3n) elements.  The library never frees them.
 *  - A context owns all workspace (cell lists, pair masks, partial sums,
 *    counters, the sticky device error word), sized at sdpd_create for n.
 *  - Calls are asynchronous on the stream given at sdpd_create unless they
 *    return statistics (then they synchronise that stream).  One context must
 *    not be used from two host threads at once.
 *  - Every call returns an sdpd_status.  Argument errors are detected on the
 *    host before any launch and leave the state unchanged.  Conditions found
 *    on the device (cell overflow, negative energy in SSA mode, non-finite
 *    values) set a sticky error word that the next synchronising call
 *    returns; after such an error the state is unspecified.
 */
#ifndef SDPD_H
#define SDPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDPD_ABI_VERSION 8

typedef enum {
    SDPD_OK = 0,
    SDPD_EINVAL = -1,     /* bad argument or parameter (host check)          */
    SDPD_EHIP = -2,       /* a HIP runtime call failed                        */
    SDPD_ENOMEM = -3,     /* workspace allocation failed                      */
    SDPD_ECELLCAP = -4,   /* a cell holds more than cell_cap particles        */
    SDPD_ENEGEPS = -5,    /* SSA mode produced eps <= 0 (Sec. 3.2 of the paper) */
    SDPD_ENONFINITE = -6, /* a position, energy or density is not finite      */
    SDPD_ECAPACITY = -7   /* more active pairs than the schedule holds (64 per particle) */
} sdpd_status;

/* SPH kernel W with support h (Sec. 2.1.1): Lucy's quartic, or the paper's
 * cubic spline of eq. (sdpd-cubic-w).                                       */
typedef enum { SDPD_KERNEL_LUCY = 0, SDPD_KERNEL_CUBIC = 1 } sdpd_kernel;

/* fluctuation/dissipation scheme: exact Metropolis (EMS, Sec. 3.3.2),
 * approximate Metropolis rejecting only negative energies (AMS, Sec. 3.3.3),
 * the Shardlow-like splitting without rejection (SSA, Sec. 3.2), or none.  */
typedef enum { SDPD_FD_EMS = 0, SDPD_FD_AMS = 1, SDPD_FD_SSA = 2, SDPD_FD_NONE = 3 } sdpd_fd;

/* arithmetic of the particle passes: everything in FP64, or (MIXED) the
 * density, the pair masks and the pressure forces from FP32 positions
 * relative to the particle's cell, FP32 kernel values and FP32 sums, and
 * (EMS with Lucy's kernel and zeta = 0) the F/D pair geometry, the Gaussian
 * draws G (Box-Muller of the same Philox words) and the proposal
 * coefficients alpha, b of eq. (proposal) in FP32, while momenta, energies,
 * the equation of state, the uniform U, the proposal v' = alpha v + b G,
 * Delta, the Metropolis ratio (evaluated for those same coefficients and
 * draws) and the observables stay FP64.  MIXED decides r < h in FP32, so
 * pairs within ~1e-7 h of the cutoff may differ from FP64; its draws lie
 * within ~2e-6 of the FP64 ones.                                          */
typedef enum { SDPD_FP64 = 0, SDPD_MIXED = 1 } sdpd_prec;

/* Physical and numerical parameters.  Ideal-gas entropy closure
 *   S(eps, rho) = Cv ln eps - A kB ln(rho / rho0)          (eq. pg-eos)
 * so T = eps/Cv, P = A kB rho eps / (m Cv), C = Cv (Sec. 2.1.2).  A = 0
 * selects the default A = Cv / (3 kB) (the paper's ideal-gas entropy of
 * Sec. 4 with kB restored in its density term).
 * Requirements: n >= 0; m, h, kB, Cv, rho0, dt > 0; A > 0 or A == 0 (the
 * default); Cv > kB/2 (so that
 * d_ij < 1); eta > 0 and 0 <= zeta < 5 eta / 3 (both kappas positive);
 * box[k] / ncell[k] >= h with ncell[k] even and >= 4 (ncell[k] = 0 picks the
 * largest even integer <= box[k]/h); 1 <= cell_cap <= 64; fd_every >= 1.   */
typedef struct {
    int64_t n;            /* number of particles                            */
    double box[3];        /* periodic box lengths                           */
    double m, h, kB;      /* particle mass, smoothing length, Boltzmann     */
    double Cv, A, rho0;   /* heat capacity, EOS coefficient (0 = Cv/(3 kB)), ref. density */
    double eta, zeta;     /* shear and bulk viscosity                       */
    double dt;            /* time step                                      */
    int32_t fd_every;     /* theta: F/D every theta steps with theta*dt (Sec. 4.2) */
    int32_t kernel;       /* sdpd_kernel                                    */
    int32_t fd;           /* sdpd_fd                                        */
    int32_t prec;         /* sdpd_prec                                      */
    uint64_t seed;        /* Philox key                                     */
    uint32_t replica;     /* replica index, part of the Philox counter      */
    int32_t cell_cap;     /* max particles per cell (<= 64)                 */
    int32_t ncell[3];     /* cells per axis, 0 = automatic                  */
} sdpd_params;

/* Particle state, device pointers (see Conventions).  eps > 0.            */
typedef struct {
    double *q;            /* positions in [0, box), 3n                      */
    double *p;            /* momenta, 3n                                    */
    double *eps;          /* internal energies, n                           */
    double *rho;          /* densities, n                                   */
    double *f;            /* conservative forces, 3n                        */
    uint32_t *id;         /* particle identities (distinct), n              */
} sdpd_state;

/* Counters of one F/D sweep and observables after a step.                */
typedef struct {
    uint64_t proposed;    /* active pairs visited                           */
    uint64_t rej_energy;  /* rejected by the energy bound, eq. (energy-bound) */
    uint64_t rej_ratio;   /* rejected by the Metropolis test                */
    uint64_t marginal;    /* decisions within the rounding margin           */
    uint64_t negeps;      /* SSA moves that made an energy non-positive     */
    double E, Eint, KE;   /* total, internal and kinetic energy (Sec. 2.2.1) */
    double P[3];          /* total momentum                                 */
    double min_eps;       /* smallest internal energy                       */
} sdpd_stats;

typedef struct sdpd_ctx sdpd_ctx;

/* Create a context for params->n particles on the current HIP device.
 * hip_stream: a hipStream_t (NULL = the default stream) that every later
 * call of this context launches on.  *out receives the context.
 * Errors: SDPD_EINVAL (parameters), SDPD_ENOMEM, SDPD_EHIP.                */
int sdpd_create(const sdpd_params *params, void *hip_stream, sdpd_ctx **out);

/* Destroy a context (synchronises its stream, frees its workspace).       */
int sdpd_destroy(sdpd_ctx *ctx);

/* Cell list (not part of the paper; it defines the pair schedule, see
 * sdpd_fd_metropolis).  Sorts the state in place by (cell, id): cell c =
 * cx + nx (cy + ny cz) with ck = floor(q_k * ncell_k / box_k) clamped to
 * [0, ncell_k); within a cell by increasing id (the slot).  All six arrays
 * are permuted; cell_start[0..ncell] is kept in the context.  A cell with
 * more than cell_cap particles raises SDPD_ECELLCAP (sticky).             */
int sdpd_build_cells(sdpd_ctx *ctx, const sdpd_state *state);

/* Device pointer to the context's cell_start array (ncell+1 uint32) and
 * the cell counts per axis (for inspection; valid until the next call).   */
int sdpd_cell_info(sdpd_ctx *ctx, int32_t ncell[3], const uint32_t **cell_start);

/* Copy cell_start (ncell+1 uint32) into the HOST array dst of capacity
 * entries (sync).  SDPD_EINVAL if capacity < ncell + 1.                   */
int sdpd_copy_cell_start(sdpd_ctx *ctx, uint32_t *dst, int64_t capacity);

/* SPH density, eq. (sdpd-rho-v): rho_i = sum_j m W(r_ij) over all j with
 * r_ij < h (minimum image) including j = i.  Requires the state to be in
 * the order of the last sdpd_build_cells.  If update_eps_const_S != 0 the
 * internal energies follow the entropy-conserving update of Sec. 3.1:
 * eps_i <- eps_i (rho_new_i / rho_old_i)^(A kB / Cv), rho_old being the
 * rho array on entry.  Also records the active-pair masks that
 * sdpd_fd_metropolis uses.                                                 */
int sdpd_density(sdpd_ctx *ctx, const sdpd_state *state, int update_eps_const_S);

/* Conservative forces, eq. (cons-forces):
 *   f_i = sum_{j != i, r_ij < h} m^2 (P_i/rho_i^2 + P_j/rho_j^2) F_ij r_ij
 * with P from the closure at (eps, rho).  Requires sdpd_density since the
 * last sdpd_build_cells, on the same positions (the partners are the active
 * pairs it recorded); SDPD_EINVAL otherwise.                              */
int sdpd_forces(sdpd_ctx *ctx, const sdpd_state *state);

/* One fluctuation/dissipation sweep with time step fd_every * dt: every
 * pair with r_ij < h is updated once, EMS/AMS/SSA per params->fd (Sec. 3.2,
 * 3.3), with i the smaller id.  Pair (i, j) draws its Gaussian vector and
 * uniform from Philox4x32-10 with key seed and counter
 * (step, id_i, id_j, 2 replica + k), k = 0, 1.  Pairs are applied in
 * ascending (phase, round): phase 0 = pairs inside a cell, phase
 * 1 + 8 o + pi = pairs between cell A of coordinate parity pi and its o-th
 * forward neighbour (o = 0..12, the offsets after the centre of the
 * z-slowest 27-list); round = slot_A XOR slot_B.  Equal keys share no
 * particle.  Requires sdpd_density on the current cell order (for the pair
 * masks and rho).  If out is not NULL the counters are returned (sync).    */
int sdpd_fd_metropolis(sdpd_ctx *ctx, const sdpd_state *state, uint64_t step,
                       sdpd_stats *out);

/* nsteps full steps, step indices step0 .. step0+nsteps-1, each:
 *   p += dt/2 f; q += dt p/m (wrapped once into [0, box)); build cells;
 *   density with the entropy-conserving energy update; if step % fd_every
 *   == 0 an F/D sweep; forces; p += dt/2 f     (eq. sdpd-verlet + splitting)
 * On entry rho and f must belong to q (sdpd_build_cells, sdpd_density(0),
 * sdpd_forces).  per_step (host array of nsteps, or NULL) receives each
 * step's counters and observables; it makes the call synchronise once at
 * the end.  Without it the call is asynchronous.                          */
int sdpd_step(sdpd_ctx *ctx, const sdpd_state *state, uint64_t step0, int nsteps,
              sdpd_stats *per_step);

/* Observables of the current state (sync): E, Eint, KE, P, min_eps.       */
int sdpd_observe(sdpd_ctx *ctx, const sdpd_state *state, sdpd_stats *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of sdpd_observe (the total energy E = sum eps + |p|^2/2m and
 * the total momentum of Sec. 2.2.1) for any state, without a context and
 * without allocating anything.  params must pass the checks of sdpd_create
 * (only n and m are used); state->p (3 x n) and state->eps (n) are read, the
 * other state pointers are not used.  out: DEVICE array of 7 doubles that
 * receives E, Eint, KE, P[0], P[1], P[2], min_eps (min_eps = +inf for n = 0).
 * Asynchronous on hip_stream (NULL = the default stream): no synchronisation,
 * capturable in a HIP graph; errors of the launch are returned, nothing is
 * sticky.  Limits: n <= SDPD_OBSERVE_NOALLOC_MAX_N (SDPD_EINVAL beyond);
 * the partial sums (at most 1024 blocks x 6 doubles, 48 KiB) live in a fixed
 * device array of the library, one per device, kept until the process ends:
 * calls that overlap on one device (two streams, two threads) race on it and
 * must be ordered by the caller.  The sums are those of sdpd_observe, in the
 * same order, so the values are bit for bit identical.  SDPD_EINVAL for bad
 * parameters or NULL pointers, SDPD_EHIP for a failed launch.               */
#define SDPD_OBSERVE_NOALLOC_MAX_N 0x7fffffffLL
int sdpd_observe_noalloc(const sdpd_params *params, const sdpd_state *state, void *hip_stream,
                         double *out);

/* Wait for the context's stream and return (then clear) the first sticky
 * device error, or SDPD_OK.                                               */
int sdpd_sync(sdpd_ctx *ctx);

/* Kernel timing with HIP events on the context's stream.  sdpd_set_timing
 * (sync) switches it on or off and clears the record; while on, every launch
 * of the classes below is bracketed by two events.  sdpd_timing (sync)
 * returns, per class, the summed milliseconds and the number of launches
 * since the last call, then clears the record.  Classes: 0 cell build,
 * 1 density, 2 F/D phase kernels, 3 forces + half kick, 4 observables,
 * 5 F/D scheduling pass.                                                   */
int sdpd_set_timing(sdpd_ctx *ctx, int enable);
/* The same for the classes whose bit is set in mask (bit k = class k); the
 * other classes run without events.  SDPD_EINVAL for bits beyond class 5. */
int sdpd_set_timing_mask(sdpd_ctx *ctx, uint32_t mask);
int sdpd_timing(sdpd_ctx *ctx, double ms[6], int64_t launches[6]);

/* Execution-only tuning of the F/D sweep (results do not change).  Index k
 * is the phase class: 0 = phase 0 (pairs inside a cell), 1, 2, 3 = phases of
 * cell pairs whose offset has 1 (face), 2 (edge), 3 (corner) non-zero
 * components.
 *   fd_tasks[k]          tasks (cells or cell pairs) per workgroup, 1..64;
 *   fd_lds_particles[k]  particles one workgroup stages in LDS, >= 128;
 *   fd_lds_pairs[k]      pair entries one workgroup sorts in LDS, >= 64.
 * A workgroup whose tasks need more than its capacity processes them in
 * several batches.  The LDS of one workgroup, 36 B per particle + 4 B per
 * pair entry + 1320 B, must fit the device's per-workgroup limit.  Fields
 * equal to 0 in sdpd_tune keep the current value, and a negative LDS field
 * selects the capacities the defaults give the class's (new) task count
 * (sdpd_tune waits for the context's stream first); sdpd_get_tuning reports
 * the values in use (the defaults scale with the mean particles per cell).
 * SDPD_EINVAL for out-of-range values; nothing is changed then.          */
typedef struct {
    int32_t fd_tasks[4];
    int32_t fd_lds_particles[4];
    int32_t fd_lds_pairs[4];
} sdpd_tuning;

int sdpd_tune(sdpd_ctx *ctx, const sdpd_tuning *tuning);
int sdpd_get_tuning(sdpd_ctx *ctx, sdpd_tuning *out);

/* How the F/D sweep is launched (results are identical bit for bit).  The
 * sweep is 27 groups of mutually disjoint phases (phase 0, then 26 groups of
 * 4 inter-cell phases) that must follow one another on each cell.
 *   SDPD_SWEEP_AUTO       one launch for boxes large enough to hold several
 *                         GPU-fulls of task ranges, else one per group;
 *   SDPD_SWEEP_ONE        one persistent launch: each range waits only for
 *                         the ranges of the previous group on its cells;
 *   SDPD_SWEEP_PER_GROUP  27 launches.
 * Captured batches always use one launch per group.  sdpd_set_sweep_mode
 * returns SDPD_EINVAL for another mode or a NULL context.  sdpd_sweep_mode
 * returns the mode set (>= 0; SDPD_EINVAL for a NULL context) and writes
 * the layout the next sweep uses (SDPD_SWEEP_ONE or SDPD_SWEEP_PER_GROUP)
 * to *in_use when it is not NULL.                                          */
enum { SDPD_SWEEP_AUTO = 0, SDPD_SWEEP_ONE = 1, SDPD_SWEEP_PER_GROUP = 2 };
int sdpd_set_sweep_mode(sdpd_ctx *ctx, int mode);
int sdpd_sweep_mode(sdpd_ctx *ctx, int *in_use);

/* Autotuner of the F/D sweep's execution-only parameters: the tasks per
 * workgroup of each phase class (LDS capacities sized for them as the
 * defaults are) and, when the mode is SDPD_SWEEP_AUTO, the layout.  It times
 * `trials` sweeps (1..64) of each candidate on device-side scratch copies of
 * state->p and state->eps, by coordinate descent from the current tuning
 * (tasks x 1/2, 3/4, 3/2, 2 per class; a candidate must be 1 % faster), and
 * keeps the fastest: the results of later calls do not depend on it.  The
 * cells and masks must be current (sdpd_build_cells and sdpd_density, or a
 * step, since the last change of the state); the state is not modified.
 * Waits for the context's stream; allocates the scratch arrays (32 B per
 * particle) for the duration of the call.  Writes the tuning in use to
 * *chosen when it is not NULL.  Like sdpd_tune, invalidates captured
 * batches.  SDPD_EINVAL for invalid arguments or stale cells; on a HIP
 * error the previous tuning and mode are restored.                        */
int sdpd_autotune(sdpd_ctx *ctx, const sdpd_state *state, int trials, sdpd_tuning *chosen);

/* Batched replicas (many independent boxes advanced together).  Each box
 * is a context of its own (its parameters, replica index, stream) with its
 * state, prepared as for sdpd_step (cells, density, forces).  All contexts
 * must share the device and fd_every, have timing off, appear once, and
 * use created streams (not the null stream, which cannot be captured).
 * sdpd_batch_create captures fd_every consecutive steps of every box into
 * HIP graphs (it waits for the boxes' streams first; the graphs refer to
 * the given state arrays, which must stay allocated) in the fused layout of
 * sdpd_batch_create_layout below.  In the graph layout: one graph per
 * stream when the process has at least as many hardware queues as there
 * are streams (environment GPU_MAX_HW_QUEUES, 4 when unset), else one graph
 * that forks to and joins the boxes' streams.  sdpd_batch_run
 * replays it for steps step0 .. step0+nsteps-1 (both multiples of
 * fd_every; SDPD_EINVAL if a context was retuned with sdpd_tune after the
 * capture): every box advances exactly as with sdpd_step on its own (bit
 * for bit), the boxes of different streams concurrently.  It is
 * asynchronous: later work on a box's stream waits for it; sdpd_sync /
 * sdpd_observe on a context report errors and observables.  Steps follow
 * eq. (sdpd-verlet) with the F/D sweep of Sec. 3.3 as in sdpd_step.       */
typedef struct sdpd_batch sdpd_batch;
int sdpd_batch_create(sdpd_ctx *const *ctxs, const sdpd_state *states, int nbox,
                      sdpd_batch **out);

/* The same with an explicit layout:
 *   SDPD_BATCH_FUSED   every stage of the step runs for all boxes in one
 *                      launch (each box's workgroups and arguments as in its
 *                      own step, taken from device tables), the launches of
 *                      fd_every steps captured in a graph; the boxes are
 *                      dealt into `parts` parts of about equal particle
 *                      count (<= 0: min(GPU_MAX_HW_QUEUES, 16)), each with
 *                      its own graph and stream, which run side by side;
 *                      ~50 launches per part and step for any number of
 *                      boxes.  Boxes of any size, precision and scheme.
 *   SDPD_BATCH_FUSED_FLOW  the fused layout with the F/D sweeps of a part's
 *                      boxes in one persistent launch (their task ranges,
 *                      group by group over all boxes, handed out by one
 *                      counter; a range waits only for its own box's earlier
 *                      groups, on per-cell epochs), instead of one launch
 *                      per group of commuting phases;
 *   SDPD_BATCH_GRAPHS  each box's own launch sequence captured: one graph per
 *                      stream, or one graph forking to the boxes' streams
 *                      (see sdpd_batch_create above);
 *   SDPD_BATCH_AUTO    the fused layout (what sdpd_batch_create uses).
 * Results are identical bit for bit in every layout.  sdpd_batch_layout
 * returns the layout in use (SDPD_EINVAL for NULL).                         */
enum { SDPD_BATCH_AUTO = 0, SDPD_BATCH_FUSED = 1, SDPD_BATCH_GRAPHS = 2,
       SDPD_BATCH_FUSED_FLOW = 3 };
int sdpd_batch_create_layout(sdpd_ctx *const *ctxs, const sdpd_state *states, int nbox,
                             int layout, int parts, sdpd_batch **out);
int sdpd_batch_layout(const sdpd_batch *batch);
int sdpd_batch_run(sdpd_batch *batch, uint64_t step0, int nsteps);
int sdpd_batch_destroy(sdpd_batch *batch);

/* Adjoint of the conservative dynamics (F/D off: params.fd = SDPD_FD_NONE,
 * FP64): reverse-mode gradients of a scalar J(q_K, p_K) with respect to the
 * initial positions, momenta and internal energies and to the closure
 * coefficient A, through K steps of eq. (sdpd-verlet) with the density of
 * eq. (sdpd-rho-v), the entropy-conserving energies of Sec. 3.1 (the
 * entropies follow from eps0 and rho(q0), so rho0 cancels) and the forces of
 * eq. (cons-forces).  sdpd_adjoint_forward advances the prepared state by
 * nsteps steps (as sdpd_step does), keeping a copy of the full state every
 * checkpoint_every steps in the context; particle ids must be 0..n-1
 * (SDPD_EINVAL from the next synchronising call otherwise).
 * sdpd_adjoint_backward takes dJ/dq_K and dJ/dp_K (device, 3 x n planes,
 * indexed by particle id) and writes dJ/dq0, dJ/dp0 (device, same layout),
 * dJ/deps0 (device, n by id; may be NULL) and dJ/dA (host scalar; may be
 * NULL; its computation synchronises).  It recomputes each segment from its
 * checkpoint; memory: (nsteps / checkpoint_every + checkpoint_every + 2)
 * full states.                                                             */
int sdpd_adjoint_forward(sdpd_ctx *ctx, sdpd_state *state, int nsteps, int checkpoint_every);
int sdpd_adjoint_backward(sdpd_ctx *ctx, const double *dJ_dq, const double *dJ_dp,
                          double *dJ_dq0, double *dJ_dp0, double *dJ_deps0, double *dJ_dA);

/* The reverse pass of sdpd_adjoint_backward for a J that may also read the
 * final internal energies and densities, e.g. the mean pressure
 * P = A kB rho eps / (m Cv) of the closure of Sec. 2.1.2 with eq. (pg-eos).
 * ct: cotangents dJ/dq_K, dJ/dp_K (DEVICE, 3 x n, by id; required) and
 * dJ/deps_K, dJ/drho_K (DEVICE, n, by id; NULL = zero).  The final energies
 * follow the final densities at the entropies fixed by the initial state
 * (eps_K = eps0 (rho_K / rho(q0))^(A kB/Cv), Sec. 3.1), so dJ/deps_K reaches
 * q0 through both densities and eps0 through the entropies.
 * gr: dq0, dp0 (DEVICE, 3 x n, by id; required), deps0 (DEVICE, n, by id;
 * may be NULL) receive the gradients; the host scalars dA, dCv and drho0
 * receive the gradients with respect to the closure coefficient A, the heat
 * capacity Cv at fixed A (the conservative dynamics depends on them only
 * through A/Cv, so dCv = -(A/Cv) dA; with the default A = Cv/(3 kB) tied to
 * Cv the total derivative along the tie, dCv + dA/(3 kB), is zero) and the
 * reference density rho0 of eq. (pg-eos) (zero: rho0 cancels from the
 * dynamics).  These are the derivatives through the dynamics; terms of J's
 * own explicit dependence on A or Cv are the caller's.  Synchronises.
 * SDPD_EINVAL without a preceding sdpd_adjoint_forward or for NULL required
 * pointers.                                                                */
typedef struct {
    const double *dq, *dp;     /* 3 x n, required                          */
    const double *deps, *drho; /* n, NULL = zero                           */
} sdpd_cotangent;
typedef struct {
    double *dq0, *dp0;         /* 3 x n, required                          */
    double *deps0;             /* n, may be NULL                           */
    double dA, dCv, drho0;     /* host outputs                             */
} sdpd_gradient;
int sdpd_adjoint_vjp(sdpd_ctx *ctx, const sdpd_cotangent *ct, sdpd_gradient *gr);

/* Size of the pair schedule of the last F/D sweep (sync): the number of
 * active pairs and the number of particle entries the phase workgroups
 * staged (a particle counts once per task it takes part in).  Zeros before
 * the first sweep.                                                          */
int sdpd_fd_schedule_size(sdpd_ctx *ctx, int64_t *pairs, int64_t *staged);

const char *sdpd_strerror(int status);
int sdpd_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
