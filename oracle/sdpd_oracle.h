/*
 * sdpd_oracle.h -- plain FP64 CPU oracle for one SDPD time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Method: Faure & Stoltz, "Stable and accurate schemes for Smoothed
 * Dissipative Particle Dynamics" (arXiv:1707.04232).  Every function names the
 * section / equation of the paper it follows.  Where the paper is silent or
 * garbled the reading taken is stated next to the function.
 *
 * Data layout (shared with the C ABI of the GPU library because it is the
 * interface shape, not because code is shared): structure of arrays, a
 * 3-vector field of n particles is 3*n doubles, x[0..n) then y then z.
 */
#ifndef SDPD_ORACLE_H
#define SDPD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SO_OK = 0, SO_EINVAL = -1, SO_ENOMEM = -3, SO_ECELLCAP = -4,
       SO_ENEGEPS = -5, SO_ENONFINITE = -6 };
enum { SO_KERNEL_LUCY = 0, SO_KERNEL_CUBIC = 1 };
enum { SO_FD_EMS = 0, SO_FD_AMS = 1, SO_FD_SSA = 2, SO_FD_NONE = 3 };

typedef struct {
    int64_t n;
    double box[3];
    double m, h, kB;
    double Cv, A, rho0;     /* S(eps,rho) = Cv ln eps - A kB ln(rho/rho0) */
    double eta, zeta, dt;
    int32_t fd_every;       /* theta of the multiple-time-step variant      */
    int32_t kernel, fd_mode;
    uint64_t seed;
    uint32_t replica;
    int32_t cell_cap;
    int32_t ncell[3];       /* 0 = largest even integer <= box/h            */
} so_params;

typedef struct {
    uint64_t proposed, rej_energy, rej_ratio, marginal, negeps;
    double E, Eint, KE, P[3], min_eps;
} so_stats;

/* one record per active pair of a fluctuation/dissipation sweep, in the
 * order the sweep applied them (for schedule and decision checks)          */
typedef struct {
    int32_t phase, round;
    int32_t i, j;           /* state indices, i = smaller particle id          */
    int32_t decision;       /* 0 accepted, 1 rejected (energy), 2 rejected (ratio) */
    int32_t pad;
    double a_minus_lnU;     /* EMS log ratio minus log U (0 otherwise)        */
    double bound_gap;       /* min(eps_i,eps_j) - Delta                        */
} so_pairrec;

/* --- kernel and closure ------------------------------------------------ */
double so_kernel_w(int kernel, double h, double r);
double so_kernel_f(int kernel, double h, double r);
double so_entropy(const so_params *P, double eps, double rho);
double so_temperature(const so_params *P, double eps, double rho);
double so_pressure(const so_params *P, double eps, double rho);
double so_heat_capacity(const so_params *P, double eps, double rho);
double so_eps_at_entropy(const so_params *P, double S, double rho);

/* --- cells ------------------------------------------------------------- */
int so_grid(const so_params *P, int32_t ncell_out[3]);
int so_build_cells(const so_params *P, double *q, double *p, double *eps,
                   double *rho, double *f, uint32_t *id, uint32_t *cell_start);

/* --- density, forces --------------------------------------------------- */
int so_density(const so_params *P, const double *q, const uint32_t *cell_start,
               double *rho_out);
int so_density_bruteforce(const so_params *P, const double *q, double *rho_out);
int so_update_eps_const_entropy(const so_params *P, double *eps,
                                const double *rho_old, const double *rho_new);
int so_forces(const so_params *P, const double *q, const double *rho,
              const double *eps, const uint32_t *cell_start, double *f_out);
int so_forces_bruteforce(const so_params *P, const double *q, const double *rho,
                         const double *eps, double *f_out);

/* --- random numbers ---------------------------------------------------- */
void so_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void so_pair_draws(uint64_t seed, uint64_t step, uint32_t id_i, uint32_t id_j,
                   uint32_t replica, double G[3], double *U);

/* --- fluctuation / dissipation ----------------------------------------- */
void so_fd_coefficients(const so_params *P, double F, double rho_i, double rho_j,
                        double eps_i, double eps_j, double dt,
                        double alpha[2], double zeta[2]);
double so_fd_log_ratio(const so_params *P, double F, double rho_i, double rho_j,
                       double eps_i, double eps_j, const double v[3],
                       const double e[3], const double G[3], double dt,
                       double vnew[3], double eps_new[2]);
int so_fd_pair_list(const so_params *P, const double *q, const uint32_t *cell_start,
                    so_pairrec *out, int64_t cap, int64_t *count);
int so_fd_sweep(const so_params *P, const double *q, double *p, double *eps,
                const double *rho, const uint32_t *id, const uint32_t *cell_start,
                uint64_t step, double dt_fd, so_stats *st,
                so_pairrec *log, int64_t log_cap);
/* the same sweep where, for the pairs at positions flip_pos[0..nflip)
 * (ascending, in sweep order), the outcome of the energy bound (bit 0 of
 * flip_kind) and/or of the Metropolis test (bit 1) is inverted: a test
 * control for decisions inside the rounding margin (reading A16).
 * SO_EINVAL if flip_pos is not strictly ascending or a kind is not 0..3.   */
int so_fd_sweep_flip(const so_params *P, const double *q, double *p, double *eps,
                     const double *rho, const uint32_t *id, const uint32_t *cell_start,
                     uint64_t step, double dt_fd, so_stats *st,
                     so_pairrec *log, int64_t log_cap, const int64_t *flip_pos,
                     const int32_t *flip_kind, int64_t nflip);

/* --- full step and observables ----------------------------------------- */
int so_observe(const so_params *P, const double *p, const double *eps, so_stats *st);
int so_kick(const so_params *P, double *p, const double *f, double half_dt);
int so_drift(const so_params *P, double *q, const double *p, double dt);
int so_step(const so_params *P, double *q, double *p, double *eps, double *rho,
            double *f, uint32_t *id, uint32_t *cell_start, uint64_t step0,
            int nsteps, so_stats *per_step);

/* --- parallel variant (OpenMP; one thread when built without it) ------- */
/* so_step with density, energy update and forces spread over threads per
 * particle and the F/D sweep phase by phase over the phase's disjoint tasks
 * (reading A12): the same result bit for bit.  so_threads sets the thread
 * count (<= 0 keeps it) and returns the count in use.                      */
int so_threads(int nthreads);
int so_step_parallel(const so_params *P, double *q, double *p, double *eps, double *rho,
                     double *f, uint32_t *id, uint32_t *cell_start, uint64_t step0,
                     int nsteps, so_stats *per_step);

#ifdef __cplusplus
}
#endif
#endif
