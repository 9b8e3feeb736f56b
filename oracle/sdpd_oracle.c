/*
 * sdpd_oracle.c -- plain FP64 CPU oracle for SDPD with the Metropolized
 * fluctuation/dissipation scheme of Faure & Stoltz (arXiv:1707.04232).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline to check the HIP library.  It is single threaded,
 * unblocked and unfused on purpose, and it shares no code with the GPU path.
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (see build.py).
 *
 * Readings taken where the paper is silent or garbled (numbered as in the
 * design notes of the repository):
 *   A1  the configurations use Lucy's kernel; the paper's cubic spline is the
 *       second option of the kernel enum.
 *   A2  the second branch of the cubic spline's F is F = 48/(pi h^4 r)(1-r/h)^2
 *       (the printed h^5 is a typo: it makes F discontinuous at h/2).
 *   A3  the density sum runs over all j including j = i.
 *   A4  ideal-gas entropy S = Cv ln eps - A kB ln(rho/rho0), A = Cv/(3 kB) by
 *       default (the paper's rho term with kB restored).
 *   A6  in the relative-velocity proposal the noise amplitude is (2/m) zeta.
 *   A10 a pair is active iff r^2 < h^2 with the minimum image.
 *   A11 the pair is oriented with i = smaller particle id.
 *   A12 pairs are applied in ascending (phase, round); see so_fd_pair_list.
 *   A13 step order: half kick, drift, cells, density + constant-entropy
 *       energy update, F/D sweep, force, half kick.
 *   A15 accept iff U <= exp(a); energy bound strict.
 *   A17 Philox4x32-10 counter (step, id_i, id_j, 2 replica + draw), Box-Muller.
 *   A21 1 - alpha^2 is evaluated as -expm1(-4 gamma dt / m).
 */
#include "sdpd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SO_PI 3.14159265358979323846

/* ======================================================================= */
/* SPH kernels, Sec. 2.1.1                                                  */
/* ======================================================================= */

/* W(r) with support h.  Cubic spline: eq. (sdpd-cubic-w).  Lucy:
 * W = 105/(16 pi h^3) (1 + 3x)(1 - x)^3, x = r/h (reading A1).            */
double so_kernel_w(int kernel, double h, double r)
{
    double x = r / h;
    if (x >= 1.0) return 0.0;
    if (kernel == SO_KERNEL_LUCY)
        return 105.0 / (16.0 * SO_PI * h * h * h) * (1.0 + 3.0 * x) * pow(1.0 - x, 3);
    if (x <= 0.5)
        return 8.0 / (SO_PI * h * h * h) * (1.0 - 6.0 * x * x + 6.0 * x * x * x);
    return 16.0 / (SO_PI * h * h * h) * pow(1.0 - x, 3);
}

/* F defined by grad W(r) = -F(|r|) r (Sec. 2.1.1), i.e. F = -W'(r)/r.
 * Lucy: F = 315/(4 pi h^5) (1 - x)^2.  Cubic: the paper's first branch and
 * the corrected second branch (reading A2).                               */
double so_kernel_f(int kernel, double h, double r)
{
    double x = r / h;
    if (x >= 1.0) return 0.0;
    if (kernel == SO_KERNEL_LUCY)
        return 315.0 / (4.0 * SO_PI * pow(h, 5)) * (1.0 - x) * (1.0 - x);
    if (x <= 0.5)
        return 48.0 / (SO_PI * pow(h, 5)) * (2.0 - 3.0 * x);
    return 48.0 / (SO_PI * pow(h, 4) * r) * (1.0 - x) * (1.0 - x);
}

/* ======================================================================= */
/* Thermodynamic closure, Sec. 2.1.2 with the ideal gas of eq. (pg-eos)     */
/* ======================================================================= */

double so_entropy(const so_params *P, double eps, double rho)
{
    return P->Cv * log(eps) - P->A * P->kB * log(rho / P->rho0);
}

/* partial derivatives of the entropy function above */
static double dS_deps(const so_params *P, double eps) { return P->Cv / eps; }
static double d2S_deps2(const so_params *P, double eps) { return -P->Cv / (eps * eps); }
static double dS_drho(const so_params *P, double rho) { return -P->A * P->kB / rho; }

/* T = 1 / (dS/deps) */
double so_temperature(const so_params *P, double eps, double rho)
{
    (void)rho;
    return 1.0 / dS_deps(P, eps);
}

/* P = -(rho^2/m) (dS/drho) / (dS/deps) */
double so_pressure(const so_params *P, double eps, double rho)
{
    return -(rho * rho / P->m) * dS_drho(P, rho) / dS_deps(P, eps);
}

/* C = -(dS/deps)^2 / (d2S/deps2) */
double so_heat_capacity(const so_params *P, double eps, double rho)
{
    (void)rho;
    double g = dS_deps(P, eps);
    return -(g * g) / d2S_deps2(P, eps);
}

/* internal energy with entropy S at density rho (the energy function of
 * Sec. 3.1): solve Cv ln eps - A kB ln(rho/rho0) = S for eps.             */
double so_eps_at_entropy(const so_params *P, double S, double rho)
{
    return exp((S + P->A * P->kB * log(rho / P->rho0)) / P->Cv);
}

/* ======================================================================= */
/* Cells and the pair schedule (not in the paper; reading A12)             */
/* ======================================================================= */

/* number of cells per axis: the requested value, else the largest even
 * integer not above box/h.  Must be even and >= 4 with box/ncell >= h.    */
int so_grid(const so_params *P, int32_t nc[3])
{
    for (int k = 0; k < 3; ++k) {
        int c = P->ncell[k];
        if (c <= 0) {
            c = (int)floor(P->box[k] / P->h);
            if (c % 2) c -= 1;
        }
        if (c < 4 || c % 2 || P->box[k] / c < P->h) return SO_EINVAL;
        nc[k] = c;
    }
    return SO_OK;
}

static int cell_coord(double x, double box, int nc)
{
    int c = (int)floor(x * ((double)nc / box));
    if (c < 0) c = 0;
    if (c > nc - 1) c = nc - 1;
    return c;
}

static int64_t cell_of(const so_params *P, const int32_t nc[3], const double *q,
                       int64_t n, int64_t i)
{
    int cx = cell_coord(q[i], P->box[0], nc[0]);
    int cy = cell_coord(q[n + i], P->box[1], nc[1]);
    int cz = cell_coord(q[2 * n + i], P->box[2], nc[2]);
    return cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
}

/* neighbour of cell c under offset index k in 0..26, offsets ordered with z
 * slowest: delta = (k%3 - 1, (k/3)%3 - 1, k/9 - 1); k = 13 is c itself.   */
static int64_t cell_neighbour(const int32_t nc[3], int64_t c, int k)
{
    int cx = (int)(c % nc[0]);
    int cy = (int)((c / nc[0]) % nc[1]);
    int cz = (int)(c / ((int64_t)nc[0] * nc[1]));
    cx = (cx + (k % 3 - 1) + nc[0]) % nc[0];
    cy = (cy + ((k / 3) % 3 - 1) + nc[1]) % nc[1];
    cz = (cz + (k / 9 - 1) + nc[2]) % nc[2];
    return cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
}

static int cell_parity(const int32_t nc[3], int64_t c)
{
    int cx = (int)(c % nc[0]);
    int cy = (int)((c / nc[0]) % nc[1]);
    int cz = (int)(c / ((int64_t)nc[0] * nc[1]));
    return (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
}

typedef struct { int64_t cell; uint32_t id; int64_t idx; } sortrec;

static int cmp_sortrec(const void *a, const void *b)
{
    const sortrec *x = (const sortrec *)a, *y = (const sortrec *)b;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static int permute_d(double *a, int64_t n, int ncomp, const sortrec *r)
{
    if (!a) return SO_OK;
    double *t = (double *)malloc(sizeof(double) * (size_t)(n * ncomp));
    if (!t) return SO_ENOMEM;
    for (int c = 0; c < ncomp; ++c)
        for (int64_t k = 0; k < n; ++k) t[c * n + k] = a[c * n + r[k].idx];
    memcpy(a, t, sizeof(double) * (size_t)(n * ncomp));
    free(t);
    return SO_OK;
}

/* Sort the particles by (cell, id) and fill cell_start[ncell + 1]; the slot
 * of a particle is its rank by id inside its cell.                        */
int so_build_cells(const so_params *P, double *q, double *p, double *eps,
                   double *rho, double *f, uint32_t *id, uint32_t *cell_start)
{
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    int64_t n = P->n, ncell = (int64_t)nc[0] * nc[1] * nc[2];
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(q[i])) return SO_ENONFINITE;
    sortrec *r = (sortrec *)malloc(sizeof(sortrec) * (size_t)(n ? n : 1));
    if (!r) return SO_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        r[i].cell = cell_of(P, nc, q, n, i);
        r[i].id = id[i];
        r[i].idx = i;
    }
    qsort(r, (size_t)n, sizeof(sortrec), cmp_sortrec);
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t k = 0; k < n; ++k) cell_start[r[k].cell + 1] += 1;
    int rc = SO_OK;
    for (int64_t c = 0; c < ncell; ++c) {
        if ((int64_t)cell_start[c + 1] > P->cell_cap) rc = SO_ECELLCAP;
        cell_start[c + 1] += cell_start[c];
    }
    int e = permute_d(q, n, 3, r);
    if (!e) e = permute_d(p, n, 3, r);
    if (!e) e = permute_d(eps, n, 1, r);
    if (!e) e = permute_d(rho, n, 1, r);
    if (!e) e = permute_d(f, n, 3, r);
    if (!e && id) {
        for (int64_t k = 0; k < n; ++k) id[k] = r[k].id;
    }
    free(r);
    return e ? e : rc;
}

/* minimum-image component of a displacement (reading A10) */
static double min_image(double d, double box)
{
    if (d > 0.5 * box) return d - box;
    if (d < -0.5 * box) return d + box;
    return d;
}

static double displacement(const so_params *P, const double *q, int64_t n,
                           int64_t i, int64_t j, double r[3])
{
    r[0] = min_image(q[i] - q[j], P->box[0]);
    r[1] = min_image(q[n + i] - q[n + j], P->box[1]);
    r[2] = min_image(q[2 * n + i] - q[2 * n + j], P->box[2]);
    return r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
}

/* ======================================================================= */
/* Density, eq. (sdpd-rho-v)                                               */
/* ======================================================================= */

/* rho_i = sum_j m W(r_ij), all j with r_ij < h including j = i (A3).
 * Candidates come from the 27 cells around i's cell.                      */
static double density_at(const so_params *P, const int32_t nc[3], const double *q,
                         const uint32_t *cell_start, int64_t i)
{
    int64_t n = P->n;
    double h2 = P->h * P->h;
    int64_t c = cell_of(P, nc, q, n, i);
    double rho = 0.0;
    for (int k = 0; k < 27; ++k) {
        int64_t c2 = cell_neighbour(nc, c, k);
        for (int64_t j = cell_start[c2]; j < cell_start[c2 + 1]; ++j) {
            double r[3];
            double r2 = displacement(P, q, n, i, j, r);
            if (r2 < h2) rho += P->m * so_kernel_w(P->kernel, P->h, sqrt(r2));
        }
    }
    return rho;
}

int so_density(const so_params *P, const double *q, const uint32_t *cell_start,
               double *rho_out)
{
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    for (int64_t i = 0; i < P->n; ++i) rho_out[i] = density_at(P, nc, q, cell_start, i);
    return SO_OK;
}

/* the same sum over all N particles, no cells (a pin for so_density) */
int so_density_bruteforce(const so_params *P, const double *q, double *rho_out)
{
    int64_t n = P->n;
    double h2 = P->h * P->h;
    for (int64_t i = 0; i < n; ++i) {
        double rho = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double r[3];
            double r2 = displacement(P, q, n, i, j, r);
            if (r2 < h2) rho += P->m * so_kernel_w(P->kernel, P->h, sqrt(r2));
        }
        rho_out[i] = rho;
    }
    return SO_OK;
}

/* Sec. 3.1: along the conservative dynamics the entropies S_i are invariant,
 * so after the positions move eps_i = E(S_i, rho_i(q)).                    */
static double eps_const_entropy(const so_params *P, double eps, double rho_old,
                                double rho_new)
{
    double S = so_entropy(P, eps, rho_old);
    return so_eps_at_entropy(P, S, rho_new);
}

int so_update_eps_const_entropy(const so_params *P, double *eps,
                                const double *rho_old, const double *rho_new)
{
    for (int64_t i = 0; i < P->n; ++i) {
        eps[i] = eps_const_entropy(P, eps[i], rho_old[i], rho_new[i]);
        if (!(eps[i] > 0.0) || !isfinite(eps[i])) return SO_ENONFINITE;
    }
    return SO_OK;
}

/* ======================================================================= */
/* Conservative forces, eq. (cons-forces)                                  */
/* ======================================================================= */

/* f_i = sum_{j != i} m^2 (P_i/rho_i^2 + P_j/rho_j^2) F_ij r_ij              */
static void force_on(const so_params *P, const double *q, const double *rho,
                     const double *eps, int64_t i, int64_t j, double acc[3])
{
    int64_t n = P->n;
    double r[3];
    double r2 = displacement(P, q, n, i, j, r);
    if (!(r2 < P->h * P->h)) return;
    double Pi = so_pressure(P, eps[i], rho[i]);
    double Pj = so_pressure(P, eps[j], rho[j]);
    double F = so_kernel_f(P->kernel, P->h, sqrt(r2));
    double s = P->m * P->m * (Pi / (rho[i] * rho[i]) + Pj / (rho[j] * rho[j])) * F;
    acc[0] += s * r[0];
    acc[1] += s * r[1];
    acc[2] += s * r[2];
}

static void force_at(const so_params *P, const int32_t nc[3], const double *q,
                     const double *rho, const double *eps, const uint32_t *cell_start,
                     int64_t i, double *f_out)
{
    int64_t n = P->n;
    int64_t c = cell_of(P, nc, q, n, i);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 27; ++k) {
        int64_t c2 = cell_neighbour(nc, c, k);
        for (int64_t j = cell_start[c2]; j < cell_start[c2 + 1]; ++j)
            if (j != i) force_on(P, q, rho, eps, i, j, acc);
    }
    f_out[i] = acc[0];
    f_out[n + i] = acc[1];
    f_out[2 * n + i] = acc[2];
}

int so_forces(const so_params *P, const double *q, const double *rho,
              const double *eps, const uint32_t *cell_start, double *f_out)
{
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    for (int64_t i = 0; i < P->n; ++i) force_at(P, nc, q, rho, eps, cell_start, i, f_out);
    return SO_OK;
}

int so_forces_bruteforce(const so_params *P, const double *q, const double *rho,
                         const double *eps, double *f_out)
{
    int64_t n = P->n;
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j)
            if (j != i) force_on(P, q, rho, eps, i, j, acc);
        f_out[i] = acc[0];
        f_out[n + i] = acc[1];
        f_out[2 * n + i] = acc[2];
    }
    return SO_OK;
}

/* ======================================================================= */
/* Random numbers (reading A17)                                            */
/* ======================================================================= */

/* Philox4x32-10 of Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplies with
 * a Weyl-sequence key schedule.                                           */
void so_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double word_to_open_unit(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* The Gaussian vector G (eq. ssa-ou) and the uniform U of the EMS accept
 * test for pair (i, j) at a given step: two Philox blocks with counter
 * (step, id_i, id_j, 2*replica + draw), Box-Muller on the first block.     */
void so_pair_draws(uint64_t seed, uint64_t step, uint32_t id_i, uint32_t id_j,
                   uint32_t replica, double G[3], double *U)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w0[4], w1[4];
    uint32_t c0[4] = {(uint32_t)step, id_i, id_j, replica * 2u + 0u};
    uint32_t c1[4] = {(uint32_t)step, id_i, id_j, replica * 2u + 1u};
    so_philox4x32_10(c0, key, w0);
    so_philox4x32_10(c1, key, w1);
    double u0 = word_to_open_unit(w0[0]), u1 = word_to_open_unit(w0[1]);
    double u2 = word_to_open_unit(w0[2]), u3 = word_to_open_unit(w0[3]);
    double R1 = sqrt(-2.0 * log(u0));
    double R2 = sqrt(-2.0 * log(u2));
    G[0] = R1 * cos(2.0 * SO_PI * u1);
    G[1] = R1 * sin(2.0 * SO_PI * u1);
    G[2] = R2 * cos(2.0 * SO_PI * u3);
    *U = word_to_open_unit(w1[0]);
}

/* ======================================================================= */
/* Fluctuation / dissipation, Sec. 2.2.2 and Sec. 3.2-3.3                   */
/* ======================================================================= */

/* alpha^theta and zeta^theta (theta = parallel, perpendicular) of
 * eq. (ssa-ou) from gamma, sigma of eq. (sdpd-gamma-sigma) and the kappas
 * of Sec. 2.2.2, evaluated at internal energies (eps_i, eps_j).            */
void so_fd_coefficients(const so_params *P, double F, double rho_i, double rho_j,
                        double eps_i, double eps_j, double dt,
                        double alpha[2], double zeta[2])
{
    double Ti = so_temperature(P, eps_i, rho_i), Tj = so_temperature(P, eps_j, rho_j);
    double Ci = so_heat_capacity(P, eps_i, rho_i), Cj = so_heat_capacity(P, eps_j, rho_j);
    double d = P->kB * Ti * Tj / ((Ti + Tj) * (Ti + Tj)) * (1.0 / Ci + 1.0 / Cj);
    double kappa[2];
    kappa[0] = (10.0 / 3.0 * P->eta + 4.0 * P->zeta) * P->m * P->m * F / (rho_i * rho_j);
    kappa[1] = (5.0 * P->eta / 3.0 - P->zeta) * P->m * P->m * F / (rho_i * rho_j);
    for (int t = 0; t < 2; ++t) {
        double gamma = kappa[t] * (1.0 - d);
        double sigma = 2.0 * sqrt(kappa[t] * P->kB * Ti * Tj / (Ti + Tj));
        alpha[t] = exp(-2.0 * gamma * dt / P->m);
        double one_minus_alpha2 = -expm1(-4.0 * gamma * dt / P->m);  /* A21 */
        zeta[t] = sigma * sqrt(P->m * one_minus_alpha2 / (4.0 * gamma));
    }
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Proposal of eq. (proposal) in relative-velocity form with noise (2/m) zeta
 * (reading A6), the energies of eq. (proposal-update), and the log of the
 * Metropolis ratio of eq. (metropolis-ratio):
 *   a = |G|^2/2 + log|B(v)| - (1/2) |B(v')^-1 (v - A(v') v')|^2 - log|B(v')|
 *       + sum_k [S_k(eps'_k) - S_k(eps_k)]/kB - log T_k(eps'_k) + log T_k(eps_k)
 * Returns a; fills vnew and eps_new.  Returns NAN when the proposed energies
 * are not positive (the ratio is undefined there).                         */
double so_fd_log_ratio(const so_params *P, double F, double rho_i, double rho_j,
                       double eps_i, double eps_j, const double v[3],
                       const double e[3], const double G[3], double dt,
                       double vnew[3], double eps_new[2])
{
    double alpha[2], zeta[2];
    so_fd_coefficients(P, F, rho_i, rho_j, eps_i, eps_j, dt, alpha, zeta);
    double b[2] = {2.0 / P->m * zeta[0], 2.0 / P->m * zeta[1]};
    double ve = dot3(v, e), Ge = dot3(G, e);
    for (int k = 0; k < 3; ++k) {
        double v_par = ve * e[k], v_perp = v[k] - ve * e[k];
        double G_par = Ge * e[k], G_perp = G[k] - Ge * e[k];
        vnew[k] = alpha[0] * v_par + alpha[1] * v_perp + b[0] * G_par + b[1] * G_perp;
    }
    double delta = P->m / 8.0 * (dot3(vnew, vnew) - dot3(v, v));
    eps_new[0] = eps_i - delta;
    eps_new[1] = eps_j - delta;
    if (!(eps_new[0] > 0.0 && eps_new[1] > 0.0)) return NAN;

    double alpha_r[2], zeta_r[2];
    so_fd_coefficients(P, F, rho_i, rho_j, eps_new[0], eps_new[1], dt, alpha_r, zeta_r);
    double b_r[2] = {2.0 / P->m * zeta_r[0], 2.0 / P->m * zeta_r[1]};
    /* w = v - A(v') v' */
    double vne = dot3(vnew, e), w[3];
    for (int k = 0; k < 3; ++k) {
        double par = vne * e[k], perp = vnew[k] - vne * e[k];
        w[k] = v[k] - (alpha_r[0] * par + alpha_r[1] * perp);
    }
    double we = dot3(w, e), quad = 0.0;
    for (int k = 0; k < 3; ++k) {
        double par = we * e[k], perp = w[k] - we * e[k];
        double y = par / b_r[0] + perp / b_r[1];   /* B(v')^-1 w */
        quad += y * y;
    }
    double logdetB = log(b[0]) + 2.0 * log(b[1]);
    double logdetB_r = log(b_r[0]) + 2.0 * log(b_r[1]);
    double a = 0.5 * dot3(G, G) + logdetB - 0.5 * quad - logdetB_r;
    a += (so_entropy(P, eps_new[0], rho_i) - so_entropy(P, eps_i, rho_i)) / P->kB
         - log(so_temperature(P, eps_new[0], rho_i)) + log(so_temperature(P, eps_i, rho_i));
    a += (so_entropy(P, eps_new[1], rho_j) - so_entropy(P, eps_j, rho_j)) / P->kB
         - log(so_temperature(P, eps_new[1], rho_j)) + log(so_temperature(P, eps_j, rho_j));
    return a;
}

/* margins inside which the GPU and the oracle may decide differently
 * because their elementary functions round differently (reading A16)       */
#define SO_MARGIN_RATIO 1e-9
#define SO_MARGIN_BOUND 1e-12

/* One EMS / AMS / SSA update of pair (i, j), Sec. 3.3.2 (the four steps of
 * the exact Metropolis scheme) and Sec. 3.3.3.  Returns the decision.
 * flip is a test control (reading A16): bit 0 inverts the outcome of the
 * energy bound, bit 1 the outcome of the Metropolis test, so that a check
 * can follow the other side's outcome of a test that lies inside the
 * rounding margin; the tests still run in their order (an inverted bound
 * rejection goes on to the ratio).  The arithmetic is the same either way. */
static int fd_pair(const so_params *P, const double *q, double *p, double *eps,
                   const double *rho, const uint32_t *id, int64_t i, int64_t j,
                   uint64_t step, double dt, so_stats *st, so_pairrec *rec, int flip)
{
    int64_t n = P->n;
    if (id[i] > id[j]) { int64_t t = i; i = j; j = t; }   /* A11 */
    double r[3];
    double r2 = displacement(P, q, n, i, j, r);
    double rl = sqrt(r2);
    double e[3] = {r[0] / rl, r[1] / rl, r[2] / rl};
    double F = so_kernel_f(P->kernel, P->h, rl);
    double G[3], U;
    so_pair_draws(P->seed, step, id[i], id[j], P->replica, G, &U);
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = p[k * n + i] / P->m - p[k * n + j] / P->m;

    double vnew[3], eps_new[2];
    double alpha[2], zeta[2];
    so_fd_coefficients(P, F, rho[i], rho[j], eps[i], eps[j], dt, alpha, zeta);
    double b[2] = {2.0 / P->m * zeta[0], 2.0 / P->m * zeta[1]};
    double ve = dot3(v, e), Ge = dot3(G, e);
    for (int k = 0; k < 3; ++k) {
        double v_par = ve * e[k], v_perp = v[k] - ve * e[k];
        double G_par = Ge * e[k], G_perp = G[k] - Ge * e[k];
        vnew[k] = alpha[0] * v_par + alpha[1] * v_perp + b[0] * G_par + b[1] * G_perp;
    }
    double delta = P->m / 8.0 * (dot3(vnew, vnew) - dot3(v, v));
    eps_new[0] = eps[i] - delta;
    eps_new[1] = eps[j] - delta;
    double emin = eps[i] < eps[j] ? eps[i] : eps[j];
    double gap = emin - delta;

    int decision = 0;
    double amlu = 0.0;
    st->proposed += 1;
    if (P->fd_mode == SO_FD_SSA) {
        if (!(eps_new[0] > 0.0 && eps_new[1] > 0.0)) st->negeps += 1;
    } else if ((emin > delta) == ((flip & 1) != 0)) {   /* eq. (energy-bound) */
        decision = 1;
    } else if (P->fd_mode == SO_FD_EMS) {
        double vn2[3], en2[2];
        double a = so_fd_log_ratio(P, F, rho[i], rho[j], eps[i], eps[j], v, e, G, dt,
                                   vn2, en2);
        amlu = a - log(U);
        if (fabs(amlu) <= SO_MARGIN_RATIO) st->marginal += 1;
        if ((U > exp(a)) != ((flip & 2) != 0)) decision = 2;   /* reject iff U > A */
    }
    if (P->fd_mode != SO_FD_SSA && fabs(gap) <= SO_MARGIN_BOUND * fmax(fabs(emin), fabs(delta)))
        st->marginal += 1;
    if (decision == 1) st->rej_energy += 1;
    if (decision == 2) st->rej_ratio += 1;
    if (decision == 0) {                               /* eq. (proposal-update) */
        for (int k = 0; k < 3; ++k) {
            double dp = P->m / 2.0 * (vnew[k] - v[k]);
            p[k * n + i] += dp;
            p[k * n + j] -= dp;
        }
        eps[i] = eps_new[0];
        eps[j] = eps_new[1];
    }
    if (rec) {
        rec->i = (int32_t)i;
        rec->j = (int32_t)j;
        rec->decision = decision;
        rec->a_minus_lnU = amlu;
        rec->bound_gap = gap;
    }
    return decision;
}

/* The sequential order of the pair updates (reading A12).  The paper applies
 * pairs one after the other in an unspecified order (Sec. 3.2).  Here every
 * active pair gets the key (phase, round):
 *   phase 0        pairs inside one cell; round = slot_a XOR slot_b;
 *   phase 1+8o+pi  pairs between cell A and cell A + delta_o, o = 0..12 the
 *                  13 offsets after the centre of the z-slowest 27-list,
 *                  pi the parity bits (x | y<<1 | z<<2) of A's coordinates;
 *                  round = slot in A XOR slot in A + delta_o.
 * Pairs are applied in ascending (phase, round); pairs with equal keys share
 * no particle, so their mutual order does not matter.                     */
typedef struct { int32_t phase, round; int64_t i, j; } pairkey;

static int cmp_pairkey(const void *a, const void *b)
{
    const pairkey *x = (const pairkey *)a, *y = (const pairkey *)b;
    if (x->phase != y->phase) return x->phase < y->phase ? -1 : 1;
    if (x->round != y->round) return x->round < y->round ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

static int build_pairs(const so_params *P, const double *q, const uint32_t *cell_start,
                       pairkey **out, int64_t *count)
{
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    int64_t n = P->n, ncell = (int64_t)nc[0] * nc[1] * nc[2];
    double h2 = P->h * P->h;
    int64_t cap = 1024, cnt = 0;
    pairkey *list = (pairkey *)malloc(sizeof(pairkey) * (size_t)cap);
    if (!list) return SO_ENOMEM;
    for (int64_t A = 0; A < ncell; ++A) {
        for (int k = 13; k < 27; ++k) {
            int64_t B = cell_neighbour(nc, A, k);
            for (int64_t i = cell_start[A]; i < cell_start[A + 1]; ++i) {
                for (int64_t j = cell_start[B]; j < cell_start[B + 1]; ++j) {
                    if (k == 13 && j <= i) continue;
                    double r[3];
                    if (!(displacement(P, q, n, i, j, r) < h2)) continue;
                    if (cnt == cap) {
                        cap *= 2;
                        pairkey *t = (pairkey *)realloc(list, sizeof(pairkey) * (size_t)cap);
                        if (!t) { free(list); return SO_ENOMEM; }
                        list = t;
                    }
                    int slot_a = (int)(i - cell_start[A]), slot_b = (int)(j - cell_start[B]);
                    list[cnt].phase = (k == 13) ? 0 : 1 + 8 * (k - 14) + cell_parity(nc, A);
                    list[cnt].round = slot_a ^ slot_b;
                    list[cnt].i = i;
                    list[cnt].j = j;
                    ++cnt;
                }
            }
        }
    }
    qsort(list, (size_t)cnt, sizeof(pairkey), cmp_pairkey);
    *out = list;
    *count = cnt;
    return SO_OK;
}

int so_fd_pair_list(const so_params *P, const double *q, const uint32_t *cell_start,
                    so_pairrec *out, int64_t cap, int64_t *count)
{
    pairkey *list = NULL;
    int64_t cnt = 0;
    int rc = build_pairs(P, q, cell_start, &list, &cnt);
    if (rc) return rc;
    *count = cnt;
    for (int64_t k = 0; k < cnt && k < cap; ++k) {
        memset(&out[k], 0, sizeof(so_pairrec));
        out[k].phase = list[k].phase;
        out[k].round = list[k].round;
        out[k].i = (int32_t)list[k].i;
        out[k].j = (int32_t)list[k].j;
    }
    free(list);
    return cnt > cap ? SO_EINVAL : SO_OK;
}

/* One fluctuation/dissipation sweep: every active pair once, in key order.
 * The pairs at positions flip_pos[0..nflip) of that order (ascending; may be
 * NULL) take the test inversions flip_kind[] (see fd_pair).                */
static int fd_sweep(const so_params *P, const double *q, double *p, double *eps,
                    const double *rho, const uint32_t *id, const uint32_t *cell_start,
                    uint64_t step, double dt_fd, so_stats *st, so_pairrec *log,
                    int64_t log_cap, const int64_t *flip_pos, const int32_t *flip_kind,
                    int64_t nflip)
{
    if (P->fd_mode == SO_FD_NONE) return SO_OK;
    pairkey *list = NULL;
    int64_t cnt = 0;
    int rc = build_pairs(P, q, cell_start, &list, &cnt);
    if (rc) return rc;
    int64_t next = 0;
    for (int64_t k = 0; k < cnt; ++k) {
        so_pairrec *rec = (log && k < log_cap) ? &log[k] : NULL;
        if (rec) {
            rec->phase = list[k].phase;
            rec->round = list[k].round;
        }
        int f = 0;
        while (next < nflip && flip_pos[next] < k) ++next;
        if (next < nflip && flip_pos[next] == k) f = flip_kind[next];
        fd_pair(P, q, p, eps, rho, id, list[k].i, list[k].j, step, dt_fd, st, rec, f);
    }
    free(list);
    return st->negeps ? SO_ENEGEPS : SO_OK;
}

int so_fd_sweep(const so_params *P, const double *q, double *p, double *eps,
                const double *rho, const uint32_t *id, const uint32_t *cell_start,
                uint64_t step, double dt_fd, so_stats *st,
                so_pairrec *log, int64_t log_cap)
{
    return fd_sweep(P, q, p, eps, rho, id, cell_start, step, dt_fd, st, log, log_cap, NULL, NULL,
                    0);
}

int so_fd_sweep_flip(const so_params *P, const double *q, double *p, double *eps,
                     const double *rho, const uint32_t *id, const uint32_t *cell_start,
                     uint64_t step, double dt_fd, so_stats *st,
                     so_pairrec *log, int64_t log_cap, const int64_t *flip_pos,
                     const int32_t *flip_kind, int64_t nflip)
{
    for (int64_t k = 0; k < nflip; ++k)
        if ((k > 0 && flip_pos[k] <= flip_pos[k - 1]) || flip_kind[k] < 0 || flip_kind[k] > 3)
            return SO_EINVAL;
    return fd_sweep(P, q, p, eps, rho, id, cell_start, step, dt_fd, st, log, log_cap, flip_pos,
                    flip_kind, nflip);
}

/* ======================================================================= */
/* Velocity-Verlet, eq. (sdpd-verlet), and observables                      */
/* ======================================================================= */

int so_kick(const so_params *P, double *p, const double *f, double half_dt)
{
    for (int64_t k = 0; k < 3 * P->n; ++k) p[k] += half_dt * f[k];
    return SO_OK;
}

/* q <- q + dt p / m, then each coordinate wrapped once into [0, box) */
int so_drift(const so_params *P, double *q, const double *p, double dt)
{
    int64_t n = P->n;
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) {
            double x = q[c * n + i] + dt * p[c * n + i] / P->m;
            if (x >= P->box[c]) x -= P->box[c];
            else if (x < 0.0) x += P->box[c];
            q[c * n + i] = x;
        }
    return SO_OK;
}

/* total energy E = sum_i eps_i + p_i^2/(2m) (Sec. 2.2.1), momentum, ... */
int so_observe(const so_params *P, const double *p, const double *eps, so_stats *st)
{
    int64_t n = P->n;
    double Eint = 0.0, KE = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0, mn = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        Eint += eps[i];
        KE += (p[i] * p[i] + p[n + i] * p[n + i] + p[2 * n + i] * p[2 * n + i]) / (2.0 * P->m);
        Px += p[i];
        Py += p[n + i];
        Pz += p[2 * n + i];
        if (eps[i] < mn) mn = eps[i];
    }
    st->Eint = Eint;
    st->KE = KE;
    st->E = Eint + KE;
    st->P[0] = Px; st->P[1] = Py; st->P[2] = Pz;
    st->min_eps = mn;
    return SO_OK;
}

/* nsteps full steps in the order of reading A13.  On entry rho and f must
 * belong to q (density without energy update, then forces).               */
int so_step(const so_params *P, double *q, double *p, double *eps, double *rho,
            double *f, uint32_t *id, uint32_t *cell_start, uint64_t step0,
            int nsteps, so_stats *per_step)
{
    int64_t n = P->n;
    int theta = P->fd_every > 0 ? P->fd_every : 1;
    double *rho_new = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    if (!rho_new) return SO_ENOMEM;
    int rc = SO_OK;
    for (int s = 0; s < nsteps && rc == SO_OK; ++s) {
        uint64_t step = step0 + (uint64_t)s;
        so_stats st;
        memset(&st, 0, sizeof st);
        so_kick(P, p, f, 0.5 * P->dt);
        so_drift(P, q, p, P->dt);
        rc = so_build_cells(P, q, p, eps, rho, f, id, cell_start);
        if (rc) break;
        so_density(P, q, cell_start, rho_new);
        rc = so_update_eps_const_entropy(P, eps, rho, rho_new);
        memcpy(rho, rho_new, sizeof(double) * (size_t)n);
        if (rc) break;
        if (step % (uint64_t)theta == 0)
            rc = so_fd_sweep(P, q, p, eps, rho, id, cell_start, step, theta * P->dt, &st,
                             NULL, 0);
        so_forces(P, q, rho, eps, cell_start, f);
        so_kick(P, p, f, 0.5 * P->dt);
        so_observe(P, p, eps, &st);
        if (per_step) per_step[s] = st;
    }
    free(rho_new);
    return rc;
}

/* ======================================================================= */
/* Parallel variant of the step (the CPU baseline on many cores)           */
/* ======================================================================= */

/* The same step as so_step with the independent work spread over OpenMP
 * threads: density, energy update and forces per particle (each sum in the
 * order above), and the F/D sweep phase by phase.  Inside one phase the
 * tasks -- a cell (phase 0) or a cell pair (A, A + delta_o) -- share no
 * particle (reading A12), so they run concurrently; each task applies its
 * own pairs in (round, i) order, which is the order so_fd_sweep applies
 * them in (its keys (phase, round, i) are distinct, and pairs of other
 * tasks of the phase touch other particles).  The result is the serial one
 * bit for bit.  Compiled without OpenMP it runs on one thread.            */
#ifdef _OPENMP
#include <omp.h>
#endif

int so_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static int cmp_roundkey(const void *a, const void *b)
{
    const pairkey *x = (const pairkey *)a, *y = (const pairkey *)b;
    if (x->round != y->round) return x->round < y->round ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/* the active pairs of task (A, offset k) in (round, i) order; returns the
 * count (at most 64 * 64) */
static int64_t task_pairs(const so_params *P, const int32_t nc[3], const double *q,
                          const uint32_t *cell_start, int64_t A, int k, pairkey *out)
{
    int64_t n = P->n, cnt = 0;
    double h2 = P->h * P->h;
    int64_t B = cell_neighbour(nc, A, k);
    for (int64_t i = cell_start[A]; i < cell_start[A + 1]; ++i) {
        for (int64_t j = cell_start[B]; j < cell_start[B + 1]; ++j) {
            if (k == 13 && j <= i) continue;
            double r[3];
            if (!(displacement(P, q, n, i, j, r) < h2)) continue;
            out[cnt].phase = 0;
            out[cnt].round = (int32_t)((i - cell_start[A]) ^ (j - cell_start[B]));
            out[cnt].i = i;
            out[cnt].j = j;
            ++cnt;
        }
    }
    qsort(out, (size_t)cnt, sizeof(pairkey), cmp_roundkey);
    return cnt;
}

static int fd_sweep_parallel(const so_params *P, const double *q, double *p, double *eps,
                             const double *rho, const uint32_t *id,
                             const uint32_t *cell_start, uint64_t step, double dt_fd,
                             so_stats *st)
{
    if (P->fd_mode == SO_FD_NONE) return SO_OK;
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    uint64_t proposed = 0, rej_energy = 0, rej_ratio = 0, marginal = 0, negeps = 0;
    int fail = 0;
    for (int phase = 0; phase < 105; ++phase) {
        int k = phase == 0 ? 13 : 14 + (phase - 1) / 8;
        int par = phase == 0 ? -1 : (phase - 1) % 8;
#pragma omp parallel reduction(+ : proposed, rej_energy, rej_ratio, marginal, negeps) \
    reduction(| : fail)
        {
            pairkey *buf = (pairkey *)malloc(sizeof(pairkey) * 64 * 64);
            so_stats ts;
            memset(&ts, 0, sizeof ts);
            if (!buf) fail = 1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t A = 0; A < ncell; ++A) {
                if (!buf || (par >= 0 && cell_parity(nc, A) != par)) continue;
                int64_t cnt = task_pairs(P, nc, q, cell_start, A, k, buf);
                for (int64_t e = 0; e < cnt; ++e)
                    fd_pair(P, q, p, eps, rho, id, buf[e].i, buf[e].j, step, dt_fd, &ts, NULL,
                            0);
            }
            free(buf);
            proposed += ts.proposed;
            rej_energy += ts.rej_energy;
            rej_ratio += ts.rej_ratio;
            marginal += ts.marginal;
            negeps += ts.negeps;
        }
    }
    st->proposed += proposed;
    st->rej_energy += rej_energy;
    st->rej_ratio += rej_ratio;
    st->marginal += marginal;
    st->negeps += negeps;
    if (fail) return SO_ENOMEM;
    return st->negeps ? SO_ENEGEPS : SO_OK;
}

int so_step_parallel(const so_params *P, double *q, double *p, double *eps, double *rho,
                     double *f, uint32_t *id, uint32_t *cell_start, uint64_t step0,
                     int nsteps, so_stats *per_step)
{
    int32_t nc[3];
    if (so_grid(P, nc)) return SO_EINVAL;
    int64_t n = P->n;
    int theta = P->fd_every > 0 ? P->fd_every : 1;
    double *rho_new = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    if (!rho_new) return SO_ENOMEM;
    int rc = SO_OK;
    for (int s = 0; s < nsteps && rc == SO_OK; ++s) {
        uint64_t step = step0 + (uint64_t)s;
        so_stats st;
        memset(&st, 0, sizeof st);
        so_kick(P, p, f, 0.5 * P->dt);
        so_drift(P, q, p, P->dt);
        rc = so_build_cells(P, q, p, eps, rho, f, id, cell_start);
        if (rc) break;
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t i = 0; i < n; ++i) {
            rho_new[i] = density_at(P, nc, q, cell_start, i);
            eps[i] = eps_const_entropy(P, eps[i], rho[i], rho_new[i]);
            if (!(eps[i] > 0.0) || !isfinite(eps[i])) bad = 1;
        }
        memcpy(rho, rho_new, sizeof(double) * (size_t)n);
        if (bad) {
            rc = SO_ENONFINITE;
            break;
        }
        if (step % (uint64_t)theta == 0)
            rc = fd_sweep_parallel(P, q, p, eps, rho, id, cell_start, step, theta * P->dt, &st);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) force_at(P, nc, q, rho, eps, cell_start, i, f);
        so_kick(P, p, f, 0.5 * P->dt);
        so_observe(P, p, eps, &st);
        if (per_step) per_step[s] = st;
    }
    free(rho_new);
    return rc;
}
