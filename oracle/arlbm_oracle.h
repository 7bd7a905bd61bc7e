/*
 * Plain FP64 CPU oracle for the adaptive-relaxation, Lax-Friedrichs-type
 * equilibrium vector lattice Boltzmann method (Zhang, Lin, Zhao, Zhao,
 * "A Lattice Boltzmann Method with Adaptive Relaxation Parameter and
 * Lax-Friedrichs-Type Equilibrium for Hyperbolic Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library: it is written straight from the paper, slowly and
 * plainly, to be checked by eye against Sections 2.1-2.3.
 *
 * Parity pins: every function here is pinned by a CPU test against closed
 * forms, printed tables or textbook special cases (see tests/test_oracle_*.py).
 * The shallow-water bed source is not in the paper; its discretisation is a
 * documented reading and is pinned only by conservation, lake-at-rest
 * convergence and symmetry.
 */
#ifndef ARLBM_ORACLE_H
#define ARLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_ADVECTION = 0, ORA_EULER = 1, ORA_SWE = 2, ORA_REACTIVE = 3 };
#define ORA_MMAX 6 /* most conserved fields: 3D reactive Euler */
enum { ORA_PERIODIC = 0, ORA_TRANSMISSIVE = 1, ORA_REFLECTIVE = 2 };

typedef struct ora_cfg {
    int32_t system;     /* ORA_ADVECTION / ORA_EULER / ORA_SWE / ORA_REACTIVE */
    int32_t dim;        /* 1, 2 or 3                                         */
    int32_t nx, ny;     /* cells; ny == 1 in 1D                              */
    double x0, x1, y0, y1;
    int32_t bc[4];      /* x-lo, x-hi, y-lo, y-hi                            */
    double cfl;         /* CFL number of eq. (2.21)                          */
    double eps;         /* alpha_j = alpha_bar_j + eps (Section 2.3)         */
    double gamma;       /* Euler ratio of specific heats                     */
    double g;           /* gravity for shallow water                         */
    double adv[3];      /* advection velocity per direction                  */
    double h_dry;       /* shallow-water dry threshold                       */
    double rho_floor, p_floor;
    int32_t has_bed;    /* shallow-water bed-slope source                    */
    int32_t omega_fixed_on;   /* 1: omega == omega_fixed everywhere          */
    double omega_fixed;
    /* reactive Euler (Section 5.4): heat release q, rate constant K and
     * activation temperature T_i of the Arrhenius rate R = K rho Y
     * exp(-T_i / T), T = p / rho */
    double q_heat, k_rate, t_act;
    /* third dimension (D3Q7): cells nz (1 below 3D), extent [z0, z1] with
     * (z1 - z0)/nz equal to dx, boundaries z-lo, z-hi */
    int32_t nz;
    double z0, z1;
    int32_t bc_z[2];
} ora_cfg;

typedef struct ora_lattice ora_lattice;

/* Number of conserved fields m for a system in dimension d. */
int ora_num_fields(int system, int dim);

/* Lattice life cycle. U0 is m planes [c][z][y][x] of conserved variables at cell
 * centres; bed is one plane [y][x] (or NULL).  Returns NULL on bad input. */
ora_lattice *ora_create(const ora_cfg *cfg);
void ora_destroy(ora_lattice *L);
int ora_init(ora_lattice *L, const double *U0, const double *bed, double t0);

/* Advance up to nsteps steps; when t_final > 0, stepping also stops at the
 * first step that reaches t >= t_final (whole steps, none shortened).
 * Returns the number of steps taken, or a negative error code (-1: the sum of
 * alpha_bar is zero, so the time step is undefined). */
int64_t ora_run(ora_lattice *L, int64_t nsteps, double t_final);

/* Read-back of the state. */
void ora_moments(const ora_lattice *L, double *U);       /* m planes       */
void ora_get_f(const ora_lattice *L, double *f);         /* Q*m planes     */
void ora_set_f(ora_lattice *L, const double *f);
void ora_last_omega(const ora_lattice *L, double *omega);/* 1 plane        */
double ora_time(const ora_lattice *L);
int ora_threads(void); /* threads of a parallel region (1: single-threaded build) */
int64_t ora_steps(const ora_lattice *L);
void ora_last_scalars(const ora_lattice *L, double *abar3, double *dt);
int32_t ora_flags(const ora_lattice *L);

/* Pieces of one step, exposed for the pin tests. */
/* omega field that the next step would use, from the current state. */
void ora_omega_field(ora_lattice *L, double *omega);
/* nu on the interior cells, from the current state. */
void ora_nu_field(ora_lattice *L, double *nu);
/* alpha_bar_j (eq. 2.19) of the current state; returns d values. */
void ora_alpha_bar(const ora_lattice *L, double *abar);

/* Per-state system functions (Section 2 and Section 5 systems). */
void ora_flux(const ora_cfg *c, int dir, const double *U, double *F);
double ora_max_speed(const ora_cfg *c, int dir, const double *U);
void ora_left_eigvecs(const ora_cfg *c, int dir, const double *U, double *L);
/* Source S(U) of the system (shallow-water bed slopes db = (b_x, b_y) are
 * ignored by the other systems). */
void ora_source(const ora_cfg *c, const double *U, const double *db, double *S);
/* Implicit moment update (2.8) of one cell: U = sumF + (dt/2) S(U). */
void ora_moment_update(const ora_cfg *c, const double *sumF, const double *db, double half_dt,
                       double *U);
/* Lax-Friedrichs-type equilibrium coefficients a_k, b_kj of eq. (2.20)
 * written in the general form (2.5): b is Q x d row-major. */
void ora_lf_coeffs(int dim, const double *alpha, double lambda, double *a,
                   double *b);
/* f^eq_k(U) of eq. (2.5) for all k: out is Q x m row-major. */
void ora_equilibrium(const ora_cfg *c, const double *U, const double *alpha,
                     double lambda, double *feq);

#ifdef __cplusplus
}
#endif
#endif
