/*
 * Plain FP64 CPU oracle of the adaptive-relaxation, Lax-Friedrichs-type
 * equilibrium vector LBM (Sections 2.1-2.3 of the paper).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
 * code with the GPU path.  Built with -O2 -ffp-contract=off, no fast-math.
 *
 * The oracle follows the paper's order of operations for one time step:
 *   moments (2.3) -> wave-speed bounds (2.19) and time step (2.21) ->
 *   characteristic projections and indicator (2.13)-(2.14) -> box sum (2.15)
 *   -> relaxation parameter (2.16) -> Lax-Friedrichs-type equilibrium (2.20)
 *   in the general form (2.5) with source split (2.6) -> collision at the
 *   source node and pull streaming (the implementation form after (2.7)) ->
 *   implicit moment update (2.8) -> second half source.
 *
 * Readings where the paper is silent:
 *   - left eigenvectors: L = R^{-1}, R with first component 1 in every
 *     acoustic/entropy column, shear columns (0,..,1,..) (Toro's form);
 *   - boundaries: ghost cells by a mirror index map U(-1-i) <- U(i) (depth 2
 *     for U, depth 1 for the collided populations); reflective walls negate
 *     the normal momentum and swap the mirrored population;
 *   - alpha_bar is recomputed every step from U^n; a run with a final time
 *     takes whole steps until t >= T (the last step is not shortened: a
 *     shortened step changes lambda abruptly and, with omega near 2, breaks
 *     the second-order accuracy that the paper's tables show);
 *   - the second half source uses the same step's a_k and delta t;
 *   - shallow water: a cell with h <= h_dry has u = v = 0 and zero momentum
 *     flux; the acoustic speed in L uses max(h, h_dry);
 *   - bed source S = (0, -g h db/dx, -g h db/dy), central differences of the
 *     cell-centred bed with mirrored ghosts (not in the paper);
 *   - reactive Euler (Section 5.4): with E' = E - q rho Y the system is Euler
 *     in (rho, m, E') plus the passively advected rho Y, so L = L' T where
 *     L' holds the Euler rows (zero in the rho Y column) and the species row
 *     (-Y, 0, .., 0, 1), and T maps U to (rho, m, E - q rho Y, rho Y);
 *   - reactive Euler: (2.8) reduces to one scalar equation for rho Y whose
 *     root lies in [min(0,B), max(0,B)], B = sum_k F_k of rho Y (the sink
 *     R >= 0 for rho Y >= 0 puts it there); the oracle brackets it by the
 *     Illinois variant of regula falsi until the bracket is two adjacent
 *     doubles, and the Arrhenius factor uses the C library's exp.
 *
 * Built once single-threaded (the reference timing and every test) and once
 * with OpenMP over rows (the benchmark's all-core timing): every cell's
 * arithmetic is the same in both and the only reduction is a maximum, so the
 * two builds give the same bits.
 */
#include "arlbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define G2 2 /* ghost depth of the padded moment array */

struct ora_lattice {
    ora_cfg c;
    int d, m, Q, nx, ny, nz, ncell;
    double dx;
    double *f;      /* [k][c][z][y][x], Q*m*ncell                    */
    double *bed;    /* [y][x] or NULL                                */
    double *dbed;   /* [dir][y][x] central-difference bed gradient   */
    double *omega;  /* omega used by the last step                   */
    double *Up;     /* padded moments, ghost depth 2, m planes       */
    double *nup;    /* padded nu, ghost depth 1                      */
    double *fs;     /* padded collided populations, ghost depth 1    */
    double t;
    int64_t steps;
    double last_abar[3], last_dt;
    int32_t flags;
};

/* ------------------------------------------------------------------------ */
/* The physical systems (Section 5): flux, eigenvalue bound, left           */
/* eigenvectors L_j = R_j^{-1} of the flux Jacobian in direction j.         */
/* ------------------------------------------------------------------------ */

int ora_num_fields(int system, int dim)
{
    if (system == ORA_ADVECTION) return 1;
    if (system == ORA_EULER) return dim + 2;
    if (system == ORA_SWE) return dim + 1;
    if (system == ORA_REACTIVE) return dim + 3;
    return 0;
}

typedef struct {
    double rho, vel[3], mom[3], E, p, c; /* Euler: rho; SWE: h in rho */
    double cL;                           /* SWE: speed used in L      */
    double Z, Y;                         /* reactive: rho Y and Y     */
} prim_t;

static void primitives(const ora_cfg *c, const double *U, prim_t *P, int32_t *flags)
{
    int d = c->dim;
    memset(P, 0, sizeof(*P));
    if (c->system == ORA_EULER || c->system == ORA_REACTIVE) {
        P->rho = U[0];
        P->E = U[d + 1];
        for (int i = 0; i < d; ++i) {
            P->mom[i] = U[1 + i];
            P->vel[i] = U[1 + i] / P->rho;
        }
        double q2 = P->vel[0] * P->vel[0] + P->vel[1] * P->vel[1];
        if (d == 3) q2 = q2 + P->vel[2] * P->vel[2];
        if (c->system == ORA_EULER) {
            P->p = (c->gamma - 1.0) * (P->E - 0.5 * P->rho * q2);
        } else {
            /* rho E = p/(gamma-1) + rho |u|^2 / 2 + q rho Y (Section 5.4) */
            P->Z = U[d + 2];
            P->Y = P->Z / P->rho;
            P->p = (c->gamma - 1.0) * ((P->E - 0.5 * P->rho * q2) - c->q_heat * P->Z);
        }
        double pf = P->p > c->p_floor ? P->p : c->p_floor;
        double rf = P->rho > c->rho_floor ? P->rho : c->rho_floor;
        if (flags && (P->p <= c->p_floor || P->rho <= c->rho_floor)) *flags |= 2;
        P->c = sqrt(c->gamma * pf / rf);
    } else if (c->system == ORA_SWE) {
        double h = U[0];
        P->rho = h;
        int wet = h > c->h_dry;
        for (int i = 0; i < d; ++i) {
            P->mom[i] = wet ? U[1 + i] : 0.0;
            P->vel[i] = wet ? U[1 + i] / h : 0.0;
        }
        if (flags && h < 0.0) *flags |= 2;
        P->c = sqrt(c->g * (h > 0.0 ? h : 0.0));
        P->cL = sqrt(c->g * (h > c->h_dry ? h : c->h_dry));
    }
}

void ora_flux(const ora_cfg *c, int dir, const double *U, double *F)
{
    int d = c->dim;
    if (c->system == ORA_ADVECTION) {
        F[0] = c->adv[dir] * U[0];
        return;
    }
    prim_t P;
    primitives(c, U, &P, NULL);
    if (c->system == ORA_EULER || c->system == ORA_REACTIVE) {
        F[0] = P.mom[dir];
        for (int i = 0; i < d; ++i)
            F[1 + i] = P.mom[dir] * P.vel[i] + (i == dir ? P.p : 0.0);
        F[d + 1] = P.vel[dir] * (P.E + P.p);
        if (c->system == ORA_REACTIVE) F[d + 2] = P.vel[dir] * P.Z;
    } else {
        double ph = 0.5 * c->g * P.rho * P.rho;
        F[0] = P.mom[dir];
        for (int i = 0; i < d; ++i)
            F[1 + i] = P.mom[dir] * P.vel[i] + (i == dir ? ph : 0.0);
    }
}

/* max_r |lambda^(r)(dF_dir/dU)|: |a| for advection, |u_n| + c otherwise. */
double ora_max_speed(const ora_cfg *c, int dir, const double *U)
{
    if (c->system == ORA_ADVECTION) return fabs(c->adv[dir]);
    prim_t P;
    primitives(c, U, &P, NULL);
    return fabs(P.vel[dir]) + P.c;
}

void ora_left_eigvecs(const ora_cfg *c, int dir, const double *U, double *L)
{
    int d = c->dim, m = ora_num_fields(c->system, d);
    for (int i = 0; i < m * m; ++i) L[i] = 0.0;
    if (c->system == ORA_ADVECTION) {
        L[0] = 1.0;
        return;
    }
    prim_t P;
    primitives(c, U, &P, NULL);
    if (c->system == ORA_EULER || c->system == ORA_REACTIVE) {
        double cs = P.c;
        double q2 = P.vel[0] * P.vel[0] + P.vel[1] * P.vel[1];
        if (d == 3) q2 = q2 + P.vel[2] * P.vel[2];
        double b1 = (c->gamma - 1.0) / (cs * cs);
        double b2 = 0.5 * q2 * b1;
        double un = P.vel[dir];
        int n = 1 + dir;          /* normal-momentum column           */
        int e = d + 1;            /* energy column                     */
        /* row 0: u_n - c;  row 1: entropy (u_n);  row m-1: u_n + c */
        L[0 * m + 0] = 0.5 * (b2 + un / cs);
        L[(m - 1) * m + 0] = 0.5 * (b2 - un / cs);
        L[1 * m + 0] = 1.0 - b2;
        for (int i = 0; i < d; ++i) {
            double vi = P.vel[i];
            if (1 + i == n) {
                L[0 * m + n] = -0.5 * (b1 * un + 1.0 / cs);
                L[(m - 1) * m + n] = -0.5 * (b1 * un - 1.0 / cs);
            } else {
                L[0 * m + 1 + i] = -0.5 * b1 * vi;
                L[(m - 1) * m + 1 + i] = -0.5 * b1 * vi;
            }
            L[1 * m + 1 + i] = b1 * vi;
        }
        L[0 * m + e] = 0.5 * b1;
        L[(m - 1) * m + e] = 0.5 * b1;
        L[1 * m + e] = -b1;
        /* shear rows (u_n), one per tangential direction t in increasing
         * order: -v_t, unit weight on the tangential momentum */
        for (int t = 0, r = 2; t < d; ++t) {
            if (t == dir) continue;
            L[r * m + 0] = -P.vel[t];
            L[r * m + 1 + t] = 1.0;
            ++r;
        }
        if (c->system == ORA_REACTIVE) {
            /* species row m-2 (speed u_n): (-Y, 0, .., 0, 1) in the variables
             * (rho, m, E', rho Y); then every row times T: the rho Y entry
             * gains -q times the energy entry */
            int z = d + 2;
            L[(m - 2) * m + 0] = -P.Y;
            L[(m - 2) * m + z] = 1.0;
            for (int r = 0; r < m; ++r) L[r * m + z] = L[r * m + z] - c->q_heat * L[r * m + e];
        }
    } else {
        double cs = P.cL;
        double un = P.vel[dir];
        int n = 1 + dir;
        L[0 * m + 0] = (un + cs) / (2.0 * cs);
        L[0 * m + n] = -1.0 / (2.0 * cs);
        L[(m - 1) * m + 0] = -(un - cs) / (2.0 * cs);
        L[(m - 1) * m + n] = 1.0 / (2.0 * cs);
        if (d == 2) {
            int t = 1 - dir;
            L[1 * m + 0] = -P.vel[t];
            L[1 * m + 1 + t] = 1.0;
        }
    }
}

/* Source S(U) (2.1): the shallow-water bed slope, which depends on U through
 * the depth alone, so (2.8) is solved in closed form; and the Arrhenius sink
 * of the reactive system, S = (0, .., 0, -R), R = K rho Y exp(-T_i / T),
 * T = p / rho (Section 5.4). */
static int has_bed(const ora_cfg *c) { return c->system == ORA_SWE && c->has_bed; }

/* The Arrhenius rate R at rho Y = z, with rho and (E - rho |u|^2/2) fixed
 * (p depends on z through -q z). */
static double arrhenius(const ora_cfg *c, double rho, double e_int, double z)
{
    double p = (c->gamma - 1.0) * (e_int - c->q_heat * z);
    double pf = p > c->p_floor ? p : c->p_floor;
    double rf = rho > c->rho_floor ? rho : c->rho_floor;
    double T = pf / rf;
    return (c->k_rate * z) * exp(-(c->t_act / T));
}

static void reactive_parts(const ora_cfg *c, const double *U, double *rho, double *e_int)
{
    int d = c->dim;
    double u0 = U[1] / U[0], u1 = d >= 2 ? U[2] / U[0] : 0.0;
    double q2 = u0 * u0 + u1 * u1;
    if (d == 3) q2 = q2 + (U[3] / U[0]) * (U[3] / U[0]);
    *rho = U[0];
    *e_int = U[d + 1] - 0.5 * U[0] * q2;
}

void ora_source(const ora_cfg *c, const double *U, const double *db, double *S)
{
    int d = c->dim, m = ora_num_fields(c->system, d);
    for (int i = 0; i < m; ++i) S[i] = 0.0;
    if (has_bed(c))
        for (int j = 0; j < d; ++j) S[1 + j] = -c->g * U[0] * db[j];
    if (c->system == ORA_REACTIVE) {
        double rho, e_int;
        reactive_parts(c, U, &rho, &e_int);
        S[m - 1] = -arrhenius(c, rho, e_int, U[m - 1]);
    }
}

static void source(const ora_cfg *c, const double *U, const double *db, double *S)
{
    ora_source(c, U, db, S);
}

/* Root of g(z) = (z - B) + (dt/2) R(z), the rho Y component of (2.8), in
 * the bracket [min(0,B), max(0,B)] (g <= 0 at its low end, >= 0 at its high
 * end for R >= 0).  Illinois variant of regula falsi: the secant point of the
 * bracket, with the function value kept at an end that stays twice in a row
 * halved; a bisection when the secant point does not fall strictly inside.
 * Stops at an exact zero or when the bracket is two adjacent doubles, and
 * returns the end with the smaller residual. */
static double reactive_root(const ora_cfg *c, double rho, double e_int, double B, double half_dt)
{
    double a = B < 0.0 ? B : 0.0, b = B < 0.0 ? 0.0 : B;
    double ga = (a - B) + half_dt * arrhenius(c, rho, e_int, a);
    double gb = (b - B) + half_dt * arrhenius(c, rho, e_int, b);
    if (ga == 0.0) return a;
    if (gb == 0.0) return b;
    int kept = 0; /* -1: a was kept by the last step, +1: b */
    for (int it = 0; it < 2000; ++it) {
        double z = b - gb * (b - a) / (gb - ga);
        if (!(z > a && z < b)) z = a + 0.5 * (b - a);
        if (!(z > a && z < b)) break; /* a and b are adjacent doubles */
        double gz = (z - B) + half_dt * arrhenius(c, rho, e_int, z);
        if (gz == 0.0) return z;
        if ((gz < 0.0) == (ga < 0.0)) {
            a = z;
            ga = gz;
            if (kept == 1) gb *= 0.5;
            kept = 1;
        } else {
            b = z;
            gb = gz;
            if (kept == -1) ga *= 0.5;
            kept = -1;
        }
    }
    double ra = fabs((a - B) + half_dt * arrhenius(c, rho, e_int, a));
    double rb = fabs((b - B) + half_dt * arrhenius(c, rho, e_int, b));
    return ra <= rb ? a : b;
}

/* (2.8): U = sumF + (dt/2) S(U).  Bed source: S_h = 0 and S depends on h
 * alone, so U = sumF + (dt/2) S(sumF).  Reactive: every component but rho Y
 * equals sumF; rho Y = z solves g(z) = (z - B) + (dt/2) R(z) = 0. */
void ora_moment_update(const ora_cfg *c, const double *sumF, const double *db, double half_dt,
                       double *U)
{
    int d = c->dim, m = ora_num_fields(c->system, d);
    double S[ORA_MMAX];
    for (int i = 0; i < m; ++i) U[i] = sumF[i];
    if (has_bed(c)) {
        source(c, sumF, db, S);
        for (int i = 0; i < m; ++i) U[i] = sumF[i] + half_dt * S[i];
    }
    if (c->system == ORA_REACTIVE) {
        double rho, e_int;
        reactive_parts(c, sumF, &rho, &e_int);
        U[m - 1] = reactive_root(c, rho, e_int, sumF[m - 1], half_dt);
    }
}

/* ------------------------------------------------------------------------ */
/* Lax-Friedrichs-type equilibrium (2.20) in the general form (2.5).        */
/* Velocity set: e_0 = 0, e_j = unit j, e_{j+d} = -e_j (j = 1..d).         */
/* ------------------------------------------------------------------------ */

static void velocity(int d, int k, int *ex, int *ey, int *ez)
{
    *ex = 0;
    *ey = 0;
    *ez = 0;
    if (k == 0) return;
    int j = (k - 1) % d;
    int s = k <= d ? 1 : -1;
    if (j == 0) *ex = s; else if (j == 1) *ey = s; else *ez = s;
}

void ora_lf_coeffs(int dim, const double *alpha, double lambda, double *a, double *b)
{
    int Q = 2 * dim + 1;
    double sum_alpha = 0.0;
    for (int j = 0; j < dim; ++j) sum_alpha += alpha[j];
    for (int i = 0; i < Q * dim; ++i) b[i] = 0.0;
    a[0] = 1.0 - sum_alpha / lambda;
    for (int j = 0; j < dim; ++j) {
        a[1 + j] = alpha[j] / (2.0 * lambda);
        a[1 + dim + j] = alpha[j] / (2.0 * lambda);
        b[(1 + j) * dim + j] = 1.0 / (2.0 * lambda);
        b[(1 + dim + j) * dim + j] = -1.0 / (2.0 * lambda);
    }
}

static void equilibrium_ab(const ora_cfg *c, const double *U, const double *a,
                           const double *b, double *feq)
{
    int d = c->dim, m = ora_num_fields(c->system, d), Q = 2 * d + 1;
    double F[3][ORA_MMAX];
    for (int j = 0; j < d; ++j) ora_flux(c, j, U, F[j]);
    for (int k = 0; k < Q; ++k)
        for (int r = 0; r < m; ++r) {
            double bf = 0.0;
            for (int j = 0; j < d; ++j) bf += b[k * d + j] * F[j][r];
            feq[k * m + r] = a[k] * U[r] + bf;
        }
}

void ora_equilibrium(const ora_cfg *c, const double *U, const double *alpha,
                     double lambda, double *feq)
{
    double a[7], b[21];
    ora_lf_coeffs(c->dim, alpha, lambda, a, b);
    equilibrium_ab(c, U, a, b, feq);
}

/* ------------------------------------------------------------------------ */
/* Lattice storage and boundary index maps.  Arrays are [z][y][x]; y and z  */
/* carry ghost layers only in the dimensions the lattice has.               */
/* ------------------------------------------------------------------------ */

static int gy(const ora_lattice *L, int depth) { return L->d >= 2 ? depth : 0; }
static int gz(const ora_lattice *L, int depth) { return L->d == 3 ? depth : 0; }
/* padded moments, ghost depth 2 */
static size_t iU(const ora_lattice *L, int c, int i, int j, int l)
{
    size_t px = (size_t)L->nx + 2 * G2, py = (size_t)L->ny + 2 * gy(L, G2), pz = (size_t)L->nz + 2 * gz(L, G2);
    return (((size_t)c * pz + (size_t)(l + gz(L, G2))) * py + (size_t)(j + gy(L, G2))) * px + (size_t)(i + G2);
}
/* padded nu / collided populations, ghost depth 1 */
static size_t n1(const ora_lattice *L)
{
    return ((size_t)L->nx + 2) * ((size_t)L->ny + 2 * gy(L, 1)) * ((size_t)L->nz + 2 * gz(L, 1));
}
static size_t i1(const ora_lattice *L, int i, int j, int l)
{
    size_t px = (size_t)L->nx + 2, py = (size_t)L->ny + 2 * gy(L, 1);
    return ((size_t)(l + gz(L, 1)) * py + (size_t)(j + gy(L, 1))) * px + (size_t)(i + 1);
}
static size_t iC(const ora_lattice *L, int i, int j, int l)
{
    return ((size_t)l * L->ny + j) * L->nx + i;
}
static size_t iF(const ora_lattice *L, int k, int c, int i, int j, int l)
{
    return ((size_t)k * L->m + c) * (size_t)L->ncell + iC(L, i, j, l);
}
static size_t iFs(const ora_lattice *L, int k, int c, int i, int j, int l)
{
    return ((size_t)k * L->m + c) * n1(L) + i1(L, i, j, l);
}
static int bc_side(const ora_cfg *c, int side) { return side < 4 ? c->bc[side] : c->bc_z[side - 4]; }
static int extent(const ora_lattice *L, int dir) { return dir == 0 ? L->nx : (dir == 1 ? L->ny : L->nz); }

/* Mirror/wrap map of an index outside [0,n) onto the interior.  *refl is set
 * when the boundary on that side is a reflective wall. */
static int bc_map(int i, int n, int bclo, int bchi, int *refl)
{
    *refl = 0;
    if (i >= 0 && i < n) return i;
    if (i < 0) {
        if (bclo == ORA_PERIODIC) return ((i % n) + n) % n;
        *refl = bclo == ORA_REFLECTIVE;
        return -1 - i;
    }
    if (bchi == ORA_PERIODIC) return i % n;
    *refl = bchi == ORA_REFLECTIVE;
    return 2 * n - 1 - i;
}

/* Population index reflected across a wall normal to direction dir. */
static int mirror_k(int d, int k, int dir)
{
    if (k == 0) return 0;
    int j = (k - 1) % d;
    if (j != dir) return k;
    return k <= d ? k + d : k - d;
}

ora_lattice *ora_create(const ora_cfg *cfg)
{
    int d = cfg->dim;
    if (d < 1 || d > 3) return NULL;
    if (cfg->nx < 4 || (d >= 2 && cfg->ny < 4) || (d == 1 && cfg->ny != 1)) return NULL;
    if ((d == 3 && cfg->nz < 4) || (d < 3 && cfg->nz != 1)) return NULL;
    if (d == 3 && cfg->system == ORA_SWE) return NULL;
    if (cfg->system == ORA_ADVECTION)
        for (int s = 0; s < 2 * d; ++s)
            if (bc_side(cfg, s) == ORA_REFLECTIVE) return NULL;
    for (int a = 0; a < d; ++a)
        if ((bc_side(cfg, 2 * a) == ORA_PERIODIC) != (bc_side(cfg, 2 * a + 1) == ORA_PERIODIC))
            return NULL;
    ora_lattice *L = calloc(1, sizeof(*L));
    L->c = *cfg;
    L->d = d;
    L->m = ora_num_fields(cfg->system, d);
    L->Q = 2 * d + 1;
    L->nx = cfg->nx;
    L->ny = cfg->ny;
    L->nz = cfg->nz;
    L->ncell = L->nx * L->ny * L->nz;
    L->dx = (cfg->x1 - cfg->x0) / cfg->nx;
    L->f = calloc((size_t)L->Q * L->m * L->ncell, sizeof(double));
    L->omega = calloc((size_t)L->ncell, sizeof(double));
    L->Up = calloc((size_t)L->m * ((size_t)L->nx + 2 * G2) * ((size_t)L->ny + 2 * gy(L, G2)) *
                       ((size_t)L->nz + 2 * gz(L, G2)), sizeof(double));
    L->nup = calloc(n1(L), sizeof(double));
    L->fs = calloc((size_t)L->Q * L->m * n1(L), sizeof(double));
    if (has_bed(cfg)) {
        L->bed = calloc((size_t)L->ncell, sizeof(double));
        L->dbed = calloc((size_t)2 * L->ncell, sizeof(double));
    }
    return L;
}

void ora_destroy(ora_lattice *L)
{
    if (!L) return;
    free(L->f);
    free(L->omega);
    free(L->Up);
    free(L->nup);
    free(L->fs);
    free(L->bed);
    free(L->dbed);
    free(L);
}

/* Moments U = sum_k f_k (2.3) of the interior, then ghost layers of depth 2:
 * the x map on interior rows first, then the y map on all columns, then the
 * z map on all rows and columns (edges and corners take the maps in turn). */
static void fill_moments(ora_lattice *L)
{
    int d = L->d, m = L->m, nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int c = 0; c < m; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < L->Q; ++k) s += L->f[iF(L, k, c, i, j, l)];
                    L->Up[iU(L, c, i, j, l)] = s;
                }
    int mom_ok = L->c.system != ORA_ADVECTION;
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = -G2; i < nx + G2; ++i) {
                if (i >= 0 && i < nx) continue;
                int refl, si = bc_map(i, nx, L->c.bc[0], L->c.bc[1], &refl);
                for (int c = 0; c < m; ++c) {
                    double v = L->Up[iU(L, c, si, j, l)];
                    if (refl && mom_ok && c == 1) v = -v;
                    L->Up[iU(L, c, i, j, l)] = v;
                }
            }
    if (d >= 2)
        for (int l = 0; l < nz; ++l)
            for (int j = -G2; j < ny + G2; ++j) {
                if (j >= 0 && j < ny) continue;
                int refl, sj = bc_map(j, ny, L->c.bc[2], L->c.bc[3], &refl);
                for (int i = -G2; i < nx + G2; ++i)
                    for (int c = 0; c < m; ++c) {
                        double v = L->Up[iU(L, c, i, sj, l)];
                        if (refl && mom_ok && c == 2) v = -v;
                        L->Up[iU(L, c, i, j, l)] = v;
                    }
            }
    if (d == 3)
        for (int l = -G2; l < nz + G2; ++l) {
            if (l >= 0 && l < nz) continue;
            int refl, sl = bc_map(l, nz, L->c.bc_z[0], L->c.bc_z[1], &refl);
            for (int j = -G2; j < ny + G2; ++j)
                for (int i = -G2; i < nx + G2; ++i)
                    for (int c = 0; c < m; ++c) {
                        double v = L->Up[iU(L, c, i, j, sl)];
                        if (refl && mom_ok && c == 3) v = -v;
                        L->Up[iU(L, c, i, j, l)] = v;
                    }
        }
}

static void load_U(const ora_lattice *L, int i, int j, int l, double *U)
{
    for (int c = 0; c < L->m; ++c) U[c] = L->Up[iU(L, c, i, j, l)];
}

/* Wave-speed bounds alpha_bar_j (2.19): global max over interior cells. */
static void alpha_bar(const ora_lattice *L, double *abar)
{
    for (int dir = 0; dir < L->d; ++dir) {
        double mx = 0.0;
#pragma omp parallel for collapse(2) reduction(max : mx) schedule(static)
        for (int l = 0; l < L->nz; ++l)
            for (int j = 0; j < L->ny; ++j)
                for (int i = 0; i < L->nx; ++i) {
                    double U[ORA_MMAX];
                    load_U(L, i, j, l, U);
                    double s = ora_max_speed(&L->c, dir, U);
                    if (s > mx) mx = s;
                }
        abar[dir] = mx;
    }
}

/* Indicator nu (2.13)-(2.14) on interior cells and ghost cells of depth 1. */
static void compute_nu(ora_lattice *L)
{
    int d = L->d, m = L->m;
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = -gz(L, 1); l < L->nz + gz(L, 1); ++l)
        for (int j = -gy(L, 1); j < L->ny + gy(L, 1); ++j)
            for (int i = -1; i < L->nx + 1; ++i) {
                double Uz[ORA_MMAX], Um[ORA_MMAX], Upl[ORA_MMAX], Lm[ORA_MMAX * ORA_MMAX];
                double dm[ORA_MMAX], dp[ORA_MMAX], dU[ORA_MMAX];
                load_U(L, i, j, l, Uz);
                double nu = 0.0;
                for (int dir = 0; dir < d; ++dir) {
                    int ox = dir == 0, oy = dir == 1, oz = dir == 2;
                    load_U(L, i - ox, j - oy, l - oz, Um);
                    load_U(L, i + ox, j + oy, l + oz, Upl);
                    ora_left_eigvecs(&L->c, dir, Uz, Lm);
                    /* Delta_{j,-} W = L_j(U_i)(U_i - U_{i-n_j}) */
                    for (int c = 0; c < m; ++c) dU[c] = Uz[c] - Um[c];
                    for (int r = 0; r < m; ++r) {
                        double s = 0.0;
                        for (int c = 0; c < m; ++c) s += Lm[r * m + c] * dU[c];
                        dm[r] = s;
                    }
                    /* Delta_{j,+} W = L_j(U_i)(U_{i+n_j} - U_i) */
                    for (int c = 0; c < m; ++c) dU[c] = Upl[c] - Uz[c];
                    for (int r = 0; r < m; ++r) {
                        double s = 0.0;
                        for (int c = 0; c < m; ++c) s += Lm[r * m + c] * dU[c];
                        dp[r] = s;
                    }
                    for (int r = 0; r < m; ++r) {
                        double adm = fabs(dm[r]), adp = fabs(dp[r]);
                        double theta = fabs(dp[r] - dm[r]) / (adm + adp + L->dx) + adm + adp;
                        nu += theta;
                    }
                }
                L->nup[i1(L, i, j, l)] = nu;
            }
}

/* Box sum (2.15) over {-1,0,1}^d (z outermost, x innermost) and the
 * relaxation parameter (2.16). */
static void compute_omega(ora_lattice *L)
{
    int d = L->d;
    int zr = d == 3 ? 1 : 0, yr = d >= 2 ? 1 : 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < L->nz; ++l)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double w;
                if (L->c.omega_fixed_on) {
                    w = L->c.omega_fixed;
                } else {
                    double nt = 0.0;
                    for (int kl = -zr; kl <= zr; ++kl)
                        for (int kj = -yr; kj <= yr; ++kj)
                            for (int ki = -1; ki <= 1; ++ki) nt += L->nup[i1(L, i + ki, j + kj, l + kl)];
                    w = 1.0 + 1.0 / (1.0 + nt);
                }
                L->omega[iC(L, i, j, l)] = w;
            }
}

int ora_init(ora_lattice *L, const double *U0, const double *bed, double t0)
{
    int m = L->m, n = L->ncell;
    if (has_bed(&L->c)) {
        if (!bed) return -2;
        memcpy(L->bed, bed, sizeof(double) * n);
        /* central differences with mirrored (or wrapped) ghost values */
        for (int dir = 0; dir < L->d; ++dir)
            for (int j = 0; j < L->ny; ++j)
                for (int i = 0; i < L->nx; ++i) {
                    int r1, r2, ip, im, jp, jm;
                    if (dir == 0) {
                        ip = bc_map(i + 1, L->nx, L->c.bc[0], L->c.bc[1], &r1);
                        im = bc_map(i - 1, L->nx, L->c.bc[0], L->c.bc[1], &r2);
                        jp = jm = j;
                    } else {
                        jp = bc_map(j + 1, L->ny, L->c.bc[2], L->c.bc[3], &r1);
                        jm = bc_map(j - 1, L->ny, L->c.bc[2], L->c.bc[3], &r2);
                        ip = im = i;
                    }
                    double bp = bed[(size_t)jp * L->nx + ip];
                    double bm = bed[(size_t)jm * L->nx + im];
                    L->dbed[(size_t)dir * n + (size_t)j * L->nx + i] = (bp - bm) / (2.0 * L->dx);
                }
    }
    /* moments of U0 at the cell centres, then f = f^eq(U0) with the step-0
     * coefficients, so that sum_k f_k = U0 (up to rounding). */
    for (int c = 0; c < m; ++c)
        for (int l = 0; l < L->nz; ++l)
            for (int j = 0; j < L->ny; ++j)
                for (int i = 0; i < L->nx; ++i)
                    L->Up[iU(L, c, i, j, l)] = U0[(size_t)c * n + iC(L, i, j, l)];
    double abar[3] = {0, 0, 0}, alpha[3];
    alpha_bar(L, abar);
    double sa = 0.0;
    for (int j = 0; j < L->d; ++j) sa += abar[j];
    if (!(sa > 0.0)) return -1;
    double dt = L->c.cfl * L->dx / sa;
    double lambda = L->dx / dt;
    for (int j = 0; j < L->d; ++j) alpha[j] = abar[j] + L->c.eps;
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < L->nz; ++l)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double U[ORA_MMAX], feq[7 * ORA_MMAX];
                load_U(L, i, j, l, U);
                ora_equilibrium(&L->c, U, alpha, lambda, feq);
                for (int k = 0; k < L->Q; ++k)
                    for (int c = 0; c < m; ++c) L->f[iF(L, k, c, i, j, l)] = feq[k * m + c];
            }
    L->t = t0;
    L->steps = 0;
    L->flags = 0;
    return 0;
}

static int one_step(ora_lattice *L)
{
    int d = L->d, m = L->m, Q = L->Q, nx = L->nx, ny = L->ny, nz = L->nz;
    const ora_cfg *cf = &L->c;
    fill_moments(L);

    /* (2.19), (2.21): bounds, alpha_j = alpha_bar_j + eps, delta t, lambda */
    double abar[3] = {0, 0, 0}, alpha[3] = {0, 0, 0};
    alpha_bar(L, abar);
    double sa = 0.0;
    for (int j = 0; j < d; ++j) sa += abar[j];
    if (!(sa > 0.0)) return -1;
    double dt = cf->cfl * L->dx / sa;
    double lambda = L->dx / dt;
    for (int j = 0; j < d; ++j) alpha[j] = abar[j] + cf->eps;
    double a[7], b[21];
    ora_lf_coeffs(d, alpha, lambda, a, b);
    double hdt = 0.5 * dt;

    compute_nu(L);
    compute_omega(L);

    /* collision at every interior source node */
    int bsrc = has_bed(cf);
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double U[ORA_MMAX], feq[7 * ORA_MMAX], S[ORA_MMAX], db[2] = {0, 0};
                load_U(L, i, j, l, U);
                equilibrium_ab(cf, U, a, b, feq);
                if (bsrc)
                    for (int dir = 0; dir < d; ++dir)
                        db[dir] = L->dbed[(size_t)dir * L->ncell + (size_t)j * nx + i];
                source(cf, U, db, S);
                double w = L->omega[iC(L, i, j, l)];
                for (int k = 0; k < Q; ++k)
                    for (int c = 0; c < m; ++c) {
                        double fk = L->f[iF(L, k, c, i, j, l)];
                        L->fs[iFs(L, k, c, i, j, l)] =
                            fk - w * (fk - feq[k * m + c]) + hdt * (a[k] * S[c]);
                    }
            }

    /* ghost collided populations on the faces (depth 1): for the face normal
     * to dir, every cell of the face plane outside the lattice along dir */
    for (int side = 0; side < 2 * d; ++side) {
        int dir = side / 2, hi = side % 2;
        int n_along = extent(L, dir);
        int g = hi ? n_along : -1;
        int refl, mi = bc_map(g, n_along, bc_side(cf, 2 * dir), bc_side(cf, 2 * dir + 1), &refl);
        for (int l = 0; l < (dir == 2 ? 1 : nz); ++l)
            for (int j = 0; j < (dir == 1 ? 1 : ny); ++j)
                for (int i = 0; i < (dir == 0 ? 1 : nx); ++i) {
                    int gi = dir == 0 ? g : i, gj = dir == 1 ? g : j, gl = dir == 2 ? g : l;
                    int si = dir == 0 ? mi : i, sj = dir == 1 ? mi : j, sl = dir == 2 ? mi : l;
                    for (int k = 0; k < Q; ++k) {
                        int ks = refl ? mirror_k(d, k, dir) : k;
                        for (int c = 0; c < m; ++c) {
                            double v = L->fs[iFs(L, ks, c, si, sj, sl)];
                            if (refl && c == 1 + dir) v = -v;
                            L->fs[iFs(L, k, c, gi, gj, gl)] = v;
                        }
                    }
                }
    }

    /* pull streaming F_k(x) = f*_k(x - e_k), implicit moments (2.8), and the
     * second half source f_k = F_k + dt/2 s_k(U^{n+1}) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double Fk[7 * ORA_MMAX], sumF[ORA_MMAX], Un[ORA_MMAX], S[ORA_MMAX], db[2] = {0, 0};
                for (int c = 0; c < m; ++c) sumF[c] = 0.0;
                for (int k = 0; k < Q; ++k) {
                    int ex, ey, ez;
                    velocity(d, k, &ex, &ey, &ez);
                    for (int c = 0; c < m; ++c) {
                        Fk[k * m + c] = L->fs[iFs(L, k, c, i - ex, j - ey, l - ez)];
                        sumF[c] += Fk[k * m + c];
                    }
                }
                if (bsrc)
                    for (int dir = 0; dir < d; ++dir)
                        db[dir] = L->dbed[(size_t)dir * L->ncell + (size_t)j * nx + i];
                /* (2.8) for U^{n+1}, then S(U^{n+1}) for the second half source */
                ora_moment_update(cf, sumF, db, hdt, Un);
                source(cf, Un, db, S);
                for (int k = 0; k < Q; ++k)
                    for (int c = 0; c < m; ++c)
                        L->f[iF(L, k, c, i, j, l)] = Fk[k * m + c] + hdt * (a[k] * S[c]);
            }

    for (size_t q = 0; q < (size_t)Q * m * L->ncell; ++q)
        if (!isfinite(L->f[q])) {
            L->flags |= 1;
            break;
        }
    L->t += dt;
    L->steps += 1;
    for (int j = 0; j < 3; ++j) L->last_abar[j] = abar[j];
    L->last_dt = dt;
    return 0;
}

int64_t ora_run(ora_lattice *L, int64_t nsteps, double t_final)
{
    int64_t n = 0;
    while (n < nsteps) {
        if (t_final > 0.0 && L->t >= t_final) break;
        int rc = one_step(L);
        if (rc < 0) return rc;
        ++n;
    }
    return n;
}

void ora_moments(const ora_lattice *L, double *U)
{
    for (int c = 0; c < L->m; ++c)
        for (int l = 0; l < L->nz; ++l)
            for (int j = 0; j < L->ny; ++j)
                for (int i = 0; i < L->nx; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < L->Q; ++k) s += L->f[iF(L, k, c, i, j, l)];
                    U[(size_t)c * L->ncell + iC(L, i, j, l)] = s;
                }
}

void ora_get_f(const ora_lattice *L, double *f)
{
    memcpy(f, L->f, sizeof(double) * (size_t)L->Q * L->m * L->ncell);
}

void ora_set_f(ora_lattice *L, const double *f)
{
    memcpy(L->f, f, sizeof(double) * (size_t)L->Q * L->m * L->ncell);
}

void ora_last_omega(const ora_lattice *L, double *omega)
{
    memcpy(omega, L->omega, sizeof(double) * (size_t)L->ncell);
}

/* Threads a parallel region of this build uses (1 without OpenMP). */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double ora_time(const ora_lattice *L) { return L->t; }
int64_t ora_steps(const ora_lattice *L) { return L->steps; }
int32_t ora_flags(const ora_lattice *L) { return L->flags; }

void ora_last_scalars(const ora_lattice *L, double *abar3, double *dt)
{
    for (int j = 0; j < 3; ++j) abar3[j] = L->last_abar[j];
    *dt = L->last_dt;
}

void ora_omega_field(ora_lattice *L, double *omega)
{
    fill_moments(L);
    compute_nu(L);
    compute_omega(L);
    memcpy(omega, L->omega, sizeof(double) * (size_t)L->ncell);
}

void ora_nu_field(ora_lattice *L, double *nu)
{
    fill_moments(L);
    compute_nu(L);
    for (int l = 0; l < L->nz; ++l)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) nu[iC(L, i, j, l)] = L->nup[i1(L, i, j, l)];
}

void ora_alpha_bar(const ora_lattice *L, double *abar)
{
    fill_moments((ora_lattice *)L);
    for (int j = 0; j < L->d; ++j) abar[j] = 0.0;
    alpha_bar(L, abar);
}
