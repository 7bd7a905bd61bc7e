/*
 * arlbm.h - C ABI of the MI355X adaptive-relaxation lattice Boltzmann library.
 *
 * One time step of the method of Zhang, Lin, Zhao and Zhao ("A Lattice
 * Boltzmann Method with Adaptive Relaxation Parameter and Lax-Friedrichs-Type
 * Equilibrium for Hyperbolic Systems") runs as a single fused HIP kernel on a
 * gfx950 GPU:
 *   moments U = sum_k f_k (eq. 2.3) -> characteristic projections and
 *   smoothness indicator (eqs. 2.9-2.10, 2.13-2.14) -> box sum (2.11, 2.15)
 *   -> relaxation parameter omega = 1 + 1/(1 + nu~) (2.12, 2.16) ->
 *   Lax-Friedrichs-type equilibrium with the global wave-speed bound
 *   (2.17-2.20) and time step (2.21) -> source split (2.6) -> collision at
 *   the source node and pull streaming (the implementation form of 2.2) ->
 *   implicit moment update (2.8) and second half source.
 *
 * Systems (Section 5): scalar advection, compressible Euler (gamma law),
 * shallow water, and reactive Euler with one-step Arrhenius kinetics
 * (Section 5.4), in 1D (D1Q3) and 2D (D2Q5), and (all but shallow water) in
 * 3D (D3Q7: the formulation of Section 2.3 with d = 3), with an optional
 * shallow-water bed-slope source S = (0, -g h db/dx, -g h db/dy) (not in the
 * paper).
 *
 * Conserved fields per system (plane order):
 *   advection      u
 *   Euler          rho, rho u, [rho v,] rho E       E = p/(gamma-1) + rho|u|^2/2
 *   shallow water  h, h u, [h v]
 *   reactive       rho, rho u, [rho v,] rho E, rho Y
 *                  rho E = p/(gamma-1) + rho|u|^2/2 + q rho Y, and the source
 *                  S = (0, .., 0, -R), R = K rho Y exp(-T_i rho / p)
 *
 * Conventions
 *  - Every function returns 0 (ARLBM_OK) or a negative ARLBM_E* code.  No
 *    exception crosses the ABI.  arlbm_last_error() describes the last failure.
 *  - Host arrays are FP64, structure of arrays: plane c of a field with m
 *    components starts at c*nx*ny, x is fastest, then y.  Host pointers are
 *    borrowed for the duration of the call only.
 *  - Device pointers are HIP device addresses on the current device.
 *  - A handle is not thread-safe; all its work runs in order on the HIP stream
 *    given at creation (NULL = the default stream).
 *  - Cells are cell-centred: x_i = x0 + (i + 1/2) dx, dx = (x1 - x0)/nx, and
 *    in 2D the same dx must hold along y (the paper's uniform grid).
 */
#ifndef ARLBM_H
#define ARLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ARLBM_ABI_VERSION 4

/* Systems, boundary conditions, precisions, relaxation modes. */
enum { ARLBM_ADVECTION = 0, ARLBM_EULER = 1, ARLBM_SWE = 2, ARLBM_REACTIVE = 3 };
enum { ARLBM_PERIODIC = 0, ARLBM_TRANSMISSIVE = 1, ARLBM_REFLECTIVE = 2 };
enum { ARLBM_F32 = 0, ARLBM_F64 = 1 };
enum { ARLBM_OMEGA_ADAPTIVE = 0, ARLBM_OMEGA_FIXED = 1 };

/* Error codes. */
#define ARLBM_OK 0
#define ARLBM_EINVAL (-1)      /* bad configuration or argument               */
#define ARLBM_ENOMEM (-2)      /* device allocation failed                    */
#define ARLBM_EDEVICE (-3)     /* a HIP call failed (message kept)            */
#define ARLBM_ENONFINITE (-4)  /* a moment became NaN/Inf                     */
#define ARLBM_EPOSITIVITY (-5) /* rho or p at/below floor, or h < -h_dry seen  */
#define ARLBM_EDEGENERATE (-6) /* sum of wave-speed bounds is 0: dt undefined */
#define ARLBM_EBUSY (-7)       /* handle is owned by a server                 */
#define ARLBM_EBUDGET (-8)     /* request can never fit the server budget     */

/* Status flag bits (arlbm_status.flags). */
#define ARLBM_FLAG_NONFINITE 1u
#define ARLBM_FLAG_POSITIVITY 2u
#define ARLBM_FLAG_DEGENERATE 4u

typedef struct arlbm_config {
    int32_t abi_version;  /* ARLBM_ABI_VERSION                                  */
    int32_t system;       /* ARLBM_ADVECTION / _EULER / _SWE / _REACTIVE        */
    int32_t dim;          /* 1, 2 or 3 (3D: not shallow water)                  */
    int32_t precision;    /* ARLBM_F32 or ARLBM_F64: storage and arithmetic     */
    int64_t nx, ny, nz;   /* cells; ny = 1 in 1D, nz = 1 below 3D; else >= 4    */
    double x0, x1, y0, y1, z0, z1; /* domain; the spacing is the same on every
                             axis the lattice has: (x1-x0)/nx = (y1-y0)/ny = ..  */
    int32_t bc[6];        /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; periodic must be
                             paired; reflective is rejected for advection      */
    double cfl;           /* in (0, 1): delta t = CFL dx / sum_j alpha_bar_j    */
    double eps;           /* alpha_j = alpha_bar_j + eps, eps > 0 (paper: 1e-10)*/
    double gamma;         /* Euler ratio of specific heats (> 1)                */
    double g;             /* shallow-water gravity (> 0)                        */
    double adv_speed[3];  /* advection velocity per direction                   */
    double h_dry;         /* shallow-water dry threshold (FP64 compare)         */
    double rho_floor, p_floor; /* Euler floors used in the sound speed          */
    int32_t has_bed;      /* shallow water: bed-slope source on                 */
    int32_t omega_mode;   /* ARLBM_OMEGA_ADAPTIVE (eq. 2.16) or _FIXED          */
    double omega_fixed;   /* omega when fixed, in (0, 2]                        */
    double q_heat;        /* reactive: heat release q (>= 0)                    */
    double k_rate;        /* reactive: Arrhenius rate constant K (>= 0)         */
    double t_act;         /* reactive: activation temperature T_i (>= 0)        */
} arlbm_config;

/* Byte sizes of the device buffers of one lattice (each 256-byte aligned). */
typedef struct arlbm_sizes {
    size_t f_bytes;       /* one distribution buffer: Q*m planes                */
    size_t u_bytes;       /* one moment buffer: m planes                        */
    size_t bed_bytes;     /* bed plane (0 without a bed)                        */
    size_t scalar_bytes;  /* per-lattice device scalars                         */
    size_t omega_bytes;   /* omega export plane                                 */
    size_t total_bytes;   /* 2 f + 2 u + bed + scalars (omega export excluded)  */
    size_t alignment;     /* required alignment of caller buffers               */
    int32_t m, q;         /* fields per cell, velocities per cell (2d+1)        */
} arlbm_sizes;

/* Caller-owned device buffers (e.g. torch tensors).  They must outlive the
 * handle.  omega may be NULL (export disabled). */
typedef struct arlbm_buffers {
    void *f[2];
    void *u[2];
    void *bed;
    void *scalars;
    void *omega;
} arlbm_buffers;

typedef struct arlbm_status {
    double t;             /* simulated time                                     */
    double last_dt;       /* delta t of the last step                           */
    double abar[3];       /* wave-speed bounds of the current state (eq. 2.19)  */
    int64_t step;         /* steps that advanced the state since set_state      */
    int64_t first_bad_step; /* first step whose result set a flag, or -1        */
    uint32_t flags;       /* ARLBM_FLAG_* bits seen so far                      */
    uint32_t reserved;
} arlbm_status;

typedef struct arlbm_lattice arlbm_lattice;

/* Fill *cfg with defaults: ABI version, EULER, 1D, F32, nx = 64, ny = nz = 1,
 * unit domain, transmissive, CFL 0.5, eps 1e-10, gamma 1.4, g 9.81,
 * advection speed (1, 0, 0), h_dry 1e-6, floors 1e-12, adaptive omega. */
int arlbm_config_init(arlbm_config *cfg);

/* Validate cfg and report buffer sizes.  EINVAL on a bad configuration. */
int arlbm_query_sizes(const arlbm_config *cfg, arlbm_sizes *out);

/* Create a lattice.  bufs == NULL: the library allocates (and frees in
 * destroy) every buffer; otherwise the caller's buffers are bound (each at
 * least the queried size and aligned).  stream is a hipStream_t or NULL.
 * Validates CFL in (0,1), eps > 0 and the sizes; the eps bound of
 * Theorem 4.3, eps < (1/d)(1/CFL - 1) sum_j alpha_bar_j, needs the state and
 * is checked by arlbm_set_state. */
int arlbm_create(const arlbm_config *cfg, const arlbm_buffers *bufs, void *stream,
                 arlbm_lattice **out);

/* Set the initial state from host FP64 planes U0 (m planes) and, with a bed,
 * bed (one plane); t0 is the starting time.  Rejects non-finite values,
 * rho <= 0 or p <= 0 (Euler), h < 0 (shallow water) with EPOSITIVITY, a zero
 * wave-speed bound with EDEGENERATE and an eps above the Theorem 4.3 bound
 * with EINVAL (the first problem a sequential pass over the cells would
 * meet; the checks of large states run on several host threads).
 * Initialises f = f^eq(U0) with the step-0 coefficients and synchronises the
 * stream.  Arrays of 8 MB and more move through two pinned 16 MB chunks of
 * the library's, used in turn. */
int arlbm_set_state(arlbm_lattice *h, const double *U0, const double *bed, double t0);

/* Same, with U0 (and bed) already on the device as FP64 planes. */
int arlbm_set_state_device(arlbm_lattice *h, const double *U0_dev, const double *bed_dev,
                           double t0);

/* Enqueue n time steps (asynchronous: one kernel launch per step on the
 * handle's stream, no host round trip).  Device-side problems are latched in
 * the status flags and reported by arlbm_sync. */
int arlbm_step(arlbm_lattice *h, int64_t n);

/* Whole steps until the simulated time reaches t_final (t >= t_final; the
 * last step is not shortened, which keeps the scheme second order) or until
 * max_steps steps were taken.  Synchronises a few times to size its batches
 * of launches; a launch that finds t >= t_final leaves the state unchanged,
 * so the result does not depend on the batching.  *steps_taken (may be NULL)
 * receives the number of steps that advanced the state. */
int arlbm_step_until(arlbm_lattice *h, double t_final, int64_t max_steps, int64_t *steps_taken);

/* Wait for the stream and report the status.  Returns ENONFINITE,
 * EDEGENERATE or EPOSITIVITY when the matching flag is set (status still
 * filled), else 0.  EPOSITIVITY is advisory: the method has no positivity
 * mechanism, so a state with a density, pressure or depth below its floor is
 * still the method's result and stepping may continue; the two others mean
 * the state is no longer usable. */
int arlbm_sync(arlbm_lattice *h, arlbm_status *st);

/* Copy the current moments U = sum_k f_k to host FP64 planes (synchronises;
 * large reads are packed into the population buffer the next step writes and
 * move through the pinned chunks that arlbm_set_state uses). */
int arlbm_read_moments(arlbm_lattice *h, double *U_out);

/* Enable (1) or disable (0) writing the relaxation parameter of each step to
 * the omega plane (2.16); library-owned handles allocate the plane. */
int arlbm_set_omega_export(arlbm_lattice *h, int on);

/* Copy the omega plane of the last exported step to host FP64 (synchronises). */
int arlbm_read_omega(arlbm_lattice *h, double *omega_out);

/* Sums over all cells of each conserved field, FP64 with compensated
 * (Neumaier) summation in a fixed order, so repeated calls agree bitwise. */
int arlbm_conservation(arlbm_lattice *h, double *sums_out);

/* arlbm_conservation without any device allocation, for callers that
 * cannot allocate (a serving loop or harness that forbids hipMalloc, work
 * recorded while no allocation may happen): the per-block partial sums live
 * in a device array of the library, 256 blocks x 6 fields of doubles
 * (12 KiB), one copy per GPU, held until the process ends, instead of a
 * buffer the lattice allocates on its first request.  Same sums, bit for
 * bit.  The array is shared by every call on a GPU and keeps the last
 * call's contents (every call overwrites what it reads): calls that overlap
 * on one GPU (several streams or threads at once) race.  EINVAL for a
 * lattice of more than 6 fields (none of the systems has more); EDEVICE if
 * the array's address cannot be had. */
int arlbm_conservation_noalloc(arlbm_lattice *h, double *sums_out);

/* Checkpoint: the state is the f planes, the moment planes, the device
 * scalars and the step count.  state_bytes gives the size of the blob. */
int arlbm_state_bytes(arlbm_lattice *h, size_t *bytes);
int arlbm_save_state(arlbm_lattice *h, void *host_blob, size_t bytes);
int arlbm_load_state(arlbm_lattice *h, const void *host_blob, size_t bytes);

/* Release the handle and any library-owned buffers. */
int arlbm_destroy(arlbm_lattice *h);

/* Message of the last failure on h (or of the calling thread when h is NULL).
 * The string stays valid until the next call on the same handle/thread. */
const char *arlbm_last_error(const arlbm_lattice *h);

/* ------------------------------------------------------------------------ */
/* Serving: many FP32 lattices resident at once; each iteration advances    */
/* every resident lattice by one step in one batched launch (one per group   */
/* of lattices of one cost per row when their 2D work exceeds one round of   */
/* the waves) and a launch per 3D lattice.                                   */
/* ------------------------------------------------------------------------ */

typedef struct arlbm_server arlbm_server;

typedef struct arlbm_completion {
    uint64_t id;          /* id returned by submit                              */
    int32_t status;       /* 0 or an ARLBM_E* code (EPOSITIVITY is reported in
                             flags, with status 0)                             */
    uint32_t flags;       /* ARLBM_FLAG_* bits seen during the run              */
    int64_t steps;        /* steps taken in the server (fewer than asked when a
                             non-finite or degenerate state retired it early)  */
    int64_t first_bad_step; /* the lattice's first step whose result set a flag,
                             or -1                                             */
    double t;             /* simulated time reached                             */
    double submit_s;      /* host clock (seconds) at submit                     */
    double admit_s;       /* host clock when its lattice became resident        */
    double done_s;        /* host clock when its result was read back           */
    double *U;            /* m planes FP64: the caller's array given to
                             arlbm_server_result_into, else owned by the server
                             until the next poll; NULL if status != 0          */
    int64_t u_count;      /* number of doubles in U                             */
} arlbm_completion;

/* Create a server whose lattices never hold more than hbm_budget bytes of
 * device memory: each resident lattice takes one block of the server's pool,
 * sized to a class at most 25% above its buffers (arlbm_sizes.total_bytes),
 * and the blocks the pool keeps, in use or free for reuse, never exceed the
 * budget together.  The work table of the batched launch (about 0.3 KB per
 * resident lattice plus 16 bytes per segment) is outside the budget.
 * precision must be ARLBM_F32 or ARLBM_F64. */
int arlbm_server_create(size_t hbm_budget, int32_t precision, void *stream,
                        arlbm_server **out);

/* Queue a request: a configuration, host FP64 initial planes (and bed) copied
 * at submit time, and a step count (>= 1, else EINVAL).  EBUDGET if its block
 * can never fit the budget.  1D and 2D lattices advance in the iteration's
 * batched launch; a 3D lattice, or a 2D one whose population buffer spans
 * 4 GiB or more, runs its step as launches of its own after it, on the same
 * stream.  A lattice whose state becomes non-finite (or whose wave-speed
 * bounds sum to zero) is retired at a later call, before its step count,
 * and completes with ENONFINITE (EDEGENERATE); the others are unaffected. */
int arlbm_server_submit(arlbm_server *s, const arlbm_config *cfg, const double *U0,
                        const double *bed, int64_t nsteps, uint64_t *id);

/* Queue a request that resumes a saved lattice: blob holds bytes written by
 * arlbm_save_state for a lattice of configuration cfg in the server's
 * precision (copied at submit time); the lattice takes nsteps (>= 1) more
 * steps from the saved step and time, exactly as the saved lattice would have
 * on its own.  EINVAL if the blob does not match cfg (header, sizes), or if
 * cfg has a bed; EBUDGET as for submit. */
int arlbm_server_submit_state(arlbm_server *s, const arlbm_config *cfg, const void *blob,
                              size_t bytes, int64_t nsteps, uint64_t *id);

/* One serving iteration: admit queued requests while the budget allows, run
 * one batched step for every resident lattice, and retire finished ones
 * (their moments are read back).  *resident and *queued report the counts
 * after the iteration (either may be NULL). */
int arlbm_server_iterate(arlbm_server *s, int32_t *resident, int32_t *queued);

/* As arlbm_server_iterate, with up to max_launches (>= 1) steps (each the
 * step's launches) after the admissions, fewer where a resident lattice
 * would otherwise pass its step count: retirements and results are those of
 * one step per call,
 * while the host keeps more work queued on the GPU (requests submitted
 * meanwhile wait for the next call).  *launched (may be NULL) receives the
 * steps made.  EINVAL if max_launches < 1. */
int arlbm_server_iterate_n(arlbm_server *s, int32_t max_launches, int32_t *resident,
                           int32_t *queued, int32_t *launched);

/* Give a queued request (submitted, not yet admitted by an iteration) a
 * destination for its result: dst holds count = m * nx * ny * nz doubles (m
 * planes FP64, the layout of arlbm_read_moments), is owned by the caller and
 * must stay valid until the request's completion has been polled or the
 * server destroyed.  At retirement the moments are copied from the pinned
 * read-back block straight into dst (several host threads), and the
 * completion's U points at dst: the caller needs no copy of its own.  dst is
 * written only if the request completes with status 0.  EINVAL if no queued
 * request has this id, or count is not the result's size. */
int arlbm_server_result_into(arlbm_server *s, uint64_t id, double *dst, int64_t count);

/* Pop up to max finished requests into out; *n receives the count. */
int arlbm_server_poll(arlbm_server *s, arlbm_completion *out, int32_t max, int32_t *n);

/* Bytes of device memory charged to resident lattices (their blocks). */
int arlbm_server_memory(arlbm_server *s, size_t *bytes_in_use);

/* Bytes of device memory the server's pool holds for lattices: blocks in use
 * and free blocks kept for reuse (never above the budget). */
int arlbm_server_pool_bytes(arlbm_server *s, size_t *bytes_held);

int arlbm_server_destroy(arlbm_server *s);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* The batched launch's work list for lattices of configurations cfgs[0..n-1]
 * served together (3D lattices, which run launches of their own, take no
 * part), for a launch of at most `waves` waves, computed on the host as the
 * server computes it (no GPU needed).  On return the list has *nsegs items
 * and the launch *nwaves waves; item k is segs[4k .. 4k+3] = (lattice index,
 * strip, first row, end row) for a 2D lattice, (lattice index, first strip,
 * 0, end strip) for a 1D one (strips are 58 output columns, or 120 where the
 * lattice runs two columns per lane).  The list is cut into 8 queues, one per
 * XCD: queue q holds items queue_start[q] .. queue_start[q+1]-1
 * (queue_start has 9 entries).  EINVAL on a bad configuration or when segs
 * (4 max_segs entries) is too small (the counts are still set). */
int arlbm_plan_schedule(const arlbm_config *cfgs, int32_t n, int32_t waves, int32_t *queue_start,
                        int32_t *segs, int32_t max_segs, int32_t *nsegs, int32_t *nwaves);

/* How the server splits lattices of configurations cfgs[0..n-1] served
 * together into batched launches of at most `waves` waves, computed on the
 * host (no GPU needed).  When their 2D work needs more than one round of
 * the waves, the lattices are split into groups that each fit one round, and
 * each group is one launch of the step, the groups one after the other;
 * otherwise there is one group.  On return group_of[i] (n entries, caller
 * owned) is lattice i's group in 0 .. *ngroups-1, or -1 for a 3D lattice
 * (its step is a launch of its own).  arlbm_plan_schedule on the
 * configurations of one group gives that launch's work list.  EINVAL on a
 * bad configuration or argument. */
int arlbm_plan_groups(const arlbm_config *cfgs, int32_t n, int32_t waves, int32_t *group_of, int32_t *ngroups);

/* The Arrhenius factor's exponential exactly as the kernels evaluate it,
 * callable on the host (no GPU needed): arlbm_kernel_exp is the FP64 kernels'
 * (Cody-Waite reduction, degree-13 series), arlbm_kernel_expf the FP32
 * kernels' (degree 7).  Section 5.4: R = K rho Y exp(-T_i / T). */
double arlbm_kernel_exp(double x);
float arlbm_kernel_expf(float x);

/* Vector registers per lane of the fused step kernel for a precision, system
 * and dimension (from the code object; in 2D the kernel that a lattice of
 * even nx runs), or -1. */
int arlbm_step_kernel_vgprs(int32_t precision, int32_t system, int32_t dim);

#ifdef __cplusplus
}
#endif
#endif /* ARLBM_H */
