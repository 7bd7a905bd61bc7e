// Internal types shared by the HIP kernels and the host runtime of libarlbm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arlbm {

// Cells produced per wave along x.  With one column per lane a wave of 64
// lanes covers x0-3 .. x0+60: the 3-cell halo on each side feeds the
// radius-2 indicator stencil and the radius-1 pull (omega is needed one cell
// beyond the outputs).  With V columns per lane the halo is rounded up to
// whole lanes, so that every lane's V columns start V-aligned.
constexpr int kWave = 64;
constexpr int kHalo = 3;
constexpr int kOutW = kWave - 2 * kHalo;  // 58
__host__ __device__ constexpr int strip_halo(int v) { return (kHalo + v - 1) / v * v; }
__host__ __device__ constexpr int strip_out_w(int v) { return kWave * v - 2 * strip_halo(v); }
static_assert(strip_out_w(1) == kOutW && strip_out_w(2) == 120, "strip geometry");
constexpr int kBlock = 256;               // 4 independent waves per block
constexpr int kWavesPerBlock = kBlock / kWave;

enum Variant : int32_t {
    V_ADV1 = 0, V_EUL1 = 1, V_SWE1 = 2, V_REU1 = 3,
    V_ADV2 = 4, V_EUL2 = 5, V_SWE2 = 6, V_REU2 = 7,
    V_ADV3 = 8, V_EUL3 = 9, V_REU3 = 11
};

__host__ __device__ constexpr int variant_of(int system, int dim) { return (dim - 1) * 4 + system; }
__host__ __device__ constexpr int num_fields(int system, int dim) {
    return system == 0 ? 1 : (system == 1 ? dim + 2 : (system == 2 ? dim + 1 : dim + 3));
}

// Per-lattice device scalars (FP64), kept resident between launches.
// One copy of a wave-speed slot: one 128-byte line, v[0..2] the directions.
struct AbarCopy {
    unsigned long long v[16];
};
// Copies per slot.  A wave maxes its bounds into copy (wave index mod
// kAbarCopies) and readers take the max over the copies: with a single copy
// the waves of a launch queued on one line at about 11 ns per atomic, about
// 9 us of a 2048^2 2D step.  Atomics on one line serialize even at different
// addresses: copies packed 16 to a line measured 0.1586 against 0.1574 ms per
// 2048^2 Euler step and 17.2 against 7.9 us per 262144-cell 1D step.
constexpr int kAbarCopies = 64;
struct DevScalars {
    // alpha_bar bit patterns (non-negative doubles order like unsigned
    // integers, so the grid-wide max is an integer atomic max).  Three slots:
    // step n reads slot n%3, maxes into (n+1)%3 and clears (n+2)%3.
    AbarCopy abar[3][kAbarCopies];
    double last_dt;
    unsigned long long first_bad_step;  // min over flagged steps (~0 = none)
    unsigned int flags;
    unsigned int pad;
    // time of the state step n reads (slot n%3; the step writes slot (n+1)%3,
    // so every wave of a launch sees the same value)
    double t[3];
    unsigned long long null_launches;   // launches that found t >= t_stop (left the state as it was)
};
static_assert(sizeof(DevScalars) == 3 * kAbarCopies * sizeof(AbarCopy) + 56, "DevScalars layout");

// Everything a kernel needs to know about one lattice.  Uploaded once at
// creation (and at admission in the server); the step index is derived from
// the launch's iteration counter: n = iter - iter0.
struct LatticeDesc {
    void *f[2];
    void *u[2];
    const void *bed;
    void *omega;
    DevScalars *sc;
    int32_t variant, nx, ny, nz, bc[6];
    int32_t omega_fixed_on;
    int32_t band_h;       // rows per strip (2D)
    int32_t ncols;        // strips along x
    int64_t iter0;
    double t_stop;        // a launch whose state time is >= t_stop copies f unchanged (null step)
    int64_t plane;        // nx * ny * nz
    int64_t pstride;      // elements between planes: plane rounded up to 64, plus a pad
    int32_t omega_on;     // omega export plane present (else omega is null and never written)
    int32_t cpl;          // 2D: columns per lane of the step's strips (1, or 2 when nx is even)
    int32_t buf;          // 2D: population buffers below 4 GiB, addressed by buffer resources
    int32_t abar_n;       // copies of each wave-speed slot in use: a power of two <= kAbarCopies, fixed per lattice
    double dx, cfl, eps, gamma, g, adv[3], h_dry, rho_floor, p_floor, omega_fixed;
    double q_heat, k_rate, t_act;  // reactive Euler: heat release, rate constant, activation temperature
};

// One work item of a batched launch.  2D: rows y0 .. y1-1 of strip col.
// 1D: strips col .. y1-1 (y0 unused).  The item that holds the lattice's
// first cell (col 0, row 0) also updates its scalars.
struct Segment {
    int32_t lattice;
    int32_t col;
    int32_t y0;
    int32_t y1;
};

// Conservation sums: per-block compensated partial sums of each field, over
// kConsBlocks blocks, for at most kConsMaxFields fields (3D reactive Euler).
constexpr int kConsBlocks = 256;
constexpr int kConsMaxFields = 6;

// Work queues of a batched launch: one per XCD, counters 128 bytes apart.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;

}  // namespace arlbm

// Host-side launchers, implemented once per precision (kernels.hip is
// compiled twice, FP32 and FP64, both without contraction).
#define ARLBM_DECLARE_LAUNCHERS(NS)                                                                    \
    namespace arlbm {                                                                                  \
    namespace NS {                                                                                     \
    hipError_t reduce_abar(const LatticeDesc &h, const double *U0, int slot, hipStream_t s);          \
    hipError_t init(const LatticeDesc &h, const double *U0, const double *bed64, int slot_in,         \
                    hipStream_t s);                                                                    \
    hipError_t step_single(const LatticeDesc &h, int64_t iter, hipStream_t s);                        \
    hipError_t steps1d(const LatticeDesc &h, int64_t iter0, int32_t nsteps, hipStream_t s);           \
    hipError_t step_batched(const LatticeDesc *d_descs, const Segment *d_segs, const int32_t *d_qstart, \
                            unsigned *d_counters, int32_t parity, int32_t nwaves, int64_t iter,        \
                            hipStream_t s);                                                            \
    hipError_t conservation(const void *u, int64_t plane, int64_t pstride, int m, double *partial,    \
                            int nblocks, hipStream_t s);                                               \
    hipError_t moments(const void *f, void *u, int64_t plane, int64_t pstride, int m, int q,          \
                       hipStream_t s);                                                                 \
    hipError_t to_double(const void *src, double *dst, int64_t plane, int64_t pstride, int m,         \
                         hipStream_t s);                                                               \
    int step_kernel_vgprs(int variant, int cpl);                                                       \
    int step_waves_per_cu(int variant, int cpl);                                                       \
    }                                                                                                  \
    }

ARLBM_DECLARE_LAUNCHERS(f32)
ARLBM_DECLARE_LAUNCHERS(f64)

namespace arlbm {
// out[i] = descs[i].sc->flags for i < n (either precision: the scalars are FP64).
hipError_t gather_flags_launch(const LatticeDesc *descs, int32_t n, unsigned *out, hipStream_t s);
// Device address of this GPU's copy of the conservation scratch (a
// file-scope device array of kConsBlocks * kConsMaxFields doubles), looked up
// once per device with that device current.
hipError_t conservation_scratch(double **out);
}  // namespace arlbm
