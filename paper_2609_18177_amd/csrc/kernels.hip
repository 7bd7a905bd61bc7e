// Kernel instantiations and launchers for one storage precision.  Built twice
// by the package's build step, -DARLBM_F64=0 (float) and -DARLBM_F64=1
// (double), both with -ffp-contract=off so every rounding follows the written
// expression order.
#include "arlbm_internal.h"
#include "step.hpp"
#include "step3d.hpp"

#include <mutex>

namespace arlbm {
static int cell_grid_flags(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b > 64 ? 64 : (b < 1 ? 1 : b));
}
}  // namespace arlbm

#if ARLBM_F64
#define ARLBM_NS f64
typedef double real;
#else
#define ARLBM_NS f32
typedef float real;
#endif

namespace arlbm {
namespace ARLBM_NS {

static int grid_for(int64_t items, int per_block)
{
    int64_t b = (items + per_block - 1) / per_block;
    b = (b + 7) / 8 * 8;  // multiple of 8: the XCD-aware remap is a bijection
    return (int)(b < 8 ? 8 : b);
}

// Compute units of the current device (cached per device).
static int num_cus()
{
    constexpr int kMaxDevices = 64;
    static int cus[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    if (cus[dev] <= 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

static int cell_grid(int64_t cells)
{
    int64_t b = (cells + kBlock - 1) / kBlock;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

template <int SYS, int D>
static hipError_t reduce_impl(const LatticeDesc &h, const double *U0, int slot, hipStream_t s)
{
    hipLaunchKernelGGL((k_reduce_abar<SYS, D, real>), dim3(cell_grid(h.plane)), dim3(kBlock), 0, s, h, U0, slot);
    return hipGetLastError();
}

template <int SYS, int D>
static hipError_t init_impl(const LatticeDesc &h, const double *U0, const double *bed64, int slot_in,
                            hipStream_t s)
{
    hipLaunchKernelGGL((k_init<SYS, D, real>), dim3(cell_grid(h.plane)), dim3(kBlock), 0, s, h, U0, bed64,
                       slot_in);
    return hipGetLastError();
}

template <int SYS, int D>
static hipError_t step_impl(const LatticeDesc &h, int64_t iter, hipStream_t s)
{
    if constexpr (D == 3) {
        // one fused pass: tiles x plane chunks filling the chip once
        using G = Tile3<SYS, real>;
        const int nt = k3_tiles(h.nx, h.ny, G::TX, G::TY);
        const int nb = nt * k3_chunks(nt, h.nz, num_cus());
        hipLaunchKernelGGL((k3_step<SYS, real>), dim3(nb), dim3(G::kThreads), 0, s, h, iter);
    } else {
        const int64_t nbands = D == 2 ? (h.ny + h.band_h - 1) / h.band_h : 1;
        const int64_t nwork = (int64_t)h.ncols * nbands;
        const dim3 g(grid_for(nwork, kWavesPerBlock)), b(kBlock);
        if constexpr (D == 2) {
            constexpr bool kBed = SYS == 2;  // the bed source exists for shallow water only
            const bool bed = kBed && h.bed;
#define ARLBM_L2(BED, V, BUF) hipLaunchKernelGGL((k_step_single<SYS, D, BED, real, V, BUF>), g, b, 0, s, h, iter, (int32_t)nwork)
            if (h.cpl == 2) {
                if (h.buf) {
                    if (bed) ARLBM_L2(kBed, 2, true); else ARLBM_L2(false, 2, true);
                } else {
                    if (bed) ARLBM_L2(kBed, 2, false); else ARLBM_L2(false, 2, false);
                }
            } else if (h.buf) {
                if (bed) ARLBM_L2(kBed, 1, true); else ARLBM_L2(false, 1, true);
            } else {
                if (bed) ARLBM_L2(kBed, 1, false); else ARLBM_L2(false, 1, false);
            }
#undef ARLBM_L2
        } else {
            hipLaunchKernelGGL((k_step_single<SYS, D, false, real>), g, b, 0, s, h, iter, (int32_t)nwork);
        }
    }
    return hipGetLastError();
}

#define ARLBM_DISPATCH(v, CALL)                  \
    switch (v) {                                 \
    case V_ADV1: return CALL(0, 1);              \
    case V_EUL1: return CALL(1, 1);              \
    case V_SWE1: return CALL(2, 1);              \
    case V_ADV2: return CALL(0, 2);              \
    case V_EUL2: return CALL(1, 2);              \
    case V_SWE2: return CALL(2, 2);              \
    case V_REU1: return CALL(3, 1);              \
    case V_REU2: return CALL(3, 2);              \
    case V_ADV3: return CALL(0, 3);              \
    case V_EUL3: return CALL(1, 3);              \
    case V_REU3: return CALL(3, 3);              \
    default: return hipErrorInvalidValue;        \
    }

hipError_t reduce_abar(const LatticeDesc &h, const double *U0, int slot, hipStream_t s)
{
#define C_(S, D) reduce_impl<S, D>(h, U0, slot, s)
    ARLBM_DISPATCH(h.variant, C_)
#undef C_
}

hipError_t init(const LatticeDesc &h, const double *U0, const double *bed64, int slot_in, hipStream_t s)
{
#define C_(S, D) init_impl<S, D>(h, U0, bed64, slot_in, s)
    ARLBM_DISPATCH(h.variant, C_)
#undef C_
}

hipError_t step_single(const LatticeDesc &h, int64_t iter, hipStream_t s)
{
#define C_(S, D) step_impl<S, D>(h, iter, s)
    ARLBM_DISPATCH(h.variant, C_)
#undef C_
}

hipError_t steps1d(const LatticeDesc &h, int64_t iter0, int32_t nsteps, hipStream_t s)
{
    const int nw = h.ncols < 16 ? h.ncols : 16;  // one wave per strip up to 16
    const dim3 g(1), b(64 * nw);
    switch (h.variant) {
    case V_ADV1: hipLaunchKernelGGL((k_steps1d<0, real>), g, b, 0, s, h, iter0, nsteps); break;
    case V_EUL1: hipLaunchKernelGGL((k_steps1d<1, real>), g, b, 0, s, h, iter0, nsteps); break;
    case V_SWE1: hipLaunchKernelGGL((k_steps1d<2, real>), g, b, 0, s, h, iter0, nsteps); break;
    case V_REU1: hipLaunchKernelGGL((k_steps1d<3, real>), g, b, 0, s, h, iter0, nsteps); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t step_batched(const LatticeDesc *d_descs, const Segment *d_segs, const int32_t *d_qstart,
                        unsigned *d_counters, int32_t parity, int32_t nwaves, int64_t iter, hipStream_t s)
{
    hipLaunchKernelGGL((k_step_batched<real>), dim3(grid_for(nwaves, kWavesPerBlock)), dim3(kBlock), 0, s,
                       d_descs, d_segs, d_qstart, d_counters, parity, iter);
    return hipGetLastError();
}

hipError_t conservation(const void *u, int64_t plane, int64_t pstride, int m, double *partial, int nblocks,
                        hipStream_t s)
{
    hipLaunchKernelGGL((k_conservation<real>), dim3(nblocks), dim3(kBlock), 0, s, (const real *)u, plane, pstride, m,
                       partial);
    return hipGetLastError();
}

hipError_t moments(const void *f, void *u, int64_t plane, int64_t pstride, int m, int q, hipStream_t s)
{
    hipLaunchKernelGGL((k_moments<real>), dim3(cell_grid(plane)), dim3(kBlock), 0, s, (const real *)f, (real *)u, plane,
                       pstride, m, q);
    return hipGetLastError();
}

hipError_t to_double(const void *src, double *dst, int64_t plane, int64_t pstride, int m, hipStream_t s)
{
    hipLaunchKernelGGL((k_to_double<real>), dim3(cell_grid(plane * m)), dim3(kBlock), 0, s, (const real *)src, dst,
                       plane, pstride, m);
    return hipGetLastError();
}

// The single-lattice step kernel of a variant (2D: with cpl columns per lane,
// buffer-resource addressing).
template <int SYS, bool BED>
static const void *step_fn2(int cpl)
{
    return cpl == 2 ? (const void *)&k_step_single<SYS, 2, BED, real, 2, true>
                    : (const void *)&k_step_single<SYS, 2, BED, real, 1, true>;
}
static const void *step_fn(int variant, int cpl)
{
    switch (variant) {
    case V_ADV1: return (const void *)&k_step_single<0, 1, false, real>;
    case V_EUL1: return (const void *)&k_step_single<1, 1, false, real>;
    case V_SWE1: return (const void *)&k_step_single<2, 1, false, real>;
    case V_REU1: return (const void *)&k_step_single<3, 1, false, real>;
    case V_ADV2: return step_fn2<0, false>(cpl);
    case V_EUL2: return step_fn2<1, false>(cpl);
    case V_SWE2: return step_fn2<2, true>(cpl);
    case V_REU2: return step_fn2<3, false>(cpl);
    case V_ADV3: return (const void *)&k3_step<0, real>;
    case V_EUL3: return (const void *)&k3_step<1, real>;
    case V_REU3: return (const void *)&k3_step<3, real>;
    default: return nullptr;
    }
}

// Waves of the single-lattice step kernel resident per CU at full occupancy.
int step_waves_per_cu(int variant, int cpl)
{
    const void *fn = step_fn(variant, cpl);
    if (!fn) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlock, 0) != hipSuccess) return 0;
    return blocks * kWavesPerBlock;
}

int step_kernel_vgprs(int variant, int cpl)
{
    hipFuncAttributes a;
    const void *fn = step_fn(variant, cpl);
    if (!fn) return -1;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) return -1;
    return a.numRegs;
}

}  // namespace ARLBM_NS

#if !ARLBM_F64
extern "C" double arlbm_kernel_exp(double x) { return arrhenius_exp(x); }
extern "C" float arlbm_kernel_expf(float x) { return arrhenius_exp(x); }

__global__ __launch_bounds__(kBlock) void k_gather_flags(const LatticeDesc *descs, int32_t n, unsigned *out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = descs[i].sc->flags;
}

hipError_t gather_flags_launch(const LatticeDesc *descs, int32_t n, unsigned *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_flags, dim3(cell_grid_flags(n)), dim3(kBlock), 0, s, descs, n, out);
    return hipGetLastError();
}

// Partial sums of the allocation-free conservation sums: one copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device array: only the address hipGetSymbolAddress
// returns (per device) reaches a kernel.
static __device__ __align__(256) double scratch[kConsBlocks * kConsMaxFields];

hipError_t conservation_scratch(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}
#endif
}  // namespace arlbm
