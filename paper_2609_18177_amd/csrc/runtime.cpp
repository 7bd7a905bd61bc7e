// Host runtime of libarlbm: the C ABI declared in include/arlbm.h.
//
// A lattice owns (or borrows) two population buffers and two moment buffers
// (ping-pong), an optional bed plane, an optional omega plane and a 128-byte
// block of device scalars.  Stepping enqueues one fused kernel per step on the
// handle's stream; the host never reads the device between steps.  The server
// keeps many lattices resident and advances all of them with one batched
// launch per iteration.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <sys/mman.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "arlbm.h"
#include "arlbm_internal.h"

using namespace arlbm;

namespace {

thread_local std::string g_thread_err;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int q_of(int dim) { return 2 * dim + 1; }

// Validation of a configuration; returns an empty string when valid.
std::string check_config(const arlbm_config *c)
{
    if (!c) return "config is NULL";
    if (c->abi_version != ARLBM_ABI_VERSION) return "abi_version mismatch";
    if (c->system < 0 || c->system > 3) return "unknown system";
    if (c->dim < 1 || c->dim > 3) return "dim must be 1, 2 or 3";
    if (c->precision != ARLBM_F32 && c->precision != ARLBM_F64) return "precision must be F32 or F64";
    if (c->nx < 4) return "nx must be >= 4";
    if (c->dim == 1 && c->ny != 1) return "ny must be 1 in 1D";
    if (c->dim >= 2 && c->ny < 4) return "ny must be >= 4";
    if (c->dim < 3 && c->nz != 1) return "nz must be 1 below 3D";
    if (c->dim == 3 && c->nz < 4) return "nz must be >= 4";
    if (c->dim == 3 && c->system == ARLBM_SWE) return "shallow water is 1D or 2D";
    if (c->nx > (1 << 26) || c->ny > (1 << 26) || c->nz > (1 << 26)) return "lattice too large";
    // kernels address cells within a plane with 32-bit offsets
    if (c->nx * c->ny * c->nz > (int64_t)0x7fffffff) return "a plane exceeds 2^31 cells";
    if (!(c->x1 > c->x0)) return "x1 must exceed x0";
    const double dx = (c->x1 - c->x0) / (double)c->nx;
    if (c->dim >= 2) {
        if (!(c->y1 > c->y0)) return "y1 must exceed y0";
        const double dy = (c->y1 - c->y0) / (double)c->ny;
        if (std::fabs(dx - dy) > 1e-12 * dx) return "dx must equal dy (uniform lattice)";
    }
    if (c->dim == 3) {
        if (!(c->z1 > c->z0)) return "z1 must exceed z0";
        const double dz = (c->z1 - c->z0) / (double)c->nz;
        if (std::fabs(dx - dz) > 1e-12 * dx) return "dx must equal dz (uniform lattice)";
    }
    for (int s = 0; s < 2 * c->dim; ++s)
        if (c->bc[s] < 0 || c->bc[s] > 2) return "unknown boundary condition";
    for (int a = 0; a < c->dim; ++a)
        if ((c->bc[2 * a] == ARLBM_PERIODIC) != (c->bc[2 * a + 1] == ARLBM_PERIODIC))
            return "periodic boundaries must be paired on an axis";
    if (c->system == ARLBM_ADVECTION)
        for (int s = 0; s < 2 * c->dim; ++s)
            if (c->bc[s] == ARLBM_REFLECTIVE) return "reflective walls need a momentum field (not advection)";
    if (!(c->cfl > 0.0 && c->cfl < 1.0)) return "CFL must lie in (0, 1)";
    if (!(c->eps > 0.0)) return "eps must be > 0";
    const bool gas = c->system == ARLBM_EULER || c->system == ARLBM_REACTIVE;
    if (gas && !(c->gamma > 1.0)) return "gamma must be > 1";
    if (c->system == ARLBM_REACTIVE && !(c->q_heat >= 0.0 && c->k_rate >= 0.0 && c->t_act >= 0.0 &&
                                         std::isfinite(c->q_heat) && std::isfinite(c->k_rate) &&
                                         std::isfinite(c->t_act)))
        return "q_heat, k_rate and t_act must be finite and >= 0";
    if (c->system == ARLBM_SWE && !(c->g > 0.0)) return "g must be > 0";
    if (c->system == ARLBM_SWE && !(c->h_dry > 0.0)) return "h_dry must be > 0";
    if (gas && !(c->rho_floor > 0.0 && c->p_floor > 0.0)) return "floors must be > 0";
    if (c->has_bed && c->system != ARLBM_SWE) return "a bed source needs shallow water";
    if (c->system == ARLBM_ADVECTION) {
        double s = std::fabs(c->adv_speed[0]) + (c->dim >= 2 ? std::fabs(c->adv_speed[1]) : 0.0) +
                   (c->dim == 3 ? std::fabs(c->adv_speed[2]) : 0.0);
        if (!(s > 0.0)) return "advection speed must be non-zero";
    }
    if (c->omega_mode != ARLBM_OMEGA_ADAPTIVE && c->omega_mode != ARLBM_OMEGA_FIXED) return "unknown omega mode";
    if (c->omega_mode == ARLBM_OMEGA_FIXED && !(c->omega_fixed > 0.0 && c->omega_fixed <= 2.0))
        return "omega_fixed must lie in (0, 2]";
    return "";
}

// Columns per lane of the 2D step.  Two adjacent columns per lane need an
// even nx (every pair 8-byte aligned).  Measured on MI355X (2048^2 and
// 4096^2 lattices, ms per step, one column per lane -> two):
//   FP32 advection 0.0650 -> 0.0558, shallow water 0.520 -> 0.493,
//        Euler 0.1758 -> 0.1777, reactive Euler 0.290 -> 0.298;
//   FP64 shallow water 1.177 -> 1.140, Euler 0.388 -> 0.430.
// The faster width is taken per system and precision.
int columns_per_lane(const arlbm_config *c)
{
    if (c->dim != 2 || c->nx % 2 != 0) return 1;
    static const int f32[4] = {2, 1, 2, 1}, f64[4] = {1, 1, 2, 1};  // advection, Euler, shallow water, reactive
    return (c->precision == ARLBM_F64 ? f64 : f32)[c->system];
}

// Planes are stored at a stride of nx*ny rounded up to a multiple of 64
// elements (every plane starts 256-byte aligned) plus kPlanePad
// elements, so that the planes of a power-of-two lattice do not all start at
// the same offset of the memory interleave: the step reads and writes row j
// of all Q m planes together.  Measured (ms per step, pad 0 / 64 / 256 /
// 1088 elements): 2048^2 Euler FP32 0.173 / 0.166 / 0.184 / 0.167, 4096^2
// shallow water FP32 0.486 / 0.465 / 0.463 / 0.460, FP64 0.903 / 0.903 /
// 0.894 / 0.883, 256^3 Euler FP32 1.72 / 1.70 / 1.76 / 1.70.
constexpr int64_t kPlanePad = 1088;
int64_t plane_stride(const arlbm_config *c)
{
    const int64_t plane = c->nx * c->ny * c->nz;
    return (plane + 63) / 64 * 64 + kPlanePad;
}

void fill_sizes(const arlbm_config *c, arlbm_sizes *o)
{
    const int m = num_fields(c->system, c->dim), q = q_of(c->dim);
    const size_t s = c->precision == ARLBM_F64 ? 8 : 4;
    const size_t ps = (size_t)plane_stride(c);
    o->m = m;
    o->q = q;
    o->f_bytes = align_up((size_t)q * m * ps * s);
    // in 3D the moment buffers are a ping-pong kept current by the step
    o->u_bytes = align_up((size_t)m * ps * s);
    o->bed_bytes = c->has_bed ? align_up(ps * s) : 0;
    o->scalar_bytes = align_up(sizeof(DevScalars));
    o->omega_bytes = align_up(ps * s);
    o->total_bytes = 2 * o->f_bytes + 2 * o->u_bytes + o->bed_bytes + o->scalar_bytes;
    o->alignment = kAlign;
}

// Band height of the 2D step.  Each strip pays a warm-up of 3 extra moment
// rows and 2 extra indicator rows, so strips should be long; the grid should
// also fill the GPU in one round.  The number of strips is kept at or just
// below one wave per SIMD (4 per CU): measured on MI355X, one wave per SIMD
// with twice the rows beats two waves per SIMD by 15-25% for both FP32 and
// FP64 (fewer concurrent streams into HBM, half the warm-up rows), and never
// more than the waves the GPU can hold at once.
int choose_band(int64_t ny, int ncols, int64_t resident_waves, int64_t simds)
{
    if (resident_waves <= 0) resident_waves = 4096;
    if (simds < resident_waves) resident_waves = simds;  // one wave per SIMD
    int64_t nb = resident_waves / ncols;
    if (nb < 1) nb = 1;
    int64_t h = (ny + nb - 1) / nb;
    if (h < 8) h = 8;
    if (h > ny) h = ny;
    return (int)h;
}

int num_cus()
{
    static int cus = -1;
    if (cus < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            v = 256;
        cus = v;
    }
    return cus;
}

int64_t resident_waves(int precision, int variant, int cpl)
{
    const int64_t cus = num_cus();
    const int w = precision == ARLBM_F64 ? f64::step_waves_per_cu(variant, cpl)
                                         : f32::step_waves_per_cu(variant, cpl);
    return (int64_t)cus * (w > 0 ? w : 16);
}

}  // namespace

struct arlbm_lattice {
    arlbm_config cfg{};
    arlbm_sizes sz{};
    LatticeDesc desc{};
    hipStream_t stream = nullptr;
    bool owns = false;
    bool owns_omega = false;
    bool busy = false;
    int64_t step = 0;
    double *d_partial = nullptr;
    std::string err;
};

namespace {

int fail(arlbm_lattice *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    g_thread_err = msg;
    return code;
}

int hip_fail(arlbm_lattice *h, hipError_t e, const char *what)
{
    return fail(h, e == hipErrorOutOfMemory ? ARLBM_ENOMEM : ARLBM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                    \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

bool is_f64(const arlbm_lattice *h) { return h->cfg.precision == ARLBM_F64; }

hipError_t L_reduce(const arlbm_lattice *h, const double *U0, int slot)
{
    return is_f64(h) ? f64::reduce_abar(h->desc, U0, slot, h->stream) : f32::reduce_abar(h->desc, U0, slot, h->stream);
}
hipError_t L_init(const arlbm_lattice *h, const double *U0, const double *bed, int slot)
{
    return is_f64(h) ? f64::init(h->desc, U0, bed, slot, h->stream) : f32::init(h->desc, U0, bed, slot, h->stream);
}
hipError_t L_step(const arlbm_lattice *h, int64_t iter)
{
    return is_f64(h) ? f64::step_single(h->desc, iter, h->stream) : f32::step_single(h->desc, iter, h->stream);
}

void free_owned(arlbm_lattice *h)
{
    if (h->owns) {
        for (int i = 0; i < 2; ++i) {
            if (h->desc.f[i]) (void)hipFree(h->desc.f[i]);
            if (h->desc.u[i]) (void)hipFree(h->desc.u[i]);
        }
        if (h->desc.bed) (void)hipFree((void *)h->desc.bed);
        if (h->desc.sc) (void)hipFree(h->desc.sc);
    }
    if (h->owns_omega && h->desc.omega) (void)hipFree(h->desc.omega);
    if (h->d_partial) (void)hipFree(h->d_partial);
}

// Host-side admissibility of an initial state (finite, rho > 0, p > 0, h >= 0).
// memcpy of large host arrays over several threads: a fresh destination
// faults its pages in on first touch, and those faults proceed in parallel
// (measured on 32 MB: 21 ms on one thread, 4 ms on eight).
void par_copy(void *dst, const void *src, size_t bytes)
{
    constexpr size_t kPerThread = (size_t)4 << 20;
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({(size_t)8, hw, bytes / kPerThread});
    if (bytes == 0) return;
    if (nt < 2) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t chunk = (bytes / nt + 4095) / 4096 * 4096;  // nt * chunk >= bytes
    std::vector<std::thread> th;
    size_t started = 0;  // chunks 1 .. started run on threads of their own
    try {
        th.reserve(nt - 1);
        for (size_t t = 1; t < nt && t * chunk < bytes; ++t) {
            const size_t a = t * chunk, len = std::min(chunk, bytes - a);
            th.emplace_back([=] { std::memcpy((char *)dst + a, (const char *)src + a, len); });
            started = t;
        }
    } catch (...) {
        // no thread for the remaining chunks: copied below
    }
    std::memcpy(dst, src, std::min(chunk, bytes));
    const size_t rest = (started + 1) * chunk;
    if (rest < bytes) std::memcpy((char *)dst + rest, (const char *)src + rest, bytes - rest);
    for (auto &x : th) x.join();
}

// Host <-> device copies of large pageable arrays (the plain path's state
// upload and read-back): the data moves through two pinned chunks used in
// turn, the host copy of one chunk (several threads) overlapping the DMA of
// the other.  The chunk pairs are kept for the process in a free list, one
// pair per transfer in progress.  Arrays below kBounceMin go directly.
constexpr size_t kBounceChunk = (size_t)16 << 20, kBounceMin = (size_t)8 << 20;
std::mutex g_bounce_mu;
std::vector<char *> g_bounce_free;

char *bounce_take()
{
    {
        std::lock_guard<std::mutex> g(g_bounce_mu);
        if (!g_bounce_free.empty()) {
            char *b = g_bounce_free.back();
            g_bounce_free.pop_back();
            return b;
        }
    }
    void *p = nullptr;
    return hipHostMalloc(&p, 2 * kBounceChunk, hipHostMallocDefault) == hipSuccess ? (char *)p : nullptr;
}

void bounce_give(char *b)
{
    std::lock_guard<std::mutex> g(g_bounce_mu);
    g_bounce_free.push_back(b);
}

// dst (device) <- src (host), ordered on the stream; returns once the
// source has been read (the last DMA done).
hipError_t copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    char *buf = bytes >= kBounceMin ? bounce_take() : nullptr;
    if (!buf) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
    bool used[2] = {false, false};
    for (size_t off = 0, k = 0; e == hipSuccess && off < bytes; off += kBounceChunk, ++k) {
        const int b = (int)(k & 1);
        const size_t len = std::min(kBounceChunk, bytes - off);
        if (used[b]) e = hipEventSynchronize(ev[b]);  // the chunk's previous DMA has read it
        if (e != hipSuccess) break;
        par_copy(buf + b * kBounceChunk, (const char *)src + off, len);
        e = hipMemcpyAsync((char *)dst + off, buf + b * kBounceChunk, len, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(ev[b], st);
        used[b] = true;
    }
    // both chunks idle before the pair goes back to the free list
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (es == hipSuccess) bounce_give(buf);
    return e;
}

// dst (host) <- src (device) after the work ordered before it on the stream;
// returns with dst written.
hipError_t copy_d2h(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    char *buf = bytes >= kBounceMin ? bounce_take() : nullptr;
    if (!buf) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
    const size_t nchunks = (bytes + kBounceChunk - 1) / kBounceChunk;
    auto enqueue = [&](size_t k) {
        const int b = (int)(k & 1);
        const size_t off = k * kBounceChunk, len = std::min(kBounceChunk, bytes - off);
        hipError_t r = hipMemcpyAsync(buf + b * kBounceChunk, (const char *)src + off, len, hipMemcpyDeviceToHost, st);
        return r == hipSuccess ? hipEventRecord(ev[b], st) : r;
    };
    for (size_t k = 0; k < 2 && k < nchunks && e == hipSuccess; ++k) e = enqueue(k);
    for (size_t k = 0; k < nchunks && e == hipSuccess; ++k) {
        const int b = (int)(k & 1);
        const size_t off = k * kBounceChunk, len = std::min(kBounceChunk, bytes - off);
        e = hipEventSynchronize(ev[b]);
        if (e != hipSuccess) break;
        par_copy((char *)dst + off, buf + b * kBounceChunk, len);
        if (k + 2 < nchunks) e = enqueue(k + 2);  // into the chunk just emptied
    }
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (es == hipSuccess) bounce_give(buf);
    return e;
}

// Host checks of an initial state, over several threads for large lattices.
// The result is the sequential one: a non-finite value anywhere first, then
// a non-finite bed, then the first cell (lowest index) that breaks
// positivity.
int check_state(arlbm_lattice *h, const double *U0, const double *bed)
{
    const arlbm_config &c = h->cfg;
    const int64_t plane = h->desc.plane;
    const int m = h->sz.m;
    enum { kOk = 0, kRho, kP, kDepth };
    struct Part {
        bool nonfinite = false, bed_nonfinite = false;
        int64_t bad = -1;  // first cell breaking positivity
        int kind = kOk;
    };
    auto check = [&](int64_t i0, int64_t i1, Part &r) {
        for (int f = 0; f < m && !r.nonfinite; ++f)
            for (int64_t i = i0; i < i1; ++i)
                if (!std::isfinite(U0[(int64_t)f * plane + i])) {
                    r.nonfinite = true;
                    break;
                }
        if (bed)
            for (int64_t i = i0; i < i1; ++i)
                if (!std::isfinite(bed[i])) {
                    r.bed_nonfinite = true;
                    break;
                }
        if (c.system == ARLBM_EULER || c.system == ARLBM_REACTIVE) {
            const int e = c.dim + 1;
            for (int64_t i = i0; i < i1; ++i) {
                const double rho = U0[i];
                double ke = 0.0;
                for (int d = 0; d < c.dim; ++d) {
                    const double mom = U0[(1 + d) * plane + i];
                    ke += 0.5 * mom * mom / rho;
                }
                double chem = 0.0;
                if (c.system == ARLBM_REACTIVE) chem = c.q_heat * U0[(int64_t)(e + 1) * plane + i];
                const double p = (c.gamma - 1.0) * (U0[(int64_t)e * plane + i] - ke - chem);
                if (!(rho > 0.0) || !(p > 0.0)) {
                    r.bad = i;
                    r.kind = !(rho > 0.0) ? kRho : kP;
                    break;
                }
            }
        } else if (c.system == ARLBM_SWE) {
            for (int64_t i = i0; i < i1; ++i)
                if (!(U0[i] >= 0.0)) {
                    r.bad = i;
                    r.kind = kDepth;
                    break;
                }
        }
    };
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({8, hw, plane / (1 << 18)}));
    std::vector<Part> parts((size_t)nt);
    std::vector<std::thread> th;
    const int64_t per = (plane + nt - 1) / nt;
    try {
        for (int64_t t = 1; t < nt; ++t)
            th.emplace_back(check, std::min(plane, t * per), std::min(plane, (t + 1) * per), std::ref(parts[t]));
    } catch (...) {
        for (auto &x : th) x.join();
        th.clear();
        parts.assign(1, Part{});
        check(0, plane, parts[0]);
    }
    if (parts.size() == (size_t)nt) check(0, std::min(plane, per), parts[0]);
    for (auto &x : th) x.join();
    Part all;
    for (const Part &r : parts) {
        all.nonfinite |= r.nonfinite;
        all.bed_nonfinite |= r.bed_nonfinite;
        if (r.bad >= 0 && all.bad < 0) {  // parts in index order: the first one found is the lowest
            all.bad = r.bad;
            all.kind = r.kind;
        }
    }
    if (all.nonfinite) return fail(h, ARLBM_EPOSITIVITY, "initial state is not finite");
    if (all.bed_nonfinite) return fail(h, ARLBM_EPOSITIVITY, "bed is not finite");
    if (all.kind == kRho) return fail(h, ARLBM_EPOSITIVITY, "initial density must be > 0");
    if (all.kind == kP) return fail(h, ARLBM_EPOSITIVITY, "initial pressure must be > 0");
    if (all.kind == kDepth) return fail(h, ARLBM_EPOSITIVITY, "initial depth must be >= 0");
    return ARLBM_OK;
}

// The wave-speed bound of direction dir in a slot: the max over the slot's
// copies (non-negative doubles order like their bit patterns).
double abar_host(const DevScalars &sc, int slot, int dir)
{
    unsigned long long m = 0;
    for (int c = 0; c < kAbarCopies; ++c) m = std::max(m, sc.abar[slot][c].v[dir]);
    double d;
    std::memcpy(&d, &m, sizeof d);
    return d;
}

int read_scalars(arlbm_lattice *h, DevScalars *out)
{
    HIPCHK(h, hipMemcpyAsync(out, h->desc.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return ARLBM_OK;
}

// Device-side staging of the initial state into f[1] (free before step 0).
int set_state_impl(arlbm_lattice *h, const double *U0, const double *bed, bool on_device, double t0)
{
    if (h->busy) return fail(h, ARLBM_EBUSY, "lattice is owned by a server");
    const int64_t plane = h->desc.plane;
    const int m = h->sz.m;
    const bool need_bed = h->cfg.has_bed != 0;
    if (!U0) return fail(h, ARLBM_EINVAL, "U0 is NULL");
    if (need_bed && !bed) return fail(h, ARLBM_EINVAL, "configuration has a bed but bed is NULL");
    double *stage = (double *)h->desc.f[1];
    double *U0d = stage;
    double *bedd = need_bed ? stage + (size_t)m * plane : nullptr;
    if (on_device) {
        HIPCHK(h, hipMemcpyAsync(U0d, U0, sizeof(double) * m * plane, hipMemcpyDeviceToDevice, h->stream));
        if (need_bed)
            HIPCHK(h, hipMemcpyAsync(bedd, bed, sizeof(double) * plane, hipMemcpyDeviceToDevice, h->stream));
    } else {
        int rc = check_state(h, U0, need_bed ? bed : nullptr);
        if (rc) return rc;
        HIPCHK(h, copy_h2d(U0d, U0, sizeof(double) * m * plane, h->stream));
        if (need_bed) HIPCHK(h, copy_h2d(bedd, bed, sizeof(double) * plane, h->stream));
    }
    DevScalars sc{};
    sc.t[0] = t0;
    sc.first_bad_step = ~0ull;
    HIPCHK(h, hipMemcpyAsync(h->desc.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, L_reduce(h, U0d, 2));
    HIPCHK(h, L_init(h, U0d, bedd, 2));
    DevScalars got{};
    int rc = read_scalars(h, &got);
    if (rc) return rc;
    h->step = 0;
    const double ab0 = abar_host(got, 0, 0);
    const double ab1 = h->cfg.dim >= 2 ? abar_host(got, 0, 1) : 0.0;
    const double ab2 = h->cfg.dim == 3 ? abar_host(got, 0, 2) : 0.0;
    const double sa = (ab0 + ab1) + ab2;
    if (!(sa > 0.0)) return fail(h, ARLBM_EDEGENERATE, "sum of wave-speed bounds is zero: time step undefined");
    // Theorem 4.3: 0 < eps < (1/d)(1/CFL - 1) sum_j alpha_bar_j
    const double bound = (1.0 / h->cfg.dim) * (1.0 / h->cfg.cfl - 1.0) * sa;
    if (!(h->cfg.eps < bound)) return fail(h, ARLBM_EINVAL, "eps exceeds the stability bound of Theorem 4.3");
    return ARLBM_OK;
}

}  // namespace

// ------------------------------------------------------------------------
// Single lattice
// ------------------------------------------------------------------------

extern "C" int arlbm_config_init(arlbm_config *c)
{
    if (!c) return ARLBM_EINVAL;
    std::memset(c, 0, sizeof(*c));
    c->abi_version = ARLBM_ABI_VERSION;
    c->system = ARLBM_EULER;
    c->dim = 1;
    c->precision = ARLBM_F32;
    c->nx = 64;
    c->ny = 1;
    c->nz = 1;
    c->x0 = 0.0;
    c->x1 = 1.0;
    c->y0 = 0.0;
    c->y1 = 1.0;
    c->z0 = 0.0;
    c->z1 = 1.0;
    for (int i = 0; i < 6; ++i) c->bc[i] = ARLBM_TRANSMISSIVE;
    c->cfl = 0.5;
    c->eps = 1e-10;
    c->gamma = 1.4;
    c->g = 9.81;
    c->adv_speed[0] = 1.0;
    c->adv_speed[1] = 0.0;
    c->adv_speed[2] = 0.0;
    c->h_dry = 1e-6;
    c->rho_floor = 1e-12;
    c->p_floor = 1e-12;
    c->has_bed = 0;
    c->omega_mode = ARLBM_OMEGA_ADAPTIVE;
    c->omega_fixed = 2.0;
    return ARLBM_OK;
}

extern "C" int arlbm_query_sizes(const arlbm_config *cfg, arlbm_sizes *out)
{
    std::string e = check_config(cfg);
    if (!e.empty()) return fail(nullptr, ARLBM_EINVAL, e);
    if (!out) return fail(nullptr, ARLBM_EINVAL, "out is NULL");
    fill_sizes(cfg, out);
    return ARLBM_OK;
}

extern "C" int arlbm_create(const arlbm_config *cfg, const arlbm_buffers *bufs, void *stream, arlbm_lattice **out)
{
    if (!out) return fail(nullptr, ARLBM_EINVAL, "out is NULL");
    *out = nullptr;
    std::string e = check_config(cfg);
    if (!e.empty()) return fail(nullptr, ARLBM_EINVAL, e);
    arlbm_lattice *h = new arlbm_lattice();
    h->cfg = *cfg;
    fill_sizes(cfg, &h->sz);
    h->stream = (hipStream_t)stream;
    LatticeDesc &d = h->desc;
    d.variant = variant_of(cfg->system, cfg->dim);
    d.nx = (int32_t)cfg->nx;
    d.ny = (int32_t)cfg->ny;
    d.nz = (int32_t)cfg->nz;
    for (int i = 0; i < 6; ++i) d.bc[i] = cfg->bc[i];
    if (cfg->dim == 1) d.bc[2] = d.bc[3] = ARLBM_PERIODIC;
    if (cfg->dim <= 2) d.bc[4] = d.bc[5] = ARLBM_PERIODIC;
    d.omega_fixed_on = cfg->omega_mode == ARLBM_OMEGA_FIXED;
    d.cpl = columns_per_lane(cfg);
    // buffer-resource addressing: every plane offset and cell offset of the
    // population buffer in 32 bits
    d.buf = cfg->dim == 2 && h->sz.f_bytes <= 0xffffffffull ? 1 : 0;
    d.ncols = (int32_t)((cfg->nx + strip_out_w(d.cpl) - 1) / strip_out_w(d.cpl));
    // copies of each wave-speed slot: a 1D step launches one wave per strip,
    // and about 8 waves per copy keep its atomics from queueing while its
    // readers (on the critical path of a step of a few microseconds) load
    // fewer lines; 2D and 3D steps launch about a thousand waves or more
    d.abar_n = kAbarCopies;
    if (cfg->dim == 1) {
        d.abar_n = 1;
        while (d.abar_n < kAbarCopies && d.abar_n * 8 < d.ncols) d.abar_n *= 2;
    }
    d.band_h = cfg->dim == 2 ? choose_band(cfg->ny, d.ncols, resident_waves(cfg->precision, d.variant, d.cpl),
                                           4 * (int64_t)num_cus())
                             : 1;
    d.iter0 = 0;
    d.t_stop = HUGE_VAL;
    d.plane = cfg->nx * cfg->ny * cfg->nz;
    d.pstride = plane_stride(cfg);
    d.dx = (cfg->x1 - cfg->x0) / (double)cfg->nx;
    d.cfl = cfg->cfl;
    d.eps = cfg->eps;
    d.gamma = cfg->gamma;
    d.g = cfg->g;
    d.adv[0] = cfg->adv_speed[0];
    d.adv[1] = cfg->dim >= 2 ? cfg->adv_speed[1] : 0.0;
    d.adv[2] = cfg->dim == 3 ? cfg->adv_speed[2] : 0.0;
    d.h_dry = cfg->h_dry;
    d.rho_floor = cfg->rho_floor;
    d.p_floor = cfg->p_floor;
    d.omega_fixed = cfg->omega_fixed;
    d.q_heat = cfg->q_heat;
    d.k_rate = cfg->k_rate;
    d.t_act = cfg->t_act;
    if (bufs) {
        auto bad = [](const void *p) { return !p || ((uintptr_t)p % kAlign) != 0; };
        if (bad(bufs->f[0]) || bad(bufs->f[1]) || bad(bufs->u[0]) || bad(bufs->u[1]) || bad(bufs->scalars) ||
            (cfg->has_bed && bad(bufs->bed)) || (bufs->omega && ((uintptr_t)bufs->omega % kAlign) != 0)) {
            delete h;
            return fail(nullptr, ARLBM_EINVAL, "caller buffers must be non-NULL and 256-byte aligned");
        }
        for (int i = 0; i < 2; ++i) {
            d.f[i] = bufs->f[i];
            d.u[i] = bufs->u[i];
        }
        d.bed = cfg->has_bed ? bufs->bed : nullptr;
        d.sc = (DevScalars *)bufs->scalars;
        d.omega = bufs->omega;
    } else {
        h->owns = true;
        hipError_t err = hipSuccess;
        for (int i = 0; i < 2 && err == hipSuccess; ++i) {
            err = hipMalloc(&d.f[i], h->sz.f_bytes);
            if (err == hipSuccess) err = hipMalloc(&d.u[i], h->sz.u_bytes);
        }
        if (err == hipSuccess && cfg->has_bed) {
            void *b = nullptr;
            err = hipMalloc(&b, h->sz.bed_bytes);
            d.bed = b;
        }
        if (err == hipSuccess) err = hipMalloc((void **)&d.sc, h->sz.scalar_bytes);
        if (err != hipSuccess) {
            free_owned(h);
            delete h;
            return fail(nullptr, err == hipErrorOutOfMemory ? ARLBM_ENOMEM : ARLBM_EDEVICE,
                        std::string("device allocation failed: ") + hipGetErrorString(err));
        }
    }
    // without an omega plane the kernels store no omega (omega_on = 0)
    d.omega_on = d.omega ? 1 : 0;
    *out = h;
    return ARLBM_OK;
}

extern "C" int arlbm_set_state(arlbm_lattice *h, const double *U0, const double *bed, double t0)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    return set_state_impl(h, U0, bed, false, t0);
}

extern "C" int arlbm_set_state_device(arlbm_lattice *h, const double *U0, const double *bed, double t0)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    return set_state_impl(h, U0, bed, true, t0);
}

constexpr int32_t kSteps1dMaxStrips = 16, kSteps1dRun = 1024;

extern "C" int arlbm_step(arlbm_lattice *h, int64_t n)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    if (h->busy) return fail(h, ARLBM_EBUSY, "lattice is owned by a server");
    if (n < 0) return fail(h, ARLBM_EINVAL, "n must be >= 0");
    // a small 1D lattice takes its steps in launches of up to kSteps1dRun
    // steps of one workgroup (k_steps1d), the same bits as one launch per step
    if (h->cfg.dim == 1 && h->desc.ncols <= kSteps1dMaxStrips && n >= 2) {
        while (n > 0) {
            const int32_t k = (int32_t)std::min<int64_t>(n, kSteps1dRun);
            hipError_t e = is_f64(h) ? f64::steps1d(h->desc, h->step, k, h->stream)
                                     : f32::steps1d(h->desc, h->step, k, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "step launch");
            h->step += k;
            n -= k;
        }
        return ARLBM_OK;
    }
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = L_step(h, h->step);
        if (e != hipSuccess) return hip_fail(h, e, "step launch");
        ++h->step;
    }
    return ARLBM_OK;
}

extern "C" int arlbm_step_until(arlbm_lattice *h, double t_final, int64_t max_steps, int64_t *taken)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    if (h->busy) return fail(h, ARLBM_EBUSY, "lattice is owned by a server");
    if (max_steps < 0 || !(t_final == t_final)) return fail(h, ARLBM_EINVAL, "bad argument");
    DevScalars sc{};
    int rc = read_scalars(h, &sc);
    if (rc) return rc;
    const int64_t done0 = h->step - (int64_t)sc.null_launches;
    int64_t real = 0;
    h->desc.t_stop = t_final;
    while (real < max_steps) {
        const double t = sc.t[h->step % 3];
        if (t >= t_final) break;
        if (sc.flags & (ARLBM_FLAG_NONFINITE | ARLBM_FLAG_DEGENERATE)) break;
        // launch the estimated remaining steps plus one; a launch that finds
        // the state at or past t_final leaves it unchanged, so the surplus
        // costs one copy of the populations and the result does not depend
        // on the estimate
        const double est = sc.last_dt > 0.0 ? (t_final - t) / sc.last_dt : 1.0;
        int64_t k = est < 1e15 ? (int64_t)std::ceil(est) + 1 : 1;
        if (k > max_steps - real) k = max_steps - real;
        for (int64_t i = 0; i < k; ++i) {
            hipError_t e = L_step(h, h->step);
            if (e != hipSuccess) {
                h->desc.t_stop = HUGE_VAL;
                return hip_fail(h, e, "step launch");
            }
            ++h->step;
        }
        rc = read_scalars(h, &sc);
        if (rc) break;
        real = h->step - (int64_t)sc.null_launches - done0;
    }
    h->desc.t_stop = HUGE_VAL;
    if (rc) return rc;
    if (taken) *taken = real;
    return ARLBM_OK;
}

extern "C" int arlbm_sync(arlbm_lattice *h, arlbm_status *st)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    DevScalars sc{};
    int rc = read_scalars(h, &sc);
    if (rc) return rc;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        const int slot = (int)(h->step % 3);
        st->t = sc.t[slot];
        st->last_dt = sc.last_dt;
        st->abar[0] = abar_host(sc, slot, 0);
        st->abar[1] = h->cfg.dim >= 2 ? abar_host(sc, slot, 1) : 0.0;
        st->abar[2] = h->cfg.dim == 3 ? abar_host(sc, slot, 2) : 0.0;
        st->step = h->step - (int64_t)sc.null_launches;
        st->flags = sc.flags;
        st->first_bad_step = sc.first_bad_step == ~0ull ? -1 : (int64_t)sc.first_bad_step;
    }
    if (sc.flags & ARLBM_FLAG_NONFINITE) return fail(h, ARLBM_ENONFINITE, "a moment became non-finite");
    if (sc.flags & ARLBM_FLAG_DEGENERATE) return fail(h, ARLBM_EDEGENERATE, "sum of wave-speed bounds became zero");
    if (sc.flags & ARLBM_FLAG_POSITIVITY) return fail(h, ARLBM_EPOSITIVITY, "a density, pressure or depth fell below its floor");
    return ARLBM_OK;
}

// Enqueue the copy of m strided device planes (stride pstride) to dense host
// FP64 planes (FP32 data through the population buffer the step does not
// read next).
static int read_planes_async(arlbm_lattice *h, const void *src, int m, double *out)
{
    const int64_t plane = h->desc.plane, ps = h->desc.pstride;
    if (is_f64(h)) {
        HIPCHK(h, hipMemcpy2DAsync(out, sizeof(double) * plane, src, sizeof(double) * ps, sizeof(double) * plane, m,
                                   hipMemcpyDeviceToHost, h->stream));
    } else {
        double *stage = (double *)h->desc.f[(h->step + 1) & 1];
        HIPCHK(h, f32::to_double(src, stage, plane, ps, m, h->stream));
        HIPCHK(h, hipMemcpyAsync(out, stage, sizeof(double) * plane * m, hipMemcpyDeviceToHost, h->stream));
    }
    return ARLBM_OK;
}

// The same into pageable host memory, returning with out written: large
// reads are packed as FP64 into the population buffer the step does not read
// next and moved through the pinned chunks of copy_d2h.
static int read_planes(arlbm_lattice *h, const void *src, int m, double *out)
{
    const int64_t plane = h->desc.plane, ps = h->desc.pstride;
    const size_t bytes = sizeof(double) * (size_t)plane * m;
    if (bytes < kBounceMin) {
        int rc = read_planes_async(h, src, m, out);
        if (rc) return rc;
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return ARLBM_OK;
    }
    double *stage = (double *)h->desc.f[(h->step + 1) & 1];
    if (is_f64(h))
        HIPCHK(h, hipMemcpy2DAsync(stage, sizeof(double) * plane, src, sizeof(double) * ps, sizeof(double) * plane, m,
                                   hipMemcpyDeviceToDevice, h->stream));
    else
        HIPCHK(h, f32::to_double(src, stage, plane, ps, m, h->stream));
    HIPCHK(h, copy_d2h(out, stage, bytes, h->stream));
    return ARLBM_OK;
}

// Form U = sum_k f_k of the current state in u[step & 1] (the step kernels
// do not store the moments).
static int form_moments(arlbm_lattice *h)
{
    void *u = h->desc.u[h->step & 1];
    const void *f = h->desc.f[h->step & 1];
    HIPCHK(h, is_f64(h) ? f64::moments(f, u, h->desc.plane, h->desc.pstride, h->sz.m, h->sz.q, h->stream)
                        : f32::moments(f, u, h->desc.plane, h->desc.pstride, h->sz.m, h->sz.q, h->stream));
    return ARLBM_OK;
}

extern "C" int arlbm_read_moments(arlbm_lattice *h, double *U)
{
    if (!h || !U) return fail(h, ARLBM_EINVAL, "NULL argument");
    int rc = form_moments(h);
    if (rc) return rc;
    return read_planes(h, h->desc.u[h->step & 1], h->sz.m, U);
}

extern "C" int arlbm_set_omega_export(arlbm_lattice *h, int on)
{
    if (!h) return fail(nullptr, ARLBM_EINVAL, "handle is NULL");
    if (on && !h->desc.omega_on) {
        void *p = nullptr;
        HIPCHK(h, hipMalloc(&p, h->sz.omega_bytes));
        HIPCHK(h, hipMemsetAsync(p, 0, h->sz.omega_bytes, h->stream));
        h->desc.omega = p;
        h->desc.omega_on = 1;
        h->owns_omega = true;
    } else if (!on && h->desc.omega_on) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        if (h->owns_omega) (void)hipFree(h->desc.omega);
        h->desc.omega = nullptr;
        h->desc.omega_on = 0;
        h->owns_omega = false;
    }
    return ARLBM_OK;
}

extern "C" int arlbm_read_omega(arlbm_lattice *h, double *omega)
{
    if (!h || !omega) return fail(h, ARLBM_EINVAL, "NULL argument");
    if (!h->desc.omega_on) return fail(h, ARLBM_EINVAL, "omega export is off");
    return read_planes(h, h->desc.omega, 1, omega);
}

// Sums of each field from the per-block partials (compensated, in a fixed
// order), then the partials' reduction on the host in a fixed order.
static int conservation_impl(arlbm_lattice *h, double *partial, double *sums)
{
    const int m = h->sz.m;
    const void *u = h->desc.u[h->step & 1];
    hipError_t e = is_f64(h) ? f64::conservation(u, h->desc.plane, h->desc.pstride, m, partial, kConsBlocks,
                                                 h->stream)
                             : f32::conservation(u, h->desc.plane, h->desc.pstride, m, partial, kConsBlocks,
                                                 h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "conservation launch");
    double part[kConsMaxFields * kConsBlocks];
    HIPCHK(h, hipMemcpyAsync(part, partial, sizeof(double) * m * kConsBlocks, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int c = 0; c < m; ++c) {
        double s = 0.0, comp = 0.0;
        for (int b = 0; b < kConsBlocks; ++b) {
            const double v = part[c * kConsBlocks + b];
            const double t = s + v;
            comp += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
            s = t;
        }
        sums[c] = s + comp;
    }
    return ARLBM_OK;
}

extern "C" int arlbm_conservation(arlbm_lattice *h, double *sums)
{
    if (!h || !sums) return fail(h, ARLBM_EINVAL, "NULL argument");
    int rc = form_moments(h);
    if (rc) return rc;
    // per-block partials of up to kConsMaxFields fields, allocated on the
    // first request, so that a lattice that never asks allocates nothing
    if (!h->d_partial)
        HIPCHK(h, hipMalloc((void **)&h->d_partial, sizeof(double) * kConsBlocks * kConsMaxFields));
    return conservation_impl(h, h->d_partial, sums);
}

extern "C" int arlbm_conservation_noalloc(arlbm_lattice *h, double *sums)
{
    if (!h || !sums) return fail(h, ARLBM_EINVAL, "NULL argument");
    if (h->sz.m > kConsMaxFields)
        return fail(h, ARLBM_EINVAL, "the conservation scratch holds partial sums of at most 6 fields");
    double *partial = nullptr;
    HIPCHK(h, conservation_scratch(&partial));
    int rc = form_moments(h);
    if (rc) return rc;
    return conservation_impl(h, partial, sums);
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t precision, variant, nx, ny, nz, pad;
    int64_t step;
    uint64_t f_bytes, u_bytes;
};
constexpr uint64_t kMagic = 0x41524c424d535432ull;  // "ARLBMST2"
}  // namespace

extern "C" int arlbm_state_bytes(arlbm_lattice *h, size_t *bytes)
{
    if (!h || !bytes) return fail(h, ARLBM_EINVAL, "NULL argument");
    *bytes = sizeof(StateHeader) + h->sz.f_bytes + h->sz.u_bytes + sizeof(DevScalars);
    return ARLBM_OK;
}

extern "C" int arlbm_save_state(arlbm_lattice *h, void *blob, size_t bytes)
{
    size_t need = 0;
    int rc = arlbm_state_bytes(h, &need);
    if (rc) return rc;
    if (!blob || bytes < need) return fail(h, ARLBM_EINVAL, "state buffer too small");
    StateHeader hd{kMagic, h->cfg.precision, h->desc.variant, h->desc.nx, h->desc.ny, h->desc.nz, 0, h->step,
                   h->sz.f_bytes,
                   h->sz.u_bytes};
    char *p = (char *)blob;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    HIPCHK(h, hipMemcpyAsync(p, h->desc.f[h->step & 1], h->sz.f_bytes, hipMemcpyDeviceToHost, h->stream));
    p += h->sz.f_bytes;
    HIPCHK(h, hipMemcpyAsync(p, h->desc.u[h->step & 1], h->sz.u_bytes, hipMemcpyDeviceToHost, h->stream));
    p += h->sz.u_bytes;
    HIPCHK(h, hipMemcpyAsync(p, h->desc.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return ARLBM_OK;
}

extern "C" int arlbm_load_state(arlbm_lattice *h, const void *blob, size_t bytes)
{
    size_t need = 0;
    int rc = arlbm_state_bytes(h, &need);
    if (rc) return rc;
    if (!blob || bytes < need) return fail(h, ARLBM_EINVAL, "state buffer too small");
    StateHeader hd;
    std::memcpy(&hd, blob, sizeof(hd));
    if (hd.magic != kMagic || hd.precision != h->cfg.precision || hd.variant != h->desc.variant ||
        hd.nx != h->desc.nx || hd.ny != h->desc.ny || hd.nz != h->desc.nz || hd.f_bytes != h->sz.f_bytes ||
        hd.u_bytes != h->sz.u_bytes)
        return fail(h, ARLBM_EINVAL, "state blob does not match this lattice");
    h->step = hd.step;
    const char *p = (const char *)blob + sizeof(hd);
    HIPCHK(h, hipMemcpyAsync(h->desc.f[h->step & 1], p, h->sz.f_bytes, hipMemcpyHostToDevice, h->stream));
    p += h->sz.f_bytes;
    HIPCHK(h, hipMemcpyAsync(h->desc.u[h->step & 1], p, h->sz.u_bytes, hipMemcpyHostToDevice, h->stream));
    p += h->sz.u_bytes;
    HIPCHK(h, hipMemcpyAsync(h->desc.sc, p, sizeof(DevScalars), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return ARLBM_OK;
}

extern "C" int arlbm_destroy(arlbm_lattice *h)
{
    if (!h) return ARLBM_OK;
    (void)hipStreamSynchronize(h->stream);
    free_owned(h);
    delete h;
    return ARLBM_OK;
}

extern "C" const char *arlbm_last_error(const arlbm_lattice *h)
{
    return h ? h->err.c_str() : g_thread_err.c_str();
}

// Diagnostics used by the benchmark: registers of the fused step kernel
// (2D: the kernel a lattice of even nx runs).
extern "C" int arlbm_step_kernel_vgprs(int32_t precision, int32_t system, int32_t dim)
{
    if (system < 0 || system > 3 || dim < 1 || dim > 3) return -1;
    const int v = variant_of(system, dim);
    arlbm_config c{};
    c.precision = precision;
    c.system = system;
    c.dim = dim;
    c.nx = 2;
    const int cpl = columns_per_lane(&c);
    return precision == ARLBM_F64 ? f64::step_kernel_vgprs(v, cpl) : f32::step_kernel_vgprs(v, cpl);
}

// ------------------------------------------------------------------------
// Server
// ------------------------------------------------------------------------
//
// Everything a served lattice needs runs on the server's one stream, in
// order: its upload and initialisation, the batched steps, its read-back.
// Device memory therefore never needs a synchronisation before reuse: a
// block released by a retiring lattice is written by a later admission only
// after the read-back that precedes it in the stream.  Uploads and
// read-backs go through pinned host blocks, and each iteration enqueues the
// retirements, the admissions and the table upload before its batched
// launch and finishes them (result copies, admission checks) after it, so
// the host work overlaps the launch instead of leaving the GPU idle.  Served
// lattices take their buffers from a pool of device blocks in size classes:
// once the pool is warm, serving calls neither hipMalloc nor hipFree.

namespace {
// Host arrays the server keeps (queued initial states, results): left
// uninitialised when allocated, since a parallel copy fills them at once.
// Host arrays of queued states and results.  Large ones are 2 MiB aligned
// and advised for transparent huge pages, so that their first touch (the
// copy into them) takes one fault per 2 MiB instead of per 4 KiB.
struct HostArray {
    struct Free {
        void operator()(double *q) const { free(q); }
    };
    std::unique_ptr<double, Free> p;
    size_t n = 0;
    bool alloc(size_t count)  // false when the memory is not there
    {
        constexpr size_t kHuge = (size_t)2 << 20;
        const size_t bytes = sizeof(double) * count;
        void *q = nullptr;
        if (count && posix_memalign(&q, bytes >= 2 * kHuge ? kHuge : 64, bytes) != 0) q = nullptr;
        if (q && bytes >= 2 * kHuge) (void)madvise(q, bytes / kHuge * kHuge, MADV_HUGEPAGE);
        p.reset((double *)q);
        n = p ? count : 0;
        return p || count == 0;
    }
    double *data() { return p.get(); }
    const double *data() const { return p.get(); }
    size_t size() const { return n; }
};

struct Pending {
    uint64_t id;
    arlbm_config cfg;
    HostArray U0, bed;
    std::unique_ptr<char[]> blob;  // a saved state to resume instead of U0 (and its step)
    size_t blob_bytes = 0;
    int64_t step0 = 0;
    int64_t nsteps;
    double submit_s;
    size_t bytes;  // device memory charged: the size class of the lattice's block
    double *dst = nullptr;  // caller memory for the result (arlbm_server_result_into), or none
};
struct Resident {
    uint64_t id;
    arlbm_lattice *lat;
    int64_t iter0;     // the lattice's step index is iter - iter0 (iter0 = admission - step0)
    int64_t admit_it;  // server iteration at admission
    int64_t end_it;    // iteration at which it has taken its steps
    double submit_s, admit_s;
    size_t bytes;
    void *dev;       // the lattice's device block (pool)
    size_t dev_cls;  // its size class
    double *dst;     // caller memory for the result, or nullptr
};
struct Done {
    arlbm_completion c;
    HostArray U;
};
// An admission or a retirement whose transfers are in the stream, finished
// after the iteration's launch.
struct Staged {
    enum Kind { ADMIT, ADMIT_STATE, RETIRE } kind;
    uint64_t id;
    arlbm_lattice *lat;
    int64_t steps;  // retirement: steps taken in the server
    double submit_s, admit_s;
    void *host;  // pinned block: scalars [, scalars out], planes
    size_t host_cls;
    hipEvent_t ev;
    double *dst = nullptr;  // retirement: caller memory for the result, or nullptr
};

// Size classes a quarter octave apart (a block is at most 25% larger than
// asked), at least 64 KiB.
size_t size_class(size_t n)
{
    if (n <= ((size_t)1 << 16)) return (size_t)1 << 16;
    const int lg = 63 - __builtin_clzll((unsigned long long)n);
    const size_t q = (size_t)1 << (lg - 2);
    return (n + q - 1) / q * q;
}

// Free lists of device or pinned host blocks per size class.  Free blocks are
// given back (largest first) when the blocks held would exceed cap.  A free
// device block may still be read by work queued before its release (a
// retiring lattice's read-back), so giving one back first waits for the
// stream; a pinned block is released only after its transfers completed.
struct BlockPool {
    bool pinned = false;
    hipStream_t stream = nullptr;
    size_t cap = 0;
    size_t free_bytes = 0, used_bytes = 0;
    std::vector<std::pair<size_t, void *>> free_blocks;  // (class, pointer)

    void give_back(void *p)
    {
        if (pinned) {
            (void)hipHostFree(p);
        } else {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(p);
        }
    }
    void drop_largest()
    {
        auto it = std::max_element(free_blocks.begin(), free_blocks.end(),
                                   [](const auto &a, const auto &b) { return a.first < b.first; });
        free_bytes -= it->first;
        give_back(it->second);
        free_blocks.erase(it);
    }
    void *acquire(size_t n, size_t *cls_out)
    {
        const size_t cls = size_class(n);
        for (size_t i = 0; i < free_blocks.size(); ++i) {
            if (free_blocks[i].first != cls) continue;
            void *p = free_blocks[i].second;
            free_blocks[i] = free_blocks.back();
            free_blocks.pop_back();
            free_bytes -= cls;
            used_bytes += cls;
            *cls_out = cls;
            return p;
        }
        while (!free_blocks.empty() && used_bytes + free_bytes + cls > cap) drop_largest();
        void *p = nullptr;
        for (int attempt = 0; attempt < 2; ++attempt) {
            const hipError_t e = pinned ? hipHostMalloc(&p, cls, hipHostMallocDefault) : hipMalloc(&p, cls);
            if (e == hipSuccess) break;
            p = nullptr;
            (void)hipGetLastError();
            while (!free_blocks.empty()) drop_largest();
        }
        if (!p) return nullptr;
        used_bytes += cls;
        *cls_out = cls;
        return p;
    }
    void release(void *p, size_t cls)
    {
        used_bytes -= cls;
        free_blocks.emplace_back(cls, p);
        free_bytes += cls;
        while (!free_blocks.empty() && used_bytes + free_bytes > cap) drop_largest();
    }
    void clear()
    {
        while (!free_blocks.empty()) drop_largest();
    }
};
}  // namespace

struct arlbm_server {
    size_t budget = 0, in_use = 0;
    int32_t precision = ARLBM_F32;
    hipStream_t stream = nullptr;
    uint64_t next_id = 1;
    int64_t iter = 0;
    std::deque<Pending> queue;
    std::vector<Resident> resident;
    std::vector<Staged> staged;
    std::deque<Done> done;
    std::vector<Done> handed;  // results returned by the last poll
    BlockPool dev, pin;
    // device work table: descriptors, the start of each XCD's part of the
    // work list (kQueues + 1 entries), the work list; one allocation
    char *d_table = nullptr;
    size_t cap_table = 0;
    // pinned host copies of the work table, two used in turn; one is
    // rewritten only after the upload that read it (its event) has completed
    char *h_table[2] = {nullptr, nullptr};
    size_t hcap_table[2] = {0, 0};
    hipEvent_t table_ev[2] = {nullptr, nullptr};
    int table_set = 0;
    // the batched launches of a step (launch_groups): waves and the byte
    // offsets of the queue starts and items in the table
    struct Launch {
        int32_t nwaves;
        size_t off_start, off_segs;
    };
    std::vector<Launch> launches;
    // queue counters of the batched launch: two sets (launch parity) of
    // kQueues counters 128 bytes apart; a launch takes items with one set and
    // zeroes the other for the next launch
    unsigned *d_counters = nullptr;
    int64_t batched_launches = 0;  // its parity picks the counter set
    // flag words of the residents gathered after each call's launches (two
    // in turn), read by a later call once their copy has completed: a
    // lattice that became non-finite or degenerate retires early
    unsigned *d_flags = nullptr;
    size_t cap_flags = 0;
    struct FlagGather {
        unsigned *host = nullptr;  // pinned
        size_t cap = 0;
        std::vector<uint64_t> ids;  // resident ids in gather order
        hipEvent_t ev = nullptr;
        bool pending = false;
    } gather[2];
    int gather_next = 0;
    std::vector<uint64_t> failing;  // residents seen with a fatal flag
    bool dirty = true;
    std::string err;
};

namespace {

int sfail(arlbm_server *s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    g_thread_err = msg;
    return code;
}

// Byte offsets of a lattice's buffers inside its device block, in the order
// f[0], f[1], u[0], u[1], bed, scalars (every size is a multiple of 256).
arlbm_buffers carve(void *blk, const arlbm_sizes &sz, bool has_bed)
{
    char *b = (char *)blk;
    arlbm_buffers r{};
    r.f[0] = b;
    r.f[1] = b + sz.f_bytes;
    r.u[0] = b + 2 * sz.f_bytes;
    r.u[1] = b + 2 * sz.f_bytes + sz.u_bytes;
    r.bed = has_bed ? b + 2 * sz.f_bytes + 2 * sz.u_bytes : nullptr;
    r.scalars = b + 2 * sz.f_bytes + 2 * sz.u_bytes + sz.bed_bytes;
    r.omega = nullptr;
    return r;
}

// A served lattice's handle: its buffers belong to the server's pool and
// no kernel touches them after this point in the stream, so nothing waits.
void drop_handle(arlbm_lattice *h)
{
    free_owned(h);
    delete h;
}

void push_failed(arlbm_server *s, uint64_t id, int rc, double submit_s)
{
    Done d{};
    d.c.id = id;
    d.c.status = rc;
    d.c.submit_s = submit_s;
    d.c.done_s = now_s();
    s->done.push_back(std::move(d));
}

// Served lattices that the batched kernel does not step: 3D lattices (their
// fused z-marching step keeps tiles of moments and indicators in LDS, a
// launch shape of its own) and 2D lattices whose population buffer spans
// 4 GiB or more (the batched kernel addresses planes through 32-bit buffer
// offsets).
bool own_launch(const LatticeDesc &d) { return d.variant >= V_ADV3 || (d.variant >= V_ADV2 && !d.buf); }

// Work list of the batched launch.  The work of every resident 1D and 2D
// lattice is cut into items (row bands of 2D strips, runs of 1D strips),
// and the launch's waves, one per SIMD, take items from a queue until it is
// empty.  The items are taken in list order, so the items the waves hold at
// any moment are neighbours in the list: the list holds each lattice's bands
// in order, each band's strips left to right, so those waves march over the
// same rows of neighbouring strips (their halo columns are in each other's
// L2, and the concurrent reads cover whole plane rows).  The list is cut
// into kQueues parts, one per XCD; a wave takes items from its XCD's part
// first (blocks are dealt to the XCDs round robin, so block b runs on XCD
// b mod 8), its first one as a static deal would give it, then from the
// part with the most items left.
//
// Item height: the whole work is r rounds of the launch's waves, with r as
// small as keeps bands of at most 256 rows, and every 2D lattice is cut into
// bands of equal height, about h = (strip rows) / (r waves) rows (at least
// 8); in a single round h is the lowest height whose items all fit the
// waves.  A lattice alone thus gets the single-lattice kernel's bands, one
// per wave (2048^2 Euler: 28 bands of 74 rows of its 36 strips); a large mix
// gets about r items per wave, which the queues balance.  Lattices with the
// tallest bands come first.  Each part holds a contiguous range of the bands
// (equal counts in one round, so that every band is a wave's first item;
// about equal work over several rounds), then every kQueues-th 1D run, the
// largest first: the runs fill the waves whose bands end early.  A run
// spreads the 1D strips over the waves the bands leave free (a 1D lattice
// alone: about one strip per wave, as in the single-lattice kernel), or,
// when the bands leave fewer than an eighth of the waves free, over all of
// them in runs of at least 8 strips; it is never longer than about one 2D
// item's work.  Cost model, in population values a wave moves: a 2D item
// of h rows costs (h + 6) rows of 64 V lanes by Q m values (the march reads
// 3 rows of moments beyond each end and collides one row beyond each end);
// a 1D strip costs 64 Q m values plus a latency share of one 1280-value row,
// and a run two strips more.
//
// Measured on the 65 lattices of the fixed serving mix (ms per launch):
// parts of equal work in one round and the 1D runs at the end of the list
// put a few bands of one part behind its XCD's waves, and the other XCDs'
// waves first took the small 1D runs the list ended with (the mix's 2D
// Euler lattices with its 1D ones 0.552, with one 1D lattice 0.469 against
// 0.387 alone; now 0.395); the whole mix 0.826 -> 0.809.  Bands of exactly h
// rows with the rows left over as short items (0.83), the last eighth of
// the 2D work in bands a quarter as tall (0.88), and one round of bands up
// to 384 rows (0.90) measured slower.  Dealing the items statically
// instead (consecutive items per wave) gave the same times for one item per
// wave, but two or more put a wave's items one after the other on its own,
// so neighbouring waves no longer marched over neighbouring strips: 4096^2
// shallow water 0.46 -> 0.70 ms per step, all 512 requests of the serving
// mix resident 21 -> 15 GLUPS; and cutting strips into row ranges dealt
// down each strip put the waves of one XCD at scattered rows (2048^2 Euler
// 51% slower than the single-lattice kernel).
constexpr int kWarmRows2d = 6, kWarmStrips1d = 2, kMinRows2d = 8, kMaxRows2d = 256;
constexpr int64_t kStrip1dLatency = 1280, kRowValues = 1280, kRun1dMix = 8;

int64_t batched_waves() { return 4 * (int64_t)num_cus(); }  // one wave per SIMD

struct SchedLattice {
    int32_t lattice;
    bool one_d;
    int32_t ncols;  // strips
    int64_t ny;     // 2D rows
    int64_t unit;   // cost per row (2D) or per strip (1D)
};

// The band height h of a one-launch schedule for these lattices and its
// rounds r (items per wave): the lowest height at most kMaxRows2d that puts
// at most one item on every wave, else two or more rounds.
void band_height(const std::vector<SchedLattice> &lats, int64_t W, int64_t &h, int64_t &r)
{
    int64_t S = 0;  // 2D strip rows
    for (const SchedLattice &l : lats)
        if (!l.one_d) S += (int64_t)l.ncols * l.ny;
    h = kMaxRows2d;
    r = 1;
    if (S > 0) {
        r = std::max<int64_t>(1, (S + W * kMaxRows2d - 1) / (W * kMaxRows2d));
        h = std::max<int64_t>(kMinRows2d, (S + W * r - 1) / (W * r));
        auto items_at = [&](int64_t hh) {
            int64_t n = 0;
            for (const SchedLattice &l : lats)
                if (!l.one_d) n += (int64_t)l.ncols * ((l.ny + std::min(hh, l.ny) - 1) / std::min(hh, l.ny));
            return n;
        };
        if (r == 1) {
            // one round: the lowest height whose items all fit the waves (a
            // second round for a few items would double the step time)
            while (items_at(h) > W && h < kMaxRows2d) ++h;
            if (items_at(h) > W) {
                r = 2;
                h = std::max<int64_t>(kMinRows2d, (S + W * r - 1) / (W * r));
            }
        }
    }
}

// Items in queue order and the start of each XCD's part (kQueues + 1
// entries); returns the number of waves to launch.
int64_t build_schedule(const std::vector<SchedLattice> &lats, int64_t W, std::vector<Segment> &segs,
                       std::vector<int32_t> &qstart)
{
    segs.clear();
    qstart.assign(kQueues + 1, 0);
    int64_t h, r;
    band_height(lats, W, h, r);
    // each lattice in bands of equal height, at most h; lattices with the
    // tallest bands first
    struct Item {
        Segment seg;
        double cost;
    };
    std::vector<Item> big, small;
    std::vector<std::pair<int64_t, const SchedLattice *>> order;  // (band height, lattice)
    for (const SchedLattice &l : lats) {
        if (l.one_d) continue;
        const int64_t hl = std::min(h, l.ny);
        const int64_t nb = (l.ny + hl - 1) / hl;
        order.push_back({(l.ny + nb - 1) / nb, &l});
    }
    std::stable_sort(order.begin(), order.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    for (const auto &o : order) {
        const SchedLattice &l = *o.second;
        for (int64_t y0 = 0; y0 < l.ny; y0 += o.first) {
            const int64_t y1 = std::min<int64_t>(l.ny, y0 + o.first);
            for (int32_t c = 0; c < l.ncols; ++c)
                big.push_back({{l.lattice, c, (int32_t)y0, (int32_t)y1}, (double)(y1 - y0 + kWarmRows2d) * (double)l.unit});
        }
    }
    // 1D runs, no longer than about one 2D item's work.  Where the 2D items
    // leave at least an eighth of the waves free, the 1D strips are spread
    // over those (a 1D lattice alone: about one strip per wave); otherwise
    // over all the waves in runs of at least kRun1dMix strips, which the
    // waves take as their 2D items end.
    int64_t strips1d = 0;
    for (const SchedLattice &l : lats)
        if (l.one_d) strips1d += l.ncols;
    const int64_t free_waves = W - (int64_t)big.size();
    const int64_t spread = free_waves > 0 && free_waves >= W / 8 ? (strips1d + free_waves - 1) / free_waves
                                               : std::max<int64_t>((strips1d + W - 1) / W, kRun1dMix);
    for (const SchedLattice &l : lats) {
        if (!l.one_d) continue;
        const int64_t cap = std::max<int64_t>(1, (h + kWarmRows2d) * kRowValues / l.unit - kWarmStrips1d);
        const int64_t per = std::max<int64_t>(1, std::min(spread, cap));
        for (int64_t c = 0; c < l.ncols; c += per) {
            const int64_t e = std::min<int64_t>(l.ncols, c + per);
            small.push_back({{l.lattice, (int32_t)c, 0, (int32_t)e}, (double)(e - c + kWarmStrips1d) * (double)l.unit});
        }
    }
    std::stable_sort(small.begin(), small.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    // each queue: a contiguous part of the bands, then every kQueues-th of
    // the smaller items (largest first), which fill the waves that finish
    // early.  In one round the parts have equal counts, so that every band is
    // a first item (a queue with more bands than its XCD's waves would leave
    // the extra ones to waves that first take the other queues' small items);
    // over several rounds they carry about equal work.
    std::vector<size_t> bstart(kQueues + 1, big.size());
    bstart[0] = 0;
    if (r == 1) {
        const size_t per = (big.size() + kQueues - 1) / kQueues;
        for (int q = 1; q < kQueues; ++q) bstart[q] = std::min(big.size(), per * q);
    } else {
        double total = 0.0;
        for (const Item &it : big) total += it.cost;
        double acc = 0.0;
        int q = 1;
        for (size_t k = 0; k < big.size() && q < kQueues; ++k) {
            acc += big[k].cost;
            while (q < kQueues && acc >= total * q / kQueues) bstart[q++] = k + 1;
        }
    }
    for (int q = 0; q < kQueues; ++q) {
        qstart[q] = (int32_t)segs.size();
        for (size_t k = bstart[q]; k < bstart[q + 1]; ++k) segs.push_back(big[k].seg);
        for (size_t k = q; k < small.size(); k += kQueues) segs.push_back(small[k].seg);
    }
    qstart[kQueues] = (int32_t)segs.size();
    return std::min<int64_t>(W, (int64_t)segs.size());
}

// Launch groups of the batched step.  When the resident 2D work needs more
// than one round of the waves, one launch would deal several bands to each
// wave, and its items differ in cost per row (a shallow-water strip of two
// columns per lane moves 1.5 times an Euler strip's bytes per row, one of one
// column 0.75 times): the waves end far apart.  The lattices are instead
// split into groups of one cost per strip row, each group one launch of one
// round sized to fill the waves, the launches one after the other on the
// stream (every lattice in exactly one group, so it is stepped once per
// iteration with the same bits).  A class with fewer than kMinGroupRows
// rows per wave joins the class nearest in cost; a class still needing more
// than one round is split, largest lattices first into the group with the
// least work, into the fewest groups that each fit one round (a single
// lattice that does not cannot be shortened by any split); the 1D lattices
// join the heaviest group, whose waves take their runs as bands end; past
// kMaxGroups groups, one launch.  The fixed serving mix (20 Euler, 15 + 8
// shallow-water and 22 1D lattices) took 0.812 ms per step in one launch,
// 0.722 in two (Euler; shallow water and 1D), 0.848 in two of mixed classes
// balanced by work, 0.902 in one launch of one round with bands of equal
// cost (158-487 rows); in the three classes 0.708 with the 1D lattices in
// the lightest group, 0.712 in a launch of their own, 0.690 in the
// heaviest.
// Returns the group of each lattice (0 .. groups-1).
constexpr int64_t kMaxGroups = 8, kMinGroupRows = 24;
std::vector<int32_t> launch_groups(const std::vector<SchedLattice> &lats, int64_t W, int64_t &ngroups)
{
    std::vector<int32_t> grp(lats.size(), 0);
    ngroups = 1;
    int64_t h, r;
    band_height(lats, W, h, r);
    if (r == 1) return grp;
    auto rows = [&](size_t i) { return lats[i].one_d ? (int64_t)0 : (int64_t)lats[i].ncols * lats[i].ny; };
    // classes of one cost per strip row
    struct Class {
        int64_t unit, rows;
        std::vector<size_t> members;
    };
    std::vector<Class> cls;
    for (size_t i = 0; i < lats.size(); ++i) {
        if (lats[i].one_d) continue;
        auto it = std::find_if(cls.begin(), cls.end(), [&](const Class &c) { return c.unit == lats[i].unit; });
        if (it == cls.end()) {
            cls.push_back({lats[i].unit, 0, {}});
            it = cls.end() - 1;
        }
        it->rows += rows(i);
        it->members.push_back(i);
    }
    auto ratio = [](int64_t a, int64_t b) { return a > b ? (double)a / (double)b : (double)b / (double)a; };
    auto merge_into_nearest = [&](size_t k) {
        size_t best = k;
        for (size_t j = 0; j < cls.size(); ++j)
            if (j != k && (best == k || ratio(cls[j].unit, cls[k].unit) < ratio(cls[best].unit, cls[k].unit)))
                best = j;
        cls[best].rows += cls[k].rows;
        cls[best].members.insert(cls[best].members.end(), cls[k].members.begin(), cls[k].members.end());
        cls.erase(cls.begin() + (long)k);
    };
    for (bool again = true; again && cls.size() > 1;) {
        again = false;
        size_t k = 0;
        for (size_t j = 1; j < cls.size(); ++j)
            if (cls[j].rows < cls[k].rows) k = j;
        if (cls[k].rows < W * kMinGroupRows) {
            merge_into_nearest(k);
            again = true;
        }
    }
    while ((int64_t)cls.size() > kMaxGroups) {
        size_t k = 0;
        for (size_t j = 1; j < cls.size(); ++j)
            if (cls[j].rows < cls[k].rows) k = j;
        merge_into_nearest(k);
    }
    // each class in the fewest groups that fit one round
    std::vector<std::vector<size_t>> groups;
    for (Class &c : cls) {
        std::stable_sort(c.members.begin(), c.members.end(), [&](size_t a, size_t b) { return rows(a) > rows(b); });
        const int64_t nmax = std::min<int64_t>(kMaxGroups, (int64_t)c.members.size());
        std::vector<std::vector<size_t>> best;
        for (int64_t g = 1; g <= nmax && best.empty(); ++g) {
            std::vector<std::vector<size_t>> part(g);
            std::vector<int64_t> load(g, 0);
            for (size_t i : c.members) {
                const int64_t k = std::min_element(load.begin(), load.end()) - load.begin();
                part[k].push_back(i);
                load[k] += rows(i);
            }
            bool ok = true;
            for (const auto &pg : part) {
                std::vector<SchedLattice> sub;
                for (size_t i : pg) sub.push_back(lats[i]);
                int64_t hk, rk;
                band_height(sub, W, hk, rk);
                ok = ok && (rk == 1 || pg.size() == 1);
            }
            if (ok) best = part;
        }
        if (best.empty()) best.push_back(c.members);
        for (auto &pg : best) groups.push_back(pg);
    }
    if (groups.size() < 2 || (int64_t)groups.size() > kMaxGroups) return grp;
    std::vector<double> cost(groups.size(), 0.0);
    for (size_t k = 0; k < groups.size(); ++k)
        for (size_t i : groups[k]) {
            grp[i] = (int32_t)k;
            cost[k] += (double)rows(i) * (double)lats[i].unit;
        }
    const int32_t heavy = (int32_t)(std::max_element(cost.begin(), cost.end()) - cost.begin());
    for (size_t i = 0; i < lats.size(); ++i)
        if (lats[i].one_d) grp[i] = heavy;
    ngroups = (int64_t)groups.size();
    return grp;
}

// A schedule item of lattice i from its descriptor (1D and 2D lattices the
// batched kernel steps).
SchedLattice sched_lattice(int32_t i, const LatticeDesc &d)
{
    const int m = num_fields(d.variant % 4, d.variant / 4 + 1);
    if (d.variant >= V_ADV2) return {i, false, d.ncols, d.ny, (int64_t)kWave * d.cpl * 5 * m};
    return {i, true, d.ncols, 1, (int64_t)kWave * 3 * m + kStrip1dLatency};
}

int rebuild_table(arlbm_server *s)
{
    std::vector<LatticeDesc> descs;
    std::vector<SchedLattice> lats;
    for (size_t i = 0; i < s->resident.size(); ++i) {
        LatticeDesc d = s->resident[i].lat->desc;
        d.iter0 = s->resident[i].iter0;
        descs.push_back(d);
        if (!own_launch(d)) lats.push_back(sched_lattice((int32_t)i, d));
    }
    // one schedule per launch group, laid out after the descriptors
    int64_t ng = 0;
    const std::vector<int32_t> grp = lats.empty() ? std::vector<int32_t>() : launch_groups(lats, batched_waves(), ng);
    std::vector<std::vector<Segment>> segs(ng);
    std::vector<std::vector<int32_t>> qstart(ng);
    std::vector<arlbm_server::Launch> launches(ng);
    size_t bytes = align_up(sizeof(LatticeDesc) * descs.size());
    for (int64_t k = 0; k < ng; ++k) {
        std::vector<SchedLattice> sub;
        for (size_t i = 0; i < lats.size(); ++i)
            if (grp[i] == k) sub.push_back(lats[i]);
        launches[k].nwaves = (int32_t)build_schedule(sub, batched_waves(), segs[k], qstart[k]);
        launches[k].off_start = bytes;
        launches[k].off_segs = bytes + align_up(sizeof(int32_t) * (kQueues + 1));
        bytes = launches[k].off_segs + align_up(sizeof(Segment) * segs[k].size());
    }
    hipError_t e;
    // the device table grows by reallocation, after the launches that still
    // read the old one
    if (bytes > s->cap_table) {
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, hipGetErrorString(e));
        if (s->d_table) (void)hipFree(s->d_table);
        s->d_table = nullptr;
        s->cap_table = std::max<size_t>(bytes * 2, (size_t)1 << 16);
        e = hipMalloc((void **)&s->d_table, s->cap_table);
        if (e != hipSuccess) {
            s->cap_table = 0;
            return sfail(s, ARLBM_ENOMEM, "work table allocation failed");
        }
    }
    if (!descs.empty()) {
        // the upload is ordered after the launches that read the previous
        // table; its source, a pinned copy, is rewritten two rebuilds later,
        // after its own upload has completed
        const int k = s->table_set;
        s->table_set ^= 1;
        if (!s->table_ev[k]) {
            e = hipEventCreateWithFlags(&s->table_ev[k], hipEventDisableTiming);
            if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("event: ") + hipGetErrorString(e));
        } else {
            e = hipEventSynchronize(s->table_ev[k]);
            if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("table event: ") + hipGetErrorString(e));
        }
        if (bytes > s->hcap_table[k]) {
            if (s->h_table[k]) (void)hipHostFree(s->h_table[k]);
            s->h_table[k] = nullptr;
            s->hcap_table[k] = s->cap_table;
            e = hipHostMalloc((void **)&s->h_table[k], s->hcap_table[k], hipHostMallocDefault);
            if (e != hipSuccess) {
                s->hcap_table[k] = 0;
                return sfail(s, ARLBM_ENOMEM, "pinned work table allocation failed");
            }
        }
        char *h = s->h_table[k];
        std::memcpy(h, descs.data(), sizeof(LatticeDesc) * descs.size());
        for (int64_t g = 0; g < ng; ++g) {
            std::memcpy(h + launches[g].off_start, qstart[g].data(), sizeof(int32_t) * qstart[g].size());
            if (!segs[g].empty())
                std::memcpy(h + launches[g].off_segs, segs[g].data(), sizeof(Segment) * segs[g].size());
        }
        e = hipMemcpyAsync(s->d_table, h, bytes, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->table_ev[k], s->stream);
        if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
    }
    s->launches = launches;
    s->dirty = false;
    return ARLBM_OK;
}

// Pinned staging layout of an admission: initial scalars, scalars read back
// after the initialisation, the U0 planes, the bed plane.
struct AdmitLayout {
    size_t sc_in, sc_out, u0, bed, total;
};
AdmitLayout admit_layout(const arlbm_sizes &sz, int64_t plane, bool has_bed)
{
    AdmitLayout l;
    l.sc_in = 0;
    l.sc_out = align_up(sizeof(DevScalars));
    l.u0 = l.sc_out + align_up(sizeof(DevScalars));
    l.bed = l.u0 + align_up(sizeof(double) * sz.m * plane);
    l.total = l.bed + (has_bed ? sizeof(double) * plane : 0);
    return l;
}

// A saved state (arlbm_save_state): header, the f planes, the moment planes,
// the device scalars.
namespace {
struct StateView {
    const StateHeader *hd;
    const char *f, *u, *sc;
};
StateView state_view(const char *blob)
{
    StateView v;
    v.hd = (const StateHeader *)blob;
    v.f = blob + sizeof(StateHeader);
    v.u = v.f + v.hd->f_bytes;
    v.sc = v.u + v.hd->u_bytes;
    return v;
}
}  // namespace

// Admission: a device block from the pool, the handle, the host checks of the
// initial state, then the upload and initialisation enqueued (as set_state
// does, without its wait); the wave-speed checks follow in finish_staged.  A
// resumed state is uploaded as saved (populations, moments, scalars) and
// continues from its step and time.
void admit_enqueue(arlbm_server *s, Pending &p)
{
    arlbm_sizes sz;
    fill_sizes(&p.cfg, &sz);
    const bool has_bed = p.cfg.has_bed != 0;
    const bool resume = p.blob != nullptr;
    size_t dcls = 0;
    void *blk = s->dev.acquire(sz.total_bytes, &dcls);
    if (!blk) {
        g_thread_err = "device allocation failed";
        push_failed(s, p.id, ARLBM_ENOMEM, p.submit_s);
        return;
    }
    const arlbm_buffers b = carve(blk, sz, has_bed);
    arlbm_lattice *lat = nullptr;
    int rc = arlbm_create(&p.cfg, &b, s->stream, &lat);
    if (rc == ARLBM_OK && !resume) rc = check_state(lat, p.U0.data(), has_bed ? p.bed.data() : nullptr);
    const int64_t plane = (int64_t)p.cfg.nx * p.cfg.ny * p.cfg.nz;
    const AdmitLayout L = admit_layout(sz, plane, has_bed);
    const size_t host_bytes = resume ? p.blob_bytes : L.total;
    size_t hcls = 0;
    char *host = nullptr;
    if (rc == ARLBM_OK) {
        host = (char *)s->pin.acquire(host_bytes, &hcls);
        if (!host) rc = fail(lat, ARLBM_ENOMEM, "pinned staging allocation failed");
    }
    hipEvent_t ev = nullptr;
    if (rc == ARLBM_OK) {
        hipError_t e = hipSuccess;
        if (resume) {
            par_copy(host, p.blob.get(), p.blob_bytes);
            const StateView v = state_view(host);
            const int par = (int)(p.step0 & 1);
            e = hipMemcpyAsync(lat->desc.f[par], v.f, sz.f_bytes, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lat->desc.u[par], v.u, sz.u_bytes, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lat->desc.sc, v.sc, sizeof(DevScalars), hipMemcpyHostToDevice, s->stream);
        } else {
            DevScalars init{};
            init.t[0] = 0.0;
            init.first_bad_step = ~0ull;
            std::memcpy(host + L.sc_in, &init, sizeof init);
            par_copy(host + L.u0, p.U0.data(), sizeof(double) * sz.m * plane);
            if (has_bed) par_copy(host + L.bed, p.bed.data(), sizeof(double) * plane);
            double *U0d = (double *)lat->desc.f[1];
            double *bedd = has_bed ? U0d + (size_t)sz.m * plane : nullptr;
            e = hipMemcpyAsync(U0d, host + L.u0, sizeof(double) * sz.m * plane, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess && has_bed)
                e = hipMemcpyAsync(bedd, host + L.bed, sizeof(double) * plane, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lat->desc.sc, host + L.sc_in, sizeof(DevScalars), hipMemcpyHostToDevice,
                                   s->stream);
            if (e == hipSuccess) e = L_reduce(lat, U0d, 2);
            if (e == hipSuccess) e = L_init(lat, U0d, bedd, 2);
            if (e == hipSuccess)
                e = hipMemcpyAsync(host + L.sc_out, lat->desc.sc, sizeof(DevScalars), hipMemcpyDeviceToHost,
                                   s->stream);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
        if (e != hipSuccess) {
            rc = hip_fail(lat, e, "admission upload");
            // a transfer may be in the stream: wait before the blocks return
            (void)hipStreamSynchronize(s->stream);
            if (ev) (void)hipEventDestroy(ev);
        }
    }
    if (rc != ARLBM_OK) {
        if (host) s->pin.release(host, hcls);
        if (lat) drop_handle(lat);
        s->dev.release(blk, dcls);
        push_failed(s, p.id, rc, p.submit_s);
        return;
    }
    lat->step = p.step0;
    lat->busy = true;
    const double t_admit = now_s();
    s->resident.push_back({p.id, lat, s->iter - p.step0, s->iter, s->iter + p.nsteps, p.submit_s, t_admit, p.bytes,
                           blk, dcls, p.dst});
    s->staged.push_back({resume ? Staged::ADMIT_STATE : Staged::ADMIT, p.id, lat, 0, p.submit_s, t_admit, host,
                         hcls, ev});
    s->in_use += p.bytes;
    s->dirty = true;
}

// Retirement: the moments and scalars of the lattice's state enqueued into a
// pinned block; the device block goes back to the pool at once (stream order
// keeps it intact until the read-back has run).
int retire_enqueue(arlbm_server *s, const Resident &r)
{
    arlbm_lattice *h = r.lat;
    h->step = s->iter - r.iter0;  // the batched launches advanced it
    h->busy = false;
    const int64_t steps = s->iter - r.admit_it;
    const size_t o_u = align_up(sizeof(DevScalars));
    const size_t nU = (size_t)h->sz.m * h->desc.plane;
    size_t hcls = 0;
    char *host = (char *)s->pin.acquire(o_u + sizeof(double) * nU, &hcls);
    int rc = host ? ARLBM_OK : fail(h, ARLBM_ENOMEM, "pinned staging allocation failed");
    hipEvent_t ev = nullptr;
    if (rc == ARLBM_OK) rc = form_moments(h);
    if (rc == ARLBM_OK) rc = read_planes_async(h, h->desc.u[h->step & 1], h->sz.m, (double *)(host + o_u));
    if (rc == ARLBM_OK) {
        hipError_t e = hipMemcpyAsync(host, h->desc.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
        if (e != hipSuccess) {
            rc = hip_fail(h, e, "read-back");
            if (ev) (void)hipEventDestroy(ev);
        }
    }
    if (rc != ARLBM_OK) {
        (void)hipStreamSynchronize(s->stream);
        if (host) s->pin.release(host, hcls);
        drop_handle(h);
        s->dev.release(r.dev, r.dev_cls);
        s->in_use -= r.bytes;
        push_failed(s, r.id, rc, r.submit_s);
        return rc;
    }
    s->staged.push_back({Staged::RETIRE, r.id, h, steps, r.submit_s, r.admit_s, host, hcls, ev, r.dst});
    s->dev.release(r.dev, r.dev_cls);
    s->in_use -= r.bytes;
    return ARLBM_OK;
}

// Finish what admissions and retirements enqueued before the launch: copy
// results out of their pinned blocks and check the admitted lattices'
// wave-speed bounds (Theorem 4.3's bound on eps, a nonzero sum), as
// set_state does.  An admitted lattice that fails leaves the mix with its
// error; the steps launched with it (as many as the call's launches) touched
// only its own buffers.
int finish_staged(arlbm_server *s)
{
    int first_err = ARLBM_OK;
    for (Staged &g : s->staged) {
        hipError_t e = hipEventSynchronize(g.ev);
        (void)hipEventDestroy(g.ev);
        if (e != hipSuccess && first_err == ARLBM_OK)
            first_err = sfail(s, ARLBM_EDEVICE, std::string("staged transfer: ") + hipGetErrorString(e));
        arlbm_lattice *h = g.lat;
        if (g.kind == Staged::RETIRE) {
            DevScalars sc;
            std::memcpy(&sc, g.host, sizeof sc);
            Done d{};
            d.c.id = g.id;
            d.c.steps = g.steps;
            d.c.submit_s = g.submit_s;
            d.c.admit_s = g.admit_s;
            d.c.t = sc.t[h->step % 3];
            d.c.flags = sc.flags;
            d.c.first_bad_step = sc.first_bad_step == ~0ull ? -1 : (int64_t)sc.first_bad_step;
            int rc = e != hipSuccess ? ARLBM_EDEVICE : ARLBM_OK;
            if (rc == ARLBM_OK && (sc.flags & ARLBM_FLAG_NONFINITE)) rc = ARLBM_ENONFINITE;
            if (rc == ARLBM_OK && (sc.flags & ARLBM_FLAG_DEGENERATE)) rc = ARLBM_EDEGENERATE;
            // the positivity flag is advisory: the moments are still the result
            if (rc == ARLBM_OK) {
                const double *U = (const double *)((const char *)g.host + align_up(sizeof(DevScalars)));
                const size_t nU = (size_t)h->sz.m * h->desc.plane;
                if (g.dst) {
                    // straight into the caller's array: no copy at poll
                    par_copy(g.dst, U, sizeof(double) * nU);
                    d.c.U = g.dst;
                    d.c.u_count = (int64_t)nU;
                } else if (d.U.alloc(nU)) {
                    par_copy(d.U.data(), U, sizeof(double) * nU);
                } else {
                    rc = ARLBM_ENOMEM;
                }
            }
            d.c.status = rc;
            d.c.done_s = now_s();
            s->done.push_back(std::move(d));
            drop_handle(h);
        } else if (g.kind == Staged::ADMIT) {
            arlbm_sizes sz = h->sz;
            const AdmitLayout L = admit_layout(sz, h->desc.plane, h->cfg.has_bed != 0);
            DevScalars got;
            std::memcpy(&got, (const char *)g.host + L.sc_out, sizeof got);
            const double ab0 = abar_host(got, 0, 0);
            const double ab1 = h->cfg.dim >= 2 ? abar_host(got, 0, 1) : 0.0;
            const double ab2 = h->cfg.dim == 3 ? abar_host(got, 0, 2) : 0.0;
            const double sa = (ab0 + ab1) + ab2;
            int rc = e != hipSuccess ? ARLBM_EDEVICE : ARLBM_OK;
            if (rc == ARLBM_OK && !(sa > 0.0))
                rc = fail(h, ARLBM_EDEGENERATE, "sum of wave-speed bounds is zero: time step undefined");
            const double bound = (1.0 / h->cfg.dim) * (1.0 / h->cfg.cfl - 1.0) * sa;
            if (rc == ARLBM_OK && !(h->cfg.eps < bound))
                rc = fail(h, ARLBM_EINVAL, "eps exceeds the stability bound of Theorem 4.3");
            if (rc != ARLBM_OK) {
                for (size_t i = 0; i < s->resident.size(); ++i) {
                    if (s->resident[i].lat != h) continue;
                    s->dev.release(s->resident[i].dev, s->resident[i].dev_cls);
                    s->in_use -= s->resident[i].bytes;
                    s->resident.erase(s->resident.begin() + i);
                    break;
                }
                s->dirty = true;
                push_failed(s, g.id, rc, g.submit_s);
                drop_handle(h);
            }
        }
        s->pin.release(g.host, g.host_cls);
    }
    s->staged.clear();
    return first_err;
}

// Ids of residents whose gathered flags show a non-finite or degenerate
// state, from every gather whose copy has completed (never waits).
void take_gathers(arlbm_server *s)
{
    for (auto &g : s->gather) {
        if (!g.pending || hipEventQuery(g.ev) != hipSuccess) continue;
        for (size_t i = 0; i < g.ids.size(); ++i)
            if (g.host[i] & (ARLBM_FLAG_NONFINITE | ARLBM_FLAG_DEGENERATE)) s->failing.push_back(g.ids[i]);
        g.pending = false;
    }
}

// Enqueue the gather of the residents' flag words (after the launches, with
// the table the launches read), unless both gathers are still in flight.
int gather_flags(arlbm_server *s)
{
    const size_t n = s->resident.size();
    if (n == 0) return ARLBM_OK;
    auto &g = s->gather[s->gather_next];
    if (g.pending) return ARLBM_OK;
    hipError_t e = hipSuccess;
    if (n > s->cap_flags) {
        if (s->d_flags) {
            e = hipStreamSynchronize(s->stream);
            (void)hipFree(s->d_flags);
        }
        s->d_flags = nullptr;
        s->cap_flags = std::max<size_t>(2 * n, 256);
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_flags, sizeof(unsigned) * s->cap_flags);
        if (e != hipSuccess) {
            s->cap_flags = 0;
            return sfail(s, ARLBM_ENOMEM, "flag gather allocation failed");
        }
    }
    if (n > g.cap) {
        if (g.host) (void)hipHostFree(g.host);
        g.host = nullptr;
        g.cap = s->cap_flags;
        e = hipHostMalloc((void **)&g.host, sizeof(unsigned) * g.cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            g.cap = 0;
            return sfail(s, ARLBM_ENOMEM, "pinned flag gather allocation failed");
        }
    }
    if (!g.ev) {
        e = hipEventCreateWithFlags(&g.ev, hipEventDisableTiming);
        if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("event: ") + hipGetErrorString(e));
    }
    e = gather_flags_launch((const LatticeDesc *)s->d_table, (int32_t)n, s->d_flags, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g.host, s->d_flags, sizeof(unsigned) * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipEventRecord(g.ev, s->stream);
    if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("flag gather: ") + hipGetErrorString(e));
    g.ids.clear();
    for (const Resident &r : s->resident) g.ids.push_back(r.id);
    g.pending = true;
    s->gather_next ^= 1;
    return ARLBM_OK;
}

// Queue a request after the checks common to both submit calls.
int queue_request(arlbm_server *s, Pending &&p, uint64_t *id)
{
    p.id = s->next_id++;
    p.submit_s = now_s();
    s->queue.push_back(std::move(p));
    if (id) *id = s->queue.back().id;
    return ARLBM_OK;
}

}  // namespace

extern "C" int arlbm_server_create(size_t budget, int32_t precision, void *stream, arlbm_server **out)
{
    if (!out) return sfail(nullptr, ARLBM_EINVAL, "out is NULL");
    if (precision != ARLBM_F32 && precision != ARLBM_F64) return sfail(nullptr, ARLBM_EINVAL, "bad precision");
    arlbm_server *s = new (std::nothrow) arlbm_server();
    if (!s) return sfail(nullptr, ARLBM_ENOMEM, "host memory for the server");
    s->budget = budget;
    s->precision = precision;
    s->stream = (hipStream_t)stream;
    // device blocks held for lattices (in use or free): at most the budget;
    // pinned staging blocks (in use or free): at most 4 GiB, room to keep the
    // admission and read-back blocks of large lattices for reuse (a 4096^2
    // shallow-water state takes 671 and 470 MB; with a 1 GiB cap each solve
    // gave one back and pinned the other again: 4096^2 solve 1035 ms, of
    // which 920 ms of steps)
    s->dev.cap = budget;
    s->dev.stream = s->stream;
    s->pin.stream = s->stream;
    s->pin.pinned = true;
    s->pin.cap = (size_t)4 << 30;
    const size_t cbytes = sizeof(unsigned) * 2 * kQueues * kQueueStride;
    hipError_t e = hipMalloc((void **)&s->d_counters, cbytes);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_counters, 0, cbytes, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        if (s->d_counters) (void)hipFree(s->d_counters);
        delete s;
        return sfail(nullptr, e == hipErrorOutOfMemory ? ARLBM_ENOMEM : ARLBM_EDEVICE,
                     std::string("queue counters: ") + hipGetErrorString(e));
    }
    *out = s;
    return ARLBM_OK;
}

extern "C" int arlbm_server_submit(arlbm_server *s, const arlbm_config *cfg, const double *U0, const double *bed,
                                   int64_t nsteps, uint64_t *id)
{
    if (!s || !cfg || !U0) return sfail(s, ARLBM_EINVAL, "bad argument");
    if (nsteps < 1) return sfail(s, ARLBM_EINVAL, "nsteps must be >= 1");
    arlbm_config c = *cfg;
    c.precision = s->precision;
    std::string e = check_config(&c);
    if (!e.empty()) return sfail(s, ARLBM_EINVAL, e);
    if (c.has_bed && !bed) return sfail(s, ARLBM_EINVAL, "bed is NULL");
    arlbm_sizes sz;
    fill_sizes(&c, &sz);
    Pending p;
    p.bytes = size_class(sz.total_bytes);
    if (p.bytes > s->budget) return sfail(s, ARLBM_EBUDGET, "request can never fit the HBM budget");
    p.cfg = c;
    const size_t plane = (size_t)c.nx * c.ny * c.nz;
    if (!p.U0.alloc((size_t)sz.m * plane) || (c.has_bed && !p.bed.alloc(plane)))
        return sfail(s, ARLBM_ENOMEM, "host memory for the queued state");
    par_copy(p.U0.data(), U0, sizeof(double) * p.U0.size());
    if (c.has_bed) par_copy(p.bed.data(), bed, sizeof(double) * plane);
    p.nsteps = nsteps;
    return queue_request(s, std::move(p), id);
}

extern "C" int arlbm_server_submit_state(arlbm_server *s, const arlbm_config *cfg, const void *blob, size_t bytes,
                                         int64_t nsteps, uint64_t *id)
{
    if (!s || !cfg || !blob) return sfail(s, ARLBM_EINVAL, "bad argument");
    if (nsteps < 1) return sfail(s, ARLBM_EINVAL, "nsteps must be >= 1");
    arlbm_config c = *cfg;
    c.precision = s->precision;
    std::string e = check_config(&c);
    if (!e.empty()) return sfail(s, ARLBM_EINVAL, e);
    if (c.has_bed) return sfail(s, ARLBM_EINVAL, "a lattice with a bed cannot be resumed in the server");
    arlbm_sizes sz;
    fill_sizes(&c, &sz);
    const size_t need = sizeof(StateHeader) + sz.f_bytes + sz.u_bytes + sizeof(DevScalars);
    if (bytes < need) return sfail(s, ARLBM_EINVAL, "state blob too small");
    StateHeader hd;
    std::memcpy(&hd, blob, sizeof hd);
    if (hd.magic != kMagic || hd.precision != c.precision || hd.variant != variant_of(c.system, c.dim) ||
        hd.nx != c.nx || hd.ny != c.ny || hd.nz != c.nz || hd.f_bytes != sz.f_bytes || hd.u_bytes != sz.u_bytes ||
        hd.step < 0)
        return sfail(s, ARLBM_EINVAL, "state blob does not match the configuration");
    Pending p;
    p.bytes = size_class(sz.total_bytes);
    if (p.bytes > s->budget) return sfail(s, ARLBM_EBUDGET, "request can never fit the HBM budget");
    p.cfg = c;
    p.blob.reset(new (std::nothrow) char[need]);
    if (!p.blob) return sfail(s, ARLBM_ENOMEM, "host memory for the queued state");
    par_copy(p.blob.get(), blob, need);
    p.blob_bytes = need;
    p.step0 = hd.step;
    p.nsteps = nsteps;
    return queue_request(s, std::move(p), id);
}

extern "C" int arlbm_server_result_into(arlbm_server *s, uint64_t id, double *dst, int64_t count)
{
    if (!s || !dst) return sfail(s, ARLBM_EINVAL, "bad argument");
    for (Pending &p : s->queue) {
        if (p.id != id) continue;
        const int64_t need = (int64_t)num_fields(p.cfg.system, p.cfg.dim) * p.cfg.nx * p.cfg.ny * p.cfg.nz;
        if (count != need) return sfail(s, ARLBM_EINVAL, "count is not the size of the request's result");
        p.dst = dst;
        return ARLBM_OK;
    }
    return sfail(s, ARLBM_EINVAL, "no queued request has this id");
}

extern "C" int arlbm_server_iterate(arlbm_server *s, int32_t *n_res, int32_t *n_queued)
{
    return arlbm_server_iterate_n(s, 1, n_res, n_queued, nullptr);
}

extern "C" int arlbm_server_iterate_n(arlbm_server *s, int32_t max_launches, int32_t *n_res, int32_t *n_queued,
                                      int32_t *n_launched)
{
    if (!s) return sfail(nullptr, ARLBM_EINVAL, "server is NULL");
    if (max_launches < 1) return sfail(s, ARLBM_EINVAL, "max_launches must be >= 1");
    if (n_launched) *n_launched = 0;
    take_gathers(s);
    // retire lattices whose steps are complete, or whose state became
    // non-finite or degenerate (read-backs enqueued)
    for (size_t i = 0; i < s->resident.size();) {
        const Resident r = s->resident[i];
        const bool failing = std::find(s->failing.begin(), s->failing.end(), r.id) != s->failing.end();
        if (s->iter >= r.end_it || failing) {
            s->resident.erase(s->resident.begin() + i);
            s->dirty = true;
            (void)retire_enqueue(s, r);  // a failure is reported in its completion
        } else {
            ++i;
        }
    }
    s->failing.clear();
    // admit queued requests in arrival order while the budget allows
    while (!s->queue.empty() && s->in_use + s->queue.front().bytes <= s->budget) {
        Pending p = std::move(s->queue.front());
        s->queue.pop_front();
        admit_enqueue(s, p);
    }
    if (s->dirty) {
        int rc = rebuild_table(s);
        if (rc) return rc;
    }
    // launches this call: as many as asked, but no resident lattice past its
    // step count, so retirements fall on the same iteration as one launch
    // per call would give (every resident has a step left: finished lattices
    // retired above, and a request asks for at least one step)
    int64_t nl = s->resident.empty() ? 0 : max_launches;
    for (const Resident &r : s->resident) nl = std::min<int64_t>(nl, r.end_it - s->iter);
    for (int64_t l = 0; l < nl; ++l) {
        hipError_t e = hipSuccess;
        for (const arlbm_server::Launch &g : s->launches) {
            if (g.nwaves <= 0) continue;
            const LatticeDesc *dd = (const LatticeDesc *)s->d_table;
            const int32_t *dq = (const int32_t *)(s->d_table + g.off_start);
            const Segment *dg = (const Segment *)(s->d_table + g.off_segs);
            const int32_t par = (int32_t)(s->batched_launches & 1);
            e = s->precision == ARLBM_F64
                    ? f64::step_batched(dd, dg, dq, s->d_counters, par, g.nwaves, s->iter, s->stream)
                    : f32::step_batched(dd, dg, dq, s->d_counters, par, g.nwaves, s->iter, s->stream);
            ++s->batched_launches;
            if (e != hipSuccess) break;
        }
        if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("batched launch: ") + hipGetErrorString(e));
        // lattices outside the batched kernel (3D; 2D beyond 4 GiB of
        // populations) run their own step after it, on the same stream
        for (const Resident &r : s->resident) {
            if (!own_launch(r.lat->desc)) continue;
            LatticeDesc d = r.lat->desc;
            d.iter0 = r.iter0;
            e = s->precision == ARLBM_F64 ? f64::step_single(d, s->iter, s->stream)
                                          : f32::step_single(d, s->iter, s->stream);
            if (e != hipSuccess) return sfail(s, ARLBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
        }
        ++s->iter;
        if (n_launched) ++*n_launched;
    }
    if (nl > 0) {
        int rc = gather_flags(s);
        if (rc) return rc;
    }
    // result copies and admission checks, while the launch runs
    int rc = finish_staged(s);
    if (rc) return rc;
    if (n_res) *n_res = (int32_t)s->resident.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return ARLBM_OK;
}

extern "C" int arlbm_server_poll(arlbm_server *s, arlbm_completion *out, int32_t max, int32_t *n)
{
    if (!s || !n || (max > 0 && !out)) return sfail(s, ARLBM_EINVAL, "bad argument");
    s->handed.clear();
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        s->handed.push_back(std::move(s->done.front()));
        s->done.pop_front();
        ++k;
    }
    for (int32_t i = 0; i < k; ++i) {
        Done &d = s->handed[i];
        out[i] = d.c;
        if (d.c.status != ARLBM_OK) {
            out[i].U = nullptr;
            out[i].u_count = 0;
        } else if (!d.c.U) {  // a result in the server's own memory
            out[i].U = d.U.data();
            out[i].u_count = (int64_t)d.U.size();
        }
    }
    *n = k;
    return ARLBM_OK;
}

extern "C" int arlbm_server_memory(arlbm_server *s, size_t *bytes)
{
    if (!s || !bytes) return sfail(s, ARLBM_EINVAL, "bad argument");
    *bytes = s->in_use;
    return ARLBM_OK;
}

extern "C" int arlbm_server_pool_bytes(arlbm_server *s, size_t *bytes)
{
    if (!s || !bytes) return sfail(s, ARLBM_EINVAL, "bad argument");
    *bytes = s->dev.used_bytes + s->dev.free_bytes;
    return ARLBM_OK;
}

extern "C" int arlbm_server_destroy(arlbm_server *s)
{
    if (!s) return ARLBM_OK;
    (void)hipStreamSynchronize(s->stream);
    (void)finish_staged(s);
    for (auto &r : s->resident) {
        drop_handle(r.lat);
        s->dev.release(r.dev, r.dev_cls);
    }
    s->dev.clear();
    s->pin.clear();
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->d_flags) (void)hipFree(s->d_flags);
    if (s->d_counters) (void)hipFree(s->d_counters);
    for (int k = 0; k < 2; ++k) {
        if (s->h_table[k]) (void)hipHostFree(s->h_table[k]);
        if (s->table_ev[k]) (void)hipEventDestroy(s->table_ev[k]);
        if (s->gather[k].host) (void)hipHostFree(s->gather[k].host);
        if (s->gather[k].ev) (void)hipEventDestroy(s->gather[k].ev);
    }
    delete s;
    return ARLBM_OK;
}

// Schedule entries of the 1D and 2D lattices among configurations
// cfgs[0..n-1] (lattice index = configuration index); "" or the first
// configuration error.
std::string plan_lattices(const arlbm_config *cfgs, int32_t n, std::vector<SchedLattice> &lats)
{
    for (int32_t i = 0; i < n; ++i) {
        std::string e = check_config(&cfgs[i]);
        if (!e.empty()) return e;
        if (cfgs[i].dim == 3) continue;
        LatticeDesc d{};
        d.variant = variant_of(cfgs[i].system, cfgs[i].dim);
        d.cpl = columns_per_lane(&cfgs[i]);
        d.ncols = (int32_t)((cfgs[i].nx + strip_out_w(d.cpl) - 1) / strip_out_w(d.cpl));
        d.ny = (int32_t)cfgs[i].ny;
        lats.push_back(sched_lattice(i, d));
    }
    return "";
}

extern "C" int arlbm_plan_groups(const arlbm_config *cfgs, int32_t n, int32_t waves, int32_t *group_of,
                                 int32_t *ngroups)
{
    if (!cfgs || n < 0 || waves < 1 || !ngroups || (n > 0 && !group_of))
        return sfail(nullptr, ARLBM_EINVAL, "bad argument");
    std::vector<SchedLattice> lats;
    std::string e = plan_lattices(cfgs, n, lats);
    if (!e.empty()) return sfail(nullptr, ARLBM_EINVAL, e);
    int64_t ng = 1;
    const std::vector<int32_t> grp = lats.empty() ? std::vector<int32_t>() : launch_groups(lats, waves, ng);
    for (int32_t i = 0; i < n; ++i) group_of[i] = -1;
    for (size_t k = 0; k < lats.size(); ++k) group_of[lats[k].lattice] = grp[k];
    *ngroups = lats.empty() ? 0 : (int32_t)ng;
    return ARLBM_OK;
}

extern "C" int arlbm_plan_schedule(const arlbm_config *cfgs, int32_t n, int32_t waves, int32_t *queue_start,
                                   int32_t *segs, int32_t max_segs, int32_t *nsegs, int32_t *nwaves)
{
    if (!cfgs || n < 0 || waves < 1 || !nsegs || !nwaves || !queue_start)
        return sfail(nullptr, ARLBM_EINVAL, "bad argument");
    std::vector<SchedLattice> lats;
    std::string e = plan_lattices(cfgs, n, lats);
    if (!e.empty()) return sfail(nullptr, ARLBM_EINVAL, e);
    std::vector<Segment> sg;
    std::vector<int32_t> qs(kQueues + 1, 0);
    const int64_t nw = lats.empty() ? 0 : build_schedule(lats, waves, sg, qs);
    *nwaves = (int32_t)nw;
    *nsegs = (int32_t)sg.size();
    for (int q = 0; q <= kQueues; ++q) queue_start[q] = qs[q];
    if ((int64_t)sg.size() > max_segs || (!sg.empty() && !segs))
        return sfail(nullptr, ARLBM_EINVAL, "output array too small");
    for (size_t k = 0; k < sg.size(); ++k) {
        segs[4 * k + 0] = sg[k].lattice;
        segs[4 * k + 1] = sg[k].col;
        segs[4 * k + 2] = sg[k].y0;
        segs[4 * k + 3] = sg[k].y1;
    }
    return ARLBM_OK;
}
