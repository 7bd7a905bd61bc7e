// Fused collide-and-stream step of the adaptive-relaxation LBM on gfx950.
//
// Work decomposition.  One wave64 owns a strip of output columns and a band
// of rows.  With one column per lane, lane l sits on column x = x0 - 3 + l
// (58 outputs); with two, on columns x0 - 4 + 2l and the next (120 outputs).
// The halo on each side is carried by the wave itself: x-neighbours come
// from lane shuffles and no barriers are used.  The wave marches up its band;
// per row it loads the populations f (Q m planes), forms the moments U of the
// row two ahead from them, and keeps a rolling window in registers:
//
//   U rows j-2, j-1, j           -> nu at row j-1            (eqs. 2.13-2.14)
//   nu rows j-3, j-2, j-1 (+x+-1) -> nu~, omega at row j-2   (eqs. 2.15-2.16)
//   f, U, omega at row r = j-2   -> collided f*_k (source node, eq. 2.2)
//   f*_{+y}(r-2), f*_{0,+x,-x}(r-1), f*_{-y}(r) -> pulled F_k at row r-1
//   sum_k F_k, (2.8), second half source -> f^{n+1}, U^{n+1} written once.
//
// Every population is written once per step and read from HBM once: the
// loaded rows wait for the collision two rows later in a register ring
// (FP32) or in two LDS slots of the wave (FP64); the step stores nothing but
// the populations.  The grid-wide
// wave-speed bound of the next step (eq. 2.19) is reduced in registers, across
// the wave by shuffles, and committed with one 64-bit atomic max per wave and
// direction into a triple-buffered slot.  The kernel launch boundary is the
// grid barrier that the global maximum needs.
//
// Plane layout: plane c of a buffer starts at c * pstride, pstride = nx ny
// rounded up to 64 elements plus a pad that keeps the planes of a
// power-of-two lattice from all starting at the same offset of the memory
// interleave.  Lanes that must not write (halo lanes, warm-up
// rows) are masked off and make no memory request.  (Storing them to shared
// slots in a tail of every plane instead kept the row loop free of branches,
// but every wave on every XCD then wrote the same few lines, which cost more
// than the branch: 0.169 -> 0.166 ms per 2048^2 Euler step without it.)
//
// Ghost cells: U at ghost positions follows the boundary index map (periodic
// wrap, or mirror U(-1-i) = U(i) with the normal momentum negated at
// reflective walls); populations pulled from a mirror ghost are the
// destination's own collided populations (transmissive: same direction;
// reflective: the mirrored direction with the normal momentum negated).
#pragma once

#include "arlbm_internal.h"
#include "physics.hpp"

namespace arlbm {

// ---------------------------------------------------------------- helpers --

// Value held by lane l-1 (x - 1) / lane l+1 (x + 1), by one DPP wavefront
// shift (wave_shr:1 / wave_shl:1); the edge lane keeps its own value (edge
// lanes only produce halo values that are never used).
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v) { return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false); }
template <int CTRL, typename T>
__device__ __forceinline__ T wave_shift(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_shift<CTRL>(__builtin_bit_cast(int, v)));
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)dpp_shift<CTRL>((int)(unsigned)b);
        const unsigned hi = (unsigned)dpp_shift<CTRL>((int)(unsigned)(b >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}
template <typename T>
__device__ __forceinline__ T from_left(T v) { return wave_shift<0x138>(v); }   // wave_shr:1
template <typename T>
__device__ __forceinline__ T from_right(T v) { return wave_shift<0x130>(v); }  // wave_shl:1

// Compile-time phase of an unrolled loop.
template <int N>
struct Phase {
    static constexpr int value = N;
};

// Loads and stores of one plane at a 32-bit per-lane element offset from the
// plane's (uniform) base pointer.
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned elem_off)
{
    return base[elem_off];
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned elem_off, T v)
{
    base[elem_off] = v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

// Relaxation parameter from the summed indicator (2.12/2.16): 1 + 1/(1 + nt).
// FP32 takes the hardware reciprocal (1 ulp), FP64 the IEEE quotient.
template <typename T>
__device__ __forceinline__ T omega_of(T nt)
{
    if constexpr (sizeof(T) == 4)
        return T(1) + __builtin_amdgcn_rcpf(T(1) + nt);
    else
        return T(1) + T(1) / (T(1) + nt);
}

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// Boundary index map for a coordinate in [-reach, n-1+reach] (clamped first:
// lanes further out only carry unused halo values; n >= 4 >= reach keeps the
// image inside the lattice).  refl is set for a reflective wall on the side
// the index fell off.
__device__ __forceinline__ int bc_map(int i, int n, int lo, int hi, bool &refl, int reach = kHalo)
{
    refl = false;
    i = i < -reach ? -reach : (i > n - 1 + reach ? n - 1 + reach : i);
    if (i < 0) {
        if (lo == 0) return i + n;
        refl = lo == 2;
        return -1 - i;
    }
    if (i >= n) {
        if (hi == 0) return i - n;
        refl = hi == 2;
        return 2 * n - 1 - i;
    }
    return i;
}

// Per-step coefficients of the Lax-Friedrichs-type equilibrium, computed in
// FP64 from the wave-speed bounds of U^n (eqs. 2.19-2.21):
//   dt = CFL dx / sum_j abar_j, lambda = dx / dt, alpha_j = abar_j + eps,
//   a_0 = 1 - sum_j alpha_j / lambda, a_{+-j} = alpha_j / (2 lambda),
//   b_{+j} = 1 / (2 lambda), b_{-j} = -1 / (2 lambda)   (general form 2.5).
template <typename T>
struct Coefs {
    T a0, ap[3], bp, bm, hdt, omega_fixed;
    double dt;
};

// Mask of the copy index: abar_n - 1, kept inside the slot's kAbarCopies
// copies whatever the descriptor holds.
__device__ __forceinline__ int abar_mask(const LatticeDesc &L)
{
    return (L.abar_n - 1) & (kAbarCopies - 1);
}
// Wave-speed bound of direction dir in a slot: the max over the lattice's
// L.abar_n copies, lane l reading copy l mod abar_n.  Every lane of the wave
// takes part; the result is the same in all lanes (made uniform).
__device__ __forceinline__ double abar_of(const LatticeDesc &L, int slot, int dir)
{
    static_assert(kAbarCopies == kWave, "one copy per lane");
    double v = bitsd(L.sc->abar[slot][threadIdx.x & abar_mask(L)].v[dir]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    const unsigned long long b = dbits(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return bitsd(((unsigned long long)hi << 32) | lo);
}
// Copy of a slot this wave maxes into.
__device__ __forceinline__ int abar_copy(const LatticeDesc &L)
{
    return (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & abar_mask(L));
}

template <int D, typename T>
__device__ __forceinline__ bool step_coefs(const LatticeDesc &L, int64_t n, Coefs<T> &cf)
{
    const DevScalars *sc = L.sc;
    const int slot = (int)(n % 3);
    const double ab0 = abar_of(L, slot, 0);
    const double ab1 = D >= 2 ? abar_of(L, slot, 1) : 0.0;
    const double ab2 = D == 3 ? abar_of(L, slot, 2) : 0.0;
    const double sa = D == 3 ? (ab0 + ab1) + ab2 : (D == 2 ? ab0 + ab1 : ab0);
    if (!(sa > 0.0) || !(sa < 1.0e300)) return false;
    const double dt = L.cfl * L.dx / sa;
    const double lam = L.dx / dt;
    const double al0 = ab0 + L.eps, al1 = ab1 + L.eps, al2 = ab2 + L.eps;
    const double sum_alpha = D == 3 ? (al0 + al1) + al2 : (D == 2 ? al0 + al1 : al0);
    cf.a0 = T(1.0 - sum_alpha / lam);
    cf.ap[0] = T(al0 / (2.0 * lam));
    cf.ap[1] = T(al1 / (2.0 * lam));
    cf.ap[2] = T(al2 / (2.0 * lam));
    cf.bp = T(1.0 / (2.0 * lam));
    cf.bm = T(-1.0 / (2.0 * lam));
    cf.hdt = T(0.5 * dt);
    cf.omega_fixed = T(L.omega_fixed);
    cf.dt = dt;
    return true;
}

template <typename T>
__device__ __forceinline__ Phys<T> make_phys(const LatticeDesc &L)
{
    Phys<T> P;
    P.gamma = T(L.gamma);
    P.gm1 = T(L.gamma - 1.0);
    P.g = T(L.g);
    P.half_g = T(0.5 * L.g);
    P.adv[0] = T(L.adv[0]);
    P.adv[1] = T(L.adv[1]);
    P.adv[2] = T(L.adv[2]);
    P.dx = T(L.dx);
    P.p_floor_t = T(L.p_floor);
    P.rho_floor_t = T(L.rho_floor);
    P.h_dry_t = T(L.h_dry);
    P.qh = T(L.q_heat);
    P.kr = T(L.k_rate);
    P.ti = T(L.t_act);
    P.h_dry = L.h_dry;
    P.rho_floor = L.rho_floor;
    P.p_floor = L.p_floor;
    return P;
}

// Work of the lattice's first wave in a launch (all its lanes): advance t,
// record dt, clear the slot that the next step will max into (lane l clears
// copy l).
__device__ __forceinline__ void scalar_update(const LatticeDesc &L, int64_t n, double dt)
{
    DevScalars *sc = L.sc;
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0) {
        sc->t[(n + 1) % 3] = sc->t[n % 3] + dt;
        sc->last_dt = dt;
    }
    if (lane <= abar_mask(L)) {
        AbarCopy &c = sc->abar[(n + 2) % 3][lane];
        c.v[0] = 0ull;
        c.v[1] = 0ull;
        c.v[2] = 0ull;
    }
}

// A launch whose state time has reached the stop time leaves the state
// unchanged: populations are copied to the output buffer (the ping-pong
// stays consistent), t and the wave-speed bounds carry over to the next slot.
__device__ __forceinline__ bool stopped(const LatticeDesc &L, int64_t n)
{
    return L.sc->t[n % 3] >= L.t_stop;
}
// (all lanes of the lattice's first wave; lane l carries and clears copy l)
__device__ __forceinline__ void null_scalars(const LatticeDesc &L, int64_t n)
{
    DevScalars *sc = L.sc;
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0) {
        sc->t[(n + 1) % 3] = sc->t[n % 3];
        sc->null_launches = sc->null_launches + 1ull;
    }
    if (lane <= abar_mask(L)) {
        const AbarCopy &from = sc->abar[n % 3][lane];
        AbarCopy &to = sc->abar[(n + 1) % 3][lane];
        AbarCopy &clr = sc->abar[(n + 2) % 3][lane];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            to.v[d] = from.v[d];
            clr.v[d] = 0ull;
        }
    }
}
template <typename T>
__device__ __forceinline__ void null_copy(const LatticeDesc &L, int64_t n, int planes, int x, bool xout, int ya,
                                          int yb, bool first)
{
    const T *fin = (const T *)L.f[n & 1];
    T *fout = (T *)L.f[(n + 1) & 1];
    if (xout)
        for (int y = ya; y < yb; ++y)
            for (int p = 0; p < planes; ++p) {
                const unsigned o = (unsigned)(y * L.nx + x);
                sto(fout + (size_t)p * L.pstride, o, ldo(fin + (size_t)p * L.pstride, o));
            }
    if (first) null_scalars(L, n);
}

__device__ __forceinline__ void flag_degenerate(const LatticeDesc &L, int64_t n)
{
    atomicOr(&L.sc->flags, 4u);
    atomicMin(&L.sc->first_bad_step, (unsigned long long)n - L.sc->null_launches);
}

// Commit the wave's bounds and flags for the next step.
template <typename T>
__device__ __forceinline__ void commit(const LatticeDesc &L, int64_t n, T s0, T s1, unsigned flags, int dims,
                                       T s2 = T(0))
{
    const double m0 = (double)wave_max<T>(s0);
    const double m1 = dims >= 2 ? (double)wave_max<T>(s1) : 0.0;
    const double m2 = dims == 3 ? (double)wave_max<T>(s2) : 0.0;
    const unsigned long long anyf = __ballot(flags != 0u);
    unsigned fl = flags;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) fl |= __shfl_xor(fl, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        AbarCopy &c = L.sc->abar[(n + 1) % 3][abar_copy(L)];
        atomicMax(&c.v[0], dbits(m0));
        if (dims >= 2) atomicMax(&c.v[1], dbits(m1));
        if (dims == 3) atomicMax(&c.v[2], dbits(m2));
        if (anyf) {
            atomicOr(&L.sc->flags, fl);
            atomicMin(&L.sc->first_bad_step, (unsigned long long)n - L.sc->null_launches);
        }
    }
}

template <typename T>
__device__ __forceinline__ bool finite_val(T v) { return __builtin_isfinite(v); }

// ------------------------------------------------------------------ 1D ----

// A 1D segment: strips c0 .. c1-1 of 58 output cells each, one after the
// other in one wave.  The step's coefficients are formed once, the next
// strip's populations are requested before the current one is collided, and
// the wave commits its bounds once for the whole segment.
template <int SYS, typename T>
__device__ __forceinline__ void seg1d(const LatticeDesc &L, int64_t iter, int c0, int c1)
{
    constexpr int D = 1, M = SysInfo<SYS, 1>::M, Q = 3;
    const int64_t n = iter - L.iter0;
    const bool first = c0 == 0;
    Coefs<T> cf;
    if (!step_coefs<D, T>(L, n, cf)) {
        if (first && (threadIdx.x & 63) == 0) flag_degenerate(L, n);
        return;
    }
    const Phys<T> P = make_phys<T>(L);
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = L.nx;
    const int64_t plane = L.pstride;
    if (stopped(L, n)) {
        for (int col = c0; col < c1; ++col) {
            const int xs = col * kOutW - kHalo + lane;
            null_copy<T>(L, n, Q * M, xs, lane >= kHalo && lane < kWave - kHalo && xs < nx, 0, 1,
                         first && col == c0);
        }
        return;
    }
    const T *fin = (const T *)L.f[n & 1];
    T *fout = (T *)L.f[(n + 1) & 1];
    constexpr bool src = SYS == 2;
    const bool has_bed = src && L.bed != nullptr;
    // populations (with the ghost map) of strip col
    auto load = [&](int col, T (&f)[Q][M], T &b) {
        bool r;
        const unsigned xo = (unsigned)bc_map(col * kOutW - kHalo + lane, nx, L.bc[0], L.bc[1], r);
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int c = 0; c < M; ++c) f[k][c] = ldo(fin + (size_t)(k * M + c) * plane, xo);
        if (has_bed) b = ((const T *)L.bed)[xo];
    };
    T s0 = T(0);
    unsigned flags = 0;
    T f[Q][M], b = T(0);
    load(c0, f, b);
    for (int col = c0; col < c1; ++col) {
        T fnx[Q][M], bnx = T(0);
        const bool more = col + 1 < c1;
        if (more) load(col + 1, fnx, bnx);
        const int x = col * kOutW - kHalo + lane;
        bool rx;
        (void)bc_map(x, nx, L.bc[0], L.bc[1], rx);
        const bool out = lane >= kHalo && lane < kWave - kHalo && x < nx;

        // moments (with ghost map) and neighbours
        T U[M], UL[M], UR[M];
#pragma unroll
        for (int c = 0; c < M; ++c) U[c] = f[0][c] + f[1][c] + f[2][c];  // (2.3), velocity order
        if constexpr (SYS != 0)
            if (rx) U[1] = -U[1];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            UL[c] = from_left(U[c]);
            UR[c] = from_right(U[c]);
        }
        Prim<T> q;
        primitives<SYS, D, T>(U, P, q);
        // indicator nu (2.9)-(2.10), 3-point sum (2.11), omega (2.12)
        T nu = T(0);
        add_theta<SYS, D, T>(0, q, U, UL, UR, P, nu);
        const T nuL = from_left(nu), nuR = from_right(nu);
        const T nt = nuL + nu + nuR;
        const T w = L.omega_fixed_on ? cf.omega_fixed : omega_of<T>(nt);
        if (L.omega_on && out) ((T *)L.omega)[x] = w;

        // bed slope by central differences
        T db = T(0);
        if constexpr (src)
            if (has_bed) db = ddiv<T>(from_right(b) - from_left(b), T(2) * P.dx);

        // equilibrium (2.18) and collision at this source node
        T F[M];
        flux<SYS, D, T>(0, U, q, P, F);
        T fs[Q][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const T u = U[c];
            const T feq0 = cf.a0 * u;
            const T feq1 = cf.ap[0] * u + cf.bp * F[c];
            const T feq2 = cf.ap[0] * u + cf.bm * F[c];
            const T f0 = f[0][c], f1 = f[1][c], f2 = f[2][c];
            fs[0][c] = f0 - w * (f0 - feq0);
            fs[1][c] = f1 - w * (f1 - feq1);
            fs[2][c] = f2 - w * (f2 - feq2);
        }
        if constexpr (src) {
            if (has_bed) {
                const T S1 = -P.g * U[0] * db;
                fs[0][1] = fs[0][1] + cf.hdt * (cf.a0 * S1);
                fs[1][1] = fs[1][1] + cf.hdt * (cf.ap[0] * S1);
                fs[2][1] = fs[2][1] + cf.hdt * (cf.ap[0] * S1);
            }
        }
        if constexpr (SYS == 3) {  // Arrhenius sink of rho Y, first half (2.6)
            const T SY = -arrhenius_rate<T>(P, U[0], reactive_eint<D, T>(U), U[M - 1], nullptr);
            fs[0][M - 1] = fs[0][M - 1] + cf.hdt * (cf.a0 * SY);
            fs[1][M - 1] = fs[1][M - 1] + cf.hdt * (cf.ap[0] * SY);
            fs[2][M - 1] = fs[2][M - 1] + cf.hdt * (cf.ap[0] * SY);
        }
        // pull streaming: F_+(x) = f*_+(x-1), F_-(x) = f*_-(x+1)
        T Fp[M], Fm[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Fp[c] = from_left(fs[1][c]);
            Fm[c] = from_right(fs[2][c]);
        }
        if (x == 0 && L.bc[0] != 0) {
#pragma unroll
            for (int c = 0; c < M; ++c) Fp[c] = L.bc[0] == 1 ? fs[1][c] : (c == 1 ? -fs[2][c] : fs[2][c]);
        }
        if (x == nx - 1 && L.bc[1] != 0) {
#pragma unroll
            for (int c = 0; c < M; ++c) Fm[c] = L.bc[1] == 1 ? fs[2][c] : (c == 1 ? -fs[1][c] : fs[1][c]);
        }
        // moments (2.8) and second half source
        T fn[Q][M], Un[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            fn[0][c] = fs[0][c];
            fn[1][c] = Fp[c];
            fn[2][c] = Fm[c];
        }
        if constexpr (src) {
            if (has_bed) {
                const T h = fs[0][0] + Fp[0] + Fm[0];
                const T S1 = -P.g * h * db;
                fn[0][1] = fn[0][1] + cf.hdt * (cf.a0 * S1);
                fn[1][1] = fn[1][1] + cf.hdt * (cf.ap[0] * S1);
                fn[2][1] = fn[2][1] + cf.hdt * (cf.ap[0] * S1);
            }
        }
        if constexpr (SYS == 3) {  // (2.8) for rho Y, then the second half source
            T sumF[M];
#pragma unroll
            for (int c = 0; c < M; ++c) sumF[c] = fs[0][c] + Fp[c] + Fm[c];
            const T eint = reactive_eint<D, T>(sumF);
            const T z = reactive_solve<T>(P, sumF[0], eint, sumF[M - 1], cf.hdt);
            const T SY = -arrhenius_rate<T>(P, sumF[0], eint, z, nullptr);
            fn[0][M - 1] = fn[0][M - 1] + cf.hdt * (cf.a0 * SY);
            fn[1][M - 1] = fn[1][M - 1] + cf.hdt * (cf.ap[0] * SY);
            fn[2][M - 1] = fn[2][M - 1] + cf.hdt * (cf.ap[0] * SY);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) Un[c] = fn[0][c] + fn[1][c] + fn[2][c];
        if (out) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
#pragma unroll
                for (int c = 0; c < M; ++c) sto(fout + (size_t)(k * M + c) * plane, (unsigned)x, fn[k][c]);
#pragma unroll
            for (int c = 0; c < M; ++c)
                if (!finite_val<T>(Un[c])) flags |= 1u;
            Prim<T> qn;
            primitives<SYS, D, T>(Un, P, qn);
            flags |= qn.flags;
            const T sp = max_speed<SYS, T>(0, qn, P);
            if (finite_val<T>(sp) && sp > s0) s0 = sp;
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
#pragma unroll
                for (int c = 0; c < M; ++c) f[k][c] = fnx[k][c];
            b = bnx;
        }
    }
    if (first) scalar_update(L, n, cf.dt);
    commit<T>(L, n, s0, T(0), flags, 1);
}

// Several steps of a small 1D lattice in one launch: one workgroup, one wave
// per strip (at most 16 strips), a barrier between steps.  Before it every
// wave waits for its stores and wave-speed atomics to complete.  The
// barrier's workgroup-scope fences then make them visible to the other waves:
// the waves of one workgroup run on one CU and share its L1, which the CU
// keeps coherent with its own stores and atomics, so the next step reads the
// populations, times and slots the step wrote without dropping any cache
// lines.  A step then costs no launch: a 256-cell advection solve of 512
// steps took 2.23 ms in one launch per step, 1.52 ms here with an acquire at
// device scope after the barrier (which invalidates the L1), 1.33 ms without;
// 900 cells of Euler over 1500 steps 9.07 -> 6.73 ms.  With several strips
// per wave the strips follow one another: 4096 cells (71 strips on 16 waves)
// took 25 ms against 9.8 ms, so larger lattices keep one launch per step.
template <int SYS, typename T>
__global__ __launch_bounds__(1024) void k_steps1d(LatticeDesc L, int64_t iter0, int32_t nsteps)
{
    const int nw = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
    const int c0 = (int)((int64_t)w * L.ncols / nw), c1 = (int)((int64_t)(w + 1) * L.ncols / nw);
    for (int s = 0; s < nsteps; ++s) {
        if (c0 < c1) seg1d<SYS, T>(L, iter0 + s, c0, c1);
        __builtin_amdgcn_s_waitcnt(0);  // vmcnt, expcnt and lgkmcnt all zero
        __syncthreads();
    }
}

// ------------------------------------------------------------------ 2D ----

// Loads and stores of a lane's V adjacent columns as one V-element access
// (the first column is V-aligned).
template <int V, typename T>
__device__ __forceinline__ void ldv(const T *base, unsigned off, T (&out)[V])
{
    if constexpr (V == 1) {
        out[0] = base[off];
    } else {
        typedef T vec_t __attribute__((ext_vector_type(V)));
        const vec_t v = *(const vec_t *)(base + off);
#pragma unroll
        for (int i = 0; i < V; ++i) out[i] = v[i];
    }
}
template <int V, typename T>
__device__ __forceinline__ void stv(T *base, unsigned off, const T (&in)[V])
{
    if constexpr (V == 1) {
        base[off] = in[0];
    } else {
        typedef T vec_t __attribute__((ext_vector_type(V)));
        vec_t v;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = in[i];
        *(vec_t *)(base + off) = v;
    }
}

// Population planes of the 2D step, read from f^n and written to f^{n+1}.
// BUF = false: 64-bit plane pointers.  BUF = true: one buffer resource per
// buffer, the plane as a scalar byte offset and the cell as a 32-bit vector
// byte offset, so a plane access costs no vector address arithmetic; used
// when the whole population buffer spans less than 4 GiB.
template <typename T, int V, bool BUF>
struct PlaneIO;

template <typename T, int V>
struct PlaneIO<T, V, false> {
    const T *in;
    T *out;
    int64_t ps;
    __device__ __forceinline__ PlaneIO(const LatticeDesc &L, int64_t n)
        : in((const T *)L.f[n & 1]), out((T *)L.f[(n + 1) & 1]), ps(L.pstride) {}
    __device__ __forceinline__ void ld(int p, unsigned e, T (&o)[V]) const { ldv<V>(in + (size_t)p * ps, e, o); }
    __device__ __forceinline__ void st(int p, unsigned e, const T (&v)[V]) const { stv<V>(out + (size_t)p * ps, e, v); }
};

template <typename T, int V>
struct PlaneIO<T, V, true> {
    // a lane's V values as one vector; loads and stores move it whole (the
    // returned word vector is bit-cast as a unit, never indexed)
    typedef T vec_t __attribute__((ext_vector_type(V == 1 ? 2 : V)));
    static constexpr int kBytes = (int)sizeof(T) * V;
    __amdgpu_buffer_rsrc_t rin, rout;
    unsigned psb;  // plane stride in bytes
    __device__ __forceinline__ PlaneIO(const LatticeDesc &L, int64_t n)
        // raw buffers (stride 0): the range check covers the vector offset
        // only, so num_records = 2^32 - 1 never clips; the descriptor's third
        // word is the gfx9 untyped 32-bit format
        : rin(__builtin_amdgcn_make_buffer_rsrc(L.f[n & 1], 0, -1, 0x00020000)),
          rout(__builtin_amdgcn_make_buffer_rsrc(L.f[(n + 1) & 1], 0, -1, 0x00020000)),
          psb((unsigned)(L.pstride * (int64_t)sizeof(T))) {}
    __device__ __forceinline__ void ld(int p, unsigned e, T (&o)[V]) const
    {
        const int vo = (int)(e * (unsigned)sizeof(T)), so = (int)((unsigned)p * psb);
        if constexpr (kBytes == 4) {
            o[0] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rin, vo, so, 0));
        } else if constexpr (V == 1) {
            o[0] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rin, vo, so, 0));
        } else if constexpr (kBytes == 8) {
            const vec_t v = __builtin_bit_cast(vec_t, __builtin_amdgcn_raw_buffer_load_b64(rin, vo, so, 0));
            o[0] = v[0];
            o[1] = v[1];
        } else {
            const vec_t v = __builtin_bit_cast(vec_t, __builtin_amdgcn_raw_buffer_load_b128(rin, vo, so, 0));
            o[0] = v[0];
            o[1] = v[1];
        }
    }
    __device__ __forceinline__ void st(int p, unsigned e, const T (&v)[V]) const
    {
        const int vo = (int)(e * (unsigned)sizeof(T)), so = (int)((unsigned)p * psb);
        typedef unsigned w2_t __attribute__((__vector_size__(2 * sizeof(unsigned))));
        typedef unsigned w4_t __attribute__((__vector_size__(4 * sizeof(unsigned))));
        if constexpr (kBytes == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[0]), rout, vo, so, 0);
        } else if constexpr (V == 1) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(w2_t, v[0]), rout, vo, so, 0);
        } else {
            vec_t t;
            t[0] = v[0];
            t[1] = v[1];
            if constexpr (kBytes == 8)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(w2_t, t), rout, vo, so, 0);
            else
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(w4_t, t), rout, vo, so, 0);
        }
    }
};

// One wave marches a strip of strip_out_w(V) output columns up the rows
// ya .. yb-1; lane l holds the V columns xa .. xa+V-1, xa = x0 - strip_halo(V) + V l.
// With V = 2 every row access of a wave is one 512-byte span at an 8-byte
// aligned start instead of a 256-byte span at a 4-byte aligned one: fewer
// cache lines per byte, and a halo of 4 columns in 128 instead of 3 in 64.
// At a mirror ghost (x < 0 or x >= nx, transmissive or reflective) a lane's
// two columns map to cells in descending order: the lane loads the ascending
// pair and swaps it; the wave-uniform test keeps interior strips free of it.
template <int SYS, bool BED, typename T, int V, bool BUF = false>
__device__ __forceinline__ void strip2d(const LatticeDesc &L, int64_t iter, int col, int ya, int yb, bool first,
                                        T *lds = nullptr)
{
    constexpr int D = 2, M = SysInfo<SYS, 2>::M, Q = 5;
    constexpr int HC = strip_halo(V), OW = strip_out_w(V);
    const int64_t n = iter - L.iter0;
    Coefs<T> cf;
    if (!step_coefs<D, T>(L, n, cf)) {
        if (first && (threadIdx.x & 63) == 0) flag_degenerate(L, n);
        return;
    }
    const Phys<T> P = make_phys<T>(L);
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = L.nx, ny = L.ny;
    const int xa = col * OW - HC + lane * V;  // this lane's first column
    // with V = 2, nx is even and xa is even, so xa < nx covers both columns
    const bool xout = lane * V >= HC && lane * V < kWave * V - HC && xa < nx;
    if (stopped(L, n)) {
#pragma unroll
        for (int v = 0; v < V; ++v) null_copy<T>(L, n, Q * M, xa + v, xout, ya, yb, first && v == 0);
        return;
    }
    const PlaneIO<T, V, BUF> io(L, n);
    const T *bed = (const T *)L.bed;
    T *om = (T *)L.omega;
    const int bxl = L.bc[0], bxh = L.bc[1], byl = L.bc[2], byh = L.bc[3];
    int xm[V];
    bool rx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) xm[v] = bc_map(xa + v, nx, bxl, bxh, rx[v], HC);
    // first cell of the lane's load and whether its columns come in descending order
    int xl = xm[0];
    bool swp = false;
    if constexpr (V == 2) {
        xl = (xm[0] < xm[1] ? xm[0] : xm[1]) & ~1;
        swp = xm[0] > xm[1];
    }
    const bool anyswap = V > 1 && __ballot(swp) != 0ull;
    const T two_dx = T(2) * P.dx;

    auto fix = [&](T (&a)[V]) {
        if constexpr (V == 2) {
            const T a0 = a[0], a1 = a[1];
            a[0] = swp ? a1 : a0;
            a[1] = swp ? a0 : a1;
        }
    };
    auto fixF = [&](T (*f)[M][V]) {
        if (anyswap) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
#pragma unroll
                for (int c = 0; c < M; ++c) fix(f[k][c]);
        }
    };
    // Moments of a population row j as loaded: U = sum_k f_k (2.3), summed
    // in velocity order, put in column order; the ghost map negates the
    // normal momentum at walls.  (Selects, not a branch on the wave-uniform
    // swap flag: a branch here would make the compiler wait for every memory
    // operation in flight, the previous row's stores included.)
    auto sumU = [&](int j, const T (*f)[M][V], T (*out)[M]) {
        bool ry;
        (void)bc_map(j, ny, byl, byh, ry);
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int c = 0; c < M; ++c) {
                T sum = f[0][c][v];
#pragma unroll
                for (int k = 1; k < Q; ++k) sum = sum + f[k][c][v];
                out[v][c] = sum;
            }
        if constexpr (V == 2) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                T t[2] = {out[0][c], out[1][c]};
                fix(t);
                out[0][c] = t[0];
                out[1][c] = t[1];
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (SYS != 0) {
                if (rx[v]) out[v][1] = -out[v][1];
                if (ry) out[v][2] = -out[v][2];
            }
        }
    };
    auto loadF = [&](int r, T (*out)[M][V]) {
        bool ry;
        const int rm = bc_map(r, ny, byl, byh, ry);
        const unsigned off = (unsigned)(rm * nx + xl);
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int c = 0; c < M; ++c) io.ld(k * M + c, off, out[k][c]);
    };
    auto loadU = [&](int j, T (*out)[M]) {
        T f[Q][M][V];
        loadF(j, f);
        sumU(j, f, out);
    };
    auto loadB = [&](int j, T (&out)[V]) {
        bool ry;
        const int jm = bc_map(j, ny, byl, byh, ry);
        ldv<V>(bed, (unsigned)(jm * nx + xl), out);
    };
    // values at columns x-1 / x+1 of the lane's columns
    auto left_of = [&](const T (&a)[V], T (&o)[V]) {
        o[0] = from_left(a[V - 1]);
#pragma unroll
        for (int v = 1; v < V; ++v) o[v] = a[v - 1];
    };
    auto right_of = [&](const T (&a)[V], T (&o)[V]) {
        o[V - 1] = from_right(a[0]);
#pragma unroll
        for (int v = 0; v < V - 1; ++v) o[v] = a[v + 1];
    };

    T U0[V][M], U1[V][M], U2[V][M];     // U rows j-2, j-1, j
    T Unx[V][M];                        // U row j+1 (in flight, FP64)
    T N0[V], N0l[V], N0r[V];            // nu rows j-3, j-2, j-1 and at x -+ 1
    T N1[V], N1l[V], N1r[V];
    T N2[V], N2l[V], N2r[V];
    T B0[V], B1[V], B2[V], Bnx[V];      // bed rows r-1, r, r+1; row r+2 in flight
    T dbx_prev[V], dby_prev[V];         // bed slope of the previous f* row
    T P1[V][M], P2[V][M];               // f*_{+y} of rows r-1 and r-2
    T G0[V][M], Gpx[V][M], Gmx[V][M], Gmy[V][M]; // row r-1: f*_0, pulled +x, pulled -x, own f*_{-y}
#pragma unroll
    for (int v = 0; v < V; ++v) {
        N0[v] = N0l[v] = N0r[v] = N1[v] = N1l[v] = N1r[v] = N2[v] = N2l[v] = N2r[v] = T(0);
        B0[v] = B1[v] = B2[v] = Bnx[v] = dbx_prev[v] = dby_prev[v] = T(0);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            U0[v][c] = U1[v][c] = U2[v][c] = T(0);
            P1[v][c] = P2[v][c] = G0[v][c] = Gpx[v][c] = Gmx[v][c] = Gmy[v][c] = T(0);
        }
    }
    T s0 = T(0), s1 = T(0);
    unsigned flags = 0;

    // primitives of the U1 row that the last nu_row() formed: the next row()
    // collides that row (as U0) and takes them instead of forming them again.
    // Only with one column per lane: the two-column strips are at the
    // register limit, and carrying them cost the batched kernel's
    // two-column shallow-water strips 19% (more spills), against 1% gained
    // by 2D Euler.
    constexpr bool kCarry = V == 1;
    Prim<T> Qn[V];
    auto nu_row = [&]() {  // nu at the row of U1 (eqs. 2.13-2.14)
        T UL[V][M], UR[V][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            UL[0][c] = from_left(U1[V - 1][c]);
            UR[V - 1][c] = from_right(U1[0][c]);
#pragma unroll
            for (int v = 1; v < V; ++v) {
                UL[v][c] = U1[v - 1][c];
                UR[v - 1][c] = U1[v][c];
            }
        }
        T nu[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            primitives<SYS, D, T>(U1[v], P, Qn[v]);
            nu[v] = T(0);
            add_theta<SYS, D, T>(0, Qn[v], U1[v], UL[v], UR[v], P, nu[v]);
            add_theta<SYS, D, T>(1, Qn[v], U1[v], U0[v], U2[v], P, nu[v]);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            N0[v] = N1[v]; N0l[v] = N1l[v]; N0r[v] = N1r[v];
            N1[v] = N2[v]; N1l[v] = N2l[v]; N1r[v] = N2r[v];
            N2[v] = nu[v];
        }
        left_of(nu, N2l);
        right_of(nu, N2r);
    };
    auto pushU = [&](const T (*u)[M]) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int c = 0; c < M; ++c) {
                U0[v][c] = U1[v][c];
                U1[v][c] = U2[v][c];
                U2[v][c] = u[v][c];
            }
    };
    auto roll_U = [&](int j) {  // U2 <- row j (prefetched), then prefetch row j+1
        pushU(Unx);
        loadU(j + 1, Unx);
    };

    // Every population row is read from memory once and kept until the
    // collision two rows later uses it.  FP32 keeps the rows in a register
    // ring (4 Q m V registers).  FP64 would need twice the registers: with an
    // LDS buffer (lds != nullptr) rows j-1 and j go to two LDS slots of the
    // wave (the row in flight stays in registers); without one it reads the
    // row again in the iteration that collides it, from L2 when it is still
    // there (measured: mostly not, 2.2x the algorithmic reads at 2048^2).
    // FP32 reactive Euler (25 values per row) also reads rows again: its
    // step is bound by the kinetics' arithmetic, and the LDS slots measured
    // 3.5% slower there (0.281 -> 0.291 ms at 2048^2).
    constexpr bool kRing = sizeof(T) == 4 && Q * M <= 20;
    const bool use_lds = sizeof(T) == 8 && lds != nullptr;
    // The ring's rotation copies a row still in flight, so the row loop waits
    // for its loads within the step.  Unrolling the loop by the ring's period
    // makes the slots fixed registers (no copy; the wait falls in the next
    // row's step) at the price of a 4x body and more registers.  Measured on
    // MI355X (ms per step, rotating -> unrolled): advection 0.0540 -> 0.0512,
    // Euler 0.169 -> 0.179, shallow water 0.478 -> 0.492; so only advection
    // unrolls.
    constexpr bool kUnroll = kRing && SYS == 0;
    // Without the unrolled ring, shallow water (15 values per row) prefetches
    // two rows ahead.
    constexpr bool kPf2 = kRing && !kUnroll && SYS == 2;
    // f rows j-1, j, j+1 (in flight), and j+2 (in flight) with two rows of
    // prefetch, kept as loaded; a row is put in column order when the
    // collision takes it.  Unrolled: row x in slot (x - ya + 1) mod 4.
    constexpr bool kRot = kRing && !kUnroll;
    T Rb[kRot ? Q : 1][M][V], Rc[kRot ? Q : 1][M][V], Rn[kRot ? Q : 1][M][V], Rm[kPf2 ? Q : 1][M][V];
    T R[kUnroll ? 4 : 1][kUnroll ? Q : 1][M][V];
    constexpr bool kLdsPath = sizeof(T) == 8;  // compiled for FP64 only
    T Rl[kLdsPath ? Q : 1][M][V];              // FP64 LDS ring: the row in flight
    // LDS slot (row & 1) of the wave: value i of lane l at ((slot Q m + i) 64 + l) V
    auto lds_put = [&](int row, const T (*f)[M][V]) {
        T *base = lds + ((row & 1) * Q * M * kWave + lane) * V;
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int c = 0; c < M; ++c) stv<V>(base, (unsigned)((k * M + c) * kWave * V), f[k][c]);
    };
    auto lds_get = [&](int row, T (*f)[M][V]) {
        const T *base = lds + ((row & 1) * Q * M * kWave + lane) * V;
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int c = 0; c < M; ++c) ldv<V>(base, (unsigned)((k * M + c) * kWave * V), f[k][c]);
    };

    // prologue: moment rows ya-3 .. ya, indicator rows ya-2 .. ya-1
    if constexpr (BED) {
        loadB(ya - 2, B1);
        loadB(ya - 1, B2);
        loadB(ya, Bnx);
        fix(B1);
        fix(B2);
    }
    if constexpr (kUnroll) {
        T Ut[V][M];
        loadU(ya - 3, Ut);
        pushU(Ut);
        loadU(ya - 2, Ut);
        pushU(Ut);
        loadF(ya - 1, R[0]);
        sumU(ya - 1, R[0], Ut);
        pushU(Ut);
        nu_row();
        loadF(ya, R[1]);
        sumU(ya, R[1], Ut);
        pushU(Ut);
        nu_row();
        loadF(ya + 1, R[2]);
    } else if constexpr (kRing) {
        T Ut[V][M];
        loadU(ya - 3, Ut);
        pushU(Ut);
        loadU(ya - 2, Ut);
        pushU(Ut);
        loadF(ya - 1, Rb);
        sumU(ya - 1, Rb, Ut);
        pushU(Ut);
        nu_row();
        loadF(ya, Rc);
        sumU(ya, Rc, Ut);
        pushU(Ut);
        nu_row();
        loadF(ya + 1, Rn);
        if constexpr (kPf2) loadF(ya + 2, Rm);
    } else if (kLdsPath && use_lds) {
        T Ut[V][M], Rt[Q][M][V];
        loadU(ya - 3, Ut);
        pushU(Ut);
        loadU(ya - 2, Ut);
        pushU(Ut);
        loadF(ya - 1, Rt);
        sumU(ya - 1, Rt, Ut);
        lds_put(ya - 1, Rt);
        pushU(Ut);
        nu_row();
        // the row in flight into the loop is requested before row ya, whose
        // wait then covers it: the loop's wait for its row in flight need not
        // drain the stores of the row before
        loadF(ya + 1, Rl);
        loadF(ya, Rt);
        sumU(ya, Rt, Ut);
        lds_put(ya, Rt);
        pushU(Ut);
        nu_row();
    } else {
        loadU(ya - 3, Unx);
        roll_U(ya - 3);
        roll_U(ya - 2);
        roll_U(ya - 1);
        nu_row();
        roll_U(ya);
        nu_row();
    }

    // steady state: the step of row j takes U(j), loads row j+1, computes nu
    // at row j-1, omega and f* at row r = j-2 from its populations fcur, and
    // writes destination row j-3
    auto row = [&](int j, T (*fcur)[M][V]) __attribute__((always_inline)) {
        const int r = j - 2;
        T dbx[V], dby[V];
        if constexpr (BED) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                B0[v] = B1[v];
                B1[v] = B2[v];
                B2[v] = Bnx[v];
            }
            fix(B2);
            loadB(r + 2, Bnx);
        }
        Prim<T> Qc[V];  // primitives of the row collided here (formed by the last nu_row)
        if constexpr (kCarry) {
#pragma unroll
            for (int v = 0; v < V; ++v) Qc[v] = Qn[v];
        }
        nu_row();
        // 3x3 box sum (2.15) in row-major order, relaxation parameter (2.16)
        T w[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T nt = N0l[v] + N0[v] + N0r[v] + N1l[v] + N1[v] + N1r[v] + N2l[v] + N2[v] + N2r[v];
            w[v] = L.omega_fixed_on ? cf.omega_fixed : omega_of<T>(nt);
        }
        // halo lanes and rows outside the band store nothing (masked lanes
        // make no memory request; a shared slot for them cost about 13% of
        // the step in write traffic to the same lines from every wave)
        if (L.omega_on && xout && r >= ya && r < yb) stv<V>(om, (unsigned)(r * nx + xa), w);
        if constexpr (BED) {
            T bl[V], br[V];
            left_of(B1, bl);
            right_of(B1, br);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                dbx[v] = ddiv<T>(br[v] - bl[v], two_dx);
                dby[v] = ddiv<T>(B2[v] - B0[v], two_dx);
            }
        }
        // equilibrium (2.20) and collision at the source nodes of row r
        T fs[V][Q][M];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (!kCarry) primitives<SYS, D, T>(U0[v], P, Qc[v]);
            const Prim<T> &q = Qc[v];
            T Fx[M], Fy[M];
            flux<SYS, D, T>(0, U0[v], q, P, Fx);
            flux<SYS, D, T>(1, U0[v], q, P, Fy);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const T u = U0[v][c];
                const T feq[Q] = {cf.a0 * u, cf.ap[0] * u + cf.bp * Fx[c], cf.ap[1] * u + cf.bp * Fy[c],
                                  cf.ap[0] * u + cf.bm * Fx[c], cf.ap[1] * u + cf.bm * Fy[c]};
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    const T fk = fcur[k][c][v];
                    fs[v][k][c] = fk - w[v] * (fk - feq[k]);
                }
            }
            if constexpr (BED) {
                const T S1 = -P.g * U0[v][0] * dbx[v], S2 = -P.g * U0[v][0] * dby[v];
                const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[0], cf.ap[1]};
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    fs[v][k][1] = fs[v][k][1] + cf.hdt * (ak[k] * S1);
                    fs[v][k][2] = fs[v][k][2] + cf.hdt * (ak[k] * S2);
                }
            }
            if constexpr (SYS == 3) {  // Arrhenius sink of rho Y, first half (2.6)
                const T SY = -arrhenius_rate<T>(P, U0[v][0], reactive_eint<D, T>(U0[v]), U0[v][M - 1], nullptr);
                const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[0], cf.ap[1]};
#pragma unroll
                for (int k = 0; k < Q; ++k) fs[v][k][M - 1] = fs[v][k][M - 1] + cf.hdt * (ak[k] * SY);
            }
        }
        // x pulls with the ghost map at the two x walls
        T px[V][M], mx[V][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            px[0][c] = from_left(fs[V - 1][1][c]);
            mx[V - 1][c] = from_right(fs[0][3][c]);
#pragma unroll
            for (int v = 1; v < V; ++v) {
                px[v][c] = fs[v - 1][1][c];
                mx[v - 1][c] = fs[v][3][c];
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (xa + v == 0 && bxl != 0) {
#pragma unroll
                for (int c = 0; c < M; ++c)
                    px[v][c] = bxl == 1 ? fs[v][1][c] : (c == 1 ? -fs[v][3][c] : fs[v][3][c]);
            }
            if (xa + v == nx - 1 && bxh != 0) {
#pragma unroll
                for (int c = 0; c < M; ++c)
                    mx[v][c] = bxh == 1 ? fs[v][3][c] : (c == 1 ? -fs[v][1][c] : fs[v][1][c]);
            }
        }
        // destination row d = r-1: F_0, F_{+x}, F_{+y}, F_{-x}, F_{-y}
        const int d = r - 1;
        {
            T Fk[Q][M][V];
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    Fk[0][c][v] = G0[v][c];
                    Fk[1][c][v] = Gpx[v][c];
                    Fk[2][c][v] = P2[v][c];
                    Fk[3][c][v] = Gmx[v][c];
                    Fk[4][c][v] = fs[v][4][c];
                }
            if (d == ny - 1 && byh != 0) {
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int c = 0; c < M; ++c) Fk[4][c][v] = byh == 1 ? Gmy[v][c] : (c == 2 ? -P1[v][c] : P1[v][c]);
            }
            const bool ok = xout && d >= ya;
            T Un[V][M];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T sumF[M];
#pragma unroll
                for (int c = 0; c < M; ++c)
                    sumF[c] = Fk[0][c][v] + Fk[1][c][v] + Fk[2][c][v] + Fk[3][c][v] + Fk[4][c][v];
                if constexpr (BED) {
                    const T S1 = -P.g * sumF[0] * dbx_prev[v], S2 = -P.g * sumF[0] * dby_prev[v];
                    const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[0], cf.ap[1]};
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        Fk[k][1][v] = Fk[k][1][v] + cf.hdt * (ak[k] * S1);
                        Fk[k][2][v] = Fk[k][2][v] + cf.hdt * (ak[k] * S2);
                    }
                }
                if constexpr (SYS == 3) {  // (2.8) for rho Y, then the second half source
                    const T eint = reactive_eint<D, T>(sumF);
                    const T z = reactive_solve<T>(P, sumF[0], eint, sumF[M - 1], cf.hdt);
                    const T SY = -arrhenius_rate<T>(P, sumF[0], eint, z, nullptr);
                    const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[0], cf.ap[1]};
#pragma unroll
                    for (int k = 0; k < Q; ++k) Fk[k][M - 1][v] = Fk[k][M - 1][v] + cf.hdt * (ak[k] * SY);
                }
#pragma unroll
                for (int c = 0; c < M; ++c)
                    Un[v][c] = Fk[0][c][v] + Fk[1][c][v] + Fk[2][c][v] + Fk[3][c][v] + Fk[4][c][v];
            }
            if (ok) {
                const unsigned o = (unsigned)(d * nx + xa);
#pragma unroll
                for (int k = 0; k < Q; ++k)
#pragma unroll
                    for (int c = 0; c < M; ++c) io.st(k * M + c, o, Fk[k][c]);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                Prim<T> qn;
                primitives<SYS, D, T>(Un[v], P, qn);
                const T v0 = max_speed<SYS, T>(0, qn, P), v1 = max_speed<SYS, T>(1, qn, P);
                bool fin_ok = true;
#pragma unroll
                for (int c = 0; c < M; ++c) fin_ok = fin_ok && finite_val<T>(Un[v][c]);
                if (ok) {
                    flags |= qn.flags | (fin_ok ? 0u : 1u);
                    if (finite_val<T>(v0) && v0 > s0) s0 = v0;
                    if (finite_val<T>(v1) && v1 > s1) s1 = v1;
                }
            }
        }
        // roll the pulled-population window
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                P2[v][c] = P1[v][c];
                P1[v][c] = fs[v][2][c];
                G0[v][c] = fs[v][0][c];
                Gpx[v][c] = px[v][c];
                Gmx[v][c] = mx[v][c];
                Gmy[v][c] = fs[v][4][c];
            }
            if (r == 0 && byl != 0) {
#pragma unroll
                for (int c = 0; c < M; ++c) P2[v][c] = byl == 1 ? fs[v][2][c] : (c == 2 ? -fs[v][4][c] : fs[v][4][c]);
            }
            if constexpr (BED) {
                dbx_prev[v] = dbx[v];
                dby_prev[v] = dby[v];
            }
        }
    };
    if constexpr (kUnroll) {
        // phase S of the ring: row j in slot S+2, row j+1 loaded into slot
        // S+3, row j-2 (fcur) in slot S
        auto phase = [&](auto phase_tag, int j) __attribute__((always_inline)) {
            constexpr int S = decltype(phase_tag)::value;
            T Ut[V][M];
            sumU(j, R[(S + 2) & 3], Ut);
            pushU(Ut);
            loadF(j + 1, R[(S + 3) & 3]);
            fixF(R[S]);
            row(j, R[S]);
        };
        const int nrows = yb + 2 - ya;  // steps j = ya+1 .. yb+2
        int i = 0;
        for (; i + 4 <= nrows; i += 4) {
            phase(Phase<0>(), ya + 1 + i);
            phase(Phase<1>(), ya + 2 + i);
            phase(Phase<2>(), ya + 3 + i);
            phase(Phase<3>(), ya + 4 + i);
        }
        if (i < nrows) phase(Phase<0>(), ya + 1 + i);
        if (i + 1 < nrows) phase(Phase<1>(), ya + 2 + i);
        if (i + 2 < nrows) phase(Phase<2>(), ya + 3 + i);
    } else {
        for (int j = ya + 1; j <= yb + 2; ++j) {
            T fcur[Q][M][V];
            if constexpr (kRing) {
                T Ut[V][M];
                sumU(j, Rn, Ut);
                pushU(Ut);
#pragma unroll
                for (int k = 0; k < Q; ++k)
#pragma unroll
                    for (int c = 0; c < M; ++c)
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            fcur[k][c][v] = Rb[k][c][v];
                            Rb[k][c][v] = Rc[k][c][v];
                            Rc[k][c][v] = Rn[k][c][v];
                            if constexpr (kPf2) Rn[k][c][v] = Rm[k][c][v];
                        }
                if constexpr (kPf2)
                    loadF(j + 2, Rm);
                else
                    loadF(j + 1, Rn);
                fixF(fcur);
            } else if (kLdsPath && use_lds) {
                T Ut[V][M];
                sumU(j, Rl, Ut);
                pushU(Ut);
                // row j-2 out of the slot that row j then takes (the LDS
                // operations of a wave complete in order)
                lds_get(j - 2, fcur);
                lds_put(j, Rl);
                loadF(j + 1, Rl);
                fixF(fcur);
            } else {
                roll_U(j);
                loadF(j - 2, fcur);
                fixF(fcur);
            }
            row(j, fcur);
        }
    }
    if (first) scalar_update(L, n, cf.dt);
    commit<T>(L, n, s0, s1, flags, 2);
}

// -------------------------------------------------------------- kernels ---

// Block -> work mapping that keeps consecutive work items on one XCD
// (blocks are dealt round-robin over the 8 XCDs; gridDim.x is a multiple of 8).
__device__ __forceinline__ int logical_wave()
{
    const int b = blockIdx.x, nb = gridDim.x;
    const int lb = (b & 7) * (nb >> 3) + (b >> 3);
    return __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + (int)(threadIdx.x >> 6));
}

// FP64 2D steps keep two population rows per wave in LDS (measured per step
// at 2048^2 and 4096^2: Euler 0.375 -> 0.318 ms, shallow water 1.086 ->
// 0.909, reactive 0.517 -> 0.493, advection 0.117 -> 0.126, so advection,
// whose rows are 5 values, reads them again; kernels whose slots would not
// fit the CU's 160 KB of LDS do too).  Elements of one wave's two slots:
template <int SYS, typename T, int V>
__host__ __device__ constexpr int lds_ring_elems()
{
    return sizeof(T) == 8 && SYS != 0 &&
                   kWavesPerBlock * 2 * 5 * SysInfo<SYS, 2>::M * kWave * V * sizeof(T) <= 160 * 1024
               ? 2 * 5 * SysInfo<SYS, 2>::M * kWave * V
               : 0;
}

template <int SYS, int D, bool BED, typename T, int V = 1, bool BUF = false>
__global__ __launch_bounds__(kBlock) void k_step_single(LatticeDesc L, int64_t iter, int32_t nwork)
{
    const int w = logical_wave();
    if (w >= nwork) return;
    if constexpr (D == 1) {
        seg1d<SYS, T>(L, iter, w, w + 1);
    } else {
        const int col = w % L.ncols, ya = (w / L.ncols) * L.band_h;
        const int yb = ya + L.band_h < L.ny ? ya + L.band_h : L.ny;
        constexpr int kRing = lds_ring_elems<SYS, T, V>();
        if constexpr (kRing > 0) {
            __shared__ T ring[kWavesPerBlock * kRing];
            strip2d<SYS, BED, T, V, BUF>(L, iter, col, ya, yb, w == 0, ring + (threadIdx.x >> 6) * kRing);
        } else {
            strip2d<SYS, BED, T, V, BUF>(L, iter, col, ya, yb, w == 0);
        }
    }
}

// One 2D segment of the batched step with the lattice's own strip width and
// buffer-resource addressing (served lattices whose population buffer spans
// 4 GiB or more run a launch of their own).
template <int SYS, bool BED, typename T, int V>
__device__ __forceinline__ void seg2d(const LatticeDesc &L, int64_t iter, const Segment &g, T *lds)
{
    constexpr int kRing = lds_ring_elems<SYS, T, V>();
    strip2d<SYS, BED, T, V, true>(L, iter, g.col, g.y0, g.y1, g.col == 0 && g.y0 == 0,
                                  kRing > 0 ? lds : nullptr);
}
template <int SYS, bool BED, typename T>
__device__ __forceinline__ void seg2d_cpl(const LatticeDesc &L, int64_t iter, const Segment &g, T *lds)
{
    // the widths the single-lattice path takes per system and precision
    // (two columns per lane need an even nx)
    constexpr bool kTwo = SYS == 2 || (SYS == 0 && sizeof(T) == 4);
    if (kTwo && L.cpl == 2) seg2d<SYS, BED, T, kTwo ? 2 : 1>(L, iter, g, lds);
    else seg2d<SYS, BED, T, 1>(L, iter, g, lds);
}

// Batched step: persistent waves take work items (a row band of one 2D strip
// or a run of 1D strips of one lattice) from per-XCD queues until every queue
// is empty.  Queue q holds items qstart[q] .. qstart[q+1]-1 of the work list.
// Blocks are dealt to the 8 XCDs round robin, so block b runs on XCD b mod 8,
// where its wave k has rank r = 4 (b / 8) + k among the XCD's w waves.  A
// wave's first item is item r of its XCD's queue, as a static deal would give
// it (a lattice alone thus runs in the single-lattice kernel's layout: one
// band of one strip per wave, neighbouring strips on neighbouring waves of
// one XCD); the items after the first w of each queue are taken through its
// counter (item w + counter), first from the wave's own queue, then from the
// queue with the most items left.  The counters of this launch are set
// `parity` (kQueues counters kQueueStride words apart), the parity of the
// number of batched launches made before it; the launch zeroes the other set,
// which the previous batched launch used and the next one takes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_step_batched(const LatticeDesc *__restrict__ descs,
                                                          const Segment *__restrict__ segs,
                                                          const int32_t *__restrict__ qstart,
                                                          unsigned *__restrict__ counters, int32_t parity,
                                                          int64_t iter)
{
    constexpr int kRing = lds_ring_elems<2, T, 2>() > lds_ring_elems<3, T, 1>() ? lds_ring_elems<2, T, 2>()
                                                                                 : lds_ring_elems<3, T, 1>();
    __shared__ T ring[kWavesPerBlock * (kRing > 0 ? kRing : 1)];
    T *lds = ring + (threadIdx.x >> 6) * kRing;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned *ctr = counters + (parity & 1) * (kQueues * kQueueStride);
    if (blockIdx.x == 0 && threadIdx.x < kQueues)
        counters[((parity + 1) & 1) * (kQueues * kQueueStride) + threadIdx.x * kQueueStride] = 0u;
    const int wpx = (int)(gridDim.x / kQueues) * kWavesPerBlock;  // waves per XCD (gridDim.x: a multiple of 8)
    auto run = [&](int item) {
        const Segment g = segs[item];
        const LatticeDesc &L = descs[g.lattice];
        switch (L.variant) {
        case V_ADV1: seg1d<0, T>(L, iter, g.col, g.y1); break;
        case V_EUL1: seg1d<1, T>(L, iter, g.col, g.y1); break;
        case V_SWE1: seg1d<2, T>(L, iter, g.col, g.y1); break;
        case V_REU1: seg1d<3, T>(L, iter, g.col, g.y1); break;
        case V_ADV2: seg2d_cpl<0, false, T>(L, iter, g, lds); break;
        case V_EUL2: seg2d_cpl<1, false, T>(L, iter, g, lds); break;
        case V_SWE2:
            if (L.bed) seg2d_cpl<2, true, T>(L, iter, g, lds);
            else seg2d_cpl<2, false, T>(L, iter, g, lds);
            break;
        case V_REU2: seg2d_cpl<3, false, T>(L, iter, g, lds); break;
        default: break;
        }
    };
    int c = (int)(blockIdx.x & (kQueues - 1));
    const int rank = (int)__builtin_amdgcn_readfirstlane((blockIdx.x / kQueues) * kWavesPerBlock +
                                                         (threadIdx.x >> 6));
    // the wave's first item (static), else -1; later items from the counters
    int item = rank < qstart[c + 1] - qstart[c] ? qstart[c] + rank : -1;
    // every failed take means another wave took an item, so the loop ends;
    // the bound on failed takes in a row makes the end certain
    for (int failed = 0; failed < 4096;) {
        if (item < 0) {
            const int lo = qstart[c], n = qstart[c + 1] - lo;
            int i = n;  // (the first wpx items went to the waves' first takes)
            if (wpx < n) {
                unsigned got = 0u;
                if (lane == 0) got = atomicAdd(&ctr[c * kQueueStride], 1u);
                i = wpx + (int)__builtin_amdgcn_readfirstlane(got);
            }
            if (i < n) {
                item = lo + i;
            } else {
                ++failed;
                // queue c is empty: read every counter at once (lane q reads
                // queue q) and go on with the queue that has the most items
                // left; stop when none has any
                int left = -1;
                if (lane < kQueues) {
                    const unsigned taken =
                        __hip_atomic_load(&ctr[lane * kQueueStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int nq = qstart[lane + 1] - qstart[lane];
                    const long long next = (long long)wpx + (long long)taken;
                    left = next < nq ? nq - (int)next : 0;
                }
                int key = left < 0 ? -1 : left * kQueues + (kQueues - 1 - lane);
#pragma unroll
                for (int o = 4; o > 0; o >>= 1) {
                    const int other = __shfl_xor(key, o, kWave);
                    key = other > key ? other : key;
                }
                key = (int)__builtin_amdgcn_readfirstlane((unsigned)key);
                if (key < kQueues) break;  // no queue has items left
                c = kQueues - 1 - key % kQueues;
                continue;
            }
        }
        failed = 0;
        run(item);
        item = -1;
    }
}

// Wave-speed bound of the initial state: atomic max of max_r |lambda_j^(r)|.
template <int SYS, int D, typename T>
__global__ __launch_bounds__(kBlock) void k_reduce_abar(LatticeDesc L, const double *U0, int slot)
{
    constexpr int M = SysInfo<SYS, D>::M;
    const Phys<T> P = make_phys<T>(L);
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.plane;
         i += (int64_t)gridDim.x * blockDim.x) {
        T U[M];
#pragma unroll
        for (int c = 0; c < M; ++c) U[c] = T(U0[(int64_t)c * L.plane + i]);
        Prim<T> q;
        primitives<SYS, D, T>(U, P, q);
        const T v0 = max_speed<SYS, T>(0, q, P);
        if (finite_val<T>(v0) && v0 > s0) s0 = v0;
        if constexpr (D >= 2) {
            const T v1 = max_speed<SYS, T>(1, q, P);
            if (finite_val<T>(v1) && v1 > s1) s1 = v1;
        }
        if constexpr (D == 3) {
            const T v2 = max_speed<SYS, T>(2, q, P);
            if (finite_val<T>(v2) && v2 > s2) s2 = v2;
        }
    }
    const double m0 = (double)wave_max<T>(s0), m1 = (double)wave_max<T>(s1), m2 = (double)wave_max<T>(s2);
    if ((threadIdx.x & 63) == 0) {
        AbarCopy &c = L.sc->abar[slot][abar_copy(L)];
        atomicMax(&c.v[0], dbits(m0));
        if (D >= 2) atomicMax(&c.v[1], dbits(m1));
        if (D == 3) atomicMax(&c.v[2], dbits(m2));
    }
}

// f = f^eq(U0) with the coefficients of U0's bounds (slot_in); U = sum_k f_k;
// bounds of U into slot 0; bed converted to the storage precision.
template <int SYS, int D, typename T>
__global__ __launch_bounds__(kBlock) void k_init(LatticeDesc L, const double *U0, const double *bed64, int slot_in)
{
    constexpr int M = SysInfo<SYS, D>::M, Q = SysInfo<SYS, D>::Q;
    const Phys<T> P = make_phys<T>(L);
    // coefficients of the initial state, same formulas as a step
    const double ab0 = abar_of(L, slot_in, 0);
    const double ab1 = D >= 2 ? abar_of(L, slot_in, 1) : 0.0;
    const double ab2 = D == 3 ? abar_of(L, slot_in, 2) : 0.0;
    const double sa = D == 3 ? (ab0 + ab1) + ab2 : (D == 2 ? ab0 + ab1 : ab0);
    const double dt = L.cfl * L.dx / sa;
    const double lam = L.dx / dt;
    const double al0 = ab0 + L.eps, al1 = ab1 + L.eps, al2 = ab2 + L.eps;
    const double sum_alpha = D == 3 ? (al0 + al1) + al2 : (D == 2 ? al0 + al1 : al0);
    const T a0 = T(1.0 - sum_alpha / lam);
    const T ap[3] = {T(al0 / (2.0 * lam)), T(al1 / (2.0 * lam)), T(al2 / (2.0 * lam))};
    const T bp = T(1.0 / (2.0 * lam)), bm = T(-1.0 / (2.0 * lam));
    T *f = (T *)L.f[0];
    T *u = (T *)L.u[0];
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.plane;
         i += (int64_t)gridDim.x * blockDim.x) {
        T U[M], F[D][M];
#pragma unroll
        for (int c = 0; c < M; ++c) U[c] = T(U0[(int64_t)c * L.plane + i]);
        Prim<T> q;
        primitives<SYS, D, T>(U, P, q);
#pragma unroll
        for (int j = 0; j < D; ++j) flux<SYS, D, T>(j, U, q, P, F[j]);
        T Un[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T feq[Q];
            feq[0] = a0 * U[c];
            // velocities: k = 1..D the +j directions, k = D+1..2D the -j directions
#pragma unroll
            for (int j = 0; j < D; ++j) {
                feq[1 + j] = ap[j] * U[c] + bp * F[j][c];
                feq[1 + D + j] = ap[j] * U[c] + bm * F[j][c];
            }
            T s = feq[0];
#pragma unroll
            for (int k = 1; k < Q; ++k) s = s + feq[k];
#pragma unroll
            for (int k = 0; k < Q; ++k) f[(int64_t)(k * M + c) * L.pstride + i] = feq[k];
            Un[c] = s;
            u[(int64_t)c * L.pstride + i] = s;
        }
        if (bed64 && L.bed) ((T *)L.bed)[i] = T(bed64[i]);
        Prim<T> qn;
        primitives<SYS, D, T>(Un, P, qn);
        const T v0 = max_speed<SYS, T>(0, qn, P);
        if (finite_val<T>(v0) && v0 > s0) s0 = v0;
        if constexpr (D >= 2) {
            const T v1 = max_speed<SYS, T>(1, qn, P);
            if (finite_val<T>(v1) && v1 > s1) s1 = v1;
        }
        if constexpr (D == 3) {
            const T v2 = max_speed<SYS, T>(2, qn, P);
            if (finite_val<T>(v2) && v2 > s2) s2 = v2;
        }
    }
    const double m0 = (double)wave_max<T>(s0), m1 = (double)wave_max<T>(s1), m2 = (double)wave_max<T>(s2);
    if ((threadIdx.x & 63) == 0) {
        AbarCopy &c = L.sc->abar[0][abar_copy(L)];
        atomicMax(&c.v[0], dbits(m0));
        if (D >= 2) atomicMax(&c.v[1], dbits(m1));
        if (D == 3) atomicMax(&c.v[2], dbits(m2));
    }
}

// Moments U = sum_k f_k of every cell (velocity order), for read-back and
// conservation sums; the step kernels themselves never store U.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(const T *f, T *u, int64_t plane, int64_t pstride, int m, int q)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < m; ++c) {
            T s = f[(int64_t)c * pstride + i];
            for (int k = 1; k < q; ++k) s = s + f[(int64_t)(k * m + c) * pstride + i];
            u[(int64_t)c * pstride + i] = s;
        }
}

// Per-block compensated (Neumaier) sums of each moment plane, in a fixed
// order: partial[c * gridDim.x + block].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_conservation(const T *u, int64_t plane, int64_t pstride, int m,
                                                          double *partial)
{
    __shared__ double ss[kBlock], cc[kBlock];
    const int64_t per = (plane + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < plane ? lo + per : plane;
    for (int c = 0; c < m; ++c) {
        double s = 0.0, e = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double v = (double)u[(int64_t)c * pstride + i];
            const double t = s + v;
            e += __builtin_fabs(s) >= __builtin_fabs(v) ? (s - t) + v : (v - t) + s;
            s = t;
        }
        ss[threadIdx.x] = s;
        cc[threadIdx.x] = e;
        __syncthreads();
        for (int h = kBlock / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                const double a = ss[threadIdx.x], b = ss[threadIdx.x + h];
                const double t = a + b;
                const double err = __builtin_fabs(a) >= __builtin_fabs(b) ? (a - t) + b : (b - t) + a;
                ss[threadIdx.x] = t;
                cc[threadIdx.x] = cc[threadIdx.x] + cc[threadIdx.x + h] + err;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = ss[0] + cc[0];
        __syncthreads();
    }
}

// m planes at stride pstride -> dense FP64 planes of `plane` values.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_double(const T *src, double *dst, int64_t plane, int64_t pstride,
                                                       int m)
{
    const int64_t n = plane * m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / plane, k = i - c * plane;
        dst[i] = (double)src[c * pstride + k];
    }
}

}  // namespace arlbm
