// One time step of the method on a D3Q7 lattice (Section 2.3 with d = 3:
// e_0 = 0, e_j the unit vectors, e_{j+3} = -e_j) in one fused pass.  The
// moments U = sum_k f_k (eq. 2.3) of the current state are kept in the
// ping-pong buffer u[n&1]: written by the initialisation and by each step for
// the next one, so that the indicator reads U instead of the populations.
// A population pulled from a ghost position outside a non-periodic face is
// the destination's own collided population: the same velocity
// (transmissive) or the mirrored one with the normal momentum negated
// (reflective), as in the 1D/2D kernels.
#pragma once

#include "step.hpp"

namespace arlbm {

// Cell index of (i, j, l).
__device__ __forceinline__ int64_t cell3(const LatticeDesc &L, int i, int j, int l)
{
    return ((int64_t)l * L.ny + j) * L.nx + i;
}

// U at any position within three cells of the lattice (positions further out
// are clamped; their values go unused): each axis through its boundary index
// map; reflective maps negate that axis's momentum.
template <int M, typename T>
__device__ __forceinline__ void load_U3(const LatticeDesc &L, const T *u, int i, int j, int l, bool mom, T *U)
{
    bool rx, ry, rz;
    const int im = bc_map(i, L.nx, L.bc[0], L.bc[1], rx);
    const int jm = bc_map(j, L.ny, L.bc[2], L.bc[3], ry);
    const int lm = bc_map(l, L.nz, L.bc[4], L.bc[5], rz);
    const int64_t c0 = cell3(L, im, jm, lm);
#pragma unroll
    for (int c = 0; c < M; ++c) U[c] = u[(int64_t)c * L.pstride + c0];
    if (mom) {
        if (rx) U[1] = -U[1];
        if (ry) U[2] = -U[2];
        if (rz) U[3] = -U[3];
    }
}

// ------------------------------------------------------- fused 3D step ---
//
// One pass per step.  A block owns an x-y tile of TX x TY destination
// columns and a range of planes [za, zb), and marches up through the planes.
// LDS holds the moments of four planes over the tile and a three-cell halo,
// the indicator of three planes over the tile and a two-cell halo, and omega
// of one plane over the tile and a one-cell halo.  Iteration s has two
// phases, each closed by a barrier:
//
//   1. moments of plane s+3 into LDS (read from HBM an iteration ahead);
//      omega of plane s: box sum (2.15) over the indicator planes s-1 .. s+1,
//      z outermost and x innermost, then (2.16);
//   2. in the first TX*TY threads (one per tile column), the collision at
//      plane s (eqs. 2.2, 2.5, 2.6, 2.20).  A column's thread collides its
//      cell's rest and +-z populations and the in-plane ones it pulls from
//      its four neighbours (their moments and omega from LDS, the population
//      from HBM, read by this thread only).  The +z population goes to the
//      destination one plane up, the -z one to the destination one plane
//      down, which is then complete: the moment update (2.8), the second half
//      source, the moments of the new state and the next step's wave-speed
//      bounds (2.19).  The thread then requests the next plane's populations,
//      which arrive during the rest of the iteration.  Then (all threads) the
//      indicator (2.13-2.14) of plane s+2 over the tile and a two-cell halo,
//      from the LDS moments of planes s+1 .. s+3, and (FP32 Euler and
//      reactive Euler) the request of plane s+4's moments.
//
// Every population of the old state is read from HBM once and every
// population and moment of the new state written once; the old moments are
// read once per tile and its halo.  The indicator of a halo cell is
// evaluated by every tile that needs it (720 evaluations per 512 columns in
// FP32).  Sums keep the order of the cell-parallel formulation (k = 0 .. 6
// in 2.8, the box sum as above), so FP64 results are the oracle's bits.
//
// Tiles of 32 x 16 columns.  Euler (FP32 and FP64) and FP64 advection: 512
// threads, all of them destination threads (two waves per SIMD, up to 256
// registers), each evaluating one or two indicator cells.  FP32 advection:
// 768 threads, the first 512 the destination threads.  A 256^3 lattice is
// 128 tiles in two plane chunks: one block per CU.  Measured at 256^3 Euler
// FP32 (ms per step): tiles of 8 rows with the indicator in waves of its own
// 1.34; tiles of 16 rows in 768 threads of 168 registers 1.23-1.27; the same
// with populations requested two planes ahead (8 waves of 256 registers)
// 1.29; requesting each group of the next plane as soon as its registers are
// free 1.68; the collision before the indicator 1.195; with the
// non-temporal accesses below 1.135-1.17; with the late moment loads (below)
// 1.16-1.18, and in 512 threads 1.136-1.14 (768 threads spilled 20 bytes per
// lane; 512 threads of 32 x 24 tiles: 2.03; 32 x 8 tiles: 1.53; advection in
// 512 threads: 0.33 -> 0.37).  Euler FP64: 16 x 16 tiles of 448 threads (one
// destination wave per SIMD) 4.09; 16 x 32 and 32 x 16 of 512 threads 3.18
// and 3.07 (the three-pass version before the fusion: 3.2).
template <int SYS, typename T>
struct Tile3 {
    // FP32 reactive Euler (six fields, the Arrhenius rate at every pulled
    // source) in tiles of 8 rows: 448 threads of 249 registers instead of 768
    // spilling 384 bytes each (256^3: 2.73 -> 2.45 ms per step; advection in
    // tiles of 24 rows, 1024 threads: 0.33 -> 0.44, not kept).  FP64 reactive
    // Euler keeps 16 x 16 tiles (six fields of a 32 x 16 tile and its halo
    // exceed the LDS), of 256 threads that all collide: one wave per SIMD,
    // with room for 512 registers, against 448 threads of which 256 collide
    // and spill 464 bytes each (256^3: 10.3 -> 5.3 ms per step; in FP32 the
    // same made reactive Euler slower, 2.41 -> 2.76).
    static constexpr bool kWide64 = sizeof(T) == 8 && SYS != 3;
    static constexpr int TX = sizeof(T) == 4 || kWide64 ? 32 : 16;
    static constexpr int TY = SYS == 3 && sizeof(T) == 4 ? 8 : 16;
    static constexpr int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;  // moments: tile + 3
    static constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;  // indicator: tile + 2
    static constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;  // omega: tile + 1
    static constexpr int NT = TX * TY;
    static constexpr int kDest = (NT + kWave - 1) / kWave * kWave;  // destination threads
    // every thread collides and evaluates one or two indicator cells, or (FP32
    // advection and reactive Euler) one indicator cell each
    static constexpr bool kAllDest = sizeof(T) == 8 || SYS == 1;
    static constexpr int kThreads = kAllDest ? kDest : ((N2 > NT ? N2 : NT) + kWave - 1) / kWave * kWave;
    static constexpr int kUPer = (N3 + kThreads - 1) / kThreads;  // cells per thread: moments,
    static constexpr int kNPer = (N2 + kThreads - 1) / kThreads;  // indicator,
    static constexpr int kWPer = (N1 + kThreads - 1) / kThreads;  // omega
};

// Launch shape of the fused step: tiles x plane chunks, enough blocks to
// give every CU one (chunks of at least 8 planes).
__host__ __device__ inline int k3_tiles(int nx, int ny, int tx, int ty)
{
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
}
__host__ __device__ inline int k3_chunks(int ntiles, int nz, int num_cus)
{
    const int c = (num_cus + ntiles - 1) / ntiles;
    const int cmax = nz / 8 > 1 ? nz / 8 : 1;
    return c < 1 ? 1 : (c > cmax ? cmax : c);
}

// A 3D velocity mirrored through its axis (1 <-> 4, 2 <-> 5, 3 <-> 6).
__device__ __forceinline__ int mirror3(int k) { return k <= 3 ? k + 3 : k - 3; }

// Populations of the old state read (except the +-x pulls, below) and the
// new state stored non-temporal: nothing reads them again in this step, and
// they stay out of the way of the moments the tiles' halos read from L2
// (256^3 Euler FP32, ms per step: stores 1.200 -> 1.156, then loads 1.163 ->
// 1.135; in the 2D kernels either made the step 2-30% slower).
template <typename T>
__device__ __forceinline__ void sto_nt(T *base, unsigned off, T v)
{
    __builtin_nontemporal_store(v, base + off);
}
template <typename T>
__device__ __forceinline__ T ldo_nt(const T *base, unsigned off)
{
    return __builtin_nontemporal_load(base + off);
}

// A uniform base pointer and plane stride made opaque where they are used:
// the compiler then forms each field's address there (a few scalar ops)
// instead of holding one 64-bit address per field across the plane loop,
// which exceeds the scalar registers.
template <typename P>
__device__ __forceinline__ void opaque(P *&base, int64_t &stride)
{
    asm volatile("" : "+s"(base), "+s"(stride));
}

template <int SYS, typename T>
__global__ __launch_bounds__((Tile3<SYS, T>::kThreads)) void k3_step(LatticeDesc L, int64_t iter)
{
    using G = Tile3<SYS, T>;
    constexpr int D = 3, M = SysInfo<SYS, 3>::M, Q = 7;
    constexpr int TX = G::TX, TY = G::TY, W3 = G::W3, W2 = G::W2, W1 = G::W1;
    __shared__ T lu[4][M][G::N3];
    __shared__ T lnu[3][G::N2];
    __shared__ T lw[G::N1];
    // FP32 reactive Euler: the source rate of plane s over the tile + 1,
    // formed once per cell beside omega, which the pulls read for their
    // sources instead of forming it again (256^3: 2.41 -> 2.29 ms per step;
    // FP64, where the collision holds the destination threads longer, 5.61
    // -> 5.67, so it forms the rates in the collision)
    constexpr bool kRateLds = SYS == 3 && sizeof(T) == 4;
    __shared__ T lrate[kRateLds ? G::N1 : 1];

    const int64_t n = iter - L.iter0;
    const int tid = threadIdx.x;
    const T *fin = (const T *)L.f[n & 1];
    T *fout = (T *)L.f[(n + 1) & 1];
    const int64_t ps = L.pstride;
    const T *u = (const T *)L.u[n & 1];
    T *uout = (T *)L.u[(n + 1) & 1];
    if (L.sc->t[n % 3] >= L.t_stop) {  // null step: the state is at the stop time
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + tid; c < L.plane; c += stride) {
            for (int p = 0; p < Q * M; ++p) fout[(int64_t)p * ps + c] = fin[(int64_t)p * ps + c];
            for (int p = 0; p < M; ++p) uout[(int64_t)p * ps + c] = u[(int64_t)p * ps + c];
        }
        if (blockIdx.x == 0 && tid < kWave) null_scalars(L, n);
        return;
    }
    Coefs<T> cf;
    if (!step_coefs<D, T>(L, n, cf)) {
        if (blockIdx.x == 0 && tid == 0) flag_degenerate(L, n);
        return;
    }
    const Phys<T> P = make_phys<T>(L);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const unsigned nxy = (unsigned)nx * (unsigned)ny;

    // this block's tile and planes; consecutive items (x fastest, then y,
    // then the chunk) on one XCD
    const int ntx = (nx + TX - 1) / TX;
    const int ntile = ntx * ((ny + TY - 1) / TY);
    const int nchunk = (int)gridDim.x / ntile;
    int item = blockIdx.x;
    {
        const int full = (int)gridDim.x & ~7;
        if (item < full) item = (item & 7) * (full >> 3) + (item >> 3);
    }
    const int chunk = item / ntile, tile = item - chunk * ntile;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int za = (int)((int64_t)chunk * nz / nchunk), zb = (int)((int64_t)(chunk + 1) * nz / nchunk);
    const bool fixed = L.omega_fixed_on != 0;
    const T wfix = T(L.omega_fixed);
    const bool zlo_wall = L.bc[4] != 0 && za == 0, zhi_wall = L.bc[5] != 0 && zb == nz;
    // a tile on a reflective x or y face reads mirrored populations there
    const bool refl_xy = (L.bc[0] == 2 && x0 == 0) || (L.bc[1] == 2 && x0 + TX >= nx) ||
                         (L.bc[2] == 2 && y0 == 0) || (L.bc[3] == 2 && y0 + TY >= ny);

    // moments stage (all threads): thread -> cells tid, tid + kThreads, ...
    // of the tile + 3
    constexpr int UP = G::kUPer;
    auto u_load = [&](int p, T (*Ul)[M]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < UP; ++i) {
            const int c = tid + i * G::kThreads;
            if (c < G::N3) load_U3<M, T>(L, u, x0 - 3 + c % W3, y0 - 3 + c / W3, p, SYS != 0, Ul[i]);
        }
    };
    auto u_store = [&](int p, const T (*Ul)[M]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < UP; ++i) {
            const int cl = tid + i * G::kThreads;
            if (cl < G::N3)
#pragma unroll
                for (int c = 0; c < M; ++c) lu[(p + 4) & 3][c][cl] = Ul[i][c];
        }
    };
    // relaxation stage (all threads): thread -> cells tid, tid + kThreads,
    // ... of the tile + 1
    int w_idx[G::kWPer];
#pragma unroll
    for (int i = 0; i < G::kWPer; ++i) w_idx[i] = tid + i * G::kThreads;
    auto w_cell = [&](int s, int wt) __attribute__((always_inline)) {
        if (wt >= G::N1) return;
        const int wxl = wt % W1, wyl = wt / W1;
        if constexpr (kRateLds) {
            const int r3 = (wyl + 2) * W3 + wxl + 2;
            T Uc[M];
#pragma unroll
            for (int c = 0; c < M; ++c) Uc[c] = lu[(s + 4) & 3][c][r3];
            lrate[wt] = -arrhenius_rate<T>(P, Uc[0], reactive_eint<D, T>(Uc), Uc[M - 1], nullptr);
        }
        const int wr = (wyl + 1) * W2 + wxl + 1;
        T w;
        if (fixed) {
            w = wfix;
        } else {
            T nt = T(0);
#pragma unroll
            for (int kl = -1; kl <= 1; ++kl) {
                const T *nv = lnu[(s + kl + 3) % 3];
#pragma unroll
                for (int kj = -1; kj <= 1; ++kj)
#pragma unroll
                    for (int ki = -1; ki <= 1; ++ki) nt = nt + nv[wr + kj * W2 + ki];
            }
            w = omega_of<T>(nt);
        }
        lw[wt] = w;
        if (L.omega_on && s >= za && s < zb) {
            const int gx = x0 - 1 + wxl, gy = y0 - 1 + wyl;
            if (wxl >= 1 && wxl <= TX && wyl >= 1 && wyl <= TY && gx < nx && gy < ny)
                ((T *)L.omega)[cell3(L, gx, gy, s)] = w;
        }
    };
    auto w_stage = [&](int s) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < G::kWPer; ++i) w_cell(s, w_idx[i]);
    };
    // indicator stage (all threads): thread -> cells tid, tid + kThreads,
    // ... of the tile + 2
    const bool is_dest = tid < G::kDest;
    int nu_r[G::kNPer];
#pragma unroll
    for (int i = 0; i < G::kNPer; ++i) {
        const int vt = tid + i * G::kThreads;
        nu_r[i] = (vt / W2 + 1) * W3 + vt % W2 + 1;
    }
    auto nu_cell = [&](int p, int vt, int nr) __attribute__((always_inline)) {
        if (fixed || vt >= G::N2) return;
        const int sc = (p + 4) & 3, sm = (p + 3) & 3, sp = (p + 5) & 3;
        T Uc[M], Um[M], Up[M];
#pragma unroll
        for (int c = 0; c < M; ++c) Uc[c] = lu[sc][c][nr];
        Prim<T> qc;
        primitives<SYS, D, T>(Uc, P, qc);
        T nu = T(0);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Um[c] = lu[sc][c][nr - 1];
            Up[c] = lu[sc][c][nr + 1];
        }
        add_theta<SYS, D, T>(0, qc, Uc, Um, Up, P, nu);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Um[c] = lu[sc][c][nr - W3];
            Up[c] = lu[sc][c][nr + W3];
        }
        add_theta<SYS, D, T>(1, qc, Uc, Um, Up, P, nu);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Um[c] = lu[sm][c][nr];
            Up[c] = lu[sp][c][nr];
        }
        add_theta<SYS, D, T>(2, qc, Uc, Um, Up, P, nu);
        lnu[(p + 3) % 3][vt] = nu;
    };
    auto nu_stage = [&](int p) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < G::kNPer; ++i) nu_cell(p, tid + i * G::kThreads, nu_r[i]);
    };

    // destination stage (the first waves): thread -> column of the tile
    const int tx = tid % TX, ty = tid / TX;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool live = tid < G::NT && gx < nx && gy < ny;
    const int dr3 = (ty + 3) * W3 + tx + 3, dr1 = (ty + 1) * W1 + tx + 1;
    const unsigned doff = live ? (unsigned)gy * (unsigned)nx + (unsigned)gx : 0u;
    // the in-plane pulls j = 0 .. 3 of k = 1 (+x), 2 (+y), 4 (-x), 5 (-y):
    // the source's offset in the plane, and bit j of own_m when the source is
    // this cell itself (a transmissive or reflective face), of refl_m when
    // the population is read mirrored with its normal momentum negated
    unsigned poff[4];
    unsigned own_m = 0, refl_m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = j < 2 ? j + 1 : j + 2;
        const int dir = (k - 1) % 3;
        const int sgn = k <= 3 ? 1 : -1;
        int sx = gx - (dir == 0 ? sgn : 0), sy = gy - (dir == 1 ? sgn : 0);
        const int s_ax = dir == 0 ? sx : sy, n_ax = dir == 0 ? nx : ny;
        if (s_ax < 0 || s_ax >= n_ax) {
            const int b = L.bc[2 * dir + (s_ax < 0 ? 0 : 1)];
            if (b == 0) {
                if (dir == 0) sx = s_ax < 0 ? nx - 1 : 0;
                else sy = s_ax < 0 ? ny - 1 : 0;
            } else {
                sx = gx;
                sy = gy;
                own_m |= 1u << j;
                if (b == 2) refl_m |= 1u << j;
            }
        }
        poff[j] = live ? (unsigned)sy * (unsigned)nx + (unsigned)sx : 0u;
    }
    auto pull_r3 = [&](int j) __attribute__((always_inline)) -> int {
        const int k = j < 2 ? j + 1 : j + 2;
        const int dir = (k - 1) % 3, sgn = k <= 3 ? 1 : -1;
        return (own_m >> j) & 1u ? dr3 : dr3 - (dir == 1 ? sgn * W3 : sgn);
    };
    auto pull_r1 = [&](int j) __attribute__((always_inline)) -> int {
        const int k = j < 2 ? j + 1 : j + 2;
        const int dir = (k - 1) % 3, sgn = k <= 3 ? 1 : -1;
        return (own_m >> j) & 1u ? dr1 : dr1 - (dir == 1 ? sgn * W1 : sgn);
    };

    T smax[3] = {T(0), T(0), T(0)};
    unsigned flags = 0;
    T carryS[M], carryF3[M], carryL[6];
#pragma unroll
    for (int c = 0; c < M; ++c) carryS[c] = carryF3[c] = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) carryL[k] = T(0);

    const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[2], cf.ap[0], cf.ap[1], cf.ap[2]};
    // source rate at a node with moments U whose rate is not in LDS
    auto src_rate = [&](const T *U) __attribute__((always_inline)) -> T {
        if constexpr (SYS == 3) return -arrhenius_rate<T>(P, U[0], reactive_eint<D, T>(U), U[M - 1], nullptr);
        else return T(0);
    };
    // collided population of velocity k read as ks (b of ks) at a node with
    // moments U, flux F along k's axis, omega w and source SY
    auto collide = [&](int k, int ks, const T *fk, const T *U, const T *F, T w, T SY, T *out)
        __attribute__((always_inline)) {
        const T a = ak[k];
        const T bk = ks <= 3 ? cf.bp : cf.bm;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const T feq = k == 0 ? a * U[c] : a * U[c] + bk * F[c];
            T fs = fk[c] - w * (fk[c] - feq);
            if constexpr (SYS == 3)
                if (c == M - 1) fs = fs + cf.hdt * (a * SY);
            out[c] = fs;
        }
    };
    // completes a destination from S = sum of its populations k = 0 .. 5 (the
    // last components Lk for the reactive system) and its -z population F6
    auto finish = [&](unsigned cell, const T *S, const T *Lk, const T *F6) __attribute__((always_inline)) {
        T *fo = fout, *uo = uout;
        int64_t ps = L.pstride, pu = L.pstride;
        opaque(fo, ps);
        opaque(uo, pu);
        T Un[M];
#pragma unroll
        for (int c = 0; c < M; ++c) Un[c] = S[c] + F6[c];
        if constexpr (SYS == 3) {
            const T eint = reactive_eint<D, T>(Un);
            const T z = reactive_solve<T>(P, Un[0], eint, Un[M - 1], cf.hdt);
            const T SY = -arrhenius_rate<T>(P, Un[0], eint, z, nullptr);
            T last[Q];
#pragma unroll
            for (int k = 0; k < 6; ++k) last[k] = Lk[k] + cf.hdt * (ak[k] * SY);
            last[6] = F6[M - 1] + cf.hdt * (ak[6] * SY);
            T sn = last[0];
#pragma unroll
            for (int k = 1; k < Q; ++k) sn = sn + last[k];
            Un[M - 1] = sn;
#pragma unroll
            for (int k = 0; k < Q; ++k) sto_nt(fo + (int64_t)(k * M + M - 1) * ps, cell, last[k]);
#pragma unroll
            for (int c = 0; c < M - 1; ++c) sto_nt(fo + (int64_t)(6 * M + c) * ps, cell, F6[c]);
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) sto_nt(fo + (int64_t)(6 * M + c) * ps, cell, F6[c]);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) sto_nt(uo + (int64_t)c * pu, cell, Un[c]);
        Prim<T> qn;
        primitives<SYS, D, T>(Un, P, qn);
        bool ok = true;
#pragma unroll
        for (int c = 0; c < M; ++c) ok = ok && finite_val<T>(Un[c]);
        flags |= qn.flags | (ok ? 0u : 1u);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T v = max_speed<SYS, T>(d, qn, P);
            if (finite_val<T>(v) && v > smax[d]) smax[d] = v;
        }
    };

    // populations a destination thread needs at source plane s: its own
    // k = 0, 3, 6 and the four in-plane pulls (requested an iteration ahead)
    auto dest_load = [&](int s, T (&fown)[3][M], T (&fpull)[4][M]) __attribute__((always_inline)) {
        if (!live) return;
        const bool mid = s >= za && s < zb;
        const bool need3 = mid || (s == za - 1 && !zlo_wall);
        const bool need6 = mid || (s == zb && !zhi_wall);
        bool rz;
        const int sm = bc_map(s, nz, L.bc[4], L.bc[5], rz);
        const unsigned pb = (unsigned)sm * nxy;
        const T *fi = fin;
        int64_t ps = L.pstride;
        opaque(fi, ps);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            fown[0][c] = mid ? ldo_nt(fi + (int64_t)(0 * M + c) * ps, pb + doff) : T(0);
            fown[1][c] = need3 ? ldo_nt(fi + (int64_t)(3 * M + c) * ps, pb + doff) : T(0);
            fown[2][c] = need6 ? ldo_nt(fi + (int64_t)(6 * M + c) * ps, pb + doff) : T(0);
        }
        if (!mid) return;
        // the +-x pulls read one cell of the line the neighbouring tile
        // reads the rest of at about the same time: they are kept in L2
        // (non-temporal, the line was often gone by the second read: 256^3
        // Euler FP32 read 2.81 GB per step instead of 2.73, at equal time)
        if (!refl_xy) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = j < 2 ? j + 1 : j + 2;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    const T *src = fi + (int64_t)(k * M + c) * ps;
                    fpull[j][c] = k == 1 || k == 4 ? ldo(src, pb + poff[j]) : ldo_nt(src, pb + poff[j]);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = j < 2 ? j + 1 : j + 2;
                const int ks = (refl_m >> j) & 1u ? mirror3(k) : k;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    const T *src = fi + (int64_t)(ks * M + c) * ps;
                    fpull[j][c] = k == 1 || k == 4 ? ldo(src, pb + poff[j]) : ldo_nt(src, pb + poff[j]);
                }
            }
        }
    };
    auto dest_stage = [&](int s, const T (&fown)[3][M], const T (&fpull)[4][M]) __attribute__((always_inline)) {
        if (!live) return;
        const bool mid = s >= za && s < zb;
        const bool need3 = mid || (s == za - 1 && !zlo_wall);
        const bool need6 = mid || (s == zb && !zhi_wall);
        if (!need3 && !need6) return;
        const int sl = (s + 4) & 3;
        T Uo[M], Fz[M];
#pragma unroll
        for (int c = 0; c < M; ++c) Uo[c] = lu[sl][c][dr3];
        Prim<T> qo;
        primitives<SYS, D, T, false>(Uo, P, qo);
        flux<SYS, D, T>(2, Uo, qo, P, Fz);
        const T wo = lw[dr1];
        const T SYo = kRateLds ? lrate[dr1] : src_rate(Uo);
        T F3[M], F6[M];
        collide(3, 3, fown[1], Uo, Fz, wo, SYo, F3);
        collide(6, 6, fown[2], Uo, Fz, wo, SYo, F6);
        // the destination one plane down is complete
        if (s - 1 >= za && s - 1 < zb) finish((unsigned)(s - 1) * nxy + doff, carryS, carryL, F6);
        if (!mid) {
#pragma unroll
            for (int c = 0; c < M; ++c) carryF3[c] = F3[c];
            return;
        }
        const unsigned cell = (unsigned)s * nxy + doff;
        T *fo = fout;
        int64_t ps = L.pstride;
        opaque(fo, ps);
        constexpr int CW = SYS == 3 ? M - 1 : M;  // components final before (2.8)
        T S[M], Lk[6], F[M];
        // k = 0, then the pulls and +z in k order, summed as they come
        collide(0, 0, fown[0], Uo, Fz, wo, SYo, F);
#pragma unroll
        for (int c = 0; c < M; ++c) S[c] = F[c];
#pragma unroll
        for (int c = 0; c < CW; ++c) sto_nt(fo + (int64_t)(0 * M + c) * ps, cell, F[c]);
        Lk[0] = F[M - 1];
#pragma unroll
        for (int k = 1; k < 6; ++k) {
            if (k == 3) {
                // +z: from the plane below, or at a wall this cell's own
                // (mirrored at a reflective one)
                if (s == 0 && zlo_wall) {
#pragma unroll
                    for (int c = 0; c < M; ++c) F[c] = L.bc[4] == 2 ? (c == 3 ? -F6[c] : F6[c]) : F3[c];
                } else {
#pragma unroll
                    for (int c = 0; c < M; ++c) F[c] = carryF3[c];
                }
            } else {
                const int j = k < 3 ? k - 1 : k - 2;
                const int dir = (k - 1) % 3;
                const int ks = (refl_m >> j) & 1u ? mirror3(k) : k;
                const int r3 = pull_r3(j);
                T Us[M], Fs[M];
#pragma unroll
                for (int c = 0; c < M; ++c) Us[c] = lu[sl][c][r3];
                Prim<T> qs;
                primitives<SYS, D, T, false>(Us, P, qs);
                flux<SYS, D, T>(dir, Us, qs, P, Fs);
                collide(k, ks, fpull[j], Us, Fs, lw[pull_r1(j)], kRateLds ? lrate[pull_r1(j)] : src_rate(Us), F);
                if (1 + dir < M && ((refl_m >> j) & 1u)) F[1 + dir] = -F[1 + dir];
            }
#pragma unroll
            for (int c = 0; c < M; ++c) S[c] = S[c] + F[c];
#pragma unroll
            for (int c = 0; c < CW; ++c) sto_nt(fo + (int64_t)(k * M + c) * ps, cell, F[c]);
            Lk[k] = F[M - 1];
        }
        if (s == nz - 1 && zhi_wall) {
            // -z at the top wall: this cell's own (mirrored at a reflective one)
#pragma unroll
            for (int c = 0; c < M; ++c) F[c] = L.bc[5] == 2 ? (c == 3 ? -F3[c] : F3[c]) : F6[c];
            finish(cell, S, Lk, F);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            carryS[c] = S[c];
            carryF3[c] = F3[c];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) carryL[k] = Lk[k];
    };

    // prologue: moments of planes za-3 .. za+1, indicator of za-2 .. za
    for (int p = za - 3; p <= za + 1; ++p) {
        T Ul[UP][M];
        u_load(p, Ul);
        u_store(p, Ul);
        __syncthreads();
        if (p >= za - 1) nu_stage(p - 1);
    }
    T Unext[UP][M];
    u_load(za + 2, Unext);
    T fown[3][M], fpull[4][M];
    if (is_dest) dest_load(za - 1, fown, fpull);
    __syncthreads();
    // FP32 Euler and reactive Euler request the moments of plane s + 4 after
    // the indicator, so that they hold no registers during the collision, and
    // put them into LDS after the next omega (256^3 Euler FP32: 1.19 -> 1.16
    // ms per step; with it advection took 0.33 -> 0.38, Euler FP64 in 16 x 32
    // tiles 3.18 -> 3.33)
    constexpr bool kLate = sizeof(T) == 4 && SYS != 0;
    for (int s = za - 1; s <= zb; ++s) {
        if (!kLate && s + 3 <= zb + 2) {
            u_store(s + 3, Unext);
            if (s + 4 <= zb + 2) u_load(s + 4, Unext);
        }
        w_stage(s);
        if (kLate && s + 3 <= zb + 2) u_store(s + 3, Unext);
        __syncthreads();
        // the collision first: the next plane's populations are requested
        // before the indicator is evaluated, so they arrive during it and the
        // next first phase (indicator first: 1.27 ms per 256^3 Euler FP32
        // step; collision first: 1.195)
        if (is_dest) {
            dest_stage(s, fown, fpull);
            if (s < zb) dest_load(s + 1, fown, fpull);
        }
        if (s + 2 <= zb + 1) nu_stage(s + 2);
        if (kLate && s + 4 <= zb + 2) u_load(s + 4, Unext);
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid < kWave) scalar_update(L, n, cf.dt);
    commit<T>(L, n, smax[0], smax[1], flags, 3, smax[2]);
}

}  // namespace arlbm
