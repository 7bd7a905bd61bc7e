// One time step of the method on a D3Q7 lattice (Section 2.3 with d = 3:
// e_0 = 0, e_j the unit vectors, e_{j+3} = -e_j), as three cell-parallel
// passes.  The moments U = sum_k f_k (eq. 2.3) of the current state are kept
// in the ping-pong buffer u[n&1]: written by the initialisation and by each
// step for the next one.
//
//   k3_nu       indicator nu (eqs. 2.13-2.14) on the lattice padded by one
//               ghost cell per side, from U with the boundary index maps;
//   k3_omega    box sum over {-1,0,1}^3 (eq. 2.15, z outermost, x innermost)
//               and omega (eq. 2.16) of every cell;
//   k3_collide  per destination cell x and velocity k: collision at the
//               source node x - e_k (eqs. 2.2, 2.5, 2.6, 2.20), pull, the
//               moment update (2.8) and the second half source; the moments
//               of the new populations into u[(n+1)&1]; the next step's
//               wave-speed bounds (2.19) reduced across the wave and
//               committed with one atomic max per wave and direction.
//
// Threads walk cells in column tiles marching in z (x fastest within a tile
// row), so every plane access is coalesced (shifts by e_k move whole rows or
// planes) and the neighbours a cell reads were fetched by the same XCD just
// before.  Waves whose cells all lie one cell inside the lattice skip the
// boundary maps and ghost rules.  A population pulled from a
// ghost position outside a non-periodic face is the destination's own
// collided population: the same velocity (transmissive) or the mirrored one
// with the normal momentum negated (reflective), as in the 1D/2D kernels.
#pragma once

#include "step.hpp"

namespace arlbm {

// Cell index of (i, j, l) and the padded index of (i, j, l), i in [-1, nx].
__device__ __forceinline__ int64_t cell3(const LatticeDesc &L, int i, int j, int l)
{
    return ((int64_t)l * L.ny + j) * L.nx + i;
}
__device__ __forceinline__ int64_t pad3(const LatticeDesc &L, int i, int j, int l)
{
    return ((int64_t)(l + 1) * (L.ny + 2) + (j + 1)) * (L.nx + 2) + (i + 1);
}

// Cells of a 3D pass in XCD-contiguous slabs.  Blocks are dealt round-robin
// over the 8 XCDs, so block b works on slab b mod 8 (cells [s S, (s+1) S),
// S = ceil(total / 8)) and strides over it with the slab's other blocks: each
// XCD sweeps one contiguous range, and the neighbours a cell reads (a row or
// a plane away) were mostly fetched into that XCD's L2 shortly before.  The
// grid is a multiple of 8 blocks.  Every thread of a wave runs the same
// number of iterations (lim is a whole number of strides past begin).
struct Slab {
    int64_t begin, end, first, step, lim;
};
__device__ __forceinline__ Slab slab_of(int64_t total)
{
    Slab r;
    const int b = blockIdx.x, nbx = gridDim.x >> 3;
    const int64_t S = (total + 7) / 8;
    r.begin = (int64_t)(b & 7) * S;
    r.end = r.begin + S < total ? r.begin + S : total;
    r.step = (int64_t)nbx * blockDim.x;
    r.first = r.begin + (int64_t)(b >> 3) * blockDim.x + threadIdx.x;
    const int64_t len = r.end > r.begin ? r.end - r.begin : 0;
    r.lim = r.begin + (len + r.step - 1) / r.step * r.step;
    return r;
}

// Column tiles of TX x (1024 / TX) cells marching in z.  An iteration index
// g maps to (tile, z, offset in the tile) with the offset fastest, then z,
// then the tile: cells a plane apart are 1024 iterations apart and those a
// row apart TX, so a cell's neighbours are fetched by the same XCD at about
// the same time, and the working set of a tile column (a few planes of 1024
// cells) stays in L2 where a whole lattice plane would not.  Tiles
// overhanging the lattice leave their outside cells idle.  The indicator pass
// walks the lattice padded by one cell (nx + 2 wide), where a 256-wide tile
// would leave most of a second tile idle.  Measured (ms per 256^3 FP32 Euler
// step): all passes 64 x 16 / 128 x 8 / 256 x 4: 1.75 / 1.70 / 1.69; collide
// 1.30 ms at 128 x 8 and 1.23 at 256 x 4, indicator 0.31 and 0.36; with the
// collide and relaxation passes at 256 x 4, the indicator at 128 x 8 / 64 x
// 16: 1.645 / 1.638 (FP64 3.264 / 3.236); the relaxation no better at 128 or
// 64 wide.
constexpr int kTileW = 256, kTileWNu = 64, kTileWOmega = 256;  // tile widths: collide, indicator, relaxation
constexpr int kTileShift = 10;
template <int TX>
struct Tiling {
    static constexpr int kTY = (1 << kTileShift) / TX;
    static_assert(TX * kTY == 1 << kTileShift, "tile size");
    int nx, ny, nz, ntx;
    int64_t total;
};
template <int TX>
__device__ __forceinline__ Tiling<TX> tiling_of(int nx, int ny, int nz)
{
    constexpr int kTY = Tiling<TX>::kTY;
    Tiling<TX> t;
    t.nx = nx;
    t.ny = ny;
    t.nz = nz;
    t.ntx = (nx + TX - 1) / TX;
    const int nty = (ny + kTY - 1) / kTY;
    t.total = ((int64_t)t.ntx * nty * nz) << kTileShift;
    return t;
}
template <int TX>
__device__ __forceinline__ bool tile_cell(const Tiling<TX> &t, int64_t g, int &i, int &j, int &l)
{
    const int o = (int)(g & ((1 << kTileShift) - 1));
    const unsigned rest = (unsigned)(g >> kTileShift);
    const unsigned tile = rest / (unsigned)t.nz;
    l = (int)(rest - tile * (unsigned)t.nz);
    const unsigned ty = tile / (unsigned)t.ntx;
    i = (int)(tile - ty * (unsigned)t.ntx) * TX + (o & (TX - 1));
    j = (int)ty * Tiling<TX>::kTY + (o / TX);
    return i < t.nx && j < t.ny;
}

// U at any position within two cells of the lattice: each axis through its
// boundary index map; reflective maps negate that axis's momentum.
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

template <int SYS, typename T>
__global__ __launch_bounds__(kBlock) void k3_nu(LatticeDesc L, int64_t iter)
{
    constexpr int M = SysInfo<SYS, 3>::M;
    const Phys<T> P = make_phys<T>(L);
    const T *u = (const T *)L.u[(iter - L.iter0) & 1];
    T *nu_out = (T *)L.nu3;
    const int px = L.nx + 2, py = L.ny + 2;
    const int64_t npad = (int64_t)px * py * (L.nz + 2);
    const auto tl = tiling_of<kTileWNu>(px, py, L.nz + 2);
    const Slab sl = slab_of(tl.total);
    for (int64_t g = sl.first; g < sl.end; g += sl.step) {
        int i, j, l;
        if (!tile_cell(tl, g, i, j, l)) continue;
        const int64_t gp = ((int64_t)l * py + j) * px + i;  // padded index
        --i;
        --j;
        --l;
        // cells whose neighbours are all inside the lattice read them
        // directly; a wave with any other cell takes the boundary maps
        const bool inner = i >= 1 && i <= L.nx - 2 && j >= 1 && j <= L.ny - 2 && l >= 1 && l <= L.nz - 2;
        auto cell_nu = [&](auto inner_tag) __attribute__((always_inline)) {
            constexpr bool kInner = decltype(inner_tag)::value;
            const int64_t ps = L.pstride;
            const int64_t c0 = kInner ? cell3(L, i, j, l) : 0;
            auto ld = [&](int di, int dj, int dl, T *U) __attribute__((always_inline)) {
                if constexpr (kInner) {
                    const int64_t cn = c0 + ((int64_t)dl * L.ny + dj) * L.nx + di;
#pragma unroll
                    for (int c = 0; c < M; ++c) U[c] = u[(int64_t)c * ps + cn];
                } else {
                    load_U3<M, T>(L, u, i + di, j + dj, l + dl, SYS != 0, U);
                }
            };
            T Uc[M], Um[M], Up[M];
            ld(0, 0, 0, Uc);
            Prim<T> qc;
            primitives<SYS, 3, T>(Uc, P, qc);
            T nu = T(0);
#pragma unroll
            for (int dir = 0; dir < 3; ++dir) {
                const int ox = dir == 0, oy = dir == 1, oz = dir == 2;
                ld(-ox, -oy, -oz, Um);
                ld(ox, oy, oz, Up);
                add_theta<SYS, 3, T>(dir, qc, Uc, Um, Up, P, nu);
            }
            nu_out[gp] = nu;
        };
        if (__ballot(!inner) == 0ull)
            cell_nu(Phase<1>());
        else
            cell_nu(Phase<0>());
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k3_omega(LatticeDesc L, int64_t iter)
{
    const T *nu = (const T *)L.nu3;
    const int64_t npad = (int64_t)(L.nx + 2) * (L.ny + 2) * (L.nz + 2);
    T *w_out = (T *)L.nu3 + npad;
    const T wfix = T(L.omega_fixed);
    const auto tl = tiling_of<kTileWOmega>(L.nx, L.ny, L.nz);
    const Slab sl = slab_of(tl.total);
    for (int64_t g = sl.first; g < sl.end; g += sl.step) {
        int i, j, l;
        if (!tile_cell(tl, g, i, j, l)) continue;
        const int64_t c = cell3(L, i, j, l);
        T w;
        if (L.omega_fixed_on) {
            w = wfix;
        } else {
            T nt = T(0);
#pragma unroll
            for (int kl = -1; kl <= 1; ++kl)
#pragma unroll
                for (int kj = -1; kj <= 1; ++kj)
#pragma unroll
                    for (int ki = -1; ki <= 1; ++ki) nt = nt + nu[pad3(L, i + ki, j + kj, l + kl)];
            w = omega_of<T>(nt);
        }
        w_out[c] = w;
        if (L.omega_on) ((T *)L.omega)[c] = w;
    }
}

template <int SYS, typename T>
__global__ __launch_bounds__(kBlock) void k3_collide(LatticeDesc L, int64_t iter)
{
    constexpr int D = 3, M = SysInfo<SYS, 3>::M, Q = 7;
    const int64_t n = iter - L.iter0;
    const bool first_thread = blockIdx.x == 0 && threadIdx.x == 0;
    const bool first_wave = blockIdx.x == 0 && threadIdx.x < kWave;
    const T *fin = (const T *)L.f[n & 1];
    T *fout = (T *)L.f[(n + 1) & 1];
    const int64_t ps = L.pstride;
    const T *u = (const T *)L.u[n & 1];
    T *uout = (T *)L.u[(n + 1) & 1];
    if (L.sc->t[n % 3] >= L.t_stop) {  // null step: the state is at the stop time
        const Slab sl = slab_of(L.plane);
        for (int64_t c = sl.first; c < sl.end; c += sl.step) {
            for (int p = 0; p < Q * M; ++p) fout[(int64_t)p * ps + c] = fin[(int64_t)p * ps + c];
            for (int p = 0; p < M; ++p) uout[(int64_t)p * ps + c] = u[(int64_t)p * ps + c];
        }
        if (first_wave) null_scalars(L, n);
        return;
    }
    Coefs<T> cf;
    if (!step_coefs<D, T>(L, n, cf)) {
        if (first_thread) flag_degenerate(L, n);
        return;
    }
    const Phys<T> P = make_phys<T>(L);
    const T *wv = (const T *)L.nu3 + (int64_t)(L.nx + 2) * (L.ny + 2) * (L.nz + 2);
    const T ak[Q] = {cf.a0, cf.ap[0], cf.ap[1], cf.ap[2], cf.ap[0], cf.ap[1], cf.ap[2]};
    T smax[3] = {T(0), T(0), T(0)};
    unsigned flags = 0;
    // every lane of a wave runs the same number of iterations (the reduction
    // below needs the whole wave)
    const auto tl = tiling_of<kTileW>(L.nx, L.ny, L.nz);
    const Slab sl = slab_of(tl.total);
    for (int64_t g = sl.first; g < sl.lim; g += sl.step) {
        int i = 0, j = 0, l = 0;
        const bool live = g < sl.end && tile_cell(tl, g, i, j, l);
        if (!live) i = j = l = 0;
        const int64_t c = cell3(L, i, j, l);
        const int pos[3] = {i, j, l};
        const int ext[3] = {L.nx, L.ny, L.nz};
        T Fk[Q][M];
        // a wave whose cells all pull from inside the lattice skips the ghost rules
        const bool inner = live && i >= 1 && i <= L.nx - 2 && j >= 1 && j <= L.ny - 2 && l >= 1 && l <= L.nz - 2;
        auto pull = [&](auto inner_tag) __attribute__((always_inline)) {
        constexpr bool kInner = decltype(inner_tag)::value;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            // velocity k: 0 rest; 1..3 +x,+y,+z; 4..6 -x,-y,-z
            const int dir = k == 0 ? 0 : (k - 1) % 3;
            const int sgn = k == 0 ? 0 : (k <= 3 ? 1 : -1);
            int src[3] = {i, j, l};
            src[dir] -= sgn;
            int ks = k;
            bool negate = false;
            if (!kInner && k != 0 && (src[dir] < 0 || src[dir] >= ext[dir])) {
                const int side = src[dir] < 0 ? 2 * dir : 2 * dir + 1;
                const int b = L.bc[side];
                if (b == 0) {
                    src[dir] = src[dir] < 0 ? ext[dir] - 1 : 0;  // periodic wrap
                } else {
                    src[dir] = pos[dir];  // the destination's own collided population
                    if (b == 2) {
                        ks = k <= 3 ? k + 3 : k - 3;
                        negate = true;
                    }
                }
            }
            const int64_t s = cell3(L, src[0], src[1], src[2]);
            T U[M];
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) U[c2] = u[(int64_t)c2 * ps + s];
            Prim<T> q;
            primitives<SYS, D, T>(U, P, q);
            // a mirrored velocity keeps its axis, so a_k and the flux
            // direction are those of k; only the sign of b_k follows ks
            T F[M];
            if (k != 0) flux<SYS, D, T>(dir, U, q, P, F);
            const T w = wv[s];
            const T a = k == 0 ? cf.a0 : cf.ap[dir];
            const T bk = ks <= 3 ? cf.bp : cf.bm;
            T SY = T(0);
            if constexpr (SYS == 3) SY = -arrhenius_rate<T>(P, U[0], reactive_eint<D, T>(U), U[M - 1], nullptr);
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) {
                const T fk = fin[(int64_t)(ks * M + c2) * ps + s];
                const T feq = k == 0 ? a * U[c2] : a * U[c2] + bk * F[c2];
                T fs = fk - w * (fk - feq);
                if constexpr (SYS == 3)
                    if (c2 == M - 1) fs = fs + cf.hdt * (a * SY);
                Fk[k][c2] = (negate && c2 == 1 + dir) ? -fs : fs;
            }
        }
        };
        if (__ballot(!inner) == 0ull)
            pull(Phase<1>());
        else
            pull(Phase<0>());
        // moments (2.8) and the second half source
        T sumF[M];
#pragma unroll
        for (int c2 = 0; c2 < M; ++c2) {
            T sf = Fk[0][c2];
#pragma unroll
            for (int k = 1; k < Q; ++k) sf = sf + Fk[k][c2];
            sumF[c2] = sf;
        }
        if constexpr (SYS == 3) {
            const T eint = reactive_eint<D, T>(sumF);
            const T z = reactive_solve<T>(P, sumF[0], eint, sumF[M - 1], cf.hdt);
            const T SY = -arrhenius_rate<T>(P, sumF[0], eint, z, nullptr);
#pragma unroll
            for (int k = 0; k < Q; ++k) Fk[k][M - 1] = Fk[k][M - 1] + cf.hdt * (ak[k] * SY);
        }
        T Un[M];
#pragma unroll
        for (int c2 = 0; c2 < M; ++c2) {
            T sn = Fk[0][c2];
#pragma unroll
            for (int k = 1; k < Q; ++k) sn = sn + Fk[k][c2];
            Un[c2] = sn;
        }
        if (live) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
#pragma unroll
                for (int c2 = 0; c2 < M; ++c2) fout[(int64_t)(k * M + c2) * ps + c] = Fk[k][c2];
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) uout[(int64_t)c2 * ps + c] = Un[c2];
            Prim<T> qn;
            primitives<SYS, D, T>(Un, P, qn);
            bool fin_ok = true;
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) fin_ok = fin_ok && finite_val<T>(Un[c2]);
            flags |= qn.flags | (fin_ok ? 0u : 1u);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T v = max_speed<SYS, T>(d, qn, P);
                if (finite_val<T>(v) && v > smax[d]) smax[d] = v;
            }
        }
    }
    if (first_wave) scalar_update(L, n, cf.dt);
    commit<T>(L, n, smax[0], smax[1], flags, 3, smax[2]);
}

}  // namespace arlbm
