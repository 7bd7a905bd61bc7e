// Per-cell physics of the four balance laws on the device: primitive
// variables, physical fluxes F_j(U), the eigenvalue bound max_r |lambda_j^(r)|
// and the characteristic projections L_j(U_i)(U_a - U_b) entering the
// smoothness indicator (eqs. 2.13-2.14).
//
// Operation order.  In the FP64 build (compiled without contraction) every
// expression keeps the association written here, which follows the textbook
// forms: p = (gamma-1)(E - (rho/2)|u|^2), c = sqrt(gamma p / rho),
// b1 = (gamma-1)/(c c), b2 = (|u|^2/2) b1, left eigenvectors L = R^{-1} for
// right eigenvectors whose acoustic and entropy columns start with 1 and whose
// shear column is the unit tangential momentum.  Matrix-vector products sum
// their non-zero terms in column order.
//
// Reactive Euler (Section 5.4), U = (rho, rho u[, rho v], rho E, rho Y):
// p = (gamma-1)((E - (rho/2)|u|^2) - q rho Y).  With E' = E - q rho Y the
// system is Euler in (rho, m, E') plus the advected rho Y, so its left
// eigenvectors are the Euler rows with a rho Y entry of -q times their energy
// entry, plus the species row (-Y, 0, .., 0, 1); rows in the order u-c,
// entropy, [shear,] species, u+c.
#pragma once

#include <hip/hip_runtime.h>

namespace arlbm {

template <typename T>
struct Phys {
    T gamma, gm1, g, half_g, adv[3], dx, p_floor_t, rho_floor_t, h_dry_t;
    T qh, kr, ti;  // reactive: heat release q, rate constant K, activation temperature T_i
    double h_dry, rho_floor, p_floor;
};

// Division and square root in the storage precision.  FP64: the IEEE
// quotient and root (the oracle's arithmetic).  FP32: the hardware reciprocal
// and root (about 1 ulp), named explicitly, so that every kernel and every
// inlined copy rounds the same way.  Left to the compiler, a quotient it
// speculates or merges (under a select, say) can fall back to the correctly
// rounded sequence in one kernel and not in another, and a one-ulp difference
// in the wave-speed bound then moves every cell of the next step.
template <typename T>
__device__ __forceinline__ T ddiv(T a, T b);
template <>
__device__ __forceinline__ double ddiv<double>(double a, double b) { return a / b; }
template <>
__device__ __forceinline__ float ddiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
template <typename T>
__device__ __forceinline__ T dsqrt(T v);
template <>
__device__ __forceinline__ double dsqrt<double>(double v) { return __builtin_sqrt(v); }
template <>
__device__ __forceinline__ float dsqrt<float>(float v) { return __builtin_amdgcn_sqrtf(v); }

template <typename T>
__device__ __forceinline__ T dabs(T v) { return __builtin_fabs(v); }
template <>
__device__ __forceinline__ float dabs<float>(float v) { return __builtin_fabsf(v); }

template <int SYS, int D>
struct SysInfo {
    static constexpr int M = SYS == 0 ? 1 : (SYS == 1 ? D + 2 : (SYS == 2 ? D + 1 : D + 3));
    static constexpr int Q = 2 * D + 1;
};

template <typename T>
struct Prim {
    T rho, E, p, c, cL;
    T vel[3], mom[3];
    T Z, Y;  // reactive: rho Y and Y
    unsigned flags;
};

// Primitive variables.  Euler: floors enter only the sound speed (a state at
// or below a floor raises the positivity flag).  Shallow water: a cell with
// h <= h_dry (FP64 compare) has zero velocity and momentum flux and the
// acoustic speed in L uses max(h, h_dry); depths within h_dry of zero are dry,
// so only h < -h_dry raises the positivity flag.  kSpeed = false leaves out
// the sound speeds and the flags (what the flux alone needs is the same).
template <int SYS, int D, typename T, bool kSpeed = true>
__device__ __forceinline__ void primitives(const T *U, const Phys<T> &P, Prim<T> &q)
{
    q.flags = 0;
    q.vel[1] = q.vel[2] = T(0);
    q.mom[1] = q.mom[2] = T(0);
    q.Z = q.Y = T(0);
    if constexpr (SYS == 1 || SYS == 3) {
        q.rho = U[0];
        q.E = U[D + 1];
        q.mom[0] = U[1];
        q.vel[0] = ddiv<T>(U[1], q.rho);
        T q2;
        if constexpr (D >= 2) {
            q.mom[1] = U[2];
            q.vel[1] = ddiv<T>(U[2], q.rho);
            q2 = q.vel[0] * q.vel[0] + q.vel[1] * q.vel[1];
            if constexpr (D == 3) {
                q.mom[2] = U[3];
                q.vel[2] = ddiv<T>(U[3], q.rho);
                q2 = q2 + q.vel[2] * q.vel[2];
            }
        } else {
            q2 = q.vel[0] * q.vel[0];
        }
        if constexpr (SYS == 1) {
            q.p = P.gm1 * (q.E - T(0.5) * q.rho * q2);
        } else {
            q.Z = U[D + 2];
            q.Y = ddiv<T>(q.Z, q.rho);
            q.p = P.gm1 * ((q.E - T(0.5) * q.rho * q2) - P.qh * q.Z);
        }
        if constexpr (kSpeed) {
            const bool pok = double(q.p) > P.p_floor, rok = double(q.rho) > P.rho_floor;
            const T pf = pok ? q.p : P.p_floor_t;
            const T rf = rok ? q.rho : P.rho_floor_t;
            if (!(pok && rok)) q.flags |= 2u;
            q.c = dsqrt<T>(ddiv<T>(P.gamma * pf, rf));
            q.cL = q.c;
        } else {
            q.c = q.cL = T(0);
        }
    } else if constexpr (SYS == 2) {
        const T h = U[0];
        q.rho = h;
        const bool wet = double(h) > P.h_dry;
        q.mom[0] = wet ? U[1] : T(0);
        q.vel[0] = wet ? ddiv<T>(U[1], h) : T(0);
        if constexpr (D == 2) {
            q.mom[1] = wet ? U[2] : T(0);
            q.vel[1] = wet ? ddiv<T>(U[2], h) : T(0);
        }
        if constexpr (kSpeed) {
            if (double(h) < -P.h_dry) q.flags |= 2u;
            q.c = dsqrt<T>(P.g * (h > T(0) ? h : T(0)));
            q.cL = dsqrt<T>(P.g * (wet ? h : P.h_dry_t));
        } else {
            q.c = q.cL = T(0);
        }
        q.E = q.p = T(0);
    } else {
        q.rho = U[0];
        q.E = q.p = q.c = q.cL = T(0);
        q.vel[0] = q.mom[0] = T(0);
    }
}

// Physical flux F_dir(U) (Section 5 systems).
template <int SYS, int D, typename T>
__device__ __forceinline__ void flux(int dir, const T *U, const Prim<T> &q, const Phys<T> &P, T *F)
{
    if constexpr (SYS == 0) {
        F[0] = P.adv[dir] * U[0];
    } else if constexpr (SYS == 1 || SYS == 3) {
        const T md = q.mom[dir], vd = q.vel[dir];
        F[0] = md;
#pragma unroll
        for (int i = 0; i < D; ++i) F[1 + i] = (i == dir) ? md * q.vel[i] + q.p : md * q.vel[i];
        F[D + 1] = vd * (q.E + q.p);
        if constexpr (SYS == 3) F[D + 2] = vd * q.Z;
    } else {
        const T md = q.mom[dir];
        const T ph = P.half_g * q.rho * q.rho;
        F[0] = md;
#pragma unroll
        for (int i = 0; i < D; ++i) F[1 + i] = (i == dir) ? md * q.vel[i] + ph : md * q.vel[i];
    }
}

// max_r |lambda_dir^(r)(U)| of eq. (2.19).
template <int SYS, typename T>
__device__ __forceinline__ T max_speed(int dir, const Prim<T> &q, const Phys<T> &P)
{
    if constexpr (SYS == 0) return dabs<T>(P.adv[dir]);
    else return dabs<T>(q.vel[dir]) + q.c;
}

// Indicator of eq. (2.13) for one field: |dp - dm| / (|dm| + |dp| + dx) + |dm| + |dp|.
template <typename T>
__device__ __forceinline__ T theta(T dm, T dp, T dx)
{
    const T adm = dabs<T>(dm), adp = dabs<T>(dp);
    return ddiv<T>(dabs<T>(dp - dm), adm + adp + dx) + adm + adp;
}

// Adds sum_r theta^(r,dir) to nu, with L_dir evaluated at the centre state
// (primitives qc), backward difference dU- = Uc - Um and forward dU+ = Up - Uc.
template <int SYS, int D, typename T>
__device__ __forceinline__ void add_theta(int dir, const Prim<T> &qc, const T *Uc, const T *Um,
                                          const T *Up, const Phys<T> &P, T &nu)
{
    constexpr int M = SysInfo<SYS, D>::M;
    T a[M], b[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        a[c] = Uc[c] - Um[c];
        b[c] = Up[c] - Uc[c];
    }
    const T dx = P.dx;
    if constexpr (SYS == 0) {
        nu = nu + theta<T>(a[0], b[0], dx);
    } else if constexpr ((SYS == 1 || SYS == 3) && D == 3) {
        // 3D: rows u-c, entropy, shear (two tangential directions in
        // increasing order), [species,] u+c; columns rho, m_x, m_y, m_z, E[, rho Y]
        const T cs = qc.c;
        const T q2 = (qc.vel[0] * qc.vel[0] + qc.vel[1] * qc.vel[1]) + qc.vel[2] * qc.vel[2];
        const T b1 = ddiv<T>(P.gm1, cs * cs);
        const T b2 = T(0.5) * q2 * b1;
        const T un = qc.vel[dir];
        const T hb1 = T(0.5) * b1;
        const T r0c0 = T(0.5) * (b2 + ddiv<T>(un, cs)), r0cn = T(-0.5) * (b1 * un + ddiv<T>(T(1), cs));
        const T r3c0 = T(0.5) * (b2 - ddiv<T>(un, cs)), r3cn = T(-0.5) * (b1 * un - ddiv<T>(T(1), cs));
        T r0[3], r3[3], r1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T tang = T(-0.5) * b1 * qc.vel[i];
            r0[i] = i == dir ? r0cn : tang;
            r3[i] = i == dir ? r3cn : tang;
            r1[i] = b1 * qc.vel[i];
        }
        const T r1c0 = T(1) - b2;
        T dm0 = r0c0 * a[0] + r0[0] * a[1] + r0[1] * a[2] + r0[2] * a[3] + hb1 * a[4];
        T dp0 = r0c0 * b[0] + r0[0] * b[1] + r0[1] * b[2] + r0[2] * b[3] + hb1 * b[4];
        T dm1 = r1c0 * a[0] + r1[0] * a[1] + r1[1] * a[2] + r1[2] * a[3] + (-b1) * a[4];
        T dp1 = r1c0 * b[0] + r1[0] * b[1] + r1[1] * b[2] + r1[2] * b[3] + (-b1) * b[4];
        T dm4 = r3c0 * a[0] + r3[0] * a[1] + r3[1] * a[2] + r3[2] * a[3] + hb1 * a[4];
        T dp4 = r3c0 * b[0] + r3[0] * b[1] + r3[1] * b[2] + r3[2] * b[3] + hb1 * b[4];
        if constexpr (SYS == 3) {
            const T zac = -(P.qh * hb1), zen = P.qh * b1;
            dm0 = dm0 + zac * a[5];
            dp0 = dp0 + zac * b[5];
            dm1 = dm1 + zen * a[5];
            dp1 = dp1 + zen * b[5];
            dm4 = dm4 + zac * a[5];
            dp4 = dp4 + zac * b[5];
        }
        const int t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
        const T dm2 = (-qc.vel[t1]) * a[0] + a[1 + t1];
        const T dp2 = (-qc.vel[t1]) * b[0] + b[1 + t1];
        const T dm3 = (-qc.vel[t2]) * a[0] + a[1 + t2];
        const T dp3 = (-qc.vel[t2]) * b[0] + b[1 + t2];
        nu = nu + theta<T>(dm0, dp0, dx);
        nu = nu + theta<T>(dm1, dp1, dx);
        nu = nu + theta<T>(dm2, dp2, dx);
        nu = nu + theta<T>(dm3, dp3, dx);
        if constexpr (SYS == 3) {
            const T dms = (-qc.Y) * a[0] + a[5];
            const T dps = (-qc.Y) * b[0] + b[5];
            nu = nu + theta<T>(dms, dps, dx);
        }
        nu = nu + theta<T>(dm4, dp4, dx);
    } else if constexpr (SYS == 1) {
        const T cs = qc.c;
        T q2;
        if constexpr (D == 2) q2 = qc.vel[0] * qc.vel[0] + qc.vel[1] * qc.vel[1];
        else q2 = qc.vel[0] * qc.vel[0];
        const T b1 = ddiv<T>(P.gm1, cs * cs);
        const T b2 = T(0.5) * q2 * b1;
        const T un = qc.vel[dir];
        const T r0c0 = T(0.5) * (b2 + ddiv<T>(un, cs));
        const T r0cn = T(-0.5) * (b1 * un + ddiv<T>(T(1), cs));
        const T r3c0 = T(0.5) * (b2 - ddiv<T>(un, cs));
        const T r3cn = T(-0.5) * (b1 * un - ddiv<T>(T(1), cs));
        const T hb1 = T(0.5) * b1;
        const T r1c0 = T(1) - b2;
        if constexpr (D == 1) {
            const T r1c1 = b1 * qc.vel[0];
            // rows: u-c, u (entropy), u+c; columns: rho, rho u, E
            const T dm0 = r0c0 * a[0] + r0cn * a[1] + hb1 * a[2];
            const T dp0 = r0c0 * b[0] + r0cn * b[1] + hb1 * b[2];
            const T dm1 = r1c0 * a[0] + r1c1 * a[1] + (-b1) * a[2];
            const T dp1 = r1c0 * b[0] + r1c1 * b[1] + (-b1) * b[2];
            const T dm2 = r3c0 * a[0] + r3cn * a[1] + hb1 * a[2];
            const T dp2 = r3c0 * b[0] + r3cn * b[1] + hb1 * b[2];
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm1, dp1, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
        } else {
            const int t = 1 - dir;
            const T vt = qc.vel[t];
            const T r0ct = T(-0.5) * b1 * vt;  // tangential-momentum column of the acoustic rows
            const T r1c1 = b1 * qc.vel[0], r1c2 = b1 * qc.vel[1];
            // acoustic rows: column 1 is normal for dir 0, tangential for dir 1
            const T r0c1 = dir == 0 ? r0cn : r0ct, r0c2 = dir == 0 ? r0ct : r0cn;
            const T r3c1 = dir == 0 ? r3cn : r0ct, r3c2 = dir == 0 ? r0ct : r3cn;
            const T dm0 = r0c0 * a[0] + r0c1 * a[1] + r0c2 * a[2] + hb1 * a[3];
            const T dp0 = r0c0 * b[0] + r0c1 * b[1] + r0c2 * b[2] + hb1 * b[3];
            const T dm1 = r1c0 * a[0] + r1c1 * a[1] + r1c2 * a[2] + (-b1) * a[3];
            const T dp1 = r1c0 * b[0] + r1c1 * b[1] + r1c2 * b[2] + (-b1) * b[3];
            // shear row: -v_t rho + (rho v_t)
            const T at = dir == 0 ? a[2] : a[1], bt = dir == 0 ? b[2] : b[1];
            const T dm2 = (-vt) * a[0] + at;
            const T dp2 = (-vt) * b[0] + bt;
            const T dm3 = r3c0 * a[0] + r3c1 * a[1] + r3c2 * a[2] + hb1 * a[3];
            const T dp3 = r3c0 * b[0] + r3c1 * b[1] + r3c2 * b[2] + hb1 * b[3];
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm1, dp1, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
            nu = nu + theta<T>(dm3, dp3, dx);
        }
    } else if constexpr (SYS == 3) {
        const T cs = qc.c;
        T q2;
        if constexpr (D == 2) q2 = qc.vel[0] * qc.vel[0] + qc.vel[1] * qc.vel[1];
        else q2 = qc.vel[0] * qc.vel[0];
        const T b1 = ddiv<T>(P.gm1, cs * cs);
        const T b2 = T(0.5) * q2 * b1;
        const T un = qc.vel[dir];
        const T r0c0 = T(0.5) * (b2 + ddiv<T>(un, cs));
        const T r0cn = T(-0.5) * (b1 * un + ddiv<T>(T(1), cs));
        const T r3c0 = T(0.5) * (b2 - ddiv<T>(un, cs));
        const T r3cn = T(-0.5) * (b1 * un - ddiv<T>(T(1), cs));
        const T hb1 = T(0.5) * b1;
        const T r1c0 = T(1) - b2;
        const T zac = -(P.qh * hb1);  // rho Y entry of the acoustic rows
        const T zen = P.qh * b1;      // rho Y entry of the entropy row
        const T mY = -qc.Y;
        if constexpr (D == 1) {
            const T r1c1 = b1 * qc.vel[0];
            // rows: u-c, u (entropy), u (species), u+c; columns: rho, rho u, E, rho Y
            const T dm0 = r0c0 * a[0] + r0cn * a[1] + hb1 * a[2] + zac * a[3];
            const T dp0 = r0c0 * b[0] + r0cn * b[1] + hb1 * b[2] + zac * b[3];
            const T dm1 = r1c0 * a[0] + r1c1 * a[1] + (-b1) * a[2] + zen * a[3];
            const T dp1 = r1c0 * b[0] + r1c1 * b[1] + (-b1) * b[2] + zen * b[3];
            const T dm2 = mY * a[0] + a[3];
            const T dp2 = mY * b[0] + b[3];
            const T dm3 = r3c0 * a[0] + r3cn * a[1] + hb1 * a[2] + zac * a[3];
            const T dp3 = r3c0 * b[0] + r3cn * b[1] + hb1 * b[2] + zac * b[3];
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm1, dp1, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
            nu = nu + theta<T>(dm3, dp3, dx);
        } else {
            const int t = 1 - dir;
            const T vt = qc.vel[t];
            const T r0ct = T(-0.5) * b1 * vt;
            const T r1c1 = b1 * qc.vel[0], r1c2 = b1 * qc.vel[1];
            const T r0c1 = dir == 0 ? r0cn : r0ct, r0c2 = dir == 0 ? r0ct : r0cn;
            const T r3c1 = dir == 0 ? r3cn : r0ct, r3c2 = dir == 0 ? r0ct : r3cn;
            // rows: u-c, entropy, shear, species, u+c; columns: rho, rho u, rho v, E, rho Y
            const T dm0 = r0c0 * a[0] + r0c1 * a[1] + r0c2 * a[2] + hb1 * a[3] + zac * a[4];
            const T dp0 = r0c0 * b[0] + r0c1 * b[1] + r0c2 * b[2] + hb1 * b[3] + zac * b[4];
            const T dm1 = r1c0 * a[0] + r1c1 * a[1] + r1c2 * a[2] + (-b1) * a[3] + zen * a[4];
            const T dp1 = r1c0 * b[0] + r1c1 * b[1] + r1c2 * b[2] + (-b1) * b[3] + zen * b[4];
            const T at = dir == 0 ? a[2] : a[1], bt = dir == 0 ? b[2] : b[1];
            const T dm2 = (-vt) * a[0] + at;
            const T dp2 = (-vt) * b[0] + bt;
            const T dm3 = mY * a[0] + a[4];
            const T dp3 = mY * b[0] + b[4];
            const T dm4 = r3c0 * a[0] + r3c1 * a[1] + r3c2 * a[2] + hb1 * a[3] + zac * a[4];
            const T dp4 = r3c0 * b[0] + r3c1 * b[1] + r3c2 * b[2] + hb1 * b[3] + zac * b[4];
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm1, dp1, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
            nu = nu + theta<T>(dm3, dp3, dx);
            nu = nu + theta<T>(dm4, dp4, dx);
        }
    } else {
        const T cs = qc.cL;
        const T un = qc.vel[dir];
        const T l00 = ddiv<T>(un + cs, T(2) * cs);
        const T l0n = ddiv<T>(T(-1), T(2) * cs);
        const T l20 = ddiv<T>(-(un - cs), T(2) * cs);
        const T l2n = ddiv<T>(T(1), T(2) * cs);
        const T an = a[1 + dir], bn = b[1 + dir];
        const T dm0 = l00 * a[0] + l0n * an;
        const T dp0 = l00 * b[0] + l0n * bn;
        const T dm2 = l20 * a[0] + l2n * an;
        const T dp2 = l20 * b[0] + l2n * bn;
        if constexpr (D == 1) {
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
        } else {
            const int t = 1 - dir;
            const T vt = qc.vel[t];
            const T dm1 = (-vt) * a[0] + a[1 + t];
            const T dp1 = (-vt) * b[0] + b[1 + t];
            nu = nu + theta<T>(dm0, dp0, dx);
            nu = nu + theta<T>(dm1, dp1, dx);
            nu = nu + theta<T>(dm2, dp2, dx);
        }
    }
}

// ---------------------------------------------------------------- reactive --

// exp(x) for the Arrhenius factor, by a fixed algorithm (so that results do
// not depend on the math library): Cody-Waite reduction x = k ln2 + r,
// |r| <= ln2/2, with ln2 split into a head whose trailing bits are zero (k
// times the head is exact) and a tail; the Taylor series of exp(r) in Horner
// form; scaling by 2^k.  FP64 to degree 13 (truncation below 5e-18).  Host
// callable, so that tests pin it against the C library.
__host__ __device__ __forceinline__ double arrhenius_exp(double x)
{
    const double inv_ln2 = 1.44269504088896338700e+00;
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    if (x != x) return x;
    if (x < -746.0) return 0.0;
    if (x > 710.0) return __builtin_huge_val();
    const double k = __builtin_rint(x * inv_ln2);
    const double r = (x - k * ln2_hi) - k * ln2_lo;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return __builtin_ldexp(p, (int)k);
}
// FP32 kinetics: the same in single precision, ln2's head with 9 trailing
// zero bits (k times it is exact for the |k| <= 150 of the float range) and
// the series to degree 7 (truncation below 6e-9, a tenth of an FP32 ulp).
// Against the FP64 exponential, reactive Euler FP32 steps went 2.31 -> 2.22
// ms at 256^3 and 0.266 -> 0.262 ms at 2048^2.
__host__ __device__ __forceinline__ float arrhenius_exp(float x)
{
    const float inv_ln2 = 1.44269502f;
    const float ln2_hi = 0.693145752f;
    const float ln2_lo = 1.42860677e-6f;
    if (x != x) return x;
    if (x < -104.0f) return 0.0f;
    if (x > 89.0f) return __builtin_huge_valf();
    const float k = __builtin_rintf(x * inv_ln2);
    const float r = (x - k * ln2_hi) - k * ln2_lo;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return __builtin_ldexpf(p, (int)k);
}

// Arrhenius rate R = K z exp(-T_i / T), T = p / rho, at rho Y = z with rho
// and e_int = E - (rho/2)|u|^2 fixed; dRdz (if asked) its derivative in z.
template <typename T>
__device__ __forceinline__ T arrhenius_rate(const Phys<T> &P, T rho, T e_int, T z, T *dRdz)
{
    const T p = P.gm1 * (e_int - P.qh * z);
    const bool pok = double(p) > P.p_floor, rok = double(rho) > P.rho_floor;
    const T pf = pok ? p : P.p_floor_t;
    const T rf = rok ? rho : P.rho_floor_t;
    const T Tm = ddiv<T>(pf, rf);
    const T e = arrhenius_exp(-ddiv<T>(P.ti, Tm));
    const T R = (P.kr * z) * e;
    if (dRdz) {
        const T dlog = pok ? ddiv<T>((P.ti * rf) * (P.gm1 * P.qh), pf * pf) : T(0);
        *dRdz = P.kr * e * (T(1) - z * dlog);
    }
    return R;
}

// Internal energy part E - (rho/2)|u|^2 of a reactive state, in the same
// association as the primitive variables.
template <int D, typename T>
__device__ __forceinline__ T reactive_eint(const T *U)
{
    const T u0 = ddiv<T>(U[1], U[0]);
    const T u1 = D >= 2 ? ddiv<T>(U[2], U[0]) : T(0);
    T q2 = u0 * u0 + u1 * u1;
    if constexpr (D == 3) {
        const T u2 = ddiv<T>(U[3], U[0]);
        q2 = q2 + u2 * u2;
    }
    return U[D + 1] - T(0.5) * U[0] * q2;
}

// rho Y component of (2.8): z solves g(z) = (z - B) + (dt/2) R(z) = 0 on the
// bracket [min(0,B), max(0,B)], by Newton steps that fall back to bisection
// when they leave the bracket (or the slope is not positive); stops when a
// Newton step no longer changes z (or a bisection lands on z), or after 40
// iterations.
template <typename T>
__device__ __forceinline__ T reactive_solve(const Phys<T> &P, T rho, T e_int, T B, T half_dt)
{
    T lo = B < T(0) ? B : T(0), hi = B < T(0) ? T(0) : B;
    T z = B;
    for (int it = 0; it < 40; ++it) {
        T dR;
        const T g = (z - B) + half_dt * arrhenius_rate<T>(P, rho, e_int, z, &dR);
        if (g == T(0)) break;
        if (g > T(0)) hi = z;
        else lo = z;
        const T dg = T(1) + half_dt * dR;
        T zn = z - ddiv<T>(g, dg);
        if (dg > T(0) && zn == z) break;  // the Newton step no longer moves z
        if (!(dg > T(0)) || !(zn > lo && zn < hi)) zn = T(0.5) * (lo + hi);
        if (zn == z) break;
        z = zn;
    }
    return z;
}

}  // namespace arlbm
