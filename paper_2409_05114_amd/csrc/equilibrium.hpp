// Entropic equilibrium of the RD3Q81 model on the GPU (Sec. III of
// Atif et al., arXiv:2409.05114).
//
// f_i^eq = rho w_i exp(mu + zeta.c_i + gamma c_i^2): the minimiser of
// H = <f, log(f/w) - 1> with the conserved moments of Eq. (conslaws).  The
// five multipliers lambda = (mu, zeta_x, zeta_y, zeta_z, gamma) solve the
// 5x5 Newton system of Sec. III, J dlambda = m - <g, P>, with
// P_i = (1, c_i, c_i^2), g_i = w_i exp(lambda.P_i) per unit density,
// J = <g, P P^T> and m = (1, u, u^2 + 3 theta).
//
// Shell factorisation.  Within a shell w_i exp(mu + gamma c_i^2) is one
// number, and the sum of exp(zeta.c_i) over the shell's sign/permutation
// orbit factorises into products of cosh and sinh of k zeta_a.  With
// X_a = exp(zeta_a / 2), every exp(k zeta_a) is a power X_a^(2k), so one
// evaluation of all fifteen Jacobian entries costs 5 exponentials, a few
// reciprocals and ~300 multiply-adds instead of 81 exponentials.  The
// per-direction equilibrium is the shell factor times three powers.
//
// Safeguard.  Far from the solution a Newton step is scaled down so that no
// multiplier moves by more than 1 (a step cap, which needs no extra state;
// from the Maxwellian initial guess it converges wherever a backtracking
// line search on the convex dual does).  Near the solution every step is a
// full Newton step.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm81 {

template <class T>
struct Math;

template <>
struct Math<double> {
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static constexpr double TOL = 1e-9;  // step size that ends the iteration
    static constexpr int MAXIT = 40;
};

template <>
struct Math<float> {
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
    static __device__ __forceinline__ float log(float x) { return __logf(x); }
    static __device__ __forceinline__ float rcp(float x) {
        return __builtin_amdgcn_rcpf(x);
    }
    static constexpr float TOL = 3e-5f;
    static constexpr int MAXIT = 20;
};

// Visit every shell but the rest shell with the quantities that depend on
// the multipliers: f(IC<S>, px, mx, py, my, pz, mz, e) with p = X_a^n and
// m = X_a^-n for n = SHELL_N[S] (so p = exp(k zeta_a) for the per-component
// magnitude k = n / 2 of the shell) and e = exp(mu + gamma c_S^2).  Shells are
// visited in increasing n so that the powers are built by repeated
// multiplication and each is live only while it is needed.  Returns
// exp(mu), the rest shell's factor.
template <class T, class F>
__device__ __forceinline__ T visit_shells(const T lam[5], F &&f) {
    const T A = Math<T>::exp(lam[0]);
    const T g1 = Math<T>::exp(T(0.25) * lam[4]);  // exp(gamma c^2) = g1^(4 c^2)
    const T x1 = Math<T>::exp(T(0.5) * lam[1]);
    const T y1 = Math<T>::exp(T(0.5) * lam[2]);
    const T z1 = Math<T>::exp(T(0.5) * lam[3]);
    const T xm1 = Math<T>::rcp(x1), ym1 = Math<T>::rcp(y1),
            zm1 = Math<T>::rcp(z1);
    const T g2 = g1 * g1, g3 = g2 * g1, g4 = g2 * g2, g8 = g4 * g4;
    // n = 1: BCC-1/2
    f(IC<7>{}, x1, xm1, y1, ym1, z1, zm1, A * g3);
    // n = 2: SC-1, FCC-1, BCC-1
    const T x2 = x1 * x1, y2 = y1 * y1, z2 = z1 * z1;
    const T xm2 = xm1 * xm1, ym2 = ym1 * ym1, zm2 = zm1 * zm1;
    f(IC<1>{}, x2, xm2, y2, ym2, z2, zm2, A * g4);
    f(IC<5>{}, x2, xm2, y2, ym2, z2, zm2, A * g8);
    f(IC<8>{}, x2, xm2, y2, ym2, z2, zm2, A * (g8 * g4));
    // n = 3: BCC-3/2
    const T g16 = g8 * g8;
    {
        const T x3 = x2 * x1, y3 = y2 * y1, z3 = z2 * z1;
        const T xm3 = xm2 * xm1, ym3 = ym2 * ym1, zm3 = zm2 * zm1;
        f(IC<9>{}, x3, xm3, y3, ym3, z3, zm3, A * ((g16 * g8) * g3));
    }
    // n = 4: SC-2, FCC-2
    const T x4 = x2 * x2, y4 = y2 * y2, z4 = z2 * z2;
    const T xm4 = xm2 * xm2, ym4 = ym2 * ym2, zm4 = zm2 * zm2;
    const T g32 = g16 * g16;
    f(IC<2>{}, x4, xm4, y4, ym4, z4, zm4, A * g16);
    f(IC<6>{}, x4, xm4, y4, ym4, z4, zm4, A * g32);
    // n = 5: BCC-5/2
    const T g64 = g32 * g32;
    {
        const T x5 = x4 * x1, y5 = y4 * y1, z5 = z4 * z1;
        const T xm5 = xm4 * xm1, ym5 = ym4 * ym1, zm5 = zm4 * zm1;
        f(IC<10>{}, x5, xm5, y5, ym5, z5, zm5, A * ((g64 * g8) * g3));
    }
    // n = 6: SC-3
    {
        const T x6 = x4 * x2, y6 = y4 * y2, z6 = z4 * z2;
        const T xm6 = xm4 * xm2, ym6 = ym4 * ym2, zm6 = zm4 * zm2;
        f(IC<3>{}, x6, xm6, y6, ym6, z6, zm6, A * (g32 * g4));
    }
    // n = 8: SC-4
    {
        const T x8 = x4 * x4, y8 = y4 * y4, z8 = z4 * z4;
        const T xm8 = xm4 * xm4, ym8 = ym4 * ym4, zm8 = zm4 * zm4;
        f(IC<4>{}, x8, xm8, y8, ym8, z8, zm8, A * g64);
    }
    return A;
}

// X^(2 c) for a doubled velocity component a = 2c in {-n, 0, n}, given
// p = X^n and m = X^-n.
template <int A_, class T>
__device__ __forceinline__ T pick(T p, T m) {
    if constexpr (A_ == 0)
        return T(1);
    else if constexpr (A_ > 0)
        return p;
    else
        return m;
}

// Moments <g, P P^T> of the exponential family, per unit density.
template <class T>
struct Sums {
    T t0, tx, ty, tz, t2;       // <g, P>: the conserved moments
    T txx, tyy, tzz, txy, txz, tyz, t2x, t2y, t2z, t4;
};

template <class T>
__device__ __forceinline__ Sums<T> family_sums(const T lam[5]) {
    Sums<T> s{};
    const T A = visit_shells(lam, [&](auto S_, T px, T pmx, T py, T pmy, T pz,
                                      T pmz, T e) {
        constexpr int S = decltype(S_)::value;
        constexpr T k = T(0.5 * SHELL_N[S]);  // per-component magnitude
        constexpr T k2 = k * k;
        constexpr T c2 = T(0.25 * SHELL_C2X4[S]);
        const T g = T(shell_weight(S)) * e;
        // 2 cosh(k zeta_a) and 2 sinh(k zeta_a)
        const T cx = px + pmx, sx = px - pmx;
        const T cy = py + pmy, sy = py - pmy;
        const T cz = pz + pmz, sz = pz - pmz;
        T m0, mx, my, mz, mxx, myy, mzz, mxy, mxz, myz;
        if constexpr (SHELL_KIND[S] == SC) {
            // +-k e_a
            m0 = cx + cy + cz;
            mx = k * sx;
            my = k * sy;
            mz = k * sz;
            mxx = k2 * cx;
            myy = k2 * cy;
            mzz = k2 * cz;
            mxy = mxz = myz = T(0);
        } else if constexpr (SHELL_KIND[S] == FCC) {
            // k(+-e_a +- e_b), a < b
            const T cyz = cy + cz, cxz = cx + cz, cxy = cx + cy;
            m0 = cx * cyz + cy * cz;
            mx = k * sx * cyz;
            my = k * sy * cxz;
            mz = k * sz * cxy;
            mxx = k2 * cx * cyz;
            myy = k2 * cy * cxz;
            mzz = k2 * cz * cxy;
            mxy = k2 * sx * sy;
            mxz = k2 * sx * sz;
            myz = k2 * sy * sz;
        } else {
            // h(+-1, +-1, +-1)
            const T cyz = cy * cz;
            m0 = cx * cyz;
            mx = k * sx * cyz;
            my = k * sy * cx * cz;
            mz = k * sz * cx * cy;
            mxx = myy = mzz = k2 * m0;
            mxy = k2 * sx * sy * cz;
            mxz = k2 * sx * sz * cy;
            myz = k2 * sy * sz * cx;
        }
        s.t0 += g * m0;
        s.tx += g * mx;
        s.ty += g * my;
        s.tz += g * mz;
        s.txx += g * mxx;
        s.tyy += g * myy;
        s.tzz += g * mzz;
        if constexpr (SHELL_KIND[S] != SC) {
            s.txy += g * mxy;
            s.txz += g * mxz;
            s.tyz += g * myz;
        }
        const T gc2 = g * c2;
        s.t2x += gc2 * mx;
        s.t2y += gc2 * my;
        s.t2z += gc2 * mz;
        s.t4 += (gc2 * c2) * m0;
    });
    s.t0 += T(shell_weight(0)) * A;
    s.t2 = s.txx + s.tyy + s.tzz;
    return s;
}

// Solve J d = r for the symmetric positive definite 5x5 J (LDL^T).
// Returns false when a pivot is not positive.
template <class T>
__device__ __forceinline__ bool solve5(const Sums<T> &s, const T r[5], T d[5]) {
    T a[5][5];
    a[0][0] = s.t0;
    a[1][0] = s.tx;  a[1][1] = s.txx;
    a[2][0] = s.ty;  a[2][1] = s.txy; a[2][2] = s.tyy;
    a[3][0] = s.tz;  a[3][1] = s.txz; a[3][2] = s.tyz; a[3][3] = s.tzz;
    a[4][0] = s.t2;  a[4][1] = s.t2x; a[4][2] = s.t2y; a[4][3] = s.t2z;
    a[4][4] = s.t4;
    T L[5][5], D[5], iD[5];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        T dj = a[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k] * D[k];
        ok = ok && (dj > T(0));
        D[j] = dj;
        iD[j] = Math<T>::rcp(dj);
#pragma unroll
        for (int i = j + 1; i < 5; ++i) {
            T v = a[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k] * D[k];
            L[i][j] = v * iD[j];
        }
    }
    T y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        T v = r[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v;
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        T v = y[i] * iD[i];
#pragma unroll
        for (int k = i + 1; k < 5; ++k) v -= L[k][i] * d[k];
        d[i] = v;
    }
    return ok;
}

// Newton iteration for the multipliers per unit density.  Inputs: velocity
// u, specific energy e = u^2 + 3 theta and theta (for the initial guess).
// Initial guess: the multipliers of the continuous Maxwellian at (u, theta)
// relative to the lattice weights, mu = -(3/2) ln(theta/theta0) -
// u^2/(2 theta), zeta = u / theta, gamma = (1/theta0 - 1/theta)/2; their
// Taylor series at u = 0 is the series of Appendix B.
// Returns the number of Newton directions computed, or -1 when the cap was
// reached or the Jacobian was not positive definite.
template <class T>
__device__ __forceinline__ int solve_multipliers(T ux, T uy, T uz, T e, T theta,
                                                 T lam[5]) {
    const T it_ = Math<T>::rcp(theta);
    const T usq = ux * ux + uy * uy + uz * uz;
    lam[0] = T(-1.5) * Math<T>::log(theta * T(1.0 / THETA0)) - T(0.5) * usq * it_;
    lam[1] = ux * it_;
    lam[2] = uy * it_;
    lam[3] = uz * it_;
    lam[4] = T(0.5 / THETA0) - T(0.5) * it_;
    T d[5];
    int status = -1;
    for (int it = 0; it < Math<T>::MAXIT; ++it) {
        const Sums<T> s = family_sums(lam);
        const T r[5] = {T(1) - s.t0, ux - s.tx, uy - s.ty, uz - s.tz,
                        e - s.t2};
        if (!solve5(s, r, d)) break;
        T dmax = T(0);
#pragma unroll
        for (int a = 0; a < 5; ++a) dmax = fmax(dmax, fabs(d[a]));
        if (!(dmax == dmax)) break;  // NaN
        // far from the solution, limit the step to 1 in every multiplier
        const T sc = dmax > T(1) ? Math<T>::rcp(dmax) : T(1);
#pragma unroll
        for (int a = 0; a < 5; ++a) lam[a] += sc * d[a];
        if (dmax < Math<T>::TOL) {
            status = it + 1;
            break;
        }
    }
    return status;
}

}  // namespace lbm81
