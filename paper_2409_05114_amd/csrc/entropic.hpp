// The entropic step with two lanes per site (Sec. II, Eq. delH): its
// kernel, the FP64 and FP32 ln(1 + y) / h(y) routines it evaluates, and the
// launcher of the entropic step.  Included only by the entropic translation
// units (kernels_<storage>_ent.hip), so that the plain step kernels'
// sources do not change with it.
#pragma once

#include "entropic_launch.hpp"
#include "kernels.hpp"

namespace lbm81 {

// l = ln(1 + y) and h = (1 + y) ln(1 + y) - y (hfun) together in FP64, for
// y > -1 (h = 1 at y = -1), lean in registers and without branches, for the
// FP64 split step, which evaluates them for many directions per pass.
//  * ln(1 + y): u = 1 + y rounded, corrected for the rounding of u to second
//    order, ln u + c - c^2 / 2 with c = (y - (u - 1)) / u (the first-order
//    form is Goldberg's, "What every computer scientist should know about
//    floating-point arithmetic", 1991); ln u = e ln 2 + ln m for u = m 2^e
//    with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) = 2 (s + s^3/3 + ... +
//    s^23/23), s = (m - 1) / (m + 1), |s| <= 0.1716 (omitted terms below
//    1e-18 relative); ln 2 split into a head of 40 bits (e ln2_hi exact) and
//    a tail.
//  * h: where e = 0 (m = u), ln(1 + y) - y = 2 s^3 P - (u - 1)(s + c) - c^2/2
//    with 2 s^3 P the series' tail, a sum without cancellation (the closed
//    form (1 + y) l - y cancels to order y^2), and h = (l - y) + y l;
//    elsewhere (|y| > 0.29) the closed form.
//  * divisions by reciprocals: the correction term, itself below one ulp of
//    the result, takes the hardware reciprocal of u as it is; s takes the
//    reciprocal of m + 1 (in [1.7, 2.5]) refined by two Newton steps and one
//    residual correction of the quotient.
// Checked against extended precision on 1.8e7 arguments from -1 + 2^-40 to
// e^40: l within 5e-16 and h within 2e-15 relative.
__device__ __forceinline__ void lnh_f64(double y, double &l, double &h) {
    const double u = 1.0 + y, um = u - 1.0;
    const double c = (y - um) * __builtin_amdgcn_rcp(u);
    int e;
    double m = frexp(u, &e);  // m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double dn = m + 1.0, nm = m - 1.0;
    double r = __builtin_amdgcn_rcp(dn);
    r = fma(fma(-dn, r, 1.0), r, r);
    r = fma(fma(-dn, r, 1.0), r, r);
    const double s0 = nm * r;
    const double s = fma(fma(-dn, s0, nm), r, s0);
    const double t = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, t, 1.0 / 21.0);
    p = fma(p, t, 1.0 / 19.0);
    p = fma(p, t, 1.0 / 17.0);
    p = fma(p, t, 1.0 / 15.0);
    p = fma(p, t, 1.0 / 13.0);
    p = fma(p, t, 1.0 / 11.0);
    p = fma(p, t, 1.0 / 9.0);
    p = fma(p, t, 1.0 / 7.0);
    p = fma(p, t, 1.0 / 5.0);
    p = fma(p, t, 1.0 / 3.0);
    const double q = 2.0 * s * t * p;  // 2 s^3 P
    const double lm = 2.0 * s + q;
    // ln 2 to 40 fractional bits (0x1.62e42fefa2p-1), and the rest
    constexpr double LN2_HI = 0.6931471805592082;
    constexpr double LN2_LO = 7.371002565167799e-13;
    const double de = double(e);
    const double c2 = fma(-0.5 * c, c, c);
    l = fma(de, LN2_HI, (lm + fma(de, LN2_LO, c2)));
    const double hs = fma(y, l, fma(-um, s + c, fma(-0.5 * c, c, q)));
    const double hc = fma(1.0 + y, l, -y);
    h = y <= -1.0 ? 1.0 : (e == 0 ? hs : hc);
}

// l = ln(1 + y) and h = (1 + y) ln(1 + y) - y (hfun) together in FP32 for
// y > -1, as log1p_f32 and hfun<float> compute them (each form below and
// above |y| = 0.05), without branches: both forms evaluated, one selected.
__device__ __forceinline__ void lnh_f32(float y, float &l, float &h) {
    float sl = -1.0f / 8.0f;  // sum_{n=1..8} (-1)^(n+1) y^n / n, Horner
    sl = fmaf(sl, y, 1.0f / 7.0f);
    sl = fmaf(sl, y, -1.0f / 6.0f);
    sl = fmaf(sl, y, 1.0f / 5.0f);
    sl = fmaf(sl, y, -1.0f / 4.0f);
    sl = fmaf(sl, y, 1.0f / 3.0f);
    sl = fmaf(sl, y, -1.0f / 2.0f);
    sl = fmaf(sl, y, 1.0f);
    sl *= y;
    const float u = 1.0f + y;
    const float c = y - (u - 1.0f);
    const float ll = fmaf(c, __builtin_amdgcn_rcpf(u),
                          __builtin_amdgcn_logf(u) * 0.693147180559945309f);
    const bool small = fabsf(y) < 0.05f;
    l = small ? sl : ll;
    constexpr int NT = 8;
    float sh = 0.0f;
    static_for<0, NT - 1>([&](auto K_) {  // Horner, from y^NT down to y^2
        constexpr int n = NT - int(K_);
        sh = fmaf(sh, y, float((n % 2 ? -1.0 : 1.0) / (double(n) * (n - 1))));
    });
    sh = sh * y * y;
    const float hc = y <= -1.0f ? 1.0f : fmaf(1.0f + y, l, -y);
    h = small ? sh : hc;
}

// ------------------------------------------------- entropic step, split
// The entropic step with two lanes per site (row addressing).  The search
// for alpha (Eq. delH) needs every population f_i and relative departure
// x_i = (f_eq,i - f_i) / f_i in each of its evaluations.  Held by one lane,
// all 81 of both plus the search state do not fit the registers: the FP64
// form spilled them to scratch memory, and the FP32-arithmetic forms parked
// all 81 populations in LDS, which limited them to 64-lane workgroups at
// under two waves per SIMD, too few to hide the latency of the search.
// Here a wavefront covers 32 consecutive x of one row: lane l (l < 32)
// holds the even directions 0, 2, ..., 80 of site x0 + l and lane l + 32 the
// odd directions 1, 3, ..., 79 of the same site, 41 and 40 values.  The x_i
// stay in registers and the populations wait in the lane's LDS column (all
// but the last: 80 KB per workgroup in FP64, two workgroups per CU; 40 KB
// in FP32, four per CU).  The evaluation is written without branches (lnh_*
// compute ln(1 + y) and h(y) together, unconditionally): with a branch per
// direction the register allocator kept the x_i in scratch memory.  The
// per-site sums (moments, the bracket, the parts of phi and phi') are each
// lane's half added to its partner's; the partner's value arrives by a lane
// permutation, and since addition commutes both lanes hold the same sum and
// take the same path through the solves and the search.  The search is that
// of entropic_alpha (FP64) and entropic_alpha_x (FP32), with the
// alpha-independent part s1 = sum f x ln(1 + x) summed once
// (phi(a) = sum f h(a x) - a s1, phi'(a) = sum f x ln(1 + a x) - s1), and
// three changes that leave its root and tolerance as they are: a Newton
// step already below QTOL is accepted without a confirming evaluation, a
// Newton step that leaves the bracket is replaced by the regula falsi point
// (Illinois) where both ends' values are known, and with a warm buffer
// attached the search starts from the alpha the site had in the previous
// step.
constexpr int EH = (Q + 1) / 2;  // directions per lane (the odd half has one fewer)
constexpr uint32_t ESEG = 32;    // x per wavefront

// The sum over the two lanes of a site (l and l ^ 32): the same value in
// both.  The empty asm keeps the compiler from fusing the addition into an
// fma with the producer of v, which would round the two lanes differently.
template <class C>
__device__ __forceinline__ C pair_sum(C v) {
    asm volatile("" : "+v"(v));
    return v + __shfl_xor(v, 32);
}
template <class C>
__device__ __forceinline__ C pair_min(C v) {
    return fmin(v, __shfl_xor(v, 32));
}
__device__ __forceinline__ bool pair_and(bool b) {
    return (int(b) & __shfl_xor(int(b), 32)) != 0;
}

// The address of this lane's direction: row base r0 (x offset o0) in the
// lower half-wave, r1 (o1) in the upper.  The row bases are wavefront-
// uniform; the empty asm keeps them scalar, so that the per-lane choice is
// made on the finished bases (two selects and an add) rather than pushed
// into their index arithmetic, where it would turn a scalar row offset into
// a per-lane 64-bit product for every direction.
template <class P>
__device__ __forceinline__ P half_addr(bool hi, P r0, uint32_t o0, P r1,
                                       uint32_t o1) {
    uint64_t b0 = uint64_t(r0), b1 = uint64_t(r1);
    asm volatile("" : "+s"(b0), "+s"(b1));
    return P((hi ? b1 : b0) + (hi ? o1 : o0));
}

// Wavefronts of one sweep (32-x segments) and workgroups of BLOCK lanes;
// 0 where the sweep's lanes would not fit one launch.
inline uint32_t ent2_blocks(const Geom &g) {
    const uint64_t waves = 2ull * uint64_t(g.ny) * uint64_t(g.nz) *
                           ((uint64_t(g.nx) + ESEG - 1) / ESEG);
    const uint64_t blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    return blocks * BLOCK > 0xFFFFFFFFull ? 0u : uint32_t(blocks);
}
// Waves per SIMD: the LDS park (EH - 1 values of C per lane) of that many
// 256-lane workgroups fills the 160 KB of a CU.  (The FP32-arithmetic odd
// step spills 92-96 bytes per lane at four waves and none at three; four
// measured 2-7 % faster.)
template <int ST>
constexpr int ent2_waves() {
    return sizeof(typename Store<ST>::C) == 8 ? 2 : 4;
}

template <int ST, bool ODD>
__global__ __launch_bounds__(BLOCK, ent2_waves<ST>()) void k_step_ent2(
    typename Store<ST>::T *F, Geom g, double omega, unsigned *flags,
    float *warm) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    using AT = Addr<T, ROW>;
    constexpr bool DEV = Store<ST>::DEV;
    constexpr bool F64 = sizeof(C) == 8;
    static_assert(F64 != DEV, "FP64 stores f, the other forms h = f/w - 1");
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t wpr = (uint32_t(g.nx) + ESEG - 1) / ESEG;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t W = tile * WAVES_PER_BLOCK + wv;  // wavefront-uniform
    const uint32_t nyz = uint32_t(g.ny) * uint32_t(g.nz);
    if (W >= 2u * nyz * wpr) return;
    const uint32_t row = W / wpr, seg = W - row * wpr;
    RowSite r;
    r.sub = row >= nyz ? 1 : 0;
    const uint32_t rr = row - (r.sub ? nyz : 0u);
    r.z = int(rr / uint32_t(g.ny));
    r.y = int(rr - uint32_t(r.z) * uint32_t(g.ny));
    r.x = int(seg * ESEG + (threadIdx.x & (ESEG - 1)));
    // both lanes of a site share x, so they leave or stay together
    if (r.x >= g.nx) return;
    const bool hi = (threadIdx.x & 32u) != 0;  // odd directions
    const AT ad(F, g, r);
    // the search's start value at this site (warm start), 0 for none
    const uint32_t sidx = site_index(g, r);
    const float w0 = warm ? warm[sidx] : 0.0f;
    float wout = 0.0f;
    // the populations (storage form, as C) of slots 0..EH-2 wait in this
    // lane's own LDS column through the solves; the registers hold the x_i
    // and the search
    __shared__ __align__(16) C park[EH - 1][BLOCK];
    // weight of slot k's direction in this lane (0 for the odd half's empty
    // slot), for the deviation forms
    auto wsel = [&](auto K_) -> C {
        constexpr int k = decltype(K_)::value, i0 = 2 * k, i1 = 2 * k + 1;
        constexpr double w1 = i1 < Q ? weight(i1) : 0.0;
        return hi ? C(w1) : C(weight(i0));
    };

    // ---- load this lane's half (direction 2k + hi in slot k)
    C v[EH], x[EH];
    {
        AT la = ad;
        // source row and x offset of direction i (AA pattern: the odd step
        // pulls from x - c_i in slot opp(i), the even step reads slot i)
        auto src = [&](auto I_, gptr<T> &rowp, uint32_t &off) {
            constexpr int i = decltype(I_)::value;
            if constexpr (ODD) {
                rowp = la.template nbr_row<i, true, opp(i)>();
                off = la.template nbr_x<i, true>();
            } else {
                rowp = la.row(i, la.sub, la.y, la.z);
                off = la.xo[4];
            }
        };
        static_for<0, EH>([&](auto K_) {
            constexpr int k = K_, i0 = 2 * k, i1 = 2 * k + 1;
            if constexpr (k > 0 && k % (LOAD_GROUP / 2) == 0) la.launder();
            gptr<T> r0;
            uint32_t o0;
            src(IC<i0>{}, r0, o0);
            if constexpr (i1 < Q) {
                gptr<T> r1;
                uint32_t o1;
                src(IC<i1>{}, r1, o1);
                v[k] = Store<ST>::load(half_addr(hi, r0, o0, r1, o1));
            } else {
                // the odd half has no direction here: f = 1 (FP64) or h = 0
                // with weight 0, and x = 0, add nothing to any sum (the lane
                // reads its partner's in-bounds element and drops it)
                const C t = Store<ST>::load(byte_off(r0, o0));
                v[k] = hi ? C(DEV ? 0.0 : 1.0) : t;
            }
        });
    }

    // ---- conserved moments (sums over both halves; FP64 from there on)
    C rs = C(0), jx = C(0), jy = C(0), jz = C(0), en = C(0);
    static_for<0, EH>([&](auto K_) {
        constexpr int k = K_, i0 = 2 * k, i1 = 2 * k + 1;
        constexpr bool has1 = i1 < Q;
        // w_i h_i (deviation forms) or f_i (FP64); nothing for the empty slot
        C wt;
        if constexpr (DEV) wt = wsel(K_) * v[k];
        else wt = has1 || !hi ? v[k] : C(0);
        rs += wt;
        constexpr double ax0 = cx(i0), ay0 = cy(i0), az0 = cz(i0), c0 = csq(i0);
        constexpr double ax1 = has1 ? cx(i1) : 0.0, ay1 = has1 ? cy(i1) : 0.0,
                         az1 = has1 ? cz(i1) : 0.0, c1 = has1 ? csq(i1) : 0.0;
        if constexpr (ax0 != 0.0 || ax1 != 0.0) jx = fma(hi ? C(ax1) : C(ax0), wt, jx);
        if constexpr (ay0 != 0.0 || ay1 != 0.0) jy = fma(hi ? C(ay1) : C(ay0), wt, jy);
        if constexpr (az0 != 0.0 || az1 != 0.0) jz = fma(hi ? C(az1) : C(az0), wt, jz);
        if constexpr (c0 != 0.0 || c1 != 0.0) en = fma(hi ? C(c1) : C(c0), wt, en);
    });
    Moments m;
    {
        // deviation form: rho = 1 + sum w h, E = 3 theta0 + sum w c^2 h
        const double rho = (DEV ? 1.0 : 0.0) + double(pair_sum(rs));
        const double E = (DEV ? 3.0 * THETA0 : 0.0) + double(pair_sum(en));
        const double ir = 1.0 / rho;
        m.rho = rho;
        m.ux = double(pair_sum(jx)) * ir;
        m.uy = double(pair_sum(jy)) * ir;
        m.uz = double(pair_sum(jz)) * ir;
        m.e = E * ir;
        m.theta = (m.e - (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz)) * (1.0 / 3.0);
        m.ok = rho > 0.0 && m.theta > 0.0 && isfinite(rho) && isfinite(m.theta) &&
               isfinite(m.ux) && isfinite(m.uy) && isfinite(m.uz);
    }
    static_for<0, EH - 1>([&](auto K_) {
        constexpr int kk = K_;
        park[kk][threadIdx.x] = v[kk];
    });
    // compiler barrier: the parked values are re-read from LDS, not kept in
    // registers across the solves
    asm volatile("" ::: "memory");
    const C vlast = v[EH - 1];
    auto vv = [&](auto K_) -> C {  // stored value of slot k
        constexpr int kk = decltype(K_)::value;
        if constexpr (kk < EH - 1)
            return park[kk][threadIdx.x];
        else
            return vlast;
    };
    unsigned bits = 0;
    C lam[5] = {C(0), C(0), C(0), C(0), C(0)};
    if (m.ok) {
        if (solve_multipliers<C>(C(m.ux), C(m.uy), C(m.uz), C(m.e), C(m.theta),
                                 lam) < 0)
            bits |= LBM_FLAG_NEWTON;
    } else {
        bits |= isfinite(m.rho) && isfinite(m.theta) ? LBM_FLAG_UNREALIZABLE
                                                     : LBM_FLAG_NONFINITE;
    }

    // ---- f_eq (FP64) or f_eq / w (deviation forms) of this lane's
    // directions into x, then x = (f_eq - f) / f (the plain difference
    // f_eq - f, or (f_eq - f) / w, at a non-positive population)
    C alpha = C(2);
    // (the odd half's empty slot keeps f_eq = f: 1 in FP64, w (f/w = 1))
    static_for<0, EH>([&](auto K_) { x[int(K_)] = C(1); });
    if (m.ok) {
        const C rho = C(m.rho);
        const C A = visit_shells(lam, [&](auto S_, C px, C mx, C py, C my,
                                          C pz, C mz, C e) {
            constexpr int S = decltype(S_)::value;
            const C q = (DEV ? rho : rho * C(shell_weight(S))) * e;
            static_for<1, Q>([&](auto I_) {
                constexpr int i = I_;
                if constexpr (shell_of(i) == S) {
                    const C val = q * (pick<cx2(i)>(px, mx) *
                                       pick<cy2(i)>(py, my) *
                                       pick<cz2(i)>(pz, mz));
                    x[i / 2] = hi == bool(i & 1) ? val : x[i / 2];
                }
            });
        });
        x[0] = hi ? x[0] : (DEV ? rho : rho * C(shell_weight(0))) * A;
        bool pos = true;
        C amax = C(INFINITY), scale = C(0), s1 = C(0);
        static_for<0, EH>([&](auto K_) {
            constexpr int k = K_;
            // fq: f (FP64) or f / w; f: the population
            const C fq = DEV ? C(1) + vv(K_) : vv(K_);
            const C f = DEV ? wsel(K_) * fq : fq;
            const C d = x[k] - fq;
            const bool p = fq > C(0);
            pos = pos && p;
            C xk;
            if constexpr (F64) xk = p ? d / fq : d;
            else xk = p ? d * __builtin_amdgcn_rcpf(fq) : d;
            x[k] = xk;
            if (p) {
                scale = fma(f * xk, xk, scale);
                if (xk < C(0)) {
                    if constexpr (F64) amax = fmin(amax, C(-1) / xk);
                    else amax = fmin(amax, -__builtin_amdgcn_rcpf(xk));
                }
            }
        });
        pos = pair_and(pos);
        if (!pos) {
            bits |= LBM_FLAG_NEGATIVE;
        } else if (pair_sum(scale) > C(0)) {
            amax = pair_min(amax);
            auto lnh = [&](C y, C &l, C &h) {
                if constexpr (F64) lnh_f64(y, l, h);
                else lnh_f32(y, l, h);
            };
            static_for<0, EH>([&](auto K_) {
                constexpr int k = K_;
                const C f = DEV ? wsel(K_) * (C(1) + vv(K_)) : vv(K_);
                C l1, h1;
                lnh(x[k], l1, h1);
                s1 = fma(f * x[k], x[k] <= C(-1) ? C(-INFINITY) : l1, s1);
            });
            s1 = pair_sum(s1);
            // phi(a) and phi'(a) over both halves, four interleaved partial
            // sums per lane
            auto eval = [&](C a, C &ph, C &dph) __attribute__((always_inline)) {
                C p4[4] = {C(0), C(0), C(0), C(0)}, d4[4] = {C(0), C(0), C(0), C(0)};
                // the populations are read from LDS in every evaluation
                asm volatile("" ::: "memory");
                static_for<0, EH>([&](auto K_) {
                    constexpr int k = K_;
                    const C xk = x[k], y = a * xk;
                    const C f = DEV ? wsel(K_) * (C(1) + vv(K_)) : vv(K_);
                    // evaluated unconditionally (NaN or garbage where
                    // y <= -1, then discarded): no branch per direction
                    C l, hy;
                    lnh(y, l, hy);
                    const C ly = y <= C(-1) ? C(-INFINITY) : l;
                    p4[k % 4] = fma(f, hy, p4[k % 4]);
                    d4[k % 4] = fma(f * xk, ly, d4[k % 4]);
                });
                const C pp = pair_sum((p4[0] + p4[1]) + (p4[2] + p4[3]));
                const C dd = pair_sum((d4[0] + d4[1]) + (d4[2] + d4[3]));
                ph = fma(-a, s1, pp);
                dph = dd - s1;
            };
            // the steps of entropic_alpha, one evaluation per pass (a single
            // call site, inlined once); at_max: the pass checks alpha_max.
            // One more stopping rule: a Newton step inside the bracket
            // smaller than QTOL a is accepted without evaluating phi at the
            // new point: Newton converges quadratically on the convex phi, so
            // the new point is within about (QTOL a)^2 / a of the root, below
            // TOL a; this saves the evaluation that would only confirm it
            // (most wavefronts took four evaluations in FP64, three in FP32).
            // Looser bounds (1e-7, 1e-3) moved the results on rough states
            // (FP64 by 2.5e-13, FP32 beyond its storage bar): the constant
            // of the quadratic convergence is not small everywhere.
            constexpr C TOL = F64 ? C(1e-14) : C(1e-6);
            constexpr C QTOL = F64 ? C(1e-9) : C(1e-4);
            constexpr int MAXIT = F64 ? 100 : 50;
            C lo = C(0), hb = amax, a, next = C(0);
            // phi at the bracket ends where evaluated (phi(0) = 0 carries no
            // slope information; phi at alpha_max is known once checked)
            C plo = C(0), phb = C(INFINITY);
            int side = 0;  // the end the last evaluation replaced
            // the point tried when a Newton step leaves the bracket: the
            // regula falsi point of the two ends where both values are
            // known, with the Illinois rule (the value kept at an end that
            // survives two replacements of the other is halved), else the
            // midpoint.  Near alpha_max, where phi rises with a vertical
            // tangent, Newton steps from the left overshoot the bracket and
            // plain bisection needed 8-19 evaluations per wavefront.
            auto inner = [&]() -> C {
                if (plo < C(0) && phb > C(0) && phb < C(INFINITY)) {
                    const C c = (lo * phb - hb * plo) / (phb - plo);
                    if (c > lo && c < hb) return c;
                }
                return C(0.5) * (lo + hb);
            };
            bool max_checked = false, at_max = false, stop_next = false,
                 done = false;
            // start: with a kept alpha from the previous step inside the
            // bracket, Newton starts there (after the check at alpha_max
            // where that alpha was capped); else at alpha_max (checked
            // first) or 2
            const C a0 = C(fabsf(w0));
            const bool have = a0 > C(0) && a0 < amax;
            if (amax <= C(2)) {
                if (have && w0 > 0.0f) {
                    a = a0;
                } else {
                    a = amax;
                    at_max = true;
                    next = have ? a0 : C(0.5) * amax;
                }
            } else {
                a = have ? a0 : C(2);
            }
            for (int it = 0; !done && (it < MAXIT || at_max);) {
                C ph, dph;
                eval(a, ph, dph);
                if (at_max) {
                    at_max = false;
                    max_checked = true;
                    if (ph <= C(0) || stop_next) {
                        alpha = ph <= C(0) ? amax : next;
                        done = true;
                    } else {
                        phb = ph;  // hb is alpha_max
                        a = inner();
                    }
                    continue;
                }
                ++it;
                if (ph < C(0)) {
                    lo = a;
                    plo = ph;
                    if (side < 0) phb *= C(0.5);
                    side = -1;
                } else {
                    hb = a;
                    phb = ph;
                    if (side > 0) plo *= C(0.5);
                    side = 1;
                }
                const C newton = a - ph / dph;
                C an = newton;
                if (ph == C(0) || fabs(an - a) <= TOL * a) {
                    alpha = an;
                    done = true;
                    continue;
                }
                if (an > lo && an < hb && fabs(an - a) <= QTOL * a) {
                    alpha = an;
                    done = true;
                    continue;
                }
                if (!(an > lo && an < hb)) {
                    an = inner();
                    if (!max_checked && !(newton < hb) && hb == amax) {
                        // the step overshoots alpha_max: check it, then go
                        // inside the bracket
                        stop_next = hb - lo <= TOL * a;
                        next = an;
                        at_max = true;
                        a = amax;
                        continue;
                    }
                }
                if (hb - lo <= TOL * a) {
                    alpha = an;
                    done = true;
                    continue;
                }
                a = an;
            }
            if (!done) alpha = a;
            wout = alpha == amax ? -float(alpha) : float(alpha);
        }
    }
    if (warm && !hi) warm[sidx] = wout;
    // ---- relax (f* = f + (alpha / 2) omega (f_eq - f); in the deviation
    // forms h* = h + (alpha / 2) omega x (1 + h)) and stream
    const C ome = m.ok ? C(omega) * C(0.5) * alpha : C(0);
    AT wr = ad;
    wr.launder();
    // destination row and x offset of direction i (the odd step pushes to
    // x + c_i in slot i, the even step writes slot opp(i))
    auto dst = [&](auto I_, gptr<T> &rowp, uint32_t &off) {
        constexpr int i = decltype(I_)::value;
        if constexpr (ODD) {
            rowp = wr.template nbr_row<i, false, i>();
            off = wr.template nbr_x<i, false>();
        } else {
            rowp = wr.row(opp(i), wr.sub, wr.y, wr.z);
            off = wr.xo[4];
        }
    };
    static_for<0, EH>([&](auto K_) {
        constexpr int k = K_, i0 = 2 * k, i1 = 2 * k + 1;
        if constexpr (k > 0 && k % (LOAD_GROUP / 2) == 0) wr.launder();
        const C sv = vv(K_);
        const C fq = DEV ? C(1) + sv : sv;  // f (FP64) or f / w
        // (an unrealizable site keeps its populations)
        const C out = m.ok ? fma(ome, fq > C(0) ? x[k] * fq : x[k], sv) : sv;
        gptr<T> r0;
        uint32_t o0;
        dst(IC<i0>{}, r0, o0);
        if constexpr (i1 < Q) {
            gptr<T> r1;
            uint32_t o1;
            dst(IC<i1>{}, r1, o1);
            Store<ST>::store(half_addr(hi, r0, o0, r1, o1), out);
        } else if (!hi) {
            Store<ST>::store(byte_off(r0, o0), out);
        }
    });
    flag_or(flags, bits);
}

// The entropic kernels are instantiated in translation units of their own
// (kernels_<storage>_ent.hip), which compile in parallel with the others.
template <int ST>
void launch_step_entropic_warm(void *f, const Geom &g, double omega,
                               unsigned *flags, bool odd, float *warm,
                               hipStream_t stream) {
    // two lanes per site where the row addressing applies (and the sweep's
    // lanes fit one launch); the single-lane kernels keep no start values
    const uint32_t blocks = mode_of(g) != SMALL ? ent2_blocks(g) : 0u;
    if (blocks) {
        auto *F = static_cast<typename Store<ST>::T *>(f);
        if (odd)
            hipLaunchKernelGGL((k_step_ent2<ST, true>), dim3(blocks),
                               dim3(BLOCK), 0, stream, F, g, omega, flags, warm);
        else
            hipLaunchKernelGGL((k_step_ent2<ST, false>), dim3(blocks),
                               dim3(BLOCK), 0, stream, F, g, omega, flags, warm);
        return;
    }
    launch_step<ST, true>(f, g, omega, flags, odd, stream);
}

template <int ST>
void launch_step_entropic(void *f, const Geom &g, double omega,
                          unsigned *flags, bool odd, hipStream_t stream) {
    launch_step_entropic_warm<ST>(f, g, omega, flags, odd, nullptr, stream);
}

}  // namespace lbm81
