// Device code of the RD3Q81 library: storage forms, grid addressing, the
// fused site update and the kernels.  Included once per storage form by the
// kernels_*.hip translation units, which instantiate and launch them.
//
// Method (Atif et al., arXiv:2409.05114): per site, moments of the 81
// populations (Eq. conslaws) -> entropic equilibrium by Newton on five
// multipliers (Sec. III, equilibrium.hpp) -> trapezoidal BGK relaxation with
// alpha = 2, beta = 1/(2 tau + 1) (Eq. discretelbm) -> streaming along c_i on
// the body-centred grid (cube corners + cube centres; half-integer links
// switch sub-lattice).
//
// Memory layout (types.hpp): direction planes or row tiles, x fastest in
// both, so every per-direction access of a wavefront is a contiguous
// (possibly shifted) run of 64 elements.  Streaming is in place with the AA pattern:
//   even step (count even -> odd): read slot i at x, collide, write the
//     post-collision f*_i to slot opp(i) at the same x;
//   odd step (count odd -> even): read f_i from slot opp(i) at x - c_i,
//     collide, write f*_i to slot i at x + c_i.
// In the odd step a thread writes exactly the 81 addresses it read, so
// no two threads touch the same address within a launch; the kernel
// boundary between steps is the only barrier the scheme needs.
//
// Storage forms: FP64 stores f_i; FP32/FP16/BF16 store h_i = f_i / w_i - 1
// and compute in FP32, with the temperature recovered from the energy moment
// in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "equilibrium.hpp"
#include "lattice.hpp"
#include "lbm81.h"
#include "types.hpp"

namespace lbm81 {



// ---------------------------------------------------------------- storage
template <int ST>
struct Store;

template <>
struct Store<LBM_F64> {
    using T = double;  // stored
    using C = double;  // computed
    static constexpr bool DEV = false;
    // Occupancy target (waves per SIMD) and how many of the 81 values are
    // parked in LDS during the equilibrium solve (see site_update).
    static constexpr int WAVES = 2;
    static constexpr int NLDS = 40;
    // Route odd-step stores through LDS so that every store instruction
    // covers whole cache lines (see site_update).
    static constexpr bool XCH = false;
    static constexpr bool TILED = tiled_layout(LBM_F64);
    template <class P>
    static __device__ __forceinline__ C load(P p) { return *p; }
    template <class P>
    static __device__ __forceinline__ void store(P p, C v) { *p = v; }
};

template <>
struct Store<LBM_F32> {
    using T = float;
    using C = float;
    static constexpr bool DEV = true;
    static constexpr int WAVES = 4;
    static constexpr int NLDS = 40;
    static constexpr bool XCH = false;
    static constexpr bool TILED = tiled_layout(LBM_F32);
    template <class P>
    static __device__ __forceinline__ C load(P p) { return *p; }
    template <class P>
    static __device__ __forceinline__ void store(P p, C v) { *p = v; }
};

template <>
struct Store<LBM_F16> {
    using T = _Float16;
    using C = float;
    static constexpr bool DEV = true;
    static constexpr int WAVES = 3;
    static constexpr int NLDS = 40;
    static constexpr bool XCH = true;
    static constexpr bool TILED = tiled_layout(LBM_F16);
    template <class P>
    static __device__ __forceinline__ C load(P p) { return float(*p); }
    // The FP32 value is rounded to FP16 (round to nearest even) as it
    // stands: the empty asm keeps the compiler from fusing the producing
    // FMA into a mixed-precision FMA that rounds once to FP16, which it does
    // in some code paths and not in others (the stored bits would then
    // depend on the path).
    template <class P>
    static __device__ __forceinline__ void store(P p, C v) {
        asm volatile("" : "+v"(v));
        *p = _Float16(v);
    }
};

template <>
struct Store<LBM_BF16> {
    using T = __bf16;
    using C = float;
    static constexpr bool DEV = true;
    static constexpr int WAVES = 3;
    static constexpr int NLDS = 40;
    static constexpr bool XCH = true;
    static constexpr bool TILED = tiled_layout(LBM_BF16);
    template <class P>
    static __device__ __forceinline__ C load(P p) { return float(*p); }
    // round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
    template <class P>
    static __device__ __forceinline__ void store(P p, C v) { *p = __bf16(v); }
};

// The 16-bit forms keep direction planes (Addr<T, ROW> forms row offsets
// inside a plane in 32 bits for 2-byte elements).
static_assert(!Store<LBM_F16>::TILED && !Store<LBM_BF16>::TILED,
              "16-bit forms must keep direction planes");

// ----------------------------------------------------------------- geometry

// A pointer into the global address space.  Row-mode addressing works on
// these throughout: the step kernels launder their base pointers (see
// Addr::launder), and a generic pointer from there on would turn every
// store into a flat store with a 64-bit address per lane instead of a
// scalar base plus a 32-bit lane offset.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> global(T *p) {
    return (gptr<T>)p;
}




// v = u + o, with u in [0, n) and o in [LO, HI] (compile-time bounds within
// [-4, 5], n >= 4 in row mode), wrapped into [0, n): only the side the
// offset can cross is checked.
template <int LO, int HI>
__device__ __forceinline__ int wrap_off(int v, int n) {
    if constexpr (LO >= 0)
        return v >= n ? v - n : v;
    else if constexpr (HI <= 0)
        return v < 0 ? v + n : v;
    else {
        v = v < 0 ? v + n : v;
        return v >= n ? v - n : v;
    }
}

// v in [-4, n + 4) wrapped into [0, n).
template <bool SMALLW>
__device__ __forceinline__ int wrap(int v, int n) {
    if constexpr (SMALLW) {
        int r = v % n;
        return r < 0 ? r + n : r;
    } else {
        v = v < 0 ? v + n : v;
        return v >= n ? v - n : v;
    }
}

// Shift of the neighbour index along one axis for a link with doubled
// component a, moving by -c (SRC) or +c.  Integer links stay on the
// sub-lattice and shift by -+a/2.  Half links switch sub-lattice; the shift
// is sub + o with o = -(a+1)/2 (SRC) or (a-1)/2 (exact integers for odd a).
template <int A_, bool SRC>
constexpr int half_off() {
    return SRC ? -(A_ + 1) / 2 : (A_ - 1) / 2;
}
template <int A_, bool SRC>
constexpr int int_off() {
    return SRC ? -A_ / 2 : A_ / 2;
}

// Element offset of x within its row.
__device__ __forceinline__ uint32_t x_el(uint32_t x, uint32_t ts) {
    return (x / TILE) * ts + (x % TILE);
}
// Element offset of a site's direction slot 0 (add slot * ss).
__device__ __forceinline__ uint64_t site_el(const Geom &g, uint32_t s) {
    const uint32_t row = s / uint32_t(g.nx);
    const uint32_t x = s - row * uint32_t(g.nx);
    return uint64_t(row) * g.rs + x_el(x, g.ts);
}

template <class T>
__device__ __forceinline__ T *byte_off(T *base, uint32_t bytes) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + bytes);
}
template <class T>
__device__ __forceinline__ const T *byte_off(const T *base, uint32_t bytes) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                       bytes);
}
template <class T>
__device__ __forceinline__ gptr<T> byte_off(gptr<T> base, uint32_t bytes) {
    using gchar = __attribute__((address_space(1))) char;
    return (gptr<T>)((gchar *)base + bytes);
}

template <class T, int MODE>
struct Addr;

// Site of this lane in ROW mode for workgroup tile `tile`: wavefront-
// uniform sub-lattice, y, z and row segment; per-lane x.
struct RowSite {
    int sub, y, z, x;
    bool active;
};

__device__ __forceinline__ RowSite row_site(const Geom &g, uint32_t tile,
                                            uint32_t wpb = WAVES_PER_BLOCK) {
    RowSite r;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t W = tile * wpb + wv;  // wavefront-uniform
    const uint32_t row = W / g.wpr;
    const uint32_t seg = W - row * g.wpr;
    const uint32_t nyz = uint32_t(g.ny) * uint32_t(g.nz);
    r.sub = row >= nyz ? 1 : 0;
    const uint32_t rr = row - (r.sub ? nyz : 0u);
    r.z = int(rr / uint32_t(g.ny));
    r.y = int(rr - uint32_t(r.z) * uint32_t(g.ny));
    r.x = int(seg * 64u + (threadIdx.x & 63u));
    r.active = W < g.nwaves && r.x < g.nx;
    return r;
}

__device__ __forceinline__ uint32_t site_index(const Geom &g, const RowSite &r) {
    return (r.sub ? g.N : 0u) +
           (uint32_t(r.z) * uint32_t(g.ny) + uint32_t(r.y)) * uint32_t(g.nx) +
           uint32_t(r.x);
}

template <class T>
struct Addr<T, ROW> {
    // The 16-bit forms' odd step is sensitive to its scalar instruction
    // count (the neighbour-row addresses of its 162 accesses), so they take
    // a leaner form: the byte offset of a row inside its direction plane in
    // 32 bits (a 16-bit plane holds fewer than 2^31 sites, so it stays
    // below 4 GiB), wraps that test only the side an offset can cross, and
    // one row base for the slots of the own site.  That measured 1.6 %
    // faster for FP16 and 1.5 % slower for FP64, so the 8- and 4-byte forms
    // keep the 64-bit products (FP32 row tiles also span all 81 slots).
    static constexpr bool LEAN = sizeof(T) == 2;
    gptr<T> F;
    uint32_t rs, ss;
    uint32_t rsb;  // planes: bytes between consecutive rows
    int nx, ny, nz;
    int sub, y, z;  // wavefront-uniform
    uint32_t xo[9];  // per lane: bytes of wrap(x + k) within a row, k = -4..4

    __device__ __forceinline__ Addr(T *F_, const Geom &g, const RowSite &r)
        : F(global(F_)), rs(g.rs), ss(g.ss), rsb(g.rs * uint32_t(sizeof(T))),
          nx(g.nx), ny(g.ny), nz(g.nz), sub(r.sub), y(r.y), z(r.z) {
#pragma unroll
        for (int k = -4; k <= 4; ++k) {
            int v = r.x + k;
            if (k < 0) v = v < 0 ? v + nx : v;
            if (k > 0) v = v >= nx ? v - nx : v;
            xo[k + 4] = x_el(uint32_t(v), g.ts) * uint32_t(sizeof(T));
        }
    }
    // Make the compiler treat the base pointer and the row coordinates as
    // new values, so that the store addresses are computed where they are
    // used (a few scalar operations each) instead of being computed up front
    // and kept alive (spilled) across the whole collision.
    __device__ __forceinline__ void launder() {
        uint64_t b = uint64_t(F);
        // wavefront-uniform by construction (row_site)
        sub = __builtin_amdgcn_readfirstlane(sub);
        y = __builtin_amdgcn_readfirstlane(y);
        z = __builtin_amdgcn_readfirstlane(z);
        asm volatile("" : "+s"(b), "+s"(sub), "+s"(y), "+s"(z));
        F = (gptr<T>)b;
    }
    __device__ __forceinline__ gptr<T> row(int slot, int sb, int yy, int zz) const {
        const uint32_t r = (uint32_t(sb ? nz : 0) + uint32_t(zz)) * uint32_t(ny) +
                           uint32_t(yy);
        if constexpr (LEAN)
            return byte_off(F + uint64_t(slot) * ss, r * rsb);
        else
            return F + uint64_t(r) * rs + uint64_t(slot) * ss;
    }
    template <int SLOT>
    __device__ __forceinline__ gptr<T> own() const {
        if constexpr (LEAN) {
            // the row base is shared by every slot of the site
            const uint32_t r = (uint32_t(sub ? nz : 0) + uint32_t(z)) * uint32_t(ny) +
                               uint32_t(y);
            return byte_off(byte_off(F, r * rsb) + uint64_t(SLOT) * ss, xo[4]);
        } else {
            return byte_off(row(SLOT, sub, y, z), xo[4]);
        }
    }
    // Row (its x = 0 element) of the neighbour along -c_I (SRC) or +c_I in
    // slot SLOT; wavefront-uniform.
    template <int I, bool SRC, int SLOT>
    __device__ __forceinline__ gptr<T> nbr_row() const {
        constexpr int b = cy2(I), c = cz2(I);
        if constexpr (is_half(I)) {
            constexpr int oy = half_off<b, SRC>(), oz = half_off<c, SRC>();
            if constexpr (LEAN)  // sub is 0 or 1: the offset is oy or oy + 1
                return row(SLOT, 1 - sub, wrap_off<oy, oy + 1>(y + sub + oy, ny),
                           wrap_off<oz, oz + 1>(z + sub + oz, nz));
            else
                return row(SLOT, 1 - sub, wrap<false>(y + sub + oy, ny),
                           wrap<false>(z + sub + oz, nz));
        } else {
            constexpr int oy = int_off<b, SRC>(), oz = int_off<c, SRC>();
            if constexpr (LEAN) {
                const int yy = oy == 0 ? y : wrap_off<oy, oy>(y + oy, ny);
                const int zz = oz == 0 ? z : wrap_off<oz, oz>(z + oz, nz);
                return row(SLOT, sub, yy, zz);
            } else {
                const int yy = oy == 0 ? y : wrap<false>(y + oy, ny);
                const int zz = oz == 0 ? z : wrap<false>(z + oz, nz);
                return row(SLOT, sub, yy, zz);
            }
        }
    }
    // Byte offset of this lane's neighbour x within that row.
    template <int I, bool SRC>
    __device__ __forceinline__ uint32_t nbr_x() const {
        constexpr int a = cx2(I);
        if constexpr (is_half(I)) {
            constexpr int ox = half_off<a, SRC>();
            return sub ? xo[ox + 5] : xo[ox + 4];
        } else {
            return xo[int_off<a, SRC>() + 4];
        }
    }
    template <int I, bool SRC, int SLOT>
    __device__ __forceinline__ gptr<T> nbr() const {
        return byte_off(nbr_row<I, SRC, SLOT>(), nbr_x<I, SRC>());
    }
};

template <class T, int MODE>
struct Addr {
    static_assert(MODE == SMALL, "mode");
    T *F;
    uint32_t rs, ss;
    uint32_t ts;
    int nx, ny, nz;
    uint32_t N;
    int sub, x, y, z;  // per lane

    __device__ __forceinline__ Addr(T *F_, const Geom &g, uint32_t s)
        : F(F_), rs(g.rs), ss(g.ss), ts(g.ts), nx(g.nx), ny(g.ny), nz(g.nz), N(g.N) {
        sub = s >= N ? 1 : 0;
        const uint32_t i0 = s - (sub ? N : 0u);
        const uint32_t r = i0 / uint32_t(nx);
        x = int(i0 - r * uint32_t(nx));
        z = int(r / uint32_t(ny));
        y = int(r - uint32_t(z) * uint32_t(ny));
    }
    __device__ __forceinline__ void launder() {
        uint64_t b = reinterpret_cast<uint64_t>(F);
        asm volatile("" : "+s"(b));
        F = reinterpret_cast<T *>(b);
    }
    __device__ __forceinline__ T *at(int slot, int sb, int xx, int yy,
                                     int zz) const {
        const uint32_t r = (uint32_t(sb ? nz : 0) + uint32_t(zz)) * uint32_t(ny) +
                           uint32_t(yy);
        return F + uint64_t(r) * rs + uint64_t(slot) * ss + x_el(uint32_t(xx), ts);
    }
    template <int SLOT>
    __device__ __forceinline__ T *own() const {
        return at(SLOT, sub, x, y, z);
    }
    template <int I, bool SRC, int SLOT>
    __device__ __forceinline__ T *nbr() const {
        constexpr bool SW = true;
        constexpr int a = cx2(I), b = cy2(I), c = cz2(I);
        if constexpr (is_half(I)) {
            constexpr int ox = half_off<a, SRC>(), oy = half_off<b, SRC>(),
                          oz = half_off<c, SRC>();
            return at(SLOT, 1 - sub, wrap<SW>(x + sub + ox, nx),
                      wrap<SW>(y + sub + oy, ny), wrap<SW>(z + sub + oz, nz));
        } else {
            constexpr int ox = int_off<a, SRC>(), oy = int_off<b, SRC>(),
                          oz = int_off<c, SRC>();
            return at(SLOT, sub, ox == 0 ? x : wrap<SW>(x + ox, nx),
                      oy == 0 ? y : wrap<SW>(y + oy, ny),
                      oz == 0 ? z : wrap<SW>(z + oz, nz));
        }
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs
// on XCD b % 8).  Renumber them so that each XCD processes one contiguous
// range of tiles: cache lines shared by neighbouring tiles then stay in one
// L2.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t xcd = b & 7u, slot = b >> 3;
    const uint32_t per = n >> 3, rem = n & 7u;
    const uint32_t start = xcd < rem ? xcd * (per + 1u)
                                     : rem * (per + 1u) + (xcd - rem) * per;
    return start + slot;
}

// Workgroup order of a plain step sweep.  The FP64 even step reads and
// writes only its own sites' slots, so no tile shares cache lines with
// another; there the plain dispatch order, in which the eight XCDs work on
// neighbouring tiles and every direction plane is swept by one front,
// measured 1.5 % faster than XCD ranges in the buffers where the 81-plane
// pattern runs fastest.  Every other step keeps the XCD ranges (FP32 row
// tiles lose 10 % without them, the 16-bit forms 3 %).
template <int ST, bool ODD, bool ENT>
constexpr bool plain_order() {
    return ST == LBM_F64 && !ODD && !ENT;
}

// ------------------------------------------------------------- site update
// The 81 populations of a site at the current step in storage form (f for
// FP64, h = f/w - 1 otherwise).  At odd parity direction i lives in slot
// opp(i) at x - c_i.
// The row coordinates are laundered every LOAD_GROUP directions so that the
// compiler computes the addresses of one group at a time instead of all 81
// up front (which spills scalar registers).
constexpr int LOAD_GROUP = 16;

template <int ST, bool ODD, class AD>
__device__ __forceinline__ void gather(const AD &ad, typename Store<ST>::C v[Q]) {
    AD la = ad;
    static_for<0, Q>([&](auto I_) {
        constexpr int i = I_;
        if constexpr (i > 0 && i % LOAD_GROUP == 0) la.launder();
        if constexpr (ODD)
            v[i] = Store<ST>::load(la.template nbr<i, true, opp(i)>());
        else
            v[i] = Store<ST>::load(la.template own<i>());
    });
}

// Conserved moments in FP64: rho, u, e = u^2 + 3 theta and theta.
struct Moments {
    double rho, ux, uy, uz, e, theta;
    bool ok;
};

template <int ST>
__device__ __forceinline__ Moments moments_of(const typename Store<ST>::C v[Q]) {
    using C = typename Store<ST>::C;
    // per-shell sums and antisymmetric pair differences
    C ssum[NSHELL];
    static_for<0, NSHELL>([&](auto S_) { ssum[int(S_)] = C(0); });
    static_for<0, Q>([&](auto I_) {
        constexpr int i = I_;
        ssum[shell_of(i)] += v[i];
    });
    C jx = C(0), jy = C(0), jz = C(0);
    static_for<1, NPAIR + 1>([&](auto I_) {
        constexpr int i = I_;
        constexpr C wfac = Store<ST>::DEV ? C(weight(i)) : C(1);
        const C d = v[i] - v[i + NPAIR];
        if constexpr (cx2(i) != 0) jx += (wfac * C(cx(i))) * d;
        if constexpr (cy2(i) != 0) jy += (wfac * C(cy(i))) * d;
        if constexpr (cz2(i) != 0) jz += (wfac * C(cz(i))) * d;
    });
    C r = C(0), en = C(0);
    static_for<0, NSHELL>([&](auto S_) {
        constexpr int s = S_;
        constexpr C wfac = Store<ST>::DEV ? C(shell_weight(s)) : C(1);
        r += wfac * ssum[s];
        if constexpr (s > 0) en += (wfac * C(0.25 * SHELL_C2X4[s])) * ssum[s];
    });
    Moments m;
    // deviation form: rho = 1 + sum w h, E = 3 theta0 + sum w c^2 h; the
    // temperature is recovered in FP64 either way
    const double rho = Store<ST>::DEV ? 1.0 + double(r) : double(r);
    const double E = Store<ST>::DEV ? 3.0 * THETA0 + double(en) : double(en);
    const double ir = 1.0 / rho;
    m.rho = rho;
    m.ux = double(jx) * ir;
    m.uy = double(jy) * ir;
    m.uz = double(jz) * ir;
    m.e = E * ir;
    m.theta = (m.e - (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz)) * (1.0 / 3.0);
    m.ok = rho > 0.0 && m.theta > 0.0 && isfinite(rho) && isfinite(m.theta) &&
           isfinite(m.ux) && isfinite(m.uy) && isfinite(m.uz);
    return m;
}

__device__ __forceinline__ void flag_or(unsigned *flags, unsigned bits) {
    if (bits) atomicOr(flags, bits);
}

// Write f*_i = f_i + omega (f_eq_i - f_i) for every direction, in storage
// form, through `put(IC<i>, value)`.  With e_s = exp(mu + gamma c_s^2),
// f_eq_i = rho w_i e_s X^(2 c_x) Y^(2 c_y) Z^(2 c_z); in the deviation form
// h_eq_i = f_eq_i / w_i - 1.
template <int ST, class PUT>
__device__ __forceinline__ void relax_all(const typename Store<ST>::C lam[5],
                                          const typename Store<ST>::C v[Q],
                                          typename Store<ST>::C rho,
                                          typename Store<ST>::C om, PUT &&put) {
    using C = typename Store<ST>::C;
    const C keep = C(1) - om;
    const C shift = Store<ST>::DEV ? -om : C(0);
    const C orho = om * rho;
    const C A = visit_shells(lam, [&](auto S_, C px, C mx, C py, C my, C pz,
                                      C mz, C e) {
        constexpr int S = decltype(S_)::value;
        const C q = (Store<ST>::DEV ? orho : orho * C(shell_weight(S))) * e;
        static_for<1, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (shell_of(i) == S) {
                const C p = pick<cx2(i)>(px, mx) * pick<cy2(i)>(py, my) *
                            pick<cz2(i)>(pz, mz);
                put(IC<i>{}, fma(q, p, fma(keep, v[i], shift)));
            }
        });
    });
    const C q0 = (Store<ST>::DEV ? orho : orho * C(shell_weight(0))) * A;
    put(IC<0>{}, fma(q0, C(1), fma(keep, v[0], shift)));
}


// ------------------------------------------------------- series equilibrium
// The series form of the equilibrium (Sec. III; Appendix B), accurate to
// O(u^3 eta^4), eta = theta / theta0 - 1:
//   f~_i = rho W~_i [1 + u.c / theta + f2_i + f3_i],  W~_i = w_i p_s(eta),
// p_s the quartic of Eq. (zeroveleqseries) in y_s = c_s^2 / theta0, and
// the second- and third-order terms corrected by R-bar, the departure of
// the fourth moments of the unit-density weights W~ from 3 theta^2 Delta.
// By cubic symmetry every fourth moment of a shell is A_s = sum w c_x^4,
// B_s = sum w c_x^2 c_y^2 or zero, so with A = sum_s p_s A_s and
// B = sum_s p_s B_s (compile-time lattice sums):
//   <W~, c^4> = 3 A + 6 B,  R-bar = (3 A + 6 B) / (15 theta^2) - 1,
//   t_k = R-bar_kabg u_a u_b u_g
//       = (A u_k^3 + 3 B u_k (u^2 - u_k^2)) / theta^2 - 3 u^2 u_k.
// Collecting powers of u.c, the bracket of direction i in shell s is
//   K0_s + K1_s (u.c) + (u.c)^2 / (2 theta^2) + (u.c)^3 / (6 theta^3)
//   - c.t / (6 theta^2),  with g = R-bar / (2 + 5 R-bar),
//   K0_s = 1 - u^2 / (2 theta) - (5/6) g u^2 (c_s^2 - 3 theta) / theta^2,
//   K1_s = 1 / theta - u^2 / (2 theta^2) + (5/6) u^2 R-bar / theta^2
//          - (5/6) g u^2 (c_s^2 - 3 theta) / theta^3.
// Mass, momentum and energy of f~ are those of the fluid (exactly, up to
// rounding).  It is used at a site only where every f~_i is positive
// (series_positive); elsewhere the step solves for the entropic
// equilibrium.
constexpr double shell_m4(int s, bool xxxx) {
    double a = 0.0;
    for (int i = 0; i < Q; ++i)
        if (shell_of(i) == s)
            a += weight(i) * (xxxx ? cx(i) * cx(i) * cx(i) * cx(i)
                                   : cx(i) * cx(i) * cy(i) * cy(i));
    return a;
}
// coefficients of p_s(eta) = 1 + a1 eta + a2 eta^2 + a3 eta^3 + a4 eta^4
constexpr double wpoly(int s, int n) {
    const double y = 0.25 * SHELL_C2X4[s] / THETA0;
    switch (n) {
    case 1: return (y - 3.0) / 2.0;
    case 2: return (y * y - 10.0 * y + 15.0) / 8.0;
    case 3: return (y * y * y - 21.0 * y * y + 105.0 * y - 105.0) / 48.0;
    default:
        return (y * y * y * y - 36.0 * y * y * y + 378.0 * y * y - 1260.0 * y +
                945.0) / 384.0;
    }
}

template <class C>
struct Series {
    C rho, eta, th, ux, uy, uz, u2, g, rb, tx, ty, tz;
    template <int S>
    __device__ __forceinline__ C p() const {  // p_S(eta)
        // (constexpr locals: evaluated by the compiler, not at run time)
        constexpr double a1 = wpoly(S, 1), a2 = wpoly(S, 2), a3 = wpoly(S, 3),
                         a4 = wpoly(S, 4);
        return fma(eta, fma(eta, fma(eta, fma(eta, C(a4), C(a3)), C(a2)), C(a1)),
                   C(1));
    }
};

template <class C>
__device__ __forceinline__ Series<C> series_of(const Moments &m) {
    Series<C> q;
    q.rho = C(m.rho);
    q.th = C(m.theta);
    q.eta = C(m.theta * (1.0 / THETA0) - 1.0);
    q.ux = C(m.ux);
    q.uy = C(m.uy);
    q.uz = C(m.uz);
    q.u2 = q.ux * q.ux + q.uy * q.uy + q.uz * q.uz;
    C A = C(0), B = C(0);
    static_for<1, NSHELL>([&](auto S_) {
        constexpr int s = S_;
        constexpr double as = shell_m4(s, true), bs = shell_m4(s, false);
        const C ps = q.template p<s>();
        A = fma(ps, C(as), A);
        B = fma(ps, C(bs), B);
    });
    const C ith2 = C(1) / (q.th * q.th);
    q.rb = (C(3) * A + C(6) * B) * ith2 * C(1.0 / 15.0) - C(1);
    q.g = q.rb / (C(2) + C(5) * q.rb);
    auto tk = [&](C uk) {
        return (A * uk * uk * uk + C(3) * B * uk * (q.u2 - uk * uk)) * ith2 -
               C(3) * q.u2 * uk;
    };
    q.tx = tk(q.ux);
    q.ty = tk(q.uy);
    q.tz = tk(q.uz);
    return q;
}

// fn(IC<i>, f~_i / w_i) for every direction
template <class C, class FN>
__device__ __forceinline__ void series_visit(const Series<C> &q, FN &&fn) {
    const C ith = C(1) / q.th;
    const C ith2 = ith * ith;
    const C k2 = C(0.5) * ith2, k3 = C(1.0 / 6.0) * ith2 * ith;
    const C gu = C(5.0 / 6.0) * q.g * q.u2 * ith2;  // (5/6) g u^2 / theta^2
    const C k0 = C(1) - C(0.5) * q.u2 * ith;
    const C k1 = ith - C(0.5) * q.u2 * ith2 + C(5.0 / 6.0) * q.rb * q.u2 * ith2;
    const C tfac = C(-1.0 / 6.0) * ith2;
    static_for<0, NSHELL>([&](auto S_) {
        constexpr int s = S_;
        constexpr double c2s = 0.25 * SHELL_C2X4[s];
        const C d = C(c2s) - C(3) * q.th;  // c_s^2 - 3 theta
        const C K0 = fma(-gu, d, k0);
        const C K1 = fma(-gu * ith, d, k1);
        const C rp = q.rho * q.template p<s>();
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (shell_of(i) == s) {
                constexpr double ax = cx(i), ay = cy(i), az = cz(i);
                C uc = C(0), ct = C(0);
                if constexpr (cx2(i) != 0) { uc = fma(C(ax), q.ux, uc); ct = fma(C(ax), q.tx, ct); }
                if constexpr (cy2(i) != 0) { uc = fma(C(ay), q.uy, uc); ct = fma(C(ay), q.ty, ct); }
                if constexpr (cz2(i) != 0) { uc = fma(C(az), q.uz, uc); ct = fma(C(az), q.tz, ct); }
                const C br = fma(uc, fma(uc, fma(uc, k3, k2), K1), fma(tfac, ct, K0));
                fn(IC<i>{}, rp * br);
            }
        });
    });
}

template <class C>
__device__ __forceinline__ bool series_positive(const Series<C> &q) {
    bool pos = true;
    series_visit(q, [&](auto, C fw) { pos = pos && fw > C(0); });
    return pos;
}

// f*_i = f_i + omega (f~_i - f_i), in storage form, through put(IC<i>, value)
template <int ST, class PUT>
__device__ __forceinline__ void relax_series(
    const Series<typename Store<ST>::C> &q, const typename Store<ST>::C v[Q],
    typename Store<ST>::C om, PUT &&put) {
    using C = typename Store<ST>::C;
    const C keep = C(1) - om;
    const C shift = Store<ST>::DEV ? -om : C(0);
    series_visit(q, [&](auto I_, C fw) {
        constexpr int i = decltype(I_)::value;
        constexpr double wi = weight(i);
        const C e = Store<ST>::DEV ? fw : C(wi) * fw;
        put(I_, fma(om, e, fma(keep, v[i], shift)));
    });
}

// ------------------------------------------------------- entropic collision
// h(y) = (1 + y) ln(1 + y) - y for y >= -1 (h(-1) = 1), given l = ln(1 + y);
// by its Taylor series sum_{n>=2} (-1)^n y^n / (n (n - 1)) for small |y|,
// where the closed form cancels.
template <class C>
__device__ __forceinline__ C hfun(C y, C l) {
    constexpr bool F64 = sizeof(C) == 8;
    constexpr int NT = F64 ? 14 : 8;  // highest power of the series
    if (fabs(y) < (F64 ? C(0.01) : C(0.05))) {
        C s = C(0);
        static_for<0, NT - 1>([&](auto K_) {  // Horner, from y^NT down to y^2
            constexpr int n = NT - int(K_);
            s = fma(s, y, C((n % 2 ? -1.0 : 1.0) / (double(n) * (n - 1))));
        });
        return s * y * y;
    }
    return y <= C(-1) ? C(1) : fma(C(1) + y, l, -y);
}

// ln(1 + y) in FP32 for y > -1, cheaply: for |y| < 0.05 its Taylor series
// (8 terms, truncation below 1e-11 relative); above, the hardware base-2
// logarithm of u = 1 + y with the rounding of u corrected to first order,
// ln u + (y - (u - 1)) / u (Goldberg, "What every computer scientist should
// know about floating-point arithmetic", 1991).  A few ulp, against ~80
// instructions of compensated arithmetic in the library's log1pf.
__device__ __forceinline__ float log1p_f32(float y) {
    if (fabsf(y) < 0.05f) {
        float s = -1.0f / 8.0f;  // sum_{n=1..8} (-1)^(n+1) y^n / n, Horner
        s = fmaf(s, y, 1.0f / 7.0f);
        s = fmaf(s, y, -1.0f / 6.0f);
        s = fmaf(s, y, 1.0f / 5.0f);
        s = fmaf(s, y, -1.0f / 4.0f);
        s = fmaf(s, y, 1.0f / 3.0f);
        s = fmaf(s, y, -1.0f / 2.0f);
        s = fmaf(s, y, 1.0f);
        return s * y;
    }
    const float u = 1.0f + y;
    const float c = y - (u - 1.0f);
    return fmaf(c, __builtin_amdgcn_rcpf(u),
                __builtin_amdgcn_logf(u) * 0.693147180559945309f);
}

// Calls fn(i, f_i, x_i) for every direction, x_i = (f_eq,i - f_i) / f_i,
// with f_eq from the multipliers (f_eq,i = rho w_i e_s X^2cx Y^2cy Z^2cz as
// in relax_all) and f_i from get(IC<i>) in storage form.
template <int ST, class GET, class FN>
__device__ __forceinline__ void for_each_deviation(
    const typename Store<ST>::C lam[5], typename Store<ST>::C rho, GET &&get,
    FN &&fn) {
    using C = typename Store<ST>::C;
    auto one = [&](auto I_, C qp) {  // qp = f_eq / w (dev) or f_eq (FP64)
        constexpr int i = decltype(I_)::value;
        const C v = get(I_);
        if constexpr (Store<ST>::DEV) {
            const C fw = C(1) + v;  // f / w
            fn(I_, C(weight(i)) * fw, (qp - fw) / fw);
        } else {
            fn(I_, v, (qp - v) / v);
        }
    };
    const C A = visit_shells(lam, [&](auto S_, C px, C mx, C py, C my, C pz,
                                      C mz, C e) {
        constexpr int S = decltype(S_)::value;
        const C q = (Store<ST>::DEV ? rho : rho * C(shell_weight(S))) * e;
        static_for<1, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (shell_of(i) == S)
                one(I_, q * (pick<cx2(i)>(px, mx) * pick<cy2(i)>(py, my) *
                             pick<cz2(i)>(pz, mz)));
        });
    });
    one(IC<0>{}, (Store<ST>::DEV ? rho : rho * C(shell_weight(0))) * A);
}

// Entropic alpha (Sec. II, Eq. delH): the positive root of
//   phi(alpha) = H[f + alpha (f_eq - f)] - H[f],  H[g] = sum g (ln(g/w) - 1),
// evaluated as phi = sum_i f_i [h(alpha x_i) - alpha x_i ln(1 + x_i)] (equal
// to the difference because f_eq carries the conserved moments of f and
// ln(f_eq / w) is a combination of 1, c and c^2; every term is of second
// order in x, so nothing cancels near equilibrium).  phi(0) = 0,
// phi'(0) < 0 and phi is convex: Newton's method from alpha = 2 inside the
// bracket (0, alpha_max), alpha_max = min over x_i < 0 of -1/x_i (the
// populations stay non-negative); bisection when a step leaves the bracket;
// alpha_max itself when phi is still negative there.  At equilibrium
// alpha = 2.  A site with a non-positive population gets alpha = 2 and sets
// LBM_FLAG_NEGATIVE.
template <int ST, class GET>
__device__ __forceinline__ typename Store<ST>::C entropic_alpha(
    const typename Store<ST>::C lam[5], typename Store<ST>::C rho, GET &&get,
    unsigned &bits) {
    using C = typename Store<ST>::C;
    constexpr bool F64 = sizeof(C) == 8;
    constexpr C TOL = F64 ? C(1e-14) : C(1e-6);
    constexpr int MAXIT = F64 ? 100 : 50;  // a root next to alpha_max converges slowly
    bool pos = true;
    C amax = C(INFINITY), scale = C(0);
    for_each_deviation<ST>(lam, rho, get, [&](auto, C f, C x) {
        pos = pos && f > C(0);
        scale = fma(f * x, x, scale);
        if (x < C(0)) amax = fmin(amax, C(-1) / x);
    });
    if (!pos) {
        bits |= LBM_FLAG_NEGATIVE;
        return C(2);
    }
    if (!(scale > C(0))) return C(2);
    auto eval = [&](C a, C &ph, C &dph) {
        ph = C(0);
        dph = C(0);
        for_each_deviation<ST>(lam, rho, get, [&](auto, C f, C x) {
            const C y = a * x;
            const C l1 = log1p(x);
            const C ly = y <= C(-1) ? C(-INFINITY) : log1p(y);
            ph = fma(f, hfun(y, ly) - y * l1, ph);
            dph = fma(f * x, ly - l1, dph);
        });
    };
    C lo = C(0), hi = amax, ph, dph, a;
    bool max_checked = false;
    if (amax <= C(2)) {
        eval(amax, ph, dph);
        if (ph <= C(0)) return amax;
        max_checked = true;
        a = C(0.5) * amax;
    } else {
        a = C(2);
    }
    for (int it = 0; it < MAXIT; ++it) {
        eval(a, ph, dph);
        if (ph < C(0))
            lo = a;
        else
            hi = a;
        C an = a - ph / dph;
        if (ph == C(0) || fabs(an - a) <= TOL * a) return an;
        if (!(an > lo && an < hi)) {
            if (!max_checked && !(an < hi) && hi == amax) {
                // the root may lie beyond alpha_max: is phi still negative?
                C pm, dm;
                eval(amax, pm, dm);
                max_checked = true;
                if (pm <= C(0)) return amax;
            }
            an = C(0.5) * (lo + hi);
        }
        if (hi - lo <= TOL * a) return an;
        a = an;
    }
    return a;
}

// Entropic alpha for the FP32-compute forms, with the 81 relative departures
// x_i held in registers beside the deviations h_i (get(IC<i>), from
// registers or the thread's LDS column).  Same root as
// entropic_alpha (Sec. II, Eq. delH), reached without re-deriving f_eq in
// every evaluation:
//  * one pass over the shells of the equilibrium writes x_i to xv (for a
//    non-positive population the plain difference f_eq,i/w_i - f_i/w_i is
//    written instead, and alpha = 2 is returned with LBM_FLAG_NEGATIVE) and
//    sums s1 = sum f x ln(1 + x);
//  * phi(a) = sum f h(a x) - a s1 and phi'(a) = sum f x ln(1 + a x) - s1:
//    one logarithm (log1p_f32) per direction and evaluation.  Both sums are
//    of the order of sum f x^2, and so is their rounding error, as is phi',
//    so the root moves by a few ulps only; divisions are reciprocal
//    multiplies (1 ulp);
//  * the search takes the same steps as entropic_alpha, written as one
//    evaluation per pass (`at_max`: the pass is the check at alpha_max) so
//    that the evaluation has a single call site and is inlined: called as a
//    function it could reach the register-resident values only through a
//    copy on the stack.
template <int ST, class GET>
__device__ __forceinline__ float entropic_alpha_x(const float lam[5],
                                                  float rho, GET &&get,
                                                  float xv[Q],
                                                  unsigned &bits) {
    using C = float;
    static_assert(Store<ST>::DEV && sizeof(typename Store<ST>::C) == 4,
                  "deviation storage with FP32 arithmetic");
    constexpr C TOL = C(1e-6);
    constexpr int MAXIT = 50;
    bool pos = true;
    C amax = C(INFINITY), scale = C(0), s1 = C(0);
    auto one = [&](auto I_, C qp) {  // qp = f_eq,i / w_i
        constexpr int i = decltype(I_)::value;
        const C fw = C(1) + get(I_);  // f_i / w_i
        const C d = qp - fw;
        const bool p = fw > C(0);
        pos = pos && p;
        const C x = p ? d * __builtin_amdgcn_rcpf(fw) : d;
        xv[i] = x;
        const C f = C(weight(i)) * fw;
        scale = fma(f * x, x, scale);
        s1 = fma(f * x, log1p_f32(x), s1);
        if (x < C(0)) amax = fmin(amax, -__builtin_amdgcn_rcpf(x));
    };
    const C A = visit_shells(lam, [&](auto S_, C px, C mx, C py, C my, C pz,
                                      C mz, C e) {
        constexpr int S = decltype(S_)::value;
        const C q = rho * e;
        static_for<1, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (shell_of(i) == S)
                one(I_, q * (pick<cx2(i)>(px, mx) * pick<cy2(i)>(py, my) *
                             pick<cz2(i)>(pz, mz)));
        });
    });
    one(IC<0>{}, rho * A);
    if (!pos) {
        bits |= LBM_FLAG_NEGATIVE;
        return C(2);
    }
    if (!(scale > C(0))) return C(2);
    // four interleaved partial sums: the 81 terms are independent, and one
    // running sum would chain 81 dependent FMAs per evaluation
    auto eval = [&](C a, C &ph, C &dph) __attribute__((always_inline)) {
        C p4[4] = {C(0), C(0), C(0), C(0)}, d4[4] = {C(0), C(0), C(0), C(0)};
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            const C x = xv[i];
            const C f = C(weight(i)) * (C(1) + get(I_));
            const C y = a * x;
            const C ly = y <= C(-1) ? C(-INFINITY) : log1p_f32(y);
            p4[i % 4] = fma(f, hfun(y, ly), p4[i % 4]);
            d4[i % 4] = fma(f * x, ly, d4[i % 4]);
        });
        ph = fma(-a, s1, (p4[0] + p4[1]) + (p4[2] + p4[3]));
        dph = ((d4[0] + d4[1]) + (d4[2] + d4[3])) - s1;
    };
    C lo = C(0), hi = amax, a, next = C(0);
    bool max_checked = false, at_max = false, stop_next = false;
    if (amax <= C(2)) {
        a = amax;
        at_max = true;
        next = C(0.5) * amax;
    } else {
        a = C(2);
    }
    // MAXIT Newton iterates at most, plus the one check at alpha_max
    for (int it = 0; it < MAXIT || at_max;) {
        C ph, dph;
        eval(a, ph, dph);
        if (at_max) {
            at_max = false;
            max_checked = true;
            if (ph <= C(0) || stop_next) return ph <= C(0) ? amax : next;
            a = next;
            continue;
        }
        ++it;
        if (ph < C(0))
            lo = a;
        else
            hi = a;
        const C newton = a - ph / dph;
        C an = newton;
        if (ph == C(0) || fabs(an - a) <= TOL * a) return an;
        if (!(an > lo && an < hi)) {
            an = C(0.5) * (lo + hi);
            if (!max_checked && !(newton < hi) && hi == amax) {
                // the step overshoots alpha_max: check it, then bisect
                stop_next = hi - lo <= TOL * a;
                next = an;
                at_max = true;
                a = amax;
                continue;
            }
        }
        if (hi - lo <= TOL * a) return an;
        a = an;
    }
    return a;
}

// The entropic step of the FP32-compute forms keeps x_i resident beside the
// populations (entropic_alpha_x) and has the registers of 2 waves per SIMD.
template <int ST, bool ENT>
constexpr bool ent_resident() {
    return ENT && sizeof(typename Store<ST>::C) == 4;
}
template <int ST, bool ENT>
constexpr int step_waves() {
    return ent_resident<ST, ENT>() ? 2 : Store<ST>::WAVES;
}
// Populations parked in the thread's LDS column during the solves (see
// site_update).  The resident entropic step parks all 81, since its
// registers hold the 81 x_i: with any of the populations left in registers
// the compiler keeps the whole array in scratch memory instead (0.7-1.2 KB
// per lane), and the step becomes bound by the latency of those accesses.
// Its workgroups have 64 lanes (one wavefront, 20.7 KB of LDS), so that
// seven share a CU; with 256 lanes (83 KB) only one fits.
template <int ST, bool ENT>
constexpr int park_count() {
    return ent_resident<ST, ENT>() ? Q : Store<ST>::NLDS;
}
template <int ST, bool ENT>
constexpr int step_block() {
    return ent_resident<ST, ENT>() ? 64 : BLOCK;
}

// Directions whose odd-step destination x differs from the source x (for
// some sub-lattice): every half link and every integer link with c_x != 0.
// Only these go through the LDS exchange of site_update; xch_slot numbers
// them consecutively.
constexpr bool needs_xch(int i) { return is_half(i) || cx2(i) != 0; }
constexpr int xch_slot(int i) {
    int k = 0;
    for (int j = 0; j < i; ++j) k += needs_xch(j) ? 1 : 0;
    return k;
}
constexpr int NXCH = xch_slot(Q);
static_assert(NXCH == 56, "8 SC + 16 FCC + 32 BCC directions move along x");
// Also route the (equally shifted) odd-step loads through the exchange.
constexpr bool XCH_LOADS = true;

// One site update: moments -> equilibrium -> relax -> stream (AA pattern).
//
// The 81 populations must survive the equilibrium solve, which needs many
// registers itself.  The last NL of them are parked in this thread's own
// LDS column meanwhile (no other thread reads them, so no barrier), which
// keeps the kernel at its occupancy target without spilling to scratch
// memory.  LDS per workgroup: NL x BLOCK values (park_count).
//
// XCH (odd step, 16-bit storage, every workgroup covering whole rows): the
// odd step writes direction i at x + c_i, so a wavefront's 64 stores are
// shifted against the 128-byte lines and every store instruction splits
// into two partial lines, which costs a third of the store bandwidth.
// Instead each lane puts its post-collision values at their destination x
// in a row buffer in LDS (overlaying the parking area once every lane has
// re-read its parked values), and after a barrier each lane stores the
// values that land on its own x, so every wavefront store covers whole
// lines.  Same values, same addresses; only which lane stores what changes.
//
// `lds` is the workgroup's LDS buffer of lds_bytes<ST, XCH, ENT>() bytes.
template <int ST, bool XCH, bool ENT = false>
constexpr size_t lds_bytes() {
    using C = typename Store<ST>::C;
    using T = typename Store<ST>::T;
    constexpr size_t park =
        size_t(park_count<ST, ENT>()) * step_block<ST, ENT>() * sizeof(C);
    constexpr size_t xbuf = XCH ? size_t(NXCH) * BLOCK * sizeof(T) : 0;
    return park > xbuf ? park : xbuf;
}

template <int ST, bool ODD, bool XCH, bool ENT, class AD, bool SER = false>
__device__ __forceinline__ void site_update(const AD &ad, double omega,
                                            unsigned *flags,
                                            unsigned char *lds) {
    static_assert(!SER || (!XCH && !ENT), "the series step is a plain BGK step");
    using C = typename Store<ST>::C;
    using T = typename Store<ST>::T;
    constexpr int NL = park_count<ST, ENT>();
    constexpr int BS = step_block<ST, ENT>();
    static_assert(!XCH || BS == BLOCK, "the row exchange spans BLOCK lanes");
    C(*park)[BS] = reinterpret_cast<C(*)[BS]>(lds);
    C v[Q];
    if constexpr (XCH && XCH_LOADS) {
        // each lane loads its own x of every source row (whole-line loads)
        // into the row buffer and then takes its value at x - c_i from it
        // planes: a lane's x offsets are wrap(x + k) * sizeof(T)
        static_assert(!Store<ST>::TILED, "exchange positions assume planes");
        T *xb = reinterpret_cast<T *>(lds);
        // byte offset of this lane's row in a direction's row buffer
        const uint32_t rb = uint32_t(threadIdx.x * sizeof(T)) - ad.xo[4];
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (needs_xch(i)) {
                constexpr int slot = xch_slot(i);  // a compile-time constant
                xb[slot * BLOCK + threadIdx.x] =
                    *byte_off(ad.template nbr_row<i, true, opp(i)>(), ad.xo[4]);
            }
        });
        __syncthreads();
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (needs_xch(i)) {
                constexpr int slot = xch_slot(i);
                v[i] = Store<ST>::load(byte_off(xb + slot * BLOCK,
                                                rb + ad.template nbr_x<i, true>()));
            } else  // same x: a whole-line load already
                v[i] = Store<ST>::load(ad.template nbr<i, true, opp(i)>());
        });
        __syncthreads();  // the buffer becomes the parking area
    } else {
        gather<ST, ODD>(ad, v);
    }
    const Moments m = moments_of<ST>(v);
    static_for<Q - NL, Q>([&](auto I_) {
        constexpr int i = I_;
        park[i - (Q - NL)][threadIdx.x] = v[i];
    });
    // compiler barrier: the parked values must be re-read from LDS, not kept
    // in registers across the solve
    asm volatile("" ::: "memory");
    unsigned bits = 0;
    C lam[5] = {C(0), C(0), C(0), C(0), C(0)};
    C om = C(omega);
    // series equilibrium where it is positive (SER), else the Newton solve
    Series<C> sq{};
    bool ser = false;
    if constexpr (SER) {
        if (m.ok) {
            sq = series_of<C>(m);
            ser = series_positive(sq);
        }
    }
    if (m.ok) {
        if (!ser && solve_multipliers<C>(C(m.ux), C(m.uy), C(m.uz), C(m.e),
                                         C(m.theta), lam) < 0)
            bits |= LBM_FLAG_NEWTON;
    } else {
        bits |= isfinite(m.rho) && isfinite(m.theta) ? LBM_FLAG_UNREALIZABLE
                                                     : LBM_FLAG_NONFINITE;
        om = C(0);  // the site keeps its populations
    }
    if constexpr (ENT && !ent_resident<ST, ENT>()) {
        // alpha beta = (alpha / 2) omega; the parked values are read from
        // LDS where the search needs them
        if (m.ok) {
            const C alpha = entropic_alpha<ST>(
                lam, C(m.rho),
                [&](auto I_) -> C {
                    constexpr int i = decltype(I_)::value;
                    if constexpr (i < Q - NL)
                        return v[i];
                    else
                        return park[i - (Q - NL)][threadIdx.x];
                },
                bits);
            om *= C(0.5) * alpha;
        }
    }
    asm volatile("" ::: "memory");
    if constexpr (!ent_resident<ST, ENT>()) {
        static_for<Q - NL, Q>([&](auto I_) {
            constexpr int i = I_;
            v[i] = park[i - (Q - NL)][threadIdx.x];
        });
    }
    AD wr = ad;
    wr.launder();
    if constexpr (ent_resident<ST, ENT>()) {
        static_assert(!XCH, "the entropic step stores directly");
        // h*_i = h_i + (alpha / 2) omega (f_eq,i - f_i) / w_i with
        // (f_eq,i - f_i) / w_i = x_i f_i / w_i (or the plain difference,
        // kept in xv, at a non-positive population)
        // the parked deviations stay in the thread's LDS column
        auto hv = [&](auto I_) -> C {
            constexpr int i = decltype(I_)::value;
            if constexpr (i < Q - NL)
                return v[i];
            else
                return park[i - (Q - NL)][threadIdx.x];
        };
        C xv[Q];
        C ome = C(0);
        if (m.ok) {
            const C alpha = entropic_alpha_x<ST>(lam, C(m.rho), hv, xv, bits);
            ome = om * C(0.5) * alpha;
        } else {
            static_for<0, Q>([&](auto I_) { xv[decltype(I_)::value] = C(0); });
        }
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            const C h = hv(I_);
            const C fw = C(1) + h;
            const C out = fma(ome, fw > C(0) ? xv[i] * fw : xv[i], h);
            if constexpr (ODD)
                Store<ST>::store(wr.template nbr<i, false, i>(), out);
            else
                Store<ST>::store(wr.template own<opp(i)>(), out);
        });
    } else if constexpr (XCH) {
        static_assert(ODD, "the exchange serves the shifted odd-step stores");
        // every lane of the workgroup gets here (whole rows, no idle lane)
        __syncthreads();  // parked values re-read: the LDS is free
        T *xb = reinterpret_cast<T *>(lds);
        const uint32_t rb = uint32_t(threadIdx.x * sizeof(T)) - wr.xo[4];
        relax_all<ST>(lam, v, C(m.ok ? m.rho : 1.0), om, [&](auto I_, C out) {
            constexpr int i = decltype(I_)::value;
            constexpr int slot = xch_slot(i);
            if constexpr (needs_xch(i))
                Store<ST>::store(byte_off(xb + slot * BLOCK,
                                          rb + wr.template nbr_x<i, false>()),
                                 out);
            else  // lands on the same x: already a whole-line store
                Store<ST>::store(wr.template nbr<i, false, i>(), out);
        });
        __syncthreads();
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (needs_xch(i)) {
                constexpr int slot = xch_slot(i);
                const T val = xb[slot * BLOCK + threadIdx.x];
                *byte_off(wr.template nbr_row<i, false, i>(), wr.xo[4]) = val;
            }
        });
    } else {
        auto put = [&](auto I_, C out) {
            constexpr int i = decltype(I_)::value;
            if constexpr (ODD)
                Store<ST>::store(wr.template nbr<i, false, i>(), out);
            else
                Store<ST>::store(wr.template own<opp(i)>(), out);
        };
        if (SER && ser)
            relax_series<ST>(sq, v, om, put);
        else
            relax_all<ST>(lam, v, C(m.ok ? m.rho : 1.0), om, put);
    }
    flag_or(flags, bits);
}

// ------------------------------------------------------------------ kernels
template <int ST, bool ODD, int MODE, bool ENT, bool SER = false>
// (The second bound is in workgroups per CU: step_waves waves per SIMD.)
__global__ __launch_bounds__((step_block<ST, ENT>()),
                             (step_waves<ST, ENT>() * 256 / step_block<ST, ENT>()))
void k_step(typename Store<ST>::T *F,
                                                Geom g, double omega,
                                                unsigned *flags) {
    using T = typename Store<ST>::T;
    constexpr uint32_t BS = step_block<ST, ENT>();
    __shared__ __align__(16) unsigned char lds[lds_bytes<ST, MODE == ROWX, ENT>()];
    const uint32_t tile = plain_order<ST, ODD, ENT>()
                              ? uint32_t(blockIdx.x)
                              : xcd_tile(blockIdx.x, gridDim.x);
    if constexpr (MODE == ROWX) {
        // the host launches ROWX only where every lane holds a site
        static_assert(ODD && Store<ST>::XCH, "ROWX kernel");
        site_update<ST, ODD, true, ENT>(Addr<T, ROW>(F, g, row_site(g, tile, BS / 64)),
                                        omega, flags, lds);
    } else if constexpr (MODE == ROW) {
        const RowSite r = row_site(g, tile, BS / 64);
        if (!r.active) return;
        site_update<ST, ODD, false, ENT, Addr<T, ROW>, SER>(
            Addr<T, ROW>(F, g, r), omega, flags, lds);
    } else {
        const uint32_t s = tile * BS + threadIdx.x;
        if (s >= g.nsites) return;
        site_update<ST, ODD, false, ENT, Addr<T, MODE>, SER>(
            Addr<T, MODE>(F, g, s), omega, flags, lds);
    }
}

// f = f_eq(rho, u, theta), solved in FP64, natural slots (step count 0).
template <int ST>
__global__ __launch_bounds__(BLOCK) void k_init(typename Store<ST>::T *F,
                                                Geom g, const double *rho,
                                                const double *u,
                                                const double *theta,
                                                unsigned *flags) {
    const uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.nsites) return;
    const double r = rho[s], ux = u[s], uy = u[g.nsites + s],
                 uz = u[2 * size_t(g.nsites) + s], th = theta[s];
    const bool ok = r > 0.0 && th > 0.0 && isfinite(r) && isfinite(th) &&
                    isfinite(ux) && isfinite(uy) && isfinite(uz);
    double lam[5] = {0, 0, 0, 0, 0};
    unsigned bits = 0;
    if (ok) {
        if (solve_multipliers<double>(ux, uy, uz,
                                      ux * ux + uy * uy + uz * uz + 3.0 * th,
                                      th, lam) < 0)
            bits |= LBM_FLAG_NEWTON;
    } else {
        bits |= LBM_FLAG_UNREALIZABLE;
    }
    const double rr = ok ? r : 1.0;
    const uint64_t base = site_el(g, s);
    using C = typename Store<ST>::C;
    auto put = [&](auto I_, double fw) {  // fw = f_eq / w
        constexpr int i = decltype(I_)::value;
        const C out = Store<ST>::DEV ? C(fw - 1.0) : C(weight(i) * fw);
        Store<ST>::store(F + base + uint64_t(i) * g.ss, out);
    };
    const double A = visit_shells(lam, [&](auto S_, double px, double mx,
                                           double py, double my, double pz,
                                           double mz, double e) {
        constexpr int S = decltype(S_)::value;
        static_for<1, Q>([&](auto I_) {
            constexpr int i = I_;
            if constexpr (shell_of(i) == S)
                put(I_, rr * e * (pick<cx2(i)>(px, mx) * pick<cy2(i)>(py, my) *
                                  pick<cz2(i)>(pz, mz)));
        });
    });
    put(IC<0>{}, rr * A);
    flag_or(flags, bits);
}

// Per-site FP64 moments and/or populations of the current state.
template <int ST, bool ODD, int MODE>
__global__ __launch_bounds__(BLOCK) void k_gather(typename Store<ST>::T *F,
                                                  Geom g, double *rho,
                                                  double *u, double *theta,
                                                  double *fout) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    C v[Q];
    uint32_t s;
    if constexpr (MODE == ROW) {
        const RowSite r = row_site(g, blockIdx.x);
        if (!r.active) return;
        s = site_index(g, r);
        gather<ST, ODD>(Addr<T, ROW>(F, g, r), v);
    } else {
        s = blockIdx.x * BLOCK + threadIdx.x;
        if (s >= g.nsites) return;
        gather<ST, ODD>(Addr<T, MODE>(F, g, s), v);
    }
    double f[Q];
    static_for<0, Q>([&](auto I_) {
        constexpr int i = I_;
        f[i] = Store<ST>::DEV ? weight(i) * (1.0 + double(v[i])) : double(v[i]);
    });
    if (fout) {
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            fout[size_t(i) * g.nsites + s] = f[i];
        });
    }
    if (rho || u || theta) {
        double r = 0, jx = 0, jy = 0, jz = 0, en = 0;
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            r += f[i];
            if constexpr (cx2(i) != 0) jx += cx(i) * f[i];
            if constexpr (cy2(i) != 0) jy += cy(i) * f[i];
            if constexpr (cz2(i) != 0) jz += cz(i) * f[i];
            en += csq(i) * f[i];
        });
        const double ux = jx / r, uy = jy / r, uz = jz / r;
        if (rho) rho[s] = r;
        if (u) {
            u[s] = ux;
            u[g.nsites + s] = uy;
            u[2 * size_t(g.nsites) + s] = uz;
        }
        if (theta) theta[s] = (en / r - (ux * ux + uy * uy + uz * uz)) / 3.0;
    }
}

// Block-wise FP64 totals in a fixed order.  The memory holds every
// population of the current state once; at odd parity direction i sits in
// slot opp(i), which only flips the sign of the momentum.
template <int ST>
__global__ __launch_bounds__(BLOCK) void k_totals_part(
    const typename Store<ST>::T *F, Geom g, int odd, double *part) {
    __shared__ double sh[5][BLOCK];
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < g.nsites;
         s += TOT_BLOCKS * BLOCK) {
        double r = 0, jx = 0, jy = 0, jz = 0, en = 0;
        const uint64_t base = site_el(g, s);
        static_for<0, Q>([&](auto I_) {
            constexpr int i = I_;
            const double v = double(Store<ST>::load(F + base + uint64_t(i) * g.ss));
            const double f = Store<ST>::DEV ? weight(i) * (1.0 + v) : v;
            r += f;
            if constexpr (cx2(i) != 0) jx += cx(i) * f;
            if constexpr (cy2(i) != 0) jy += cy(i) * f;
            if constexpr (cz2(i) != 0) jz += cz(i) * f;
            en += csq(i) * f;
        });
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += jz;
        acc[4] += en;
    }
    const double sign = odd ? -1.0 : 1.0;
    acc[1] *= sign;
    acc[2] *= sign;
    acc[3] *= sign;
    for (int a = 0; a < 5; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < unsigned(w))
            for (int a = 0; a < 5; ++a)
                sh[a][threadIdx.x] += sh[a][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) part[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

static __global__ __launch_bounds__(BLOCK) void k_totals_final(const double *part,
                                                        double *out) {
    __shared__ double sh[5][BLOCK];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < TOT_BLOCKS; b += BLOCK)
        for (int a = 0; a < 5; ++a) acc[a] += part[b * 5 + a];
    for (int a = 0; a < 5; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < unsigned(w))
            for (int a = 0; a < 5; ++a)
                sh[a][threadIdx.x] += sh[a][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

// Batched step over many resident simulations (serving): tiles of BLOCK
// sites are numbered consecutively over the simulations (BatchArgs), one
// workgroup per tile in the plain step's XCD-aware order, and a binary
// search over the descriptors' first tiles finds the tile's simulation.
// (A persistent grid that loops over the tiles, strided or in contiguous
// ranges per workgroup, ran 5-20 % slower than the plain step on the same
// grids; one workgroup per tile matches it.)  Every simulation of one launch
// is at the same streaming parity, and in an odd-step launch of a 16-bit
// form either every simulation takes the LDS row exchange of the odd step
// (XCHK: its workgroups cover whole rows, as in the plain ROWX step) or none
// does; the host groups them so.  Keeping the two odd-step paths in
// separate kernels matters: compiled together, the register allocation of
// the combined kernel issued the row path's 81 loads one at a time (a wait
// for each load before the next), and the batched odd step ran at a third
// of the plain step's rate.  A tile belongs to one simulation, so the whole
// workgroup takes the same path.
template <int ST, bool ODD, bool XCHK>
__global__ __launch_bounds__(BLOCK, Store<ST>::WAVES) void k_step_batch(BatchArgs a) {
    using T = typename Store<ST>::T;
    static_assert(!XCHK || (ODD && Store<ST>::XCH), "the exchange serves odd steps");
    __shared__ __align__(16) unsigned char lds[lds_bytes<ST, XCHK>()];
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    // the last simulation whose first tile is at or before this one
    int lo = 0, hi = a.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.d[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    const BatchDesc &d = a.d[lo];
    const RowSite r = row_site(d.g, tile - d.tile0);
    if constexpr (XCHK) {  // every lane of the tile holds a site
        site_update<ST, ODD, true, false>(
            Addr<T, ROW>(static_cast<T *>(d.f), d.g, r), d.omega, d.flags, lds);
    } else if (r.active) {
        site_update<ST, ODD, false, false>(
            Addr<T, ROW>(static_cast<T *>(d.f), d.g, r), d.omega, d.flags, lds);
    }
}

// ---------------------------------------------------------------- launchers
// One step of the whole grid.  The entropic collision is compute-bound, so
// its odd step keeps the plain row addressing (no LDS exchange).
template <int ST, bool ENT, bool SER = false>
void launch_step(void *f, const Geom &g, double omega, unsigned *flags,
                 bool odd, hipStream_t stream) {
    auto *F = static_cast<typename Store<ST>::T *>(f);
    constexpr int BS = step_block<ST, ENT>();
    const dim3 grid(sweep_blocks(g, BS)), block(BS);
    const int mode = mode_of(g);
#define LBM_STEP(ODD, MODE)                                                  \
    hipLaunchKernelGGL((k_step<ST, ODD, MODE, ENT, SER>), grid, block, 0,    \
                       stream, F, g, omega, flags)
    if (odd) {
        if constexpr (Store<ST>::XCH && !ENT && !SER) {
            if (mode == ROWX) {
                LBM_STEP(true, ROWX);
                return;
            }
        }
        if (mode != SMALL) LBM_STEP(true, ROW);
        else LBM_STEP(true, SMALL);
    } else {
        if (mode != SMALL) LBM_STEP(false, ROW);
        else LBM_STEP(false, SMALL);
    }
#undef LBM_STEP
}

// The series-equilibrium kernels likewise (kernels_<storage>_ser.hip); they
// take the plain row addressing.
template <int ST>
void launch_step_series(void *f, const Geom &g, double omega,
                        unsigned *flags, bool odd, hipStream_t stream) {
    launch_step<ST, false, true>(f, g, omega, flags, odd, stream);
}

template <int ST>
void Launch<ST>::step(void *f, const Geom &g, double omega, unsigned *flags,
                      bool odd, int collision, hipStream_t stream) {
    if (collision == LBM_COLLIDE_ENTROPIC)
        launch_step_entropic<ST>(f, g, omega, flags, odd, stream);
    else if (collision == LBM_COLLIDE_SERIES)
        launch_step_series<ST>(f, g, omega, flags, odd, stream);
    else
        launch_step<ST, false>(f, g, omega, flags, odd, stream);
}

template <int ST>
void Launch<ST>::init(void *f, const Geom &g, const double *rho,
                      const double *u, const double *theta, unsigned *flags,
                      hipStream_t stream) {
    auto *F = static_cast<typename Store<ST>::T *>(f);
    hipLaunchKernelGGL((k_init<ST>), dim3((g.nsites + BLOCK - 1) / BLOCK),
                       dim3(BLOCK), 0, stream, F, g, rho, u, theta, flags);
}

template <int ST>
void Launch<ST>::gather(void *f, const Geom &g, bool odd, double *rho,
                        double *u, double *theta, double *fout,
                        hipStream_t stream) {
    auto *F = static_cast<typename Store<ST>::T *>(f);
    const dim3 grid(sweep_blocks(g)), block(BLOCK);
    const int mode = mode_of(g);
#define LBM_GATHER(ODD, MODE)                                                 \
    hipLaunchKernelGGL((k_gather<ST, ODD, MODE>), grid, block, 0, stream, F, \
                       g, rho, u, theta, fout)
    if (odd) {
        if (mode != SMALL) LBM_GATHER(true, ROW);
        else LBM_GATHER(true, SMALL);
    } else {
        if (mode != SMALL) LBM_GATHER(false, ROW);
        else LBM_GATHER(false, SMALL);
    }
#undef LBM_GATHER
}

template <int ST>
void Launch<ST>::totals(const void *f, const Geom &g, bool odd, void *ws,
                        hipStream_t stream) {
    const auto *F = static_cast<const typename Store<ST>::T *>(f);
    char *w = static_cast<char *>(ws);
    hipLaunchKernelGGL((k_totals_part<ST>), dim3(TOT_BLOCKS), dim3(BLOCK), 0,
                       stream, F, g, int(odd),
                       reinterpret_cast<double *>(w + WS_PART));
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(BLOCK), 0, stream,
                       reinterpret_cast<const double *>(w + WS_PART),
                       reinterpret_cast<double *>(w + WS_OUT));
}

template <int ST>
void Launch<ST>::batch(const BatchArgs &a, bool odd, bool xch,
                       hipStream_t stream) {
    // one workgroup per tile of every simulation in the batch
    const dim3 grid(a.ntiles);
    if (odd && xch) {
        if constexpr (Store<ST>::XCH)
            hipLaunchKernelGGL((k_step_batch<ST, true, true>), grid,
                               dim3(BLOCK), 0, stream, a);
    } else if (odd) {
        hipLaunchKernelGGL((k_step_batch<ST, true, false>), grid,
                           dim3(BLOCK), 0, stream, a);
    } else {
        hipLaunchKernelGGL((k_step_batch<ST, false, false>), grid,
                           dim3(BLOCK), 0, stream, a);
    }
}

}  // namespace lbm81
