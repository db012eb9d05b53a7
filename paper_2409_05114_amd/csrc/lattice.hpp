// RD3Q81 velocity set and weights, built at compile time (Table "tab:weights"
// of Atif et al., arXiv:2409.05114).
//
// Directions are ordered so that the kernels can address a direction and its
// opposite without a table: 0 is rest, 1..40 are one representative of every
// +-pair and d + 40 is the opposite of d.  Velocities are stored doubled
// (2 c_i), so every component is a small integer; a direction is
// "half-integer" (moves between the corner and centre sub-lattices) when its
// doubled components are odd.
//
// Shells (index, kind, per-component magnitude):
//   0 rest; 1..4 SC-k, k = 1..4; 5, 6 FCC-k, k = 1, 2;
//   7..10 BCC-h, h = 1/2, 1, 3/2, 5/2.
// The weights are the degree-5 polynomials of the table evaluated at
// theta0 in double-double arithmetic and rounded once, and the rest weight is
// 1 minus the sum of the others (mass trace <w, 1> = 1, Sec. III).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm81 {

constexpr int Q = 81;
constexpr int NPAIR = 40;
constexpr int NSHELL = 11;

// ------------------------------------------------ double-double arithmetic
// Error-free transformations (Dekker / Knuth) usable in constant
// expressions, so host and device passes fold to the same doubles.
struct DD {
    double hi, lo;
};

constexpr DD two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

constexpr DD split(double a) {
    double t = 134217729.0 * a;  // 2^27 + 1
    double hi = t - (t - a);
    return {hi, a - hi};
}

constexpr DD two_prod(double a, double b) {
    double p = a * b;
    DD sa = split(a), sb = split(b);
    double e = ((sa.hi * sb.hi - p) + sa.hi * sb.lo + sa.lo * sb.hi) +
               sa.lo * sb.lo;
    return {p, e};
}

constexpr DD dd_add(DD a, DD b) {
    DD s = two_sum(a.hi, b.hi);
    double e = s.lo + a.lo + b.lo;
    return two_sum(s.hi, e);
}

constexpr DD dd_mul(DD a, DD b) {
    DD p = two_prod(a.hi, b.hi);
    double e = p.lo + (a.hi * b.lo + a.lo * b.hi);
    return two_sum(p.hi, e);
}

constexpr DD dd_div(DD a, double d) {
    double q1 = a.hi / d;
    DD p = two_prod(q1, d);
    DD r = dd_add(a, DD{-p.hi, -p.lo});
    double q2 = r.hi / d;
    return two_sum(q1, q2);
}

// theta0 = 0.821035006329447750282591763 (caption of Table "tab:weights"),
// split into the nearest double and the remainder.
constexpr DD THETA0_DD{0.8210350063294477, 4.729410296325315e-17};
constexpr double THETA0 = THETA0_DD.hi;

// (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) / d at t = theta0 (Horner).
constexpr DD weight_poly(double a1, double a2, double a3, double a4, double a5,
                         double d) {
    DD p{a5, 0.0};
    p = dd_add(dd_mul(p, THETA0_DD), DD{a4, 0.0});
    p = dd_add(dd_mul(p, THETA0_DD), DD{a3, 0.0});
    p = dd_add(dd_mul(p, THETA0_DD), DD{a2, 0.0});
    p = dd_add(dd_mul(p, THETA0_DD), DD{a1, 0.0});
    p = dd_mul(p, THETA0_DD);
    return dd_div(p, d);
}

// Shell weights in double-double, Table "tab:weights".
constexpr DD SHELL_W_DD[NSHELL] = {
    {0.0, 0.0},  // rest: filled from the mass trace below
    weight_poly(388800, -2508408, 7033852, -7856469, 2838528, 486000),
    weight_poly(-388800, 3091608, -8269102, 8694819, -2838528, 3888000),
    weight_poly(388800, -3199608, 8977852, -9120069, 2838528, 30618000),
    weight_poly(-97200, 809352, -2315338, 2396961, -709632, 108864000),
    weight_poly(0, 0, 8, -9, 0, 12),
    weight_poly(0, 0, -2, 9, 0, 768),
    weight_poly(0, 24300, -103834, 126963, -44352, 7776),
    weight_poly(0, -24300, 189022, -328275, 177408, 272160),
    weight_poly(0, 2700, -24778, 67995, -44352, 699840),
    weight_poly(0, -972, 11818, -43371, 44352, 68040000),
};

constexpr int SHELL_SIZE[NSHELL] = {1, 6, 6, 6, 6, 12, 12, 8, 8, 8, 8};
// per-component magnitude of the shell, doubled (2k or 2h)
constexpr int SHELL_N[NSHELL] = {0, 2, 4, 6, 8, 2, 4, 1, 2, 3, 5};
// |c|^2 of the shell, times 4 (an integer for every shell)
constexpr int SHELL_C2X4[NSHELL] = {0, 4, 16, 36, 64, 8, 32, 3, 12, 27, 75};
enum ShellKind { REST = 0, SC = 1, FCC = 2, BCC = 3 };
constexpr int SHELL_KIND[NSHELL] = {REST, SC, SC, SC, SC, FCC, FCC,
                                    BCC, BCC, BCC, BCC};

constexpr double rest_weight() {
    DD s{0.0, 0.0};
    for (int k = 1; k < NSHELL; ++k)
        s = dd_add(s, dd_mul(SHELL_W_DD[k], DD{double(SHELL_SIZE[k]), 0.0}));
    DD r = dd_add(DD{1.0, 0.0}, DD{-s.hi, -s.lo});
    return r.hi + r.lo;
}

constexpr double shell_weight(int s) {
    return s == 0 ? rest_weight() : SHELL_W_DD[s].hi + SHELL_W_DD[s].lo;
}

// --------------------------------------------------------- velocity table
struct Dir {
    int8_t x, y, z;  // 2 c_i
    int8_t shell;
};

struct DirTable {
    Dir d[Q];
};

constexpr DirTable make_dirs() {
    DirTable t{};
    t.d[0] = Dir{0, 0, 0, 0};
    int n = 1;
    // SC-k: +k e_a
    for (int k = 1; k <= 4; ++k)
        for (int a = 0; a < 3; ++a) {
            int8_t v[3] = {0, 0, 0};
            v[a] = int8_t(2 * k);
            t.d[n++] = Dir{v[0], v[1], v[2], int8_t(k)};
        }
    // FCC-k: k(e_a + e_b), k(e_a - e_b)
    for (int k = 1; k <= 2; ++k)
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                for (int sb = 1; sb >= -1; sb -= 2) {
                    int8_t v[3] = {0, 0, 0};
                    v[a] = int8_t(2 * k);
                    v[b] = int8_t(2 * k * sb);
                    t.d[n++] = Dir{v[0], v[1], v[2], int8_t(4 + k)};
                }
    // BCC-h: h(+1, +-1, +-1)
    const int hn[4] = {1, 2, 3, 5};
    for (int m = 0; m < 4; ++m)
        for (int sy = 1; sy >= -1; sy -= 2)
            for (int sz = 1; sz >= -1; sz -= 2)
                t.d[n++] = Dir{int8_t(hn[m]), int8_t(hn[m] * sy),
                               int8_t(hn[m] * sz), int8_t(7 + m)};
    // opposites
    for (int i = 1; i <= NPAIR; ++i)
        t.d[i + NPAIR] = Dir{int8_t(-t.d[i].x), int8_t(-t.d[i].y),
                             int8_t(-t.d[i].z), t.d[i].shell};
    return t;
}

constexpr DirTable DIRS = make_dirs();

constexpr int opp(int i) { return i == 0 ? 0 : (i <= NPAIR ? i + NPAIR : i - NPAIR); }
constexpr int cx2(int i) { return DIRS.d[i].x; }
constexpr int cy2(int i) { return DIRS.d[i].y; }
constexpr int cz2(int i) { return DIRS.d[i].z; }
constexpr int shell_of(int i) { return DIRS.d[i].shell; }
constexpr bool is_half(int i) { return (DIRS.d[i].x & 1) != 0; }
constexpr double weight(int i) { return shell_weight(shell_of(i)); }
constexpr double cx(int i) { return 0.5 * cx2(i); }
constexpr double cy(int i) { return 0.5 * cy2(i); }
constexpr double cz(int i) { return 0.5 * cz2(i); }
constexpr double csq(int i) { return 0.25 * SHELL_C2X4[shell_of(i)]; }

// Compile-time checks of the construction.
constexpr bool check_table() {
    int count[NSHELL] = {};
    for (int i = 0; i < Q; ++i) {
        count[shell_of(i)]++;
        int c2 = cx2(i) * cx2(i) + cy2(i) * cy2(i) + cz2(i) * cz2(i);
        if (c2 != SHELL_C2X4[shell_of(i)]) return false;
        if (cx2(opp(i)) != -cx2(i) || cy2(opp(i)) != -cy2(i) ||
            cz2(opp(i)) != -cz2(i))
            return false;
        bool hx = cx2(i) & 1, hy = cy2(i) & 1, hz = cz2(i) & 1;
        if (hx != hy || hy != hz) return false;
    }
    for (int s = 0; s < NSHELL; ++s)
        if (count[s] != SHELL_SIZE[s]) return false;
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < i; ++j)
            if (cx2(i) == cx2(j) && cy2(i) == cy2(j) && cz2(i) == cz2(j))
                return false;
    return true;
}
static_assert(check_table(), "RD3Q81 velocity table is inconsistent");
static_assert(rest_weight() > 0.11 && rest_weight() < 0.12, "rest weight");

// ----------------------------------------------------------- static_for
template <int N>
struct IC {
    static constexpr int value = N;
    constexpr operator int() const { return N; }
};

template <int B, int E, class F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(IC<B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace lbm81
