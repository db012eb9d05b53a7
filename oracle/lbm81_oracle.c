/*
 * RD3Q81 lattice Boltzmann oracle: a plain, slow, FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * with the GPU library: the lattice, the equilibrium solver, the collision and
 * the streaming are all written out again here from the paper
 * (Atif et al., "Lattice Boltzmann Model for Transonic Flows",
 * arXiv:2409.05114).
 *
 * What it computes, step by step, and where the paper defines it:
 *   - lattice: 81 velocities and their weights w_i(theta0), Table "tab:weights"
 *     (Appendix); the rest weight is not printed and is 1 - sum of the others
 *     (mass trace, Sec. III, Eq. condRed1);
 *   - physical grid: body-centred cubic, i.e. the integer cube corners plus one
 *     replica site at every cube centre, so the half-integer links land on
 *     lattice sites (Sec. I, replica grid; Sec. V calls the model a
 *     body-centred cubic LBM);
 *   - moments rho, rho u, rho u^2 + 3 rho theta, Eq. (conslaws), Sec. II;
 *   - entropic equilibrium f_i = w_i rho exp(mu + zeta.c_i + gamma c_i^2),
 *     Sec. III, the minimiser of H = <f, log(f/w) - 1> under the conservation
 *     constraints; the multipliers are found by Newton's method on the
 *     5x5 linear system of Sec. III (the paper's linearised exp), here with a
 *     backtracking safeguard on the convex dual so that it cannot diverge;
 *   - update f_i(x + c_i, t + 1) = f_i + alpha beta (f_i^eq - f_i) with
 *     alpha = 2, beta = 1 / (2 tau + 1) (dt = 1), Eq. (discretelbm), Sec. II;
 *     streaming is done by pushing into a second buffer;
 *   - entropic variant: alpha is the positive root of
 *     H[f + alpha (f_eq - f)] = H[f], Eq. (delH), Sec. II;
 *   - series variant: the series form of the equilibrium (Sec. III;
 *     Appendix B: quartic weights, Eq. zeroveleqseries, and the third-order
 *     velocity term), used at a site when all 81 of its values are
 *     positive, else the Newton solution;
 *   - diagnostics of the Taylor-Green vortex (kinetic energy, enstrophy),
 *     Sec. IV.C.
 *
 * Every function is written for clarity, not speed.  OpenMP parallelises the
 * loops over sites only; each site's arithmetic is sequential.
 *
 * Population layout (oracle-private): f[site * 81 + i], site =
 * ((sub * nz + z) * ny + y) * nx + x, sub 0 = cube corners at (x, y, z),
 * sub 1 = cube centres at (x + 1/2, y + 1/2, z + 1/2).  Field arrays
 * (rho, theta: [site]; u: [3][site]) use the same site order.
 *
 * Return codes: 0 on success; a negative number -k when k sites were
 * unrealizable (rho <= 0, theta <= 0, non-finite) or failed to converge; -1000000000
 * for a bad argument.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 81
#define BAD_ARG (-1000000000)

/* ---------------------------------------------------------------- lattice */

/* theta0 as printed in the caption of Table "tab:weights". */
static const long double THETA0_LD = 0.821035006329447750282591763L;

static double g_c[Q][3];   /* velocities c_i (half-integers are exact)   */
static double g_w[Q];      /* weights w_i = W_i(theta0)                  */
static int g_ready = 0;

/* p(t) = (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) / d, in long double. */
static long double poly5(long double t, long double a1, long double a2,
                         long double a3, long double a4, long double a5,
                         long double d)
{
    long double t2 = t * t, t3 = t2 * t, t4 = t3 * t, t5 = t4 * t;
    return (a1 * t + a2 * t2 + a3 * t3 + a4 * t4 + a5 * t5) / d;
}

static void add_dir(int *n, double cx, double cy, double cz, long double w,
                    long double *wsum)
{
    g_c[*n][0] = cx;
    g_c[*n][1] = cy;
    g_c[*n][2] = cz;
    g_w[*n] = (double)w;
    *wsum += w;
    (*n)++;
}

/* Build the 81 velocities shell by shell as listed in Table "tab:weights":
 * rest; SC-k = k(+-1,0,0) and permutations, k = 1..4; FCC-k =
 * k(+-1,+-1,0) and permutations, k = 1, 2; BCC-h = h(+-1,+-1,+-1),
 * h = 1/2, 1, 3/2, 5/2. */
static void build_lattice(void)
{
    if (g_ready)
        return;
    const long double t = THETA0_LD;
    long double w_sc[5], w_fcc[3], w_bcc[4];
    w_sc[1] = poly5(t, 388800, -2508408, 7033852, -7856469, 2838528, 486000);
    w_sc[2] = poly5(t, -388800, 3091608, -8269102, 8694819, -2838528, 3888000);
    w_sc[3] = poly5(t, 388800, -3199608, 8977852, -9120069, 2838528, 30618000);
    w_sc[4] = poly5(t, -97200, 809352, -2315338, 2396961, -709632, 108864000);
    w_fcc[1] = poly5(t, 0, 0, 8, -9, 0, 12);
    w_fcc[2] = poly5(t, 0, 0, -2, 9, 0, 768);
    w_bcc[0] = poly5(t, 0, 24300, -103834, 126963, -44352, 7776);    /* h=1/2 */
    w_bcc[1] = poly5(t, 0, -24300, 189022, -328275, 177408, 272160); /* h=1   */
    w_bcc[2] = poly5(t, 0, 2700, -24778, 67995, -44352, 699840);     /* h=3/2 */
    w_bcc[3] = poly5(t, 0, -972, 11818, -43371, 44352, 68040000);    /* h=5/2 */
    const double bcc_h[4] = {0.5, 1.0, 1.5, 2.5};

    int n = 1; /* slot 0 is the rest velocity, filled last */
    long double wsum = 0.0L;
    for (int k = 1; k <= 4; ++k)
        for (int a = 0; a < 3; ++a)
            for (int s = -1; s <= 1; s += 2) {
                double v[3] = {0, 0, 0};
                v[a] = s * k;
                add_dir(&n, v[0], v[1], v[2], w_sc[k], &wsum);
            }
    for (int k = 1; k <= 2; ++k)
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                for (int sa = -1; sa <= 1; sa += 2)
                    for (int sb = -1; sb <= 1; sb += 2) {
                        double v[3] = {0, 0, 0};
                        v[a] = sa * k;
                        v[b] = sb * k;
                        add_dir(&n, v[0], v[1], v[2], w_fcc[k], &wsum);
                    }
    for (int m = 0; m < 4; ++m)
        for (int sx = -1; sx <= 1; sx += 2)
            for (int sy = -1; sy <= 1; sy += 2)
                for (int sz = -1; sz <= 1; sz += 2)
                    add_dir(&n, sx * bcc_h[m], sy * bcc_h[m], sz * bcc_h[m],
                            w_bcc[m], &wsum);
    /* rest weight: mass trace <w, 1> = 1 (Sec. III) */
    g_c[0][0] = g_c[0][1] = g_c[0][2] = 0.0;
    g_w[0] = (double)(1.0L - wsum);
    g_ready = (n == Q);
}

int lbo_lattice(double *c_out, double *w_out, double *theta0_out)
{
    build_lattice();
    if (!g_ready)
        return BAD_ARG;
    for (int i = 0; i < Q; ++i) {
        c_out[3 * i + 0] = g_c[i][0];
        c_out[3 * i + 1] = g_c[i][1];
        c_out[3 * i + 2] = g_c[i][2];
        w_out[i] = g_w[i];
    }
    *theta0_out = (double)THETA0_LD;
    return 0;
}

/* ------------------------------------------------------------ equilibrium */

/* Solve A x = b for a symmetric positive definite 5x5 A (Cholesky).
 * Returns 0, or -1 if A is not positive definite. */
static int spd_solve5(double A[5][5], const double b[5], double x[5])
{
    double L[5][5] = {{0}};
    for (int j = 0; j < 5; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k)
            d -= L[j][k] * L[j][k];
        if (!(d > 0.0))
            return -1;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 5; ++i) {
            double s = A[i][j];
            for (int k = 0; k < j; ++k)
                s -= L[i][k] * L[j][k];
            L[i][j] = s / L[j][j];
        }
    }
    double y[5];
    for (int i = 0; i < 5; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k)
            s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = 4; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 5; ++k)
            s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return 0;
}

/* Moment basis P_i = (1, c_x, c_y, c_z, c^2) of the conserved quantities,
 * Eq. (conslaws). */
static void basis(int i, double P[5])
{
    P[0] = 1.0;
    P[1] = g_c[i][0];
    P[2] = g_c[i][1];
    P[3] = g_c[i][2];
    P[4] = g_c[i][0] * g_c[i][0] + g_c[i][1] * g_c[i][1] + g_c[i][2] * g_c[i][2];
}

/* Populations of the exponential family at multipliers lam, per unit density:
 * g_i = w_i exp(mu + zeta.c_i + gamma c_i^2) (Sec. III).  Also returns the
 * dual objective Phi(lam) = sum_i g_i - lam.m, whose gradient is the moment
 * residual and whose Hessian is the matrix of the Sec. III linear system. */
static double family(const double lam[5], const double m[5], double g[Q])
{
    double phi = 0.0;
    for (int i = 0; i < Q; ++i) {
        double P[5];
        basis(i, P);
        double e = 0.0;
        for (int a = 0; a < 5; ++a)
            e += lam[a] * P[a];
        g[i] = g_w[i] * exp(e);
        phi += g[i];
    }
    for (int a = 0; a < 5; ++a)
        phi -= lam[a] * m[a];
    return phi;
}

/* Entropic equilibrium f_eq(rho, u, theta) (Sec. III).
 *
 * Works per unit density: the multipliers depend on (u, theta) only, since
 * rho multiplies every population.  Targets m = (1, u, u^2 + 3 theta).
 * Initial guess: the multipliers of the continuous Maxwellian at (u, theta)
 * relative to the lattice weights, mu = -(3/2) ln(theta/theta0) - u^2/(2 theta),
 * zeta = u/theta, gamma = (1/theta0 - 1/theta)/2; at u = 0 their Taylor series
 * in eta = theta/theta0 - 1 is the series of Appendix B (mu^(0), gamma^(0)).
 * Iteration: the 5x5 Newton system of Sec. III, J dlam = m - <g, P>, with
 * J = <g, P P^T>; a step that does not decrease the convex dual Phi is halved
 * (Armijo).  Converged when |dlam|_inf < 1e-12, then one more Newton step.
 *
 * Returns the number of iterations (>= 1), or -1 on non-convergence within
 * 100 iterations or a non-positive-definite Jacobian. */
static int solve_equilibrium(double rho, const double u[3], double theta,
                             double feq[Q], double lam_out[5])
{
    const double th0 = (double)THETA0_LD;
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double m[5] = {1.0, u[0], u[1], u[2], usq + 3.0 * theta};
    double lam[5] = {-1.5 * log(theta / th0) - usq / (2.0 * theta),
                     u[0] / theta, u[1] / theta, u[2] / theta,
                     0.5 / th0 - 0.5 / theta};
    double g[Q], gt[Q], lt[5];
    double phi = family(lam, m, g);
    int it, extra = 0, status = -1;
    for (it = 1; it <= 100; ++it) {
        double J[5][5] = {{0}}, r[5], d[5];
        for (int a = 0; a < 5; ++a)
            r[a] = m[a];
        for (int i = 0; i < Q; ++i) {
            double P[5];
            basis(i, P);
            for (int a = 0; a < 5; ++a) {
                r[a] -= g[i] * P[a];
                for (int b = 0; b < 5; ++b)
                    J[a][b] += g[i] * P[a] * P[b];
            }
        }
        if (spd_solve5(J, r, d) != 0)
            break;
        double dmax = 0.0, slope = 0.0;
        for (int a = 0; a < 5; ++a) {
            dmax = fmax(dmax, fabs(d[a]));
            slope -= r[a] * d[a]; /* grad Phi . d  (< 0) */
        }
        if (!isfinite(dmax))
            break;
        double t = 1.0, phit = 0.0;
        for (int k = 0; k < 60; ++k) {
            for (int a = 0; a < 5; ++a)
                lt[a] = lam[a] + t * d[a];
            phit = family(lt, m, gt);
            /* Near the solution Phi is flat to rounding; full steps there. */
            if (dmax * t < 1e-3 || phit <= phi + 1e-4 * t * slope)
                break;
            t *= 0.5;
        }
        memcpy(lam, lt, sizeof lam);
        memcpy(g, gt, sizeof g);
        phi = phit;
        if (extra) {
            status = it;
            break;
        }
        if (dmax * t < 1e-12 && t == 1.0)
            extra = 1;
    }
    for (int i = 0; i < Q; ++i)
        feq[i] = rho * g[i];
    if (lam_out)
        memcpy(lam_out, lam, sizeof lam);
    return status;
}

int lbo_equilibrium(double rho, double ux, double uy, double uz, double theta,
                    double *feq, double *lam_out)
{
    build_lattice();
    if (!g_ready)
        return BAD_ARG;
    if (!(rho > 0.0) || !(theta > 0.0) || !isfinite(ux) || !isfinite(uy) ||
        !isfinite(uz) || !isfinite(rho) || !isfinite(theta))
        return -1;
    const double u[3] = {ux, uy, uz};
    double lam[5];
    int it = solve_equilibrium(rho, u, theta, feq, lam);
    if (lam_out)
        memcpy(lam_out, lam, sizeof lam);
    return it;
}

/* ----------------------------------------------------------------- moments */

/* rho = <f, 1>, rho u = <f, c>, rho u^2 + 3 rho theta = <f, c^2>
 * (Eq. conslaws).  Returns 0, or -1 if the state is unrealizable. */
static int site_moments(const double *f, double *rho, double u[3],
                        double *theta)
{
    double r = 0.0, j[3] = {0, 0, 0}, e = 0.0;
    for (int i = 0; i < Q; ++i) {
        double csq = g_c[i][0] * g_c[i][0] + g_c[i][1] * g_c[i][1] +
                     g_c[i][2] * g_c[i][2];
        r += f[i];
        j[0] += f[i] * g_c[i][0];
        j[1] += f[i] * g_c[i][1];
        j[2] += f[i] * g_c[i][2];
        e += f[i] * csq;
    }
    *rho = r;
    for (int a = 0; a < 3; ++a)
        u[a] = j[a] / r;
    *theta = (e / r - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    if (!(r > 0.0) || !(*theta > 0.0) || !isfinite(r) || !isfinite(*theta) ||
        !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2]))
        return -1;
    return 0;
}

/* ---------------------------------------------------------------- geometry */

static long long wrap(long long v, long long n)
{
    long long r = v % n;
    return r < 0 ? r + n : r;
}

/* Site that the population of direction i leaving site s lands on after one
 * streaming step: position p = (x, y, z) + sub (1/2, 1/2, 1/2) moves to
 * p + c_i; a half-integer link switches sublattice.  Computed with doubled
 * coordinates so that every quantity is an integer; periodic in x, y, z. */
static long long stream_target(long long s, int i, int nx, int ny, int nz)
{
    long long x = s % nx, y = (s / nx) % ny, z = (s / ((long long)nx * ny)) % nz;
    long long sub = s / ((long long)nx * ny * nz);
    long long X2 = 2 * x + sub + (long long)llround(2.0 * g_c[i][0]);
    long long Y2 = 2 * y + sub + (long long)llround(2.0 * g_c[i][1]);
    long long Z2 = 2 * z + sub + (long long)llround(2.0 * g_c[i][2]);
    long long nsub = ((X2 % 2) + 2) % 2; /* same parity in all three axes */
    long long tx = wrap((X2 - nsub) / 2, nx);
    long long ty = wrap((Y2 - nsub) / 2, ny);
    long long tz = wrap((Z2 - nsub) / 2, nz);
    return ((nsub * nz + tz) * ny + ty) * nx + tx;
}

/* ------------------------------------------------------------- public API */

void lbo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int lbo_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* f = f_eq(rho, u, theta) at every site. */
int lbo_init(int nx, int ny, int nz, const double *rho, const double *u,
             const double *theta, double *f)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || !g_ready)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    long long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long long s = 0; s < ns; ++s) {
        const double us[3] = {u[s], u[ns + s], u[2 * ns + s]};
        if (!(rho[s] > 0.0) || !(theta[s] > 0.0) || !isfinite(rho[s]) ||
            !isfinite(theta[s]) || !isfinite(us[0]) || !isfinite(us[1]) ||
            !isfinite(us[2])) {
            for (int i = 0; i < Q; ++i)
                f[s * Q + i] = NAN;
            bad++;
            continue;
        }
        if (solve_equilibrium(rho[s], us, theta[s], f + s * Q, NULL) < 0)
            bad++;
    }
    return bad ? (int)(-bad) : 0;
}

/* ------------------------------------------------------ entropic collision */

/* h(y) = (1 + y) ln(1 + y) - y for y >= -1 (h(-1) = 1), by its Taylor series
 * sum_{n>=2} (-1)^n y^n / (n (n - 1)) where |y| is small (the closed form
 * cancels there). */
static long double hfun(long double y)
{
    if (y <= -1.0L)
        return 1.0L;
    if (fabsl(y) < 0.01L) {
        long double sum = 0.0L, p = y * y;
        for (int n = 2; n <= 14; ++n) {
            sum += ((n % 2) ? -p : p) / ((long double)n * (n - 1));
            p *= y;
        }
        return sum;
    }
    return (1.0L + y) * log1pl(y) - y;
}

/* Entropic alpha (Sec. II, Eq. delH): the positive root of
 *   phi(alpha) = H[f + alpha (f_eq - f)] - H[f],  H[g] = sum_i g_i (ln(g_i / w_i) - 1),
 * the convex entropy whose minimiser under the conservation constraints is
 * f_eq (Sec. III).  With D_i = f_eq,i - f_i and x_i = D_i / f_i the
 * difference is evaluated in the algebraically equal form
 *   phi(alpha) = sum_i f_i [ h(alpha x_i) - alpha x_i ln(1 + x_i) ],
 * which uses sum_i D_i = 0 and sum_i D_i ln(f_eq,i / w_i) = 0 (f_eq carries
 * the mass, momentum and energy of f, and ln(f_eq / w) is a combination of
 * 1, c and c^2); every term is then of second order in x, so nothing
 * cancels near equilibrium.  phi(0) = 0, phi'(0) < 0 and phi is convex, so
 * the positive root is unique when it exists; it is found by Newton's method
 * kept inside a bracket (bisection when a step leaves it).  The root must
 * keep every population non-negative, alpha <= alpha_max =
 * min over x_i < 0 of -1 / x_i; if phi is still negative there, alpha =
 * alpha_max.  At equilibrium (x = 0) alpha = 2, the limit of the root.
 * Returns the number of iterations, or -1 if f has a non-positive entry. */
static int entropic_alpha(const double *f, const double *feq, double *alpha)
{
    long double x[Q], scale = 0.0L, amax = INFINITY;
    for (int i = 0; i < Q; ++i) {
        if (!(f[i] > 0.0))
            return -1;
        x[i] = ((long double)feq[i] - f[i]) / f[i];
        scale += (long double)f[i] * x[i] * x[i];
        if (x[i] < 0.0L && -1.0L / x[i] < amax)
            amax = -1.0L / x[i];
    }
    if (scale == 0.0L) {
        *alpha = 2.0;
        return 0;
    }
    /* phi and phi' at a */
#define PHI(a, ph, dph)                                                    \
    do {                                                                   \
        ph = 0.0L;                                                         \
        dph = 0.0L;                                                        \
        for (int i = 0; i < Q; ++i) {                                      \
            const long double l1 = log1pl(x[i]);                           \
            ph += f[i] * (hfun((a) * x[i]) - (a) * x[i] * l1);             \
            dph += f[i] * x[i] *                                           \
                   (((a) * x[i] <= -1.0L ? -INFINITY : log1pl((a) * x[i])) - l1); \
        }                                                                  \
    } while (0)
    long double lo = 0.0L, hi = amax, ph, dph;
    if (isfinite(amax)) {
        PHI(amax, ph, dph);
        if (ph <= 0.0L) {
            *alpha = (double)amax;
            return 0;
        }
    } else {
        hi = 4.0L;
        for (;;) { /* grow until phi > 0 (phi grows at least linearly) */
            PHI(hi, ph, dph);
            if (ph > 0.0L)
                break;
            lo = hi;
            hi *= 2.0L;
        }
    }
    long double a = (2.0L > lo && 2.0L < hi) ? 2.0L : 0.5L * (lo + hi);
    for (int it = 1; it <= 200; ++it) {
        PHI(a, ph, dph);
        if (ph < 0.0L)
            lo = a;
        else
            hi = a;
        long double an = a - ph / dph;
        if (ph == 0.0L || fabsl(an - a) <= 2e-16L * a) {
            *alpha = (double)an;
            return it;
        }
        if (!(an > lo && an < hi)) /* Newton left the bracket: bisect */
            an = 0.5L * (lo + hi);
        if (hi - lo <= 2e-16L * a) {
            *alpha = (double)an;
            return it;
        }
        a = an;
    }
#undef PHI
    *alpha = (double)a;
    return 200;
}

int lbo_entropic_alpha(const double *f, const double *feq, double *alpha)
{
    build_lattice();
    if (!f || !feq || !alpha || !g_ready)
        return BAD_ARG;
    return entropic_alpha(f, feq, alpha);
}

/* H[f] = sum_i f_i (ln(f_i / w_i) - 1) in long double (for checks). */
double lbo_entropy(const double *f)
{
    build_lattice();
    long double h = 0.0L;
    for (int i = 0; i < Q; ++i)
        h += (long double)f[i] * (logl((long double)f[i] / g_w[i]) - 1.0L);
    return (double)h;
}


/* ------------------------------------------------------ series equilibrium */

/* The series form of the equilibrium, accurate to O(u^3 eta^4) (Sec. III;
 * Appendix B, "Discrete equilibrium at nonzero velocity"):
 *   f~_i = rho W~_i [1 + u.c_i / theta + f2_i + f3_i]
 * with eta = theta / theta0 - 1, y_i = c_i^2 / theta0 and the quartic
 * temperature-dependent weights of Eq. (zeroveleqseries) per unit density
 *   W~_i = w_i [1 + eta/2 (y - 3) + eta^2/8 (y^2 - 10 y + 15)
 *               + eta^3/48 (y^3 - 21 y^2 + 105 y - 105)
 *               + eta^4/384 (y^4 - 36 y^3 + 378 y^2 - 1260 y + 945)],
 *   f2_i = [(u.c)^2 - theta u^2] / (2 theta^2)
 *          - (5/3) u^2 / (2 theta^2) Rb / (2 + 5 Rb) (c^2 - 3 theta),
 *   f3_i = [(u.c)^3 - 3 theta u^2 (u.c)] / (6 theta^3)
 *          - 5 / (6 theta^3) Rb u^2 / (2 + 5 Rb) (u.c) (c^2 - 3 theta)
 *          + [5 (u.c) u^2 Rb - c_k Rb_kabg u_a u_b u_g] / (6 theta^2),
 *   Rb_kabg = <W~, c_k c_a c_b c_g> / theta^2 - Delta_kabg,
 *   Rb = <W~, c^2 c^2> / (15 theta^2) - 1,
 * Delta_kabg = d_ka d_bg + d_kb d_ag + d_kg d_ab (so Delta_kabg u_a u_b u_g
 * = 3 u^2 u_k).  The R-bar moments are those of the unit-density weights:
 * the moments they correct (15 rho theta^2, ...) carry rho.
 * Returns 1 if every value is positive, 0 otherwise. */
static int series_equilibrium(double rho, const double u[3], double theta,
                              double *feq)
{
    const double th0 = (double)THETA0_LD;
    const double eta = theta / th0 - 1.0;
    double wt[Q];
    for (int i = 0; i < Q; ++i) {
        const double y = (g_c[i][0] * g_c[i][0] + g_c[i][1] * g_c[i][1] +
                          g_c[i][2] * g_c[i][2]) / th0;
        wt[i] = g_w[i] *
                (1.0 + eta / 2.0 * (y - 3.0) +
                 eta * eta / 8.0 * (y * y - 10.0 * y + 15.0) +
                 eta * eta * eta / 48.0 *
                     (y * y * y - 21.0 * y * y + 105.0 * y - 105.0) +
                 eta * eta * eta * eta / 384.0 *
                     (y * y * y * y - 36.0 * y * y * y + 378.0 * y * y -
                      1260.0 * y + 945.0));
    }
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double th2 = theta * theta, th3 = th2 * theta;
    /* s4 = <W~, c^4>; t_k = Rb_kabg u_a u_b u_g */
    double s4 = 0.0, t[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < Q; ++j) {
        const double c2 = g_c[j][0] * g_c[j][0] + g_c[j][1] * g_c[j][1] +
                          g_c[j][2] * g_c[j][2];
        const double uc = u[0] * g_c[j][0] + u[1] * g_c[j][1] + u[2] * g_c[j][2];
        s4 += wt[j] * c2 * c2;
        for (int a = 0; a < 3; ++a)
            t[a] += wt[j] * g_c[j][a] * uc * uc * uc;
    }
    for (int a = 0; a < 3; ++a)
        t[a] = t[a] / th2 - 3.0 * u2 * u[a];
    const double rb = s4 / (15.0 * th2) - 1.0;
    const double g = rb / (2.0 + 5.0 * rb);
    int pos = 1;
    for (int i = 0; i < Q; ++i) {
        const double c2 = g_c[i][0] * g_c[i][0] + g_c[i][1] * g_c[i][1] +
                          g_c[i][2] * g_c[i][2];
        const double uc = u[0] * g_c[i][0] + u[1] * g_c[i][1] + u[2] * g_c[i][2];
        const double ct = g_c[i][0] * t[0] + g_c[i][1] * t[1] + g_c[i][2] * t[2];
        const double f2 = (uc * uc - theta * u2) / (2.0 * th2) -
                          5.0 / 3.0 * u2 / (2.0 * th2) * g * (c2 - 3.0 * theta);
        const double f3 = (uc * uc * uc - 3.0 * theta * u2 * uc) / (6.0 * th3) -
                          5.0 / (6.0 * th3) * g * u2 * uc * (c2 - 3.0 * theta) +
                          (5.0 * uc * u2 * rb - ct) / (6.0 * th2);
        feq[i] = rho * wt[i] * (1.0 + uc / theta + f2 + f3);
        if (!(feq[i] > 0.0))
            pos = 0;
    }
    return pos;
}

/* Series equilibrium at one point (see series_equilibrium): 1 if every
 * value is positive, 0 if not (the step then takes the Newton solution),
 * -1 for rho <= 0, theta <= 0 or non-finite input. */
int lbo_series_equilibrium(double rho, double ux, double uy, double uz,
                           double theta, double *feq)
{
    build_lattice();
    if (!g_ready)
        return BAD_ARG;
    if (!(rho > 0.0) || !(theta > 0.0) || !isfinite(ux) || !isfinite(uy) ||
        !isfinite(uz) || !isfinite(rho) || !isfinite(theta))
        return -1;
    const double u[3] = {ux, uy, uz};
    return series_equilibrium(rho, u, theta, feq);
}

/* mode 0: nsteps of collide + stream; mode 1: stream only; mode 2: collide
 * only (no streaming).  entropic = 0: alpha = 2 (Eq. discretelbm);
 * entropic = 1: alpha from Eq. delH at every site (entropic_alpha).
 * series = 1: the series equilibrium where it is positive, else Newton.
 * f is updated in place; scratch has the size of f. */
static int step_impl(int nx, int ny, int nz, double tau, int nsteps, int mode,
                     int entropic, int series, double *f, double *scratch)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || nsteps < 0 || !(tau > 0.0) ||
        mode < 0 || mode > 2 || !g_ready)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    /* alpha beta with alpha = 2 and beta = dt / (2 tau + dt), dt = 1 */
    const double omega = 2.0 / (2.0 * tau + 1.0);
    long long bad = 0;
    for (int step = 0; step < nsteps; ++step) {
#pragma omp parallel for schedule(static) reduction(+ : bad)
        for (long long s = 0; s < ns; ++s) {
            double post[Q];
            const double *fs = f + s * Q;
            memcpy(post, fs, sizeof post);
            if (mode != 1) {
                double rho, u[3], theta, feq[Q];
                if (site_moments(fs, &rho, u, &theta) != 0) {
                    bad++; /* unrealizable: the site keeps its populations */
                } else {
                    if (!(series && series_equilibrium(rho, u, theta, feq)) &&
                        solve_equilibrium(rho, u, theta, feq, NULL) < 0)
                        bad++;
                    double ab = omega; /* alpha beta */
                    if (entropic) {
                        double alpha;
                        if (entropic_alpha(fs, feq, &alpha) < 0)
                            bad++; /* a non-positive population: keep BGK */
                        else
                            ab = alpha / (2.0 * tau + 1.0);
                    }
                    for (int i = 0; i < Q; ++i)
                        post[i] = fs[i] + ab * (feq[i] - fs[i]);
                }
            }
            if (mode == 2) {
                memcpy(scratch + s * Q, post, sizeof post);
            } else {
                for (int i = 0; i < Q; ++i)
                    scratch[stream_target(s, i, nx, ny, nz) * Q + i] = post[i];
            }
        }
        memcpy(f, scratch, (size_t)ns * Q * sizeof(double));
    }
    return bad ? (int)(-(bad > 1000000000 ? 1000000000 : bad)) : 0;
}

int lbo_step(int nx, int ny, int nz, double tau, int nsteps, int mode,
             double *f, double *scratch)
{
    return step_impl(nx, ny, nz, tau, nsteps, mode, 0, 0, f, scratch);
}

int lbo_step_entropic(int nx, int ny, int nz, double tau, int nsteps, int mode,
                      double *f, double *scratch)
{
    return step_impl(nx, ny, nz, tau, nsteps, mode, 1, 0, f, scratch);
}

int lbo_step_series(int nx, int ny, int nz, double tau, int nsteps, int mode,
                    double *f, double *scratch)
{
    return step_impl(nx, ny, nz, tau, nsteps, mode, 0, 1, f, scratch);
}

/* Sites of f whose series equilibrium is not positive everywhere (where a
 * series step takes the Newton solution); unrealizable sites not counted. */
long long lbo_series_fallbacks(int nx, int ny, int nz, const double *f)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || !g_ready)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    long long n = 0;
#pragma omp parallel for schedule(static) reduction(+ : n)
    for (long long s = 0; s < ns; ++s) {
        double rho, u[3], theta, feq[Q];
        if (site_moments(f + s * Q, &rho, u, &theta) == 0 &&
            !series_equilibrium(rho, u, theta, feq))
            n++;
    }
    return n;
}

/* Per-site rho, u ([3][site]) and theta from the populations. */
int lbo_moments(int nx, int ny, int nz, const double *f, double *rho,
                double *u, double *theta)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || !g_ready)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    long long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long long s = 0; s < ns; ++s) {
        double r, us[3], th;
        if (site_moments(f + s * Q, &r, us, &th) != 0)
            bad++;
        rho[s] = r;
        u[s] = us[0];
        u[ns + s] = us[1];
        u[2 * ns + s] = us[2];
        theta[s] = th;
    }
    return bad ? (int)(-bad) : 0;
}

/* Domain totals of the conserved densities: sum rho, sum rho u (3),
 * sum (rho u^2 + 3 rho theta), accumulated in long double. */
int lbo_totals(int nx, int ny, int nz, const double *f, double *out)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || !g_ready)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    long double t[5] = {0, 0, 0, 0, 0};
    for (long long s = 0; s < ns; ++s)
        for (int i = 0; i < Q; ++i) {
            const long double v = f[s * Q + i];
            t[0] += v;
            t[1] += v * g_c[i][0];
            t[2] += v * g_c[i][1];
            t[3] += v * g_c[i][2];
            t[4] += v * (g_c[i][0] * g_c[i][0] + g_c[i][1] * g_c[i][1] +
                         g_c[i][2] * g_c[i][2]);
        }
    for (int a = 0; a < 5; ++a)
        out[a] = (double)t[a];
    return 0;
}

/* Mean kinetic energy and mean enstrophy of a flow field (Sec. IV.C, the
 * compressible Taylor-Green vortex diagnostics):
 *   KE  = <rho u.u / 2>,   eps = <rho w.w / 2>,   w = curl u,
 * where <.> is the mean over all sites (each sub-lattice holds one site per
 * cell volume, so the site mean is the volume mean).  The paper does not say
 * how the curl is discretised; here every derivative is the second-order
 * central difference between the two sites one cell away along that axis on
 * the same sub-lattice, periodic:  d/dy q(x, y, z) = (q(y + 1) - q(y - 1)) / 2.
 * rho: [site], u: [3][site] in the oracle's site order.  out[0] = KE,
 * out[1] = eps (sums in long double). */
int lbo_diagnostics(int nx, int ny, int nz, const double *rho, const double *u,
                    double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !rho || !u || !out)
        return BAD_ARG;
    const long long ns = 2LL * nx * ny * nz;
    const double *ux = u, *uy = u + ns, *uz = u + 2 * ns;
    long double ke = 0.0L, en = 0.0L;
    for (int sub = 0; sub < 2; ++sub)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
#define SITE(xx, yy, zz) \
    ((((long long)sub * nz + wrap(zz, nz)) * ny + wrap(yy, ny)) * nx + wrap(xx, nx))
                    const long long s = SITE(x, y, z);
                    const long long xp = SITE(x + 1, y, z), xm = SITE(x - 1, y, z);
                    const long long yp = SITE(x, y + 1, z), ym = SITE(x, y - 1, z);
                    const long long zp = SITE(x, y, z + 1), zm = SITE(x, y, z - 1);
#undef SITE
                    /* w = (d_y u_z - d_z u_y, d_z u_x - d_x u_z, d_x u_y - d_y u_x) */
                    const double wx = 0.5 * (uz[yp] - uz[ym]) - 0.5 * (uy[zp] - uy[zm]);
                    const double wy = 0.5 * (ux[zp] - ux[zm]) - 0.5 * (uz[xp] - uz[xm]);
                    const double wz = 0.5 * (uy[xp] - uy[xm]) - 0.5 * (ux[yp] - ux[ym]);
                    const double uu = ux[s] * ux[s] + uy[s] * uy[s] + uz[s] * uz[s];
                    ke += 0.5L * rho[s] * uu;
                    en += 0.5L * rho[s] * (wx * wx + wy * wy + wz * wz);
                }
    out[0] = (double)(ke / ns);
    out[1] = (double)(en / ns);
    return 0;
}

/* Streaming target of direction i from site s (exposed for geometry pins). */
long long lbo_stream_target(int nx, int ny, int nz, long long s, int i)
{
    build_lattice();
    if (nx < 1 || ny < 1 || nz < 1 || i < 0 || i >= Q || s < 0 ||
        s >= 2LL * nx * ny * nz)
        return -1;
    return stream_target(s, i, nx, ny, nz);
}
