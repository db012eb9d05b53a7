/* Drives every entry point of the CPU oracle on small and degenerate grids,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (test_oracle_sanitize.py compiles it together with oracle/lbm81_oracle.c
 * and fails on any report).  Inputs: smooth fields plus a small
 * deterministic jitter, so that every step, the entropic alpha search and
 * the diagnostics take their ordinary paths; then the argument checks. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#define Q 81

int lbo_lattice(double *c_out, double *w_out, double *theta0_out);
int lbo_equilibrium(double rho, double ux, double uy, double uz, double theta,
                    double *feq, double *lam_out);
void lbo_set_threads(int n);
int lbo_init(int nx, int ny, int nz, const double *rho, const double *u,
             const double *theta, double *f);
int lbo_entropic_alpha(const double *f, const double *feq, double *alpha);
double lbo_entropy(const double *f);
int lbo_step(int nx, int ny, int nz, double tau, int nsteps, int mode,
             double *f, double *scratch);
int lbo_step_entropic(int nx, int ny, int nz, double tau, int nsteps, int mode,
                      double *f, double *scratch);
int lbo_moments(int nx, int ny, int nz, const double *f, double *rho,
                double *u, double *theta);
int lbo_totals(int nx, int ny, int nz, const double *f, double *out);
int lbo_diagnostics(int nx, int ny, int nz, const double *rho, const double *u,
                    double *out);
long long lbo_stream_target(int nx, int ny, int nz, long long s, int i);
int lbo_series_equilibrium(double rho, double ux, double uy, double uz,
                           double theta, double *feq);
int lbo_step_series(int nx, int ny, int nz, double tau, int nsteps, int mode,
                    double *f, double *scratch);
long long lbo_series_fallbacks(int nx, int ny, int nz, const double *f);

static unsigned long long lcg = 88172645463325252ULL;
static double jitter(void) { /* uniform in [-1, 1) */
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 4503599627370496.0 - 1.0;
}

static int run(int nx, int ny, int nz)
{
    const long long ns = 2LL * nx * ny * nz;
    double c[3 * Q], w[Q], theta0;
    if (lbo_lattice(c, w, &theta0) != 0) return 1;
    double *rho = malloc(sizeof(double) * ns);
    double *u = malloc(sizeof(double) * 3 * ns);
    double *th = malloc(sizeof(double) * ns);
    double *f = malloc(sizeof(double) * Q * ns);
    double *scratch = malloc(sizeof(double) * Q * ns);
    if (!rho || !u || !th || !f || !scratch) return 1;
    const double cs = sqrt(5.0 / 3.0 * theta0);
    for (long long s = 0; s < ns; ++s) {
        const double ph = 2.0 * 3.141592653589793 * (double)(s % nx) / nx;
        rho[s] = 1.0 + 0.1 * sin(ph) + 0.01 * jitter();
        u[s] = 0.5 * cs * cos(ph) + 0.01 * jitter();
        u[ns + s] = 0.2 * cs * jitter();
        u[2 * ns + s] = 0.1 * cs * jitter();
        th[s] = theta0 * (1.0 + 0.05 * jitter());
    }
    int bad = 0;
    bad |= lbo_init(nx, ny, nz, rho, u, th, f) != 0;
    double tot0[5], tot1[5], diag[2];
    bad |= lbo_totals(nx, ny, nz, f, tot0) != 0;
    for (int mode = 0; mode < 3; ++mode) {
        bad |= lbo_step(nx, ny, nz, 0.7, 2, mode, f, scratch) != 0;
        bad |= lbo_step_entropic(nx, ny, nz, 0.55, 2, mode, f, scratch) != 0;
        bad |= lbo_step_series(nx, ny, nz, 0.6, 2, mode, f, scratch) < 0;
    }
    bad |= lbo_totals(nx, ny, nz, f, tot1) != 0;
    bad |= fabs(tot1[0] - tot0[0]) > 1e-12 * tot0[0];
    bad |= lbo_moments(nx, ny, nz, f, rho, u, th) != 0;
    bad |= lbo_diagnostics(nx, ny, nz, rho, u, diag) != 0;
    bad |= !(diag[0] >= 0.0 && diag[1] >= 0.0);
    double feq[Q], lam[5], alpha;
    bad |= lbo_equilibrium(rho[0], u[0], u[ns], u[2 * ns], th[0], feq, lam) < 0;
    bad |= lbo_entropic_alpha(f, feq, &alpha) < 0;
    bad |= lbo_series_equilibrium(rho[0], u[0], u[ns], u[2 * ns], th[0], feq) < 0;
    bad |= lbo_series_fallbacks(nx, ny, nz, f) < 0;
    bad |= lbo_series_equilibrium(-1.0, 0.0, 0.0, 0.0, 1.0, feq) != -1;
    bad |= !isfinite(lbo_entropy(f));
    for (long long s = 0; s < ns; ++s)
        for (int i = 0; i < Q; ++i) {
            const long long t = lbo_stream_target(nx, ny, nz, s, i);
            bad |= t < 0 || t >= ns;
        }
    /* argument checks: rejected without touching memory */
    bad |= lbo_init(0, ny, nz, rho, u, th, f) == 0;
    bad |= lbo_diagnostics(nx, ny, nz, NULL, u, diag) == 0;
    bad |= lbo_stream_target(nx, ny, nz, ns, 0) != -1;
    bad |= lbo_stream_target(nx, ny, nz, 0, Q) != -1;
    free(rho); free(u); free(th); free(f); free(scratch);
    if (bad) fprintf(stderr, "failure on %d x %d x %d\n", nx, ny, nz);
    return bad;
}

int main(void)
{
    lbo_set_threads(2);
    const int shapes[][3] = {{1, 1, 1}, {2, 3, 1}, {5, 4, 3}, {7, 2, 2}, {16, 1, 1}};
    int bad = 0;
    for (unsigned k = 0; k < sizeof shapes / sizeof shapes[0]; ++k)
        bad |= run(shapes[k][0], shapes[k][1], shapes[k][2]);
    if (!bad) printf("ok\n");
    return bad;
}
