/*
 * Host check of the oracle's C code (test infrastructure only): calls every
 * entry point of precompute.c on small grids in 1, 2 and 3 dimensions, with
 * both interpolation schemes, serially and on several threads, plus the
 * error paths (out-of-grid points, NaN, bad arguments), and checks the
 * invariants the statistics must satisfy.  Built with
 * -fsanitize=address,undefined by the test-suite, so any out-of-bounds
 * access, leak or undefined behaviour in the oracle fails the build's run.
 * Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_stencils(int d, const int64_t *m, const double *g0, const double *h,
                    const double *x, int64_t n, int64_t *nodes, double *wts,
                    int64_t *cells, int64_t *bad);
int oracle_precompute(int d, const int64_t *m, const double *g0, const double *h,
                      const double *x, const double *y, int64_t n, double *wtw,
                      double *wty, double *yty, int64_t *bad);
int oracle_precompute_abs(int d, const int64_t *m, const double *g0, const double *h,
                          const double *x, const double *y, int64_t n, double *wtw,
                          double *wty, double *yty, int64_t *bad);
int oracle_precompute_omp(int d, const int64_t *m, const double *g0, const double *h,
                          const double *x, const double *y, int64_t n, double *wtw,
                          double *wty, double *yty, int64_t *bad, int nthreads);
int oracle_probe_sketches(int d, const int64_t *m, const double *g0, const double *h,
                          const double *x, int64_t n, uint64_t seed, int nprobe,
                          double *out, int64_t *bad);
int oracle_interpolate(int d, const int64_t *m, const double *g0, const double *h,
                       const double *mu_grid, const double *xq, int64_t nq, double *out,
                       int64_t *bad);
void oracle_wtw_matvec(int d, const int64_t *m, const double *wtw, const double *v,
                       double *u, int k);
void oracle_wtw_matvec_omp(int d, const int64_t *m, const double *wtw, const double *v,
                           double *u, int k, int nthreads);
void oracle_set_interp(int kind);
double oracle_probe_value(uint64_t seed, uint64_t j, uint64_t i);

static int failures = 0;

static void check(int ok, const char *what, int d, int interp) {
    if (!ok) {
        fprintf(stderr, "FAILED: %s (d=%d interp=%d)\n", what, d, interp);
        ++failures;
    }
}

/* Deterministic uniform numbers in [0, 1) (a linear congruential step). */
static uint64_t lcg = 12345;
static double unif(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static void run(int d, const int64_t *m, int interp) {
    oracle_set_interp(interp);
    double g0[3], h[3];
    int64_t M = 1;
    for (int k = 0; k < d; ++k) {
        h[k] = 1.0 / (double)(m[k] - 3);
        g0[k] = -h[k];
        M *= m[k];
    }
    const int64_t n = 1537;
    int nb = 1, s = 1;
    for (int k = 0; k < d; ++k) {
        nb *= 7;
        s *= 4;
    }
    double *x = malloc(sizeof(double) * (size_t)(d * n));
    double *y = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) x[k * n + i] = unif();
        y[i] = unif() - 0.5;
    }
    x[0] = 0.0;        /* on the lower boundary: u = h / h = 1 exactly */
    double *wtw = malloc(sizeof(double) * (size_t)(M * nb));
    double *wtw2 = malloc(sizeof(double) * (size_t)(M * nb));
    double *wabs = malloc(sizeof(double) * (size_t)(M * nb));
    double *wty = malloc(sizeof(double) * (size_t)M);
    double *wty2 = malloc(sizeof(double) * (size_t)M);
    double yty = 0.0, yty2 = 0.0;
    int64_t bad = -1;
    check(oracle_precompute(d, m, g0, h, x, y, n, wtw, wty, &yty, &bad) == 0, "precompute", d,
          interp);
    check(oracle_precompute_abs(d, m, g0, h, x, y, n, wabs, wty2, &yty2, &bad) == 0,
          "precompute_abs", d, interp);
    check(oracle_precompute_omp(d, m, g0, h, x, y, n, wtw2, wty2, &yty2, &bad, 3) == 0,
          "precompute_omp", d, interp);
    /* invariants: 1^T W^T W 1 = n (weights sum to 1), symmetry through the
     * product, |W^T W| <= |W|^T |W|, threaded = serial to rounding */
    double *one = malloc(sizeof(double) * (size_t)M);
    double *u = malloc(sizeof(double) * (size_t)M);
    double *u2 = malloc(sizeof(double) * (size_t)M);
    for (int64_t j = 0; j < M; ++j) one[j] = 1.0;
    oracle_wtw_matvec(d, m, wtw, one, u, 1);
    oracle_wtw_matvec_omp(d, m, wtw, one, u2, 1, 4);
    double tot = 0.0, diff = 0.0;
    for (int64_t j = 0; j < M; ++j) {
        tot += u[j];
        diff += fabs(u[j] - u2[j]);
    }
    check(fabs(tot - (double)n) < 1e-9 * n, "1^T W^T W 1 = n", d, interp);
    check(diff == 0.0, "threaded product = serial product", d, interp);
    double maxd = 0.0, maxa = 0.0;
    for (int64_t e = 0; e < M * nb; ++e) {
        if (fabs(wtw[e]) > wabs[e] * (1.0 + 1e-12) + 1e-300) maxd = 1.0;
        if (fabs(wtw[e] - wtw2[e]) > maxa) maxa = fabs(wtw[e] - wtw2[e]);
    }
    check(maxd == 0.0, "|W^T W| <= |W|^T |W|", d, interp);
    check(maxa < 1e-12, "threaded statistics = serial", d, interp);
    /* stencils, sketches, interpolation */
    int64_t *nodes = malloc(sizeof(int64_t) * (size_t)(n * s));
    double *wts = malloc(sizeof(double) * (size_t)(n * s));
    int64_t *cells = malloc(sizeof(int64_t) * (size_t)n);
    check(oracle_stencils(d, m, g0, h, x, n, nodes, wts, cells, &bad) == 0, "stencils", d,
          interp);
    int wsum_ok = 1;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int a = 0; a < s; ++a) {
            acc += wts[i * s + a];
            if (nodes[i * s + a] < 0 || nodes[i * s + a] >= M) wsum_ok = 0;
        }
        if (fabs(acc - 1.0) > 1e-12) wsum_ok = 0;
    }
    check(wsum_ok, "stencil weights sum to 1, nodes in range", d, interp);
    double *sk = malloc(sizeof(double) * (size_t)(3 * M));
    check(oracle_probe_sketches(d, m, g0, h, x, n, 7, 3, sk, &bad) == 0, "sketches", d, interp);
    double *q = malloc(sizeof(double) * (size_t)n);
    check(oracle_interpolate(d, m, g0, h, one, x, n, q, &bad) == 0, "interpolate", d, interp);
    int interp_ok = 1;
    for (int64_t i = 0; i < n; ++i)
        if (fabs(q[i] - 1.0) > 1e-12) interp_ok = 0;
    check(interp_ok, "interpolating a constant", d, interp);
    /* error paths: out of grid (with its index), NaN, bad arguments */
    x[(d - 1) * n + 700] = 1.5;
    bad = -1;
    check(oracle_precompute(d, m, g0, h, x, y, n, wtw, wty, &yty, &bad) == -2 && bad == 700,
          "out-of-grid point reported", d, interp);
    bad = -1;
    check(oracle_precompute_omp(d, m, g0, h, x, y, n, wtw, wty, &yty, &bad, 4) == -2 &&
              bad == 700,
          "out-of-grid point reported (threaded)", d, interp);
    x[(d - 1) * n + 700] = NAN;
    check(oracle_stencils(d, m, g0, h, x, n, nodes, wts, cells, &bad) == -2, "NaN rejected", d,
          interp);
    check(oracle_precompute(0, m, g0, h, x, y, n, wtw, wty, &yty, &bad) == -1, "d = 0", d,
          interp);
    check(oracle_precompute(d, m, g0, h, x, y, -1, wtw, wty, &yty, &bad) == -1, "n < 0", d,
          interp);
    check(oracle_probe_value(0, 0, 0) == 1.0 || oracle_probe_value(0, 0, 0) == -1.0,
          "probe value", d, interp);
    free(x); free(y); free(wtw); free(wtw2); free(wabs); free(wty); free(wty2);
    free(one); free(u); free(u2); free(nodes); free(wts); free(cells); free(sk); free(q);
}

int main(void) {
    const int64_t m1[1] = {40}, m2[2] = {17, 13}, m3[3] = {9, 8, 7};
    for (int interp = 0; interp < 2; ++interp) {
        run(1, m1, interp);
        run(2, m2, interp);
        run(3, m3, interp);
    }
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer check: all checks passed\n");
    return 0;
}
