/*
 * Oracle (test infrastructure only) -- plain, serial, FP64 CPU reference for
 * the one-shot O(n) pass of "Faster Kernel Interpolation for Gaussian
 * Processes" (Yadav, Sheldon, Musco).  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this code; the product
 * path never does.
 *
 * What it computes, each as its plain definition:
 *   - the cubic-convolution interpolation stencil w_x of a point (Sec. 3,
 *     Def. 3 and the basis-function description under Fig. 1: basis j is
 *     centred at grid node j and supported on [j-2, j+2); Keys' cubic kernel
 *     with a = -1/2), or the linear-interpolation stencil (Sec. 2.3: 2^d
 *     nonzeros; Claim 2 with r = 1), selected by oracle_set_interp and kept
 *     in the same four-node frame with zero outer weights;
 *   - the sufficient statistics W^T W = sum_i w_i w_i^T, W^T y = sum_i y_i w_i
 *     and y^T y = sum_i y_i^2 (Sec. 3.1 "Precomputation"; proof of Claim 2),
 *     accumulated serially in input order;
 *   - Rademacher probe sketches W^T z_j with z_j drawn from SplitMix64
 *     (stochastic log-determinant estimation, Sec. 2.2 / Sec. 5);
 *   - interpolation mu(x) = w_x^T mu_G (Fact 2, mean);
 *   - the banded product u = (W^T W) v in the stencil-diagonal layout.
 *
 * Grid convention: dimension k has m[k] nodes at g0[k] + j*h[k]; nodes are
 * flattened in C order (dimension 0 slowest).  A point is interpolable iff
 * 1 <= u_k <= m_k - 2 with u_k = (x_k - g0_k)/h_k, so that all four stencil
 * nodes exist.  The base node is i_k = min(floor(u_k), m_k - 3) and the
 * fractional offset t_k = u_k - i_k lies in [0, 1]; the stencil nodes are
 * i_k-1 .. i_k+2.
 *
 * W^T W is returned in the stencil-diagonal layout [m][7^d]: entry (j, o) is
 * (W^T W)[j, j+o] for the offset o in [-3,3]^d enumerated in C order; entries
 * whose partner node j+o lies outside the grid are zero (Claim 2: at most
 * (4r-1)^d = 7^d nonzeros per row for cubic interpolation, r = 2).
 *
 * The *_omp variants (for timing the oracle on all host cores) split the
 * points into one contiguous chunk per thread, accumulate each chunk
 * serially into the thread's own arrays and add the threads' arrays in
 * thread order, so their result is deterministic for a given thread count
 * (the serial functions stay the reference).
 *
 * Error behaviour: functions return 0 on success, -2 when a point lies outside
 * the interpolable region (index of the first such point in *bad), -1 on
 * invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Keys cubic-convolution weights (a = -1/2) for the nodes i-1, i, i+1, i+2 of
 * a point at fractional offset t in [0,1] from node i.  With s = 1 - t the
 * four Keys polynomials factor as
 *   w0 = -t s^2 / 2,  w1 = s (1 + 4s - 3s^2) / 2,
 *   w2 = t (1 + 4t - 3t^2) / 2,  w3 = -t^2 s / 2
 * (expanding gives (-t^3 + 2t^2 - t)/2, (3t^3 - 5t^2 + 2)/2,
 * (-3t^3 + 4t^2 + t)/2, (t^3 - t^2)/2).  Evaluated this way every weight is
 * accurate to a few units in its own last place, also where it is tiny
 * (t or s near 0): the expanded form cancels there and leaves an absolute
 * error of order 2^-52, which would swamp entries of W^T W built from
 * products of such weights.  The quadratic factors lie in [1, 2] on [0, 1]. */
static void keys_weights(double t, double w[4]) {
    double s = 1.0 - t;
    w[0] = -0.5 * t * (s * s);
    w[1] = 0.5 * s * (1.0 + 4.0 * s - 3.0 * (s * s));
    w[2] = 0.5 * t * (1.0 + 4.0 * t - 3.0 * (t * t));
    w[3] = -0.5 * (t * t) * s;
}

/* Linear interpolation between nodes i and i+1, in the same frame. */
static void linear_weights(double t, double w[4]) {
    w[0] = 0.0;
    w[1] = 1.0 - t;
    w[2] = t;
    w[3] = 0.0;
}

/* 0: Keys cubic (default); 1: linear.  Set before each call by the Python
 * wrapper from the grid description. */
static int g_interp = 0;

void oracle_set_interp(int kind) { g_interp = kind == 1 ? 1 : 0; }

static void stencil_weights(double t, double w[4]) {
    if (g_interp == 1)
        linear_weights(t, w);
    else
        keys_weights(t, w);
}

/* Per-dimension grid coordinate, base node and fractional offset.
 * Returns 0 if interpolable, -2 otherwise (including NaN). */
static int locate_1d(double x, double g0, double h, int64_t m, int64_t *base,
                     double *t) {
    double u = (x - g0) / h;
    if (!(u >= 1.0 && u <= (double)(m - 2))) return -2;
    double fl = floor(u);
    int64_t i = (int64_t)fl;
    if (i > m - 3) i = m - 3;
    *base = i;
    *t = u - (double)i;
    return 0;
}

/* Stencil of one point: up to 64 (node, weight) pairs (4^d).  Also returns
 * the cell key: the C-order index of (i_0 - 1, ..., i_{d-1} - 1) over a grid
 * of (m_k - 3) cells per dimension. */
static int stencil(int d, const int64_t *m, const double *g0, const double *h,
                   const double *xs /* d coords */, int64_t *nodes,
                   double *wts, int64_t *cell) {
    int64_t base[3];
    double w1[3][4];
    for (int k = 0; k < d; ++k) {
        double t;
        if (locate_1d(xs[k], g0[k], h[k], m[k], &base[k], &t)) return -2;
        stencil_weights(t, w1[k]);
    }
    int64_t c = 0;
    for (int k = 0; k < d; ++k) c = c * (m[k] - 3) + (base[k] - 1);
    *cell = c;
    int cnt = 1;
    for (int k = 0; k < d; ++k) cnt *= 4;
    for (int s = 0; s < cnt; ++s) {
        int rem = s;
        int a[3];
        for (int k = d - 1; k >= 0; --k) { a[k] = rem % 4; rem /= 4; }
        int64_t j = 0;
        double w = 1.0;
        for (int k = 0; k < d; ++k) {
            j = j * m[k] + (base[k] - 1 + a[k]);
            w *= w1[k][a[k]];
        }
        nodes[s] = j;
        wts[s] = w;
    }
    return 0;
}

static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

/* Flat index of offset (node_b - node_a) in the [-3,3]^d C-order enumeration. */
static int offset_index(int d, const int64_t *m, int64_t ja, int64_t jb) {
    int64_t ca[3], cb[3];
    for (int k = d - 1; k >= 0; --k) {
        ca[k] = ja % m[k]; ja /= m[k];
        cb[k] = jb % m[k]; jb /= m[k];
    }
    int oi = 0;
    for (int k = 0; k < d; ++k) oi = oi * 7 + (int)(cb[k] - ca[k] + 3);
    return oi;
}

/* Stencil of each point: nodes [n][4^d], weights [n][4^d], cell key [n]. */
int oracle_stencils(int d, const int64_t *m, const double *g0, const double *h,
                    const double *x /* [d][n] */, int64_t n, int64_t *nodes,
                    double *wts, int64_t *cells, int64_t *bad) {
    if (d < 1 || d > 3 || n < 0) return -1;
    int s = ipow(4, d);
    double xs[3];
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) xs[k] = x[(int64_t)k * n + i];
        if (stencil(d, m, g0, h, xs, nodes + i * s, wts + i * s, cells + i)) {
            if (bad) *bad = i;
            return -2;
        }
    }
    return 0;
}

/* Sufficient statistics, serially in input order (absw = 0), or the same
 * sums over the absolute weights, |W|^T |W| and |W|^T |y| (absw = 1): the
 * scale of the rounding error of any summation order of W^T W, used by the
 * tests' error bounds.
 * wtw: [M][7^d] zero-initialised here; wty: [M]; yty: scalar. */
static int precompute_impl(int d, const int64_t *m, const double *g0,
                           const double *h, const double *x, int64_t ldx,
                           const double *y, int64_t n, double *wtw, double *wty,
                           double *yty, int64_t *bad, int absw) {
    if (d < 1 || d > 3 || n < 0) return -1;
    int64_t M = 1;
    for (int k = 0; k < d; ++k) {
        if (m[k] < 4) return -1;
        M *= m[k];
    }
    int s = ipow(4, d), nb = ipow(7, d);
    memset(wtw, 0, sizeof(double) * (size_t)(M * nb));
    memset(wty, 0, sizeof(double) * (size_t)M);
    double acc_yy = 0.0;
    int64_t nodes[64];
    double wts[64];
    double xs[3];
    for (int64_t i = 0; i < n; ++i) {
        int64_t cell;
        for (int k = 0; k < d; ++k) xs[k] = x[(int64_t)k * ldx + i];
        if (stencil(d, m, g0, h, xs, nodes, wts, &cell)) {
            if (bad) *bad = i;
            return -2;
        }
        if (absw)
            for (int a = 0; a < s; ++a) wts[a] = fabs(wts[a]);
        const double yi = absw ? fabs(y[i]) : y[i];
        for (int a = 0; a < s; ++a) {
            wty[nodes[a]] += yi * wts[a];
            for (int b = 0; b < s; ++b) {
                int oi = offset_index(d, m, nodes[a], nodes[b]);
                wtw[nodes[a] * nb + oi] += wts[a] * wts[b];
            }
        }
        acc_yy += y[i] * y[i];
    }
    *yty = acc_yy;
    return 0;
}

int oracle_precompute(int d, const int64_t *m, const double *g0,
                      const double *h, const double *x /* [d][n] */,
                      const double *y, int64_t n, double *wtw, double *wty,
                      double *yty, int64_t *bad) {
    return precompute_impl(d, m, g0, h, x, n, y, n, wtw, wty, yty, bad, 0);
}

int oracle_precompute_abs(int d, const int64_t *m, const double *g0,
                          const double *h, const double *x /* [d][n] */,
                          const double *y, int64_t n, double *wtw, double *wty,
                          double *yty, int64_t *bad) {
    return precompute_impl(d, m, g0, h, x, n, y, n, wtw, wty, yty, bad, 1);
}

/* SplitMix64 finaliser (Vigna, public domain) applied to a counter. */
static uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Raw SplitMix64 output for a counter value (exported for the generator's
 * published test vectors). */
uint64_t oracle_splitmix64(uint64_t z) { return splitmix64(z); }

/* Rademacher probe entry z_j[i] in {+1,-1}: the top bit of SplitMix64 of the
 * counter (seed << 48) ^ (j << 40) ^ i. */
double oracle_probe_value(uint64_t seed, uint64_t j, uint64_t i) {
    uint64_t r = splitmix64((seed << 48) ^ (j << 40) ^ i);
    return (r >> 63) ? -1.0 : 1.0;
}

/* Probe sketches W^T z_j for j = 0..nprobe-1, serially in input order.
 * out: [nprobe][M]. */
int oracle_probe_sketches(int d, const int64_t *m, const double *g0,
                          const double *h, const double *x, int64_t n,
                          uint64_t seed, int nprobe, double *out,
                          int64_t *bad) {
    if (d < 1 || d > 3 || n < 0 || nprobe < 0) return -1;
    int64_t M = 1;
    for (int k = 0; k < d; ++k) M *= m[k];
    memset(out, 0, sizeof(double) * (size_t)(M * nprobe));
    int s = ipow(4, d);
    int64_t nodes[64];
    double wts[64];
    double xs[3];
    for (int64_t i = 0; i < n; ++i) {
        int64_t cell;
        for (int k = 0; k < d; ++k) xs[k] = x[(int64_t)k * n + i];
        if (stencil(d, m, g0, h, xs, nodes, wts, &cell)) {
            if (bad) *bad = i;
            return -2;
        }
        for (int j = 0; j < nprobe; ++j) {
            double z = oracle_probe_value(seed, (uint64_t)j, (uint64_t)i);
            for (int a = 0; a < s; ++a) out[(int64_t)j * M + nodes[a]] += z * wts[a];
        }
    }
    return 0;
}

/* mu(x_q) = w_{x_q}^T mu_G for each query point. */
int oracle_interpolate(int d, const int64_t *m, const double *g0,
                       const double *h, const double *mu_grid,
                       const double *xq /* [d][nq] */, int64_t nq,
                       double *out, int64_t *bad) {
    int s = ipow(4, d);
    int64_t nodes[64];
    double wts[64];
    double xs[3];
    for (int64_t i = 0; i < nq; ++i) {
        int64_t cell;
        for (int k = 0; k < d; ++k) xs[k] = xq[(int64_t)k * nq + i];
        if (stencil(d, m, g0, h, xs, nodes, wts, &cell)) {
            if (bad) *bad = i;
            return -2;
        }
        double acc = 0.0;
        for (int a = 0; a < s; ++a) acc += wts[a] * mu_grid[nodes[a]];
        out[i] = acc;
    }
    return 0;
}

/* u = (W^T W) v with W^T W in the stencil-diagonal layout [M][7^d];
 * v, u: [k][M] (k right-hand sides). */
void oracle_wtw_matvec(int d, const int64_t *m, const double *wtw,
                       const double *v, double *u, int k) {
    int64_t M = 1;
    for (int q = 0; q < d; ++q) M *= m[q];
    int nb = ipow(7, d);
    for (int r = 0; r < k; ++r) {
        for (int64_t j = 0; j < M; ++j) {
            int64_t c[3], rem = j;
            for (int q = d - 1; q >= 0; --q) { c[q] = rem % m[q]; rem /= m[q]; }
            double acc = 0.0;
            for (int oi = 0; oi < nb; ++oi) {
                int o[3], orem = oi;
                for (int q = d - 1; q >= 0; --q) { o[q] = orem % 7 - 3; orem /= 7; }
                int64_t jj = 0;
                int inside = 1;
                for (int q = 0; q < d; ++q) {
                    int64_t cq = c[q] + o[q];
                    if (cq < 0 || cq >= m[q]) { inside = 0; break; }
                    jj = jj * m[q] + cq;
                }
                if (inside) acc += wtw[j * nb + oi] * v[(int64_t)r * M + jj];
            }
            u[(int64_t)r * M + j] = acc;
        }
    }
}

/* oracle_precompute on `nthreads` threads (<= 0: all available). */
int oracle_precompute_omp(int d, const int64_t *m, const double *g0,
                          const double *h, const double *x, const double *y,
                          int64_t n, double *wtw, double *wty, double *yty,
                          int64_t *bad, int nthreads) {
    if (d < 1 || d > 3 || n < 0) return -1;
    int64_t M = 1;
    for (int k = 0; k < d; ++k) {
        if (m[k] < 4) return -1;
        M *= m[k];
    }
    int T = 1;
#ifdef _OPENMP
    T = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const int nb = ipow(7, d);
    double **tw = calloc((size_t)T, sizeof(double *));
    double **ty = calloc((size_t)T, sizeof(double *));
    double *tyy = calloc((size_t)T, sizeof(double));
    int64_t *tbad = malloc(sizeof(int64_t) * (size_t)T);
    int *trc = calloc((size_t)T, sizeof(int));
    int rc = 0;
    if (!tw || !ty || !tyy || !tbad || !trc) rc = -1;
    for (int t = 0; t < T && rc == 0; ++t) {
        tw[t] = malloc(sizeof(double) * (size_t)(M * nb));
        ty[t] = malloc(sizeof(double) * (size_t)M);
        if (!tw[t] || !ty[t]) rc = -1;
    }
    if (rc == 0) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static, 1)
#endif
        for (int t = 0; t < T; ++t) {
            const int64_t b0 = n * t / T, b1 = n * (t + 1) / T;
            int64_t bi = -1;
            trc[t] = precompute_impl(d, m, g0, h, x + b0, n, y + b0, b1 - b0, tw[t], ty[t],
                                     &tyy[t], &bi, 0);
            tbad[t] = bi >= 0 ? b0 + bi : -1;
        }
    }
    if (rc == 0) {
        for (int t = 0; t < T; ++t)
            if (trc[t] != 0) {
                rc = trc[t];
                if (rc == -2 && bad) *bad = tbad[t];
                break;
            }
    }
    if (rc == 0) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static)
#endif
        for (int64_t i = 0; i < M * nb; ++i) {
            double acc = 0.0;
            for (int t = 0; t < T; ++t) acc += tw[t][i];
            wtw[i] = acc;
        }
        for (int64_t j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int t = 0; t < T; ++t) acc += ty[t][j];
            wty[j] = acc;
        }
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += tyy[t];
        *yty = acc;
    }
    for (int t = 0; t < T; ++t) {
        if (tw) free(tw[t]);
        if (ty) free(ty[t]);
    }
    free(tw);
    free(ty);
    free(tyy);
    free(tbad);
    free(trc);
    return rc;
}

/* oracle_wtw_matvec on `nthreads` threads (rows split between threads; each
 * row's sum in the serial order, so the result equals the serial one). */
void oracle_wtw_matvec_omp(int d, const int64_t *m, const double *wtw,
                           const double *v, double *u, int k, int nthreads) {
    int64_t M = 1;
    for (int q = 0; q < d; ++q) M *= m[q];
    int nb = ipow(7, d);
    int T = 1;
#ifdef _OPENMP
    T = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)T;
    for (int r = 0; r < k; ++r) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static)
#endif
        for (int64_t j = 0; j < M; ++j) {
            int64_t c[3], rem = j;
            for (int q = d - 1; q >= 0; --q) { c[q] = rem % m[q]; rem /= m[q]; }
            double acc = 0.0;
            for (int oi = 0; oi < nb; ++oi) {
                int o[3], orem = oi;
                for (int q = d - 1; q >= 0; --q) { o[q] = orem % 7 - 3; orem /= 7; }
                int64_t jj = 0;
                int inside = 1;
                for (int q = 0; q < d; ++q) {
                    int64_t cq = c[q] + o[q];
                    if (cq < 0 || cq >= m[q]) { inside = 0; break; }
                    jj = jj * m[q] + cq;
                }
                if (inside) acc += wtw[j * nb + oi] * v[(int64_t)r * M + jj];
            }
            u[(int64_t)r * M + j] = acc;
        }
    }
}
