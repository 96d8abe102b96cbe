// Persistent batched block conjugate gradients over many independent SKI
// problems of uneven size.
//
// Every right-hand side b of every problem is solved with the factorized CG
// in the form of Claims 3 and 4: r = W r_hat + c_r b, p = W p_hat + c_p b,
// x = W x_hat + c_x b, which needs only b_hat = W^T b and ||b||^2 (the data
// vector y: W^T y, y^T y; a Rademacher probe z_j: its sketch and n).  A
// probe starts from x_0 = 0 (c_r = c_p = 1, r_hat = 0).  The data vector
// starts from x_0 = y / s2 (c_x = 1 / s2, c_r = c_p = 0, r_hat_0 =
// -K_G W^T y / s2): its residual then stays in the span of W and every c_r b
// term vanishes, which is the simplified factorized CG of the appendix.  The
// x_0 = 0 form carries W^T W x_hat by recurrence and its reconstruction
// u_x + c_x b_hat drifts from the true solution once ||r|| falls below about
// 1e-9 ||y||; in the simplified form the drift stays at rounding level.  One
// launch covers the whole batch: workgroup g owns one work item (a problem
// and a group of at most NR right-hand sides) and runs its CG to the end
// with workgroup barriers only, so workgroups never wait on each other and
// each one exits when all its right-hand sides have converged or the
// iteration cap is reached.  Inside an item the right-hand sides advance
// together: one read of the stored W^T W per iteration serves all of them.
//
// One iteration is four passes over the item's vectors:
//   (A) s_p = u_r + beta s_p, z_p = v_r + beta z_p (the direction update of
//       the previous iteration, fused here), and the dots s_p.ap, ap.b_hat
//       with ap = z_p + c_p kappa_b (never stored);
//   (B) u_x += alpha s_p, r_hat -= alpha ap;
//   (C) u_r = W^T W r_hat with two consecutive rows per thread (the x
//       values of a stencil row are shared by neighbouring rows) and the
//       dots r_hat.u_r, r_hat.b_hat fused; with an FP32-stored matrix the
//       x windows of a tile of rows are staged through LDS;
//   (D) v_r = s K_G u_r + s2 r_hat: line products per grid dimension, dense
//       Toeplitz passes for 2-D grids with both dimensions up to 128 nodes,
//       else short lines by the register line FFT (strided lines staged
//       through an LDS transpose) and long lines by the four-step FFT.
// Each pass issues a chunk's loads together, so an iteration of an item is
// a short chain of memory round trips.
#include <hip/hip_runtime.h>

#include "common.h"
#include "line_fft.h"

namespace fkgp {
namespace {

constexpr int kMaxWaves = 8;        // waves per work item: 4 or 8 (256 or 512 threads)
constexpr int kStrBlock = 32;       // strided lines per LDS transpose block

// Sum of NV per-thread values over the workgroup, in a fixed order (wave
// shuffles, then the waves in order).  Result in out[v] for all threads.
template <int NV>
__device__ inline void wg_sum(double (&v)[NV], double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) x += __shfl_xor(x, s);
        if (lane == 0) red[k * kMaxWaves + wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double acc = 0.0;
        for (int w = 0; w < nw; ++w) acc += red[threadIdx.x * kMaxWaves + w];
        out[threadIdx.x] = acc;
    }
    __syncthreads();
}

// Geometry of the line passes of one item.
struct PassGeom {
    int m_line;         // line length
    int64_t S;          // stride of a line's entries
    int64_t per_vec;    // lines per vector (M / m_line)
    int64_t M;          // vector length
    int64_t ldr;        // stride between padded r_hat vectors
    int64_t halo;
};

// Base offsets (vector layout and padded r_hat layout) of line li of vector r.
__device__ inline void line_base(const PassGeom& pg, int r, int64_t li, int64_t& base,
                                 int64_t& abase) {
    const int64_t outer = li / pg.S, inner = li - outer * pg.S;
    const int64_t start = outer * pg.m_line * pg.S + inner;
    base = r * pg.M + start;
    abase = r * pg.ldr + pg.halo + start;
}

// Lines read in place by the register line FFT (contiguous lines, and
// strided lines shorter than 32 nodes), one line pair per wave (64/L pairs
// when L < 64).  A vector of several lines pairs its own lines (an odd one
// leaves the last pair half empty), so its result does not depend on the
// other right-hand sides of the item; one-line vectors (1-D) are paired with
// each other.  dst = scale * conv(src) (+ add_coef * addv).
template <int LG>
__device__ void pass_reg_direct(const double* src, double* dst, const int* act, int na,
                                const PassGeom& pg, const cplx<double>* tws, const double* lams,
                                double scale, const double* addv, double add_coef) {
    constexpr int L = 1 << LG;
    constexpr int R = line_regs<LG>();
    constexpr int G = L >= 64 ? 1 : 64 / L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_lane = L >= 64 ? lane : (lane & (L - 1));
    const int g_lane = L >= 64 ? 0 : lane / L;
    const bool cross = pg.per_vec == 1;
    const int64_t ppv = (pg.per_vec + 1) / 2;   // pairs per vector (several lines)
    const int64_t npairs = cross ? (na + 1) / 2 : ppv * na;
    const int nw = blockDim.x >> 6;
    for (int64_t pb = (int64_t)wave * G; pb < npairs; pb += (int64_t)nw * G) {
        const int64_t pair = pb + g_lane;
        int64_t base[2] = {0, 0}, abase[2] = {0, 0};
        bool ok[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int64_t ri, li;
            if (cross) {
                ri = 2 * pair + h;
                li = 0;
                ok[h] = pair < npairs && ri < na;
            } else {
                ri = pair / ppv;
                li = 2 * (pair - ri * ppv) + h;
                ok[h] = pair < npairs && li < pg.per_vec;
            }
            if (ok[h]) line_base(pg, act[ri], li, base[h], abase[h]);
        }
        // all loads first, the added vector's too (a node past the line's
        // end reads its last node, an absent line reads line 0 of vector 0;
        // both are masked)
        double xa[R], xb[R], aa[R], ab[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int e = q * 64 + e_lane;
            const int64_t off = (int64_t)(e < pg.m_line ? e : pg.m_line - 1) * pg.S;
            xa[q] = src[base[0] + off];
            xb[q] = src[base[1] + off];
            if (addv) {
                aa[q] = addv[abase[0] + off];
                ab[q] = addv[abase[1] + off];
            }
        }
        cplx<double> z[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const bool in = q * 64 + e_lane < pg.m_line;
            z[q].re = (in && ok[0]) ? xa[q] : 0.0;
            z[q].im = (in && ok[1]) ? xb[q] : 0.0;
        }
        conv_line_regs<double, LG>(z, e_lane, tws, lams);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int e = q * 64 + e_lane;
            if (e >= pg.m_line) continue;
            if (ok[0]) {
                double v = scale * z[q].re;
                if (addv) v += add_coef * aa[q];
                dst[base[0] + e * pg.S] = v;
            }
            if (ok[1]) {
                double v = scale * z[q].im;
                if (addv) v += add_coef * ab[q];
                dst[base[1] + e * pg.S] = v;
            }
        }
    }
}

// Strided lines (2-D, dimension 0: stride m1, m1 lines per vector) by the
// register line FFT through an LDS transpose: blocks of kStrBlock adjacent
// lines are loaded and stored with coalesced rows.  T: kStrBlock x (m0 + 1).
template <int LG>
__device__ void pass_reg_strided(const double* src, double* dst, const int* act, int na,
                                 const PassGeom& pg, const cplx<double>* tws,
                                 const double* lams, double scale, const double* addv,
                                 double add_coef, double* T) {
    constexpr int R = line_regs<LG>();
    static_assert((1 << LG) >= 64, "strided pass expects lines of at least 32 nodes");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6, nt = blockDim.x;
    const int m = pg.m_line;
    const int ms = m + 1;
    const int S = (int)pg.S;
    const int nblk = (S + kStrBlock - 1) / kStrBlock;
    for (int bi = 0; bi < na * nblk; ++bi) {
        const int r = act[bi / nblk];
        const int i0 = (bi % nblk) * kStrBlock;
        const int nv = min(kStrBlock, S - i0);
        const double* s0 = src + (int64_t)r * pg.M + i0;
        // loads in batches of 8 per thread, issued before their LDS stores
        // (a column past the block reads the block's last column, masked)
        for (int idx0 = threadIdx.x; idx0 < kStrBlock * m; idx0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = idx0 + u * nt;
                const int e = idx / kStrBlock, l = idx - e * kStrBlock;
                const int ec = idx < kStrBlock * m ? e : m - 1;
                v[u] = s0[(int64_t)ec * S + (l < nv ? l : nv - 1)];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = idx0 + u * nt;
                const int e = idx / kStrBlock, l = idx - e * kStrBlock;
                if (idx < kStrBlock * m) T[l * ms + e] = l < nv ? v[u] : 0.0;
            }
        }
        __syncthreads();
        for (int pr = wave; pr < kStrBlock / 2; pr += nw) {
            cplx<double> z[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int e = q * 64 + lane;
                z[q].re = e < m ? T[(2 * pr) * ms + e] : 0.0;
                z[q].im = e < m ? T[(2 * pr + 1) * ms + e] : 0.0;
            }
            conv_line_regs<double, LG>(z, lane, tws, lams);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int e = q * 64 + lane;
                if (e < m) {
                    T[(2 * pr) * ms + e] = z[q].re;
                    T[(2 * pr + 1) * ms + e] = z[q].im;
                }
            }
        }
        __syncthreads();
        double* d0 = dst + (int64_t)r * pg.M + i0;
        const double* a0 = addv ? addv + (int64_t)r * pg.ldr + pg.halo + i0 : nullptr;
        for (int idx0 = threadIdx.x; idx0 < kStrBlock * m; idx0 += 8 * nt) {
            double av[8];
            if (a0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = idx0 + u * nt;
                    const int e = idx / kStrBlock, l = idx - e * kStrBlock;
                    const int ec = idx < kStrBlock * m ? e : m - 1;
                    av[u] = a0[(int64_t)ec * S + (l < nv ? l : nv - 1)];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = idx0 + u * nt;
                const int e = idx / kStrBlock, l = idx - e * kStrBlock;
                if (idx < kStrBlock * m && l < nv) {
                    double v = scale * T[l * ms + e];
                    if (a0) v += add_coef * av[u];
                    d0[(int64_t)e * S + l] = v;
                }
            }
        }
        __syncthreads();
    }
}

// Long lines by the four-step FFT, one line pair at a time for the whole
// workgroup (Y: L complex scratch of this item); pairs formed as in
// pass_reg_direct.
template <int LG1, int LG2>
__device__ void pass_long(const double* src, double* dst, const int* act, int na,
                          const PassGeom& pg, const cplx<double>* tw1, const cplx<double>* tw2,
                          const cplx<double>* twh, const double* lamp, double scale,
                          const double* addv, double add_coef, cplx<double>* Y) {
    const bool cross = pg.per_vec == 1;
    const int64_t ppv = (pg.per_vec + 1) / 2;
    const int64_t npairs = cross ? (na + 1) / 2 : ppv * na;
    for (int64_t pair = 0; pair < npairs; ++pair) {
        int64_t base[2] = {0, 0}, abase[2] = {0, 0};
        int64_t ri[2], li[2];
        if (cross) {
            ri[0] = 2 * pair;
            ri[1] = 2 * pair + 1;
            li[0] = li[1] = 0;
        } else {
            ri[0] = ri[1] = pair / ppv;
            li[0] = 2 * (pair - ri[0] * ppv);
            li[1] = li[0] + 1;
        }
        const bool hb = cross ? ri[1] < na : li[1] < pg.per_vec;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int hh = hb ? h : 0;
            line_base(pg, act[ri[hh]], li[hh], base[h], abase[h]);
        }
        wg_conv_long<double, LG1, LG2>(src + base[0], hb ? src + base[1] : nullptr, pg.S,
                                       pg.m_line, dst + base[0], hb ? dst + base[1] : nullptr,
                                       scale, addv ? addv + abase[0] : nullptr,
                                       (addv && hb) ? addv + abase[1] : nullptr, add_coef, Y,
                                       twh, lamp, tw1, tw2);
    }
}

// Dense Toeplitz line passes (2-D problems with both m_k <= kBatchTzMax):
// out[j] = sum_k c[|j - k|] u[k] along each line, 64 lines on the lanes of a
// wave and kBatchTzNJ consecutive outputs in its registers, the lines staged
// through LDS.  The column comes reflected and zero-padded:
// ext[q] = c[|q - (NJ - 1) - (m - 1)|] for |.| < m, else 0, so that the NJ
// values an output block needs at step k form one contiguous wave-uniform
// slice; a block of NJ steps reads the 2 NJ - 1 values it spans once.  For
// lines of ~100 nodes this takes about half the instructions of a 256-point
// FFT convolution, with no cross-lane traffic, and is exact to the plain
// summation bound.
constexpr int kTzNJ = kBatchTzNJ;

// acc[t] += sum_{k in [kb, kb + NJ)} ext[j0 - k + m - 1 + t + NJ - 1] u[k]
// (TAIL: steps past the line's end read a valid node and are masked).
template <bool TAIL>
__device__ __forceinline__ void tz_block(double (&acc)[kTzNJ], const double* ext,
                                         const double* urow, int ustride, int j0, int kb,
                                         int m) {
    constexpr int NJ = kTzNJ;
    const int base = j0 - kb + m - 1;   // index into ext without the left pad
    double E[2 * NJ - 1];
#pragma unroll
    for (int q = 0; q < 2 * NJ - 1; ++q) E[q] = ext[base + q];   // pad NJ - 1 cancels -NJ + 1
    double u[NJ];
#pragma unroll
    for (int s = 0; s < NJ; ++s) {
        const int k = kb + s;
        const double v = urow[(int64_t)(TAIL ? (k < m ? k : m - 1) : k) * ustride];
        u[s] = (!TAIL || k < m) ? v : 0.0;
    }
#pragma unroll
    for (int s = 0; s < NJ; ++s)
#pragma unroll
        for (int t = 0; t < NJ; ++t) acc[t] = fma(E[NJ - 1 - s + t], u[s], acc[t]);
}

// One output block: acc[t] = out[j0 + t] of the lane's line.
__device__ __forceinline__ void tz_line_block(double (&acc)[kTzNJ], const double* ext,
                                              const double* urow, int ustride, int j0, int m) {
    constexpr int NJ = kTzNJ;
#pragma unroll
    for (int t = 0; t < NJ; ++t) acc[t] = 0.0;
    int kb = 0;
#pragma unroll 1
    for (; kb + NJ <= m; kb += NJ) tz_block<false>(acc, ext, urow, ustride, j0, kb, m);
    if (kb < m) tz_block<true>(acc, ext, urow, ustride, j0, kb, m);
}

// Pass along dimension 1 (contiguous lines: row i0 of the m0 x m1 vector):
// dst[i0][j] = sum_k c1[|j - k|] src[i0][k].  Blocks of 64 rows are staged
// as S[row][k] with an odd row stride (conflict-free lane reads).
__device__ void tz_rows(const double* src, double* dst, int m0, int m1, const double* ext1,
                        double* S) {
    constexpr int NJ = kTzNJ;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6, nt = blockDim.x;
    const int ls = m1 | 1;
    const int njb = (m1 + NJ - 1) / NJ;
    for (int rb = 0; rb < m0; rb += 64) {
        const int nrow = min(64, m0 - rb);
        const double* s0 = src + (int64_t)rb * m1;
        const int cnt = nrow * m1;
        for (int i0 = threadIdx.x; i0 < cnt; i0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * nt;
                v[u] = s0[i < cnt ? i : cnt - 1];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * nt;
                if (i < cnt) {
                    const int row = i / m1;
                    S[row * ls + (i - row * m1)] = v[u];
                }
            }
        }
        __syncthreads();
        // lanes past the block's last row compute on another row and store nothing
        const double* urow = S + (lane < nrow ? lane : 0) * ls;
        for (int jb = wave; jb < njb; jb += nw) {
            const int j0 = jb * NJ;
            double acc[NJ];
            tz_line_block(acc, ext1, urow, 1, j0, m1);
            if (lane < nrow) {
                double* d = dst + (int64_t)(rb + lane) * m1;
#pragma unroll
                for (int t = 0; t < NJ; ++t)
                    if (j0 + t < m1) d[j0 + t] = acc[t];
            }
        }
        __syncthreads();
    }
}

// Pass along dimension 0 (strided lines: column i1): dst[j][i1] = scale *
// sum_k c0[|j - k|] src[k][i1] + add_coef * addv[j m1 + i1] (addv: padded
// r_hat, halo applied by the caller).  Blocks of 64 columns are staged as
// S[k][col]; src == dst allowed (a block's reads precede its writes).
__device__ void tz_cols(const double* src, double* dst, int m0, int m1, const double* ext0,
                        double scale, const double* addv, double add_coef, double* S) {
    constexpr int NJ = kTzNJ;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6, nt = blockDim.x;
    const int njb = (m0 + NJ - 1) / NJ;
    for (int cb = 0; cb < m1; cb += 64) {
        const int ncol = min(64, m1 - cb);
        const int cnt = m0 * 64;
        for (int i0 = threadIdx.x; i0 < cnt; i0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * nt;
                const int k = (i < cnt ? i : cnt - 1) >> 6, c = i & 63;
                v[u] = src[(int64_t)k * m1 + cb + (c < ncol ? c : ncol - 1)];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u * nt;
                if (i < cnt) S[i] = v[u];
            }
        }
        __syncthreads();
        const int col = cb + (lane < ncol ? lane : ncol - 1);
        for (int jb = wave; jb < njb; jb += nw) {
            const int j0 = jb * NJ;
            double a[NJ];
#pragma unroll
            for (int t = 0; t < NJ; ++t) {
                const int j = j0 + t < m0 ? j0 + t : m0 - 1;
                a[t] = addv[(int64_t)j * m1 + col];
            }
            double acc[NJ];
            tz_line_block(acc, ext0, S + lane, 64, j0, m0);
            if (lane < ncol) {
#pragma unroll
                for (int t = 0; t < NJ; ++t)
                    if (j0 + t < m0)
                        dst[(int64_t)(j0 + t) * m1 + col] = fma(add_coef, a[t], scale * acc[t]);
            }
        }
        __syncthreads();
    }
}

// Spectrum data of one dimension as the kernel sees it.
struct DimSpec {
    int lg;                       // log2 of the circulant length
    const cplx<double>* tw;       // register path: L/2 twiddles (LDS); long: w_L1 (LDS)
    const cplx<double>* tw2;      // long: w_L2 (LDS)
    const cplx<double>* twh;      // long: w_L, t < L/2 (global)
    const double* lam;            // register path: bit-reversed (LDS); long: four-step order
};

__device__ void line_pass(const DimSpec& ds, bool strided, const double* src, double* dst,
                          const int* act, int na, const PassGeom& pg, double scale,
                          const double* addv, double add_coef, double* T, cplx<double>* Y) {
    if (ds.lg > kBatchRegMaxLog2) {
        switch (ds.lg) {
#define FKGP_BL(LG, A, B)                                                                   \
    case LG:                                                                                \
        pass_long<A, B>(src, dst, act, na, pg, ds.tw, ds.tw2, ds.twh, ds.lam, scale, addv,  \
                        add_coef, Y);                                                       \
        break;
            FKGP_BL(9, 4, 5) FKGP_BL(10, 5, 5) FKGP_BL(11, 5, 6) FKGP_BL(12, 6, 6)
            FKGP_BL(13, 6, 7) FKGP_BL(14, 7, 7)
#undef FKGP_BL
            default:
                break;
        }
        return;
    }
    if (strided && ds.lg >= 6) {
        switch (ds.lg) {
#define FKGP_BS(LG)                                                                          \
    case LG:                                                                                 \
        pass_reg_strided<LG>(src, dst, act, na, pg, ds.tw, ds.lam, scale, addv, add_coef, T); \
        break;
            FKGP_BS(6) FKGP_BS(7) FKGP_BS(8)
#undef FKGP_BS
            default:
                break;
        }
        return;
    }
    switch (ds.lg) {
#define FKGP_BC(LG)                                                                          \
    case LG:                                                                                 \
        pass_reg_direct<LG>(src, dst, act, na, pg, ds.tw, ds.lam, scale, addv, add_coef);    \
        break;
        FKGP_BC(3) FKGP_BC(4) FKGP_BC(5) FKGP_BC(6) FKGP_BC(7) FKGP_BC(8)
#undef FKGP_BC
        default:
            break;
    }
}

// (C): u_r = W^T W r_hat for the active right-hand sides, RW = 2
// consecutive rows per thread (eight x values per stencil row serve 2 x 7
// products; wider blocks cost more registers than the saved loads are
// worth); v[2r] += r_hat.u_r, v[2r+1] += r_hat.b_hat over those rows.
template <int NR, class TA, int D>
__device__ void spmv_rows(const TA* __restrict__ A, const double* rp, double* ur,
                          const double* bh, const int* done, int nr, int64_t M, int64_t ldr,
                          int64_t halo, int m1, double (&v)[2 * NR]) {
    constexpr int RW = 2;
    constexpr int NB = D == 1 ? 7 : 49;
    constexpr int NA = D == 1 ? 1 : 7;
    const int64_t nq = (M + RW - 1) / RW;
#pragma unroll 1
    for (int64_t qd = threadIdx.x; qd < nq; qd += blockDim.x) {
        const int64_t j0 = RW * qd;
        const TA* At = A + ((j0 / kRowTile) * NB) * kRowTile + (j0 % kRowTile);
        double acc[NR][RW];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int q = 0; q < RW; ++q) acc[r][q] = 0.0;
#pragma unroll 1
        for (int a = 0; a < NA; ++a) {
            double av[7][RW];
#pragma unroll
            for (int b = 0; b < 7; ++b) {
                const TA* ap = At + (a * 7 + b) * kRowTile;
#pragma unroll
                for (int q = 0; q < RW; ++q) av[b][q] = (double)ap[q];
            }
            const int64_t off = (D == 1 ? 0 : (int64_t)(a - 3) * m1) - 3;
            if constexpr (NR <= 4) {
                // the x windows of every slot are loaded with the matrix row
                // (each slot owns a padded r_hat, inactive ones included), so
                // a stencil row costs one round trip
                double xv[NR][RW + 6];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const double* xb = rp + r * ldr + halo + j0 + off;
#pragma unroll
                    for (int c = 0; c < RW + 6; ++c) xv[r][c] = xb[c];
                }
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r >= nr || done[r]) continue;
#pragma unroll
                    for (int b = 0; b < 7; ++b)
#pragma unroll
                        for (int q = 0; q < RW; ++q)
                            acc[r][q] = fma(av[b][q], xv[r][q + b], acc[r][q]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r >= nr || done[r]) continue;
                    const double* xb = rp + r * ldr + halo + j0 + off;
                    double xv[RW + 6];
#pragma unroll
                    for (int c = 0; c < RW + 6; ++c) xv[c] = xb[c];
#pragma unroll
                    for (int b = 0; b < 7; ++b)
#pragma unroll
                        for (int q = 0; q < RW; ++q)
                            acc[r][q] = fma(av[b][q], xv[q + b], acc[r][q]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= nr || done[r]) continue;
            const double* xc = rp + r * ldr + halo + j0;
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                if (j0 + q < M) {
                    ur[r * M + j0 + q] = acc[r][q];
                    v[2 * r] = fma(xc[q], acc[r][q], v[2 * r]);
                    v[2 * r + 1] = fma(xc[q], bh[r * M + j0 + q], v[2 * r + 1]);
                }
            }
        }
    }
}

// Rows per tile of the staged product below (its LDS: batch_stage_doubles).
template <int BB>
constexpr int kStageRows = 2 * BB;

// (C) with FP32-stored W^T W, the x windows staged through LDS: per tile of
// 2 BB rows, the active slots' r_hat over the tile plus the stencil margin
// h = 3 m1 + 3 (2-D) or 3 (1-D) go to X[r][.] with all loads issued
// together, while each thread loads the 49 (7) entries of its two rows;
// after one barrier the products read x from LDS.  A tile costs one memory
// round trip instead of one per stencil row.  The products and dots are
// summed in the same order as spmv_rows, so the results are bitwise the
// same.  The window of padded index halo + t0 - h + i (halo = h) is
// clamped to the padded vector; clamped slots serve no valid row.
template <int NR, int D, int BB>
__device__ void spmv_rows_staged(const float* __restrict__ A, const double* rp, double* ur,
                                 const double* bh, const int* done, int nr, int64_t M,
                                 int64_t ldr, int m1, double* X, double (&v)[2 * NR]) {
    constexpr int RW = 2;
    constexpr int TR = kStageRows<BB>;
    constexpr int NB = D == 1 ? 7 : 49;
    constexpr int NA = D == 1 ? 1 : 7;
    constexpr int SU = 4;   // staged loads per thread and slot per batch
    const int h = (D == 1 ? 0 : 3 * m1) + 3;
    const int WL = TR + 2 * h;
    const int tid = threadIdx.x;
#pragma unroll 1
    for (int64_t t0 = 0; t0 < M; t0 += TR) {
        // window loads first (every active slot), then this thread's rows of A
#pragma unroll 1
        for (int i0 = tid; i0 < WL; i0 += SU * BB) {
            double w[NR][SU];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r >= nr || done[r]) continue;
                const double* xr = rp + r * ldr;
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int64_t pi = t0 + i0 + u * BB;   // = halo + t0 - h + i
                    w[r][u] = xr[pi < ldr ? pi : ldr - 1];
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r >= nr || done[r]) continue;
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int i = i0 + u * BB;
                    if (i < WL) X[r * WL + i] = w[r][u];
                }
            }
        }
        const int64_t j0 = t0 + RW * tid;
        const bool row_ok = j0 < M;
        const float* At = A + ((row_ok ? j0 : 0) / kRowTile) * NB * kRowTile +
                          ((row_ok ? j0 : 0) % kRowTile);
        float2 av[NB];
#pragma unroll
        for (int o = 0; o < NB; ++o) av[o] = *reinterpret_cast<const float2*>(At + o * kRowTile);
        __syncthreads();
        if (row_ok) {
            double acc[NR][RW];
#pragma unroll
            for (int r = 0; r < NR; ++r)
#pragma unroll
                for (int q = 0; q < RW; ++q) acc[r][q] = 0.0;
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int wb = RW * tid + h + (D == 1 ? 0 : (a - 3) * m1) - 3;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r >= nr || done[r]) continue;
                    double xv[RW + 6];
#pragma unroll
                    for (int c = 0; c < RW + 6; ++c) xv[c] = X[r * WL + wb + c];
#pragma unroll
                    for (int b = 0; b < 7; ++b) {
                        const float2 ab = av[a * 7 + b];
                        acc[r][0] = fma((double)ab.x, xv[b], acc[r][0]);
                        acc[r][1] = fma((double)ab.y, xv[1 + b], acc[r][1]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r >= nr || done[r]) continue;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    if (j0 + q < M) {
                        const double xc = X[r * WL + RW * tid + h + q];
                        ur[r * M + j0 + q] = acc[r][q];
                        v[2 * r] = fma(xc, acc[r][q], v[2 * r]);
                        v[2 * r + 1] = fma(xc, bh[r * M + j0 + q], v[2 * r + 1]);
                    }
                }
            }
        }
        __syncthreads();   // X is rewritten by the next tile
    }
}

// BB threads per work item (256 or 512); the register budget allows two
// waves per SIMD (two 256-thread items or one 512-thread item per CU).
template <int NR, int BB>
__global__ __launch_bounds__(BB, 2) void batch_cg_kernel(const BatchProb* __restrict__ probs,
                                                         const BatchItem* __restrict__ items,
                                                         double tol, int maxiter,
                                                         int64_t lds_doubles) {
    constexpr int kBB = BB;
    extern __shared__ double lds_dyn[];
    __shared__ double red[2 * NR * kMaxWaves];
    __shared__ double sums[2 * NR];
    __shared__ double rho[NR], cr[NR], cp[NR], cx[NR], pb[NR], alpha[NR], beta[NR], eps[NR];
    __shared__ double bb[NR];   // ||b||^2 of each right-hand side (y^T y, or n for a probe)
    __shared__ int done[NR], iters[NR];

    const BatchItem it = items[blockIdx.x];
    const BatchProb P = probs[it.prob];
    const int nr = it.nr;
    const int64_t M = P.M, halo = P.halo, ldr = batch_rhat_stride(M, halo);
    const int tid = threadIdx.x;
    // spectra into LDS (long dimensions: only the sub-length twiddles)
    DimSpec dsp[2] = {};
    double* T = nullptr;
    const bool tz = P.col[0] != nullptr;   // dense Toeplitz line passes
    double* ext[2] = {nullptr, nullptr};
    if (tz) {
        // reflected, zero-padded columns (see tz_block), then the staging block
        double* q = lds_dyn;
        for (int k = 0; k < 2; ++k) {
            const int m = P.m[k], n = 2 * m + 2 * kTzNJ;
            for (int i = tid; i < n; i += kBB) {
                const int o = i - (kTzNJ - 1) - (m - 1);
                q[i] = (o > -m && o < m) ? P.col[k][o < 0 ? -o : o] : 0.0;
            }
            ext[k] = q;
            q += n;
        }
        T = q;
    } else {
        unsigned char* p = reinterpret_cast<unsigned char*>(lds_dyn);
        for (int k = 0; k < P.d; ++k) {
            const int lg = P.log2L[k], L = 1 << lg;
            const cplx<double>* twg = static_cast<const cplx<double>*>(P.tw[k]);
            DimSpec& ds = dsp[k];
            ds.lg = lg;
            if (lg > kBatchRegMaxLog2) {
                int lg1, lg2;
                long_split(lg, lg1, lg2);
                const int L1 = 1 << lg1, L2 = 1 << lg2;
                cplx<double>* t1 = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L1 / 2);
                cplx<double>* t2 = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L2 / 2);
                for (int i = tid; i < L1 / 2; i += kBB) t1[i] = twg[i * L2];
                for (int i = tid; i < L2 / 2; i += kBB) t2[i] = twg[i * L1];
                ds.tw = t1;
                ds.tw2 = t2;
                ds.twh = twg;
                ds.lam = P.lam[k];
            } else {
                cplx<double>* t = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L / 2);
                double* lm = reinterpret_cast<double*>(p);
                p += sizeof(double) * L;
                for (int i = tid; i < L / 2; i += kBB) t[i] = twg[i];
                for (int i = tid; i < L; i += kBB) lm[i] = P.lam[k][i];
                ds.tw = t;
                ds.tw2 = nullptr;
                ds.twh = nullptr;
                ds.lam = lm;
            }
        }
        T = reinterpret_cast<double*>(p);   // strided-pass transpose block
    }
    // vectors of this item
    double* rp = it.work;                        // [NR][ldr] padded r_hat
    double* sp = rp + (int64_t)NR * ldr;         // [NR][M] each
    double* zp = sp + NR * M;
    double* ux = zp + NR * M;
    double* ur = ux + NR * M;
    double* vr = ur + NR * M;
    const double* bh = P.bh + (int64_t)it.r0 * M;
    const double* kb = P.kb + (int64_t)it.r0 * M;
#pragma unroll 1
    for (int64_t i = tid; i < (int64_t)NR * ldr; i += kBB) rp[i] = 0.0;
#pragma unroll 1
    for (int64_t i = tid; i < (int64_t)5 * NR * M; i += kBB) sp[i] = 0.0;
    // the data right-hand side in the simplified form: r_hat_0 into its slot
    const bool pre = P.r0y != nullptr && it.r0 == 0 && nr > 0;
    __syncthreads();
    if (pre) {
#pragma unroll 1
        for (int64_t i = tid; i < M; i += kBB) rp[halo + i] = P.r0y[i];
    }
    if (tid < NR) {
        const bool act = tid < nr;
        const bool simple = pre && tid == 0;
        const double bn = act ? P.bnorm2[it.r0 + tid] : 0.0;
        rho[tid] = bn;
        bb[tid] = bn;
        cr[tid] = simple ? 0.0 : 1.0;
        cp[tid] = simple ? 0.0 : 1.0;
        cx[tid] = simple ? 1.0 / P.s2 : 0.0;
        pb[tid] = 0.0;
        alpha[tid] = 0.0;
        beta[tid] = 0.0;
        eps[tid] = tol * tol * bn;
        done[tid] = (!act || !(bn > 0.0)) ? 1 : 0;
        iters[tid] = 0;
    }
    __syncthreads();

    // the staged banded product (FP32-stored matrix) when its windows fit in
    // the LDS past the spectra (they share it with the strided-pass transpose)
    const bool stage = P.a_f32 && batch_stage_doubles(P.d, P.m[1], NR, kBB) <=
                                      lds_doubles - (int64_t)(T - lds_dyn);
    PassGeom pg1{}, pg0{};
    if (P.d == 1) {
        pg0 = PassGeom{P.m[0], 1, 1, M, ldr, halo};
    } else {
        pg1 = PassGeom{P.m[1], 1, P.m[0], M, ldr, halo};
        pg0 = PassGeom{P.m[0], P.m[1], P.m[1], M, ldr, halo};
    }

    // iteration -1 (items holding a simplified data right-hand side): only
    // (C) and (D), giving u_r = W^T W r_hat_0, v_r = B(r_hat_0).v and rho_0 =
    // r_hat_0 . u_r; the probes of the item have r_hat = 0 and keep
    // rho = ||b||^2
    for (int iter = pre ? -1 : 0; iter < maxiter; ++iter) {
        int act[NR];
        int na = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nr && !done[r]) act[na++] = r;
        if (na == 0) break;
        if (iter >= 0) {
        // (A) direction update (beta = 0 on the first pass: p_hat = r_hat)
        {
            double v[2 * NR];
#pragma unroll
            for (int k = 0; k < 2 * NR; ++k) v[k] = 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (r >= nr || done[r]) continue;
                const double b = beta[r], c = cp[r];
                double* spr = sp + r * M;
                double* zpr = zp + r * M;
                const double* urr = ur + r * M;
                const double* vrr = vr + r * M;
                const double* kbr = kb + r * M;
                const double* bhr = bh + r * M;
                // every load of a chunk is issued before the first use (the
                // tail reads a valid element and masks it): one round trip
#pragma unroll 1
                for (int64_t i0 = tid; i0 < M; i0 += 4 * kBB) {
                    double s0[4], u0[4], z0[4], v0[4], k4[4], b4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t i = i0 + u * kBB;
                        const int64_t ic = i < M ? i : M - 1;
                        s0[u] = spr[ic];
                        u0[u] = urr[ic];
                        z0[u] = zpr[ic];
                        v0[u] = vrr[ic];
                        k4[u] = kbr[ic];
                        b4[u] = bhr[ic];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t i = i0 + u * kBB;
                        const bool in = i < M;
                        const double s = in ? fma(b, s0[u], u0[u]) : 0.0;
                        const double z = in ? fma(b, z0[u], v0[u]) : 0.0;
                        const double kk = in ? k4[u] : 0.0;
                        const double bb4 = in ? b4[u] : 0.0;
                        if (in) {
                            spr[i] = s;
                            zpr[i] = z;
                        }
                        const double a = fma(c, kk, z);
                        v[2 * r] = fma(s, a, v[2 * r]);
                        v[2 * r + 1] = fma(a, bb4, v[2 * r + 1]);
                    }
                }
            }
            wg_sum<2 * NR>(v, red, sums);
        }
        if (tid < nr && !done[tid]) {
            const int r = tid;
            const double apc = P.s2 * cp[r];
            const double pap = sums[2 * r] + apc * pb[r] + cp[r] * sums[2 * r + 1] +
                               cp[r] * apc * bb[r];
            const double a = rho[r] / pap;
            if (!isfinite(a)) {
                done[r] = 2;
            } else {
                if (iters[r] < kMaxLanczos) P.alphas[(it.r0 + r) * kMaxLanczos + iters[r]] = a;
                alpha[r] = a;
                cx[r] += a * cp[r];
                cr[r] -= a * apc;
            }
        }
        __syncthreads();
        // (B) u_x += alpha s_p; r_hat -= alpha (z_p + c_p kappa_b)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= nr || done[r]) continue;
            const double a = alpha[r], c = cp[r];
            const double* spr = sp + r * M;
            const double* zpr = zp + r * M;
            const double* kbr = kb + r * M;
            double* uxr = ux + r * M;
            double* rpr = rp + r * ldr + halo;
#pragma unroll 1
            for (int64_t i0 = tid; i0 < M; i0 += 4 * kBB) {
                double s0[4], x0[4], k4[4], z0[4], r0v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t i = i0 + u * kBB;
                    const int64_t ic = i < M ? i : M - 1;
                    s0[u] = spr[ic];
                    x0[u] = uxr[ic];
                    k4[u] = kbr[ic];
                    z0[u] = zpr[ic];
                    r0v[u] = rpr[ic];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t i = i0 + u * kBB;
                    if (i < M) {
                        uxr[i] = fma(a, s0[u], x0[u]);
                        rpr[i] = fma(-a, fma(c, k4[u], z0[u]), r0v[u]);
                    }
                }
            }
        }
        __syncthreads();
        }   // iter >= 0
        // (C) u_r = W^T W r_hat with the dots r_hat.u_r and r_hat.b_hat
        {
            double v[2 * NR];
#pragma unroll
            for (int k = 0; k < 2 * NR; ++k) v[k] = 0.0;
            if (stage) {
                if (P.d == 1)
                    spmv_rows_staged<NR, 1, BB>(static_cast<const float*>(P.A), rp, ur, bh,
                                                done, nr, M, ldr, 1, T, v);
                else
                    spmv_rows_staged<NR, 2, BB>(static_cast<const float*>(P.A), rp, ur, bh,
                                                done, nr, M, ldr, P.m[1], T, v);
            } else if (P.d == 1) {
                if (P.a_f32)
                    spmv_rows<NR, float, 1>(static_cast<const float*>(P.A), rp, ur, bh, done,
                                             nr, M, ldr, halo, 1, v);
                else
                    spmv_rows<NR, double, 1>(static_cast<const double*>(P.A), rp, ur, bh,
                                              done, nr, M, ldr, halo, 1, v);
            } else {
                if (P.a_f32)
                    spmv_rows<NR, float, 2>(static_cast<const float*>(P.A), rp, ur, bh, done,
                                             nr, M, ldr, halo, P.m[1], v);
                else
                    spmv_rows<NR, double, 2>(static_cast<const double*>(P.A), rp, ur, bh,
                                              done, nr, M, ldr, halo, P.m[1], v);
            }
            wg_sum<2 * NR>(v, red, sums);
        }
        // rho' = <r, r>, convergence, beta
        if (tid < nr && !done[tid]) {
            const int r = tid;
            const double rn = sums[2 * r] + 2.0 * cr[r] * sums[2 * r + 1] + cr[r] * cr[r] * bb[r];
            if (iter < 0) {   // initial residual norm; no step taken yet
                rho[r] = rn;
                pb[r] = sums[2 * r + 1];
                if (!(rn > eps[r])) done[r] = 1;
            } else {
            iters[r] += 1;
            if (!(rn > eps[r])) {
                done[r] = 1;
                rho[r] = rn;
            } else {
                const double b = rn / rho[r];
                if (iters[r] - 1 < kMaxLanczos)
                    P.betas[(it.r0 + r) * kMaxLanczos + iters[r] - 1] = b;
                beta[r] = b;
                rho[r] = rn;
                pb[r] = sums[2 * r + 1] + b * pb[r];
                cp[r] = cr[r] + b * cp[r];
            }
            }
        }
        __syncthreads();
        // (D) v_r = s K_G u_r + s2 r_hat for the right-hand sides still active
        na = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nr && !done[r]) act[na++] = r;
        // The line FFTs carry two lines as one complex line, and rounding
        // mixes the two at the level of u times the larger one.  The data
        // right-hand side in its simplified form has vectors orders of
        // magnitude larger than a probe's, and the loss of orthogonality of
        // CG amplifies such a perturbation of a probe step by step (the
        // Lanczos log-determinant drifts after ~25 steps), so its lines are
        // never paired with a probe's: the passes run over [y] and the
        // probes separately.
        if (na > 0) {
            const bool split = !tz && pre && act[0] == 0 && na > 1;
            const int ng = split ? 2 : 1;
            for (int gi = 0; gi < ng; ++gi) {
                const int* ga = split && gi == 1 ? act + 1 : act;
                const int gn = split ? (gi == 0 ? 1 : na - 1) : na;
                if (tz) {
                    for (int q = 0; q < gn; ++q) {
                        const int r = ga[q];
                        tz_rows(ur + r * M, vr + r * M, P.m[0], P.m[1], ext[1], T);
                    }
                    __syncthreads();
                    for (int q = 0; q < gn; ++q) {
                        const int r = ga[q];
                        tz_cols(vr + r * M, vr + r * M, P.m[0], P.m[1], ext[0], P.so,
                                rp + r * ldr + halo, P.s2, T);
                    }
                } else if (P.d == 1) {
                    line_pass(dsp[0], false, ur, vr, ga, gn, pg0, P.so, rp, P.s2, T, it.yscr);
                } else {
                    line_pass(dsp[1], false, ur, vr, ga, gn, pg1, 1.0, nullptr, 0.0, T,
                              it.yscr);
                    __syncthreads();
                    line_pass(dsp[0], true, vr, vr, ga, gn, pg0, P.so, rp, P.s2, T, it.yscr);
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
    // outputs: W^T x = u_x + c_x b_hat, and the final states
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r >= nr) continue;
        const double c = cx[r];
        double* out = P.wx + (int64_t)(it.r0 + r) * M;
#pragma unroll 1
        for (int64_t i = tid; i < M; i += kBB) out[i] = fma(c, bh[r * M + i], ux[r * M + i]);
    }
    if (tid < nr) {
        PState s{};
        s.rho = rho[tid];
        s.cr = cr[tid];
        s.cp = cp[tid];
        s.cx = cx[tid];
        s.pb = pb[tid];
        s.alpha = alpha[tid];
        s.beta = beta[tid];
        s.eps = eps[tid];
        s.done = done[tid];
        s.iters = iters[tid];
        P.ps[it.r0 + tid] = s;
    }
}

template <int NR, int BB>
fkgp_status launch_nr(const BatchProb* probs, const BatchItem* items, int nitems, size_t lds,
                      double tol, int maxiter, hipStream_t s) {
    if (lds > 64 * 1024)
        FKGP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_cg_kernel<NR, BB>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    batch_cg_kernel<NR, BB><<<nitems, BB, lds, s>>>(probs, items, tol, maxiter,
                                                    (int64_t)(lds / sizeof(double)));
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

}  // namespace

size_t batch_work_doubles(int64_t M, int64_t halo, int nr) {
    return (size_t)nr * batch_rhat_stride(M, halo) + (size_t)5 * nr * M;
}

size_t batch_lds_bytes(int d, const int* m, const int* log2L) {
    if (batch_tz(d, m)) return sizeof(double) * (size_t)batch_tz_doubles(m);
    size_t l = 0;
    for (int k = 0; k < d; ++k) {
        if (log2L[k] > kBatchRegMaxLog2) {
            int lg1, lg2;
            long_split(log2L[k], lg1, lg2);
            l += (size_t)8 * ((1 << lg1) + (1 << lg2));   // both sub-length twiddles
        } else {
            l += (size_t)16 * (1 << log2L[k]);            // twiddles + spectrum
        }
    }
    if (d == 2 && log2L[0] <= kBatchRegMaxLog2)
        l += (size_t)8 * kStrBlock * (m[0] + 1);          // strided-pass transpose
    return l;
}

fkgp_status launch_batch_cg(const BatchProb* probs_dev, const BatchItem* items_dev, int nitems,
                            size_t lds, double tol, int maxiter, int nr, int block,
                            hipStream_t s) {
    if (nitems == 0) return FKGP_OK;
    const int key = nr * 10000 + block;
    switch (key) {
        case 20256:
            return launch_nr<2, 256>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        case 40256:
            return launch_nr<4, 256>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        case 80256:
            return launch_nr<8, 256>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        case 20512:
            return launch_nr<2, 512>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        case 40512:
            return launch_nr<4, 512>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        case 80512:
            return launch_nr<8, 512>(probs_dev, items_dev, nitems, lds, tol, maxiter, s);
        default:
            set_error("batched solver: right-hand sides per item must be 2, 4 or 8 and the "
                      "workgroup 256 or 512 threads");
            return FKGP_EINVAL;
    }
}

}  // namespace fkgp
