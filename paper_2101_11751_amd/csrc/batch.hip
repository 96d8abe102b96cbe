// Persistent batched block conjugate gradients over many independent SKI
// problems of uneven size.
//
// Every right-hand side b of every problem is solved with the factorized CG
// from x_0 = 0 (Claims 3 and 4): r = W r_hat + c_r b, p = W p_hat + c_p b,
// x = W x_hat + c_x b, which needs only b_hat = W^T b and ||b||^2 (the data
// vector y: W^T y, y^T y; a Rademacher probe z_j: its sketch and n).  One
// launch covers the whole batch: workgroup g owns one work item (a problem
// and a group of at most kBatchRhs right-hand sides) and runs its CG to the
// end with workgroup barriers only, so workgroups never wait on each other
// and each one exits when all its right-hand sides have converged or the
// iteration cap is reached.  Inside an item the right-hand sides advance
// together: one read of the stored W^T W per iteration serves all of them,
// and the K_G product convolves their grid lines with the register-resident
// line FFT (two real lines per complex line).
#include <hip/hip_runtime.h>

#include "common.h"
#include "line_fft.h"

namespace fkgp {
namespace {

constexpr int kBatchBlock = 256;
constexpr int kBatchWaves = kBatchBlock / 64;

// Sum of NV per-thread values over the workgroup, in a fixed order (wave
// shuffles, then the waves in order).  Result in out[v] for all threads.
template <int NV>
__device__ inline void wg_sum(double (&v)[NV], double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) x += __shfl_xor(x, s);
        if (lane == 0) red[k * kBatchWaves + wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double acc = 0.0;
        for (int w = 0; w < kBatchWaves; ++w) acc += red[threadIdx.x * kBatchWaves + w];
        out[threadIdx.x] = acc;
    }
    __syncthreads();
}

// One pass of line convolutions over all lines (of all nr vectors) along a
// grid dimension: lines of length m_line with stride S inside [outer][m][S]
// vectors of length M.  dst = scale * conv(src) (+ add_coef * addv, addv in
// padded layout with leading dimension ldx and offset halo).
template <int LG>
__device__ void wg_line_pass(const double* src, double* dst, int nr, int64_t M, int m_line,
                             int64_t S, const cplx<double>* tws, const double* lams,
                             double scale, const double* addv, int64_t ldx, int64_t halo,
                             double add_coef) {
    constexpr int L = 1 << LG;
    constexpr int R = line_regs<LG>();
    constexpr int G = L >= 64 ? 1 : 64 / L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_lane = L >= 64 ? lane : (lane & (L - 1));
    const int g_lane = L >= 64 ? 0 : lane / L;
    const int64_t lines_per_vec = M / m_line;
    const int64_t nlines = lines_per_vec * nr;
    const int64_t npairs = (nlines + 1) / 2;
    for (int64_t pb = (int64_t)wave * G; pb < npairs; pb += (int64_t)kBatchWaves * G) {
        const int64_t pair = pb + g_lane;
        int64_t base[2];
        int64_t abase[2];
        bool ok[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t l = 2 * pair + h;
            ok[h] = pair < npairs && l < nlines;
            const int64_t r = ok[h] ? l / lines_per_vec : 0;
            const int64_t li = ok[h] ? l - r * lines_per_vec : 0;
            const int64_t outer = li / S, inner = li - outer * S;
            const int64_t start = outer * m_line * S + inner;
            base[h] = r * M + start;
            abase[h] = r * ldx + halo + start;
        }
        cplx<double> z[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int e = q * 64 + e_lane;
            const bool in = e < m_line;
            z[q].re = (in && ok[0]) ? src[base[0] + e * S] : 0.0;
            z[q].im = (in && ok[1]) ? src[base[1] + e * S] : 0.0;
        }
        conv_line_regs<double, LG>(z, e_lane, tws, lams);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int e = q * 64 + e_lane;
            if (e >= m_line) continue;
            if (ok[0]) {
                double v = scale * z[q].re;
                if (addv) v += add_coef * addv[abase[0] + e * S];
                dst[base[0] + e * S] = v;
            }
            if (ok[1]) {
                double v = scale * z[q].im;
                if (addv) v += add_coef * addv[abase[1] + e * S];
                dst[base[1] + e * S] = v;
            }
        }
    }
}

// Long lines: the workgroup convolves one line pair at a time with the
// four-step FFT (tw1/tw2 in LDS, half-circle twiddles twh and the four-step
// spectrum in global memory, Y: L complex scratch of this work item).
template <int LG1, int LG2>
__device__ void wg_line_pass_long(const double* src, double* dst, int nr, int64_t M, int m_line,
                                  int64_t S, const cplx<double>* tw1, const cplx<double>* tw2,
                                  const cplx<double>* twh, const double* lamp, double scale,
                                  const double* addv, int64_t ldx, int64_t halo, double add_coef,
                                  cplx<double>* Y) {
    const int64_t lines_per_vec = M / m_line;
    const int64_t nlines = lines_per_vec * nr;
    for (int64_t la = 0; la < nlines; la += 2) {
        int64_t base[2] = {0, 0}, abase[2] = {0, 0};
        const bool hb = la + 1 < nlines;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t l = (h == 0 || hb) ? la + h : la;
            const int64_t r = l / lines_per_vec;
            const int64_t li = l - r * lines_per_vec;
            const int64_t outer = li / S, inner = li - outer * S;
            const int64_t start = outer * m_line * S + inner;
            base[h] = r * M + start;
            abase[h] = r * ldx + halo + start;
        }
        wg_conv_long<double, LG1, LG2>(src + base[0], hb ? src + base[1] : nullptr, S, m_line,
                                       dst + base[0], hb ? dst + base[1] : nullptr, scale,
                                       addv ? addv + abase[0] : nullptr,
                                       (addv && hb) ? addv + abase[1] : nullptr, add_coef, Y,
                                       twh, lamp, tw1, tw2);
    }
}

__device__ void wg_line_pass_any(int lg, const double* src, double* dst, int nr, int64_t M,
                                 int m_line, int64_t S, const cplx<double>* tws,
                                 const double* lams, double scale, const double* addv,
                                 int64_t ldx, int64_t halo, double add_coef,
                                 const cplx<double>* tw2, const cplx<double>* twh,
                                 cplx<double>* Y) {
    switch (lg) {
#define FKGP_WLL(LG, A, B)                                                                  \
    case LG:                                                                                \
        wg_line_pass_long<A, B>(src, dst, nr, M, m_line, S, tws, tw2, twh, lams, scale,     \
                                addv, ldx, halo, add_coef, Y);                              \
        break;
        FKGP_WLL(12, 6, 6) FKGP_WLL(13, 6, 7) FKGP_WLL(14, 7, 7)
#undef FKGP_WLL
#define FKGP_WLP(LG)                                                                     \
    case LG:                                                                             \
        wg_line_pass<LG>(src, dst, nr, M, m_line, S, tws, lams, scale, addv, ldx, halo, \
                         add_coef);                                                      \
        break;
        FKGP_WLP(3) FKGP_WLP(4) FKGP_WLP(5) FKGP_WLP(6) FKGP_WLP(7) FKGP_WLP(8)
        FKGP_WLP(9) FKGP_WLP(10) FKGP_WLP(11)
#undef FKGP_WLP
        default:
            break;
    }
}

template <class TA>
__device__ void wg_spmv(const TA* __restrict__ A, const double* __restrict__ rp,
                        double* __restrict__ ur, int nr, const int* done, int64_t M,
                        int64_t ldx, int64_t halo, int NB, const int* offs) {
    for (int64_t j = threadIdx.x; j < M; j += kBatchBlock) {
        double acc[kBatchRhs];
#pragma unroll
        for (int r = 0; r < kBatchRhs; ++r) acc[r] = 0.0;
        const double* xj = rp + halo + j;
        for (int o = 0; o < NB; ++o) {
            const double a = (double)A[dia_index(j, o, NB)];
            const int off = offs[o];
#pragma unroll
            for (int r = 0; r < kBatchRhs; ++r)
                if (r < nr) acc[r] = fma(a, xj[r * ldx + off], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < kBatchRhs; ++r)
            if (r < nr && !done[r]) ur[r * M + j] = acc[r];
    }
}

__global__ __launch_bounds__(kBatchBlock) void batch_cg_kernel(const BatchProb* __restrict__ probs,
                                                               const BatchItem* __restrict__ items,
                                                               double tol, int maxiter) {
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[2 * kBatchRhs * kBatchWaves];
    __shared__ double sums[2 * kBatchRhs];
    __shared__ double rho[kBatchRhs], cr[kBatchRhs], cp[kBatchRhs], cx[kBatchRhs],
        pb[kBatchRhs], alpha[kBatchRhs], beta[kBatchRhs], eps[kBatchRhs];
    __shared__ int done[kBatchRhs], iters[kBatchRhs];
    __shared__ int offs[49];
    __shared__ int all_done;

    const BatchItem it = items[blockIdx.x];
    const BatchProb P = probs[it.prob];
    const int nr = it.nr;
    const int64_t M = P.M, halo = P.halo, ldx = M + 2 * halo;
    const int tid = threadIdx.x;
    // spectra of both dimensions into LDS (long lines: only the twiddles of
    // the two four-step sub-lengths; spectrum and w_L stay in global memory)
    cplx<double>* tws[2] = {nullptr, nullptr};
    cplx<double>* tw2s[2] = {nullptr, nullptr};
    const cplx<double>* twhs[2] = {nullptr, nullptr};
    const double* lams[2] = {nullptr, nullptr};
    {
        unsigned char* p = lds_raw;
        for (int k = 0; k < P.d; ++k) {
            const int L = 1 << P.log2L[k];
            const cplx<double>* twg = static_cast<const cplx<double>*>(P.tw[k]);
            if (P.log2L[k] > kMaxRegLog2) {
                int lg1, lg2;
                long_split(P.log2L[k], lg1, lg2);
                const int L1 = 1 << lg1, L2 = 1 << lg2;
                tws[k] = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L1 / 2);
                tw2s[k] = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L2 / 2);
                for (int i = tid; i < L1 / 2; i += kBatchBlock) tws[k][i] = twg[i * L2];
                for (int i = tid; i < L2 / 2; i += kBatchBlock) tw2s[k][i] = twg[i * L1];
                twhs[k] = twg;
                lams[k] = P.lam[k];
            } else {
                tws[k] = reinterpret_cast<cplx<double>*>(p);
                p += sizeof(cplx<double>) * (L / 2);
                double* lm = reinterpret_cast<double*>(p);
                p += sizeof(double) * L;
                for (int i = tid; i < L / 2; i += kBatchBlock) tws[k][i] = twg[i];
                for (int i = tid; i < L; i += kBatchBlock) lm[i] = P.lam[k][i];
                lams[k] = lm;
            }
        }
    }
    if (tid < P.NB) {
        int o = tid, off = 0;
        if (P.d == 1) {
            off = o - 3;
        } else {
            off = (o / 7 - 3) * P.m[1] + (o % 7 - 3);
        }
        offs[tid] = off;
    }
    // vectors of this item
    double* rp = it.work;                  // [nr][ldx] padded r_hat
    double* ap = rp + (int64_t)kBatchRhs * ldx;
    double* sp = ap + kBatchRhs * M;
    double* zp = sp + kBatchRhs * M;
    double* ux = zp + kBatchRhs * M;
    double* ur = ux + kBatchRhs * M;
    double* vr = ur + kBatchRhs * M;
    const double* bh = P.bh + (int64_t)it.r0 * M;
    const double* kb = P.kb + (int64_t)it.r0 * M;
    for (int64_t i = tid; i < (int64_t)kBatchRhs * ldx; i += kBatchBlock) rp[i] = 0.0;
    for (int64_t i = tid; i < (int64_t)kBatchRhs * M; i += kBatchBlock) {
        sp[i] = 0.0;
        zp[i] = 0.0;
        ux[i] = 0.0;
    }
    if (tid < kBatchRhs) {
        const bool act = tid < nr;
        const double bn = act ? P.bnorm2[it.r0 + tid] : 0.0;
        rho[tid] = bn;
        cr[tid] = 1.0;
        cp[tid] = 1.0;
        cx[tid] = 0.0;
        pb[tid] = 0.0;
        alpha[tid] = 0.0;
        beta[tid] = 0.0;
        eps[tid] = tol * tol * bn;
        done[tid] = (!act || !(bn > 0.0)) ? 1 : 0;
        iters[tid] = 0;
    }
    __syncthreads();

    for (int iter = 0; iter < maxiter; ++iter) {
        if (tid == 0) {
            int a = 1;
            for (int r = 0; r < nr; ++r) a &= done[r];
            all_done = a;
        }
        __syncthreads();
        if (all_done) break;
        // ap = z_p + c_p kappa_b; s_p.ap and ap.b_hat
        {
            double v[2 * kBatchRhs];
#pragma unroll
            for (int k = 0; k < 2 * kBatchRhs; ++k) v[k] = 0.0;
#pragma unroll
            for (int r = 0; r < kBatchRhs; ++r) {
                if (r >= nr || done[r]) continue;
                const double c = cp[r];
                for (int64_t i = tid; i < M; i += kBatchBlock) {
                    const double a = fma(c, kb[r * M + i], zp[r * M + i]);
                    ap[r * M + i] = a;
                    v[2 * r] = fma(sp[r * M + i], a, v[2 * r]);
                    v[2 * r + 1] = fma(a, bh[r * M + i], v[2 * r + 1]);
                }
            }
            wg_sum<2 * kBatchRhs>(v, red, sums);
        }
        if (tid < nr && !done[tid]) {
            const int r = tid;
            const double apc = P.s2 * cp[r];
            const double pap = sums[2 * r] + apc * pb[r] + cp[r] * sums[2 * r + 1] +
                               cp[r] * apc * P.n;
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
        // u_x += alpha s_p; r_hat -= alpha ap
#pragma unroll
        for (int r = 0; r < kBatchRhs; ++r) {
            if (r >= nr || done[r]) continue;
            const double a = alpha[r];
            for (int64_t i = tid; i < M; i += kBatchBlock) {
                ux[r * M + i] = fma(a, sp[r * M + i], ux[r * M + i]);
                rp[r * ldx + halo + i] = fma(-a, ap[r * M + i], rp[r * ldx + halo + i]);
            }
        }
        __syncthreads();
        // u_r = W^T W r_hat
        if (P.a_f32)
            wg_spmv<float>(static_cast<const float*>(P.A), rp, ur, nr, done, M, ldx, halo, P.NB,
                           offs);
        else
            wg_spmv<double>(static_cast<const double*>(P.A), rp, ur, nr, done, M, ldx, halo,
                            P.NB, offs);
        __syncthreads();
        // v_r = s K u_r + s2 r_hat
        if (P.d == 1) {
            wg_line_pass_any(P.log2L[0], ur, vr, nr, M, P.m[0], 1, tws[0], lams[0], P.so, rp,
                             ldx, halo, P.s2, tw2s[0], twhs[0], it.yscr);
        } else {
            wg_line_pass_any(P.log2L[1], ur, vr, nr, M, P.m[1], 1, tws[1], lams[1], 1.0,
                             nullptr, ldx, halo, 0.0, tw2s[1], twhs[1], it.yscr);
            __syncthreads();
            wg_line_pass_any(P.log2L[0], vr, vr, nr, M, P.m[0], P.m[1], tws[0], lams[0], P.so,
                             rp, ldx, halo, P.s2, tw2s[0], twhs[0], it.yscr);
        }
        __syncthreads();
        // rho' = <r, r>, beta
        {
            double v[2 * kBatchRhs];
#pragma unroll
            for (int k = 0; k < 2 * kBatchRhs; ++k) v[k] = 0.0;
#pragma unroll
            for (int r = 0; r < kBatchRhs; ++r) {
                if (r >= nr || done[r]) continue;
                for (int64_t i = tid; i < M; i += kBatchBlock) {
                    const double x = rp[r * ldx + halo + i];
                    v[2 * r] = fma(x, ur[r * M + i], v[2 * r]);
                    v[2 * r + 1] = fma(x, bh[r * M + i], v[2 * r + 1]);
                }
            }
            wg_sum<2 * kBatchRhs>(v, red, sums);
        }
        if (tid < nr && !done[tid]) {
            const int r = tid;
            const double rn = sums[2 * r] + 2.0 * cr[r] * sums[2 * r + 1] + cr[r] * cr[r] * P.n;
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
        __syncthreads();
        // s_p = u_r + beta s_p; z_p = v_r + beta z_p
#pragma unroll
        for (int r = 0; r < kBatchRhs; ++r) {
            if (r >= nr || done[r]) continue;
            const double b = beta[r];
            for (int64_t i = tid; i < M; i += kBatchBlock) {
                sp[r * M + i] = fma(b, sp[r * M + i], ur[r * M + i]);
                zp[r * M + i] = fma(b, zp[r * M + i], vr[r * M + i]);
            }
        }
        __syncthreads();
    }
    // outputs: W^T x = u_x + c_x b_hat, and the final states
#pragma unroll
    for (int r = 0; r < kBatchRhs; ++r) {
        if (r >= nr) continue;
        const double c = cx[r];
        double* out = P.wx + (int64_t)(it.r0 + r) * M;
        for (int64_t i = tid; i < M; i += kBatchBlock) out[i] = fma(c, bh[r * M + i], ux[r * M + i]);
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

}  // namespace

size_t batch_work_doubles(int64_t M, int64_t halo) {
    return (size_t)kBatchRhs * (M + 2 * halo) + (size_t)6 * kBatchRhs * M;
}

fkgp_status launch_batch_cg(const BatchProb* probs_dev, const BatchItem* items_dev, int nitems,
                            size_t lds, double tol, int maxiter, hipStream_t s) {
    if (nitems == 0) return FKGP_OK;
    if (lds > 64 * 1024)
        FKGP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_cg_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    batch_cg_kernel<<<nitems, kBatchBlock, lds, s>>>(probs_dev, items_dev, tol, maxiter);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

}  // namespace fkgp
