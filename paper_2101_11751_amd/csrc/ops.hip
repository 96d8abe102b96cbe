// Per-iteration operators of the factorized solvers: the banded W^T W
// product and K_G = s * T_0 (x) ... (x) T_{d-1} (Sec. 2.3: multilevel
// Toeplitz for a stationary kernel on an equispaced grid, applied with FFTs),
// plus interpolation to query points (Fact 2 mean).
//
// K_G is applied one dimension at a time.  Each line of the grid along
// dimension k is convolved with the symmetric Toeplitz column of T_k through
// a circulant embedding of length L >= 2 m_k - 1 (a power of two), entirely
// in registers: two real lines are packed into one complex line (the
// circulant is real, so real and imaginary parts stay separate), transformed
// by a radix-2 decimation-in-frequency FFT (natural in, bit-reversed out),
// scaled by the real spectrum stored in bit-reversed order, and transformed
// back by the matching decimation-in-time inverse (bit-reversed in, natural
// out).  No padded grid ever touches HBM.  Butterfly spans below 64 use
// wavefront shuffles; larger spans are within a lane's registers.  Each wave
// owns its line pair and reads it straight from global memory (strided
// lines are gathered: the vectors are small and stay in L2), so thousands
// of independent waves hide each other's latency; circulants longer than
// 2048 points take a four-step FFT by one workgroup per line pair.
#include <hip/hip_runtime.h>

#include "common.h"
#include "line_fft.h"

namespace fkgp {
namespace {


// ---------------------------------------------------------------------------
// Line geometry.  Data of k vectors [k][M] are viewed as [outer][m_line][S]:
// line l = (outer, inner) with outer = l / S, inner = l % S.
// ---------------------------------------------------------------------------
struct LineGeom {
    int m_line;
    int64_t S;         // stride between consecutive entries of a line
    int64_t nlines;    // k * M / m_line
};

__device__ inline int64_t line_addr(const LineGeom& lg, int64_t l, int e) {
    const int64_t outer = l / lg.S;
    const int64_t inner = l - outer * lg.S;
    return outer * (int64_t)lg.m_line * lg.S + (int64_t)e * lg.S + inner;
}

constexpr int kLineBlock = 256;

// Two adjacent values as one vector access (16 bytes for FP64, 8 for FP32).
template <class T>
struct Vec2Of;
template <>
struct Vec2Of<double> { using type = double2; };
template <>
struct Vec2Of<float> { using type = float2; };

// The two lines of a pair are adjacent in memory (the next inner index of a
// strided dimension with an even stride) and start at an even element:
// element e of both lines is then one 2-vector, aligned wherever the array
// pointer is (checked with vec2_aligned).
__device__ inline bool pair_adjacent(const bool (&ok)[2], const int64_t (&base)[2], int S32) {
    return ok[0] && ok[1] && base[1] == base[0] + 1 && (base[0] & 1) == 0 && (S32 & 1) == 0;
}

template <class T>
__device__ inline bool vec2_aligned(const T* p) {
    return (reinterpret_cast<uintptr_t>(p) & (2 * sizeof(T) - 1)) == 0;
}

// Store of a line pass: element e = r*64 + e_lane of the (up to two) lines
// at base[h] with stride S32 gets scale * z (+ add_coef * addv); or, with
// fz.s set, the CG direction update of CgStep2 consumes the value in place
// and the last workgroup finishes s^T z.  `active`: this wave holds results
// (all threads of the block must call it when fz.s is set).
template <class T, int R>
__device__ __forceinline__ void line_store(const cplx<T> (&z)[R], int e_lane, bool active,
                                           const bool (&ok)[2], const int64_t (&base)[2],
                                           int S32, int m, T* out, T scale,
                                           const T* __restrict__ addv, T add_coef,
                                           const CgStep2& fz, bool adj = false) {
    using V2 = typename Vec2Of<T>::type;
    if (fz.s) {
        __shared__ double red[kLineBlock];
        const int tid = threadIdx.x;
        double acc = 0.0;
        if (active) {
            const double beta = fz.st->beta;
            const T* uu = static_cast<const T*>(fz.u);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = r * 64 + e_lane;
                if (e >= m) continue;
                if (adj) {   // both lines through 2-vector accesses
                    const int64_t a = base[0] + (int64_t)(e * S32);
                    T v0 = scale * z[r].re, v1 = scale * z[r].im;
                    if (addv) {
                        v0 += add_coef * addv[a];
                        v1 += add_coef * addv[a + 1];
                    }
                    const V2 u2 = *reinterpret_cast<const V2*>(uu + a);
                    const double2 s2 = *reinterpret_cast<const double2*>(fz.s + a);
                    const double2 z2 = *reinterpret_cast<const double2*>(fz.z + a);
                    const double sn0 = fma(beta, s2.x, (double)u2.x);
                    const double sn1 = fma(beta, s2.y, (double)u2.y);
                    const double zn0 = fma(beta, z2.x, (double)v0);
                    const double zn1 = fma(beta, z2.y, (double)v1);
                    *reinterpret_cast<double2*>(fz.s + a) = double2{sn0, sn1};
                    *reinterpret_cast<double2*>(fz.z + a) = double2{zn0, zn1};
                    if (fz.p) {
                        const double2 p2 = *reinterpret_cast<const double2*>(fz.p + a);
                        const double2 r2 = *reinterpret_cast<const double2*>(fz.r + a);
                        *reinterpret_cast<double2*>(fz.p + a) =
                            double2{fma(beta, p2.x, r2.x), fma(beta, p2.y, r2.y)};
                    }
                    acc = fma(sn0, zn0, acc);
                    acc = fma(sn1, zn1, acc);
                    continue;
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (!ok[h]) continue;
                    const int64_t a = base[h] + (int64_t)(e * S32);
                    T v = scale * (h == 0 ? z[r].re : z[r].im);
                    if (addv) v += add_coef * addv[a];
                    const double sn = fma(beta, fz.s[a], (double)uu[a]);
                    const double zn = fma(beta, fz.z[a], (double)v);
                    fz.s[a] = sn;
                    fz.z[a] = zn;
                    if (fz.p) fz.p[a] = fma(beta, fz.p[a], fz.r[a]);
                    acc = fma(sn, zn, acc);
                }
            }
        }
        red[tid] = acc;
        __syncthreads();
        for (int s2 = kLineBlock / 2; s2 > 0; s2 >>= 1) {
            if (tid < s2) red[tid] += red[tid + s2];
            __syncthreads();
        }
        last_block_finish(fz.lb, red[0], red);
        return;
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + e_lane;
        if (e >= m) continue;
        if (adj) {
            const int64_t a = base[0] + (int64_t)(e * S32);
            T v0 = scale * z[r].re, v1 = scale * z[r].im;
            if (addv) {
                v0 += add_coef * addv[a];
                v1 += add_coef * addv[a + 1];
            }
            V2 o;
            o.x = v0;
            o.y = v1;
            *reinterpret_cast<V2*>(out + a) = o;
            continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!ok[h]) continue;
            const int64_t a = base[h] + (int64_t)(e * S32);
            T v = scale * (h == 0 ? z[r].re : z[r].im);
            if (addv) v += add_coef * addv[a];
            out[a] = v;
        }
    }
}

// The two innermost dimensions of a 3-D grid in one pass, by the dense
// products with their symmetric Toeplitz factors (Sec. 2.3: each factor of
// K_G is the Toeplitz matrix of the kernel on an equispaced line):
// y[o, :, :] = T_1 x[o, :, :] T_2, exact up to rounding (no truncation of
// the band), for slabs of m_1 x m_2 <= 4096 nodes with m_1 <= 128, m_2 <= 64.
// Where the line FFT spends its time in the latency of each pass's exchange
// chain (two launches and two round trips through memory), this is one
// launch at m_1 + m_2 FMAs per node.
//
// Workgroup (slab o, part p): the slab (contiguous in memory) is loaded into
// LDS once, T_2 is applied along every row (all rows: the next product
// needs them), then T_1 along the columns for this part's output rows, which
// are written straight out (parts read the whole slab and write disjoint
// rows, so an in-place call takes one part).  Both products use register
// blocks of 8 x 8: per block, 8 reads of the data, 15 of the column
// c[|i - j|] (held in LDS padded with zeros beyond the band) and 64 FMAs.
// No divisions in the index arithmetic except per-thread setup.
constexpr int kSlabR = 8;
constexpr int kSlabMaxM1 = 128, kSlabMaxM2 = 64, kSlabMaxNodes = 4096;

__host__ __device__ inline int slab_pad(int m) { return (m + kSlabR - 1) / kSlabR * kSlabR; }

// Rows of the column product per part: 8-row blocks times the column count
// that fills 256 threads.
__host__ __device__ inline int slab_part_rows(int m2) {
    const int blocks = 256 / m2 > 0 ? 256 / m2 : 1;
    return blocks * kSlabR;
}

// register-blocked Toeplitz product along one direction of an LDS tile:
// out(i0 + r) = sum_j c[|i0 + r - j|] v(j), r < R, with v(j) = V[j * sv] and
// cx[t] = c[|t - R - (m - 1)|] (zero outside the band).
template <class T>
__device__ __forceinline__ void slab_block(const T* V, int sv, const T* cx, int m, int i0,
                                           T (&acc)[kSlabR]) {
    constexpr int R = kSlabR;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    const int mp = slab_pad(m);
    for (int jb = 0; jb < mp; jb += R) {
        T xv[R], cw[2 * R - 1];
#pragma unroll
        for (int q = 0; q < R; ++q) xv[q] = V[(jb + q) * sv];
        const int cb = i0 - jb + m;   // cx[cb + t] = c[|i - j|], t = r - q + R - 1
#pragma unroll
        for (int t = 0; t < 2 * R - 1; ++t) cw[t] = cx[cb + t];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < R; ++q) acc[r] = fma(cw[r - q + R - 1], xv[q], acc[r]);
    }
}

template <class T>
__global__ __launch_bounds__(256) void toeplitz_slab(const T* in, T* out, int m1, int m2,
                                                     int parts, int prow,
                                                     const T* __restrict__ col1,
                                                     const T* __restrict__ col2,
                                                     const int* __restrict__ skip) {
    constexpr int R = kSlabR;
    extern __shared__ unsigned char slab_lds[];
    if (skip && *skip) return;
    const int tid = threadIdx.x;
    const int mp1 = slab_pad(m1), mp2 = slab_pad(m2);
    const int sx = mp2 + 1;                      // row stride of X and Y (odd: LDS banks)
    T* X = reinterpret_cast<T*>(slab_lds);       // [mp1][sx], zero padded
    T* Y = X + mp1 * sx;                         // [mp1][sx]
    T* c1x = Y + mp1 * sx;                       // [2 mp1 + 2R]
    T* c2x = c1x + 2 * mp1 + 2 * R;              // [2 mp2 + 2R]
    const unsigned b = xcd_block();
    const int64_t slab = b / (unsigned)parts;
    const int part = (int)(b - slab * (unsigned)parts);
    const int ns = m1 * m2;
    const T* src = in + slab * ns;
    T* dst = out + slab * ns;
    // load the slab: element idx = tid + 256 e sits at (idx / m2, idx % m2),
    // stepped without per-element division
    {
        constexpr int kMaxE = kSlabMaxNodes / 256;
        T v[kMaxE];
#pragma unroll
        for (int e = 0; e < kMaxE; ++e) {
            const int idx = tid + 256 * e;
            v[e] = idx < ns ? src[idx] : T(0);
        }
        for (int t = tid; t < mp1 * sx; t += 256) {   // zero everything first
            X[t] = T(0);
            Y[t] = T(0);
        }
        for (int t = tid; t < 2 * mp1 + 2 * R; t += 256) {
            const int dl = t - R - (m1 - 1);
            const int a = dl < 0 ? -dl : dl;
            c1x[t] = a < m1 ? col1[a] : T(0);
        }
        for (int t = tid; t < 2 * mp2 + 2 * R; t += 256) {
            const int dl = t - R - (m2 - 1);
            const int a = dl < 0 ? -dl : dl;
            c2x[t] = a < m2 ? col2[a] : T(0);
        }
        __syncthreads();
        const int q256 = 256 / m2, r256 = 256 - q256 * m2;
        int row = tid / m2, cl = tid - (tid / m2) * m2;
#pragma unroll
        for (int e = 0; e < kMaxE; ++e) {
            if (tid + 256 * e < ns) X[row * sx + cl] = v[e];
            row += q256;
            cl += r256;
            if (cl >= m2) {
                cl -= m2;
                ++row;
            }
        }
    }
    __syncthreads();
    // T_2 along the rows: task (row i, column block k), column blocks fastest
    {
        const int nb2 = mp2 / R;
        const int ntask = m1 * nb2;
        for (int task = tid; task < ntask; task += 256) {
            const int i = task / nb2, k = task - (task / nb2) * nb2;
            T acc[R];
            slab_block<T>(X + i * sx, 1, c2x, m2, k * R, acc);
#pragma unroll
            for (int r = 0; r < R; ++r) Y[i * sx + k * R + r] = acc[r];
        }
    }
    __syncthreads();
    // T_1 along the columns for this part's prow rows: task (row block,
    // column), columns fastest (consecutive lanes read consecutive Y entries
    // and write consecutive outputs)
    {
        const int r_lo = part * prow;
        const int r_hi = min(m1, r_lo + prow);
        const int nbr = (r_hi - r_lo + R - 1) / R;
        const int ntask = nbr * m2;
        for (int task = tid; task < ntask; task += 256) {
            const int kb = task / m2, c = task - (task / m2) * m2;
            const int i0 = r_lo + kb * R;
            T acc[R];
            slab_block<T>(Y + c, sx, c1x, m1, i0, acc);
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (i0 + r < r_hi) dst[(i0 + r) * m2 + c] = acc[r];
        }
    }
}

// The outermost dimension (stride S = M / m_0 per vector, m_0 <= 128) by
// the dense product with its Toeplitz factor, the last pass of K_G after the
// slab pass: y[i, c] = scale * sum_j c0[|i - j|] x[j, c] (+ add_coef *
// addv), c < S, for k vectors.  A workgroup owns 16 adjacent columns c of
// one vector and all m_0 rows (rows are 16 consecutive values: one 128-byte
// chunk per row), thread (row block, column) forms 8 rows of one column by
// the register-blocked product; the store takes the line passes' epilogue,
// including the fused CG direction update (CgStep2).  Every global load of
// the pass (tile, column, epilogue operands) is issued up front; all index
// arithmetic is multiplications and additions.
constexpr int kColsC = 16;

template <class T>
__global__ __launch_bounds__(256) void toeplitz_cols(const T* x, T* y, int m0, int64_t S,
                                                     int64_t tiles_per_vec,
                                                     const T* __restrict__ col, T scale,
                                                     const T* __restrict__ addv, T add_coef,
                                                     const int* __restrict__ skip, CgStep2 fz) {
    constexpr int R = kSlabR, C = kColsC, CS = C + 1;
    constexpr int MP = 16 * R;                     // rows covered (m_0 <= 128)
    constexpr int kE = MP * C / 256;               // tile entries per thread (8)
    __shared__ T tile[MP * CS];
    __shared__ T cx[2 * MP + 2 * R];
    __shared__ double red[256];
    if (skip && *skip) return;
    const int tid = threadIdx.x;
    const unsigned b = xcd_block();
    const int64_t vec = b / tiles_per_vec;
    const int64_t c0 = (int64_t)(b - vec * tiles_per_vec) * C;
    const int64_t base = vec * (int64_t)m0 * S + c0;
    const int c = tid % C, rb = tid / C;           // column, row block / load row offset
    const bool cok = c0 + c < S;
    // entries (i = rb + 16 e, c): address base + i S + c
    T v[kE], av[kE], uv[kE];
    double sv[kE], zv[kE], pv[kE], rv[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int i = rb + 16 * e;
        v[e] = (cok && i < m0) ? x[base + (int64_t)i * S + c] : T(0);
    }
    // epilogue operands of this thread's outputs (rows rb * R + r)
    const int i0 = rb * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        const bool ok = cok && i < m0;
        const int64_t a = base + (int64_t)i * S + c;
        av[r] = (ok && addv) ? addv[a] : T(0);
        if (fz.s) {
            sv[r] = ok ? fz.s[a] : 0.0;
            zv[r] = ok ? fz.z[a] : 0.0;
            uv[r] = ok ? static_cast<const T*>(fz.u)[a] : T(0);
            if (fz.p) {
                pv[r] = ok ? fz.p[a] : 0.0;
                rv[r] = ok ? fz.r[a] : 0.0;
            }
        }
    }
    for (int t = tid; t < 2 * MP + 2 * R; t += 256) {
        const int dl = t - R - (m0 - 1);
        const int a = dl < 0 ? -dl : dl;
        cx[t] = a < m0 ? col[a] : T(0);
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) tile[(rb + 16 * e) * CS + c] = v[e];   // zeros where absent
    __syncthreads();
    T acc[R];
    slab_block<T>(tile + c, CS, cx, m0, i0, acc);
    double part = 0.0;
    const double beta = fz.s ? fz.st->beta : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        if (!cok || i >= m0) continue;
        const int64_t a = base + (int64_t)i * S + c;
        T w = scale * acc[r];
        if (addv) w += add_coef * av[r];
        if (fz.s) {
            const double sn = fma(beta, sv[r], (double)uv[r]);
            const double zn = fma(beta, zv[r], (double)w);
            fz.s[a] = sn;
            fz.z[a] = zn;
            if (fz.p) fz.p[a] = fma(beta, pv[r], rv[r]);
            part = fma(sn, zn, part);
        } else {
            y[a] = w;
        }
    }
    if (fz.s) {
        red[tid] = part;
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (tid < s2) red[tid] += red[tid + s2];
            __syncthreads();
        }
        last_block_finish(fz.lb, red[0], red);
    }
}

// Barrier-free variant: each wave convolves its own line pair (64/L pairs
// when L < 64), loading the lines straight from global memory (strided
// lines are gathered; the vector is small enough to stay in L2) with
// twiddles and spectrum read through the cache.  Many independent waves
// hide each other's latency, where a block-wide LDS transpose leaves one
// dependent load-FFT-store chain per CU.  Optionally fuses the CG direction
// update into the store (see CgStep2).
template <class T, int LOG2L>
__global__ __launch_bounds__(kLineBlock) void line_conv_direct(
    const T* in, T* out, LineGeom lg, const T* __restrict__ lam_br,
    const cplx<T>* __restrict__ tw, T scale, const T* __restrict__ addv, T add_coef,
    const int* __restrict__ skip, CgStep2 fz) {
    constexpr int L = 1 << LOG2L;
    constexpr int R = L >= 64 ? L / 64 : 1;
    constexpr int G = L >= 64 ? 1 : 64 / L;
    if (skip && *skip) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int e_lane = L >= 64 ? lane : (lane & (L - 1));
    const int g_lane = L >= 64 ? 0 : (lane / L);
    const int64_t npairs = (lg.nlines + 1) / 2;
    const int64_t pair = ((int64_t)xcd_block() * (kLineBlock / 64) + (tid >> 6)) * G + g_lane;
    const int m = lg.m_line;
    const int S32 = (int)lg.S;
    int64_t base[2] = {0, 0};
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t l = 2 * pair + h;
        ok[h] = pair < npairs && l < lg.nlines;
        if (ok[h]) base[h] = line_addr(lg, l, 0);
    }
    using V2 = typename Vec2Of<T>::type;
    const bool pair_adj = pair_adjacent(ok, base, S32);
    const bool adj = pair_adj && vec2_aligned(in + base[0]);
    bool adj_st = pair_adj && vec2_aligned(out + base[0]);
    if (fz.s)
        adj_st = pair_adj && vec2_aligned(fz.s + base[0]) && vec2_aligned(fz.z + base[0]) &&
                 vec2_aligned(static_cast<const T*>(fz.u) + base[0]) &&
                 (!fz.p || (vec2_aligned(fz.p + base[0]) && vec2_aligned(fz.r + base[0])));
    cplx<T> z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + e_lane;
        const bool in_line = e < m;
        if (adj) {
            V2 v;
            v.x = T(0);
            v.y = T(0);
            if (in_line) v = *reinterpret_cast<const V2*>(in + base[0] + (int64_t)(e * S32));
            z[r].re = v.x;
            z[r].im = v.y;
        } else {
            z[r].re = (in_line && ok[0]) ? in[base[0] + (int64_t)(e * S32)] : T(0);
            z[r].im = (in_line && ok[1]) ? in[base[1] + (int64_t)(e * S32)] : T(0);
        }
    }
    conv_line_regs<T, LOG2L>(z, e_lane, tw, lam_br);
    line_store<T, R>(z, e_lane, true, ok, base, S32, m, out, scale, addv, add_coef, fz, adj_st);
}

// Line pairs split over two waves (used for L >= 512; at 256 points the
// duplicated gathers and the exchange cost more than the shorter chains
// save).  The circulant input is zero in its upper half (m <= L/2), so the
// first decimation-in-frequency stage (span L/2) needs no exchange: wave
// half 0 keeps x[e], wave half 1 takes x[e] w^e (e < L/2, both load the same
// entries).  Each wave then runs the
// remaining length-L/2 transform (the even twiddles), the spectrum entries of
// its half of the bit-reversed order and the inverse stages up to span L/4;
// the last inverse stage (span L/2) adds the upper half's b conj(w^e)
// through LDS, forming only the outputs e < L/2 (m <= L/2 are needed).
// Half the registers and butterflies of a one-wave line per wave, twice the
// waves: shorter dependent chains and more latency hiding.
template <class T, int LOG2L>
__global__ __launch_bounds__(kLineBlock) void line_conv_split(
    const T* in, T* out, LineGeom lg, const T* __restrict__ lam_br,
    const cplx<T>* __restrict__ tw, T scale, const T* __restrict__ addv, T add_coef,
    const int* __restrict__ skip, CgStep2 fz) {
    constexpr int L = 1 << LOG2L;
    constexpr int H = L / 2;
    constexpr int R = H / 64;
    constexpr int kPairs = kLineBlock / 128;
    static_assert(H >= 64, "split lines need L >= 128");
    __shared__ cplx<T> xch[kPairs][H];
    if (skip && *skip) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int half = wave & 1, slot = wave >> 1;
    const int64_t npairs = (lg.nlines + 1) / 2;
    const int64_t pair = (int64_t)xcd_block() * kPairs + slot;
    const int m = lg.m_line;
    const int S32 = (int)lg.S;
    int64_t base[2] = {0, 0};
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t l = 2 * pair + h;
        ok[h] = pair < npairs && l < lg.nlines;
        if (ok[h]) base[h] = line_addr(lg, l, 0);
    }
    using V2 = typename Vec2Of<T>::type;
    const bool pair_adj = pair_adjacent(ok, base, S32);
    const bool adj = pair_adj && vec2_aligned(in + base[0]);
    bool adj_st = pair_adj && vec2_aligned(out + base[0]);
    if (fz.s)
        adj_st = pair_adj && vec2_aligned(fz.s + base[0]) && vec2_aligned(fz.z + base[0]) &&
                 vec2_aligned(static_cast<const T*>(fz.u) + base[0]) &&
                 (!fz.p || (vec2_aligned(fz.p + base[0]) && vec2_aligned(fz.r + base[0])));
    cplx<T> z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        const bool in_line = e < m;
        if (adj) {
            V2 v;
            v.x = T(0);
            v.y = T(0);
            if (in_line) v = *reinterpret_cast<const V2*>(in + base[0] + (int64_t)(e * S32));
            z[r].re = v.x;
            z[r].im = v.y;
        } else {
            z[r].re = (in_line && ok[0]) ? in[base[0] + (int64_t)(e * S32)] : T(0);
            z[r].im = (in_line && ok[1]) ? in[base[1] + (int64_t)(e * S32)] : T(0);
        }
    }
    if (half) {   // first DIF stage, upper outputs: (x[e] - 0) w^e
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] = cmul(z[r], tw[r * 64 + lane]);
    }
    dif_regs<T, LOG2L - 1, 2>(z, lane, tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T lmb = lam_br[half * H + r * 64 + lane];
        z[r].re *= lmb;
        z[r].im *= lmb;
    }
    dit_regs<T, LOG2L - 1, 2>(z, lane, tw);
    if (half) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = r * 64 + lane;
            xch[slot][e] = cmul_conj(z[r], tw[e]);
        }
    }
    __syncthreads();
    if (!half) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const cplx<T> t = xch[slot][r * 64 + lane];
            z[r].re += t.re;
            z[r].im += t.im;
        }
    }
    line_store<T, R>(z, lane, half == 0, ok, base, S32, m, out, scale, addv, add_coef, fz,
                     adj_st);
}

// Long lines: one workgroup per line pair at a time (grid-stride over the
// pairs), four-step convolution through its own L-point scratch.
template <class T, int LG1, int LG2, int BS>
__global__ __launch_bounds__(BS) void line_conv_long(
    const T* in, T* out, LineGeom lg, const T* __restrict__ lamp,
    const cplx<T>* __restrict__ twh, T scale, const T* addv, T add_coef,
    const int* __restrict__ skip, cplx<T>* __restrict__ scr) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2;
    if (skip && *skip) return;
    __shared__ cplx<T> tw1[L1 / 2], tw2[L2 / 2];
    for (int t = threadIdx.x; t < L1 / 2; t += BS) tw1[t] = twh[t * L2];
    for (int t = threadIdx.x; t < L2 / 2; t += BS) tw2[t] = twh[t * L1];
    __syncthreads();
    cplx<T>* Y = scr + (int64_t)blockIdx.x * (L1 * L2);
    const int64_t npairs = (lg.nlines + 1) / 2;
    for (int64_t pair = blockIdx.x; pair < npairs; pair += gridDim.x) {
        const int64_t la = 2 * pair, lb = la + 1;
        const bool hb = lb < lg.nlines;
        const int64_t ba = line_addr(lg, la, 0);
        const int64_t bb = hb ? line_addr(lg, lb, 0) : 0;
        wg_conv_long<T, LG1, LG2>(in + ba, hb ? in + bb : nullptr, lg.S, lg.m_line, out + ba,
                                  hb ? out + bb : nullptr, scale, addv ? addv + ba : nullptr,
                                  (addv && hb) ? addv + bb : nullptr, add_coef, Y, twh, lamp,
                                  tw1, tw2);
    }
}

// Long lines with few line pairs: the three phases of the four-step
// convolution (see wg_conv_long) as three launches, one column or row per
// wave, so that a single long line spreads over the whole chip instead of
// one workgroup.  Block b of a phase handles pair b / per_pair and the four
// columns (rows) 4 (b % per_pair) .. + 3.  Y: L complex per pair.
template <class T, int LG1, int LG2, int BS>
__global__ __launch_bounds__(BS) void fs_cols_fwd(const T* in, LineGeom lg,
                                                   const cplx<T>* __restrict__ twh,
                                                   const int* __restrict__ skip,
                                                   cplx<T>* __restrict__ scr) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2, L = L1 * L2;
    constexpr int R1 = line_regs<LG1>();
    constexpr int W = BS / 64;   // consecutive columns per block
    if (skip && *skip) return;
    __shared__ cplx<T> tw1[L1 / 2];
    for (int t = threadIdx.x; t < L1 / 2; t += BS) tw1[t] = twh[t * L2];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned b = xcd_block();
    const int64_t pair = b / (L2 / W);
    const int n2 = (int)(b % (L2 / W)) * W + wave;
    const int64_t la = 2 * pair, lb = la + 1;
    const bool hb = lb < lg.nlines;
    const T* srcA = in + line_addr(lg, la, 0);
    const T* srcB = hb ? in + line_addr(lg, lb, 0) : nullptr;
    cplx<T> z[R1];
#pragma unroll
    for (int q = 0; q < R1; ++q) {
        const int n = L2 * (q * 64 + lane) + n2;
        z[q].re = (n < lg.m_line) ? srcA[(int64_t)n * lg.S] : T(0);
        z[q].im = (n < lg.m_line && srcB) ? srcB[(int64_t)n * lg.S] : T(0);
    }
    dif_regs<T, LG1>(z, lane, tw1);
    cplx<T>* Y = scr + pair * L;
#pragma unroll
    for (int q = 0; q < R1; ++q) {
        const int p1 = q * 64 + lane;
        unsigned t = ((unsigned)n2 * bitrev_bits((unsigned)p1, LG1)) & (unsigned)(L - 1);
        cplx<T> w;
        if (t < (unsigned)(L / 2)) {
            w = twh[t];
        } else {
            const cplx<T> v = twh[t - L / 2];
            w = {-v.re, -v.im};
        }
        Y[p1 * L2 + n2] = cmul(z[q], w);
    }
}

template <class T, int LG1, int LG2>
__global__ __launch_bounds__(256) void fs_rows(const cplx<T>* __restrict__ twh,
                                               const T* __restrict__ lamp,
                                               const int* __restrict__ skip,
                                               cplx<T>* __restrict__ scr) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2, L = L1 * L2;
    constexpr int R2 = line_regs<LG2>();
    if (skip && *skip) return;
    __shared__ cplx<T> tw2[L2 / 2];
    for (int t = threadIdx.x; t < L2 / 2; t += 256) tw2[t] = twh[t * L1];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned b = xcd_block();
    const int64_t pair = b / (L1 / 4);
    const int p1 = (int)(b % (L1 / 4)) * 4 + wave;
    cplx<T>* Y = scr + pair * L;
    cplx<T> z[R2];
#pragma unroll
    for (int q = 0; q < R2; ++q) z[q] = Y[p1 * L2 + q * 64 + lane];
    dif_regs<T, LG2>(z, lane, tw2);
#pragma unroll
    for (int q = 0; q < R2; ++q) {
        const T lm = lamp[p1 * L2 + q * 64 + lane];
        z[q].re *= lm;
        z[q].im *= lm;
    }
    dit_regs<T, LG2>(z, lane, tw2);
    const unsigned br = bitrev_bits((unsigned)p1, LG1);
#pragma unroll
    for (int q = 0; q < R2; ++q) {
        const int n2 = q * 64 + lane;
        const unsigned t = ((unsigned)n2 * br) & (unsigned)(L - 1);
        cplx<T> w;
        if (t < (unsigned)(L / 2)) {
            w = twh[t];
        } else {
            const cplx<T> v = twh[t - L / 2];
            w = {-v.re, -v.im};
        }
        Y[p1 * L2 + n2] = cmul_conj(z[q], w);
    }
}

template <class T, int LG1, int LG2, int BS>
__global__ __launch_bounds__(BS) void fs_cols_inv(T* out, LineGeom lg,
                                                   const cplx<T>* __restrict__ twh, T scale,
                                                   const T* addv, T add_coef,
                                                   const int* __restrict__ skip,
                                                   const cplx<T>* __restrict__ scr) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2, L = L1 * L2;
    constexpr int R1 = line_regs<LG1>();
    constexpr int W = BS / 64;   // consecutive columns per block
    if (skip && *skip) return;
    __shared__ cplx<T> tw1[L1 / 2];
    for (int t = threadIdx.x; t < L1 / 2; t += BS) tw1[t] = twh[t * L2];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned b = xcd_block();
    const int64_t pair = b / (L2 / W);
    const int n2 = (int)(b % (L2 / W)) * W + wave;
    const int64_t la = 2 * pair, lb = la + 1;
    const bool hb = lb < lg.nlines;
    const int64_t ba = line_addr(lg, la, 0), bb = hb ? line_addr(lg, lb, 0) : 0;
    const cplx<T>* Y = scr + pair * L;
    cplx<T> z[R1];
#pragma unroll
    for (int q = 0; q < R1; ++q) z[q] = Y[(q * 64 + lane) * L2 + n2];
    dit_regs<T, LG1>(z, lane, tw1);
#pragma unroll
    for (int q = 0; q < R1; ++q) {
        const int n = L2 * (q * 64 + lane) + n2;
        if (n >= lg.m_line) continue;
        const int64_t o = (int64_t)n * lg.S;
        T va = scale * z[q].re;
        if (addv) va += add_coef * addv[ba + o];
        out[ba + o] = va;
        if (hb) {
            T vb = scale * z[q].im;
            if (addv) vb += add_coef * addv[bb + o];
            out[bb + o] = vb;
        }
    }
}

// Few pairs of circulants of at least 2^kSplitPhasesLog2 points take the
// three-launch path.
constexpr int kSplitPhasesLog2 = 12;
// Column phases: 16 consecutive columns per block (one per wave), so the
// strided accesses of neighbouring columns meet in one L2, when that still
// gives kFsWideMinBlocks blocks; else 4 columns per block (more blocks).
constexpr int64_t kFsWideMinBlocks = 512;
constexpr int64_t kSplitPhasesMaxPairs = 128;

// Blocks of a barrier-free pass: one line pair per wave (64/L per wave for
// L < 64), four waves per block.
// Lines of at least kSplitLog2 points are split over two waves per pair.
constexpr int kSplitLog2 = 9;

// Workgroups of a register-resident line pass (one per 4 pairs, one per 2
// pairs when split, 64/L pairs per wave for L < 64).
static unsigned line_direct_blocks(int log2L, const LineGeom& lg) {
    const int64_t npairs = (lg.nlines + 1) / 2;
    if (log2L >= kSplitLog2)
        return (unsigned)std::max<int64_t>(1, (npairs + kLineBlock / 128 - 1) / (kLineBlock / 128));
    const int64_t G = log2L >= 6 ? 1 : (64 >> log2L);
    const int64_t waves = (npairs + G - 1) / G;
    return (unsigned)std::max<int64_t>(1, (waves + kLineBlock / 64 - 1) / (kLineBlock / 64));
}

template <class T>
fkgp_status launch_line_conv(int log2L, int lg1, const T* in, T* out, const LineGeom& lg,
                             const T* lam, const cplx<T>* tw, T scale, const T* addv,
                             T add_coef, const int* skip, cplx<T>* scr, hipStream_t s,
                             const CgStep2* fuse = nullptr) {
    if (lg1 > 0) {
        int want1, want2;
        long_split(log2L, want1, want2);
        if (!scr || log2L < kFewLinesMinLog2 || lg1 != want1) {
            set_error("spectra not laid out for the standalone line FFT");
            return FKGP_EINVAL;
        }
        const int64_t npairs = (lg.nlines + 1) / 2;
        const unsigned grid = (unsigned)std::min<int64_t>(npairs, kLongWGs);
        if (grid == 0) return FKGP_OK;
        if (log2L >= kSplitPhasesLog2 && npairs <= kSplitPhasesMaxPairs) {
#define FKGP_FS(LG, A, B)                                                                      \
    case LG: {                                                                                 \
        const int64_t c16 = npairs * ((1 << B) / 16);                                          \
        const unsigned gr = (unsigned)(npairs * ((1 << A) / 4));                               \
        if (c16 >= kFsWideMinBlocks) {                                                         \
            fs_cols_fwd<T, A, B, 1024><<<(unsigned)c16, 1024, 0, s>>>(in, lg, tw, skip, scr);  \
            fs_rows<T, A, B><<<gr, 256, 0, s>>>(tw, lam, skip, scr);                           \
            fs_cols_inv<T, A, B, 1024><<<(unsigned)c16, 1024, 0, s>>>(out, lg, tw, scale,      \
                                                                      addv, add_coef, skip,    \
                                                                      scr);                    \
        } else {                                                                               \
            const unsigned c4 = (unsigned)(npairs * ((1 << B) / 4));                           \
            fs_cols_fwd<T, A, B, 256><<<c4, 256, 0, s>>>(in, lg, tw, skip, scr);               \
            fs_rows<T, A, B><<<gr, 256, 0, s>>>(tw, lam, skip, scr);                           \
            fs_cols_inv<T, A, B, 256><<<c4, 256, 0, s>>>(out, lg, tw, scale, addv, add_coef,   \
                                                          skip, scr);                          \
        }                                                                                      \
        break;                                                                                 \
    }
            switch (log2L) {
                FKGP_FS(12, 6, 6)
                FKGP_FS(13, 6, 7)
                FKGP_FS(14, 7, 7)
                FKGP_FS(15, 7, 8)
                FKGP_FS(16, 8, 8)
                FKGP_FS(17, 8, 9)
                default:
                    set_error("no split four-step pass for this length");
                    return FKGP_EINVAL;
            }
#undef FKGP_FS
            FKGP_HIP(hipGetLastError());
            return FKGP_OK;
        }
        // few pairs: 16 waves per pair (the phases' independent columns and
        // rows spread over more waves); else 4 waves and more workgroups
        const bool wide = npairs <= kFewLines;
#define FKGP_LL(LG, A, B)                                                                      \
    case LG:                                                                                   \
        if (wide)                                                                              \
            line_conv_long<T, A, B, 1024><<<grid, 1024, 0, s>>>(in, out, lg, lam, tw, scale,   \
                                                                 addv, add_coef, skip, scr);   \
        else                                                                                   \
            line_conv_long<T, A, B, kLineBlock><<<grid, kLineBlock, 0, s>>>(                   \
                in, out, lg, lam, tw, scale, addv, add_coef, skip, scr);                       \
        break;
        switch (log2L) {
            FKGP_LL(10, 5, 5)
            FKGP_LL(11, 5, 6)
            FKGP_LL(12, 6, 6)
            FKGP_LL(13, 6, 7)
            FKGP_LL(14, 7, 7)
            FKGP_LL(15, 7, 8)
            FKGP_LL(16, 8, 8)
            FKGP_LL(17, 8, 9)
            default:
                set_error("grid dimension too long for the line FFT (at most 65536 nodes)");
                return FKGP_EINVAL;
        }
#undef FKGP_LL
        FKGP_HIP(hipGetLastError());
        return FKGP_OK;
    }
    // lines per block: enough blocks to cover the chip (>= ~2 per CU), at
    // least 8 lines for strided dimensions (64-byte coalesced rows), at most
    // what fits in 48 KiB of LDS; even.
    if (log2L > kMaxRegLog2) {
        set_error("spectra not laid out for the standalone line FFT");
        return FKGP_EINVAL;
    }
    CgStep2 fz{};
    if (fuse) fz = *fuse;
    const unsigned grid = line_direct_blocks(log2L, lg);
#define FKGP_LC(LG)                                                                          \
    case LG:                                                                                 \
        line_conv_direct<T, LG><<<grid, kLineBlock, 0, s>>>(in, out, lg, lam, tw, scale,      \
                                                             addv, add_coef, skip, fz);      \
        break;
#define FKGP_LS(LG)                                                                          \
    case LG:                                                                                 \
        line_conv_split<T, LG><<<grid, kLineBlock, 0, s>>>(in, out, lg, lam, tw, scale,       \
                                                            addv, add_coef, skip, fz);       \
        break;
    switch (log2L) {
        FKGP_LC(3) FKGP_LC(4) FKGP_LC(5) FKGP_LC(6) FKGP_LC(7) FKGP_LC(8) FKGP_LS(9)
        FKGP_LS(10) FKGP_LS(11)   // kSplitLog2 = 9
        default:
            set_error("grid dimension too long for the register-resident line FFT");
            return FKGP_EINVAL;
    }
#undef FKGP_LC
#undef FKGP_LS
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// ---------------------------------------------------------------------------
// Spectra and twiddles (FP64 on the device, cast to the working dtype).
// ---------------------------------------------------------------------------
// One-dimensional kernel at lag j (r = j h / l) or, with deriv, its
// derivative in log l (r dk/dlog l = -r dk/dr).
__device__ inline double kernel_col(int kind, int j, double h, double ell, bool deriv) {
    const double r = (double)j * h / ell;
    switch (kind) {
        case FKGP_KERNEL_MATERN12: {
            const double e = exp(-r);
            return deriv ? r * e : e;
        }
        case FKGP_KERNEL_MATERN32: {
            const double a = sqrt(3.0) * r, e = exp(-a);
            return deriv ? 3.0 * r * r * e : (1.0 + a) * e;
        }
        case FKGP_KERNEL_MATERN52: {
            const double a = sqrt(5.0) * r, e = exp(-a);
            return deriv ? (5.0 / 3.0) * r * r * (1.0 + a) * e
                         : (1.0 + a + (5.0 / 3.0) * r * r) * e;
        }
        default: {
            const double c = exp(-0.5 * r * r);
            return deriv ? c * r * r : c;
        }
    }
}

__device__ inline unsigned bitrev(unsigned v, int bits) {
    return __brev(v) >> (32 - bits);
}

// lam_br[e] = (1/L) sum_j c_emb[j] cos(2 pi j f / L), f = bitrev(e) (or the
// four-step order of long lines, lg1 > 0); the
// circulant embedding is c_emb[j] = c[min(j, L-j)] for min(j, L-j) < m,
// else 0 (symmetric, so the DFT is real).
template <class T>
__global__ void spectrum_kernel(T* __restrict__ lam_br, int log2L, int lg1, int m, double h,
                                double ell, bool deriv, int kind) {
    const int L = 1 << log2L;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= L) return;
    unsigned f;
    if (lg1 > 0) {   // four-step order: e = p1 * L2 + p2
        const int lg2 = log2L - lg1;
        const unsigned p1 = (unsigned)e >> lg2, p2 = (unsigned)e & ((1u << lg2) - 1u);
        f = bitrev(p1, lg1) + (bitrev(p2, lg2) << lg1);
    } else {
        f = bitrev((unsigned)e, log2L);
    }
    double acc = kernel_col(kind, 0, h, ell, deriv);
    for (int j = 1; j < m; ++j) {
        if (L - j < j) break;
        const unsigned long long ph = ((unsigned long long)j * f) & (unsigned long long)(L - 1);
        const double c = cospi(2.0 * (double)ph / (double)L);
        const double v = kernel_col(kind, j, h, ell, deriv);
        acc += (L - j == j) ? v * c : 2.0 * v * c;
    }
    lam_br[e] = (T)(acc / (double)L);
}

// The same spectrum for a long circulant (four-step order, lg1 = LG1) from
// its forward four-step FFT, one workgroup: (1) length-L1 DIF over n1 of the
// embedded column c_emb[L2 n1 + n2] for every n2, times w_L^{n2 k1}; (2) per
// row p1, length-L2 DIF over n2, which leaves lambda[k1 + L1 k2] at
// (p1, p2) with k1 = bitrev(p1), k2 = bitrev(p2).  FP64 throughout, with
// twiddles from sincospi; Y: L complex FP64 scratch.
template <class T, int LG1, int LG2>
__global__ __launch_bounds__(1024) void spectrum_long_kernel(T* __restrict__ lam, int m,
                                                             double h, double ell, bool deriv,
                                                             int kind,
                                                             cplx<double>* __restrict__ Y) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2, L = L1 * L2;
    constexpr int R1 = line_regs<LG1>(), R2 = line_regs<LG2>();
    static_assert(L1 >= 64 && L2 >= 64, "one column or row per wave");
    __shared__ cplx<double> tw1[L1 / 2], tw2[L2 / 2];
    for (int t = threadIdx.x; t < L1 / 2; t += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)t / (double)L1, &sn, &cs);
        tw1[t] = {cs, -sn};
    }
    for (int t = threadIdx.x; t < L2 / 2; t += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)t / (double)L2, &sn, &cs);
        tw2[t] = {cs, -sn};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int n2 = wave; n2 < L2; n2 += nw) {
        cplx<double> z[R1];
#pragma unroll
        for (int q = 0; q < R1; ++q) {
            const int n = L2 * (q * 64 + lane) + n2;
            const int j = min(n, L - n);
            z[q] = {j < m ? kernel_col(kind, j, h, ell, deriv) : 0.0, 0.0};
        }
        dif_regs<double, LG1>(z, lane, tw1);
#pragma unroll
        for (int q = 0; q < R1; ++q) {
            const int p1 = q * 64 + lane;
            const unsigned long long t =
                ((unsigned long long)n2 * bitrev_bits((unsigned)p1, LG1)) & (unsigned long long)(L - 1);
            double sn, cs;
            sincospi(2.0 * (double)t / (double)L, &sn, &cs);
            Y[p1 * L2 + n2] = cmul(z[q], cplx<double>{cs, -sn});
        }
    }
    __syncthreads();
    for (int p1 = wave; p1 < L1; p1 += nw) {
        cplx<double> z[R2];
#pragma unroll
        for (int q = 0; q < R2; ++q) z[q] = Y[p1 * L2 + q * 64 + lane];
        dif_regs<double, LG2>(z, lane, tw2);
#pragma unroll
        for (int q = 0; q < R2; ++q) lam[p1 * L2 + q * 64 + lane] = (T)(z[q].re / (double)L);
    }
}

template <class T>
__global__ void twiddle_kernel(cplx<T>* __restrict__ tw, int log2L) {
    const int L = 1 << log2L;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L / 2) return;
    double sn, cs;
    sincospi(2.0 * (double)t / (double)L, &sn, &cs);
    tw[t] = {(T)cs, (T)(-sn)};
}

// ---------------------------------------------------------------------------
// Banded W^T W product in stencil-diagonal layout A[o][j], o in [-3,3]^d.
// ---------------------------------------------------------------------------
struct DiaGeom {
    int d;
    int64_t M;
    int64_t stride[3];   // flat stride of each dimension
    int ext[3];          // 7 for active dims, 1 otherwise
};

template <class TA, class T, int K>
__global__ __launch_bounds__(256) void spmv_dia_kernel(const TA* __restrict__ A,
                                                       const T* __restrict__ xpad,
                                                       T* __restrict__ u, DiaGeom dg,
                                                       int64_t halo, int64_t ldx,
                                                       const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= dg.M) return;
    T acc[K];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = T(0);
    const T* xj = xpad + halo + j;
    const int NB = dg.ext[0] * dg.ext[1] * dg.ext[2];
    int oi = 0;
    for (int a = 0; a < dg.ext[0]; ++a) {
        const int64_t oa = (dg.ext[0] == 7 ? (a - 3) : 0) * dg.stride[0];
        for (int b = 0; b < dg.ext[1]; ++b) {
            const int64_t ob = oa + (dg.ext[1] == 7 ? (b - 3) : 0) * dg.stride[1];
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                if (c >= dg.ext[2]) break;
                const int64_t off = ob + (dg.ext[2] == 7 ? (c - 3) : 0) * dg.stride[2];
                const T av = (T)A[dia_index(j, oi, NB)];
#pragma unroll
                for (int r = 0; r < K; ++r) acc[r] += av * xj[off + r * ldx];
                ++oi;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < K; ++r) u[r * dg.M + j] = acc[r];
}

// LDS-windowed banded product for one vector.  A block owns kTileRows
// consecutive rows [j0, j0 + kTileRows); the x entries its 7^d offsets touch
// lie in 7 windows (one per offset of the slowest dimension, 1 window in 1-D)
// of kTileRows + 2*margin entries, staged once in LDS with coalesced loads.
// Thread t handles row j0 + t, so every entry load of a wave is one
// contiguous 64-element segment of a diagonal.  Optionally writes the block's
// partial of sum_j u_j x_j (the CG inner product u^T r_hat) to dotp.
constexpr int kTileRows = kRowTile;   // one row per thread

struct TileGeom {
    int64_t M, halo;
    int64_t S0;       // stride of the slowest dimension (windows), d >= 2
    int64_t S1;       // stride of the middle dimension (d == 3)
    int margin;       // 3*S1 + 3 (d = 3), 3 (d <= 2)
    int WL;           // window length kTileRows + 2*margin
};

// Accumulates one row of the product.  The stored tile is zero-padded past
// the last grid node, so entry loads need no bounds; 49 independent loads
// (one 7 x 7 slab of offsets) are in flight per step.
template <class TA, class T, int D>
__device__ __forceinline__ T tile_row(const TA* __restrict__ Ab, const T* __restrict__ win,
                                      const TileGeom& tg, int t, uint32_t wb) {
    T acc = T(0);
    if (wb == 0u) return acc;   // every block of this wavefront is zero
    if constexpr (D == 1) {
        TA av[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) av[c] = Ab[c * kTileRows];
#pragma unroll
        for (int c = 0; c < 7; ++c) acc += (T)av[c] * win[tg.margin + t + (c - 3)];
    } else {
        constexpr int NA = D == 3 ? 7 : 1;
#pragma unroll 1
        for (int a = 0; a < NA; ++a) {
            if (!((wb >> a) & 1u)) continue;   // zero slab: skip its loads
            TA av[49];
            const TA* Aa = Ab + a * 49 * kTileRows;
#pragma unroll
            for (int q = 0; q < 49; ++q) av[q] = Aa[q * kTileRows];
#pragma unroll
            for (int q = 0; q < 49; ++q) {
                // D = 3: q = (o1, o2) within slab a = o0; D = 2: q = (o0, o1)
                const int p = q / 7, c = q % 7;
                const T* w = D == 3 ? win + a * tg.WL + tg.margin + t + (p - 3) * (int)tg.S1
                                    : win + p * tg.WL + tg.margin + t;
                acc += (T)av[q] * w[c - 3];
            }
        }
    }
    return acc;
}

template <class TA, class T, int D>
__global__ __launch_bounds__(256) void spmv_tiled_kernel(const TA* __restrict__ A,
                                                         const T* __restrict__ xpad,
                                                         T* __restrict__ u, TileGeom tg,
                                                         double* __restrict__ dotp,
                                                         const int* __restrict__ skip,
                                                         const uint32_t* __restrict__ bmask,
                                                         LastBlockRed lb) {
    if (skip && *skip) return;
    extern __shared__ unsigned char lds_raw[];
    T* win = reinterpret_cast<T*>(lds_raw);
    constexpr int NW = D >= 2 ? 7 : 1;
    constexpr int kNB = D == 1 ? 7 : (D == 2 ? 49 : 343);
    const unsigned tile = xcd_block();   // neighbouring tiles share window data
    const int64_t j0 = (int64_t)tile * kTileRows;
    const int64_t ldx = tg.M + 2 * tg.halo;
    const uint32_t mk = bmask ? bmask[tile] : ~0u;
    // stage the windows (not needed when the whole tile is zero): at each
    // position the NW windows' loads are issued together, unconditionally
    // (an index past the padded vector reads its last entry and stores 0;
    // indices are never negative, the halo covers the margin)
    if (mk != 0u) {
        const int64_t start0 = tg.halo + j0 - tg.margin;
        for (int i = threadIdx.x; i < tg.WL; i += 256) {
            T v[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int64_t idx = start0 + (D >= 2 ? (int64_t)(w - 3) * tg.S0 : 0) + i;
                v[w] = xpad[idx < ldx ? idx : ldx - 1];
            }
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int64_t idx = start0 + (D >= 2 ? (int64_t)(w - 3) * tg.S0 : 0) + i;
                win[w * tg.WL + i] = idx < ldx ? v[w] : T(0);
            }
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    // this wavefront's slab bits (uniform across the wavefront)
    const uint32_t wb = __builtin_amdgcn_readfirstlane((mk >> (kMaskSlabs * (t / kWaveRows))) &
                                                       ((1u << kMaskSlabs) - 1u));
    const T acc =
        tile_row<TA, T, D>(A + (int64_t)tile * kNB * kTileRows + t, win, tg, t, wb);
    double part = 0.0;
    const int xc = (D >= 2 ? 3 * tg.WL : 0) + tg.margin + t;
    if (j0 + t < tg.M) {
        u[j0 + t] = acc;
        if (wb) part = (double)acc * (double)win[xc];
    }
    if (dotp) {
        __shared__ double red[256];
        red[t] = part;
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (t < s2) red[t] += red[t + s2];
            __syncthreads();
        }
        if (lb.ticket) {
            last_block_finish(lb, red[0], red);   // publishes dotp[blockIdx.x] itself
        } else if (t == 0) {
            dotp[blockIdx.x] = red[0];
        }
    }
}

// LDS-windowed banded product for K vectors sharing one read of the stored
// entries.  The offsets are taken slab by slab (slab a = offset a - 3 of the
// slowest dimension: 49 entries per row for d = 3, 7 for d = 2, one slab of
// 7 for d = 1); for each slab the block stages the K windows that slab
// touches (kTileRows + 2*margin entries per vector) and every thread
// multiplies its row's slab entries, held in registers, into K accumulators.
// Entry loads of the next slab are issued before the barrier that precedes
// its staging.  Zero (wavefront, slab) blocks are skipped as in the
// one-vector kernel.
template <class TA, class T, int D, int K>
__global__ __launch_bounds__(256) void spmv_multi_kernel(const TA* __restrict__ A,
                                                         const T* __restrict__ xpad,
                                                         T* __restrict__ u, TileGeom tg,
                                                         int64_t ldx,
                                                         const int* __restrict__ skip,
                                                         const uint32_t* __restrict__ bmask) {
    if (skip && *skip) return;
    extern __shared__ unsigned char lds_raw[];
    T* win = reinterpret_cast<T*>(lds_raw);   // [K][WL]
    constexpr int NS = D == 1 ? 1 : 7;        // slabs
    constexpr int SW = D == 3 ? 49 : 7;       // entries per row and slab
    constexpr int kNB = NS * SW;
    const int t = threadIdx.x;
    const unsigned tile = xcd_block();
    const int64_t j0 = (int64_t)tile * kTileRows;
    const uint32_t mk = bmask ? bmask[tile] : ~0u;
    const uint32_t wb = __builtin_amdgcn_readfirstlane((mk >> (kMaskSlabs * (t / kWaveRows))) &
                                                       ((1u << kMaskSlabs) - 1u));
    constexpr uint32_t kWaveBits = 0x204081u;   // bit 0 of each wavefront's group
    const TA* Ab = A + (int64_t)tile * kNB * kTileRows + t;
    T acc[K];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = T(0);
#pragma unroll 1
    for (int a = 0; a < NS; ++a) {
        const int bit = D == 3 ? a : 0;
        const bool mine = (wb >> bit) & 1u;
        const bool staged = ((mk >> bit) & kWaveBits) != 0u;   // uniform over the block
        TA av[SW];
        if (mine) {
#pragma unroll
            for (int q = 0; q < SW; ++q) av[q] = Ab[(a * SW + q) * kTileRows];
        }
        if (staged) {
            // the K windows: all K loads of a position in flight together
            const int64_t start =
                tg.halo + j0 + (D >= 2 ? (int64_t)(a - 3) * tg.S0 : 0) - tg.margin;
            for (int i = t; i < tg.WL; i += 256) {
                const int64_t idx = start + i;
                T v[K];
#pragma unroll
                for (int r = 0; r < K; ++r) v[r] = idx < ldx ? xpad[r * ldx + idx] : T(0);
#pragma unroll
                for (int r = 0; r < K; ++r) win[r * tg.WL + i] = v[r];
            }
        }
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int q = 0; q < SW; ++q) {
                const int p = D == 3 ? q / 7 : 0, c = D == 3 ? q % 7 : q;
                const int off = tg.margin + t + (D == 3 ? (p - 3) * (int)tg.S1 : 0) + (c - 3);
                const T e = (T)av[q];
#pragma unroll
                for (int r = 0; r < K; ++r) acc[r] += e * win[r * tg.WL + off];
            }
        }
        __syncthreads();
    }
    if (j0 + t < tg.M) {
#pragma unroll
        for (int r = 0; r < K; ++r) u[(int64_t)r * tg.M + j0 + t] = acc[r];
    }
}

// ---------------------------------------------------------------------------
// Interpolation mu(x) = sum_a w_a(x) mu_G[node_a] (FP64).
// ---------------------------------------------------------------------------
template <class Tin>
__global__ void interp_kernel(GridDev g, const double* __restrict__ mu, const Tin* x0,
                              const Tin* x1, const Tin* x2, int64_t nq,
                              double* __restrict__ out, unsigned long long* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const Tin* xs[3] = {x0, x1, x2};
    int base[3] = {1, 1, 1};
    double w[3][4] = {{0, 1, 0, 0}, {0, 1, 0, 0}, {0, 1, 0, 0}};
    bool ok = true;
    for (int k = 0; k < g.d; ++k) {
        const double u = ((double)xs[k][i] - g.g0[k]) / g.h[k];
        if (!(u >= 1.0 && u <= (double)(g.m[k] - 2))) {
            ok = false;
            break;
        }
        int b = (int)floor(u);
        if (b > g.m[k] - 3) b = g.m[k] - 3;
        base[k] = b;
        stencil_weights(g.interp, u - (double)b, w[k]);
    }
    if (!ok) {
        atomicMin(bad, (unsigned long long)i);
        out[i] = 0.0;
        return;
    }
    const int e1 = g.d > 1 ? 4 : 1, e2 = g.d > 2 ? 4 : 1;
    double acc = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < e1; ++b)
            for (int c = 0; c < e2; ++c) {
                int64_t j = base[0] - 1 + a;
                double wt = w[0][a];
                if (g.d > 1) {
                    j = j * g.m[1] + (base[1] - 1 + b);
                    wt *= w[1][b];
                }
                if (g.d > 2) {
                    j = j * g.m[2] + (base[2] - 1 + c);
                    wt *= w[2][c];
                }
                acc = fma(wt, mu[j], acc);
            }
    out[i] = acc;
}

// Interpolation weights of query point i as a grid vector: G[i][node] =
// w_i(node) for its 4^d stencil nodes (G zeroed by the caller).
template <class Tin>
__global__ void weights_kernel(GridDev g, const Tin* x0, const Tin* x1, const Tin* x2,
                               int64_t nq, int64_t M, double* __restrict__ G,
                               unsigned long long* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const Tin* xs[3] = {x0, x1, x2};
    int base[3] = {1, 1, 1};
    double w[3][4] = {{0, 1, 0, 0}, {0, 1, 0, 0}, {0, 1, 0, 0}};
    for (int k = 0; k < g.d; ++k) {
        const double u = ((double)xs[k][i] - g.g0[k]) / g.h[k];
        if (!(u >= 1.0 && u <= (double)(g.m[k] - 2))) {
            atomicMin(bad, (unsigned long long)i);
            return;
        }
        int b = (int)floor(u);
        if (b > g.m[k] - 3) b = g.m[k] - 3;
        base[k] = b;
        stencil_weights(g.interp, u - (double)b, w[k]);
    }
    const int e1 = g.d > 1 ? 4 : 1, e2 = g.d > 2 ? 4 : 1;
    double* Gi = G + i * M;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < e1; ++b)
            for (int c = 0; c < e2; ++c) {
                int64_t j = base[0] - 1 + a;
                double wt = w[0][a];
                if (g.d > 1) {
                    j = j * g.m[1] + (base[1] - 1 + b);
                    wt *= w[1][b];
                }
                if (g.d > 2) {
                    j = j * g.m[2] + (base[2] - 1 + c);
                    wt *= w[2][c];
                }
                Gi[j] = wt;
            }
}

// Stencil of query point i: first node per dimension and the four Keys
// weights per dimension (first[i][k], w[i][k][a]).
template <class Tin>
__global__ void stencil_kernel(GridDev g, const Tin* x0, const Tin* x1, const Tin* x2,
                               int64_t nq, int* __restrict__ first, double* __restrict__ w,
                               unsigned long long* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const Tin* xs[3] = {x0, x1, x2};
    for (int k = 0; k < 3; ++k) {
        double wk[4] = {1.0, 0.0, 0.0, 0.0};
        int f = 0;
        if (k < g.d) {
            const double u = ((double)xs[k][i] - g.g0[k]) / g.h[k];
            if (!(u >= 1.0 && u <= (double)(g.m[k] - 2))) {
                atomicMin(bad, (unsigned long long)i);
                return;
            }
            int b = (int)floor(u);
            if (b > g.m[k] - 3) b = g.m[k] - 3;
            stencil_weights(g.interp, u - (double)b, wk);
            f = b - 1;
        }
        first[i * 3 + k] = f;
        for (int a = 0; a < 4; ++a) w[(i * 3 + k) * 4 + a] = wk[a];
    }
}

// U[i][l] = sum over the stencil nodes j of query i of w_ij Ct[j][l]
// (one workgroup per query point, threads over l).
__global__ void love_project_kernel(GridDev g, const double* __restrict__ Ct, int k,
                                    const int* __restrict__ first,
                                    const double* __restrict__ w, double* __restrict__ U) {
    const int64_t i = blockIdx.x;
    const int e1 = g.d > 1 ? 4 : 1, e2 = g.d > 2 ? 4 : 1;
    const int f0 = first[i * 3], f1 = first[i * 3 + 1], f2 = first[i * 3 + 2];
    const double* wi = w + i * 12;
    for (int l = threadIdx.x; l < k; l += blockDim.x) {
        double acc = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < e1; ++b)
                for (int c = 0; c < e2; ++c) {
                    int64_t j = f0 + a;
                    if (g.d > 1) j = j * g.m[1] + (f1 + b);
                    if (g.d > 2) j = j * g.m[2] + (f2 + c);
                    const double wt = wi[a] * wi[4 + b] * wi[8 + c];
                    acc = fma(wt, Ct[j * k + l], acc);
                }
        U[i * k + l] = acc;
    }
}

constexpr int kGramTile = 64;
constexpr int kGramChunk = 16;
constexpr int kGramPairs = kGramTile * kGramTile / 256;

// For the tile (rows i0.., columns j0..) of the pair matrix: partial sums of
// U_i . U_j over the column chunks of this block (chunk c to block c mod
// gridDim.x, increasing order).
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ U, int k,
                                                           int nq,
                                                           double* __restrict__ partials) {
    __shared__ double sA[kGramTile][kGramChunk + 1];
    __shared__ double sB[kGramTile][kGramChunk + 1];
    const int i0 = blockIdx.y * kGramTile, j0 = blockIdx.z * kGramTile;
    const int ni = min(kGramTile, nq - i0), nj = min(kGramTile, nq - j0);
    double acc[kGramPairs];
#pragma unroll
    for (int r = 0; r < kGramPairs; ++r) acc[r] = 0.0;
    const int nchunk = (k + kGramChunk - 1) / kGramChunk;
    for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int l0 = ch * kGramChunk;
        __syncthreads();
        for (int e = threadIdx.x; e < kGramTile * kGramChunk; e += 256) {
            const int a = e / kGramChunk, ll = e % kGramChunk;
            const int l = l0 + ll;
            sA[a][ll] = (l < k && a < ni) ? U[(int64_t)(i0 + a) * k + l] : 0.0;
            sB[a][ll] = (l < k && a < nj) ? U[(int64_t)(j0 + a) * k + l] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kGramPairs; ++r) {
            const int p = threadIdx.x + 256 * r;
            const int a = p / kGramTile, b = p % kGramTile;
            double t = 0.0;
#pragma unroll 8
            for (int ll = 0; ll < kGramChunk; ++ll) t = fma(sA[a][ll], sB[b][ll], t);
            acc[r] += t;
        }
    }
    const int tile = blockIdx.y * gridDim.z + blockIdx.z;
    double* out = partials + ((int64_t)tile * gridDim.x + blockIdx.x) * (kGramTile * kGramTile);
#pragma unroll
    for (int r = 0; r < kGramPairs; ++r) out[threadIdx.x + 256 * r] = acc[r];
}

// cov[i][j] = w_i^T K_G w_j - (U_i . U_j + U_j . U_i) / 2.  The prior term
// is separable: K_G and the stencil weights are products over dimensions,
// so w_i^T K_G w_j = so prod_k sum_{a,b} w_ik[a] w_jk[b] k1(|node distance|).
__global__ void love_fin_kernel(GridDev g, int kind, double ell0, double ell1, double ell2,
                                double so, const int* __restrict__ first,
                                const double* __restrict__ w,
                                const double* __restrict__ partials, int nb, int nq, int nt,
                                double* __restrict__ cov) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)nq * nq) return;
    const int i = (int)(p / nq), j = (int)(p % nq);
    const double ell[3] = {ell0, ell1, ell2};
    // evaluated in the order of (min, max) so that cov is exactly symmetric
    const int lo = min(i, j), hi = max(i, j);
    double prior = so;
    for (int k = 0; k < g.d; ++k) {
        const int fi = first[lo * 3 + k], fj = first[hi * 3 + k];
        const double* wi = w + ((int64_t)lo * 3 + k) * 4;
        const double* wj = w + ((int64_t)hi * 3 + k) * 4;
        double t = 0.0;
        for (int a = 0; a < 4; ++a) {
            double ta = 0.0;
            for (int b = 0; b < 4; ++b) {
                const int dist = abs((fi + a) - (fj + b));
                ta = fma(wj[b], kernel_col(kind, dist, g.h[k], ell[k], false), ta);
            }
            t = fma(wi[a], ta, t);
        }
        prior *= t;
    }
    auto sum = [&](int r, int c) {
        const int tile = (r / kGramTile) * nt + c / kGramTile;
        const double* q = partials + (int64_t)tile * nb * (kGramTile * kGramTile) +
                          (r % kGramTile) * kGramTile + c % kGramTile;
        double a = 0.0;
        for (int b = 0; b < nb; ++b) a += q[(int64_t)b * (kGramTile * kGramTile)];
        return a;
    };
    cov[p] = prior - 0.5 * (sum(i, j) + sum(j, i));
}

template <class T>
__global__ void dia_to_canonical_kernel(const T* __restrict__ A, T* __restrict__ out,
                                        int64_t M, int NB) {
    __shared__ T tile[32][33];
    const int64_t j0 = (int64_t)blockIdx.x * 32;
    const int o0 = blockIdx.y * 32;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int o = o0 + r;
        const int64_t j = j0 + threadIdx.x;
        tile[r][threadIdx.x] = (o < NB && j < M) ? A[dia_index(j, o, NB)] : T(0);
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int64_t j = j0 + r;
        const int o = o0 + threadIdx.x;
        if (j < M && o < NB) out[j * NB + o] = tile[threadIdx.x][r];
    }
}

}  // namespace

int circulant_log2(int m) {
    int l = 3;
    while ((1 << l) < 2 * m - 1) ++l;
    return l;
}

template <class T>
static fkgp_status launch_spectrum_long(T* lam, int log2L, int m, double h, double ell,
                                        bool deriv, int kind, cplx<double>* Y, hipStream_t s) {
    switch (log2L) {
        case 12:
            spectrum_long_kernel<T, 6, 6><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        case 13:
            spectrum_long_kernel<T, 6, 7><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        case 14:
            spectrum_long_kernel<T, 7, 7><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        case 15:
            spectrum_long_kernel<T, 7, 8><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        case 16:
            spectrum_long_kernel<T, 8, 8><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        case 17:
            spectrum_long_kernel<T, 8, 9><<<1, 1024, 0, s>>>(lam, m, h, ell, deriv, kind, Y);
            break;
        default:
            set_error("no long-circulant spectrum for this length");
            return FKGP_EINVAL;
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status build_spectrum(const GridDev& g, int k, double ell, bool deriv, int kind,
                           fkgp_dtype dt, void* lam, int log2L, int lg1, void* scr,
                           hipStream_t s) {
    const int L = 1 << log2L;
    // four-step layouts of 2^12 points and more take the FFT whenever its
    // scratch is there (O(L log L) instead of O(L m) direct sums); beyond
    // 2^kMaxDftLog2 points they must
    if (log2L > kMaxDftLog2 || (scr && lg1 > 0 && log2L >= 12)) {
        int want1, want2;
        long_split(log2L, want1, want2);
        if (!scr || lg1 != want1) {
            set_error("long circulant spectrum needs the four-step order and its scratch");
            return FKGP_EINVAL;
        }
        cplx<double>* Y = static_cast<cplx<double>*>(scr);
        if (dt == FKGP_F32)
            return launch_spectrum_long<float>(static_cast<float*>(lam), log2L, g.m[k], g.h[k],
                                               ell, deriv, kind, Y, s);
        return launch_spectrum_long<double>(static_cast<double*>(lam), log2L, g.m[k], g.h[k],
                                            ell, deriv, kind, Y, s);
    }
    const unsigned grid = (unsigned)((L + 255) / 256);
    if (dt == FKGP_F32)
        spectrum_kernel<float><<<grid, 256, 0, s>>>(static_cast<float*>(lam), log2L, lg1,
                                                    g.m[k], g.h[k], ell, deriv, kind);
    else
        spectrum_kernel<double><<<grid, 256, 0, s>>>(static_cast<double*>(lam), log2L, lg1,
                                                     g.m[k], g.h[k], ell, deriv, kind);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status build_twiddles(int log2L, fkgp_dtype dt, void* tw, hipStream_t s) {
    const int L = 1 << log2L;
    const unsigned grid = (unsigned)((L / 2 + 255) / 256);
    if (dt == FKGP_F32)
        twiddle_kernel<float><<<grid, 256, 0, s>>>(static_cast<cplx<float>*>(tw), log2L);
    else
        twiddle_kernel<double><<<grid, 256, 0, s>>>(static_cast<cplx<double>*>(tw), log2L);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

bool toeplitz_slab_applies(const GridDev& g) {
    return g.d == 3 && g.m[0] <= 16 * kSlabR && g.m[1] <= kSlabMaxM1 && g.m[2] <= kSlabMaxM2 &&
           g.m[1] * g.m[2] <= kSlabMaxNodes;
}

static size_t slab_lds_bytes(int m1, int m2, size_t es) {
    const int mp1 = slab_pad(m1), mp2 = slab_pad(m2);
    return es * ((size_t)2 * mp1 * (mp2 + 1) + 2 * mp1 + 2 * mp2 + 4 * kSlabR);
}

int64_t toeplitz_cols_blocks(const GridDev& g, int k) {
    const int64_t S = (int64_t)g.m[1] * g.m[2];
    return (int64_t)k * ((S + kColsC - 1) / kColsC);
}

// the outermost dimension after the slab pass (in place: each workgroup
// reads and writes only its own columns)
template <class T>
static fkgp_status launch_toeplitz_cols(const GridDev& g, const T* x, T* y, int k,
                                        const T* col, T scale, const T* addv, T add_coef,
                                        const int* skip, const CgStep2* fuse, hipStream_t s) {
    CgStep2 fz{};
    if (fuse) fz = *fuse;
    const int64_t S = (int64_t)g.m[1] * g.m[2];
    const int64_t tpv = (S + kColsC - 1) / kColsC;
    const int64_t grid = (int64_t)k * tpv;
    if (grid <= 0) return FKGP_OK;
    toeplitz_cols<T><<<(unsigned)grid, 256, 0, s>>>(x, y, g.m[0], S, tpv, col, scale, addv,
                                                    add_coef, skip, fz);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// y[o] = T_1 x[o] T_2 for the nslab = k * m_0 slabs of k vectors
template <class T>
static fkgp_status launch_toeplitz_slab(const GridDev& g, const T* x, T* y, int64_t nslab,
                                        const T* col1, const T* col2, const int* skip,
                                        hipStream_t s) {
    const int m1 = g.m[1], m2 = g.m[2];
    const int prow = x == y ? slab_pad(m1) : slab_part_rows(m2);
    const int parts = (m1 + prow - 1) / prow;
    const size_t lds = slab_lds_bytes(m1, m2, sizeof(T));
    const int64_t grid = nslab * parts;
    if (grid <= 0) return FKGP_OK;
    if (lds > 64 * 1024)
        FKGP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&toeplitz_slab<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    toeplitz_slab<T><<<(unsigned)grid, 256, lds, s>>>(x, y, m1, m2, parts, prow, col1, col2,
                                                      skip);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

template <class T>
__global__ void toeplitz_col_kernel(T* __restrict__ col, int m, double h, double ell, bool deriv,
                                    int kind) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) col[j] = (T)kernel_col(kind, j, h, ell, deriv);
}

fkgp_status build_toeplitz_col(const GridDev& g, int k, double ell, bool deriv, int kind,
                               fkgp_dtype dt, void* col, hipStream_t s) {
    const unsigned grid = (unsigned)((g.m[k] + 255) / 256);
    if (dt == FKGP_F32)
        toeplitz_col_kernel<float><<<grid, 256, 0, s>>>(static_cast<float*>(col), g.m[k], g.h[k],
                                                        ell, deriv, kind);
    else
        toeplitz_col_kernel<double><<<grid, 256, 0, s>>>(static_cast<double*>(col), g.m[k],
                                                         g.h[k], ell, deriv, kind);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

template <class T>
static fkgp_status kg_apply_t(const GridDev& g, const Spectra& sp, const T* x, T* y, int k,
                              double scale, const T* addv, double add_coef, const int* skip,
                              hipStream_t s) {
    int64_t M = 1;
    for (int i = 0; i < g.d; ++i) M *= g.m[i];
    // innermost dimension first (contiguous lines), then the strided ones;
    // for 3-D grids with small inner slabs the two innermost dimensions in
    // one dense Toeplitz pass
    if (sp.col[0] && sp.col[1] && sp.col[2]) {
        fkgp_status st = launch_toeplitz_slab<T>(g, x, y, (int64_t)k * g.m[0],
                                                 static_cast<const T*>(sp.col[1]),
                                                 static_cast<const T*>(sp.col[2]), skip, s);
        if (st != FKGP_OK) return st;
        return launch_toeplitz_cols<T>(g, y, y, k, static_cast<const T*>(sp.col[0]), (T)scale,
                                       addv, (T)add_coef, skip, nullptr, s);
    }
    for (int pass = 0; pass < g.d; ++pass) {
        const int dim = g.d - 1 - pass;
        int64_t S = 1;
        for (int i = dim + 1; i < g.d; ++i) S *= g.m[i];
        LineGeom lg{g.m[dim], S, (int64_t)k * M / g.m[dim]};
        const bool last = pass == g.d - 1;
        const T* src = pass == 0 ? x : y;
        fkgp_status st = launch_line_conv<T>(
            sp.log2L[dim], sp.lg1[dim], src, y, lg, static_cast<const T*>(sp.lam[dim]),
            static_cast<const cplx<T>*>(sp.tw[dim]), last ? (T)scale : T(1),
            last ? addv : nullptr, (T)add_coef, skip, static_cast<cplx<T>*>(sp.scr[dim]), s);
        if (st != FKGP_OK) return st;
    }
    return FKGP_OK;
}

template <class T>
static fkgp_status kg_apply_fused_t(const GridDev& g, const Spectra& sp, const T* x, T* y,
                                    double scale, const T* addv, double add_coef,
                                    const int* skip, const CgStep2& fuse, bool* fused,
                                    hipStream_t s) {
    int64_t M = 1;
    for (int i = 0; i < g.d; ++i) M *= g.m[i];
    if (sp.col[0] && sp.col[1] && sp.col[2]) {
        *fused = true;
        fkgp_status st = launch_toeplitz_slab<T>(g, x, y, g.m[0], static_cast<const T*>(sp.col[1]),
                                                 static_cast<const T*>(sp.col[2]), skip, s);
        if (st != FKGP_OK) return st;
        return launch_toeplitz_cols<T>(g, y, y, 1, static_cast<const T*>(sp.col[0]), (T)scale,
                                       addv, (T)add_coef, skip, &fuse, s);
    }
    *fused = sp.lg1[0] == 0;   // the last pass (dimension 0) on the register path
    for (int pass = 0; pass < g.d; ++pass) {
        const int dim = g.d - 1 - pass;
        int64_t S = 1;
        for (int i = dim + 1; i < g.d; ++i) S *= g.m[i];
        LineGeom lg{g.m[dim], S, M / g.m[dim]};
        const bool last = pass == g.d - 1;
        const T* src = pass == 0 ? x : y;
        fkgp_status st = launch_line_conv<T>(
            sp.log2L[dim], sp.lg1[dim], src, y, lg, static_cast<const T*>(sp.lam[dim]),
            static_cast<const cplx<T>*>(sp.tw[dim]), last ? (T)scale : T(1),
            last ? addv : nullptr, (T)add_coef, skip, static_cast<cplx<T>*>(sp.scr[dim]), s,
            (last && *fused) ? &fuse : nullptr);
        if (st != FKGP_OK) return st;
    }
    return FKGP_OK;
}

fkgp_status kg_apply_fused(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x,
                           void* y, double scale, const void* addv, double add_coef,
                           const int* skip, const CgStep2& fuse, bool* fused, hipStream_t s) {
    if (dt == FKGP_F32)
        return kg_apply_fused_t<float>(g, sp, static_cast<const float*>(x),
                                       static_cast<float*>(y), scale,
                                       static_cast<const float*>(addv), add_coef, skip, fuse,
                                       fused, s);
    return kg_apply_fused_t<double>(g, sp, static_cast<const double*>(x),
                                    static_cast<double*>(y), scale,
                                    static_cast<const double*>(addv), add_coef, skip, fuse,
                                    fused, s);
}

int64_t kg_last_pass_blocks(const GridDev& g) {
    int64_t M = 1;
    for (int i = 0; i < g.d; ++i) M *= g.m[i];
    LineGeom lg{g.m[0], M / g.m[0], M / g.m[0]};
    return std::max<int64_t>(line_direct_blocks(circulant_log2(g.m[0]), lg),
                             toeplitz_cols_blocks(g, 1));
}

fkgp_status kg_apply(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x, void* y,
                     int k, double scale, const void* addv, double add_coef, void* /*work*/,
                     hipStream_t s) {
    if (dt == FKGP_F32)
        return kg_apply_t<float>(g, sp, static_cast<const float*>(x), static_cast<float*>(y), k,
                                 scale, static_cast<const float*>(addv), add_coef, nullptr, s);
    return kg_apply_t<double>(g, sp, static_cast<const double*>(x), static_cast<double*>(y), k,
                              scale, static_cast<const double*>(addv), add_coef, nullptr, s);
}

fkgp_status kg_apply_skip(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x,
                          void* y, int k, double scale, const void* addv, double add_coef,
                          const int* skip, hipStream_t s) {
    if (dt == FKGP_F32)
        return kg_apply_t<float>(g, sp, static_cast<const float*>(x), static_cast<float*>(y), k,
                                 scale, static_cast<const float*>(addv), add_coef, skip, s);
    return kg_apply_t<double>(g, sp, static_cast<const double*>(x), static_cast<double*>(y), k,
                              scale, static_cast<const double*>(addv), add_coef, skip, s);
}

int64_t dia_halo(const GridDev& g) {
    int64_t h = 0, st = 1;
    for (int i = g.d - 1; i >= 0; --i) {
        h += 3 * st;
        st *= g.m[i];
    }
    return h;
}

int64_t spmv_dot_parts(const GridDev& g) {
    int64_t M = 1;
    for (int i = 0; i < g.d; ++i) M *= g.m[i];
    return (M + kTileRows - 1) / kTileRows;
}

// Geometry of the windowed kernel; false if its LDS would exceed 96 KiB.
static bool tile_geom(const GridDev& g, size_t es, TileGeom& tg, size_t& lds) {
    tg.M = 1;
    for (int i = 0; i < g.d; ++i) tg.M *= g.m[i];
    tg.halo = dia_halo(g);
    tg.S0 = g.d >= 2 ? tg.M / g.m[0] : 0;
    tg.S1 = g.d == 3 ? g.m[2] : 0;
    tg.margin = g.d == 3 ? (int)(3 * tg.S1 + 3) : 3;
    tg.WL = kTileRows + 2 * tg.margin;
    lds = (size_t)(g.d >= 2 ? 7 : 1) * tg.WL * es;
    return lds <= 96 * 1024;
}

constexpr size_t kMultiLdsMax = 64 * 1024;

template <class TA, class T, int D, int K>
static fkgp_status launch_multi_k(unsigned grid, size_t lds, const TA* A, const T* x, T* u,
                                  const TileGeom& tg, int64_t ldx, const int* skip,
                                  const uint32_t* bmask, hipStream_t s) {
    spmv_multi_kernel<TA, T, D, K><<<grid, 256, lds, s>>>(A, x, u, tg, ldx, skip, bmask);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

template <class TA, class T, int D>
static fkgp_status launch_multi_d(int K, unsigned grid, size_t lds, const TA* A, const T* x,
                                  T* u, const TileGeom& tg, int64_t ldx, const int* skip,
                                  const uint32_t* bmask, hipStream_t s) {
    switch (K) {
        case 16: return launch_multi_k<TA, T, D, 16>(grid, lds, A, x, u, tg, ldx, skip, bmask, s);
        case 8: return launch_multi_k<TA, T, D, 8>(grid, lds, A, x, u, tg, ldx, skip, bmask, s);
        case 4: return launch_multi_k<TA, T, D, 4>(grid, lds, A, x, u, tg, ldx, skip, bmask, s);
        case 2: return launch_multi_k<TA, T, D, 2>(grid, lds, A, x, u, tg, ldx, skip, bmask, s);
        default: return launch_multi_k<TA, T, D, 1>(grid, lds, A, x, u, tg, ldx, skip, bmask, s);
    }
}

template <class TA, class T>
static fkgp_status launch_multi(int d, int K, unsigned grid, size_t lds, const TA* A, const T* x,
                                T* u, const TileGeom& tg, int64_t ldx, const int* skip,
                                const uint32_t* bmask, hipStream_t s) {
    if (d == 1) return launch_multi_d<TA, T, 1>(K, grid, lds, A, x, u, tg, ldx, skip, bmask, s);
    if (d == 2) return launch_multi_d<TA, T, 2>(K, grid, lds, A, x, u, tg, ldx, skip, bmask, s);
    return launch_multi_d<TA, T, 3>(K, grid, lds, A, x, u, tg, ldx, skip, bmask, s);
}

template <class TA, class T>
static fkgp_status spmv_t(const GridDev& g, const TA* A, const uint32_t* bmask, const T* xpad,
                          T* u, int k, int64_t halo, const int* skip, hipStream_t s,
                          double* dotp = nullptr, int* nparts = nullptr,
                          const LastBlockRed* lb = nullptr) {
    TileGeom tg;
    size_t lds;
    if (k == 1 && tile_geom(g, sizeof(T), tg, lds)) {
        LastBlockRed lbv{};
        if (lb && dotp) lbv = *lb;
        const unsigned grid = (unsigned)((tg.M + kTileRows - 1) / kTileRows);
        if (g.d == 1) {
            if (lds > 64 * 1024)
                FKGP_HIP(hipFuncSetAttribute(
                    reinterpret_cast<const void*>(&spmv_tiled_kernel<TA, T, 1>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            spmv_tiled_kernel<TA, T, 1><<<grid, 256, lds, s>>>(A, xpad, u, tg, dotp, skip, bmask,
                                                                   lbv);
        } else if (g.d == 2) {
            if (lds > 64 * 1024)
                FKGP_HIP(hipFuncSetAttribute(
                    reinterpret_cast<const void*>(&spmv_tiled_kernel<TA, T, 2>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            spmv_tiled_kernel<TA, T, 2><<<grid, 256, lds, s>>>(A, xpad, u, tg, dotp, skip, bmask,
                                                                   lbv);
        } else {
            if (lds > 64 * 1024)
                FKGP_HIP(hipFuncSetAttribute(
                    reinterpret_cast<const void*>(&spmv_tiled_kernel<TA, T, 3>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            spmv_tiled_kernel<TA, T, 3><<<grid, 256, lds, s>>>(A, xpad, u, tg, dotp, skip, bmask,
                                                                   lbv);
        }
        if (nparts) *nparts = dotp ? (int)grid : 0;
        FKGP_HIP(hipGetLastError());
        return FKGP_OK;
    }
    if (nparts) *nparts = 0;
    if (k > 1 && tile_geom(g, sizeof(T), tg, lds)) {
        const int64_t ldxm = tg.M + 2 * tg.halo;
        const unsigned grid = (unsigned)((tg.M + kTileRows - 1) / kTileRows);
        const size_t wl_bytes = (size_t)tg.WL * sizeof(T);
        for (int r0 = 0; r0 < k;) {
            const int left = k - r0;
            int K = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            while (K > 1 && K * wl_bytes > kMultiLdsMax) K /= 2;
            const T* xr = xpad + (int64_t)r0 * ldxm;
            T* ur = u + (int64_t)r0 * tg.M;
            const fkgp_status st = launch_multi<TA, T>(g.d, K, grid, K * wl_bytes, A, xr, ur, tg,
                                                       ldxm, skip, bmask, s);
            if (st != FKGP_OK) return st;
            r0 += K;
        }
        FKGP_HIP(hipGetLastError());
        return FKGP_OK;
    }
    DiaGeom dg{};
    dg.d = g.d;
    dg.M = 1;
    for (int i = 0; i < g.d; ++i) dg.M *= g.m[i];
    // map grid dims onto the three loop levels (innermost = last grid dim)
    int64_t st = 1;
    for (int lvl = 2; lvl >= 0; --lvl) {
        const int dim = g.d - 3 + lvl;
        if (dim >= 0) {
            dg.stride[lvl] = st;
            dg.ext[lvl] = 7;
            st *= g.m[dim];
        } else {
            dg.stride[lvl] = 0;
            dg.ext[lvl] = 1;
        }
    }
    const int64_t ldx = dg.M + 2 * halo;
    const unsigned grid = (unsigned)((dg.M + 255) / 256);
    for (int r0 = 0; r0 < k;) {
        const int left = k - r0;
        const T* xr = xpad + (int64_t)r0 * ldx;
        T* ur = u + (int64_t)r0 * dg.M;
        if (left >= 8) {
            spmv_dia_kernel<TA, T, 8><<<grid, 256, 0, s>>>(A, xr, ur, dg, halo, ldx, skip);
            r0 += 8;
        } else if (left >= 4) {
            spmv_dia_kernel<TA, T, 4><<<grid, 256, 0, s>>>(A, xr, ur, dg, halo, ldx, skip);
            r0 += 4;
        } else if (left >= 2) {
            spmv_dia_kernel<TA, T, 2><<<grid, 256, 0, s>>>(A, xr, ur, dg, halo, ldx, skip);
            r0 += 2;
        } else {
            spmv_dia_kernel<TA, T, 1><<<grid, 256, 0, s>>>(A, xr, ur, dg, halo, ldx, skip);
            r0 += 1;
        }
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status spmv_dia(const GridDev& g, fkgp_dtype dt, const void* A, const void* xpad, void* u,
                     int k, int64_t halo, hipStream_t s) {
    return spmv_dia_skip(g, dt, A, xpad, u, k, halo, nullptr, s);
}

fkgp_status spmv_dia_skip(const GridDev& g, fkgp_dtype dt, const void* A, const void* xpad,
                          void* u, int k, int64_t halo, const int* skip, hipStream_t s) {
    if (dt == FKGP_F32)
        return spmv_t<float, float>(g, static_cast<const float*>(A), nullptr,
                                    static_cast<const float*>(xpad), static_cast<float*>(u), k,
                                    halo, skip, s);
    return spmv_t<double, double>(g, static_cast<const double*>(A), nullptr,
                                  static_cast<const double*>(xpad), static_cast<double*>(u), k,
                                  halo, skip, s);
}

// Product with matrix dtype dta and vector dtype dtx (FP32 matrix entries are
// upcast exactly when the vectors are FP64).
fkgp_status spmv_dia_any(const GridDev& g, fkgp_dtype dta, fkgp_dtype dtx, const void* A,
                         const uint32_t* bmask, const void* xpad, void* u, int k,
                         int64_t halo, const int* skip, hipStream_t s, double* dotp,
                         int* nparts, const LastBlockRed* lb) {
    if (dta == FKGP_F32 && dtx == FKGP_F32)
        return spmv_t<float, float>(g, static_cast<const float*>(A), bmask,
                                    static_cast<const float*>(xpad), static_cast<float*>(u), k,
                                    halo, skip, s, dotp, nparts, lb);
    if (dta == FKGP_F64 && dtx == FKGP_F64)
        return spmv_t<double, double>(g, static_cast<const double*>(A), bmask,
                                      static_cast<const double*>(xpad), static_cast<double*>(u), k,
                                      halo, skip, s, dotp, nparts, lb);
    if (dta == FKGP_F32 && dtx == FKGP_F64)
        return spmv_t<float, double>(g, static_cast<const float*>(A), bmask,
                                     static_cast<const double*>(xpad), static_cast<double*>(u), k,
                                     halo, skip, s, dotp, nparts, lb);
    set_error("unsupported matrix/vector dtype combination");
    return FKGP_EINVAL;
}

// FP64 product with an FP32-stored matrix (entries upcast exactly).
fkgp_status spmv_dia_f32a_f64x(const GridDev& g, const void* A, const double* xpad, double* u,
                               int k, int64_t halo, hipStream_t s) {
    return spmv_t<float, double>(g, static_cast<const float*>(A), nullptr, xpad, u, k, halo,
                                 nullptr, s);
}

fkgp_status interpolate_points(const GridDev& g, const double* mu, const void* const* xq,
                               int64_t nq, fkgp_dtype in, double* out, unsigned long long* bad,
                               hipStream_t s) {
    if (nq == 0) return FKGP_OK;
    const unsigned grid = (unsigned)((nq + 255) / 256);
    if (in == FKGP_F32) {
        const float* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const float*>(xq[k]);
        interp_kernel<float><<<grid, 256, 0, s>>>(g, mu, p[0], p[1], p[2], nq, out, bad);
    } else {
        const double* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const double*>(xq[k]);
        interp_kernel<double><<<grid, 256, 0, s>>>(g, mu, p[0], p[1], p[2], nq, out, bad);
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status query_weights(const GridDev& g, const void* const* xq, int64_t nq, fkgp_dtype in,
                          double* G, unsigned long long* bad, hipStream_t s) {
    if (nq == 0) return FKGP_OK;
    int64_t M = 1;
    for (int i = 0; i < g.d; ++i) M *= g.m[i];
    const unsigned grid = (unsigned)((nq + 255) / 256);
    if (in == FKGP_F32) {
        const float* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const float*>(xq[k]);
        weights_kernel<float><<<grid, 256, 0, s>>>(g, p[0], p[1], p[2], nq, M, G, bad);
    } else {
        const double* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const double*>(xq[k]);
        weights_kernel<double><<<grid, 256, 0, s>>>(g, p[0], p[1], p[2], nq, M, G, bad);
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status query_stencils(const GridDev& g, const void* const* xq, int64_t nq, fkgp_dtype in,
                           int* first, double* w, unsigned long long* bad, hipStream_t s) {
    if (nq == 0) return FKGP_OK;
    const unsigned grid = (unsigned)((nq + 255) / 256);
    if (in == FKGP_F32) {
        const float* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const float*>(xq[k]);
        stencil_kernel<float><<<grid, 256, 0, s>>>(g, p[0], p[1], p[2], nq, first, w, bad);
    } else {
        const double* p[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < g.d; ++k) p[k] = static_cast<const double*>(xq[k]);
        stencil_kernel<double><<<grid, 256, 0, s>>>(g, p[0], p[1], p[2], nq, first, w, bad);
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

size_t love_partials_doubles(int nq, int k, int* nb_out) {
    const int nt = (nq + kGramTile - 1) / kGramTile;
    const int nchunk = (k + kGramChunk - 1) / kGramChunk;
    const int per_tile = std::min(256, std::max(8, 2048 / (nt * nt)));
    const int nb = std::max(1, std::min(nchunk, per_tile));
    if (nb_out) *nb_out = nb;
    return (size_t)nt * nt * nb * kGramTile * kGramTile;
}

fkgp_status love_query(const GridDev& g, int kind, const double* ell, double so,
                       const double* Ct, int k, const int* first, const double* w, int nq,
                       double* U, double* partials, double* cov, hipStream_t s) {
    int nb = 1;
    (void)love_partials_doubles(nq, k, &nb);
    const int nt = (nq + kGramTile - 1) / kGramTile;
    love_project_kernel<<<nq, 256, 0, s>>>(g, Ct, k, first, w, U);
    gram_partial_kernel<<<dim3(nb, nt, nt), 256, 0, s>>>(U, k, nq, partials);
    const int64_t P = (int64_t)nq * nq;
    love_fin_kernel<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(
        g, kind, ell[0], ell[1], ell[2], so, first, w, partials, nb, nq, nt, cov);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status dia_to_canonical(const GridDev& g, fkgp_dtype dt, const void* A, void* out,
                             hipStream_t s) {
    int64_t M = 1;
    int NB = 1;
    for (int i = 0; i < g.d; ++i) {
        M *= g.m[i];
        NB *= 7;
    }
    dim3 tb(32, 8), tg((unsigned)((M + 31) / 32), (unsigned)((NB + 31) / 32));
    if (dt == FKGP_F32)
        dia_to_canonical_kernel<float><<<tg, tb, 0, s>>>(static_cast<const float*>(A),
                                                         static_cast<float*>(out), M, NB);
    else
        dia_to_canonical_kernel<double><<<tg, tb, 0, s>>>(static_cast<const double*>(A),
                                                          static_cast<double*>(out), M, NB);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

}  // namespace fkgp
