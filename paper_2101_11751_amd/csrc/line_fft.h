// Register-resident circulant convolution of one complex line (two real
// grid lines packed as real and imaginary parts) by a symmetric Toeplitz
// column embedded in a circulant of length L = 2^LOG2L (Sec. 2.3: K_G is
// multilevel Toeplitz on an equispaced grid and is applied with FFTs).
//
// Lane layout: L >= 64: lane holds elements e = r*64 + lane, r < L/64;
// L < 64: 64/L lines per wave, lane holds element lane % L.  Radix-2
// decimation in frequency (natural order in, bit-reversed out), pointwise
// scaling by the real spectrum stored in bit-reversed order (and already
// divided by L), then the matching decimation in time with conjugate
// twiddles (bit-reversed in, natural out): no permutation pass is needed.
// Spans below 64 are exchanged across lanes (DPP moves for spans up to 8, a
// swizzle for 16, a permute for 32), larger spans stay in a lane's registers.  tws: exp(-2 pi i t / L), t < L/2; lams: spectrum.
#pragma once

#include <hip/hip_runtime.h>

namespace fkgp {

template <class T>
struct cplx {
    T re, im;
};

template <class T>
__device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ inline cplx<T> cmul_conj(cplx<T> a, cplx<T> b) {  // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

template <int LOG2L>
constexpr int line_regs() { return (1 << LOG2L) >= 64 ? (1 << LOG2L) / 64 : 1; }

// Value of lane (lane ^ S) for S < 64.  Spans 1 and 2 are quad permutes and
// spans 4 and 8 a pair of row shifts and a select (DPP: VALU latency, no LDS
// round trip); span 16 is a swizzle (xor within 32 lanes), span 32 a
// permute through the LDS crossbar.
__device__ __forceinline__ int lane_xor_b32(int v, int S) {
    switch (S) {
        case 1:
            return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 2:
            return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 4: {
            const int from_up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, false);   // row_shl:4
            const int from_dn = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, false);   // row_shr:4
            return (__lane_id() & 4) ? from_dn : from_up;
        }
        case 8: {
            const int from_up = __builtin_amdgcn_mov_dpp(v, 0x108, 0xF, 0xF, false);   // row_shl:8
            const int from_dn = __builtin_amdgcn_mov_dpp(v, 0x118, 0xF, 0xF, false);   // row_shr:8
            return (__lane_id() & 8) ? from_dn : from_up;
        }
        case 16:
            return __builtin_amdgcn_ds_swizzle(v, 0x401F);   // xor_mask 16, and_mask 31
        default:
            return __shfl_xor(v, S);
    }
}

template <class T>
__device__ __forceinline__ T lane_xor(T v, int S);

template <>
__device__ __forceinline__ float lane_xor<float>(float v, int S) {
    return __int_as_float(lane_xor_b32(__float_as_int(v), S));
}

template <>
__device__ __forceinline__ double lane_xor<double>(double v, int S) {
    const int lo = lane_xor_b32(__double2loint(v), S);
    const int hi = lane_xor_b32(__double2hiint(v), S);
    return __hiloint2double(hi, lo);
}

// TS: stride into the twiddle table (2 when tws belongs to a transform of
// twice the length: the half-length twiddles are its even entries).
template <class T, int LOG2L, int TS = 1>
__device__ __forceinline__ void dif_regs(cplx<T> (&z)[line_regs<LOG2L>()], int e_lane,
                                         const cplx<T>* __restrict__ tws) {
    constexpr int L = 1 << LOG2L;
    constexpr int R = line_regs<LOG2L>();
    // forward DIF: spans L/2 .. 1
#pragma unroll
    for (int st = LOG2L - 1; st >= 0; --st) {
        const int S = 1 << st;
        if (S >= 64) {
            const int rs = S / 64;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r & rs) continue;
                const int e = r * 64 + e_lane;
                const cplx<T> w = tws[(e & (S - 1)) * (L / (2 * S)) * TS];
                const cplx<T> a = z[r], b = z[r + rs];
                z[r] = {a.re + b.re, a.im + b.im};
                z[r + rs] = cmul(cplx<T>{a.re - b.re, a.im - b.im}, w);
            }
        } else {
            const bool upper = (e_lane & S) != 0;
            // spans 1 and 2 use the twiddles 1 and -i only: no multiplication
            const cplx<T> w = S > 2 ? tws[(e_lane & (S - 1)) * (L / (2 * S)) * TS] : cplx<T>{T(1), T(0)};
            const bool odd = (e_lane & 1) != 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> p;
                p.re = lane_xor<T>(z[r].re, S);
                p.im = lane_xor<T>(z[r].im, S);
                const cplx<T> sum{z[r].re + p.re, z[r].im + p.im};
                const cplx<T> d{p.re - z[r].re, p.im - z[r].im};
                cplx<T> dif;
                if (S == 1) dif = d;
                else if (S == 2) dif = odd ? cplx<T>{d.im, -d.re} : d;
                else dif = cmul(d, w);
                z[r] = upper ? dif : sum;
            }
        }
    }
}

template <class T, int LOG2L, int TS = 1>
__device__ __forceinline__ void dit_regs(cplx<T> (&z)[line_regs<LOG2L>()], int e_lane,
                                         const cplx<T>* __restrict__ tws) {
    constexpr int L = 1 << LOG2L;
    constexpr int R = line_regs<LOG2L>();
    // inverse DIT: spans 1 .. L/2, conjugate twiddles
#pragma unroll
    for (int st = 0; st < LOG2L; ++st) {
        const int S = 1 << st;
        if (S >= 64) {
            const int rs = S / 64;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r & rs) continue;
                const int e = r * 64 + e_lane;
                const cplx<T> w = tws[(e & (S - 1)) * (L / (2 * S)) * TS];
                const cplx<T> a = z[r];
                const cplx<T> b = cmul_conj(z[r + rs], w);
                z[r] = {a.re + b.re, a.im + b.im};
                z[r + rs] = {a.re - b.re, a.im - b.im};
            }
        } else {
            const bool upper = (e_lane & S) != 0;
            const cplx<T> w = S > 2 ? tws[(e_lane & (S - 1)) * (L / (2 * S)) * TS] : cplx<T>{T(1), T(0)};
            const bool odd = (e_lane & 1) != 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> p;
                p.re = lane_xor<T>(z[r].re, S);
                p.im = lane_xor<T>(z[r].im, S);
                const cplx<T> x = upper ? z[r] : p;
                cplx<T> t;   // x * conj(w): w = 1 (span 1), 1 or -i (span 2)
                if (S == 1) t = x;
                else if (S == 2) t = odd ? cplx<T>{-x.im, x.re} : x;
                else t = cmul_conj(x, w);
                const cplx<T> a = upper ? p : z[r];
                z[r] = upper ? cplx<T>{a.re - t.re, a.im - t.im}
                             : cplx<T>{a.re + t.re, a.im + t.im};
            }
        }
    }
}

template <class T, int LOG2L>
__device__ __forceinline__ void conv_line_regs(cplx<T> (&z)[line_regs<LOG2L>()], int e_lane,
                                               const cplx<T>* __restrict__ tws,
                                               const T* __restrict__ lams) {
    constexpr int R = line_regs<LOG2L>();
    dif_regs<T, LOG2L>(z, e_lane, tws);
    // spectrum (bit-reversed order, includes 1/L)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T lmb = lams[r * 64 + e_lane];
        z[r].re *= lmb;
        z[r].im *= lmb;
    }
    dit_regs<T, LOG2L>(z, e_lane, tws);
}

__device__ inline unsigned bitrev_bits(unsigned v, int bits) {
    return bits ? (__brev(v) >> (32 - bits)) : 0u;
}

// Long lines: four-step convolution by one workgroup, L = L1 * L2 with
// L1, L2 >= 8 and L >= 64.  With n = L2 n1 + n2: (1) length-L1 DIF over n1
// for every n2, times the twiddle w_L^{n2 k1} (k1 = bit-reversed position
// p1); (2) per row p1: length-L2 DIF over n2, spectrum in the resulting order
// (lamp[p1][p2] = lambda[k1 + L1 k2] / L), length-L2 DIT, conjugate twiddle;
// (3) length-L1 DIT over p1 for every n2 (bit-reversed in, natural out).
// Sub-lengths below 64 put 64/L1 columns (64/L2 rows) in one wave.
// Y: L complex scratch in global memory owned by this workgroup.  twh: w_L^t
// for t < L/2 (w_L^{t + L/2} = -w_L^t); tw1/tw2: w_L1^t (t < L1/2) and
// w_L2^t (t < L2/2).  Lines a and b (b may be absent) of length m with
// stride S; the result, times `scale` plus add_coef * add, is written to dst
// (src == dst allowed: every read of a line precedes every write).
template <class T, int LG1, int LG2>
__device__ void wg_conv_long(const T* srcA, const T* srcB, int64_t S, int m, T* dstA, T* dstB,
                             T scale, const T* addA, const T* addB, T add_coef, cplx<T>* Y,
                             const cplx<T>* __restrict__ twh, const T* __restrict__ lamp,
                             const cplx<T>* tw1, const cplx<T>* tw2) {
    constexpr int L1 = 1 << LG1, L2 = 1 << LG2, L = L1 * L2;
    constexpr int R1 = line_regs<LG1>(), R2 = line_regs<LG2>();
    constexpr int G1 = L1 >= 64 ? 1 : 64 / L1, G2 = L2 >= 64 ? 1 : 64 / L2;
    static_assert(LG1 >= 3 && LG2 >= 3 && L >= 64, "four-step sub-lengths too short");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int e1 = L1 >= 64 ? lane : (lane & (L1 - 1)), g1 = L1 >= 64 ? 0 : lane / L1;
    const int e2 = L2 >= 64 ? lane : (lane & (L2 - 1)), g2 = L2 >= 64 ? 0 : lane / L2;
    auto cross = [&](unsigned t) -> cplx<T> {
        t &= (unsigned)(L - 1);
        if (t < (unsigned)(L / 2)) return twh[t];
        const cplx<T> w = twh[t - L / 2];
        return {-w.re, -w.im};
    };
    // (1) columns (G1 per wave; L2 is a multiple of G1 because L >= 64)
    for (int c0 = wave * G1; c0 < L2; c0 += nw * G1) {
        const int n2 = c0 + g1;
        cplx<T> z[R1];
#pragma unroll
        for (int q = 0; q < R1; ++q) {
            const int n = L2 * (q * 64 + e1) + n2;
            z[q].re = (n < m) ? srcA[(int64_t)n * S] : T(0);
            z[q].im = (n < m && srcB) ? srcB[(int64_t)n * S] : T(0);
        }
        dif_regs<T, LG1>(z, e1, tw1);
#pragma unroll
        for (int q = 0; q < R1; ++q) {
            const int p1 = q * 64 + e1;
            Y[p1 * L2 + n2] = cmul(z[q], cross((unsigned)n2 * bitrev_bits(p1, LG1)));
        }
    }
    __syncthreads();
    // (2) rows (G2 per wave)
    for (int r0 = wave * G2; r0 < L1; r0 += nw * G2) {
        const int p1 = r0 + g2;
        cplx<T> z[R2];
#pragma unroll
        for (int q = 0; q < R2; ++q) z[q] = Y[p1 * L2 + q * 64 + e2];
        dif_regs<T, LG2>(z, e2, tw2);
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            const T lm = lamp[p1 * L2 + q * 64 + e2];
            z[q].re *= lm;
            z[q].im *= lm;
        }
        dit_regs<T, LG2>(z, e2, tw2);
        const unsigned br = bitrev_bits(p1, LG1);
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            const int n2 = q * 64 + e2;
            Y[p1 * L2 + n2] = cmul_conj(z[q], cross((unsigned)n2 * br));
        }
    }
    __syncthreads();
    // (3) columns back
    for (int c0 = wave * G1; c0 < L2; c0 += nw * G1) {
        const int n2 = c0 + g1;
        cplx<T> z[R1];
#pragma unroll
        for (int q = 0; q < R1; ++q) z[q] = Y[(q * 64 + e1) * L2 + n2];
        dit_regs<T, LG1>(z, e1, tw1);
#pragma unroll
        for (int q = 0; q < R1; ++q) {
            const int n = L2 * (q * 64 + e1) + n2;
            if (n >= m) continue;
            T va = scale * z[q].re;
            if (addA) va += add_coef * addA[(int64_t)n * S];
            dstA[(int64_t)n * S] = va;
            if (dstB) {
                T vb = scale * z[q].im;
                if (addB) vb += add_coef * addB[(int64_t)n * S];
                dstB[(int64_t)n * S] = vb;
            }
        }
    }
    __syncthreads();
}

}  // namespace fkgp
