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
// Spans below 64 are exchanged with wavefront shuffles, larger spans stay in
// a lane's registers.  tws: exp(-2 pi i t / L), t < L/2; lams: spectrum.
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

template <class T, int LOG2L>
__device__ __forceinline__ void conv_line_regs(cplx<T> (&z)[line_regs<LOG2L>()], int e_lane,
                                               const cplx<T>* __restrict__ tws,
                                               const T* __restrict__ lams) {
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
                const cplx<T> w = tws[(e & (S - 1)) * (L / (2 * S))];
                const cplx<T> a = z[r], b = z[r + rs];
                z[r] = {a.re + b.re, a.im + b.im};
                z[r + rs] = cmul(cplx<T>{a.re - b.re, a.im - b.im}, w);
            }
        } else {
            const bool upper = (e_lane & S) != 0;
            const cplx<T> w = tws[(e_lane & (S - 1)) * (L / (2 * S))];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> p;
                p.re = __shfl_xor(z[r].re, S);
                p.im = __shfl_xor(z[r].im, S);
                const cplx<T> sum{z[r].re + p.re, z[r].im + p.im};
                const cplx<T> dif = cmul(cplx<T>{p.re - z[r].re, p.im - z[r].im}, w);
                z[r] = upper ? dif : sum;
            }
        }
    }
    // spectrum (bit-reversed order, includes 1/L)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T lmb = lams[r * 64 + e_lane];
        z[r].re *= lmb;
        z[r].im *= lmb;
    }
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
                const cplx<T> w = tws[(e & (S - 1)) * (L / (2 * S))];
                const cplx<T> a = z[r];
                const cplx<T> b = cmul_conj(z[r + rs], w);
                z[r] = {a.re + b.re, a.im + b.im};
                z[r + rs] = {a.re - b.re, a.im - b.im};
            }
        } else {
            const bool upper = (e_lane & S) != 0;
            const cplx<T> w = tws[(e_lane & (S - 1)) * (L / (2 * S))];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> p;
                p.re = __shfl_xor(z[r].re, S);
                p.im = __shfl_xor(z[r].im, S);
                const cplx<T> t = cmul_conj(upper ? z[r] : p, w);
                const cplx<T> a = upper ? p : z[r];
                z[r] = upper ? cplx<T>{a.re - t.re, a.im - t.im}
                             : cplx<T>{a.re + t.re, a.im + t.im};
            }
        }
    }
}

}  // namespace fkgp
