// One-shot O(n) pass: sufficient statistics W^T W, W^T y, y^T y and probe
// sketches W^T z_j (Sec. 3.1 "Precomputation"; Claim 2 and its proof).
//
// Pipeline (all deterministic, no floating-point atomics):
//   1. cell keys: each point's base cell (FP64 grid coordinate, floor) and a
//      per-tile digit histogram for the first radix pass;
//   2. stable LSD radix sort by cell key (digits of <= 10 bits; per-wave
//      ballot matching gives stable ranks; tiles write through registers);
//      the payload carries the raw coordinates, y and (for probes) the
//      original point index;
//   3. per-cell moments in FP64, in sorted (= input) order within the cell:
//      the cubic weights are polynomials of degree 3 in the fractional
//      offset t, so sum_i w_i w_i^T over a cell is fixed by the 7^d moments
//      sum_i prod_k b6_{q_k}(t_k) (q_k <= 6), and sum_i y_i w_i by the 4^d
//      moments sum_i y_i prod_k b3_{q_k}(t_k) (q_k <= 3), in the Bernstein-
//      type bases b6_q(t) = t^q (1-t)^(6-q) and b3_q(t) = t^q (1-t)^(3-q):
//      every term is non-negative, and each product of two weights has
//      Bernstein coefficients of one sign, so an entry of W^T W assembled
//      from the moments carries no cancellation beyond that of its own
//      defining sum (monomial moments t^q cancel badly for the small
//      products near t = 0 or 1, e.g. w_{i+2}^2 = t^4 (1-t)^2 / 4);
//   4. separable assembly: one pass per dimension turns a cell moment index
//      q_k into a stencil offset o_k (resp. sums it out for the vectors),
//      giving W^T W in stencil-diagonal form, W^T y and the sketches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace fkgp {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Interpolation weights as polynomials in t: weights of the nodes i-1, i,
// i+1, i+2 of a point at offset t from node i; Keys cubic convolution
// (a = -1/2), or linear interpolation (1 - t, t on i, i+1).  The tables hold
// their coefficients in the bases b6 / b3 of the moments (see above).
// ---------------------------------------------------------------------------
struct KeysTables {
    double E[7][4][7];   // [o+3][a][q]: coeff of b6_q in w_a(t) w_{a+o}(t)
    double C[4][4];      // [a][q]: coeff of b3_q in w_a(t)
};

// Coefficients of sum_k c_k t^k (degree <= deg) on t^q (1-t)^(deg-q):
// t^k = t^k (t + (1-t))^(deg-k) = sum_j binom(deg-k, j) t^(k+j) (1-t)^(deg-k-j).
// Exact in FP64 here (dyadic coefficients times small binomials).
void monomial_to_bernstein(const double* c, int deg, double* out) {
    for (int q = 0; q <= deg; ++q) out[q] = 0.0;
    for (int k = 0; k <= deg; ++k) {
        double binom = 1.0;   // binom(deg-k, j)
        for (int j = 0; j + k <= deg; ++j) {
            out[k + j] += c[k] * binom;
            binom = binom * (double)(deg - k - j) / (double)(j + 1);
        }
    }
}

KeysTables make_tables(int interp) {
    const double keys[4][4] = {{0.0, -0.5, 1.0, -0.5},
                               {1.0, 0.0, -2.5, 1.5},
                               {0.0, 0.5, 2.0, -1.5},
                               {0.0, 0.0, -0.5, 0.5}};
    const double lin[4][4] = {{0.0, 0.0, 0.0, 0.0},
                              {1.0, -1.0, 0.0, 0.0},
                              {0.0, 1.0, 0.0, 0.0},
                              {0.0, 0.0, 0.0, 0.0}};
    const double (&w)[4][4] = interp == 1 ? lin : keys;
    KeysTables t{};
    for (int a = 0; a < 4; ++a) monomial_to_bernstein(w[a], 3, t.C[a]);
    for (int o = -3; o <= 3; ++o)
        for (int a = 0; a < 4; ++a) {
            int b = a + o;
            if (b < 0 || b > 3) continue;
            double prod[7] = {};
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q) prod[p + q] += w[a][p] * w[b][q];
            monomial_to_bernstein(prod, 6, t.E[o + 3][a]);
        }
    return t;
}

// The moment bases at t in [0,1]: b6[q] = t^q (1-t)^(6-q), b3[q] = t^q (1-t)^(3-q).
__device__ inline void moment_basis(double t, double* b6, double* b3) {
    const double s = 1.0 - t;
    double tp[7], sp[7];
    tp[0] = 1.0;
    sp[0] = 1.0;
#pragma unroll
    for (int q = 1; q < 7; ++q) {
        tp[q] = tp[q - 1] * t;
        sp[q] = sp[q - 1] * s;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) b6[q] = tp[q] * sp[6 - q];
#pragma unroll
    for (int q = 0; q < 4; ++q) b3[q] = tp[q] * sp[3 - q];
}

// Grid coordinate of one dimension: u = (x - g0)/h in FP64, interpolable iff
// 1 <= u <= m-2; base node i = min(floor(u), m-3); t = u - i in [0,1].
__device__ inline bool locate(double x, double g0, double h, int m, int& base,
                              double& t) {
    double u = (x - g0) / h;
    if (!(u >= 1.0 && u <= (double)(m - 2))) return false;
    int i = (int)floor(u);
    if (i > m - 3) i = m - 3;
    base = i;
    t = u - (double)i;
    return true;
}

template <class Tin>
__device__ inline bool cell_of(const GridDev& g, const Tin* const* xs, int64_t i,
                               uint32_t& key) {
    uint32_t c = 0;
    bool ok = true;
    for (int k = 0; k < g.d; ++k) {
        int b;
        double t;
        ok &= locate((double)xs[k][i], g.g0[k], g.h[k], g.m[k], b, t);
        if (!ok) b = 1;
        c = c * (uint32_t)g.nc[k] + (uint32_t)(b - 1);
    }
    key = ok ? c : 0u;
    return ok;
}

// The same from coordinates already in registers (unused ones ignored).
template <class Tin>
__device__ inline bool cell_of_vals(const GridDev& g, Tin x0, Tin x1, Tin x2, uint32_t& key) {
    const Tin xv[3] = {x0, x1, x2};
    uint32_t c = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= g.d) break;
        int b;
        double t;
        ok &= locate((double)xv[k], g.g0[k], g.h[k], g.m[k], b, t);
        if (!ok) b = 1;
        c = c * (uint32_t)g.nc[k] + (uint32_t)(b - 1);
    }
    key = ok ? c : 0u;
    return ok;
}

template <class Tin>
struct Coords {
    const Tin* p[3];
};

// Payload: slots [0,d) coordinates, slot d the response, slot d+1 the
// original index (bit-cast) when probes are requested.
template <class Tin>
struct PayloadOf;
template <>
struct PayloadOf<float> { using type = float4; };
template <>
struct PayloadOf<double> { using type = double4; };

__device__ inline float idx_to_slot(uint32_t i, float) { return __uint_as_float(i); }
__device__ inline double idx_to_slot(uint32_t i, double) {
    return __longlong_as_double((long long)i);
}
__device__ inline uint32_t slot_to_idx(float v) { return __float_as_uint(v); }
__device__ inline uint32_t slot_to_idx(double v) { return (uint32_t)__double_as_longlong(v); }

template <class P, class S>
__device__ inline void set_slot(P& p, int s, S v) {
    if (s == 0) p.x = v;
    else if (s == 1) p.y = v;
    else if (s == 2) p.z = v;
    else p.w = v;
}
template <class P>
__device__ inline auto get_slot(const P& p, int s) -> decltype(p.x) {
    return s == 0 ? p.x : s == 1 ? p.y : s == 2 ? p.z : p.w;
}

template <class Tin>
constexpr int items_per_thread() { return sizeof(Tin) == 4 ? 16 : 8; }
template <class Tin>
constexpr int tile_size() { return kBlock * items_per_thread<Tin>(); }

// ---------------------------------------------------------------------------
// 1. Cell keys and the first pass's per-tile digit counts.
// ---------------------------------------------------------------------------
template <class Tin>
__global__ __launch_bounds__(kBlock) void keys_and_counts(
    Coords<Tin> xs, int64_t n, GridDev g, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ counts, int ntiles, int shift, int bits,
    unsigned long long* bad, int64_t idx_base) {
    extern __shared__ uint32_t hist[];
    const int nd = 1 << bits;
    for (int i = threadIdx.x; i < nd; i += kBlock) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * tile_size<Tin>();
    const int64_t end = min(n, base + tile_size<Tin>());
    // all of the thread's coordinates are requested before the first is used
    // (no branches around the loads: past the tile's end they repeat its
    // first item, past d they read dimension 0 again; both are discarded)
    constexpr int IT = items_per_thread<Tin>();
    const Tin* px[3] = {xs.p[0], g.d > 1 ? xs.p[1] : xs.p[0], g.d > 2 ? xs.p[2] : xs.p[0]};
    Tin xv[3][IT];
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = base + (int64_t)s * kBlock + threadIdx.x;
        const int64_t ic = i < end ? i : base;
#pragma unroll
        for (int k = 0; k < 3; ++k) xv[k][s] = px[k][ic];
    }
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = base + (int64_t)s * kBlock + threadIdx.x;
        if (i >= end) break;
        uint32_t key;
        if (!cell_of_vals<Tin>(g, xv[0][s], xv[1][s], xv[2][s], key))
            atomicMin(bad, (unsigned long long)(idx_base + i));
        keys[i] = key;
        atomicAdd(&hist[(key >> shift) & (nd - 1)], 1u);
    }
    __syncthreads();
    for (int dgt = threadIdx.x; dgt < nd; dgt += kBlock)
        counts[(size_t)dgt * ntiles + blockIdx.x] = hist[dgt];
}

// Per-tile digit counts of a later pass.
template <class Tin>
__global__ __launch_bounds__(kBlock) void digit_counts(
    const uint32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ counts,
    int ntiles, int shift, int bits) {
    extern __shared__ uint32_t hist[];
    const int nd = 1 << bits;
    for (int i = threadIdx.x; i < nd; i += kBlock) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * tile_size<Tin>();
    const int64_t end = min(n, base + tile_size<Tin>());
    // the thread's keys are requested together (clamped past the tile's end,
    // then not counted), then counted
    constexpr int IT = items_per_thread<Tin>();
    uint32_t kv[IT];
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = base + (int64_t)s * kBlock + threadIdx.x;
        kv[s] = keys[i < end ? i : base];
    }
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = base + (int64_t)s * kBlock + threadIdx.x;
        if (i < end) atomicAdd(&hist[(kv[s] >> shift) & (nd - 1)], 1u);
    }
    __syncthreads();
    for (int dgt = threadIdx.x; dgt < nd; dgt += kBlock)
        counts[(size_t)dgt * ntiles + blockIdx.x] = hist[dgt];
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (digit-major counts -> scatter offsets).
// ---------------------------------------------------------------------------
constexpr int kScanChunk = 4096;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
    // Hillis-Steele over 256 threads in LDS.
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[kBlock - 1];
    uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void scan_reduce(const uint32_t* __restrict__ in,
                                                       size_t n, uint32_t* __restrict__ sums) {
    __shared__ uint32_t sh[kBlock];
    size_t base = (size_t)blockIdx.x * kScanChunk;
    uint32_t acc = 0;
    for (int i = threadIdx.x; i < kScanChunk; i += kBlock)
        if (base + i < n) acc += in[base + i];
    uint32_t total;
    block_exclusive_scan(acc, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void scan_sums(uint32_t* __restrict__ sums, int nb) {
    __shared__ uint32_t sh[kBlock];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        int i = base + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(v, sh, total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void scan_apply(const uint32_t* __restrict__ in, size_t n,
                                                      const uint32_t* __restrict__ sums,
                                                      uint32_t* __restrict__ out) {
    __shared__ uint32_t sh[kBlock];
    constexpr int per = kScanChunk / kBlock;
    size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * per;
    uint32_t v[per];
    uint32_t acc = 0;
    for (int j = 0; j < per; ++j) {
        v[j] = base + j < n ? in[base + j] : 0u;
        acc += v[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(acc, sh, total) + sums[blockIdx.x];
    for (int j = 0; j < per; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

fkgp_status exclusive_scan(const uint32_t* in, uint32_t* out, size_t n, uint32_t* sums,
                           hipStream_t s) {
    int nb = (int)((n + kScanChunk - 1) / kScanChunk);
    scan_reduce<<<nb, kBlock, 0, s>>>(in, n, sums);
    scan_sums<<<1, kBlock, 0, s>>>(sums, nb);
    scan_apply<<<nb, kBlock, 0, s>>>(in, n, sums, out);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// ---------------------------------------------------------------------------
// 2. Stable scatter of one radix pass.  Wave w of a tile owns the contiguous
// chunk [w*64*IT, (w+1)*64*IT) and walks it in steps of 64; lanes with equal
// digits in a step are matched by ballots, so ranks follow input order.
// From the per-wave digit counts the tile's items get their positions in the
// tile sorted by digit (stable); the tile then writes that sequence out in
// kStageChunks chunks of consecutive positions staged through LDS, so each
// digit's run of the tile leaves as one contiguous, coalesced range of the
// output (items stay in registers; a chunk holds a quarter of the tile).
// ---------------------------------------------------------------------------
constexpr int kStageChunks = 4;

template <class Tin>
constexpr size_t scatter_lds_bytes(int bits) {
    // whist [4][nd] (then the per-wave offsets), local start [nd], global
    // base [nd], scan scratch [kBlock], staged keys and payloads of a chunk
    return sizeof(uint32_t) * ((size_t)4 * (1u << bits) + 2 * (1u << bits) + kBlock) +
           (sizeof(uint32_t) + sizeof(typename PayloadOf<Tin>::type)) *
               (tile_size<Tin>() / kStageChunks);
}

template <class Tin, bool kRaw>
__global__ __launch_bounds__(kBlock) void radix_scatter(
    const uint32_t* __restrict__ keys_in,
    const typename PayloadOf<Tin>::type* __restrict__ pay_in, Coords<Tin> xs,
    const Tin* __restrict__ yin, int d, bool with_idx, int64_t n,
    const uint32_t* __restrict__ offsets, int ntiles, int shift, int bits,
    uint32_t* __restrict__ keys_out, typename PayloadOf<Tin>::type* __restrict__ pay_out) {
    using P = typename PayloadOf<Tin>::type;
    constexpr int IT = items_per_thread<Tin>();
    constexpr int CH = tile_size<Tin>() / kStageChunks;
    extern __shared__ __align__(16) unsigned char lds_scatter[];
    const int nd = 1 << bits;
    // the payload stage first (16-byte aligned), then the 32-bit arrays
    P* stage_pay = reinterpret_cast<P*>(lds_scatter);
    uint32_t* stage_key = reinterpret_cast<uint32_t*>(stage_pay + CH);
    uint32_t* whist = stage_key + CH;          // [4][nd]
    uint32_t* lstart = whist + 4 * nd;         // [nd]
    uint32_t* gbase = lstart + nd;             // [nd]
    uint32_t* scan_sh = gbase + nd;            // [kBlock]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * nd; i += kBlock) whist[i] = 0;
    __syncthreads();

    const int64_t tbase = (int64_t)blockIdx.x * tile_size<Tin>();
    const int64_t wbase = tbase + (int64_t)wave * 64 * IT;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[IT];
    uint32_t rank[IT];
    P pay[IT];
    // all of the thread's keys and payloads are requested before the first
    // is ranked (the ranking's wavefront barriers would otherwise hold each
    // item's loads until the previous item is done); past the end of the
    // input the loads repeat the last item (n > 0) and the key marks it void
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = wbase + (int64_t)s * 64 + lane;
        const int64_t ic = i < n ? i : n - 1;
        uint32_t k = keys_in[ic];
        P p{};
        if constexpr (kRaw) {
            // no branches around the loads: a dimension past d reads
            // dimension 0 again and discards it
            const Tin* p1 = d > 1 ? xs.p[1] : xs.p[0];
            const Tin* p2 = d > 2 ? xs.p[2] : xs.p[0];
            const Tin v0 = xs.p[0][ic];
            const Tin v1 = p1[ic];
            const Tin v2 = p2[ic];
            const Tin yv = yin[ic];
            // slots: the d coordinates, then y, then the index when asked
            // for; in 3-D there is no fifth slot, so the index takes y's
            // place and the moments read y through it (selects on uniform
            // d and with_idx, no branches)
            const Tin idx = with_idx ? idx_to_slot((uint32_t)ic, Tin(0)) : Tin(0);
            p.x = v0;
            p.y = d > 1 ? v1 : yv;
            p.z = d > 2 ? v2 : (d == 2 ? yv : idx);
            p.w = d == 3 ? (with_idx ? idx : yv) : (d == 2 ? idx : Tin(0));
        } else {
            p = pay_in[ic];
        }
        key[s] = i < n ? k : 0xffffffffu;
        pay[s] = p;
    }
    // keep the scheduler from sinking those loads back next to their uses
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        const int64_t i = wbase + (int64_t)s * 64 + lane;
        const bool valid = i < n;
        const uint32_t k = valid ? key[s] : 0u;
        const uint32_t dg = (k >> shift) & (nd - 1);
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (dg >> b) & 1u;
            const unsigned long long bb = __ballot(valid && bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t r = 0;
        if (valid) r = whist[wave * nd + dg] + before;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (valid && before + 1 == cnt) whist[wave * nd + dg] = r + 1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        rank[s] = r;
    }
    __syncthreads();
    // tile-local digit starts: exclusive scan of the tile's digit counts
    // (each thread owns nd / kBlock consecutive digits, or one)
    const int per = (nd + kBlock - 1) / kBlock;
    uint32_t tsum = 0;
    for (int q = 0; q < per; ++q) {
        const int dg = threadIdx.x * per + q;
        if (dg < nd) tsum += whist[dg] + whist[nd + dg] + whist[2 * nd + dg] + whist[3 * nd + dg];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(tsum, scan_sh, total);
    for (int q = 0; q < per; ++q) {
        const int dg = threadIdx.x * per + q;
        if (dg < nd) {
            lstart[dg] = run;
            gbase[dg] = offsets[(size_t)dg * ntiles + blockIdx.x];
            uint32_t w_run = run;
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = whist[w * nd + dg];
                whist[w * nd + dg] = w_run;   // the wave's first tile position
                w_run += c;
            }
            run = w_run;
        }
    }
    __syncthreads();
    // position of each item in the digit-sorted tile
#pragma unroll
    for (int s = 0; s < IT; ++s) {
        if (key[s] == 0xffffffffu) continue;
        const uint32_t dg = (key[s] >> shift) & (nd - 1);
        rank[s] += whist[wave * nd + dg];
    }
    // write the sorted tile out, one chunk of CH consecutive positions at a time
    for (int c = 0; c < kStageChunks; ++c) {
        const uint32_t lo = (uint32_t)(c * CH);
        if ((int)lo >= (int)total) break;   // uniform: total is the tile's item count
#pragma unroll
        for (int s = 0; s < IT; ++s) {
            if (key[s] == 0xffffffffu) continue;
            const uint32_t q = rank[s] - lo;
            if (q < (uint32_t)CH) {
                stage_key[q] = key[s];
                stage_pay[q] = pay[s];
            }
        }
        __syncthreads();
        const int cnt = min(CH, (int)total - (int)lo);
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            const uint32_t k = stage_key[q];
            const uint32_t dg = (k >> shift) & (nd - 1);
            const uint32_t pos = gbase[dg] + (lo + (uint32_t)q - lstart[dg]);
            keys_out[pos] = k;
            pay_out[pos] = stage_pay[q];
        }
        __syncthreads();
    }
}

// Segment bounds of each cell in the sorted keys: one thread per 4 keys
// (one 16-byte load plus the two neighbours).
__global__ void cell_bounds(const uint32_t* __restrict__ keys, int64_t n,
                            uint32_t* __restrict__ start, uint32_t* __restrict__ end) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    constexpr uint32_t kNone = 0xffffffffu;   // no cell has this key
    uint32_t k[6];
    k[0] = i0 > 0 ? keys[i0 - 1] : kNone;
    if (i0 + 4 <= n) {
        const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
        k[1] = v.x;
        k[2] = v.y;
        k[3] = v.z;
        k[4] = v.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < n ? keys[i0 + j] : kNone;
    }
    k[5] = i0 + 4 < n ? keys[i0 + 4] : kNone;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = i0 + j;
        if (i >= n) break;
        const uint32_t kk = k[1 + j];
        if (k[j] != kk) start[kk] = (uint32_t)i;
        if (k[j + 2] != kk) end[kk] = (uint32_t)(i + 1);
    }
}

// ---------------------------------------------------------------------------
// 3. Per-cell moments (FP64), one wave per cell, points in batches of 64.
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double rademacher(uint64_t seed, uint64_t j, uint64_t i) {
    return (splitmix64((seed << 48) ^ (j << 40) ^ i) >> 63) ? -1.0 : 1.0;
}

template <int D>
constexpr int ipow_c(int b) {
    int r = 1;
    for (int i = 0; i < D; ++i) r *= b;
    return r;
}

constexpr int kPw = 34;   // LDS row: b6 (7 per dimension), then b3 (4 per dimension), pad
constexpr int kB3 = 21;   // offset of the b3 values in a row

template <int D, class Tin>
__global__ __launch_bounds__(64) void cell_moments(
    const typename PayloadOf<Tin>::type* __restrict__ pay,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, GridDev g,
    int nprobe, uint64_t seed, int ncells, const Tin* __restrict__ yin, uint64_t idx_base,
    double* __restrict__ Mw, double* __restrict__ Mr, double* __restrict__ Myy) {
    constexpr int NW = ipow_c<D>(7);
    constexpr int NR = ipow_c<D>(4);
    extern __shared__ double smem[];
    const int nr = 1 + nprobe;
    double(*pw)[kPw] = reinterpret_cast<double(*)[kPw]>(smem);
    double* rvb = smem + 64 * kPw;   // [64][nr]
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t s0 = cstart[cell];
    const uint32_t s1 = cend[cell];
    const int ncol_r = nr * (NR / 4);

    // W moments: D=3 lane owns (q1,q2) with 7 rows q0; D<=2 lane owns one moment.
    constexpr int WROWS = (D == 3) ? 7 : 1;
    double accw[WROWS];
#pragma unroll
    for (int r = 0; r < WROWS; ++r) accw[r] = 0.0;
    // rhs moments: columns (r, trailing q) with 4 rows q0 (D>=2: trailing
    // index over dims 1..D-1; D=1: one column per rhs, 4 rows).
    constexpr int MAXG = D == 3 ? 8 : 2;   // up to 512 (3-D) or 128 columns
    double accr[MAXG][4];
#pragma unroll
    for (int gi = 0; gi < MAXG; ++gi)
#pragma unroll
        for (int r = 0; r < 4; ++r) accr[gi][r] = 0.0;
    double accyy = 0.0;

    for (uint32_t b0 = s0; b0 < s1; b0 += 64) {
        const uint32_t i = b0 + lane;
        const int cnt = (int)min(64u, s1 - b0);
        if (i < s1) {
            auto p = pay[i];
            for (int k = 0; k < D; ++k) {
                int base;
                double t;
                locate((double)get_slot(p, k), g.g0[k], g.h[k], g.m[k], base, t);
                double b6[7], b3[4];
                moment_basis(t, b6, b3);
                for (int q = 0; q < 7; ++q) pw[lane][k * 7 + q] = b6[q];
                for (int q = 0; q < 4; ++q) pw[lane][kB3 + k * 4 + q] = b3[q];
            }
            // 3-D with probes: slot 3 holds the original index, y is read
            // through it; else slot D holds y and slot D + 1 the index
            const bool y_by_idx = D == 3 && nprobe > 0;
            const uint32_t orig =
                nprobe > 0 ? slot_to_idx(get_slot(p, y_by_idx ? D : D + 1)) : 0u;
            const double yv = y_by_idx ? (double)yin[orig] : (double)get_slot(p, D);
            rvb[lane * nr] = yv;
            if (nprobe > 0) {
                // probe entries follow the point's index in the whole data
                // set (idx_base: the first point of this chunk)
                for (int j = 0; j < nprobe; ++j)
                    rvb[lane * nr + 1 + j] = rademacher(seed, j, idx_base + orig);
            }
        } else {
            for (int q = 0; q < kPw; ++q) pw[lane][q] = 0.0;
            for (int j = 0; j < nr; ++j) rvb[lane * nr + j] = 0.0;
        }
        __syncthreads();
        // W moments
        if constexpr (D == 3) {
            if (lane < 49) {
                const int q1 = lane / 7, q2 = lane % 7;
                for (int p = 0; p < cnt; ++p) {
                    const double bc = pw[p][7 + q1] * pw[p][14 + q2];
#pragma unroll
                    for (int q0 = 0; q0 < 7; ++q0) accw[q0] = fma(pw[p][q0], bc, accw[q0]);
                }
            }
        } else if constexpr (D == 2) {
            if (lane < 49) {
                const int q0 = lane / 7, q1 = lane % 7;
                for (int p = 0; p < cnt; ++p) accw[0] = fma(pw[p][q0], pw[p][7 + q1], accw[0]);
            }
        } else {
            if (lane < 7)
                for (int p = 0; p < cnt; ++p) accw[0] += pw[p][lane];
        }
        // rhs moments
#pragma unroll
        for (int gi = 0; gi < MAXG; ++gi) {
            const int col = gi * 64 + lane;
            if (col < ncol_r) {
                if constexpr (D == 1) {
                    const int r = col;
                    for (int p = 0; p < cnt; ++p) {
                        const double yv = rvb[p * nr + r];
#pragma unroll
                        for (int q = 0; q < 4; ++q) accr[gi][q] = fma(yv, pw[p][kB3 + q], accr[gi][q]);
                    }
                } else if constexpr (D == 2) {
                    const int r = col / 4, q1 = col % 4;
                    for (int p = 0; p < cnt; ++p) {
                        const double yb = rvb[p * nr + r] * pw[p][kB3 + 4 + q1];
#pragma unroll
                        for (int q0 = 0; q0 < 4; ++q0)
                            accr[gi][q0] = fma(pw[p][kB3 + q0], yb, accr[gi][q0]);
                    }
                } else {
                    const int r = col / 16, q1 = (col / 4) % 4, q2 = col % 4;
                    for (int p = 0; p < cnt; ++p) {
                        const double ybc =
                            rvb[p * nr + r] * pw[p][kB3 + 4 + q1] * pw[p][kB3 + 8 + q2];
#pragma unroll
                        for (int q0 = 0; q0 < 4; ++q0)
                            accr[gi][q0] = fma(pw[p][kB3 + q0], ybc, accr[gi][q0]);
                    }
                }
            }
        }
        if (lane == 0)
            for (int p = 0; p < cnt; ++p) accyy = fma(rvb[p * nr], rvb[p * nr], accyy);
        __syncthreads();
    }
    // write out: Mw[cell][q0..], Mr[r][cell][q], Myy[cell]
    if constexpr (D == 3) {
        if (lane < 49)
#pragma unroll
            for (int q0 = 0; q0 < 7; ++q0) Mw[(size_t)cell * NW + q0 * 49 + lane] = accw[q0];
    } else if constexpr (D == 2) {
        if (lane < 49) Mw[(size_t)cell * NW + lane] = accw[0];
    } else {
        if (lane < 7) Mw[(size_t)cell * NW + lane] = accw[0];
    }
#pragma unroll
    for (int gi = 0; gi < MAXG; ++gi) {
        const int col = gi * 64 + lane;
        if (col < ncol_r) {
            int r, rest;
            if (D == 1) { r = col; rest = 0; }
            else if (D == 2) { r = col / 4; rest = col % 4; }
            else { r = col / 16; rest = col % 16; }
            const int trail = (D == 1) ? 1 : (D == 2 ? 4 : 16);
            double* dst = Mr + ((size_t)r * ncells + cell) * NR;
#pragma unroll
            for (int q0 = 0; q0 < 4; ++q0) dst[q0 * trail + rest] = accr[gi][q0];
        }
    }
    if (lane == 0) Myy[cell] = accyy;
}

// 3-D moments (no probes), accumulated in registers.  The wave walks the
// cell's points in batches of 64: each lane loads one point (the next
// batch's load is in flight while the current batch is reduced), locates it
// and writes its basis values b6, b3 of the three coordinates and y to one
// LDS row.  Then lane l = 8 g + j of point group g (points g, g + 8, ... of
// the batch, in sorted order) accumulates, for q2 = j (j < 7; lane j = 7
// repeats q2 = 6 to keep the instruction stream uniform and discards it), the
// 49 W moments b6_q0(t0) b6_q1(t1) b6_q2(t2), and the response moments
// y b3_q0 b3_q1 b3_q2 with q2 = j / 2 and q1 = 2 (j % 2) + {0, 1} (8 of the
// 64 per lane, so the y work is spread evenly over the group).  At the end
// the 8 groups are summed in group order through LDS.  Deterministic: every
// sum has a fixed order.
constexpr int kRow3 = 34;   // LDS row: b6 x 3 (0..20), b3 x 3 (21..32), y (33)

template <class Tin>
__global__ __launch_bounds__(64) void cell_moments3(
    const typename PayloadOf<Tin>::type* __restrict__ pay,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, GridDev g,
    double* __restrict__ Mw, double* __restrict__ Mr, double* __restrict__ Myy) {
    using P = typename PayloadOf<Tin>::type;
    __shared__ __align__(16) double pts[64 * kRow3];
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const int grp = lane >> 3, j = lane & 7;
    const int q2 = j < 7 ? j : 6;
    const int q2y = j >> 1, q1y = 2 * (j & 1);
    const uint32_t s0 = cstart[cell];
    const uint32_t s1 = cend[cell];
    double acc[7][7], accy[2][4];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int k = 0; k < 7; ++k) acc[i][k] = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) accy[i][k] = 0.0;
    double accyy = 0.0;
    P cur{};
    if (s0 + lane < s1) cur = pay[s0 + lane];
    for (uint32_t b0 = s0; b0 < s1; b0 += 64) {
        const int cnt = (int)min(64u, s1 - b0);
        if (lane < cnt) {
            double* row = pts + lane * kRow3;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int base;
                double t;
                if (!locate((double)get_slot(cur, k), g.g0[k], g.h[k], g.m[k], base, t)) t = 0.0;
                moment_basis(t, row + 7 * k, row + 21 + 4 * k);
            }
            row[33] = (double)get_slot(cur, 3);
        }
        if (b0 + 64 + lane < s1) cur = pay[b0 + 64 + lane];
        __syncthreads();
        for (int p = grp; p < cnt; p += 8) {
            const double* r = pts + p * kRow3;
            double av[7], bv[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                av[q] = r[q];
                bv[q] = r[7 + q];
            }
            const double c = r[14 + q2];
#pragma unroll
            for (int q0 = 0; q0 < 7; ++q0) {
                const double ac = av[q0] * c;
#pragma unroll
                for (int q1 = 0; q1 < 7; ++q1) acc[q0][q1] = fma(ac, bv[q1], acc[q0][q1]);
            }
            const double yv = r[33];
            const double yc = yv * r[29 + q2y];
            const double y0 = yc * r[25 + q1y], y1 = yc * r[26 + q1y];
#pragma unroll
            for (int q0 = 0; q0 < 4; ++q0) {
                const double a3 = r[21 + q0];
                accy[0][q0] = fma(y0, a3, accy[0][q0]);
                accy[1][q0] = fma(y1, a3, accy[1][q0]);
            }
            accyy = fma(yv, yv, accyy);
        }
        __syncthreads();
    }
    // sum the 8 groups: 58 values per lane (49 W, 8 response, 1 y^2), in two
    // chunks of 29 through the LDS table
    constexpr int kCh = 29;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
#pragma unroll
        for (int i = 0; i < kCh; ++i) {
            const int v = ch * kCh + i;
            double x;
            if (v < 49) x = acc[v / 7][v % 7];
            else if (v < 57) x = accy[(v - 49) / 4][(v - 49) % 4];
            else x = accyy;
            pts[lane * kCh + i] = x;
        }
        __syncthreads();
        for (int o = lane; o < 8 * kCh; o += 64) {
            const int oj = o / kCh, i = o % kCh;
            const int v = ch * kCh + i;
            double sum = 0.0;
            for (int gg = 0; gg < 8; ++gg) sum += pts[(gg * 8 + oj) * kCh + i];
            if (v < 49) {
                if (oj < 7) Mw[(size_t)cell * 343 + (v / 7) * 49 + (v % 7) * 7 + oj] = sum;
            } else if (v < 57) {
                const int k = v - 49;   // (pair, q0)
                const int q1 = 2 * (oj & 1) + k / 4, q0 = k % 4;
                Mr[(size_t)cell * 64 + q0 * 16 + q1 * 4 + (oj >> 1)] = sum;
            } else if (oj == 0) {
                Myy[cell] = sum;
            }
        }
        __syncthreads();
    }
}

// 2-D moments (no probes): lane l accumulates, over the points l, l + 64,
// ... of the cell (sorted order), all 49 moments b6_q0(t0) b6_q1(t1) and the
// 16 response moments y b3_q0(t0) b3_q1(t1) in registers; the 64 lanes are
// then summed in lane order through LDS.  Cells of the 2-D workloads hold
// hundreds to thousands of points, so every lane stays busy.
template <class Tin>
__global__ __launch_bounds__(64) void cell_moments2(
    const typename PayloadOf<Tin>::type* __restrict__ pay,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, GridDev g,
    double* __restrict__ Mw, double* __restrict__ Mr, double* __restrict__ Myy) {
    __shared__ double red[64][17];
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t s0 = cstart[cell];
    const uint32_t s1 = cend[cell];
    double acc[7][7], accy[4][4];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int j = 0; j < 7; ++j) acc[i][j] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) accy[i][j] = 0.0;
    double accyy = 0.0;
    for (uint32_t i = s0 + lane; i < s1; i += 64) {
        const auto p = pay[i];
        double t[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            int base;
            if (!locate((double)get_slot(p, k), g.g0[k], g.h[k], g.m[k], base, t[k])) t[k] = 0.0;
        }
        const double yv = (double)get_slot(p, 2);
        double av[7], bv[7], a3[4], b3[4];
        moment_basis(t[0], av, a3);
        moment_basis(t[1], bv, b3);
#pragma unroll
        for (int q0 = 0; q0 < 7; ++q0)
#pragma unroll
            for (int q1 = 0; q1 < 7; ++q1) acc[q0][q1] = fma(av[q0], bv[q1], acc[q0][q1]);
#pragma unroll
        for (int q0 = 0; q0 < 4; ++q0) {
            const double ay = a3[q0] * yv;
#pragma unroll
            for (int q1 = 0; q1 < 4; ++q1) accy[q0][q1] = fma(ay, b3[q1], accy[q0][q1]);
        }
        accyy = fma(yv, yv, accyy);
    }
    // 66 values per lane (49 + 16 + 1), summed over the 64 lanes in lane order,
    // in chunks of 17 through LDS
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
#pragma unroll
        for (int j = 0; j < 17; ++j) {
            const int v = ch * 17 + j;
            double x = 0.0;
            if (v < 49) x = acc[v / 7][v % 7];
            else if (v < 65) x = accy[(v - 49) / 4][(v - 49) % 4];
            else if (v == 65) x = accyy;
            red[lane][j] = x;
        }
        __syncthreads();
        if (lane < 17) {
            const int v = ch * 17 + lane;
            double sum = 0.0;
            for (int l = 0; l < 64; ++l) sum += red[l][lane];
            if (v < 49) Mw[(size_t)cell * 49 + v] = sum;                  // q0*7 + q1
            else if (v < 65) Mr[(size_t)cell * 16 + (v - 49)] = sum;      // q0*4 + q1
            else if (v == 65) Myy[cell] = sum;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 4. Separable assembly.
// ---------------------------------------------------------------------------
struct Dims3 {
    int n[3];
};

// W^T W stage for dimension k: payload digit k (base 7) changes from a moment
// index q to an offset index o+3; spatial dimension k grows from cells to
// nodes: out[.., j_k, ..][.., o, ..] = sum_{a, q} E[o][a][q] in[.., j_k-a, ..][.., q, ..].
// One thread per (output position, payload with digit k removed): it reads
// the 4 x 7 inputs once and produces all 7 offsets.  Positions (< 2^30) use
// 32-bit arithmetic; the flat thread index is split by a compile-time 7^(d-1).
template <int D>
__global__ __launch_bounds__(256) void assemble_wtw_stage(const double* __restrict__ in,
                                                          double* __restrict__ out, Dims3 sin,
                                                          Dims3 sout, int k, KeysTables tab) {
    constexpr int P = D == 1 ? 7 : (D == 2 ? 49 : 343);
    constexpr int P0 = P / 7;
    const int64_t tot_sp = (int64_t)sout.n[0] * sout.n[1] * sout.n[2];
    // workgroups are dealt to the 8 XCDs in turn; the grid is a multiple of 8
    // and XCD x takes the x-th contiguous eighth of the node order, so the
    // neighbours that share input cells share one L2
    const unsigned per_xcd = gridDim.x / 8;
    const unsigned lb = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t idx = (int64_t)lb * blockDim.x + threadIdx.x;
    if (idx >= tot_sp * P0) return;
    const int p0i = (int)(idx % P0);
    const int sp = (int)(idx / P0);
    int pstride = 1;
    for (int i = D - 1; i > k; --i) pstride *= 7;
    const int pay0 = (p0i / pstride) * pstride * 7 + p0i % pstride;
    // output node: dimension k varies fastest over the launch (then the
    // other two in C order), so the four nodes that read the same input
    // cell run in the same or neighbouring workgroups
    int s[3];
    {
        const int ka = k == 0 ? 1 : 0, kb = k == 2 ? 1 : 2;   // the other two, in order
        int r = sp;
        s[k] = r % sout.n[k];
        r /= sout.n[k];
        s[kb] = r % sout.n[kb];
        s[ka] = r / sout.n[kb];
    }
    const int64_t spl = ((int64_t)s[0] * sout.n[1] + s[1]) * sout.n[2] + s[2];
    double acc[7];
#pragma unroll
    for (int o = 0; o < 7; ++o) acc[o] = 0.0;
    // the 4 x 7 loads are issued together: a cell outside the grid is read
    // at a clamped position and its values zeroed (no branch around loads)
    double v[4][7];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int c = s[k] - a;
        const int cc = min(max(c, 0), sin.n[k] - 1);
        int t[3] = {s[0], s[1], s[2]};
        t[k] = cc;
        const int64_t ib = (int64_t)((t[0] * sin.n[1] + t[1]) * sin.n[2] + t[2]) * P + pay0;
#pragma unroll
        for (int q = 0; q < 7; ++q) v[a][q] = in[ib + q * pstride];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int c = s[k] - a;
        const bool ok = c >= 0 && c < sin.n[k];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double x = ok ? v[a][q] : 0.0;
#pragma unroll
            for (int o = 0; o < 7; ++o) acc[o] = fma(tab.E[o][a][q], x, acc[o]);
        }
    }
    const int64_t ob = spl * P + pay0;
#pragma unroll
    for (int o = 0; o < 7; ++o) out[ob + o * pstride] = acc[o];
}

// Vector stage for dimension k (processed from the last to the first): the
// trailing payload digit q_k (base 4) is summed out:
// out[r][.., j_k, ..][p] = sum_{a, q} C[a][q] in[r][.., j_k-a, ..][p*4 + q].
__global__ void assemble_vec_stage(const double* __restrict__ in, double* __restrict__ out,
                                   Dims3 sin, Dims3 sout, int k, int Pout, int nr,
                                   KeysTables tab) {
    const int64_t sp_out = (int64_t)sout.n[0] * sout.n[1] * sout.n[2];
    const int64_t sp_in = (int64_t)sin.n[0] * sin.n[1] * sin.n[2];
    const int64_t total = sp_out * Pout * nr;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int p = (int)(idx % Pout);
    int64_t rest = idx / Pout;
    int64_t sp = rest % sp_out;
    const int r = (int)(rest / sp_out);
    int s[3];
    for (int i = 2; i >= 0; --i) {
        s[i] = (int)(sp % sout.n[i]);
        sp /= sout.n[i];
    }
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
        const int c = s[k] - a;
        if (c < 0 || c >= sin.n[k]) continue;
        int t[3] = {s[0], s[1], s[2]};
        t[k] = c;
        const int64_t ib = ((int64_t)r * sp_in + ((int64_t)t[0] * sin.n[1] + t[1]) * sin.n[2] + t[2]) *
                               (Pout * 4) + (int64_t)p * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = fma(tab.C[a][q], in[ib + q], acc);
    }
    out[idx] = acc;
}

// [M][7^d] double -> row-tiled diagonal layout in T (LDS-tiled transpose);
// rows past M in the last tile are written as zeros.
template <class T>
__global__ void transpose_to_dia(const double* __restrict__ in, T* __restrict__ out, int64_t M,
                                 int NB, uint32_t* __restrict__ bmask) {
    __shared__ double tile[32][33];
    __shared__ uint32_t occ;
    const int64_t j0 = (int64_t)blockIdx.x * 32;
    const int o0 = blockIdx.y * 32;
    if (threadIdx.x == 0 && threadIdx.y == 0) occ = 0u;
    for (int r = threadIdx.y; r < 32; r += 8) {
        int64_t j = j0 + r;
        int o = o0 + threadIdx.x;
        tile[r][threadIdx.x] = (j < M && o < NB) ? in[j * NB + o] : 0.0;
    }
    __syncthreads();
    // the block's 32 rows lie in one wavefront chunk of one row tile
    const int w = (int)((j0 % kRowTile) / kWaveRows);
    uint32_t bits = 0u;
    for (int r = threadIdx.y; r < 32; r += 8) {
        int o = o0 + r;
        int64_t j = j0 + threadIdx.x;
        if (o < NB) {
            const T v = (T)tile[threadIdx.x][r];
            out[dia_index(j, o, NB)] = v;
            if (v != T(0)) bits |= 1u << (w * kMaskSlabs + o / 49);
        }
    }
    // OR over the wavefront, then one LDS OR per wavefront (integer
    // operations: order-independent)
    for (int off = 32; off > 0; off >>= 1) bits |= (uint32_t)__shfl_xor((int)bits, off);
    if (((threadIdx.y * 32 + threadIdx.x) & 63) == 0 && bits) atomicOr(&occ, bits);
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0 && occ) atomicOr(&bmask[j0 / kRowTile], occ);
}

// Number of set bits of the block-occupancy mask (one workgroup).
__global__ __launch_bounds__(256) void count_mask_bits(const uint32_t* __restrict__ bmask,
                                                       int64_t nwords,
                                                       unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sh[256];
    unsigned long long c = 0;
    for (int64_t i = threadIdx.x; i < nwords; i += 256) c += (unsigned long long)__popc(bmask[i]);
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Deterministic sum of the per-cell sums of y^2 in two launches: 256
// workgroups each reduce one contiguous chunk in a fixed order, then one
// workgroup reduces the 256 partial sums (fixed trees throughout).
__global__ __launch_bounds__(256) void sum_chunks(const double* __restrict__ v, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ double sh[256];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = min(n, lo + chunk);
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Deterministic sum of a short array (single block, fixed tree).
__global__ __launch_bounds__(1024) void sum_fixed(const double* __restrict__ v, int64_t n,
                                                  double* __restrict__ out) {
    __shared__ double sh[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Sub-allocation from one scratch block (256-byte aligned pieces): one
// stream-ordered allocation and one free per precompute instead of a dozen
// (each allocator call costs host time).
struct Carver {
    unsigned char* base = nullptr;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += (count * sizeof(T) + 255) & ~size_t(255);
        return p;
    }
    template <class T>
    void skip(size_t count) {
        off += (count * sizeof(T) + 255) & ~size_t(255);
    }
};

// Element-wise acc (+)= v (chunked precompute: moments of the chunks summed
// in chunk order).
__global__ void add_moments(double* __restrict__ acc, const double* __restrict__ v, int64_t n,
                            int first) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc[i] = first ? v[i] : acc[i] + v[i];
}

// Kept points of a 3-D sort that carried the point index in y's slot (probe
// sketches requested): y is put back into the slot from the input, so the
// kept payload is (x, y, z, y) as without probes.
template <class Tin>
__global__ void kept_payload_with_y(const typename PayloadOf<Tin>::type* __restrict__ pay,
                                    const Tin* __restrict__ y, int64_t n,
                                    typename PayloadOf<Tin>::type* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto p = pay[i];
    p.w = y[slot_to_idx(p.w)];
    out[i] = p;
}

template <class Tin>
fkgp_status precompute_typed(const GridDev& g, const void* const* xv, const void* yv,
                             int64_t n, fkgp_dtype stats, int nprobe, uint64_t seed,
                             const StatsOut& out, unsigned long long* bad, hipStream_t s,
                             const ChunkCtl* cc) {
    using P = typename PayloadOf<Tin>::type;
    const int d = g.d;
    int64_t ncells = 1, M = 1;
    for (int k = 0; k < d; ++k) {
        ncells *= g.nc[k];
        M *= g.m[k];
    }
    int NB = 1;
    for (int k = 0; k < d; ++k) NB *= 7;
    int NR = 1;
    for (int k = 0; k < d; ++k) NR *= 4;
    const int nr = 1 + nprobe;
    Coords<Tin> xs{};
    for (int k = 0; k < d; ++k) xs.p[k] = static_cast<const Tin*>(xv[k]);
    const Tin* y = static_cast<const Tin*>(yv);

    // key bits and digit plan
    int key_bits = 1;
    while ((int64_t(1) << key_bits) < ncells) ++key_bits;
    // at most 8 bits a pass: a tile of 4096 items then leaves in runs of 16
    // or more items per digit, long enough that partial cache lines at the
    // run ends cost less than another pass (9-10 bit digits left runs of 4-8
    // items and wrote 2-3x the bytes moved)
    const int npass = (key_bits + 7) / 8;
    int dbits[8], dshift[8];
    {
        int sh = 0;
        for (int p = 0; p < npass; ++p) {
            dbits[p] = (key_bits - sh + (npass - p) - 1) / (npass - p);
            dshift[p] = sh;
            sh += dbits[p];
        }
    }
    const int ntiles = (int)((n + tile_size<Tin>() - 1) / tile_size<Tin>());

    // scratch layout: the per-cell moments and cell bounds live throughout;
    // the sort buffers and the assembly buffers share one region (the sort
    // is finished before the assembly starts)
    const size_t ncount = (size_t)ntiles << 10;
    auto sort_bytes = [&](Carver c) {
        c.skip<uint32_t>((size_t)n);
        c.skip<uint32_t>((size_t)n);
        c.skip<P>((size_t)n);
        c.skip<P>((size_t)n);
        c.skip<uint32_t>(ncount);
        c.skip<uint32_t>(ncount);
        c.skip<uint32_t>((ncount + kScanChunk - 1) / kScanChunk + 1);
        return c.off;
    };
    auto asm_bytes = [&](Carver c) {
        c.skip<double>((size_t)M * NB);
        c.skip<double>((size_t)M * NB);
        return c.off;
    };
    auto vec_bytes = [&](Carver c) {
        c.skip<double>((size_t)M * NR * nr);
        c.skip<double>((size_t)M * NR * nr);
        return c.off;
    };
    Carver whole;
    double* Mw = whole.take<double>((size_t)ncells * NB);
    double* Mr = whole.take<double>((size_t)ncells * NR * nr);
    double* Myy = whole.take<double>((size_t)ncells);
    uint32_t* cstart = whole.take<uint32_t>((size_t)ncells);
    uint32_t* cend = whole.take<uint32_t>((size_t)ncells);
    const size_t shared_off = whole.off;
    Carver z0;
    const size_t region = std::max({sort_bytes(z0), asm_bytes(z0), vec_bytes(z0)});
    unsigned char* block = nullptr;
    const DevAlloc dalloc = current_alloc();
    FKGP_HIP(alloc_async(dalloc, &block, shared_off + region, s));
    auto rebase = [&](auto* p) {
        return reinterpret_cast<decltype(p)>(block + reinterpret_cast<uintptr_t>(p));
    };
    Mw = rebase(Mw);
    Mr = rebase(Mr);
    Myy = rebase(Myy);
    cstart = rebase(cstart);
    cend = rebase(cend);
    FKGP_HIP(hipMemsetAsync(cstart, 0, sizeof(uint32_t) * ncells, s));
    FKGP_HIP(hipMemsetAsync(cend, 0, sizeof(uint32_t) * ncells, s));

    if (n > 0) {
        Carver c{block + shared_off, 0};
        uint32_t* ka = c.take<uint32_t>((size_t)n);
        uint32_t* kb = c.take<uint32_t>((size_t)n);
        P* pa = c.take<P>((size_t)n);
        P* pb = c.take<P>((size_t)n);
        uint32_t* counts = c.take<uint32_t>(ncount);
        uint32_t* offs = c.take<uint32_t>(ncount);
        uint32_t* sums = c.take<uint32_t>((ncount + kScanChunk - 1) / kScanChunk + 1);

        keys_and_counts<Tin><<<ntiles, kBlock, sizeof(uint32_t) << dbits[0], s>>>(
            xs, n, g, ka, counts, ntiles, dshift[0], dbits[0], bad, cc ? cc->idx_base : 0);
        FKGP_HIP(hipGetLastError());
        uint32_t* kin = ka;
        uint32_t* kout = kb;
        P* pin = pa;
        P* pout = pb;
        for (int p = 0; p < npass; ++p) {
            const size_t nc = (size_t)ntiles << dbits[p];
            if (p > 0) {
                digit_counts<Tin><<<ntiles, kBlock, sizeof(uint32_t) << dbits[p], s>>>(
                    kin, n, counts, ntiles, dshift[p], dbits[p]);
                FKGP_HIP(hipGetLastError());
            }
            fkgp_status st = exclusive_scan(counts, offs, nc, sums, s);
            if (st != FKGP_OK) return st;
            const size_t lds = scatter_lds_bytes<Tin>(dbits[p]);
            // the index rides along for the probes (and, for d <= 2, in the
            // kept payload); 3-D kept points keep y in its slot instead
            const bool with_idx = nprobe > 0 || (out.keep_pay != nullptr && d <= 2);
            if (p == 0)
                radix_scatter<Tin, true><<<ntiles, kBlock, lds, s>>>(
                    kin, nullptr, xs, y, d, with_idx, n, offs, ntiles, dshift[p], dbits[p],
                    kout, pout);
            else
                radix_scatter<Tin, false><<<ntiles, kBlock, lds, s>>>(
                    kin, pin, xs, y, d, with_idx, n, offs, ntiles, dshift[p], dbits[p],
                    kout, pout);
            FKGP_HIP(hipGetLastError());
            std::swap(kin, kout);
            std::swap(pin, pout);
        }
        // kin/pin now hold the sorted keys/payload
        cell_bounds<<<(unsigned)((n + 1023) / 1024), 256, 0, s>>>(kin, n, cstart, cend);
        FKGP_HIP(hipGetLastError());
        if (out.keep_pay) {
            if (d == 3 && nprobe > 0) {
                kept_payload_with_y<Tin><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
                    pin, y, n, static_cast<P*>(out.keep_pay));
                FKGP_HIP(hipGetLastError());
            } else {
                FKGP_HIP(hipMemcpyAsync(out.keep_pay, pin, sizeof(P) * (size_t)n,
                                        hipMemcpyDeviceToDevice, s));
            }
        }
        const size_t lds_mom = sizeof(double) * 64 * (kPw + nr);
        const uint64_t idx_base = cc ? (uint64_t)cc->idx_base : 0ull;   // chunk's first point
        if (d == 1)
            cell_moments<1, Tin><<<(unsigned)ncells, 64, lds_mom, s>>>(
                pin, cstart, cend, g, nprobe, seed, (int)ncells, y, idx_base, Mw, Mr, Myy);
        else if (d == 2 && nprobe == 0)
            cell_moments2<Tin><<<(unsigned)ncells, 64, 0, s>>>(pin, cstart, cend, g, Mw, Mr, Myy);
        else if (d == 2)
            cell_moments<2, Tin><<<(unsigned)ncells, 64, lds_mom, s>>>(
                pin, cstart, cend, g, nprobe, seed, (int)ncells, y, idx_base, Mw, Mr, Myy);
        else if (nprobe == 0)
            cell_moments3<Tin><<<(unsigned)ncells, 64, 0, s>>>(pin, cstart, cend, g, Mw, Mr, Myy);
        else
            cell_moments<3, Tin><<<(unsigned)ncells, 64, lds_mom, s>>>(
                pin, cstart, cend, g, nprobe, seed, (int)ncells, y, idx_base, Mw, Mr, Myy);
        FKGP_HIP(hipGetLastError());
    } else {
        FKGP_HIP(hipMemsetAsync(Mw, 0, sizeof(double) * ncells * NB, s));
        FKGP_HIP(hipMemsetAsync(Mr, 0, sizeof(double) * ncells * NR * nr, s));
        FKGP_HIP(hipMemsetAsync(Myy, 0, sizeof(double) * ncells, s));
    }
    if (cc) {   // one chunk of a streamed precompute: fold its moments in
        const int64_t nm[3] = {ncells * NB, ncells * NR * nr, ncells};
        double* acc[3] = {cc->acc_w, cc->acc_r, cc->acc_yy};
        const double* loc[3] = {Mw, Mr, Myy};
        for (int i = 0; i < 3; ++i) {
            const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nm[i] + 255) / 256, 4096));
            add_moments<<<nb, 256, 0, s>>>(acc[i], loc[i], nm[i], cc->first ? 1 : 0);
            FKGP_HIP(hipGetLastError());
        }
        if (!cc->last) {
            dev_free(dalloc, block, s);
            return FKGP_OK;
        }
        Mw = cc->acc_w;   // the assembly reads the totals
        Mr = cc->acc_r;
        Myy = cc->acc_yy;
    }

    const KeysTables tab = make_tables(g.interp);
    // --- W^T W: stages over k = d-1 .. 0 ---
    {
        Dims3 cur{{1, 1, 1}};
        for (int k = 0; k < d; ++k) cur.n[k] = g.nc[k];
        Carver c{block + shared_off, 0};
        double* bufA = c.take<double>((size_t)M * NB);
        double* bufB = c.take<double>((size_t)M * NB);
        const double* src = Mw;
        double* dst = bufA;
        for (int k = d - 1; k >= 0; --k) {
            Dims3 nxt = cur;
            nxt.n[k] = g.m[k];
            const int64_t total = (int64_t)nxt.n[0] * nxt.n[1] * nxt.n[2] * (NB / 7);
            const unsigned nbk = (unsigned)((total + 255) / 256 + 7) / 8 * 8;
            if (d == 1)
                assemble_wtw_stage<1><<<nbk, 256, 0, s>>>(src, dst, cur, nxt, k, tab);
            else if (d == 2)
                assemble_wtw_stage<2><<<nbk, 256, 0, s>>>(src, dst, cur, nxt, k, tab);
            else
                assemble_wtw_stage<3><<<nbk, 256, 0, s>>>(src, dst, cur, nxt, k, tab);
            FKGP_HIP(hipGetLastError());
            cur = nxt;
            src = dst;
            dst = (dst == bufA) ? bufB : bufA;
        }
        const int64_t Mpad = (M + kRowTile - 1) / kRowTile * kRowTile;
        dim3 tb(32, 8), tg((unsigned)(Mpad / 32), (unsigned)((NB + 31) / 32));
        if (stats == FKGP_F32)
            transpose_to_dia<float><<<tg, tb, 0, s>>>(src, static_cast<float*>(out.wtw), M, NB,
                                                      out.bmask);
        else
            transpose_to_dia<double><<<tg, tb, 0, s>>>(src, static_cast<double*>(out.wtw), M, NB,
                                                       out.bmask);
        FKGP_HIP(hipGetLastError());
        count_mask_bits<<<1, 256, 0, s>>>(out.bmask, mask_words(M), out.nzblocks);
        FKGP_HIP(hipGetLastError());
        // exact nonzero count: a separate read of the stored matrix (a few
        // thousand counter updates instead of one per wavefront above)
        fkgp_status cs = count_wtw_nonzeros(stats, out.wtw, dia_elems(M, NB), out.nnz, s);
        if (cs != FKGP_OK) return cs;
    }
    // --- W^T y and sketches: stages over k = d-1 .. 0 ---
    {
        Dims3 cur{{1, 1, 1}};
        for (int k = 0; k < d; ++k) cur.n[k] = g.nc[k];
        Carver c{block + shared_off, 0};
        double* bufA = c.take<double>((size_t)M * NR * nr);
        double* bufB = c.take<double>((size_t)M * NR * nr);
        const double* src = Mr;
        int Pin = NR;
        for (int k = d - 1; k >= 0; --k) {
            Dims3 nxt = cur;
            nxt.n[k] = g.m[k];
            const int Pout = Pin / 4;
            const int64_t total = (int64_t)nxt.n[0] * nxt.n[1] * nxt.n[2] * Pout * nr;
            double* target = (src == bufA) ? bufB : bufA;
            assemble_vec_stage<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(src, target, cur, nxt,
                                                                                k, Pout, nr, tab);
            FKGP_HIP(hipGetLastError());
            cur = nxt;
            src = target;
            Pin = Pout;
        }
        // src: [nr][M]
        FKGP_HIP(hipMemcpyAsync(out.wty, src, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
        if (nprobe > 0)
            FKGP_HIP(hipMemcpyAsync(out.sketches, src + M, sizeof(double) * M * nprobe,
                                    hipMemcpyDeviceToDevice, s));
    }
    {
        // the shared region is free again: the assembly and sketch stages
        // that used it are ordered before these launches on the stream
        Carver c{block + shared_off, 0};
        double* part = c.take<double>(256);
        sum_chunks<<<256, 256, 0, s>>>(Myy, ncells, part);
        sum_fixed<<<1, 1024, 0, s>>>(part, 256, out.yty_dev);
        FKGP_HIP(hipGetLastError());
    }
    if (out.keep_cstart) {   // cell bounds (all zero for n = 0)
        FKGP_HIP(hipMemcpyAsync(out.keep_cstart, cstart, sizeof(uint32_t) * ncells,
                                hipMemcpyDeviceToDevice, s));
        FKGP_HIP(hipMemcpyAsync(out.keep_cend, cend, sizeof(uint32_t) * ncells,
                                hipMemcpyDeviceToDevice, s));
    }
    dev_free(dalloc, block, s);
    return FKGP_OK;
}

// ---------------------------------------------------------------------------
// Plain SKI operator on the kept points (Sec. 2.3: W K_G W^T + s2 I applied
// to an n-vector, O(n + m log m) per product).  The points are in cell
// order, so W^T v is the vector assembly of the precompute with y replaced
// by v: per-cell moments sum_p v_p prod_k b3_{q_k}(t_k) (q_k <= 3, one wave per
// cell in 1-D and 2-D, four in 3-D, lanes striding over the cell's points,
// fixed xor-trees across each wave), then the separable stages that turn moment digits into the 4
// stencil offsets of each dimension.  W g gathers the 4^d stencil nodes of
// each point with the Keys weights.
// ---------------------------------------------------------------------------
// Waves per cell of ski_cell_moments: in 3-D the 64 moments are split over
// four waves by the power of the first coordinate (16 accumulators each, so
// the kernel is not held to one wave per SIMD by its registers); the four
// waves read the same points, which the first one brings into the caches.
// (Splitting the points of a 1-D or 2-D cell over four waves was slower:
// most cells hold few points.)
template <int D>
constexpr int ski_waves() { return D == 3 ? 4 : 1; }

template <class Tin, int D>
__global__ __launch_bounds__(64 * ski_waves<D>()) void ski_cell_moments(
    const typename PayloadOf<Tin>::type* __restrict__ pay, const uint32_t* __restrict__ cstart,
    const uint32_t* __restrict__ cend, GridDev g, const double* __restrict__ v,
    double* __restrict__ R) {
    constexpr int NR = ipow_c<D>(4);
    constexpr int NW = ski_waves<D>();
    constexpr int QW = NR / NW;          // moments per wave
    constexpr int KLO = NW > 1 ? 1 : 0;  // first dimension with compile-time digits
    const int64_t cell = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;     // power of the first coordinate when NW > 1
    const uint32_t s0 = cstart[cell], s1 = cend[cell];
    double acc[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) acc[q] = 0.0;
    for (uint32_t i = s0 + lane; i < s1; i += 64) {
        const auto p = pay[i];
        double tq[D][4];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int base;
            double t;
            if (!locate((double)get_slot(p, k), g.g0[k], g.h[k], g.m[k], base, t)) t = 0.0;
            const double sk = 1.0 - t;   // b3_q(t) = t^q (1-t)^(3-q)
            tq[k][0] = sk * sk * sk;
            tq[k][1] = t * sk * sk;
            tq[k][2] = t * t * sk;
            tq[k][3] = t * t * t;
        }
        double lead = v[i];
        if (NW > 1) lead *= wv == 0 ? tq[0][0] : wv == 1 ? tq[0][1] : wv == 2 ? tq[0][2] : tq[0][3];
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            double w = lead;
            int rem = q;
#pragma unroll
            for (int k = D - 1; k >= KLO; --k) {
                w *= tq[k][rem & 3];
                rem >>= 2;
            }
            acc[q] += w;
        }
    }
#pragma unroll
    for (int q = 0; q < QW; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < QW; ++q) R[cell * NR + wv * QW + q] = acc[q];
    }
}

template <class Tin, int D>
__global__ void ski_interp(const typename PayloadOf<Tin>::type* __restrict__ pay, int64_t n,
                           GridDev g, const double* __restrict__ gv,
                           const double* __restrict__ v, double s2, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const auto p = pay[i];
    int base[D];
    double w[D][4];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t;
        if (!locate((double)get_slot(p, k), g.g0[k], g.h[k], g.m[k], base[k], t)) {
            base[k] = 1;   // not reached: the precompute rejected such points
            t = 0.0;
        }
        stencil_weights(g.interp, t, w[k]);
    }
    double acc = 0.0;
    if (D == 1) {
#pragma unroll
        for (int a = 0; a < 4; ++a) acc = fma(w[0][a], gv[base[0] - 1 + a], acc);
    } else if (D == 3) {
        const int64_t m1 = g.m[1], m2 = g.m[2];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double ra = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double r = 0.0;
                const int64_t row =
                    ((int64_t)(base[0] - 1 + a) * m1 + (base[1] - 1 + b)) * m2 + (base[D - 1] - 1);
#pragma unroll
                for (int c = 0; c < 4; ++c) r = fma(w[D - 1][c], gv[row + c], r);
                ra = fma(w[1][b], r, ra);
            }
            acc = fma(w[0][a], ra, acc);
        }
    } else {
        const int64_t m1 = g.m[D - 1];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double r = 0.0;
            const int64_t row = (int64_t)(base[0] - 1 + a) * m1 + (base[D - 1] - 1);
#pragma unroll
            for (int b = 0; b < 4; ++b) r = fma(w[D - 1][b], gv[row + b], r);
            acc = fma(w[0][a], r, acc);
        }
    }
    out[i] = fma(s2, v[i], acc);
}

template <class Tin>
__global__ void ski_extract_y(const typename PayloadOf<Tin>::type* __restrict__ pay, int64_t n,
                              int d, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)get_slot(pay[i], d);
}

}  // namespace

fkgp_status ski_wt(const GridDev& g, fkgp_dtype in, const void* pay, const uint32_t* cstart,
                   const uint32_t* cend, const double* v, double* R, double* T1, double* wtv,
                   hipStream_t s) {
    const int d = g.d;
    int64_t ncells = 1;
    for (int k = 0; k < d; ++k) ncells *= g.nc[k];
    if (d == 1) {
        if (in == FKGP_F32)
            ski_cell_moments<float, 1><<<(unsigned)ncells, 64 * ski_waves<1>(), 0, s>>>(
                static_cast<const float4*>(pay), cstart, cend, g, v, R);
        else
            ski_cell_moments<double, 1><<<(unsigned)ncells, 64 * ski_waves<1>(), 0, s>>>(
                static_cast<const double4*>(pay), cstart, cend, g, v, R);
    } else if (d == 2) {
        if (in == FKGP_F32)
            ski_cell_moments<float, 2><<<(unsigned)ncells, 64 * ski_waves<2>(), 0, s>>>(
                static_cast<const float4*>(pay), cstart, cend, g, v, R);
        else
            ski_cell_moments<double, 2><<<(unsigned)ncells, 64 * ski_waves<2>(), 0, s>>>(
                static_cast<const double4*>(pay), cstart, cend, g, v, R);
    } else {
        if (in == FKGP_F32)
            ski_cell_moments<float, 3><<<(unsigned)ncells, 64 * ski_waves<3>(), 0, s>>>(
                static_cast<const float4*>(pay), cstart, cend, g, v, R);
        else
            ski_cell_moments<double, 3><<<(unsigned)ncells, 64 * ski_waves<3>(), 0, s>>>(
                static_cast<const double4*>(pay), cstart, cend, g, v, R);
    }
    FKGP_HIP(hipGetLastError());
    const KeysTables tab = make_tables(g.interp);
    Dims3 cur{{1, 1, 1}};
    for (int k = 0; k < d; ++k) cur.n[k] = g.nc[k];
    const double* src = R;
    int Pin = d == 1 ? 4 : (d == 2 ? 16 : 64);
    for (int k = d - 1; k >= 0; --k) {
        Dims3 nxt = cur;
        nxt.n[k] = g.m[k];
        const int Pout = Pin / 4;
        const int64_t total = (int64_t)nxt.n[0] * nxt.n[1] * nxt.n[2] * Pout;
        // intermediate stages alternate between the two halves of T1 (the
        // first holds nc0 nc1 m2 x 16 values in 3-D, the second follows it)
        double* target = k == 0 ? wtv : (k == d - 1 ? T1 : T1 + (int64_t)g.nc[0] * g.nc[1] * g.m[2] * 16);
        assemble_vec_stage<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(src, target, cur, nxt,
                                                                            k, Pout, 1, tab);
        FKGP_HIP(hipGetLastError());
        cur = nxt;
        src = target;
        Pin = Pout;
    }
    return FKGP_OK;
}

fkgp_status ski_w(const GridDev& g, fkgp_dtype in, const void* pay, int64_t n,
                  const double* gv, const double* v, double s2, double* out, hipStream_t s) {
    if (n == 0) return FKGP_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (g.d == 1) {
        if (in == FKGP_F32)
            ski_interp<float, 1><<<nb, 256, 0, s>>>(static_cast<const float4*>(pay), n, g, gv, v,
                                                    s2, out);
        else
            ski_interp<double, 1><<<nb, 256, 0, s>>>(static_cast<const double4*>(pay), n, g, gv,
                                                     v, s2, out);
    } else if (g.d == 2) {
        if (in == FKGP_F32)
            ski_interp<float, 2><<<nb, 256, 0, s>>>(static_cast<const float4*>(pay), n, g, gv, v,
                                                    s2, out);
        else
            ski_interp<double, 2><<<nb, 256, 0, s>>>(static_cast<const double4*>(pay), n, g, gv,
                                                     v, s2, out);
    } else {
        if (in == FKGP_F32)
            ski_interp<float, 3><<<nb, 256, 0, s>>>(static_cast<const float4*>(pay), n, g, gv, v,
                                                    s2, out);
        else
            ski_interp<double, 3><<<nb, 256, 0, s>>>(static_cast<const double4*>(pay), n, g, gv,
                                                     v, s2, out);
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status ski_y(const GridDev& g, fkgp_dtype in, const void* pay, int64_t n, double* y,
                  hipStream_t s) {
    if (n == 0) return FKGP_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (in == FKGP_F32)
        ski_extract_y<float><<<nb, 256, 0, s>>>(static_cast<const float4*>(pay), n, g.d, y);
    else
        ski_extract_y<double><<<nb, 256, 0, s>>>(static_cast<const double4*>(pay), n, g.d, y);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

namespace {
template <class T>
__global__ __launch_bounds__(256) void count_nonzero(const T* __restrict__ a, int64_t n,
                                                     unsigned long long* __restrict__ out) {
    // 16-byte loads over the bulk (the array is 256-byte aligned), then the tail
    constexpr int V = 16 / sizeof(T);
    struct alignas(16) Vec { T v[V]; };
    const Vec* av = reinterpret_cast<const Vec*>(a);
    const int64_t nv = n / V;
    unsigned cnt = 0u;
    // four independent 16-byte loads in flight per thread and step
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x; i0 < nv; i0 += 4 * stride) {
        Vec x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < nv) x[u] = av[i];
            else
#pragma unroll
                for (int j = 0; j < V; ++j) x[u].v[j] = T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < V; ++j) cnt += x[u].v[j] != T(0);
    }
    for (int64_t i = nv * V + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        cnt += a[i] != T(0);
    // one counter update per workgroup: updates of one address serialise
    // (about 15 ns each), so their number, not the read, would set the time
    __shared__ unsigned wsum[4];
    for (int off = 32; off > 0; off >>= 1) cnt += (unsigned)__shfl_xor((int)cnt, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot =
            (unsigned long long)wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (tot) atomicAdd(out, tot);
    }
}
}  // namespace

fkgp_status count_wtw_nonzeros(fkgp_dtype dt, const void* A, int64_t elems,
                               unsigned long long* out, hipStream_t s) {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((elems + 255) / 256, 1024));
    if (dt == FKGP_F32)
        count_nonzero<float><<<nb, 256, 0, s>>>(static_cast<const float*>(A), elems, out);
    else
        count_nonzero<double><<<nb, 256, 0, s>>>(static_cast<const double*>(A), elems, out);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

fkgp_status run_precompute(const GridDev& g, const void* const* x, const void* y, int64_t n,
                           fkgp_dtype in, fkgp_dtype stats, int nprobe, uint64_t seed,
                           const StatsOut& out, unsigned long long* bad, hipStream_t s,
                           const ChunkCtl* cc) {
    if (in == FKGP_F32)
        return precompute_typed<float>(g, x, y, n, stats, nprobe, seed, out, bad, s, cc);
    return precompute_typed<double>(g, x, y, n, stats, nprobe, seed, out, bad, s, cc);
}

}  // namespace fkgp
