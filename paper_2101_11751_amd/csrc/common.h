// Internal declarations shared by the HIP translation units of libfkgp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include <string>

#include "../../include/fkgp.h"

namespace fkgp {

// Grid as seen by the kernels.  Dimensions beyond d have m = 1, nc = 1.
struct GridDev {
    int d;
    int m[3];       // nodes per dimension
    int nc[3];      // cells per dimension (m - 3)
    double g0[3];   // origin
    double h[3];    // spacing
    int interp;     // 0: Keys cubic convolution, 1: linear interpolation
};

// Weights of the nodes i-1, i, i+1, i+2 of a point at fractional offset t in
// [0, 1] from node i: Keys' cubic convolution (a = -1/2; Sec. 3, Fig. 1), or
// linear interpolation between i and i+1 (Sec. 2.3: 2^d nonzeros per row of
// W), kept in the same four-node frame with zero outer weights.
__device__ inline void stencil_weights(int interp, double t, double w[4]) {
    if (interp == 1) {
        w[0] = 0.0;
        w[1] = 1.0 - t;
        w[2] = t;
        w[3] = 0.0;
        return;
    }
    const double t2 = t * t, t3 = t2 * t;
    w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
    w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
    w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
    w[3] = 0.5 * (t3 - t2);
}

constexpr int kMaxProbes = 31;

// Workgroups are dispatched round-robin over the 8 XCDs (block b to XCD
// b % 8), each with its own L2.  xcd_block() renumbers the blocks so that
// every XCD runs one contiguous range of logical blocks: neighbouring blocks
// that share cache lines (the interleaved lines of a strided pass) then share
// an L2 instead of fetching the same lines on different dies.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / kXcds, r = nb % kXcds, x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Storage of W^T W: row-tiled stencil-diagonal layout [tile][o][kRowTile],
// tile = j / kRowTile, so the entries one workgroup of the banded product
// needs (kRowTile rows x 7^d offsets) are one contiguous block.  Rows past
// the last grid node in the final tile are zero.
constexpr int kRowTile = 256;

__host__ __device__ inline int64_t dia_index(int64_t j, int o, int NB) {
    return ((j / kRowTile) * NB + o) * kRowTile + (j % kRowTile);
}

inline int64_t dia_elems(int64_t M, int NB) {
    return ((M + kRowTile - 1) / kRowTile) * NB * kRowTile;
}

// Block occupancy of the stored W^T W.  A block is one 64-row wavefront
// chunk w of a row tile times one offset slab a: the 49 offsets sharing o_0
// for d = 3 (a = o / 49), all 7^d offsets for d <= 2 (a = 0).  Word `tile`
// of the mask has bit w * kMaskSlabs + a set iff the block holds a nonzero
// stored entry; the banded product skips the loads of the other blocks (the
// points need not fill the grid's bounding box: a cylinder of points leaves
// whole wavefront chunks of W^T W zero).
constexpr int kWaveRows = 64;
constexpr int kMaskSlabs = 7;
inline int64_t mask_words(int64_t M) { return (M + kRowTile - 1) / kRowTile; }
// entries per row of one slab: 49 for d >= 2, 7 for d = 1 (slab = o / 49)
__host__ __device__ inline int mask_slab_width(int d) { return d == 1 ? 7 : 49; }

// ---- CG scalar state (capi.hip loops, fused epilogues in ops.hip) ----------
struct CgState {
    double rho;     // ||r_k||^2 in n-space (= u^T r_hat)
    double sz;      // s^T z
    double alpha;
    double beta;
    double eps;     // stop when rho <= eps
    double bnorm2;  // ||b||^2
    int done;
    int iters;
};

enum FinOp { FIN_INIT = 0, FIN_INIT_RHS = 1, FIN_RHO = 2, FIN_SZ = 3 };

// Scalar step of the CG loop once the dot product t of `op` is known.
__device__ inline void cg_state_update(CgState* st, double t, int op) {
    if (op == FIN_INIT || op == FIN_INIT_RHS) {
        st->rho = t;
        st->beta = 0.0;
        st->iters = 0;
        if (op == FIN_INIT_RHS) {
            st->bnorm2 = t;
            st->eps = st->eps * t;   // eps held tol^2 on entry
        }
        st->done = (t <= st->eps) ? 1 : 0;
    } else if (op == FIN_RHO) {
        st->iters += 1;
        if (!(t > st->eps)) {
            st->done = 1;   // converged (or NaN: stop)
            st->rho = t;
            return;
        }
        st->beta = t / st->rho;
        st->rho = t;
    } else {
        st->sz = t;
        st->alpha = st->rho / t;
        if (!isfinite(st->alpha)) st->done = 2;
    }
}

// Reduction finished by the last workgroup of a launch: every workgroup
// publishes its partial, then takes a ticket; the one holding the last
// ticket sums the partials in index order (the same order as a separate
// one-block reduction, so the result is deterministic) and applies the CG
// scalar step.  Partials and tickets use device-scope atomics, which are
// coherent across the XCDs' L2 caches without the L2 write-back a
// device-scope fence costs; the partial's exchange returns before the
// ticket is taken, so a workgroup holding the last ticket sees every
// partial.  `ticket` is zero between launches (the last workgroup resets it).
struct LastBlockRed {
    double* partials;
    unsigned* ticket;
    CgState* st;
    int op;
};

// Called by all threads of a 256-thread workgroup; `part` is the
// workgroup's partial (significant in thread 0).  sh: 256 doubles of LDS,
// free for reuse.
__device__ inline void last_block_finish(const LastBlockRed& lb, double part, double* sh) {
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        const unsigned long long old = __hip_atomic_exchange(
            reinterpret_cast<unsigned long long*>(lb.partials) + blockIdx.x,
            (unsigned long long)__double_as_longlong(part), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        asm volatile("" : : "v"(old) : "memory");   // the exchange has returned
        const unsigned t =
            __hip_atomic_fetch_add(lb.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = t == gridDim.x - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    double acc = 0.0;
    for (unsigned i = threadIdx.x; i < gridDim.x; i += 256)
        acc += __longlong_as_double((long long)__hip_atomic_load(
            reinterpret_cast<unsigned long long*>(lb.partials) + i, __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT));
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cg_state_update(lb.st, sh[0], lb.op);
        __hip_atomic_store(lb.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// CG direction update fused into the store of the last K_G line pass:
// v = s K u + s2 x is consumed in place (never stored): s = u + beta s,
// z = v + beta z, p = r + beta p (p optional), partial s.z, and the last
// workgroup finishes s.z (FIN_SZ: alpha).  u has the operator dtype.
struct CgStep2 {
    const CgState* st;
    double* s;
    double* z;
    double* p;
    const double* r;
    const void* u;
    LastBlockRed lb;
};

// ---- error plumbing -------------------------------------------------------
void set_error(const std::string& msg);
fkgp_status hip_fail(hipError_t e, const char* what);

#define FKGP_HIP(call)                                           \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::fkgp::hip_fail(e_, #call); \
    } while (0)

// ---- device buffers -------------------------------------------------------
// Device memory of the library comes from the caller's allocator when one is
// set (fkgp_set_allocator), else from stream-ordered allocations of the
// device's default pool.  Each allocation is freed through the allocator
// that made it: callers keep the DevAlloc they allocated with.
struct DevAlloc {
    void* (*alloc)(size_t bytes, void* stream, void* ctx) = nullptr;
    void (*free)(void* ptr, void* stream, void* ctx) = nullptr;
    void* ctx = nullptr;
};
DevAlloc current_alloc();
hipError_t dev_malloc(const DevAlloc& a, void** p, size_t bytes, hipStream_t s);
void dev_free(const DevAlloc& a, void* p, hipStream_t s);

template <class T>
inline hipError_t alloc_async(const DevAlloc& a, T** p, size_t count, hipStream_t s) {
    if (count == 0) count = 1;
    return dev_malloc(a, reinterpret_cast<void**>(p), count * sizeof(T), s);
}

// ---- precompute (precompute.hip) -------------------------------------------
struct StatsOut {
    void* wtw;          // row-tiled stencil-diagonal layout, stats dtype
    double* wty;        // [M]
    double* sketches;   // [nprobe][M] or null
    double* yty_dev;    // scalar
    uint32_t* bmask;    // [mask_words(M)] block occupancy, zeroed by the caller
    unsigned long long* nzblocks;   // number of set mask bits (written last)
    unsigned long long* nnz;        // nonzero stored entries of W^T W, zeroed by the caller
    // optional (d <= 2): copies of the points in cell order (payload of the
    // input dtype: coordinates, y, original index) and the cell bounds
    void* keep_pay;
    uint32_t* keep_cstart;
    uint32_t* keep_cend;
};

// Plain SKI operator pieces on kept points (precompute.hip).
// wtv[M] = W^T v for v (n doubles, cell order); R: ncells * 4^d and
// T1: M * (1, 4, 20 for d = 1, 2, 3) doubles of scratch.
fkgp_status ski_wt(const GridDev& g, fkgp_dtype in, const void* pay, const uint32_t* cstart,
                   const uint32_t* cend, const double* v, double* R, double* T1, double* wtv,
                   hipStream_t s);
// out = W gv + s2 v (n doubles, cell order), gv on the grid.
fkgp_status ski_w(const GridDev& g, fkgp_dtype in, const void* pay, int64_t n,
                  const double* gv, const double* v, double s2, double* out, hipStream_t s);
// y of the kept points (cell order).
fkgp_status ski_y(const GridDev& g, fkgp_dtype in, const void* pay, int64_t n, double* y,
                  hipStream_t s);

// One chunk of a streamed precompute: the chunk's per-cell moments are added
// to the running totals (first: copied); only the last chunk assembles the
// statistics (from the totals).  idx_base: global index of the chunk's first
// point (out-of-grid reports).
struct ChunkCtl {
    double* acc_w;    // [ncells * 7^d]
    double* acc_r;    // [ncells * 4^d]
    double* acc_yy;   // [ncells]
    int first, last;
    int64_t idx_base;
};

fkgp_status run_precompute(const GridDev& g, const void* const* x, const void* y,
                           int64_t n, fkgp_dtype in, fkgp_dtype stats,
                           int nprobe, uint64_t seed, const StatsOut& out,
                           unsigned long long* bad_dev, hipStream_t s,
                           const ChunkCtl* cc = nullptr);

// *out += number of nonzero entries among the first `elems` of A (stats dtype).
fkgp_status count_wtw_nonzeros(fkgp_dtype dt, const void* A, int64_t elems,
                               unsigned long long* out, hipStream_t s);

// ---- operators (ops.hip) -------------------------------------------------
// Longest circulant handled by the register-resident line FFT, and by the
// four-step path (grid dimensions up to 65536 nodes; the batched solver's
// passes up to 8192).
constexpr int kMaxRegLog2 = 11;
// Dimensions with at most kFewLines lines per vector and circulants of at
// least 2^kFewLinesMinLog2 points also take the four-step path.
constexpr int kFewLinesMinLog2 = 10;
constexpr int64_t kFewLines = 64;
constexpr int kMaxLineLog2 = 17;
constexpr int kMaxBatchLineLog2 = 14;
// Spectra of circulants up to 2^kMaxDftLog2 points may be direct FP64 sums;
// longer ones, and four-step layouts from 2^12 points when the scratch is
// there, come from a forward four-step FFT of the embedded column.
constexpr int kMaxDftLog2 = 14;
// Workgroups (each with its own L-point complex scratch) of a four-step pass.
constexpr int kLongWGs = 256;

// Split of a long circulant length L = 2^lg1 * 2^lg2 for the four-step path.
__host__ __device__ inline void long_split(int log2L, int& lg1, int& lg2) {
    lg1 = log2L / 2;
    lg2 = log2L - lg1;
}

struct Spectra {
    int L[3];           // circulant length per dim (power of two)
    int log2L[3];
    // [L], scaled by 1/L, stats dtype: bit-reversed order for the register
    // line FFT; for long lines (log2L > kMaxRegLog2) the four-step order
    // lam[p1 * L2 + p2] = lambda[bitrev(p1) + L1 * bitrev(p2)] / L.
    void* lam[3];
    void* tw[3];        // twiddles exp(-2 pi i t / L), t < L/2, complex stats dtype
    void* scr[3];       // long lines: kLongWGs * L complex scratch, else null
    int lg1[3];         // four-step split of dim k (0: register order)
    // 3-D grids with m_0 <= 128 whose two inner dimensions form small slabs
    // (m_1 <= 128, m_2 <= 64, m_1 m_2 <= 4096): the kernel's columns c[j],
    // j < m_k, of all three dimensions (dtype of the spectra), applied as
    // dense Toeplitz factors (a slab pass for dimensions 1 and 2, a column
    // pass for dimension 0); null otherwise
    void* col[3];
};

int circulant_log2(int m);
// Builds lam[k] for dimension k from the column of the 1-D kernel `kind`
// (fkgp_kernel; deriv: its derivative in log l).  Runs on the device in
// FP64: direct DFT sums, or (log2L > kMaxDftLog2) a four-step FFT through
// `scr` (at least L FP64 complex values).
fkgp_status build_spectrum(const GridDev& g, int k, double ell, bool deriv, int kind,
                           fkgp_dtype dt, void* lam, int log2L, int lg1, void* scr,
                           hipStream_t s);
fkgp_status build_twiddles(int log2L, fkgp_dtype dt, void* tw, hipStream_t s);
// Grids whose dimensions 1 and 2 are applied by the dense Toeplitz slab pass,
// and the column it needs: c[j] = k(j h / l) (or its derivative in log l),
// j < m_k.
bool toeplitz_slab_applies(const GridDev& g);
fkgp_status build_toeplitz_col(const GridDev& g, int k, double ell, bool deriv, int kind,
                               fkgp_dtype dt, void* col, hipStream_t s);

// y = scale * (T_0 (x) .. (x) T_{d-1}) x (+ add_coef * addv), batched over k
// vectors of length M; all arrays in dtype dt.  `work` holds M*k elements.
fkgp_status kg_apply(const GridDev& g, const Spectra& sp, fkgp_dtype dt,
                     const void* x, void* y, int k, double scale,
                     const void* addv, double add_coef, void* work,
                     hipStream_t s);

// u = A x (A: [7^d][M] offset-major), x padded by `halo` elements each side.
fkgp_status spmv_dia(const GridDev& g, fkgp_dtype dt, const void* A,
                     const void* xpad, void* u, int k, int64_t halo,
                     hipStream_t s);
fkgp_status spmv_dia_skip(const GridDev& g, fkgp_dtype dt, const void* A, const void* xpad,
                          void* u, int k, int64_t halo, const int* skip, hipStream_t s);
fkgp_status spmv_dia_f32a_f64x(const GridDev& g, const void* A, const double* xpad, double* u,
                               int k, int64_t halo, hipStream_t s);
fkgp_status kg_apply_skip(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x,
                          void* y, int k, double scale, const void* addv, double add_coef,
                          const int* skip, hipStream_t s);
// As kg_apply_skip for one vector, with the CG direction update fused into
// the last pass when that pass uses the register line FFT (*fused = true:
// y holds intermediate values only).  Otherwise y is written and *fused is
// false.  fuse->lb.partials needs kg_last_pass_blocks(g) entries.
fkgp_status kg_apply_fused(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x,
                           void* y, double scale, const void* addv, double add_coef,
                           const int* skip, const CgStep2& fuse, bool* fused, hipStream_t s);
int64_t kg_last_pass_blocks(const GridDev& g);
// dotp (optional, k == 1): per-block partials of sum_j u_j x_j; *nparts gets
// their count (0 if the path used writes none).
// lb (optional, with dotp): the last workgroup also finishes the dot
// product (partials = dotp) and applies the CG scalar step lb.op; *nparts
// is then the number of partials and the reduction is done.
// bmask (optional): the block occupancy of A; blocks without a set bit are
// not read (their entries are zero, so the result is the same).
fkgp_status spmv_dia_any(const GridDev& g, fkgp_dtype dta, fkgp_dtype dtx, const void* A,
                         const uint32_t* bmask, const void* xpad, void* u, int k,
                         int64_t halo, const int* skip,
                         hipStream_t s, double* dotp = nullptr, int* nparts = nullptr,
                         const LastBlockRed* lb = nullptr);
int64_t dia_halo(const GridDev& g);
// Upper bound on the dot partials spmv_dia_any writes (one per row tile).
int64_t spmv_dot_parts(const GridDev& g);

// G[i] (M doubles each, zeroed by the caller) = interpolation weights of
// query point i on the grid; out-of-grid points set *bad (min index).
fkgp_status query_weights(const GridDev& g, const void* const* xq, int64_t nq, fkgp_dtype in,
                          double* G, unsigned long long* bad, hipStream_t s);
// Stencils of nq query points: first[i][3] (first node per dimension) and
// w[i][3][4] (Keys weights); out-of-grid points set *bad (min index).
fkgp_status query_stencils(const GridDev& g, const void* const* xq, int64_t nq, fkgp_dtype in,
                           int* first, double* w, unsigned long long* bad, hipStream_t s);
// Rank-k covariance queries: U [nq][k] and partials (love_partials_doubles)
// are workspace; Ct [M][k]; cov [nq][nq] = w_i^T K_G w_j - U_i . U_j.
size_t love_partials_doubles(int nq, int k, int* nb_out);
fkgp_status love_query(const GridDev& g, int kind, const double* ell, double so,
                       const double* Ct, int k, const int* first, const double* w, int nq,
                       double* U, double* partials, double* cov, hipStream_t s);
fkgp_status interpolate_points(const GridDev& g, const double* mu,
                               const void* const* xq, int64_t nq,
                               fkgp_dtype in, double* out,
                               unsigned long long* bad_dev, hipStream_t s);

// ---- batched factorized CG over many problems (batch.hip) ---------------
constexpr int kMaxLanczos = 64;   // CG coefficients kept per right-hand side
constexpr int kBatchMaxRhs = 8;   // right-hand sides per work item: 2, 4 or 8
// Longest circulant the batched solver convolves with the register line FFT
// (longer ones take the four-step path, which keeps its registers low).
constexpr int kBatchRegMaxLog2 = 8;

// State of one factorized CG from x_0 = 0 (r = W r_hat + c_r b, ...).
struct PState {
    double rho, cr, cp, cx, pb, alpha, beta, eps;
    double bb;   // ||b||^2 of the right-hand side b (n for a probe)
    int done, iters;
};

template <class T>
struct cplx;   // complex pair {re, im} (line FFTs)

struct BatchProb {
    int d;
    int m[2];
    int64_t M, halo;
    int NB;
    int log2L[2];
    int a_f32;                 // stored W^T W is FP32 (else FP64)
    const void* A;             // row-tiled stencil-diagonal W^T W
    double so, s2;
    const double* bh;          // [nrhs][M] W^T b
    const double* kb;          // [nrhs][M] K_G W^T b
    const double* bnorm2;      // [nrhs] ||b||^2
    const double* r0y;         // [M] r_hat_0 = -K_G W^T y / s2 of the data right-hand
                               // side (slot 0), solved from x_0 = y / s2 with the
                               // residual in the span of W; null: slot 0 from x_0 = 0
    const void* tw[2];         // FP64 twiddles per dimension
    const double* lam[2];      // FP64 spectra per dimension
    const double* col[2];      // 2-D, both m_k <= kBatchTzMax: FP64 kernel columns
                               // c[j], j < m_k (dense Toeplitz line passes); else null
    double* alphas;            // [nrhs][kMaxLanczos]
    double* betas;             // [nrhs][kMaxLanczos]
    PState* ps;                // [nrhs]
    double* wx;                // [nrhs][M] W^T x on exit
};

struct BatchItem {
    int prob, r0, nr;
    double* work;              // batch_work_doubles(M, halo, NR) doubles
    cplx<double>* yscr;        // L complex (longest four-step line), or null
};

// Stride between the padded r_hat vectors of a work item (8 spare zeros past
// the halo: the four-row product reads up to 3 entries beyond the last row).
__host__ __device__ inline int64_t batch_rhat_stride(int64_t M, int64_t halo) {
    return M + 2 * halo + 8;
}
size_t batch_work_doubles(int64_t M, int64_t halo, int nr);
// 2-D problems with both dimensions at most kBatchTzMax nodes apply K_G in
// the batched kernel as two dense Toeplitz line passes (kBatchTzNJ
// consecutive outputs per lane, lines on the lanes); longer lines and 1-D
// problems use the line FFT.
constexpr int kBatchTzMax = 128;
constexpr int kBatchTzNJ = 8;
inline bool batch_tz(int d, const int* m) {
    return d == 2 && m[0] <= kBatchTzMax && m[1] <= kBatchTzMax;
}
// LDS (doubles) of those passes: both reflected columns (2 m + 2 NJ each)
// and the staging block, 64 lines of odd stride (pass along dimension 1) or
// m_0 rows of 64 columns (pass along dimension 0).
inline int64_t batch_tz_doubles(const int* m) {
    const int64_t ext = 2 * (int64_t)m[0] + 2 * kBatchTzNJ + 2 * (int64_t)m[1] + 2 * kBatchTzNJ;
    return ext + 64 * std::max<int64_t>(m[1] | 1, m[0]);
}
// LDS (doubles) of the batched kernel's staged banded product for nr
// right-hand sides and `block` threads: a tile of 2 block rows plus the
// stencil margin 3 m1 + 3 (2-D) or 3 (1-D) on both sides, per right-hand
// side.  It shares the LDS past the spectra with the strided-pass transpose.
__host__ __device__ inline int64_t batch_stage_doubles(int d, int m1, int nr, int block) {
    const int64_t h = (d == 1 ? 0 : 3 * (int64_t)m1) + 3;
    return (int64_t)nr * (2 * block + 2 * h);
}
// Dynamic LDS of the batched kernel for one problem (spectra, transpose).
size_t batch_lds_bytes(int d, const int* m, const int* log2L);
fkgp_status launch_batch_cg(const BatchProb* probs_dev, const BatchItem* items_dev, int nitems,
                            size_t lds, double tol, int maxiter, int nr, int block,
                            hipStream_t s);

fkgp_status dia_to_canonical(const GridDev& g, fkgp_dtype dt, const void* A,
                             void* out, hipStream_t s);

}  // namespace fkgp
