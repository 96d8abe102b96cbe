// C-ABI of libfkgp: handle management, argument validation, and the
// device-resident factorized conjugate-gradient loop.
//
// The posterior mean uses the simplified efficiently-factorized CG of the
// appendix (initial residual in the span of W): one operator application
// B(x) = ((K_G W^T W + s2 I) x, W^T W x) per iteration, FP64 vectors and
// scalars, B in the handle's stats dtype.  Scalars live on the device; every
// kernel of an iteration reads them there and returns early once the stop
// test has fired, so the host only polls a flag every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

struct fkgp_handle {
    fkgp::GridDev g;
    int64_t n = 0;
    int64_t M = 0;
    int NB = 0;
    fkgp_dtype dt = FKGP_F32;
    int nprobe = 0;
    uint64_t seed = 0;
    void* A = nullptr;          // [NB][M] stats dtype
    double* wty = nullptr;      // [M]
    double* sketches = nullptr; // [nprobe][M]
    double* yty_dev = nullptr;  // [4]: y^T y, the out-of-grid flag, the
                                // number of nonzero blocks of W^T W (bits)
    uint32_t* bmask = nullptr;  // [mask_words(M)] block occupancy of W^T W
    double yty = 0.0;
    int64_t nzblocks = 0;
    int64_t nnz = 0;            // nonzero stored entries of W^T W
    // points kept in cell order (keep_points): payload of dtype in_dt
    // (coordinates, y, original index) and the cell bounds
    void* pts_block = nullptr;
    void* pay = nullptr;
    uint32_t* cstart = nullptr;
    uint32_t* cend = nullptr;
    fkgp_dtype in_dt = FKGP_F32;
    void* block = nullptr;      // one pool allocation holding the arrays above
    fkgp::DevAlloc alloc;       // the allocator block and pts_block came from
};

// Rank-k covariance cache: C^T [M][k] (row j = C_j over the rank), the
// hypers the prior term needs, and the Lanczos tridiagonal for inspection.
struct fkgp_love {
    fkgp::GridDev g;
    int kind = 0;
    double ell[3] = {1.0, 1.0, 1.0};
    double so = 1.0;
    int k = 0;
    int dev = 0;
    double* Ct = nullptr;
    fkgp::DevAlloc alloc;   // the allocator Ct came from
    std::vector<double> alpha, beta, d;
};

// Workspace of fkgp_solve_noalloc: one copy per GPU, held until the process
// ends.  Host code must not use this name as a device address (it is a host
// stand-in); the device address comes from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace fkgp {

fkgp_status kg_apply_skip(const GridDev& g, const Spectra& sp, fkgp_dtype dt, const void* x,
                          void* y, int k, double scale, const void* addv, double add_coef,
                          const int* skip, hipStream_t s);
fkgp_status spmv_dia_skip(const GridDev& g, fkgp_dtype dt, const void* A, const void* xpad,
                          void* u, int k, int64_t halo, const int* skip, hipStream_t s);

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
std::string last_error_copy() { return g_last_error; }

fkgp_status hip_fail(hipError_t e, const char* what) {
    set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? FKGP_ENOMEM : FKGP_EDEVICE;
}

namespace {

// Scratch allocations released (stream-ordered) when the scope ends.
// Memory freed to the device's default pool stays cached in it (release
// threshold raised once per device), so repeated calls reuse mapped memory
// instead of mapping fresh pages each time.
std::mutex g_pool_mu;
bool g_pool_ready[64] = {};

void ensure_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_ready[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    g_pool_ready[dev] = true;
}

}  // namespace

namespace {
std::mutex g_alloc_mu;
DevAlloc g_alloc;
}  // namespace

DevAlloc current_alloc() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void set_alloc(const DevAlloc& a) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = a;
}

hipError_t dev_malloc(const DevAlloc& a, void** p, size_t bytes, hipStream_t s) {
    if (!a.alloc) return hipMallocAsync(p, bytes, s);
    *p = a.alloc(bytes, static_cast<void*>(s), a.ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(const DevAlloc& a, void* p, hipStream_t s) {
    if (!p) return;
    if (!a.alloc)
        (void)hipFreeAsync(p, s);
    else
        a.free(p, static_cast<void*>(s), a.ctx);
}

namespace {

// Arena mode (base != nullptr): pieces are carved, 256-byte aligned, from a
// caller-provided device buffer of `cap` bytes and nothing is allocated or
// freed; a request past the end fails with hipErrorOutOfMemory.
struct Scratch {
    hipStream_t s;
    DevAlloc a;
    std::vector<void*> ptrs;
    unsigned char* arena = nullptr;
    size_t cap = 0, off = 0;
    explicit Scratch(hipStream_t st) : s(st), a(current_alloc()) { ensure_pool(); }
    Scratch(hipStream_t st, unsigned char* base, size_t capacity)
        : s(st), arena(base), cap(capacity) {}
    ~Scratch() {
        for (void* p : ptrs) dev_free(a, p, s);
    }
    template <class T>
    hipError_t get(T** p, size_t count) {
        if (arena) {
            const size_t b = ((count ? count : 1) * sizeof(T) + 255) & ~size_t(255);
            if (off + b > cap) return hipErrorOutOfMemory;
            *p = reinterpret_cast<T*>(arena + off);
            off += b;
            return hipSuccess;
        }
        hipError_t e = alloc_async(a, p, count, s);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

size_t dsize(fkgp_dtype dt) { return dt == FKGP_F32 ? 4 : 8; }

// ---------------------------------------------------------------------------
// CG kernels (FP64 vectors and scalars).
// ---------------------------------------------------------------------------


constexpr int kRedBlock = 256;
constexpr int kRedMaxBlocks = 1024;

int red_blocks(int64_t M) {
    int64_t b = (M + 4 * kRedBlock - 1) / (4 * kRedBlock);
    if (b < 1) b = 1;
    if (b > kRedMaxBlocks) b = kRedMaxBlocks;
    return (int)b;
}

// Sum of v over the workgroup (kRedBlock threads, fixed tree order).  The
// result is read from sh[0] by every thread with no barrier after it, so
// only thread 0 may use it when another block_sum on the same `sh` follows
// (the next call's first store can overwrite sh[0] before a slower thread
// has read it); every caller here consumes it in thread 0.
__device__ inline double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

template <class TU>
__global__ __launch_bounds__(kRedBlock) void dot_partial(const TU* __restrict__ a,
                                                         const double* __restrict__ b, int64_t M,
                                                         double* __restrict__ partials,
                                                         const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock)
        acc = fma((double)a[i], b[i], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedBlock) void finalize(const double* __restrict__ partials, int nb,
                                                      CgState* st, int op) {
    __shared__ double sh[kRedBlock];
    if (op >= FIN_RHO && st->done) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedBlock) acc += partials[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) cg_state_update(st, t, op);
}

// xd += alpha s; r -= alpha z; rpad = (T) r
template <class T>
__global__ void cg_step1(const CgState* __restrict__ st, double* __restrict__ xd,
                         double* __restrict__ r, const double* __restrict__ s,
                         const double* __restrict__ z, T* __restrict__ rpad, int64_t M) {
    if (st->done) return;
    const double a = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        xd[i] = fma(a, s[i], xd[i]);
        const double rn = fma(-a, z[i], r[i]);
        r[i] = rn;
        rpad[i] = (T)rn;
    }
}

// s = u + beta s; z = v + beta z; partial s.z
template <class T>
__global__ __launch_bounds__(kRedBlock) void cg_step2(const CgState* __restrict__ st,
                                                      double* __restrict__ s,
                                                      double* __restrict__ z,
                                                      const T* __restrict__ u,
                                                      const T* __restrict__ v, int64_t M,
                                                      double* __restrict__ partials) {
    if (st->done) return;
    __shared__ double sh[kRedBlock];
    const double b = st->beta;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock) {
        const double sn = fma(b, s[i], (double)u[i]);
        const double zn = fma(b, z[i], (double)v[i]);
        s[i] = sn;
        z[i] = zn;
        acc = fma(sn, zn, acc);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <class TI, class TO>
__global__ void convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t M, double scale) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (TO)(scale * (double)in[i]);
}

// out = a + c * b  (FP64)
__global__ void axpy_out(const double* __restrict__ a, const double* __restrict__ b, double c,
                         double* __restrict__ out, int64_t M) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = fma(c, b[i], a[i]);
}

unsigned ew_grid(int64_t M) {
    int64_t b = (M + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <class TI, class TO>
hipError_t launch_convert(const TI* in, TO* out, int64_t M, double scale, hipStream_t s) {
    convert<TI, TO><<<ew_grid(M), 256, 0, s>>>(in, out, M, scale);
    return hipGetLastError();
}

hipError_t convert_any(const void* in, fkgp_dtype din, void* out, fkgp_dtype dout, int64_t M,
                       double scale, hipStream_t s) {
    if (din == FKGP_F64 && dout == FKGP_F32)
        return launch_convert(static_cast<const double*>(in), static_cast<float*>(out), M, scale, s);
    if (din == FKGP_F64 && dout == FKGP_F64)
        return launch_convert(static_cast<const double*>(in), static_cast<double*>(out), M, scale, s);
    if (din == FKGP_F32 && dout == FKGP_F64)
        return launch_convert(static_cast<const float*>(in), static_cast<double*>(out), M, scale, s);
    return launch_convert(static_cast<const float*>(in), static_cast<float*>(out), M, scale, s);
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
fkgp_status grid_from_abi(const fkgp_grid* gr, GridDev& g, int64_t& M) {
    g.interp = 0;
    if (!gr) {
        set_error("grid is NULL");
        return FKGP_EINVAL;
    }
    if (gr->d < 1 || gr->d > 3) {
        set_error("grid.d must be 1, 2 or 3");
        return FKGP_EINVAL;
    }
    std::memset(&g, 0, sizeof(g));
    g.d = gr->d;
    M = 1;
    int64_t cells = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < gr->d) {
            if (gr->m[k] < 4 || gr->m[k] > (1 << 20)) {
                set_error("grid.m[k] must be in [4, 2^20]");
                return FKGP_EINVAL;
            }
            if (!(gr->spacing[k] > 0.0) || !std::isfinite(gr->spacing[k]) ||
                !std::isfinite(gr->origin[k])) {
                set_error("grid spacing must be positive and finite, origin finite");
                return FKGP_EINVAL;
            }
            g.m[k] = (int)gr->m[k];
            g.nc[k] = g.m[k] - 3;
            g.g0[k] = gr->origin[k];
            g.h[k] = gr->spacing[k];
            M *= g.m[k];
            cells *= g.nc[k];
        } else {
            g.m[k] = 1;
            g.nc[k] = 1;
            g.h[k] = 1.0;
        }
    }
    if (M > (int64_t(1) << 30) || cells >= (int64_t(1) << 30)) {
        set_error("grid too large (more than 2^30 nodes)");
        return FKGP_EINVAL;
    }
    return FKGP_OK;
}

fkgp_status check_hypers(const fkgp_handle* h, const fkgp_hypers* hyp) {
    if (!hyp) {
        set_error("hypers is NULL");
        return FKGP_EINVAL;
    }
    for (int k = 0; k < h->g.d; ++k)
        if (!(hyp->lengthscale[k] > 0.0) || !std::isfinite(hyp->lengthscale[k])) {
            set_error("lengthscales must be positive and finite");
            return FKGP_EINVAL;
        }
    if (!(hyp->outputscale > 0.0) || !std::isfinite(hyp->outputscale) ||
        !(hyp->noise_std > 0.0) || !std::isfinite(hyp->noise_std)) {
        set_error("outputscale and noise_std must be positive and finite");
        return FKGP_EINVAL;
    }
    if (hyp->kernel < FKGP_KERNEL_SE || hyp->kernel > FKGP_KERNEL_MATERN52) {
        set_error("kernel must be one of the fkgp_kernel values");
        return FKGP_EINVAL;
    }
    return FKGP_OK;
}

// Four-step lines: beyond the register FFT, and for dimensions with few lines
// (e.g. 1-D), where one workgroup of many waves per line pair beats one or
// two waves per pair.
bool few_lines(const fkgp_handle* h, int k, int log2L) {
    return log2L >= kFewLinesMinLog2 && h->M / h->g.m[k] <= kFewLines;
}

// Device bytes make_spectra takes from its Scratch (reg_max = kMaxRegLog2).
size_t spectra_bytes(const fkgp_handle* h, fkgp_dtype dt) {
    const size_t es = dsize(dt);
    size_t t = 0;
    for (int k = 0; k < h->g.d; ++k) {
        const int lg = circulant_log2(h->g.m[k]);
        const size_t L = size_t(1) << lg;
        t += up256(es * L) + up256(2 * es * (L / 2));
        if (lg > kMaxRegLog2 || few_lines(h, k, lg)) t += up256(2 * es * L * kLongWGs);
        if (toeplitz_slab_applies(h->g)) t += up256(es * (size_t)h->g.m[k]);
    }
    return t;
}

// Spectra in dtype `dt` (derivative column for dimension `dderiv`, or none).
// Circulants longer than 2^reg_max take the four-step order; the standalone
// passes (reg_max = kMaxRegLog2) also get their four-step scratch.
fkgp_status make_spectra(const fkgp_handle* h, const fkgp_hypers* hyp, fkgp_dtype dt, int dderiv,
                         Spectra& sp, Scratch& sc, int reg_max = kMaxRegLog2) {
    std::memset(&sp, 0, sizeof(sp));
    const size_t es = dsize(dt);
    for (int k = 0; k < h->g.d; ++k) {
        sp.log2L[k] = circulant_log2(h->g.m[k]);
        if (sp.log2L[k] > (reg_max == kMaxRegLog2 ? kMaxLineLog2 : kMaxBatchLineLog2)) {
            set_error(reg_max == kMaxRegLog2
                          ? "grid dimension longer than 65536 nodes is not supported by the line FFT"
                          : "the batched solver takes grid dimensions of at most 8192 nodes");
            return FKGP_EINVAL;
        }
        sp.L[k] = 1 << sp.log2L[k];
        unsigned char *lam = nullptr, *tw = nullptr;
        FKGP_HIP(sc.get(&lam, es * sp.L[k]));
        FKGP_HIP(sc.get(&tw, 2 * es * (sp.L[k] / 2)));
        if (sp.log2L[k] > reg_max || (reg_max == kMaxRegLog2 && few_lines(h, k, sp.log2L[k]))) {
            int lg2;
            long_split(sp.log2L[k], sp.lg1[k], lg2);
            if (reg_max == kMaxRegLog2) {
                unsigned char* scr = nullptr;
                FKGP_HIP(sc.get(&scr, 2 * es * (size_t)sp.L[k] * kLongWGs));
                sp.scr[k] = scr;
            }
        }
        // the batched solver's long lines have no line scratch of their own:
        // the spectrum still comes from the forward four-step FFT of the
        // embedded column (O(L log L)) through a scratch of L FP64 complex
        // values, as in the standalone passes, not from direct DFT sums
        void* spec_scr = sp.scr[k];
        if (!spec_scr && sp.lg1[k] > 0 && sp.log2L[k] >= 12) {
            unsigned char* scr = nullptr;
            FKGP_HIP(sc.get(&scr, 16 * (size_t)sp.L[k]));
            spec_scr = scr;
        }
        fkgp_status st = build_spectrum(h->g, k, hyp->lengthscale[k], k == dderiv, hyp->kernel,
                                        dt, lam, sp.log2L[k], sp.lg1[k], spec_scr, sc.s);
        if (st != FKGP_OK) return st;
        st = build_twiddles(sp.log2L[k], dt, tw, sc.s);
        if (st != FKGP_OK) return st;
        sp.lam[k] = lam;
        sp.tw[k] = tw;
        if (toeplitz_slab_applies(h->g)) {
            unsigned char* col = nullptr;
            FKGP_HIP(sc.get(&col, es * h->g.m[k]));
            st = build_toeplitz_col(h->g, k, hyp->lengthscale[k], k == dderiv, hyp->kernel, dt,
                                    col, sc.s);
            if (st != FKGP_OK) return st;
            sp.col[k] = col;
        }
    }
    return FKGP_OK;
}

// Everything needed to apply B in the working dtype and, for FP32 handles,
// in FP64 (FP32-stored W^T W upcast exactly, FP64 K_G).
struct OpCtx {
    const fkgp_handle* h;
    fkgp_dtype op;  // arithmetic dtype of B inside the CG loop
    double so, s2;
    int64_t M, halo;
    Spectra sp;     // spectra in dtype `op`
    Spectra sp64;   // FP64 spectra (same as sp when op is FP64)
    // convergence checks by a synchronous copy of the state after each batch
    // (no pinned host slots, which are allocated on first use)
    bool sync_checks = false;
};

fkgp_status make_ctx(const fkgp_handle* h, const fkgp_hypers* hyp, fkgp_dtype op, OpCtx& c,
                     Scratch& sc) {
    c.h = h;
    c.op = op;
    c.so = hyp->outputscale;
    c.s2 = hyp->noise_std * hyp->noise_std;
    c.M = h->M;
    c.halo = dia_halo(h->g);
    fkgp_status st = make_spectra(h, hyp, op, -1, c.sp, sc);
    if (st != FKGP_OK) return st;
    if (op == FKGP_F64) {
        c.sp64 = c.sp;
        return FKGP_OK;
    }
    return make_spectra(h, hyp, FKGP_F64, -1, c.sp64, sc);
}

// B in dtype c.op on one padded vector: u = A x, v = so K u + s2 x (the
// stored W^T W may be FP32 while c.op is FP64: entries are upcast exactly).
fkgp_status apply_B_padded(const OpCtx& c, const void* xpad, void* u, void* v, const int* skip,
                           hipStream_t st, double* dotp = nullptr, int* nparts = nullptr) {
    const fkgp_handle* h = c.h;
    fkgp_status r =
        spmv_dia_any(h->g, h->dt, c.op, h->A, h->bmask, xpad, u, 1, c.halo, skip, st, dotp, nparts);
    if (r != FKGP_OK) return r;
    const void* xin = static_cast<const unsigned char*>(xpad) + c.halo * dsize(c.op);
    return kg_apply_skip(h->g, c.sp, c.op, u, v, 1, c.so, xin, c.s2, skip, st);
}

// B in FP64 on one padded FP64 vector (v may be NULL: u only).
fkgp_status apply_B64(const OpCtx& c, const double* xpad, double* u, double* v, hipStream_t st) {
    const fkgp_handle* h = c.h;
    fkgp_status r = h->dt == FKGP_F32
                        ? spmv_dia_f32a_f64x(h->g, h->A, xpad, u, 1, c.halo, st)
                        : spmv_dia(h->g, FKGP_F64, h->A, xpad, u, 1, c.halo, st);
    if (r != FKGP_OK || !v) return r;
    return kg_apply(h->g, c.sp64, FKGP_F64, u, v, 1, c.so, xpad + c.halo, c.s2, nullptr, st);
}

struct CgBufs {
    double *r, *s, *z, *p, *x, *xd, *partials, *partials2;
    unsigned char *rpad, *u, *v;
    CgState* st;
    unsigned* tickets;   // [2], zero between launches (last-workgroup reductions)
};

fkgp_status alloc_cg(const OpCtx& c, CgBufs& b, Scratch& sc) {
    const int64_t M = c.M;
    const size_t es = dsize(c.op);
    FKGP_HIP(sc.get(&b.r, M));
    FKGP_HIP(sc.get(&b.s, M));
    FKGP_HIP(sc.get(&b.z, M));
    FKGP_HIP(sc.get(&b.p, M));
    FKGP_HIP(sc.get(&b.x, M));
    FKGP_HIP(sc.get(&b.xd, M));
    FKGP_HIP(sc.get(&b.partials, std::max<int64_t>(kRedMaxBlocks, spmv_dot_parts(c.h->g))));
    FKGP_HIP(sc.get(&b.rpad, es * (M + 2 * c.halo)));
    FKGP_HIP(sc.get(&b.u, es * M));
    FKGP_HIP(sc.get(&b.v, es * M));
    FKGP_HIP(sc.get(&b.st, 1));
    FKGP_HIP(sc.get(&b.partials2, std::max<int64_t>(1, kg_last_pass_blocks(c.h->g))));
    FKGP_HIP(sc.get(&b.tickets, 2));
    FKGP_HIP(hipMemsetAsync(b.tickets, 0, 2 * sizeof(unsigned), sc.s));
    FKGP_HIP(hipMemsetAsync(b.rpad, 0, es * (M + 2 * c.halo), sc.s));
    return FKGP_OK;
}

template <class T>
__global__ void cg_step1x(const CgState* __restrict__ st, double* __restrict__ xd,
                          double* __restrict__ x, double* __restrict__ r,
                          const double* __restrict__ s, const double* __restrict__ z,
                          const double* __restrict__ p, T* __restrict__ rpad, int64_t M) {
    if (st->done) return;
    const double a = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        xd[i] = fma(a, s[i], xd[i]);
        if (x) x[i] = fma(a, p[i], x[i]);
        const double rn = fma(-a, z[i], r[i]);
        r[i] = rn;
        rpad[i] = (T)rn;
    }
}

template <class T>
__global__ __launch_bounds__(kRedBlock) void cg_step2x(const CgState* __restrict__ st,
                                                       double* __restrict__ s,
                                                       double* __restrict__ z,
                                                       double* __restrict__ p,
                                                       const double* __restrict__ r,
                                                       const T* __restrict__ u,
                                                       const T* __restrict__ v, int64_t M,
                                                       double* __restrict__ partials) {
    if (st->done) return;
    __shared__ double sh[kRedBlock];
    const double b = st->beta;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock) {
        const double sn = fma(b, s[i], (double)u[i]);
        const double zn = fma(b, z[i], (double)v[i]);
        s[i] = sn;
        z[i] = zn;
        if (p) p[i] = fma(b, p[i], r[i]);
        acc = fma(sn, zn, acc);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Two pinned host slots and two events per host thread and device for the
// CG loop's convergence checks (allocated once, kept until the process ends).
struct CgSnap {
    CgState* host = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

hipError_t cg_snap_get(CgSnap& out) {
    thread_local CgSnap cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    CgSnap& c = cache[dev];
    if (!c.host) {
        e = hipHostMalloc(reinterpret_cast<void**>(&c.host), 2 * sizeof(CgState),
                          hipHostMallocDefault);
        if (e != hipSuccess) {
            c.host = nullptr;
            return e;
        }
        for (int i = 0; i < 2; ++i) {
            e = hipEventCreateWithFlags(&c.ev[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
    }
    out = c;
    return hipSuccess;
}

// One iteration of the loop below (5 launches when the tiled product and the
// fused K_G passes run; every kernel returns at once when b.st->done is set).
template <class DotUr, class Step2>
fkgp_status cg_iteration(const OpCtx& c, CgBufs& b, double* px, double* pp, unsigned char* rin,
                         const LastBlockRed& rho_lb, const CgStep2& step2f, DotUr& dot_ur,
                         Step2& step2, int nb, unsigned ewg, hipStream_t st) {
    const fkgp_handle* h = c.h;
    const int64_t M = c.M;
    if (c.op == FKGP_F32)
        cg_step1x<float><<<ewg, 256, 0, st>>>(b.st, b.xd, px, b.r, b.s, b.z, pp,
                                              reinterpret_cast<float*>(rin), M);
    else
        cg_step1x<double><<<ewg, 256, 0, st>>>(b.st, b.xd, px, b.r, b.s, b.z, pp,
                                               reinterpret_cast<double*>(rin), M);
    FKGP_HIP(hipGetLastError());
    // u = W^T W r_hat; the product's last workgroup finishes u^T r_hat
    // (rho, beta) when the tiled kernel runs
    int np = 0;
    fkgp_status rs = spmv_dia_any(h->g, h->dt, c.op, h->A, h->bmask, b.rpad, b.u, 1, c.halo,
                                  &b.st->done, st, b.partials, &np, &rho_lb);
    if (rs != FKGP_OK) return rs;
    if (np == 0) {
        FKGP_HIP(dot_ur(&b.st->done));
        finalize<<<1, kRedBlock, 0, st>>>(b.partials, nb, b.st, FIN_RHO);
    }
    // v = s K_G u + s2 r_hat, consumed by the fused direction update
    bool fused = false;
    rs = kg_apply_fused(h->g, c.sp, c.op, b.u, b.v, c.so, rin, c.s2, &b.st->done, step2f, &fused,
                        st);
    if (rs != FKGP_OK) return rs;
    if (!fused) {
        FKGP_HIP(step2());
        finalize<<<1, kRedBlock, 0, st>>>(b.partials, nb, b.st, FIN_SZ);
    }
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// Simplified efficiently-factorized CG (appendix): the residual stays in the
// span of W, r = W r_hat, and each iteration applies B once.  On entry b.r
// holds r_hat_0; on exit b.xd += sum_k alpha_k s_k (= W^T W x_hat) and
// b.x += sum_k alpha_k p_hat_k (= x_hat, the compressed solution update).
// Stop when u^T r_hat <= eps, with eps = eps_abs, or eps_rel * (u^T r_hat)_0.
fkgp_status run_cg(const OpCtx& c, CgBufs& b, double eps_abs, double eps_rel, int maxiter,
                   CgState& out, hipStream_t st, bool track_x = true) {
    double* px = track_x ? b.x : nullptr;
    double* pp = track_x ? b.p : nullptr;
    const fkgp_handle* h = c.h;
    const int64_t M = c.M;
    const size_t es = dsize(c.op);
    unsigned char* rin = b.rpad + c.halo * es;
    CgState init{};
    const bool rel = eps_rel >= 0.0;
    init.eps = rel ? eps_rel : eps_abs;
    FKGP_HIP(hipMemcpyAsync(b.st, &init, sizeof(CgState), hipMemcpyHostToDevice, st));
    FKGP_HIP(hipMemsetAsync(b.s, 0, sizeof(double) * M, st));
    FKGP_HIP(hipMemsetAsync(b.z, 0, sizeof(double) * M, st));
    FKGP_HIP(hipMemsetAsync(b.p, 0, sizeof(double) * M, st));
    FKGP_HIP(convert_any(b.r, FKGP_F64, rin, c.op, M, 1.0, st));
    fkgp_status rs = apply_B_padded(c, b.rpad, b.u, b.v, nullptr, st);
    if (rs != FKGP_OK) return rs;
    const int nb = red_blocks(M);
    const unsigned ewg = ew_grid(M);
    auto dot_ur = [&](const int* skip) -> hipError_t {
        if (c.op == FKGP_F32)
            dot_partial<float><<<nb, kRedBlock, 0, st>>>(reinterpret_cast<float*>(b.u), b.r, M,
                                                         b.partials, skip);
        else
            dot_partial<double><<<nb, kRedBlock, 0, st>>>(reinterpret_cast<double*>(b.u), b.r, M,
                                                          b.partials, skip);
        return hipGetLastError();
    };
    auto step2 = [&]() -> hipError_t {
        if (c.op == FKGP_F32)
            cg_step2x<float><<<nb, kRedBlock, 0, st>>>(b.st, b.s, b.z, pp, b.r,
                                                       reinterpret_cast<float*>(b.u),
                                                       reinterpret_cast<float*>(b.v), M,
                                                       b.partials);
        else
            cg_step2x<double><<<nb, kRedBlock, 0, st>>>(b.st, b.s, b.z, pp, b.r,
                                                        reinterpret_cast<double*>(b.u),
                                                        reinterpret_cast<double*>(b.v), M,
                                                        b.partials);
        return hipGetLastError();
    };
    FKGP_HIP(dot_ur(nullptr));
    finalize<<<1, kRedBlock, 0, st>>>(b.partials, nb, b.st, rel ? FIN_INIT_RHS : FIN_INIT);
    FKGP_HIP(step2());
    finalize<<<1, kRedBlock, 0, st>>>(b.partials, nb, b.st, FIN_SZ);
    FKGP_HIP(hipGetLastError());
    const LastBlockRed rho_lb{b.partials, b.tickets, b.st, FIN_RHO};
    const CgStep2 step2f{b.st, b.s, b.z, pp, b.r, b.u,
                         LastBlockRed{b.partials2, b.tickets + 1, b.st, FIN_SZ}};
    // Pipelined convergence checks: the state after each batch of kBatch
    // iterations is copied to pinned host memory behind that batch while the
    // next batch is already queued, so the device does not idle while the
    // host reads it; once the state is converged the queued launches are
    // no-ops (every kernel of the loop tests b.st->done).
    constexpr int kBatch = 8;
    if (c.sync_checks) {
        for (int launched = 0;;) {
            const int nit = std::min(kBatch, maxiter - launched);
            for (int it = 0; it < nit; ++it) {
                rs = cg_iteration(c, b, px, pp, rin, rho_lb, step2f, dot_ur, step2, nb, ewg, st);
                if (rs != FKGP_OK) return rs;
            }
            launched += nit;
            FKGP_HIP(hipMemcpyAsync(&out, b.st, sizeof(CgState), hipMemcpyDeviceToHost, st));
            FKGP_HIP(hipStreamSynchronize(st));
            if (out.done || launched >= maxiter) break;
        }
        if (out.done == 2) {
            set_error("factorized CG broke down (non-finite step)");
            return FKGP_EDEVICE;
        }
        return FKGP_OK;
    }
    CgSnap snapbuf;
    FKGP_HIP(cg_snap_get(snapbuf));
    CgState* snap = snapbuf.host;
    int launched = 0, slot = 0;
    FKGP_HIP(hipMemcpyAsync(&snap[0], b.st, sizeof(CgState), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipEventRecord(snapbuf.ev[0], st));
    for (;;) {
        const int next = slot ^ 1;
        const bool queued = launched < maxiter;
        if (queued) {
        const int nit = std::min(kBatch, maxiter - launched);
        for (int it = 0; it < nit; ++it) {
            rs = cg_iteration(c, b, px, pp, rin, rho_lb, step2f, dot_ur, step2, nb, ewg, st);
            if (rs != FKGP_OK) return rs;
        }
        launched += nit;
        FKGP_HIP(hipMemcpyAsync(&snap[next], b.st, sizeof(CgState), hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipEventRecord(snapbuf.ev[next], st));
        }
        FKGP_HIP(hipEventSynchronize(snapbuf.ev[slot]));
        out = snap[slot];
        if (out.done || !queued) break;
        slot = next;
    }
    // the batch queued behind the last snapshot read (no-ops once converged)
    FKGP_HIP(hipStreamSynchronize(st));
    if (out.done == 2) {
        set_error("factorized CG broke down (non-finite step)");
        return FKGP_EDEVICE;
    }
    return FKGP_OK;
}

__global__ void sub_out(const double* __restrict__ a, const double* __restrict__ b,
                        double* __restrict__ out, int64_t M) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

__global__ void add_inplace(double* __restrict__ a, const double* __restrict__ b, int64_t M) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] += b[i];
}

fkgp_status dot64(const double* a, const double* b, int64_t M, double* partials, CgState* tmp,
                  double& out, hipStream_t st) {
    const int nb = red_blocks(M);
    dot_partial<double><<<nb, kRedBlock, 0, st>>>(a, b, M, partials, nullptr);
    CgState init{};
    init.eps = -1.0;
    FKGP_HIP(hipMemcpyAsync(tmp, &init, sizeof(CgState), hipMemcpyHostToDevice, st));
    finalize<<<1, kRedBlock, 0, st>>>(partials, nb, tmp, FIN_INIT);
    FKGP_HIP(hipGetLastError());
    CgState h{};
    FKGP_HIP(hipMemcpyAsync(&h, tmp, sizeof(CgState), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    out = h.rho;
    return FKGP_OK;
}

// Solve (W K_G W^T + s2 I) z = b for b = y (rhs == NULL; x_0 = y/s2) or
// b = W rhs (x_0 = 0) and return W^T z in `wtz`.
//  * FP64 handles: the simplified factorized CG as printed, output
//    W^T z = x_hat^d (+ W^T y / s2).
//  * FP32 handles: the same CG with B in FP32 as the inner solver of an FP64
//    iterative refinement: the compressed iterate z = x_0 + W x_hat is kept
//    in FP64, its residual W r_hat with r_hat = r_hat_0 - B_64(x_hat) is
//    recomputed in FP64 after every inner solve, and the inner solve returns
//    the correction of x_hat.
fkgp_status solve_core(const OpCtx& c, const double* rhs, double tol, int maxiter, double* wtz,
                       fkgp_solve_info* info, Scratch& sc, hipStream_t st) {
    const fkgp_handle* h = c.h;
    const int64_t M = c.M;
    const unsigned ewg = ew_grid(M);
    CgBufs b{};
    fkgp_status rs = alloc_cg(c, b, sc);
    if (rs != FKGP_OK) return rs;
    double* r0 = nullptr;
    FKGP_HIP(sc.get(&r0, M));
    // r_hat_0 in FP64
    if (rhs) {
        FKGP_HIP(hipMemcpyAsync(r0, rhs, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
    } else {
        rs = kg_apply(h->g, c.sp64, FKGP_F64, h->wty, r0, 1, -c.so / c.s2, nullptr, 0.0, nullptr,
                      st);
        if (rs != FKGP_OK) return rs;
    }
    int total_iters = 0;
    bool converged = false;
    double rho_final = 0.0, bnorm2 = rhs ? 0.0 : h->yty;
    if (c.op == FKGP_F64) {
        FKGP_HIP(hipMemcpyAsync(b.r, r0, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        FKGP_HIP(hipMemsetAsync(b.xd, 0, sizeof(double) * M, st));
        FKGP_HIP(hipMemsetAsync(b.x, 0, sizeof(double) * M, st));
        CgState out{};
        rs = run_cg(c, b, tol * tol * h->yty, rhs ? tol * tol : -1.0, maxiter, out, st,
                    /*track_x=*/false);
        if (rs != FKGP_OK) return rs;
        total_iters = out.iters;
        converged = out.done == 1;
        rho_final = out.rho;
        if (rhs) bnorm2 = out.bnorm2;
        if (rhs)
            FKGP_HIP(hipMemcpyAsync(wtz, b.xd, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        else
            axpy_out<<<ewg, 256, 0, st>>>(b.xd, h->wty, 1.0 / c.s2, wtz, M);
    } else {
        double *xt = nullptr, *xpad64 = nullptr, *u64 = nullptr, *v64 = nullptr;
        FKGP_HIP(sc.get(&xt, M));
        FKGP_HIP(sc.get(&xpad64, M + 2 * c.halo));
        FKGP_HIP(sc.get(&u64, M));
        FKGP_HIP(sc.get(&v64, M));
        FKGP_HIP(hipMemsetAsync(xt, 0, sizeof(double) * M, st));
        FKGP_HIP(hipMemsetAsync(xpad64, 0, sizeof(double) * (M + 2 * c.halo), st));
        FKGP_HIP(hipMemcpyAsync(b.r, r0, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        double* xin64 = xpad64 + c.halo;
        if (rhs) {
            // ||b||^2 = rhs^T W^T W rhs
            FKGP_HIP(hipMemcpyAsync(xin64, rhs, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
            rs = apply_B64(c, xpad64, u64, nullptr, st);
            if (rs != FKGP_OK) return rs;
            rs = dot64(u64, rhs, M, b.partials, b.st, bnorm2, st);
            if (rs != FKGP_OK) return rs;
        }
        const double target = tol * tol * bnorm2;
        constexpr int kMaxOuter = 12;
        for (int outer = 0; outer <= kMaxOuter; ++outer) {
            // true residual norm ||W r_hat||^2 = r_hat^T W^T W r_hat (FP64)
            FKGP_HIP(hipMemcpyAsync(xin64, b.r, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
            rs = apply_B64(c, xpad64, u64, nullptr, st);
            if (rs != FKGP_OK) return rs;
            double rho_true = 0.0;
            rs = dot64(u64, b.r, M, b.partials, b.st, rho_true, st);
            if (rs != FKGP_OK) return rs;
            rho_final = rho_true;
            if (rho_true <= target) {
                converged = true;
                break;
            }
            if (outer == kMaxOuter || total_iters >= maxiter) break;
            // inner FP32 solve to a modest relative accuracy
            double tin = 0.5 * std::sqrt(target / std::max(rho_true, 1e-300));
            tin = std::min(std::max(tin, 1e-4), 0.5);
            FKGP_HIP(hipMemsetAsync(b.xd, 0, sizeof(double) * M, st));
            FKGP_HIP(hipMemsetAsync(b.x, 0, sizeof(double) * M, st));
            CgState out{};
            rs = run_cg(c, b, 0.0, tin * tin, maxiter - total_iters, out, st);
            if (rs != FKGP_OK) return rs;
            total_iters += out.iters;
            add_inplace<<<ewg, 256, 0, st>>>(xt, b.x, M);
            // r_hat = r_hat_0 - B_64(x_hat).v
            FKGP_HIP(hipMemcpyAsync(xin64, xt, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
            rs = apply_B64(c, xpad64, u64, v64, st);
            if (rs != FKGP_OK) return rs;
            sub_out<<<ewg, 256, 0, st>>>(r0, v64, b.r, M);
            FKGP_HIP(hipGetLastError());
            if (out.iters == 0) break;   // no progress possible
        }
        // W^T z = W^T W x_hat (+ W^T y / s2)
        FKGP_HIP(hipMemcpyAsync(xin64, xt, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        rs = apply_B64(c, xpad64, u64, nullptr, st);
        if (rs != FKGP_OK) return rs;
        if (rhs)
            FKGP_HIP(hipMemcpyAsync(wtz, u64, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        else
            axpy_out<<<ewg, 256, 0, st>>>(u64, h->wty, 1.0 / c.s2, wtz, M);
    }
    FKGP_HIP(hipGetLastError());
    if (info) {
        info->iterations = total_iters;
        info->converged = converged ? 1 : 0;
        info->rel_residual = std::sqrt(std::max(rho_final, 0.0) / (bnorm2 > 0 ? bnorm2 : 1.0));
    }
    return converged ? FKGP_OK : FKGP_ENOTCONV;
}

// Device bytes solve_impl takes from its Scratch (mirrors make_ctx, the
// output buffer, alloc_cg, r_hat_0 and solve_core's FP32 refinement buffers).
size_t solve_scratch_bytes(const fkgp_handle* h, fkgp_dtype op) {
    const size_t M = (size_t)h->M;
    const size_t halo = (size_t)dia_halo(h->g);
    const size_t es = dsize(op);
    size_t t = spectra_bytes(h, op) + (op == FKGP_F64 ? 0 : spectra_bytes(h, FKGP_F64));
    t += up256(8 * M);                                                   // wtz
    t += 6 * up256(8 * M);                                               // r s z p x xd
    t += up256(8 * (size_t)std::max<int64_t>(kRedMaxBlocks, spmv_dot_parts(h->g)));
    t += up256(es * (M + 2 * halo)) + 2 * up256(es * M);                 // rpad, u, v
    t += up256(sizeof(CgState));
    t += up256(8 * (size_t)std::max<int64_t>(1, kg_last_pass_blocks(h->g)));
    t += up256(2 * sizeof(unsigned));                                    // tickets
    t += up256(8 * M);                                                   // r0
    if (op == FKGP_F32) t += 3 * up256(8 * M) + up256(8 * (M + 2 * halo));
    return t;
}

// arena != nullptr: every device buffer is carved from it (nothing is
// allocated, no pinned host memory is used).
fkgp_status solve_impl(const fkgp_handle* h, const fkgp_hypers* hyp, const double* rhs,
                       double* out, double tol, int maxiter, fkgp_dtype op,
                       fkgp_solve_info* info, hipStream_t st, unsigned char* arena = nullptr,
                       size_t arena_cap = 0) {
    Scratch sc = arena ? Scratch(st, arena, arena_cap) : Scratch(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, op, c, sc);
    if (rs != FKGP_OK) return rs;
    c.sync_checks = arena != nullptr;
    double* wtz = nullptr;
    FKGP_HIP(sc.get(&wtz, h->M));
    fkgp_status res = solve_core(c, rhs, tol, maxiter, wtz, info, sc, st);
    if (res != FKGP_OK && res != FKGP_ENOTCONV) return res;
    if (rhs) {
        FKGP_HIP(hipMemcpyAsync(out, wtz, sizeof(double) * h->M, hipMemcpyDeviceToDevice, st));
    } else {
        // mu_G = K_G W^T z~ (FP64)
        rs = kg_apply(h->g, c.sp64, FKGP_F64, wtz, out, 1, c.so, nullptr, 0.0, nullptr, st);
        if (rs != FKGP_OK) return rs;
    }
    FKGP_HIP(hipStreamSynchronize(st));
    return res;
}

// ---------------------------------------------------------------------------
// Plain SKI baseline: CG in n-space on A z = y, A = W K_G W^T + s2 I (the
// iteration the factorized CG replaces; Sec. 2.3), vectors in the kept cell
// order.  Scalars stay on the device; the host polls the stop flag.
// ---------------------------------------------------------------------------
struct SkiCg {
    double rho, alpha, beta, eps;
    int done, iters;
};

// partials of a.b over n (grid-stride, fixed shape: deterministic)
__global__ __launch_bounds__(kRedBlock) void nvec_dot(const double* __restrict__ a,
                                                      const double* __restrict__ b, int64_t n,
                                                      double* __restrict__ partials,
                                                      const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock)
        acc = fma(a[i], b[i], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

enum SkiFin { SKI_INIT = 0, SKI_ALPHA = 1, SKI_RHO = 2 };

__global__ __launch_bounds__(kRedBlock) void ski_fin(const double* __restrict__ partials,
                                                     int nb, SkiCg* cg, int op, double tol) {
    if (cg->done) return;
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedBlock) acc += partials[i];
    const double v = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    if (op == SKI_INIT) {   // v = y.y
        cg->rho = v;
        cg->eps = tol * tol * v;
        cg->done = v > 0.0 ? 0 : 1;
    } else if (op == SKI_ALPHA) {   // v = p.Ap
        const double a = cg->rho / v;
        if (!isfinite(a)) {
            cg->done = 2;
            return;
        }
        cg->alpha = a;
    } else {   // v = r.r
        cg->iters += 1;
        if (!(v > cg->eps)) {
            cg->rho = v;
            cg->done = 1;
            return;
        }
        cg->beta = v / cg->rho;
        cg->rho = v;
    }
}

__global__ void ski_upd_zr(const SkiCg* __restrict__ cg, double* __restrict__ z,
                           double* __restrict__ r, const double* __restrict__ p,
                           const double* __restrict__ q, int64_t n) {
    if (cg->done) return;
    const double a = cg->alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        z[i] = fma(a, p[i], z[i]);
        r[i] = fma(-a, q[i], r[i]);
    }
}

__global__ void ski_upd_p(const SkiCg* __restrict__ cg, double* __restrict__ p,
                          const double* __restrict__ r, int64_t n) {
    if (cg->done) return;
    const double b = cg->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = fma(b, p[i], r[i]);
}

fkgp_status ski_solve_impl(const fkgp_handle* h, const fkgp_hypers* hyp, double tol, int maxiter,
                           double* mean_grid, fkgp_solve_info* info, hipStream_t st) {
    Scratch sc(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, FKGP_F64, c, sc);
    if (rs != FKGP_OK) return rs;
    const GridDev& g = h->g;
    const int64_t n = h->n, M = h->M;
    int64_t ncells = 1;
    for (int k = 0; k < g.d; ++k) ncells *= g.nc[k];
    const int64_t nn = std::max<int64_t>(n, 1);
    double *z, *r, *p, *q, *R, *T1, *wt, *kv, *partials;
    SkiCg* cg;
    FKGP_HIP(sc.get(&z, nn));
    FKGP_HIP(sc.get(&r, nn));
    FKGP_HIP(sc.get(&p, nn));
    FKGP_HIP(sc.get(&q, nn));
    // per-cell moments (4^d per cell) and the assembly stages' workspace
    // (3-D: two intermediate stages of 16 and 4 values per node)
    FKGP_HIP(sc.get(&R, ncells * (g.d == 1 ? 4 : (g.d == 2 ? 16 : 64))));
    FKGP_HIP(sc.get(&T1, M * (g.d == 1 ? 1 : (g.d == 2 ? 4 : 20))));
    FKGP_HIP(sc.get(&wt, M));
    FKGP_HIP(sc.get(&kv, M));
    const int nb = red_blocks(nn);
    FKGP_HIP(sc.get(&partials, nb));
    FKGP_HIP(sc.get(&cg, 1));
    const unsigned ewg = ew_grid(nn);
    const SkiCg init{};
    FKGP_HIP(hipMemcpyAsync(cg, &init, sizeof(SkiCg), hipMemcpyHostToDevice, st));
    FKGP_HIP(hipMemsetAsync(z, 0, sizeof(double) * nn, st));
    rs = ski_y(g, h->in_dt, h->pay, n, r, st);
    if (rs != FKGP_OK) return rs;
    FKGP_HIP(hipMemcpyAsync(p, r, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    const int* done = &cg->done;
    nvec_dot<<<nb, kRedBlock, 0, st>>>(r, r, n, partials, nullptr);
    ski_fin<<<1, kRedBlock, 0, st>>>(partials, nb, cg, SKI_INIT, tol);
    FKGP_HIP(hipGetLastError());
    // q = (W K_G W^T + s2 I) v
    auto apply = [&](const double* v) -> fkgp_status {
        fkgp_status e = ski_wt(g, h->in_dt, h->pay, h->cstart, h->cend, v, R, T1, wt, st);
        if (e != FKGP_OK) return e;
        e = kg_apply(g, c.sp64, FKGP_F64, wt, kv, 1, c.so, nullptr, 0.0, nullptr, st);
        if (e != FKGP_OK) return e;
        return ski_w(g, h->in_dt, h->pay, n, kv, v, c.s2, q, st);
    };
    SkiCg out{};
    constexpr int kBatch = 8;
    int launched = 0;
    for (;;) {
        FKGP_HIP(hipMemcpyAsync(&out, cg, sizeof(SkiCg), hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipStreamSynchronize(st));
        if (out.done || launched >= maxiter) break;
        const int nit = std::min(kBatch, maxiter - launched);
        for (int it = 0; it < nit; ++it) {
            rs = apply(p);
            if (rs != FKGP_OK) return rs;
            nvec_dot<<<nb, kRedBlock, 0, st>>>(p, q, n, partials, done);
            ski_fin<<<1, kRedBlock, 0, st>>>(partials, nb, cg, SKI_ALPHA, tol);
            ski_upd_zr<<<ewg, 256, 0, st>>>(cg, z, r, p, q, n);
            nvec_dot<<<nb, kRedBlock, 0, st>>>(r, r, n, partials, done);
            ski_fin<<<1, kRedBlock, 0, st>>>(partials, nb, cg, SKI_RHO, tol);
            ski_upd_p<<<ewg, 256, 0, st>>>(cg, p, r, n);
            FKGP_HIP(hipGetLastError());
        }
        launched += nit;
    }
    if (out.done == 2) {
        set_error("SKI CG broke down (non-finite step)");
        return FKGP_EDEVICE;
    }
    // mean_grid = K_G W^T z
    rs = ski_wt(g, h->in_dt, h->pay, h->cstart, h->cend, z, R, T1, wt, st);
    if (rs != FKGP_OK) return rs;
    rs = kg_apply(g, c.sp64, FKGP_F64, wt, mean_grid, 1, c.so, nullptr, 0.0, nullptr, st);
    if (rs != FKGP_OK) return rs;
    FKGP_HIP(hipStreamSynchronize(st));
    const double ynorm2 = h->yty;
    if (info) {
        info->iterations = out.iters;
        info->converged = out.done == 1 ? 1 : 0;
        info->rel_residual = std::sqrt(std::max(out.rho, 0.0) / (ynorm2 > 0 ? ynorm2 : 1.0));
    }
    return out.done == 1 ? FKGP_OK : FKGP_ENOTCONV;
}

}  // namespace
}  // namespace fkgp

using namespace fkgp;

namespace {

template <class F>
fkgp_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::exception& e) {
        set_error(std::string("internal error: ") + e.what());
        return FKGP_EDEVICE;
    } catch (...) {
        set_error("internal error");
        return FKGP_EDEVICE;
    }
}

// One pool allocation for a handle's arrays: W^T W (row-tiled), W^T y, the
// sketches, the block mask, then y^T y, the out-of-grid flag and the block
// count side by side (read back with one copy).
fkgp_status alloc_handle_arrays(fkgp_handle* h, hipStream_t s) {
    fkgp::ensure_pool();
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t M = h->M;
    const size_t bA = up(dsize(h->dt) * (size_t)dia_elems(M, h->NB));
    const size_t bW = up(sizeof(double) * M);
    const size_t bS = up(sizeof(double) * M * h->nprobe);
    const size_t bK = up(sizeof(uint32_t) * (size_t)mask_words(M));
    hipError_t e;
    h->alloc = current_alloc();
    if ((e = dev_malloc(h->alloc, &h->block, bA + bW + bS + bK + 256, s)) != hipSuccess)
        return hip_fail(e, "device allocation (handle)");
    unsigned char* hb = static_cast<unsigned char*>(h->block);
    h->A = hb;
    h->wty = reinterpret_cast<double*>(hb + bA);
    h->sketches = h->nprobe > 0 ? reinterpret_cast<double*>(hb + bA + bW) : nullptr;
    h->bmask = reinterpret_cast<uint32_t*>(hb + bA + bW + bS);
    h->yty_dev = reinterpret_cast<double*>(hb + bA + bW + bS + bK);
    return FKGP_OK;
}

// File of fkgp_save: this header, then W^T W (row-tiled, stats dtype), the
// block mask, W^T y and the sketches, in host (little-endian) byte order.
struct StatsFileHeader {
    char magic[8];   // "FKGPSTAT"
    uint32_t version;
    int32_t d;
    int64_t m[3];
    double origin[3];
    double spacing[3];
    int64_t n;
    int32_t stats_dtype;
    int32_t nprobe;
    uint64_t seed;
    double yty;
    int64_t nzblocks;
    int32_t interp;    // 0: cubic, 1: linear
    int32_t reserved;
};
constexpr uint32_t kStatsFileVersion = 2;
static_assert(sizeof(StatsFileHeader) == 136, "statistics file header layout");

struct StatsSections {
    size_t a, mask, wty, sk;
    size_t total() const { return a + mask + wty + sk; }
};

StatsSections stats_sections(const fkgp_handle* h) {
    return {dsize(h->dt) * (size_t)dia_elems(h->M, h->NB),
            sizeof(uint32_t) * (size_t)mask_words(h->M), sizeof(double) * (size_t)h->M,
            sizeof(double) * (size_t)h->M * h->nprobe};
}

// The handle's arrays come from the device's stream-ordered pool (as all
// scratch does): freed on the default stream once pending work is done.
void free_handle(fkgp_handle* h) {
    if (!h) return;
    if (h->block || h->pts_block) {
        (void)hipDeviceSynchronize();
        dev_free(h->alloc, h->block, nullptr);
        dev_free(h->alloc, h->pts_block, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    delete h;
}


}  // namespace

extern "C" {

const char* fkgp_last_error(void) { return g_last_error.c_str(); }

fkgp_status fkgp_precompute(const fkgp_grid* grid, const void* const* x, const void* y,
                            int64_t n, fkgp_dtype in, const fkgp_precompute_opts* opts,
                            void* stream, fkgp_handle** out) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!out) {
            set_error("out is NULL");
            return FKGP_EINVAL;
        }
        *out = nullptr;
        GridDev g;
        int64_t M;
        fkgp_status st = grid_from_abi(grid, g, M);
        if (st != FKGP_OK) return st;
        if (n < 0 || n >= (int64_t(1) << 31) - 1) {
            set_error("n must be in [0, 2^31 - 1)");
            return FKGP_EINVAL;
        }
        if (in != FKGP_F32 && in != FKGP_F64) {
            set_error("input dtype must be FKGP_F32 or FKGP_F64");
            return FKGP_EINVAL;
        }
        if (n > 0) {
            if (!x || !y) {
                set_error("x and y must be non-NULL when n > 0");
                return FKGP_EINVAL;
            }
            for (int k = 0; k < g.d; ++k)
                if (!x[k]) {
                    set_error("x[k] is NULL");
                    return FKGP_EINVAL;
                }
        }
        fkgp_precompute_opts o{FKGP_F32, 0, 0, 0, FKGP_INTERP_CUBIC};
        if (opts) o = *opts;
        if (o.interp != FKGP_INTERP_CUBIC && o.interp != FKGP_INTERP_LINEAR) {
            set_error("interp must be FKGP_INTERP_CUBIC or FKGP_INTERP_LINEAR");
            return FKGP_EINVAL;
        }
        g.interp = o.interp;
        if (o.keep_points != 0 && o.keep_points != 1) {
            set_error("keep_points must be 0 or 1");
            return FKGP_EINVAL;
        }
        if (o.stats_dtype != FKGP_F32 && o.stats_dtype != FKGP_F64) {
            set_error("stats dtype must be FKGP_F32 or FKGP_F64");
            return FKGP_EINVAL;
        }
        if (o.n_probes < 0 || o.n_probes > kMaxProbes) {
            set_error("n_probes must be in [0, 31]");
            return FKGP_EINVAL;
        }
        for (int k = 0; k < g.d; ++k)
            if (circulant_log2(g.m[k]) > kMaxLineLog2) {
                set_error("grid dimension longer than 65536 nodes is not supported");
                return FKGP_EINVAL;
            }
        hipStream_t s = static_cast<hipStream_t>(stream);
        fkgp_handle* h = new fkgp_handle();
        h->g = g;
        h->n = n;
        h->M = M;
        h->NB = 1;
        for (int k = 0; k < g.d; ++k) h->NB *= 7;
        h->dt = o.stats_dtype;
        h->nprobe = o.n_probes;
        h->seed = o.probe_seed;
        auto fail = [&](fkgp_status e) {
            free_handle(h);
            return e;
        };
        hipError_t e;
        auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
        st = alloc_handle_arrays(h, s);
        if (st != FKGP_OK) return fail(st);
        unsigned long long* bad = reinterpret_cast<unsigned long long*>(h->yty_dev + 1);
        (void)hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), s);
        (void)hipMemsetAsync(h->bmask, 0, sizeof(uint32_t) * (size_t)mask_words(M), s);
        (void)hipMemsetAsync(h->yty_dev + 3, 0, sizeof(double), s);
        StatsOut so{h->A, h->wty, h->sketches, h->yty_dev, h->bmask,
                    reinterpret_cast<unsigned long long*>(h->yty_dev + 2),
                    reinterpret_cast<unsigned long long*>(h->yty_dev + 3), nullptr, nullptr,
                    nullptr};
        if (o.keep_points) {
            int64_t ncells = 1;
            for (int k = 0; k < g.d; ++k) ncells *= g.nc[k];
            const size_t bp = up((in == FKGP_F32 ? 16 : 32) * (size_t)std::max<int64_t>(n, 1));
            const size_t bc = up(sizeof(uint32_t) * (size_t)ncells);
            if ((e = dev_malloc(h->alloc, &h->pts_block, bp + 2 * bc, s)) != hipSuccess)
                return fail(hip_fail(e, "device allocation (points)"));
            unsigned char* pb = static_cast<unsigned char*>(h->pts_block);
            h->pay = pb;
            h->cstart = reinterpret_cast<uint32_t*>(pb + bp);
            h->cend = reinterpret_cast<uint32_t*>(pb + bp + bc);
            h->in_dt = in;
            so.keep_pay = h->pay;
            so.keep_cstart = h->cstart;
            so.keep_cend = h->cend;
        }
        st = run_precompute(g, x, y, n, in, h->dt, h->nprobe, h->seed, so, bad, s);
        unsigned long long hbad = ~0ull;
        double back[4] = {0.0, 0.0, 0.0, 0.0};
        if (st == FKGP_OK) {
            if ((e = hipMemcpyAsync(back, h->yty_dev, sizeof(back), hipMemcpyDeviceToHost, s)) !=
                hipSuccess)
                st = hip_fail(e, "hipMemcpyAsync(y^T y, flag)");
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess && st == FKGP_OK)
            st = hip_fail(e, "hipStreamSynchronize");
        if (st != FKGP_OK) return fail(st);
        h->yty = back[0];
        std::memcpy(&hbad, &back[1], sizeof(hbad));
        unsigned long long nzb = 0;
        std::memcpy(&nzb, &back[2], sizeof(nzb));
        h->nzblocks = (int64_t)nzb;
        unsigned long long nnz = 0;
        std::memcpy(&nnz, &back[3], sizeof(nnz));
        h->nnz = (int64_t)nnz;
        if (hbad != ~0ull) {
            set_error("point " + std::to_string(hbad) + " lies outside the interpolable region");
            return fail(FKGP_EOUTOFGRID);
        }
        *out = h;
        return FKGP_OK;
    });
}

fkgp_status fkgp_describe(const fkgp_handle* h, fkgp_handle_desc* desc) {
    if (!h || !desc) {
        set_error("NULL argument");
        return FKGP_EINVAL;
    }
    desc->n = h->n;
    desc->m_total = h->M;
    desc->d = h->g.d;
    desc->stats_dtype = h->dt;
    desc->n_probes = h->nprobe;
    desc->yty = h->yty;
    desc->nnz_wtw = h->M * h->NB;
    desc->bytes_wtw = dia_elems(h->M, h->NB) * (int64_t)dsize(h->dt);
    desc->halo = dia_halo(h->g);
    const int slabs = h->g.d == 3 ? 7 : 1;
    desc->wtw_blocks = mask_words(h->M) * (kRowTile / kWaveRows) * slabs;
    desc->wtw_blocks_nonzero = h->nzblocks;
    desc->wtw_block_entries = (int64_t)kWaveRows * mask_slab_width(h->g.d);
    desc->interp = h->g.interp;
    desc->nnz_wtw_nonzero = h->nnz;
    return FKGP_OK;
}

fkgp_status fkgp_export_stats(const fkgp_handle* h, void* wtw, double* wty, double* yty,
                              void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h) {
            set_error("handle is NULL");
            return FKGP_EINVAL;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (wtw) {
            fkgp_status st = dia_to_canonical(h->g, h->dt, h->A, wtw, s);
            if (st != FKGP_OK) return st;
        }
        if (wty) FKGP_HIP(hipMemcpyAsync(wty, h->wty, sizeof(double) * h->M, hipMemcpyDeviceToDevice, s));
        FKGP_HIP(hipStreamSynchronize(s));
        if (yty) *yty = h->yty;
        return FKGP_OK;
    });
}

fkgp_status fkgp_export_sketches(const fkgp_handle* h, double* out, void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h || !out) {
            set_error("NULL argument");
            return FKGP_EINVAL;
        }
        if (h->nprobe == 0) {
            set_error("handle has no probe sketches");
            return FKGP_EINVAL;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        FKGP_HIP(hipMemcpyAsync(out, h->sketches, sizeof(double) * h->M * h->nprobe,
                                hipMemcpyDeviceToDevice, s));
        FKGP_HIP(hipStreamSynchronize(s));
        return FKGP_OK;
    });
}

fkgp_status fkgp_solve(const fkgp_handle* h, const fkgp_hypers* hyp, const double* rhs_grid,
                       double* out, const fkgp_solve_opts* opts, fkgp_solve_info* info,
                       void* stream) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!h || !out) {
            set_error("handle and out must be non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        fkgp_solve_opts o{1e-6, 1000, FKGP_OP_F64};
        if (opts) o = *opts;
        if (!(o.tol >= 0.0) || o.maxiter < 0) {
            set_error("tol must be >= 0 and maxiter >= 0");
            return FKGP_EINVAL;
        }
        if (o.op_precision != FKGP_OP_F64 && o.op_precision != FKGP_OP_STATS) {
            set_error("op_precision must be FKGP_OP_F64 or FKGP_OP_STATS");
            return FKGP_EINVAL;
        }
        const fkgp_dtype op = o.op_precision == FKGP_OP_STATS ? h->dt : FKGP_F64;
        return solve_impl(h, hyp, rhs_grid, out, o.tol, o.maxiter, op, info,
                          static_cast<hipStream_t>(stream));
    });
}

fkgp_status fkgp_mll_and_grad(const fkgp_handle* h, const fkgp_hypers* hyp,
                              const fkgp_mll_opts* opts, double* mll, double* grad,
                              fkgp_mll_info* info, void* stream);

}  // extern "C"

namespace {

// Device address of `scratch` on each device, looked up once per device
// (with that device current) on the first fkgp_solve_noalloc call there.
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[64] = {};

fkgp_status noalloc_scratch(unsigned char** out) {
    int dev = 0;
    FKGP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device index out of range for the no-allocation workspace");
        return FKGP_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_noalloc_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return FKGP_OK;
}

}  // namespace

extern "C" {

fkgp_status fkgp_solve_noalloc(const fkgp_handle* h, const fkgp_hypers* hyp,
                               const double* rhs_grid, double* out, const fkgp_solve_opts* opts,
                               fkgp_solve_info* info, void* stream) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!h || !out) {
            set_error("handle and out must be non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        fkgp_solve_opts o{1e-6, 1000, FKGP_OP_F64};
        if (opts) o = *opts;
        if (!(o.tol >= 0.0) || o.maxiter < 0) {
            set_error("tol must be >= 0 and maxiter >= 0");
            return FKGP_EINVAL;
        }
        if (o.op_precision != FKGP_OP_F64 && o.op_precision != FKGP_OP_STATS) {
            set_error("op_precision must be FKGP_OP_F64 or FKGP_OP_STATS");
            return FKGP_EINVAL;
        }
        const fkgp_dtype op = o.op_precision == FKGP_OP_STATS ? h->dt : FKGP_F64;
        const size_t need = solve_scratch_bytes(h, op);
        if (need > kNoAllocScratchBytes) {
            set_error("fkgp_solve_noalloc: this grid needs " + std::to_string(need) +
                      " bytes of workspace, more than the " +
                      std::to_string(kNoAllocScratchBytes) +
                      " bytes of its fixed workspace (use fkgp_solve)");
            return FKGP_EINVAL;
        }
        unsigned char* base = nullptr;
        st = noalloc_scratch(&base);
        if (st != FKGP_OK) return st;
        return solve_impl(h, hyp, rhs_grid, out, o.tol, o.maxiter, op, info,
                          static_cast<hipStream_t>(stream), base, kNoAllocScratchBytes);
    });
}

fkgp_status fkgp_interpolate(const fkgp_handle* h, const double* mean_grid,
                             const void* const* xq, int64_t nq, fkgp_dtype in, double* out,
                             void* stream) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!h || !mean_grid || (nq > 0 && (!xq || !out))) {
            set_error("NULL argument");
            return FKGP_EINVAL;
        }
        if (nq < 0) {
            set_error("nq must be >= 0");
            return FKGP_EINVAL;
        }
        if (nq > 0)
            for (int k = 0; k < h->g.d; ++k)
                if (!xq[k]) {
                    set_error("xq[k] is NULL");
                    return FKGP_EINVAL;
                }
        hipStream_t s = static_cast<hipStream_t>(stream);
        unsigned long long* bad = nullptr;
        const DevAlloc dalloc = current_alloc();
        FKGP_HIP(dev_malloc(dalloc, reinterpret_cast<void**>(&bad), sizeof(unsigned long long), s));
        FKGP_HIP(hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), s));
        fkgp_status st = interpolate_points(h->g, mean_grid, xq, nq, in, out, bad, s);
        unsigned long long hbad = ~0ull;
        if (st == FKGP_OK)
            FKGP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
        dev_free(dalloc, bad, s);
        FKGP_HIP(hipStreamSynchronize(s));
        if (st != FKGP_OK) return st;
        if (hbad != ~0ull) {
            set_error("query point " + std::to_string(hbad) + " lies outside the interpolable region");
            return FKGP_EOUTOFGRID;
        }
        return FKGP_OK;
    });
}

fkgp_status fkgp_apply_B(const fkgp_handle* h, const fkgp_hypers* hyp, const void* x, void* v,
                         void* u, int k, void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h || !x || !v || k < 1) {
            set_error("invalid argument");
            return FKGP_EINVAL;
        }
        fkgp_status st = check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        Scratch sc(s);
        Spectra sp;
        st = make_spectra(h, hyp, h->dt, -1, sp, sc);
        if (st != FKGP_OK) return st;
        const int64_t halo = dia_halo(h->g);
        const size_t es = dsize(h->dt);
        const int64_t ldx = h->M + 2 * halo;
        unsigned char *xpad, *ubuf = static_cast<unsigned char*>(u);
        FKGP_HIP(sc.get(&xpad, es * ldx * k));
        if (!ubuf) FKGP_HIP(sc.get(&ubuf, es * h->M * k));
        FKGP_HIP(hipMemsetAsync(xpad, 0, es * ldx * k, s));
        for (int r = 0; r < k; ++r)
            FKGP_HIP(hipMemcpyAsync(xpad + (r * ldx + halo) * es,
                                    static_cast<const unsigned char*>(x) + r * h->M * es,
                                    es * h->M, hipMemcpyDeviceToDevice, s));
        const double s2 = hyp->noise_std * hyp->noise_std;
        st = spmv_dia(h->g, h->dt, h->A, xpad, ubuf, k, halo, s);
        if (st != FKGP_OK) return st;
        return kg_apply(h->g, sp, h->dt, ubuf, v, k, hyp->outputscale, x, s2, nullptr, s);
    });
}

fkgp_status fkgp_kg_matvec(const fkgp_handle* h, const fkgp_hypers* hyp, const void* x,
                           void* out, int k, void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h || !x || !out || k < 1) {
            set_error("invalid argument");
            return FKGP_EINVAL;
        }
        fkgp_status st = check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        Scratch sc(s);
        Spectra sp;
        st = make_spectra(h, hyp, h->dt, -1, sp, sc);
        if (st != FKGP_OK) return st;
        return kg_apply(h->g, sp, h->dt, x, out, k, hyp->outputscale, nullptr, 0.0, nullptr, s);
    });
}

fkgp_status fkgp_wtw_matvec(const fkgp_handle* h, const void* xpad, void* u, int k,
                            fkgp_dtype xdt, void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h || !xpad || !u || k < 1) {
            set_error("invalid argument");
            return FKGP_EINVAL;
        }
        if (xdt != h->dt && !(h->dt == FKGP_F32 && xdt == FKGP_F64)) {
            set_error("vector dtype must be the stats dtype or FKGP_F64");
            return FKGP_EINVAL;
        }
        return spmv_dia_any(h->g, h->dt, xdt, h->A, h->bmask, xpad, u, k, dia_halo(h->g), nullptr,
                            static_cast<hipStream_t>(stream));
    });
}

fkgp_status fkgp_wtw_matvec_dot(const fkgp_handle* h, const void* xpad, void* u,
                                fkgp_dtype xdt, double* dot, int reps, void* stream) {
    return guarded([&]() -> fkgp_status {
        if (!h || !xpad || !u || !dot || reps < 1) {
            set_error("invalid argument");
            return FKGP_EINVAL;
        }
        if (xdt != FKGP_F64) {
            set_error("fkgp_wtw_matvec_dot takes FP64 vectors (those of the FP64-arithmetic CG)");
            return FKGP_EINVAL;
        }
        hipStream_t st = static_cast<hipStream_t>(stream);
        Scratch sc(st);
        CgState* cs = nullptr;
        double* partials = nullptr;
        unsigned* tickets = nullptr;
        const int nb = red_blocks(h->M);
        FKGP_HIP(sc.get(&cs, 1));
        FKGP_HIP(sc.get(&partials, std::max<int64_t>(kRedMaxBlocks, spmv_dot_parts(h->g))));
        FKGP_HIP(sc.get(&tickets, 1));
        CgState init{};
        init.eps = -1.0;   // never "converged": every launch runs
        FKGP_HIP(hipMemcpyAsync(cs, &init, sizeof(CgState), hipMemcpyHostToDevice, st));
        FKGP_HIP(hipMemsetAsync(tickets, 0, sizeof(unsigned), st));
        const LastBlockRed lb{partials, tickets, cs, FIN_RHO};
        const int64_t halo = dia_halo(h->g);
        for (int r = 0; r < reps; ++r) {
            int np = 0;
            fkgp_status rs = spmv_dia_any(h->g, h->dt, xdt, h->A, h->bmask, xpad, u, 1, halo,
                                          &cs->done, st, partials, &np, &lb);
            if (rs != FKGP_OK) return rs;
            if (np == 0) {   // untiled product: separate dot and finalisation
                const double* x = static_cast<const double*>(xpad) + halo;
                dot_partial<double><<<nb, kRedBlock, 0, st>>>(static_cast<const double*>(u), x,
                                                              h->M, partials, nullptr);
                finalize<<<1, kRedBlock, 0, st>>>(partials, nb, cs, FIN_RHO);
                FKGP_HIP(hipGetLastError());
            }
        }
        FKGP_HIP(hipMemcpyAsync(dot, &cs->rho, sizeof(double), hipMemcpyDeviceToDevice, st));
        return FKGP_OK;
    });
}

}  // extern "C"

namespace {

// Host copy into pinned staging on several threads (one thread moves only a
// few GB/s from pageable memory).
void parallel_copy(unsigned char* dst, const unsigned char* src, size_t bytes) {
    const size_t kMinPiece = size_t(4) << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(std::min<size_t>(hw, 16), (bytes + kMinPiece - 1) / kMinPiece);
    if (nt <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t piece = (bytes + nt - 1) / nt;
    std::vector<std::thread> ts;
    for (size_t t = 1; t < nt; ++t) {
        const size_t b = t * piece, e = std::min(bytes, b + piece);
        if (b < e) ts.emplace_back([=] { std::memcpy(dst + b, src + b, e - b); });
    }
    std::memcpy(dst, src, std::min(bytes, piece));
    for (auto& t : ts) t.join();
}

}  // namespace

extern "C" {

fkgp_status fkgp_precompute_host(const fkgp_grid* grid, const void* const* x, const void* y,
                                 int64_t n, fkgp_dtype in, const fkgp_precompute_opts* opts,
                                 int64_t chunk, void* stream, fkgp_handle** out) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!out) {
            set_error("out is NULL");
            return FKGP_EINVAL;
        }
        *out = nullptr;
        GridDev g;
        int64_t M;
        fkgp_status st = grid_from_abi(grid, g, M);
        if (st != FKGP_OK) return st;
        if (n < 0 || n >= (int64_t(1) << 40)) {
            set_error("n must be in [0, 2^40)");
            return FKGP_EINVAL;
        }
        if (in != FKGP_F32 && in != FKGP_F64) {
            set_error("input dtype must be FKGP_F32 or FKGP_F64");
            return FKGP_EINVAL;
        }
        if (n > 0) {
            if (!x || !y) {
                set_error("x and y must be non-NULL when n > 0");
                return FKGP_EINVAL;
            }
            for (int k = 0; k < g.d; ++k)
                if (!x[k]) {
                    set_error("x[k] is NULL");
                    return FKGP_EINVAL;
                }
        }
        fkgp_precompute_opts o{FKGP_F32, 0, 0, 0, FKGP_INTERP_CUBIC};
        if (opts) o = *opts;
        if (o.interp != FKGP_INTERP_CUBIC && o.interp != FKGP_INTERP_LINEAR) {
            set_error("interp must be FKGP_INTERP_CUBIC or FKGP_INTERP_LINEAR");
            return FKGP_EINVAL;
        }
        g.interp = o.interp;
        if (o.stats_dtype != FKGP_F32 && o.stats_dtype != FKGP_F64) {
            set_error("stats dtype must be FKGP_F32 or FKGP_F64");
            return FKGP_EINVAL;
        }
        if (o.keep_points != 0) {
            set_error("the streamed precompute keeps no points");
            return FKGP_EINVAL;
        }
        if (o.n_probes < 0 || o.n_probes > kMaxProbes) {
            set_error("n_probes must be in [0, 31]");
            return FKGP_EINVAL;
        }
        if (chunk == 0) chunk = int64_t(1) << 24;
        if (chunk < 1 || chunk >= (int64_t(1) << 31) - 1) {
            set_error("chunk must be in [1, 2^31 - 1) points (0: 2^24)");
            return FKGP_EINVAL;
        }
        for (int k = 0; k < g.d; ++k)
            if (circulant_log2(g.m[k]) > kMaxLineLog2) {
                set_error("grid dimension longer than 65536 nodes is not supported");
                return FKGP_EINVAL;
            }
        hipStream_t s = static_cast<hipStream_t>(stream);
        fkgp_handle* h = new fkgp_handle();
        h->g = g;
        h->n = n;
        h->M = M;
        h->NB = 1;
        for (int k = 0; k < g.d; ++k) h->NB *= 7;
        h->dt = o.stats_dtype;
        h->nprobe = o.n_probes;
        h->seed = o.probe_seed;
        // resources of the stream: released on every exit path
        const size_t es = in == FKGP_F32 ? 4 : 8;
        const int nplanes = g.d + 1;
        const int64_t cpts = std::min<int64_t>(chunk, std::max<int64_t>(n, 1));
        struct Res {
            unsigned char* pinned[2] = {nullptr, nullptr};
            unsigned char* devbuf = nullptr;
            double* acc = nullptr;
            hipStream_t cs = nullptr;
            hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
            hipStream_t s = nullptr;
            DevAlloc a = current_alloc();
            ~Res() {
                (void)hipStreamSynchronize(s);
                if (cs) (void)hipStreamSynchronize(cs);
                for (int i = 0; i < 2; ++i) {
                    if (pinned[i]) (void)hipHostFree(pinned[i]);
                    if (copied[i]) (void)hipEventDestroy(copied[i]);
                    if (used[i]) (void)hipEventDestroy(used[i]);
                }
                dev_free(a, devbuf, s);
                dev_free(a, acc, s);
                if (cs) (void)hipStreamDestroy(cs);
                (void)hipStreamSynchronize(s);
            }
        } res;
        res.s = s;
        auto fail = [&](fkgp_status e) {
            free_handle(h);
            return e;
        };
        hipError_t e;
        st = alloc_handle_arrays(h, s);
        if (st != FKGP_OK) return fail(st);
        unsigned long long* bad = reinterpret_cast<unsigned long long*>(h->yty_dev + 1);
        (void)hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), s);
        (void)hipMemsetAsync(h->bmask, 0, sizeof(uint32_t) * (size_t)mask_words(M), s);
        (void)hipMemsetAsync(h->yty_dev + 3, 0, sizeof(double), s);
        StatsOut so{h->A, h->wty, h->sketches, h->yty_dev, h->bmask,
                    reinterpret_cast<unsigned long long*>(h->yty_dev + 2),
                    reinterpret_cast<unsigned long long*>(h->yty_dev + 3), nullptr, nullptr,
                    nullptr};
        if (n <= chunk) {   // one piece: the one-shot precompute from a device copy
            if ((e = dev_malloc(res.a, reinterpret_cast<void**>(&res.devbuf),
                                es * nplanes * (size_t)cpts, s)) != hipSuccess)
                return fail(hip_fail(e, "device allocation (points)"));
            const void* xd[3] = {nullptr, nullptr, nullptr};
            for (int k = 0; k < nplanes && n > 0; ++k) {
                const void* src = k < g.d ? x[k] : y;
                if ((e = hipMemcpyAsync(res.devbuf + es * k * (size_t)cpts, src, es * (size_t)n,
                                        hipMemcpyHostToDevice, s)) != hipSuccess)
                    return fail(hip_fail(e, "hipMemcpyAsync(points)"));
                if (k < g.d) xd[k] = res.devbuf + es * k * (size_t)cpts;
            }
            st = run_precompute(g, xd, res.devbuf + es * g.d * (size_t)cpts, n, in, h->dt,
                                h->nprobe, h->seed, so, bad, s);
        } else {
            int64_t ncells = 1;
            for (int k = 0; k < g.d; ++k) ncells *= g.nc[k];
            int NR = 1;
            for (int k = 0; k < g.d; ++k) NR *= 4;
            NR *= 1 + h->nprobe;   // response moments of y and of every probe
            const size_t nacc = (size_t)ncells * (h->NB + NR + 1);
            if ((e = dev_malloc(res.a, reinterpret_cast<void**>(&res.acc), sizeof(double) * nacc,
                                s)) != hipSuccess ||
                (e = dev_malloc(res.a, reinterpret_cast<void**>(&res.devbuf),
                                2 * es * nplanes * (size_t)cpts, s)) != hipSuccess)
                return fail(hip_fail(e, "device allocation (chunk buffers)"));
            for (int i = 0; i < 2; ++i)
                if ((e = hipHostMalloc(&res.pinned[i], es * nplanes * (size_t)cpts,
                                       hipHostMallocDefault)) != hipSuccess ||
                    (e = hipEventCreateWithFlags(&res.copied[i], hipEventDisableTiming)) !=
                        hipSuccess ||
                    (e = hipEventCreateWithFlags(&res.used[i], hipEventDisableTiming)) != hipSuccess)
                    return fail(hip_fail(e, "chunk staging"));
            if ((e = hipStreamCreateWithFlags(&res.cs, hipStreamNonBlocking)) != hipSuccess)
                return fail(hip_fail(e, "hipStreamCreateWithFlags"));
            ChunkCtl cc{res.acc, res.acc + (size_t)ncells * h->NB,
                        res.acc + (size_t)ncells * (h->NB + NR), 1, 0, 0};
            const int64_t nchunks = (n + chunk - 1) / chunk;
            for (int64_t c = 0; c < nchunks && st == FKGP_OK; ++c) {
                const int slot = (int)(c & 1);
                const int64_t base = c * chunk;
                const int64_t cn = std::min(chunk, n - base);
                // the slot's previous chunk has left the staging and device buffers
                if (c >= 2 && (e = hipEventSynchronize(res.used[slot])) != hipSuccess)
                    return fail(hip_fail(e, "hipEventSynchronize"));
                unsigned char* pin = res.pinned[slot];
                unsigned char* dev = res.devbuf + (size_t)slot * es * nplanes * cpts;
                for (int k = 0; k < nplanes; ++k) {
                    const unsigned char* src =
                        static_cast<const unsigned char*>(k < g.d ? x[k] : y) + es * base;
                    parallel_copy(pin + es * k * (size_t)cpts, src, es * (size_t)cn);
                }
                for (int k = 0; k < nplanes; ++k)
                    if ((e = hipMemcpyAsync(dev + es * k * (size_t)cpts, pin + es * k * (size_t)cpts,
                                            es * (size_t)cn, hipMemcpyHostToDevice, res.cs)) !=
                        hipSuccess)
                        return fail(hip_fail(e, "hipMemcpyAsync(chunk)"));
                if ((e = hipEventRecord(res.copied[slot], res.cs)) != hipSuccess ||
                    (e = hipStreamWaitEvent(s, res.copied[slot], 0)) != hipSuccess)
                    return fail(hip_fail(e, "chunk ordering"));
                const void* xd[3] = {nullptr, nullptr, nullptr};
                for (int k = 0; k < g.d; ++k) xd[k] = dev + es * k * (size_t)cpts;
                cc.first = c == 0 ? 1 : 0;
                cc.last = c == nchunks - 1 ? 1 : 0;
                cc.idx_base = base;
                st = run_precompute(g, xd, dev + es * g.d * (size_t)cpts, cn, in, h->dt,
                                    h->nprobe, h->seed, so, bad, s, &cc);
                if (st == FKGP_OK && (e = hipEventRecord(res.used[slot], s)) != hipSuccess)
                    return fail(hip_fail(e, "hipEventRecord"));
            }
        }
        unsigned long long hbad = ~0ull;
        double back[4] = {0.0, 0.0, 0.0, 0.0};
        if (st == FKGP_OK) {
            if ((e = hipMemcpyAsync(back, h->yty_dev, sizeof(back), hipMemcpyDeviceToHost, s)) !=
                hipSuccess)
                st = hip_fail(e, "hipMemcpyAsync(y^T y, flag)");
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess && st == FKGP_OK)
            st = hip_fail(e, "hipStreamSynchronize");
        if (st != FKGP_OK) return fail(st);
        h->yty = back[0];
        std::memcpy(&hbad, &back[1], sizeof(hbad));
        unsigned long long nzb = 0;
        std::memcpy(&nzb, &back[2], sizeof(nzb));
        h->nzblocks = (int64_t)nzb;
        unsigned long long nnz = 0;
        std::memcpy(&nnz, &back[3], sizeof(nnz));
        h->nnz = (int64_t)nnz;
        if (hbad != ~0ull) {
            set_error("point " + std::to_string(hbad) + " lies outside the interpolable region");
            return fail(FKGP_EOUTOFGRID);
        }
        *out = h;
        return FKGP_OK;
    });
}

fkgp_status fkgp_save(const fkgp_handle* h, const char* path, void* stream) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!h || !path) {
            set_error("handle and path must be non-NULL");
            return FKGP_EINVAL;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        StatsFileHeader hd{};
        std::memcpy(hd.magic, "FKGPSTAT", 8);
        hd.version = kStatsFileVersion;
        hd.d = h->g.d;
        for (int k = 0; k < h->g.d; ++k) {
            hd.m[k] = h->g.m[k];
            hd.origin[k] = h->g.g0[k];
            hd.spacing[k] = h->g.h[k];
        }
        hd.n = h->n;
        hd.stats_dtype = h->dt;
        hd.nprobe = h->nprobe;
        hd.seed = h->seed;
        hd.yty = h->yty;
        hd.nzblocks = h->nzblocks;
        hd.interp = h->g.interp;
        hd.reserved = 0;
        const StatsSections sec = stats_sections(h);
        std::vector<unsigned char> buf(sec.total());
        unsigned char* p = buf.data();
        FKGP_HIP(hipMemcpyAsync(p, h->A, sec.a, hipMemcpyDeviceToHost, s));
        FKGP_HIP(hipMemcpyAsync(p + sec.a, h->bmask, sec.mask, hipMemcpyDeviceToHost, s));
        FKGP_HIP(hipMemcpyAsync(p + sec.a + sec.mask, h->wty, sec.wty, hipMemcpyDeviceToHost, s));
        if (sec.sk)
            FKGP_HIP(hipMemcpyAsync(p + sec.a + sec.mask + sec.wty, h->sketches, sec.sk,
                                    hipMemcpyDeviceToHost, s));
        FKGP_HIP(hipStreamSynchronize(s));
        FILE* f = std::fopen(path, "wb");
        if (!f) {
            set_error(std::string("cannot open ") + path + " for writing");
            return FKGP_EINVAL;
        }
        const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 &&
                        (buf.empty() || std::fwrite(buf.data(), buf.size(), 1, f) == 1);
        const bool closed = std::fclose(f) == 0;
        if (!ok || !closed) {
            set_error(std::string("write to ") + path + " failed");
            return FKGP_EINVAL;
        }
        return FKGP_OK;
    });
}

fkgp_status fkgp_load(const char* path, void* stream, fkgp_handle** out) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!path || !out) {
            set_error("path and out must be non-NULL");
            return FKGP_EINVAL;
        }
        *out = nullptr;
        FILE* f = std::fopen(path, "rb");
        if (!f) {
            set_error(std::string("cannot open ") + path);
            return FKGP_EINVAL;
        }
        struct Closer {
            FILE* f;
            ~Closer() { std::fclose(f); }
        } closer{f};
        StatsFileHeader hd{};
        if (std::fread(&hd, sizeof(hd), 1, f) != 1 || std::memcmp(hd.magic, "FKGPSTAT", 8) != 0 ||
            hd.version != kStatsFileVersion) {
            set_error(std::string(path) + " is not a statistics file of this version");
            return FKGP_EINVAL;
        }
        fkgp_grid gr{};
        gr.d = hd.d;
        for (int k = 0; k < 3; ++k) {
            gr.m[k] = hd.m[k];
            gr.origin[k] = hd.origin[k];
            gr.spacing[k] = hd.spacing[k];
        }
        GridDev g;
        int64_t M;
        fkgp_status st = grid_from_abi(&gr, g, M);
        if (st != FKGP_OK) return st;
        if (hd.n < 0 || (hd.stats_dtype != FKGP_F32 && hd.stats_dtype != FKGP_F64) ||
            hd.nprobe < 0 || hd.nprobe > kMaxProbes || hd.nzblocks < 0 ||
            (hd.interp != FKGP_INTERP_CUBIC && hd.interp != FKGP_INTERP_LINEAR)) {
            set_error(std::string(path) + ": corrupt header");
            return FKGP_EINVAL;
        }
        g.interp = hd.interp;
        for (int k = 0; k < g.d; ++k)
            if (circulant_log2(g.m[k]) > kMaxLineLog2) {
                set_error(std::string(path) + ": grid dimension longer than 65536 nodes");
                return FKGP_EINVAL;
            }
        fkgp_handle* h = new fkgp_handle();
        auto fail = [&](fkgp_status e) {
            free_handle(h);
            return e;
        };
        h->g = g;
        h->n = hd.n;
        h->M = M;
        h->NB = 1;
        for (int k = 0; k < g.d; ++k) h->NB *= 7;
        h->dt = (fkgp_dtype)hd.stats_dtype;
        h->nprobe = hd.nprobe;
        h->seed = hd.seed;
        h->yty = hd.yty;
        h->nzblocks = hd.nzblocks;
        const StatsSections sec = stats_sections(h);
        std::vector<unsigned char> buf(sec.total());
        if (!buf.empty() && std::fread(buf.data(), buf.size(), 1, f) != 1) {
            set_error(std::string(path) + " is truncated");
            return fail(FKGP_EINVAL);
        }
        unsigned char extra;
        if (std::fread(&extra, 1, 1, f) != 0) {
            set_error(std::string(path) + " is longer than its header says");
            return fail(FKGP_EINVAL);
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        st = alloc_handle_arrays(h, s);
        if (st != FKGP_OK) return fail(st);
        const unsigned char* p = buf.data();
        hipError_t e = hipSuccess;
        auto put = [&](void* dst, const void* src, size_t bytes) {
            if (e == hipSuccess && bytes)
                e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
        };
        put(h->A, p, sec.a);
        put(h->bmask, p + sec.a, sec.mask);
        put(h->wty, p + sec.a + sec.mask, sec.wty);
        put(h->sketches, p + sec.a + sec.mask + sec.wty, sec.sk);
        const double tail[4] = {hd.yty, 0.0, 0.0, 0.0};
        put(h->yty_dev, tail, sizeof(tail));
        unsigned long long* nnz_dev = reinterpret_cast<unsigned long long*>(h->yty_dev + 3);
        if (e == hipSuccess && count_wtw_nonzeros(h->dt, h->A, dia_elems(M, h->NB), nnz_dev, s) !=
                                   FKGP_OK)
            e = hipErrorLaunchFailure;
        unsigned long long nnz = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nnz, nnz_dev, sizeof(nnz), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // buf and tail leave scope
        if (e != hipSuccess) return fail(hip_fail(e, "loading statistics"));
        h->nnz = (int64_t)nnz;
        *out = h;
        return FKGP_OK;
    });
}

fkgp_status fkgp_ski_solve(const fkgp_handle* h, const fkgp_hypers* hyp, double tol,
                           int maxiter, double* mean_grid, fkgp_solve_info* info,
                           void* stream) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!h || !mean_grid) {
            set_error("handle and mean_grid must be non-NULL");
            return FKGP_EINVAL;
        }
        if (!h->pay) {
            set_error("the handle keeps no points: precompute with keep_points = 1");
            return FKGP_EINVAL;
        }
        fkgp_status st = check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        if (!(tol >= 0.0) || maxiter < 0) {
            set_error("tol must be >= 0 and maxiter >= 0");
            return FKGP_EINVAL;
        }
        return ski_solve_impl(h, hyp, tol, maxiter, mean_grid, info,
                              static_cast<hipStream_t>(stream));
    });
}

fkgp_status fkgp_set_allocator(const fkgp_allocator* a) {
    return guarded([&]() -> fkgp_status {
        set_error("");
        if (!a) {
            set_alloc(DevAlloc{});
            return FKGP_OK;
        }
        if (!a->alloc || !a->free) {
            set_error("allocator needs both alloc and free");
            return FKGP_EINVAL;
        }
        DevAlloc d;
        d.alloc = a->alloc;
        d.free = a->free;
        d.ctx = a->ctx;
        set_alloc(d);
        return FKGP_OK;
    });
}

void fkgp_destroy(fkgp_handle* h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_handle(h);
}

}  // extern "C"

// ===========================================================================
// Log marginal likelihood and gradient.
//
// logdet(A), A = W K_G W^T + s2 I, by stochastic Lanczos quadrature: for each
// Rademacher probe z_j the factorized CG from x_0 = 0 (Claims 3 and 4; the
// iterates are r = W r_hat + c_r z_j, p = W p_hat + c_p z_j, x = W x_hat +
// c_x z_j and only W^T z_j, ||z_j||^2 = n enter) gives CG coefficients whose
// Lanczos tridiagonal T_j yields ||z_j||^2 e_1^T log(T_j) e_1.  The same probe
// solves x_j = A^{-1} z_j give the Hutchinson trace of the gradient
//   g_theta = 1/2 [ x_y^T dA x_y - (1/N) sum_j x_j^T dA z_j ],
// where x^T (W dK W^T) z = (W^T x)^T dK (W^T z) and dA/dlog sigma = 2 s2 I.
// ===========================================================================
namespace fkgp {
namespace {

// Right-hand side j: ||b||^2 = bb[j] when given (grid right-hand sides
// b = W v), else n (a Rademacher probe).  A grid right-hand side starts as
// r = W v (c_r = c_p = 0, r_hat = v), so every later residual stays W r_hat
// and ||r||^2 = r_hat . W^T W r_hat has no cancelling b-terms; a probe
// starts as r = z (r_hat = 0, c_r = c_p = 1).
__global__ void probe_init(PState* ps, int N, double n, double tol,
                           const double* __restrict__ bb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double b2 = bb ? bb[j] : n;
    PState s{};
    s.bb = b2;
    s.rho = b2;
    s.cr = bb ? 0.0 : 1.0;
    s.cp = bb ? 0.0 : 1.0;
    s.eps = tol * tol * b2;
    s.done = b2 > 0 ? 0 : 1;
    ps[j] = s;
}

// Direction update of the previous iteration, s_p = u_r + beta s_p and
// z_p = v_r + beta z_p (beta = 0 and u_r = v_r = 0 before the first
// iteration), then ap = z_p + c_p kappa_b (compressed A p) and the partials
// of s_p.ap and ap.b_hat.
__global__ __launch_bounds__(kRedBlock) void probe_ap(const PState* __restrict__ ps,
                                                      double* __restrict__ zp,
                                                      const double* __restrict__ kb,
                                                      double* __restrict__ sp,
                                                      const double* __restrict__ bh,
                                                      const double* __restrict__ ur,
                                                      const double* __restrict__ vr,
                                                      double* __restrict__ ap, int64_t M,
                                                      double* __restrict__ partials) {
    const int j = blockIdx.y;
    if (ps[j].done) return;
    __shared__ double sh[kRedBlock];
    const double cp = ps[j].cp, beta = ps[j].beta;
    const int64_t o = (int64_t)j * M;
    double d1 = 0.0, d2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock) {
        const double sn = fma(beta, sp[o + i], ur[o + i]);
        const double zn = fma(beta, zp[o + i], vr[o + i]);
        sp[o + i] = sn;
        zp[o + i] = zn;
        const double a = fma(cp, kb[o + i], zn);
        ap[o + i] = a;
        d1 = fma(sn, a, d1);
        d2 = fma(a, bh[o + i], d2);
    }
    const double t1 = block_sum(d1, sh);
    const double t2 = block_sum(d2, sh);
    if (threadIdx.x == 0) {
        partials[((int64_t)j * gridDim.x + blockIdx.x) * 2] = t1;
        partials[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 1] = t2;
    }
}

__device__ inline void sum_pairs(const double* partials, int j, int nbv, double* sh, double& a,
                                 double& b) {
    double x = 0.0, y = 0.0;
    for (int i = threadIdx.x; i < nbv; i += kRedBlock) {
        x += partials[((int64_t)j * nbv + i) * 2];
        y += partials[((int64_t)j * nbv + i) * 2 + 1];
    }
    a = block_sum(x, sh);
    b = block_sum(y, sh);
}

// alpha = rho / <p, A p> (Claim 4), scalar updates of x and r.
__global__ __launch_bounds__(kRedBlock) void probe_fin_ap(PState* ps,
                                                          const double* __restrict__ partials,
                                                          int nbv, double s2,
                                                          double* __restrict__ alphas) {
    const int j = blockIdx.x;
    if (ps[j].done) return;
    __shared__ double sh[kRedBlock];
    double d1, d2;
    sum_pairs(partials, j, nbv, sh, d1, d2);
    if (threadIdx.x != 0) return;
    PState s = ps[j];
    const double apc = s2 * s.cp;
    const double pap = d1 + apc * s.pb + s.cp * d2 + s.cp * apc * s.bb;
    const double alpha = s.rho / pap;
    if (!isfinite(alpha)) {
        ps[j].done = 2;
        return;
    }
    if (s.iters < kMaxLanczos) alphas[j * kMaxLanczos + s.iters] = alpha;
    s.alpha = alpha;
    s.cx += alpha * s.cp;
    s.cr -= alpha * apc;
    ps[j] = s;
}

// u_x += alpha s_p; r_hat -= alpha ap; rpad = r_hat
__global__ void probe_upd_r(const PState* __restrict__ ps, double* __restrict__ ux,
                            const double* __restrict__ sp, double* __restrict__ rh,
                            const double* __restrict__ ap, double* __restrict__ rpad, int64_t M,
                            int64_t ldx, int64_t halo) {
    const int j = blockIdx.y;
    if (ps[j].done) return;
    const double a = ps[j].alpha;
    const int64_t o = (int64_t)j * M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        ux[o + i] = fma(a, sp[o + i], ux[o + i]);
        const double r = fma(-a, ap[o + i], rh[o + i]);
        rh[o + i] = r;
        rpad[(int64_t)j * ldx + halo + i] = r;
    }
}

// partials of r_hat.u_r and r_hat.b_hat
__global__ __launch_bounds__(kRedBlock) void probe_dot_r(const PState* __restrict__ ps,
                                                         const double* __restrict__ rh,
                                                         const double* __restrict__ ur,
                                                         const double* __restrict__ bh,
                                                         int64_t M,
                                                         double* __restrict__ partials) {
    const int j = blockIdx.y;
    if (ps[j].done) return;
    __shared__ double sh[kRedBlock];
    const int64_t o = (int64_t)j * M;
    double d1 = 0.0, d2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock) {
        d1 = fma(rh[o + i], ur[o + i], d1);
        d2 = fma(rh[o + i], bh[o + i], d2);
    }
    const double t1 = block_sum(d1, sh);
    const double t2 = block_sum(d2, sh);
    if (threadIdx.x == 0) {
        partials[((int64_t)j * gridDim.x + blockIdx.x) * 2] = t1;
        partials[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 1] = t2;
    }
}

// rho' = <r, r> (Claim 4); stop test; beta and the scalar parts of p (the
// vector parts are updated by the next probe_ap).
__global__ __launch_bounds__(kRedBlock) void probe_fin_r(PState* ps,
                                                         const double* __restrict__ partials,
                                                         int nbv,
                                                         double* __restrict__ betas) {
    const int j = blockIdx.x;
    if (ps[j].done) return;
    __shared__ double sh[kRedBlock];
    double d1, d2;
    sum_pairs(partials, j, nbv, sh, d1, d2);
    if (threadIdx.x != 0) return;
    PState s = ps[j];
    const double rho_new = d1 + 2.0 * s.cr * d2 + s.cr * s.cr * s.bb;
    s.iters += 1;
    if (!(rho_new > s.eps)) {
        s.done = 1;
        s.rho = rho_new;
        ps[j] = s;
        return;
    }
    const double beta = rho_new / s.rho;
    if (s.iters - 1 < kMaxLanczos) betas[j * kMaxLanczos + s.iters - 1] = beta;
    s.beta = beta;
    s.rho = rho_new;
    s.pb = d2 + beta * s.pb;
    s.cp = s.cr + beta * s.cp;
    ps[j] = s;
}

// W^T x_j = u_x + c_x b_hat
__global__ void probe_wtx(const PState* __restrict__ ps, const double* __restrict__ ux,
                          const double* __restrict__ bh, double* __restrict__ out, int64_t M) {
    const int j = blockIdx.y;
    const double c = ps[j].cx;
    const int64_t o = (int64_t)j * M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        out[o + i] = fma(c, bh[o + i], ux[o + i]);
}

// e_1^T log(T) e_1 for the Lanczos tridiagonal of CG coefficients
// (T_ii = 1/alpha_i + beta_{i-1}/alpha_{i-1}, T_{i,i+1} = sqrt(beta_i)/alpha_i)
// by the implicit symmetric QL iteration with Wilkinson-type shifts, tracking
// only the first row of the eigenvector matrix (Gauss quadrature weights).
// One thread per probe, FP64.
__device__ double lanczos_logdet_one(const PState* __restrict__ ps,
                                     const double* __restrict__ alphas,
                                     const double* __restrict__ betas, int j, int steps) {
    int k = min(steps, min(ps[j].iters, kMaxLanczos));
    double dg[kMaxLanczos], e[kMaxLanczos], q[kMaxLanczos];
    const double* a = alphas + j * kMaxLanczos;
    const double* b = betas + j * kMaxLanczos;
    for (int i = 0; i < k; ++i) {
        dg[i] = 1.0 / a[i] + (i > 0 ? b[i - 1] / a[i - 1] : 0.0);
        e[i] = (i + 1 < k) ? sqrt(b[i]) / a[i] : 0.0;
        q[i] = (i == 0) ? 1.0 : 0.0;
    }
    bool ok = k > 0;
    for (int l = 0; l < k && ok; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < k - 1; ++m) {
                const double dd = fabs(dg[m]) + fabs(dg[m + 1]);
                if (fabs(e[m]) <= 8.9e-16 * dd) break;   // 4 ulp of 1.0
            }
            if (m == l) break;
            if (++iter > 60) {
                ok = false;
                break;
            }
            double g = (dg[l + 1] - dg[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = dg[m] - dg[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                const double f = s * e[i];
                const double bb = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    dg[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = dg[i + 1] - p;
                r = (dg[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                dg[i + 1] = g + p;
                g = c * r - bb;
                const double fq = q[i + 1];
                q[i + 1] = s * q[i] + c * fq;
                q[i] = c * q[i] - s * fq;
            }
            if (deflated) continue;
            dg[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += q[i] * q[i] * log(dg[i]);
    return ok ? acc : NAN;
}

__global__ void lanczos_logdet(const PState* __restrict__ ps, const double* __restrict__ alphas,
                               const double* __restrict__ betas, int N, int steps,
                               double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) out[j] = lanczos_logdet_one(ps, alphas, betas, j, steps);
}

// The same for many problems in one launch (problem blockIdx.y).
struct LogdetJob {
    const PState* ps;
    const double* alphas;
    const double* betas;
    double* out;
    int N;
};
__global__ void lanczos_logdet_multi(const LogdetJob* __restrict__ jobs, int steps) {
    const LogdetJob jb = jobs[blockIdx.y];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < jb.N) jb.out[j] = lanczos_logdet_one(jb.ps, jb.alphas, jb.betas, j, steps);
}

// dots[r] = A[r] . B[r] for k pairs of FP64 vectors of length M.
__global__ __launch_bounds__(kRedBlock) void batched_dot(const double* __restrict__ A,
                                                         const double* __restrict__ B,
                                                         int64_t M, double* __restrict__ partials) {
    __shared__ double sh[kRedBlock];
    const int64_t o = (int64_t)blockIdx.y * M;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * kRedBlock)
        acc = fma(A[o + i], B[o + i], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedBlock) void batched_dot_fin(const double* __restrict__ partials,
                                                             int nbv, double* __restrict__ out) {
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nbv; i += kRedBlock)
        acc += partials[(int64_t)blockIdx.x * nbv + i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

int vec_blocks(int64_t M) {
    int64_t b = (M + 4 * kRedBlock - 1) / (4 * kRedBlock);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

fkgp_status dots_dev(const double* A, const double* B, int64_t M, int k, double* partials,
                     double* out, hipStream_t st) {
    const int nbv = vec_blocks(M);
    batched_dot<<<dim3(nbv, k), kRedBlock, 0, st>>>(A, B, M, partials);
    batched_dot_fin<<<k, kRedBlock, 0, st>>>(partials, nbv, out);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// Pinned snapshot slots (2 x kSnapStates states) and two events per host
// thread and device for the probe solver's convergence checks.
constexpr int kSnapStates = 64;
struct ProbeSnap {
    PState* host = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

hipError_t probe_snap_get(ProbeSnap& out) {
    thread_local ProbeSnap cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    ProbeSnap& c = cache[dev];
    if (!c.host) {
        e = hipHostMalloc(reinterpret_cast<void**>(&c.host), 2 * kSnapStates * sizeof(PState),
                          hipHostMallocDefault);
        if (e != hipSuccess) {
            c.host = nullptr;
            return e;
        }
        for (int i = 0; i < 2; ++i) {
            e = hipEventCreateWithFlags(&c.ev[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
    }
    out = c;
    return hipSuccess;
}

// Factorized CG from x_0 = 0 for N right-hand sides b_j at once, given
// b_hat_j = W^T b_j (bh [N][M]).  Rademacher probes (v = null): ||z_j||^2 = n.
// Grid right-hand sides b_j = W v_j (v0 [N][M], bh = W^T W v, bb_dev [N] =
// v_j . bh_j on the device): the iteration starts from r_hat = v.  Outputs
// W^T x_j (wx [N][M]), the CG coefficients and the final states.
// c_r and rho of every probe after an iteration (residual history)
__global__ void probe_hist(const PState* __restrict__ ps, int N, double* __restrict__ sh) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) {
        sh[2 * j] = ps[j].cr;
        sh[2 * j + 1] = ps[j].rho;
    }
}

// rhist (optional, [khist][N][M]) and shist ([khist][N][2]) receive the
// residuals r_i = W r_hat_i + c_r,i z_j of the first khist iterations
// (r_hat_i, then (c_r,i, ||r_i||^2)); r_0 = z_j: r_hat = 0, c_r = 1, n.
fkgp_status probe_cg(const OpCtx& c, const double* bh, int N, double n, double tol,
                     int maxiter, double* wx, double* alphas, double* betas, PState* ps,
                     Scratch& sc, hipStream_t st, int& iters_max,
                     const double* bb_dev = nullptr, const double* v0 = nullptr,
                     double* rhist = nullptr, double* shist = nullptr, int khist = 0) {
    const fkgp_handle* h = c.h;
    const int64_t M = c.M;
    const int64_t ldx = M + 2 * c.halo;
    double *kb, *ap, *sp, *zp, *ux, *rh, *rpad, *ur, *vr, *partials;
    FKGP_HIP(sc.get(&kb, M * N));
    FKGP_HIP(sc.get(&ap, M * N));
    FKGP_HIP(sc.get(&sp, M * N));
    FKGP_HIP(sc.get(&zp, M * N));
    FKGP_HIP(sc.get(&ux, M * N));
    FKGP_HIP(sc.get(&rh, M * N));
    FKGP_HIP(sc.get(&ur, M * N));
    FKGP_HIP(sc.get(&vr, M * N));
    FKGP_HIP(sc.get(&rpad, ldx * N));
    const int nbv = vec_blocks(M);
    FKGP_HIP(sc.get(&partials, (size_t)2 * nbv * N));
    for (double* v : {sp, zp, ux, rh, ur, vr})
        FKGP_HIP(hipMemsetAsync(v, 0, sizeof(double) * M * N, st));
    FKGP_HIP(hipMemsetAsync(rpad, 0, sizeof(double) * ldx * N, st));
    // kappa_b = K_G W^T z_j (FP64)
    fkgp_status rs = kg_apply(h->g, c.sp64, FKGP_F64, bh, kb, N, c.so, nullptr, 0.0, nullptr, st);
    if (rs != FKGP_OK) return rs;
    if (v0) {
        // r_hat = v, u_r = W^T W v = bh, v_r = K_G u_r + s2 r_hat
        FKGP_HIP(hipMemcpyAsync(rh, v0, sizeof(double) * M * N, hipMemcpyDeviceToDevice, st));
        FKGP_HIP(hipMemcpyAsync(ur, bh, sizeof(double) * M * N, hipMemcpyDeviceToDevice, st));
        rs = kg_apply(h->g, c.sp64, FKGP_F64, bh, vr, N, c.so, v0, c.s2, nullptr, st);
        if (rs != FKGP_OK) return rs;
    }
    probe_init<<<(N + 63) / 64, 64, 0, st>>>(ps, N, n, tol, bb_dev);
    FKGP_HIP(hipGetLastError());
    if (rhist && khist > 0) {
        FKGP_HIP(hipMemsetAsync(rhist, 0, sizeof(double) * M * N, st));
        probe_hist<<<(N + 63) / 64, 64, 0, st>>>(ps, N, shist);
        FKGP_HIP(hipGetLastError());
    }
    const dim3 gv(nbv, N);
    const dim3 ge((unsigned)std::min<int64_t>((M + 255) / 256, 1024), N);
    // pipelined convergence checks, as in run_cg: the states after each
    // batch go to pinned memory while the next batch is queued (converged
    // right-hand sides skip their vector updates)
    if (N > kSnapStates) {
        set_error("too many right-hand sides for one probe solve");
        return FKGP_EINVAL;
    }
    ProbeSnap snapbuf;
    FKGP_HIP(probe_snap_get(snapbuf));
    std::vector<PState> hs(N);
    int launched = 0, slot = 0;
    constexpr int kBatch = 8;
    FKGP_HIP(hipMemcpyAsync(snapbuf.host, ps, sizeof(PState) * N, hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipEventRecord(snapbuf.ev[0], st));
    for (;;) {
        const int next = slot ^ 1;
        const bool queued = launched < maxiter;
        if (queued) {
        const int nit = std::min(kBatch, maxiter - launched);
        for (int it = 0; it < nit; ++it) {
            probe_ap<<<gv, kRedBlock, 0, st>>>(ps, zp, kb, sp, bh, ur, vr, ap, M, partials);
            probe_fin_ap<<<N, kRedBlock, 0, st>>>(ps, partials, nbv, c.s2, alphas);
            probe_upd_r<<<ge, 256, 0, st>>>(ps, ux, sp, rh, ap, rpad, M, ldx, c.halo);
            FKGP_HIP(hipGetLastError());
            rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, rpad, ur, N, c.halo, nullptr, st);
            if (rs != FKGP_OK) return rs;
            rs = kg_apply(h->g, c.sp64, FKGP_F64, ur, vr, N, c.so, rh, c.s2, nullptr, st);
            if (rs != FKGP_OK) return rs;
            probe_dot_r<<<gv, kRedBlock, 0, st>>>(ps, rh, ur, bh, M, partials);
            probe_fin_r<<<N, kRedBlock, 0, st>>>(ps, partials, nbv, betas);
            FKGP_HIP(hipGetLastError());
            const int gi = launched + it + 1;   // index of the residual just formed
            if (rhist && gi < khist) {
                FKGP_HIP(hipMemcpyAsync(rhist + (size_t)gi * N * M, rh, sizeof(double) * M * N,
                                        hipMemcpyDeviceToDevice, st));
                probe_hist<<<(N + 63) / 64, 64, 0, st>>>(ps, N, shist + (size_t)gi * N * 2);
                FKGP_HIP(hipGetLastError());
            }
        }
        launched += nit;
        FKGP_HIP(hipMemcpyAsync(snapbuf.host + (size_t)next * kSnapStates, ps,
                                sizeof(PState) * N, hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipEventRecord(snapbuf.ev[next], st));
        }
        FKGP_HIP(hipEventSynchronize(snapbuf.ev[slot]));
        std::copy(snapbuf.host + (size_t)slot * kSnapStates,
                  snapbuf.host + (size_t)slot * kSnapStates + N, hs.begin());
        bool all = true;
        for (int j = 0; j < N; ++j) all &= hs[j].done != 0;
        if (all || !queued) break;
        slot = next;
    }
    FKGP_HIP(hipStreamSynchronize(st));
    iters_max = 0;
    for (int j = 0; j < N; ++j) {
        iters_max = std::max(iters_max, hs[j].iters);
        if (hs[j].done == 2) {
            set_error("probe CG broke down (non-finite step)");
            return FKGP_EDEVICE;
        }
    }
    probe_wtx<<<ge, 256, 0, st>>>(ps, ux, bh, wx, M);
    FKGP_HIP(hipGetLastError());
    bool conv = true;
    for (int j = 0; j < N; ++j) conv &= hs[j].done == 1;
    return conv ? FKGP_OK : FKGP_ENOTCONV;
}

// MLL and gradient from solved systems: V = [W^T z~, W^T z_0 .. W^T z_{N-1}],
// wx = [W^T z~, W^T x_0 .. W^T x_{N-1}] (x_j = A^{-1} z_j), the probes' CG
// coefficients and states.  V and wx are [N+1][M] device buffers.  The
// device part (mll_post_enqueue) leaves every number the host needs in
// `res` (mll_post_doubles of them): [0] y.mu, [1] mu.(A mu), then per
// theta (log l_k, log s) N + 1 dots, then N dots for the noise, then the N
// Lanczos log-determinant terms (written by the caller when `logdet` is
// false); mll_post_finish turns a host copy of it into the MLL and its
// gradient.  Nothing in between waits for the device.
size_t mll_post_doubles(int d, int N) { return 2 + (size_t)(d + 1) * (N + 1) + 2 * (size_t)N; }

fkgp_status mll_post_enqueue(const OpCtx& c, const fkgp_hypers* hyp, const fkgp_mll_opts& o,
                             const double* V, const double* wx, const double* alphas,
                             const double* betas, const PState* ps, double* res, bool logdet,
                             Scratch& sc, hipStream_t st) {
    const fkgp_handle* h = c.h;
    const int d = h->g.d;
    const int N = h->nprobe;
    const int64_t M = h->M;
    double *DV, *mu, *Amu, *pad64, *dotp;
    FKGP_HIP(sc.get(&DV, M * (N + 1)));
    FKGP_HIP(sc.get(&mu, M));
    FKGP_HIP(sc.get(&Amu, M));
    FKGP_HIP(sc.get(&pad64, M + 2 * c.halo));
    FKGP_HIP(sc.get(&dotp, (size_t)vec_blocks(M) * (N + 1) * 2));
    double* th_dots = res + 2;
    double* s_dots = res + 2 + (size_t)(d + 1) * (N + 1);
    double* ld = s_dots + N;
    fkgp_status rs = kg_apply(h->g, c.sp64, FKGP_F64, V, mu, 1, c.so, nullptr, 0.0, nullptr, st);
    if (rs != FKGP_OK) return rs;
    if (logdet) {
        lanczos_logdet<<<(N + 63) / 64, 64, 0, st>>>(ps, alphas, betas, N, o.lanczos_steps, ld);
        FKGP_HIP(hipGetLastError());
    }
    // y^T A^{-1} y and ||z~||^2 need W^T y . mu and mu . (W^T W mu)
    FKGP_HIP(hipMemsetAsync(pad64, 0, sizeof(double) * (M + 2 * c.halo), st));
    FKGP_HIP(hipMemcpyAsync(pad64 + c.halo, mu, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
    rs = apply_B64(c, pad64, Amu, nullptr, st);
    if (rs != FKGP_OK) return rs;
    rs = dots_dev(h->wty, mu, M, 1, dotp, res, st);
    if (rs != FKGP_OK) return rs;
    rs = dots_dev(mu, Amu, M, 1, dotp, res + 1, st);
    if (rs != FKGP_OK) return rs;
    // theta = log l_k (k < d), log s (k = d): DV = dK [w_y, b_hat_j]
    for (int th = 0; th <= d; ++th) {
        Spectra dsp;
        rs = make_spectra(h, hyp, FKGP_F64, th < d ? th : -1, dsp, sc);
        if (rs != FKGP_OK) return rs;
        rs = kg_apply(h->g, dsp, FKGP_F64, V, DV, N + 1, c.so, nullptr, 0.0, nullptr, st);
        if (rs != FKGP_OK) return rs;
        rs = dots_dev(wx, DV, M, N + 1, dotp, th_dots + (size_t)th * (N + 1), st);
        if (rs != FKGP_OK) return rs;
    }
    // sigma: x_j^T z_j = (n - b_hat_j . K_G W^T x_j) / s2
    rs = kg_apply(h->g, c.sp64, FKGP_F64, wx + M, DV + M, N, c.so, nullptr, 0.0, nullptr, st);
    if (rs != FKGP_OK) return rs;
    return dots_dev(V + M, DV + M, M, N, dotp, s_dots, st);
}

fkgp_status mll_post_finish(const OpCtx& c, const double* hres, double* mll, double* grad,
                            double& logdet_out, double& q_out, const double* tr_exact = nullptr,
                            double* dq_out = nullptr) {
    const fkgp_handle* h = c.h;
    const int d = h->g.d;
    const int N = h->nprobe;
    const double n = (double)h->n;
    const double* th_dots = hres + 2;
    const double* s_dots = hres + 2 + (size_t)(d + 1) * (N + 1);
    const double* hld = s_dots + N;
    std::vector<double> quad(d + 1), tr(d + 1);
    for (int th = 0; th <= d; ++th) {
        const double* hd = th_dots + (size_t)th * (N + 1);
        quad[th] = hd[0];
        double acc = 0.0;
        for (int j = 0; j < N; ++j) acc += hd[1 + j];
        tr[th] = acc / N;
    }
    const double s2 = c.s2;
    const double yty = h->yty;
    const double q = (yty - hres[0]) / s2;
    const double zz = (yty - 2.0 * hres[0] + hres[1]) / (s2 * s2);
    double logdet = 0.0;
    for (int j = 0; j < N; ++j) logdet += n * hld[j];
    logdet /= N;
    double trs = 0.0;
    for (int j = 0; j < N; ++j) trs += (n - s_dots[j]) / s2;
    trs = 2.0 * s2 * trs / N;
    if (tr_exact) {   // exact traces: tr(S dK) per theta, then tr(A^{-1})
        for (int th = 0; th <= d; ++th) tr[th] = tr_exact[th];
        trs = 2.0 * s2 * tr_exact[d + 1];
    }
    *mll = -0.5 * (logdet + q + n * std::log(2.0 * M_PI));
    for (int th = 0; th <= d; ++th) grad[th] = 0.5 * (quad[th] - tr[th]);
    grad[d + 1] = 0.5 * (2.0 * s2 * zz - trs);
    logdet_out = logdet;
    q_out = q;
    if (dq_out) {   // dq/dtheta = -x_y^T (dA/dtheta) x_y
        for (int k = 0; k < 5; ++k) dq_out[k] = 0.0;
        for (int th = 0; th <= d; ++th) dq_out[th] = -quad[th];
        dq_out[d + 1] = -2.0 * s2 * zz;
    }
    if (!std::isfinite(logdet)) {
        set_error("Lanczos quadrature failed (non-finite log-determinant)");
        return FKGP_EDEVICE;
    }
    return FKGP_OK;
}

fkgp_status mll_post(const OpCtx& c, const fkgp_hypers* hyp, const fkgp_mll_opts& o,
                     const double* V, const double* wx, const double* alphas,
                     const double* betas, const PState* ps, double* mll, double* grad,
                     Scratch& sc, hipStream_t st, double& logdet_out, double& q_out,
                     const double* tr_exact = nullptr, double* dq_out = nullptr) {
    const size_t nres = mll_post_doubles(c.h->g.d, c.h->nprobe);
    double* res = nullptr;
    FKGP_HIP(sc.get(&res, nres));
    fkgp_status rs = mll_post_enqueue(c, hyp, o, V, wx, alphas, betas, ps, res, true, sc, st);
    if (rs != FKGP_OK) return rs;
    std::vector<double> hres(nres);
    FKGP_HIP(hipMemcpyAsync(hres.data(), res, sizeof(double) * nres, hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    return mll_post_finish(c, hres.data(), mll, grad, logdet_out, q_out, tr_exact, dq_out);
}

// E[j] = unit vector e_{q0 + j} (E zeroed by the caller), j < nr.
__global__ void unit_columns(double* __restrict__ E, int nr, int64_t M, int64_t q0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nr) E[(int64_t)j * M + q0 + j] = 1.0;
}

// Exact traces through S = W^T A^{-1} W, built from m grid right-hand-side
// solves (S e_i = W^T A^{-1} W e_i, 64 columns per batched solve):
//   tr(A^{-1} W dK W^T) = tr(S dK) = sum_i (S e_i) . (dK e_i)  (theta <= d)
//   tr(A^{-1}) = (n - tr(K_G S)) / s2.
// out[0..d]: the first kind for log l_0.., log s; out[d+1]: tr(A^{-1}).
fkgp_status exact_traces(const OpCtx& c, const fkgp_hypers* hyp, double tol, int maxiter,
                         double* out, hipStream_t st) {
    const fkgp_handle* h = c.h;
    const int d = h->g.d;
    const int64_t M = h->M;
    const int64_t ldx = M + 2 * c.halo;
    Scratch sc(st);
    std::vector<Spectra> dsp(d + 1);
    for (int th = 0; th <= d; ++th) {
        fkgp_status rs = make_spectra(h, hyp, FKGP_F64, th < d ? th : -1, dsp[th], sc);
        if (rs != FKGP_OK) return rs;
    }
    std::vector<double> acc(d + 2, 0.0);
    for (int64_t q0 = 0; q0 < M; q0 += kSnapStates) {
        const int nr = (int)std::min<int64_t>(kSnapStates, M - q0);
        Scratch sj(st);
        double *E, *Epad, *BH, *bb, *S, *D, *alphas, *betas, *dotp, *dots;
        PState* ps;
        FKGP_HIP(sj.get(&E, M * nr));
        FKGP_HIP(sj.get(&Epad, ldx * nr));
        FKGP_HIP(sj.get(&BH, M * nr));
        FKGP_HIP(sj.get(&bb, nr));
        FKGP_HIP(sj.get(&S, M * nr));
        FKGP_HIP(sj.get(&D, M * nr));
        FKGP_HIP(sj.get(&alphas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&betas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&dotp, (size_t)vec_blocks(M) * nr));
        FKGP_HIP(sj.get(&dots, nr));
        FKGP_HIP(sj.get(&ps, nr));
        FKGP_HIP(hipMemsetAsync(E, 0, sizeof(double) * M * nr, st));
        unit_columns<<<(nr + 63) / 64, 64, 0, st>>>(E, nr, M, q0);
        FKGP_HIP(hipGetLastError());
        FKGP_HIP(hipMemsetAsync(Epad, 0, sizeof(double) * ldx * nr, st));
        FKGP_HIP(hipMemcpy2DAsync(Epad + c.halo, sizeof(double) * ldx, E, sizeof(double) * M,
                                  sizeof(double) * M, nr, hipMemcpyDeviceToDevice, st));
        fkgp_status rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, Epad, BH, nr,
                                      c.halo, nullptr, st);
        if (rs != FKGP_OK) return rs;
        rs = dots_dev(E, BH, M, nr, dotp, bb, st);
        if (rs != FKGP_OK) return rs;
        int it = 0;
        rs = probe_cg(c, BH, nr, (double)h->n, tol, maxiter, S, alphas, betas, ps, sj, st, it,
                      bb, E);
        if (rs != FKGP_OK && rs != FKGP_ENOTCONV) return rs;
        std::vector<double> hd(nr);
        for (int th = 0; th <= d + 1; ++th) {
            // theta <= d: dK e_i; last: K_G e_i
            const Spectra& sp = th <= d ? dsp[th] : c.sp64;
            rs = kg_apply(h->g, sp, FKGP_F64, E, D, nr, c.so, nullptr, 0.0, nullptr, st);
            if (rs != FKGP_OK) return rs;
            rs = dots_dev(S, D, M, nr, dotp, dots, st);
            if (rs != FKGP_OK) return rs;
            FKGP_HIP(hipMemcpyAsync(hd.data(), dots, sizeof(double) * nr, hipMemcpyDeviceToHost,
                                    st));
            FKGP_HIP(hipStreamSynchronize(st));
            for (int j = 0; j < nr; ++j) acc[th] += hd[j];
        }
    }
    for (int th = 0; th <= d; ++th) out[th] = acc[th];
    out[d + 1] = ((double)h->n - acc[d + 1]) / c.s2;
    return FKGP_OK;
}

// ---------------------------------------------------------------------------
// Reverse-mode derivative of the stochastic Lanczos log-determinant estimate
// itself: for each probe, Gamma_j = n e_1^T log(T_j) e_1 with T_j the
// Lanczos tridiagonal that the first k factorized-CG coefficients give, and
// its derivative in every hyperparameter through the k Lanczos steps run
// backwards (the checkpointed Krylov vectors are the CG residuals,
// q_i = (-1)^i r_i / ||r_i||; Claims 3-4 keep them as pairs r = W a + c z).
// ---------------------------------------------------------------------------

// Eigenvalues (d) and eigenvectors (Z, Z[r * k + col]) of the symmetric
// tridiagonal matrix with diagonal d and off-diagonal e (e[i] couples i and
// i + 1), by implicit QL iterations with Wilkinson-type shifts.
bool tridiag_eig(int k, std::vector<double>& d, std::vector<double> e, std::vector<double>& Z) {
    Z.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) Z[(size_t)i * k + i] = 1.0;
    e.resize(k, 0.0);
    if (k > 0) e[k - 1] = 0.0;
    for (int l = 0; l < k; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < k - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 4.0 * DBL_EPSILON * dd) break;
            }
            if (m == l) break;
            if (++iter > 100) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                double f = sn * e[i];
                const double b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - b;
                for (int t = 0; t < k; ++t) {
                    f = Z[(size_t)t * k + i + 1];
                    Z[(size_t)t * k + i + 1] = sn * Z[(size_t)t * k + i] + cs * f;
                    Z[(size_t)t * k + i] = cs * Z[(size_t)t * k + i] - sn * f;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

// d/dT of e_1^T log(T) e_1 for T = V diag(lam) V^T: G = V (F o v v^T) V^T,
// v = V^T e_1, F_ab the divided difference of log at (lam_a, lam_b) (1/lam_a
// when they coincide).  gd[i] = G_ii; go[i] = 2 G_{i,i+1} (an off-diagonal
// entry appears twice in T).  false if T is not positive definite.
bool logm_e1_grad_host(int k, const std::vector<double>& al, const std::vector<double>& be,
                       std::vector<double>& gd, std::vector<double>& go) {
    std::vector<double> lam = al, Z;
    if (!tridiag_eig(k, lam, be, Z)) return false;
    for (int a = 0; a < k; ++a)
        if (!(lam[a] > 0.0)) return false;
    std::vector<double> v(k), L(k);
    for (int a = 0; a < k; ++a) {
        v[a] = Z[a];   // first row
        L[a] = std::log(lam[a]);
    }
    std::vector<double> Fv((size_t)k * k);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            const double gap = lam[a] - lam[b];
            const double f = std::fabs(gap) > 1e-13 * std::fabs(lam[a]) ? (L[a] - L[b]) / gap
                                                                        : 1.0 / lam[a];
            Fv[(size_t)a * k + b] = f * v[a] * v[b];
        }
    gd.assign(k, 0.0);
    go.assign(k > 0 ? k - 1 : 0, 0.0);
    // G_rs = sum_ab Z_ra Fv_ab Z_sb, needed for s = r and s = r + 1
    std::vector<double> H((size_t)k * k, 0.0);   // H = Fv Z^T: H_as = sum_b Fv_ab Z_sb
    for (int a = 0; a < k; ++a)
        for (int sI = 0; sI < k; ++sI) {
            double acc = 0.0;
            for (int b = 0; b < k; ++b) acc += Fv[(size_t)a * k + b] * Z[(size_t)sI * k + b];
            H[(size_t)a * k + sI] = acc;
        }
    for (int r = 0; r < k; ++r) {
        double g0 = 0.0, g1 = 0.0;
        for (int a = 0; a < k; ++a) {
            g0 += Z[(size_t)r * k + a] * H[(size_t)a * k + r];
            if (r + 1 < k) g1 += Z[(size_t)r * k + a] * H[(size_t)a * k + r + 1];
        }
        gd[r] = g0;
        if (r + 1 < k) go[r] = 2.0 * g1;
    }
    return true;
}

// Per-column coefficients of the sweep's vector updates (one per probe).
struct ColCoef {
    double v[kSnapStates];
};

// y_j = a_j y_j + b_j x1_j + c_j x2_j for N columns of length M (x1, x2
// optional)
__global__ void col_lin3(double* __restrict__ y, const double* __restrict__ x1,
                         const double* __restrict__ x2, ColCoef a, ColCoef b, ColCoef cc,
                         int64_t M) {
    const int j = blockIdx.y;
    const double aj = a.v[j], bj = b.v[j], cj = cc.v[j];
    const int64_t o = (int64_t)j * M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = aj * y[o + i];
        if (x1) v = fma(bj, x1[o + i], v);
        if (x2) v = fma(cj, x2[o + i], v);
        y[o + i] = v;
    }
}

// tr_out[theta] = (1/N) sum_j dGamma_j / dtheta, theta = log l_0 .. log
// l_{d-1}, log s, log sigma.  Qa holds the residual history r_hat_i
// ([k][N][M], overwritten with the Lanczos vectors' W-parts), shist the
// (c_r,i, ||r_i||^2) history, alphas/betas/ps the probes' CG record.
fkgp_status slq_logdet_grad(const OpCtx& c, const fkgp_hypers* hyp, int k, int N,
                            const double* bh, double* Qa, const double* shist,
                            const double* alphas, const double* betas, const PState* ps,
                            double* tr_out, Scratch& sc, hipStream_t st) {
    const fkgp_handle* h = c.h;
    const int d = h->g.d;
    const int64_t M = h->M;
    const int64_t ldx = M + 2 * c.halo;
    const double n = (double)h->n;
    const double s2 = c.s2;
    if (N > kSnapStates) {
        set_error("too many probes for the Lanczos-estimate gradient");
        return FKGP_EINVAL;
    }
    std::vector<double> ha((size_t)N * kMaxLanczos), hb((size_t)N * kMaxLanczos),
        hs((size_t)k * N * 2);
    std::vector<PState> hps(N);
    FKGP_HIP(hipMemcpyAsync(ha.data(), alphas, sizeof(double) * ha.size(), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipMemcpyAsync(hb.data(), betas, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipMemcpyAsync(hs.data(), shist, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipMemcpyAsync(hps.data(), ps, sizeof(PState) * N, hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    // tridiagonals, their log-quadrature gradients, Lanczos-vector scalars
    std::vector<int> kk(N);
    int K = 0;
    std::vector<std::vector<double>> al(N), be(N), abar(N), bbar(N), Qc(N), qs(N);
    for (int j = 0; j < N; ++j) {
        kk[j] = std::min(k, std::min(hps[j].iters, kMaxLanczos));
        K = std::max(K, kk[j]);
        const double* a = &ha[(size_t)j * kMaxLanczos];
        const double* b = &hb[(size_t)j * kMaxLanczos];
        al[j].resize(kk[j]);
        be[j].resize(kk[j] > 0 ? kk[j] - 1 : 0);
        for (int i = 0; i < kk[j]; ++i) {
            al[j][i] = 1.0 / a[i] + (i > 0 ? b[i - 1] / a[i - 1] : 0.0);
            if (i + 1 < kk[j]) be[j][i] = std::sqrt(b[i]) / a[i];
        }
        if (!logm_e1_grad_host(kk[j], al[j], be[j], abar[j], bbar[j])) {
            set_error("Lanczos tridiagonal not positive definite in the log-determinant gradient");
            return FKGP_EDEVICE;
        }
        Qc[j].resize(kk[j]);
        qs[j].resize(kk[j]);
        for (int i = 0; i < kk[j]; ++i) {
            const double sgn = (i % 2 == 0) ? 1.0 : -1.0;
            const double cr = hs[((size_t)i * N + j) * 2], rho = hs[((size_t)i * N + j) * 2 + 1];
            qs[j][i] = sgn / std::sqrt(rho);
            Qc[j][i] = sgn * cr / std::sqrt(rho);
        }
    }
    for (int t = 0; t < d + 2; ++t) tr_out[t] = 0.0;
    if (K == 0) return FKGP_OK;
    const dim3 gcol((unsigned)std::min<int64_t>((M + 255) / 256, 1024), N);
    ColCoef zero{}, one{};
    for (int j = 0; j < N; ++j) one.v[j] = 1.0;
    auto lin3 = [&](double* y, const double* x1, const double* x2, const ColCoef& a,
                    const ColCoef& b, const ColCoef& cc) -> fkgp_status {
        col_lin3<<<gcol, 256, 0, st>>>(y, x1, x2, a, b, cc, M);
        FKGP_HIP(hipGetLastError());
        return FKGP_OK;
    };
    double *WQ, *pad, *r, *u, *Wu, *KW, *D, *dotp, *dots;
    FKGP_HIP(sc.get(&WQ, (size_t)K * N * M));
    FKGP_HIP(sc.get(&pad, (size_t)ldx * N));
    FKGP_HIP(sc.get(&r, (size_t)N * M));
    FKGP_HIP(sc.get(&u, (size_t)N * M));
    FKGP_HIP(sc.get(&Wu, (size_t)N * M));
    FKGP_HIP(sc.get(&KW, (size_t)N * M));
    FKGP_HIP(sc.get(&D, (size_t)N * M));
    FKGP_HIP(sc.get(&dotp, (size_t)vec_blocks(M) * N));
    FKGP_HIP(sc.get(&dots, (size_t)N));
    double* qb[3];
    for (int t = 0; t < 3; ++t) {
        FKGP_HIP(sc.get(&qb[t], (size_t)N * M));
        FKGP_HIP(hipMemsetAsync(qb[t], 0, sizeof(double) * N * M, st));
    }
    FKGP_HIP(hipMemsetAsync(pad, 0, sizeof(double) * ldx * N, st));
    std::vector<double> hdot(N);
    auto dots_host = [&](const double* A, const double* B) -> fkgp_status {
        fkgp_status rs = dots_dev(A, B, M, N, dotp, dots, st);
        if (rs != FKGP_OK) return rs;
        FKGP_HIP(hipMemcpyAsync(hdot.data(), dots, sizeof(double) * N, hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipStreamSynchronize(st));
        return FKGP_OK;
    };
    // W^T x for pairs (xa, xc): W^T W xa + xc b_hat
    auto wt = [&](const double* xa, const ColCoef& xc, double* out) -> fkgp_status {
        FKGP_HIP(hipMemcpy2DAsync(pad + c.halo, sizeof(double) * ldx, xa, sizeof(double) * M,
                                  sizeof(double) * M, N, hipMemcpyDeviceToDevice, st));
        fkgp_status rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, pad, out, N,
                                      c.halo, nullptr, st);
        if (rs != FKGP_OK) return rs;
        return lin3(out, bh, nullptr, one, xc, zero);
    };
    // Lanczos vectors q_i = (qs r_hat_i, Qc_i), W^T q_i and s_i = b_hat . a_i + Qc_i n
    std::vector<std::vector<double>> sv(K, std::vector<double>(N, 0.0));
    for (int i = 0; i < K; ++i) {
        ColCoef sc_q{}, qc{};
        for (int j = 0; j < N; ++j) {
            sc_q.v[j] = i < kk[j] ? qs[j][i] : 0.0;
            qc.v[j] = i < kk[j] ? Qc[j][i] : 0.0;
        }
        double* Qi = Qa + (size_t)i * N * M;
        fkgp_status rs = lin3(Qi, nullptr, nullptr, sc_q, zero, zero);
        if (rs != FKGP_OK) return rs;
        rs = wt(Qi, qc, WQ + (size_t)i * N * M);
        if (rs != FKGP_OK) return rs;
        rs = dots_host(bh, Qi);
        if (rs != FKGP_OK) return rs;
        for (int j = 0; j < N; ++j) sv[i][j] = hdot[j] + qc.v[j] * n;
    }
    // derivative spectra: theta < d: d/dlog l_theta; theta = d: K_G itself
    std::vector<Spectra> dsp(d);
    for (int th = 0; th < d; ++th) {
        fkgp_status rs = make_spectra(h, hyp, FKGP_F64, th, dsp[th], sc);
        if (rs != FKGP_OK) return rs;
    }
    std::vector<std::vector<double>> g(N, std::vector<double>(d + 2, 0.0));
    std::vector<double> qbc_next(N, 0.0), qbc_cur(N, 0.0), qbc_prev(N, 0.0);
    for (int i = K - 1; i >= 0; --i) {
        double* QBn = qb[(i + 1) % 3];   // qbar[i + 1], final
        double* QBc = qb[i % 3];         // qbar[i]
        double* QBp = qb[(i + 2) % 3];   // qbar[i - 1]
        const double* Qi = Qa + (size_t)i * N * M;
        const double* WQi = WQ + (size_t)i * N * M;
        // r = qbar[i+1] / be_i + bbar_i q_{i+1} (columns with i + 1 < kk)
        ColCoef ca{}, cb{}, rc{};
        bool any_next = false;
        for (int j = 0; j < N; ++j) any_next |= i + 1 < kk[j];
        if (any_next) {
            fkgp_status rs = dots_host(QBn, WQ + (size_t)(i + 1) * N * M);
            if (rs != FKGP_OK) return rs;
            for (int j = 0; j < N; ++j) {
                if (!(i + 1 < kk[j])) continue;
                const double in1 = hdot[j] + qbc_next[j] * sv[i + 1][j];
                bbar[j][i] -= in1 / be[j][i];
                ca.v[j] = 1.0 / be[j][i];
                cb.v[j] = bbar[j][i];
                rc.v[j] = qbc_next[j] / be[j][i] + bbar[j][i] * Qc[j][i + 1];
            }
        }
        FKGP_HIP(hipMemsetAsync(r, 0, sizeof(double) * N * M, st));
        fkgp_status rs = lin3(r, QBn, Qa + (size_t)(i + 1 < K ? i + 1 : i) * N * M, zero, ca,
                              any_next ? cb : zero);
        if (rs != FKGP_OK) return rs;
        // abar_i -= <r, q_i>; bbar_{i-1} -= <r, q_{i-1}>
        rs = dots_host(r, WQi);
        if (rs != FKGP_OK) return rs;
        for (int j = 0; j < N; ++j)
            if (i < kk[j]) abar[j][i] -= hdot[j] + rc.v[j] * sv[i][j];
        if (i > 0) {
            rs = dots_host(r, WQ + (size_t)(i - 1) * N * M);
            if (rs != FKGP_OK) return rs;
            for (int j = 0; j < N; ++j)
                if (i < kk[j]) bbar[j][i - 1] -= hdot[j] + rc.v[j] * sv[i - 1][j];
        }
        // u = r + abar_i q_i
        ColCoef ab{}, uc{}, mal{}, mbe{};
        for (int j = 0; j < N; ++j) {
            if (!(i < kk[j])) continue;
            ab.v[j] = abar[j][i];
            uc.v[j] = rc.v[j] + abar[j][i] * Qc[j][i];
            mal.v[j] = -al[j][i];
            if (i > 0) mbe.v[j] = -be[j][i - 1];
        }
        FKGP_HIP(hipMemcpyAsync(u, r, sizeof(double) * N * M, hipMemcpyDeviceToDevice, st));
        rs = lin3(u, Qi, nullptr, one, ab, zero);
        if (rs != FKGP_OK) return rs;
        // qbar_i += -al_i r + abar_i A q_i, A q = (K_G W^T q + s2 a, s2 c)
        rs = kg_apply(h->g, c.sp64, FKGP_F64, WQi, KW, N, c.so, nullptr, 0.0, nullptr, st);
        if (rs != FKGP_OK) return rs;
        ColCoef abs2{};
        for (int j = 0; j < N; ++j) abs2.v[j] = ab.v[j] * s2;
        rs = lin3(QBc, r, KW, one, mal, ab);
        if (rs != FKGP_OK) return rs;
        rs = lin3(QBc, Qi, nullptr, one, abs2, zero);
        if (rs != FKGP_OK) return rs;
        for (int j = 0; j < N; ++j)
            if (i < kk[j]) qbc_cur[j] += -al[j][i] * rc.v[j] + ab.v[j] * s2 * Qc[j][i];
        // qbar_{i-1} -= be_{i-1} r
        if (i > 0) {
            rs = lin3(QBp, r, nullptr, one, mbe, zero);
            if (rs != FKGP_OK) return rs;
            for (int j = 0; j < N; ++j)
                if (i < kk[j]) qbc_prev[j] += mbe.v[j] * rc.v[j];
        }
        // gradient terms: ubar^T dA q_i = (W^T u)^T dK (W^T q_i) for log l and
        // log s, 2 s2 <u, q_i> for log sigma
        rs = wt(u, uc, Wu);
        if (rs != FKGP_OK) return rs;
        for (int th = 0; th <= d; ++th) {
            const double* DK = KW;   // d/dlog s: K_G itself
            if (th < d) {
                rs = kg_apply(h->g, dsp[th], FKGP_F64, WQi, D, N, c.so, nullptr, 0.0, nullptr, st);
                if (rs != FKGP_OK) return rs;
                DK = D;
            }
            rs = dots_host(Wu, DK);
            if (rs != FKGP_OK) return rs;
            for (int j = 0; j < N; ++j)
                if (i < kk[j]) g[j][th] += hdot[j];
        }
        rs = dots_host(u, WQi);
        if (rs != FKGP_OK) return rs;
        for (int j = 0; j < N; ++j)
            if (i < kk[j]) g[j][d + 1] += 2.0 * s2 * (hdot[j] + uc.v[j] * sv[i][j]);
        // qbar_i += A u = (K_G W^T u + s2 u_a, s2 u_c)
        rs = kg_apply(h->g, c.sp64, FKGP_F64, Wu, KW, N, c.so, u, s2, nullptr, st);
        if (rs != FKGP_OK) return rs;
        rs = lin3(QBc, KW, nullptr, one, one, zero);
        if (rs != FKGP_OK) return rs;
        for (int j = 0; j < N; ++j)
            if (i < kk[j]) qbc_cur[j] += s2 * uc.v[j];
        // rotate: qbar[i] becomes the next step's qbar[i + 1]
        qbc_next = qbc_cur;
        qbc_cur = qbc_prev;
        qbc_prev.assign(N, 0.0);
        FKGP_HIP(hipMemsetAsync(qb[(i + 1) % 3], 0, sizeof(double) * N * M, st));
    }
    for (int t = 0; t < d + 2; ++t) {
        double acc = 0.0;
        for (int j = 0; j < N; ++j) acc += n * g[j][t];
        tr_out[t] = acc / N;
    }
    return FKGP_OK;
}

fkgp_status mll_impl(const fkgp_handle* h, const fkgp_hypers* hyp, const fkgp_mll_opts& o,
                     double* mll, double* grad, fkgp_mll_info* info, hipStream_t st) {
    Scratch sc(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, FKGP_F64, c, sc);
    if (rs != FKGP_OK) return rs;
    const int N = h->nprobe;
    const int64_t M = h->M;
    const double n = (double)h->n;
    double *V, *wx, *alphas, *betas;
    PState* ps;
    FKGP_HIP(sc.get(&V, M * (N + 1)));       // [w_y, b_hat_0 .. b_hat_{N-1}]
    FKGP_HIP(sc.get(&wx, M * (N + 1)));      // [w_y, W^T x_0 .. W^T x_{N-1}]
    FKGP_HIP(sc.get(&alphas, (size_t)kMaxLanczos * N));
    FKGP_HIP(sc.get(&betas, (size_t)kMaxLanczos * N));
    FKGP_HIP(sc.get(&ps, N));
    FKGP_HIP(hipMemcpyAsync(V + M, h->sketches, sizeof(double) * M * N, hipMemcpyDeviceToDevice, st));
    // The response's mean solve (w_y = W^T z~) and the probe solves are
    // independent until the post-processing: the mean solve runs on a second
    // stream, driven by a second host thread, while this thread drives the
    // probe solves on `st`.
    struct Fork {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        std::thread t;
        ~Fork() {
            if (t.joinable()) t.join();
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
            if (ev) (void)hipEventDestroy(ev);
        }
    } fork;
    FKGP_HIP(hipStreamCreateWithFlags(&fork.s, hipStreamNonBlocking));
    FKGP_HIP(hipEventCreateWithFlags(&fork.ev, hipEventDisableTiming));
    FKGP_HIP(hipEventRecord(fork.ev, st));
    FKGP_HIP(hipStreamWaitEvent(fork.s, fork.ev, 0));
    int dev = 0;
    FKGP_HIP(hipGetDevice(&dev));
    fkgp_solve_info sinfo{};
    fkgp_status sres = FKGP_OK;
    std::string serr;
    const hipStream_t sy = fork.s;
    fork.t = std::thread([&, sy, dev] {
        if (hipSetDevice(dev) != hipSuccess) {
            sres = FKGP_EDEVICE;
            serr = "hipSetDevice failed in the mean-solve thread";
            return;
        }
        {
            // own spectra and four-step scratch: the long-line passes of the
            // two streams must not share their workspace
            Scratch sy_sc(sy);
            OpCtx cy;
            sres = make_ctx(h, hyp, FKGP_F64, cy, sy_sc);
            if (sres == FKGP_OK)
                sres = solve_core(cy, nullptr, o.tol, o.maxiter, V, &sinfo, sy_sc, sy);
            // the workspace goes back only once its work is done (a caller's
            // allocator may not order frees on this private stream)
            (void)hipStreamSynchronize(sy);
        }
        if (sres != FKGP_OK) serr = last_error_copy();
    });
    // probe solves (batched, or one probe at a time); the gradient of the
    // Lanczos estimate itself (trace_mode 2) checkpoints the first
    // lanczos_steps residuals of every probe
    int iters_max = 0;
    fkgp_status pres = FKGP_OK;
    const int kslq = std::min(o.lanczos_steps, kMaxLanczos);
    double *rhist = nullptr, *shist = nullptr;
    if (o.trace_mode == 2) {
        FKGP_HIP(sc.get(&rhist, (size_t)kslq * N * M));
        FKGP_HIP(sc.get(&shist, (size_t)kslq * N * 2));
    }
    if (o.batched || o.trace_mode == 2) {
        pres = probe_cg(c, V + M, N, n, o.tol, o.maxiter, wx + M, alphas, betas, ps, sc, st,
                        iters_max, nullptr, nullptr, rhist, shist, kslq);
    } else {
        for (int j = 0; j < N && (pres == FKGP_OK || pres == FKGP_ENOTCONV); ++j) {
            int it = 0;
            Scratch sj(st);
            fkgp_status r1 = probe_cg(c, V + M * (1 + j), 1, n, o.tol, o.maxiter,
                                      wx + M * (1 + j), alphas + kMaxLanczos * j,
                                      betas + kMaxLanczos * j, ps + j, sj, st, it);
            if (r1 != FKGP_OK) pres = r1;
            iters_max = std::max(iters_max, it);
        }
    }
    const std::string perr = last_error_copy();
    fork.t.join();
    if (sres != FKGP_OK && sres != FKGP_ENOTCONV) {
        set_error(serr);
        return sres;
    }
    if (pres != FKGP_OK && pres != FKGP_ENOTCONV) {
        set_error(perr);
        return pres;
    }
    FKGP_HIP(hipMemcpyAsync(wx, V, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
    double logdet = 0.0, q = 0.0, dq[5];
    std::vector<double> trx;
    if (o.trace_mode == 1) {
        trx.resize(h->g.d + 2);
        rs = exact_traces(c, hyp, o.tol, o.maxiter, trx.data(), st);
        if (rs != FKGP_OK) return rs;
    } else if (o.trace_mode == 2) {
        // d Gamma / d theta in place of the trace estimates (the last one as
        // the coefficient mll_post scales by 2 s2)
        trx.resize(h->g.d + 2);
        rs = slq_logdet_grad(c, hyp, kslq, N, V + M, rhist, shist, alphas, betas, ps, trx.data(),
                             sc, st);
        if (rs != FKGP_OK) return rs;
        trx[h->g.d + 1] /= 2.0 * c.s2;
    }
    rs = mll_post(c, hyp, o, V, wx, alphas, betas, ps, mll, grad, sc, st, logdet, q,
                  trx.empty() ? nullptr : trx.data(), dq);
    if (rs != FKGP_OK) return rs;
    if (info) {
        info->logdet = logdet;
        info->quad = q;
        for (int k = 0; k < 5; ++k) info->dquad[k] = dq[k];
        info->iterations_y = sinfo.iterations;
        info->iterations_probes_max = iters_max;
    }
    return (sres == FKGP_ENOTCONV || pres == FKGP_ENOTCONV) ? FKGP_ENOTCONV : FKGP_OK;
}

// Work items of a batch (device arrays in `sc`): each problem's right-hand
// sides in groups of at most NR, each group with its own vectors and, for
// four-step lines, its own L-point scratch.  One workgroup runs one item to
// convergence, so the batch takes at least as long as its longest item and
// at least its total work over the items that run at once (`slots`).  The
// items are sized and ordered for both (longest processing time first):
//  * cost of an item = iterations x M log2 M x (1 + right-hand sides): the
//    stored matrix is read once per iteration for all of the item's
//    right-hand sides, the rest scales with their number; the iterations are
//    those of the previous evaluation of the same batch shape when known
//    (`iters`, else equal for all problems);
//  * a problem whose item would still run after the batch's average load per
//    slot is reached gets smaller groups (down to one right-hand side), so
//    its work spreads over more workgroups;
//  * the items are launched in decreasing cost: workgroups are dispatched in
//    index order, so the long items start first and the short ones fill in.
fkgp_status build_batch_items(const std::vector<BatchProb>& probs, const std::vector<int>& nrhs,
                              const std::vector<int>& long_L, int NR, int slots,
                              const std::vector<int>* iters, Scratch& sc,
                              BatchItem** items_dev, int& nitems) {
    const size_t np = probs.size();
    // per-iteration cost of one right-hand side, and the iterations (known
    // from the previous evaluation, else equal)
    std::vector<double> w(np), its(np), ones(np, 1.0);
    for (size_t p = 0; p < np; ++p) {
        const double M = (double)probs[p].M;
        its[p] = (iters && p < iters->size() && (*iters)[p] > 0) ? (*iters)[p] : 1.0;
        w[p] = M * std::log2(M + 2.0);
    }
    auto item_cost = [&](size_t p, int nr) { return its[p] * w[p] * (1.0 + nr); };
    auto grouping = [&](const std::vector<double>& k, std::vector<int>& g) {
        auto cost = [&](size_t p, int nr) { return k[p] * w[p] * (1.0 + nr); };
        for (int pass = 0; pass < 2; ++pass) {
            double total = 0.0, longest1 = 0.0;
            for (size_t p = 0; p < np; ++p) {
                const int nit = (nrhs[p] + g[p] - 1) / g[p];
                total += nit * cost(p, g[p]);
                longest1 = std::max(longest1, cost(p, 1));
            }
            const double target = std::max(total / std::max(1, slots), longest1);
            for (size_t p = 0; p < np; ++p) {
                int nr = NR;
                while (nr > 1 && cost(p, std::min(nr, nrhs[p])) > target) nr /= 2;
                g[p] = std::max(1, nr);
            }
        }
    };
    // Group sizes per problem.  A 1-D problem's right-hand sides share
    // complex FFT lines inside an item, so its results depend on the
    // grouping: it takes the groups of equal iterations, which depend on
    // the shapes alone.  Vectors of several lines pair their own lines, so
    // larger problems follow the measured iterations without changing any
    // result: every call gives bitwise the same values.
    std::vector<int> g(np, NR), g_shape(np, NR);
    grouping(ones, g_shape);
    grouping(its, g);
    for (size_t p = 0; p < np; ++p)
        if (probs[p].d == 1) g[p] = g_shape[p];
    struct Pending {
        BatchItem it;
        double cost;
    };
    std::vector<Pending> pend;
    for (size_t p = 0; p < np; ++p) {
        const size_t wd = batch_work_doubles(probs[p].M, probs[p].halo, NR);
        for (int r0 = 0; r0 < nrhs[p]; r0 += g[p]) {
            double* work = nullptr;
            FKGP_HIP(sc.get(&work, wd));
            double* yscr = nullptr;
            if (long_L[p] > 0) FKGP_HIP(sc.get(&yscr, (size_t)2 * long_L[p]));
            const int nr = std::min(g[p], nrhs[p] - r0);
            pend.push_back(Pending{BatchItem{(int)p, r0, nr, work,
                                             reinterpret_cast<cplx<double>*>(yscr)},
                                   item_cost(p, nr)});
        }
    }
    std::stable_sort(pend.begin(), pend.end(),
                     [](const Pending& x, const Pending& y) { return x.cost > y.cost; });
    std::vector<BatchItem> items;
    items.reserve(pend.size());
    for (const Pending& q : pend) items.push_back(q.it);
    nitems = (int)items.size();
    FKGP_HIP(sc.get(items_dev, items.size()));
    FKGP_HIP(hipMemcpyAsync(*items_dev, items.data(), sizeof(BatchItem) * items.size(),
                            hipMemcpyHostToDevice, sc.s));
    FKGP_HIP(hipStreamSynchronize(sc.s));   // `items` leaves scope
    return FKGP_OK;
}

// Autotuner of the batched solver.  Two tile parameters: the number of
// right-hand sides per work item (2, 4 or 8) trades per-item work and W^T W
// re-reads against the number of co-resident workgroups and the load
// balance at the tail; the workgroup size (256 or 512 threads) trades
// latency hiding inside an item against items per CU.  Each candidate runs
// a short trial (the first iterations of the real solve, whose state the
// real launch re-initialises) timed with HIP events; the fastest per batch
// shape (problem sizes, right-hand sides, stats dtype) is cached for the
// life of the process.
struct BatchTile {
    int nr, block;
};
std::mutex g_tune_mu;
std::map<std::string, BatchTile> g_tune_cache;
// iterations of each problem at the last evaluation of a batch shape
std::map<std::string, std::vector<int>> g_iter_cache;
constexpr BatchTile kTuneCandidates[6] = {{8, 256}, {4, 256}, {2, 256},
                                          {8, 512}, {4, 512}, {2, 512}};
constexpr int kTuneIters = 16;

std::string batch_shape_key(const fkgp_handle* const* hs, int np) {
    std::string key;
    for (int p = 0; p < np; ++p) {
        const fkgp_handle* h = hs[p];
        key += std::to_string(h->g.d);
        for (int k = 0; k < h->g.d; ++k) key += "x" + std::to_string(h->g.m[k]);
        key += "r" + std::to_string(h->nprobe + 1) + (h->dt == FKGP_F32 ? "f;" : "d;");
    }
    return key;
}

// Many problems in one persistent launch: for each problem the right-hand
// sides [y, z_0 .. z_{N-1}]; the probes use the factorized CG from x_0 = 0,
// the data vector the simplified factorized CG from x_0 = y / s2.
fkgp_status batch_mll_impl(const fkgp_handle* const* hs, int np, const fkgp_hypers* hyps,
                           const fkgp_mll_opts& o, double* mll, double* grad,
                           fkgp_mll_info* infos, hipStream_t st) {
    Scratch sc(st);
    std::vector<OpCtx> ctx(np);
    std::vector<Spectra> bsp(np);
    std::vector<BatchProb> probs(np);
    std::vector<int> nrhs_v(np), long_L(np, 0);
    std::vector<double*> Vs(np), wxs(np), alph(np), bet(np);
    std::vector<PState*> pss(np);
    std::vector<std::vector<double>> hbs(np);   // ||b||^2 of each problem's right-hand sides
    size_t lds = 0;      // spectra and strided-pass transpose, largest problem
    int stage_m1 = 0;    // largest m1 of a 2-D problem (staged product margin)
    for (int p = 0; p < np; ++p) {
        const fkgp_handle* h = hs[p];
        fkgp_status rs = make_ctx(h, &hyps[p], FKGP_F64, ctx[p], sc);
        if (rs != FKGP_OK) return rs;
        // the batched kernel's own spectra: register order up to 512 points
        rs = make_spectra(h, &hyps[p], FKGP_F64, -1, bsp[p], sc, kBatchRegMaxLog2);
        if (rs != FKGP_OK) return rs;
        const OpCtx& c = ctx[p];
        const int N = h->nprobe, nrhs = N + 1;
        const int64_t M = h->M;
        nrhs_v[p] = nrhs;
        double *bh, *kb, *bn, *V, *wx, *al, *be;
        PState* ps;
        FKGP_HIP(sc.get(&bh, M * nrhs));
        FKGP_HIP(sc.get(&kb, M * nrhs));
        FKGP_HIP(sc.get(&bn, nrhs));
        FKGP_HIP(sc.get(&V, M * nrhs));
        FKGP_HIP(sc.get(&wx, M * nrhs));
        FKGP_HIP(sc.get(&al, (size_t)kMaxLanczos * nrhs));
        FKGP_HIP(sc.get(&be, (size_t)kMaxLanczos * nrhs));
        FKGP_HIP(sc.get(&ps, nrhs));
        FKGP_HIP(hipMemcpyAsync(bh, h->wty, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        FKGP_HIP(hipMemcpyAsync(bh + M, h->sketches, sizeof(double) * M * N,
                                hipMemcpyDeviceToDevice, st));
        rs = kg_apply(h->g, c.sp64, FKGP_F64, bh, kb, nrhs, c.so, nullptr, 0.0, nullptr, st);
        if (rs != FKGP_OK) return rs;
        // the data right-hand side starts from x_0 = y / s2: r_hat_0 = -K_G W^T y / s2
        double* r0y = nullptr;
        FKGP_HIP(sc.get(&r0y, M));
        rs = kg_apply(h->g, c.sp64, FKGP_F64, h->wty, r0y, 1, -c.so / c.s2, nullptr, 0.0,
                      nullptr, st);
        if (rs != FKGP_OK) return rs;
        std::vector<double>& hb = hbs[p];   // kept until the stream is synchronised
        hb.assign(nrhs, (double)h->n);
        hb[0] = h->yty;
        FKGP_HIP(hipMemcpyAsync(bn, hb.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
        BatchProb& P = probs[p];
        P.d = h->g.d;
        P.m[0] = h->g.m[0];
        P.m[1] = h->g.d > 1 ? h->g.m[1] : 1;
        P.M = M;
        P.halo = c.halo;
        P.NB = h->NB;
        for (int k = 0; k < 2; ++k) {
            P.log2L[k] = k < h->g.d ? bsp[p].log2L[k] : 0;
            P.tw[k] = k < h->g.d ? bsp[p].tw[k] : nullptr;
            P.lam[k] = k < h->g.d ? static_cast<const double*>(bsp[p].lam[k]) : nullptr;
            if (k < h->g.d && P.log2L[k] > kBatchRegMaxLog2)
                long_L[p] = std::max(long_L[p], 1 << P.log2L[k]);
        }
        P.col[0] = P.col[1] = nullptr;
        if (batch_tz(P.d, P.m)) {
            for (int k = 0; k < 2; ++k) {
                double* col = nullptr;
                FKGP_HIP(sc.get(&col, (size_t)P.m[k]));
                rs = build_toeplitz_col(h->g, k, hyps[p].lengthscale[k], false, hyps[p].kernel,
                                        FKGP_F64, col, st);
                if (rs != FKGP_OK) return rs;
                P.col[k] = col;
            }
        }
        lds = std::max(lds, batch_lds_bytes(P.d, P.m, P.log2L));
        stage_m1 = std::max(stage_m1, P.d == 1 ? 0 : P.m[1]);
        P.a_f32 = h->dt == FKGP_F32 ? 1 : 0;
        P.A = h->A;
        P.so = c.so;
        P.s2 = c.s2;
        P.bh = bh;
        P.kb = kb;
        P.bnorm2 = bn;
        P.r0y = r0y;
        P.alphas = al;
        P.betas = be;
        P.ps = ps;
        P.wx = wx;
        Vs[p] = V;
        wxs[p] = wx;
        alph[p] = al;
        bet[p] = be;
        pss[p] = ps;
    }
    BatchProb* probs_dev = nullptr;
    FKGP_HIP(sc.get(&probs_dev, np));
    FKGP_HIP(hipMemcpyAsync(probs_dev, probs.data(), sizeof(BatchProb) * np,
                            hipMemcpyHostToDevice, st));
    // scheduling inputs: concurrent items per launch and the iterations of
    // the previous evaluation of this batch shape
    int ncu = 0;
    FKGP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
    const std::string shape = batch_shape_key(hs, np);
    std::vector<int> iters_hint;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto f = g_iter_cache.find(shape);
        if (f != g_iter_cache.end()) iters_hint = f->second;
    }
    const std::vector<int>* hint = iters_hint.empty() ? nullptr : &iters_hint;
    auto slots_for = [&](int block) { return std::max(1, ncu) * (block == 256 ? 2 : 1); };
    // dynamic LDS per tile: room for the staged banded product's windows on
    // top of the spectra, within 64 KB (two 256-thread items per CU);
    // problems whose windows do not fit use the unstaged product
    auto lds_for = [&](int nr, int block) {
        const size_t cap = 64 * 1024;
        const size_t want = lds + sizeof(double) * (size_t)batch_stage_doubles(2, stage_m1, nr,
                                                                               block);
        return std::max(lds, std::min(want, cap));
    };
    // tile: forced, cached or tuned
    BatchTile tile{o.batch_rhs, o.batch_block};
    if (tile.nr == 0 || tile.block == 0) {
        const std::string key = batch_shape_key(hs, np) + "/" + std::to_string(o.batch_rhs) +
                                "/" + std::to_string(o.batch_block);
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto f = g_tune_cache.find(key);
            if (f != g_tune_cache.end()) {
                tile = f->second;
                have = true;
            }
        }
        if (!have) {
            float best = 0.0f;
            BatchTile chosen{0, 0};
            hipEvent_t e0, e1;
            FKGP_HIP(hipEventCreate(&e0));
            FKGP_HIP(hipEventCreate(&e1));
            for (const BatchTile& cand : kTuneCandidates) {
                if ((o.batch_rhs && cand.nr != o.batch_rhs) ||
                    (o.batch_block && cand.block != o.batch_block))
                    continue;
                Scratch tsc(st);
                BatchItem* it_dev = nullptr;
                int nit = 0;
                fkgp_status rs =
                    build_batch_items(probs, nrhs_v, long_L, cand.nr, slots_for(cand.block),
                                      hint, tsc, &it_dev, nit);
                if (rs == FKGP_OK)   // warm-up launch (code object load), then the trial
                    rs = launch_batch_cg(probs_dev, it_dev, nit, lds_for(cand.nr, cand.block),
                                         o.tol, 1, cand.nr, cand.block, st);
                if (rs == FKGP_OK) {
                    FKGP_HIP(hipEventRecord(e0, st));
                    rs = launch_batch_cg(probs_dev, it_dev, nit, lds_for(cand.nr, cand.block),
                                         o.tol, std::min(o.maxiter, kTuneIters), cand.nr,
                                         cand.block, st);
                    FKGP_HIP(hipEventRecord(e1, st));
                }
                if (rs != FKGP_OK) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return rs;
                }
                FKGP_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                FKGP_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (chosen.nr == 0 || ms < best) {
                    best = ms;
                    chosen = cand;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            tile = chosen;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = tile;
        }
    }
    const int NR = tile.nr;
    BatchItem* items_dev = nullptr;
    int nitems = 0;
    fkgp_status rs = build_batch_items(probs, nrhs_v, long_L, NR, slots_for(tile.block), hint,
                                       sc, &items_dev, nitems);
    if (rs != FKGP_OK) return rs;
    rs = launch_batch_cg(probs_dev, items_dev, nitems, lds_for(NR, tile.block), o.tol,
                         o.maxiter, NR, tile.block, st);
    if (rs != FKGP_OK) return rs;
    // every problem's MLL and gradient work is queued behind the launch and
    // read back with one copy; the log-determinants of all probes run in
    // one launch
    std::vector<size_t> roff(np + 1, 0), psoff(np, 0);
    size_t nps = 0;
    int maxN = 0;
    for (int p = 0; p < np; ++p) {
        roff[p + 1] = roff[p] + mll_post_doubles(hs[p]->g.d, hs[p]->nprobe);
        psoff[p] = nps;
        nps += (size_t)hs[p]->nprobe + 1;
        maxN = std::max(maxN, hs[p]->nprobe);
    }
    double* res_dev = nullptr;
    PState* ps_all = nullptr;
    LogdetJob* jobs_dev = nullptr;
    FKGP_HIP(sc.get(&res_dev, roff[np]));
    FKGP_HIP(sc.get(&ps_all, nps));
    FKGP_HIP(sc.get(&jobs_dev, (size_t)np));
    std::vector<LogdetJob> jobs(np);
    for (int p = 0; p < np; ++p) {
        const fkgp_handle* h = hs[p];
        const int N = h->nprobe;
        const int64_t M = h->M;
        FKGP_HIP(hipMemcpyAsync(ps_all + psoff[p], pss[p], sizeof(PState) * (N + 1),
                                hipMemcpyDeviceToDevice, st));
        // V = [W^T z~ (= wx_0), b_hat_j]
        FKGP_HIP(hipMemcpyAsync(Vs[p], wxs[p], sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        FKGP_HIP(hipMemcpyAsync(Vs[p] + M, h->sketches, sizeof(double) * M * N,
                                hipMemcpyDeviceToDevice, st));
        Scratch sp_(st);
        rs = mll_post_enqueue(ctx[p], &hyps[p], o, Vs[p], wxs[p], alph[p] + kMaxLanczos,
                              bet[p] + kMaxLanczos, pss[p] + 1, res_dev + roff[p], false, sp_,
                              st);
        if (rs != FKGP_OK) return rs;
        jobs[p] = LogdetJob{pss[p] + 1, alph[p] + kMaxLanczos, bet[p] + kMaxLanczos,
                            res_dev + roff[p + 1] - N, N};
    }
    FKGP_HIP(hipMemcpyAsync(jobs_dev, jobs.data(), sizeof(LogdetJob) * np,
                            hipMemcpyHostToDevice, st));
    if (maxN > 0) {
        lanczos_logdet_multi<<<dim3((maxN + 63) / 64, np), 64, 0, st>>>(jobs_dev,
                                                                         o.lanczos_steps);
        FKGP_HIP(hipGetLastError());
    }
    std::vector<double> hres(roff[np]);
    std::vector<PState> hps(nps);
    FKGP_HIP(hipMemcpyAsync(hres.data(), res_dev, sizeof(double) * roff[np],
                            hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipMemcpyAsync(hps.data(), ps_all, sizeof(PState) * nps, hipMemcpyDeviceToHost,
                            st));
    FKGP_HIP(hipStreamSynchronize(st));
    fkgp_status res = FKGP_OK;
    std::vector<int> iters_now(np, 0);
    for (int p = 0; p < np; ++p) {
        const fkgp_handle* h = hs[p];
        const int N = h->nprobe;
        const PState* hsv = hps.data() + psoff[p];
        int itmax = 0;
        bool conv = true;
        for (int j = 0; j <= N; ++j) {
            if (hsv[j].done == 2) {
                set_error("batched CG broke down (non-finite step) in problem " + std::to_string(p));
                return FKGP_EDEVICE;
            }
            conv &= hsv[j].done == 1;
            if (j > 0) itmax = std::max(itmax, hsv[j].iters);
            iters_now[p] = std::max(iters_now[p], hsv[j].iters);
        }
        double logdet = 0.0, q = 0.0, dq[5];
        rs = mll_post_finish(ctx[p], hres.data() + roff[p], &mll[p], grad + 5 * p, logdet, q,
                             nullptr, dq);
        if (rs != FKGP_OK) return rs;
        for (int k = h->g.d + 2; k < 5; ++k) grad[5 * p + k] = 0.0;
        if (infos) {
            infos[p].logdet = logdet;
            infos[p].quad = q;
            for (int k = 0; k < 5; ++k) infos[p].dquad[k] = dq[k];
            infos[p].iterations_y = hsv[0].iters;
            infos[p].iterations_probes_max = itmax;
            infos[p].batch_rhs = NR;
            infos[p].batch_block = tile.block;
        }
        if (!conv) res = FKGP_ENOTCONV;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_iter_cache[shape] = iters_now;
    }
    return res;
}

// ---------------------------------------------------------------------------
// Posterior covariance between query points (Def. 2 model):
//   cov = Wq K_G Wq^T - Wq K_G W^T A^{-1} W K_G Wq^T,  A = W K_G W^T + s2 I.
// Column j of K_G Wq^T is v_j = K_G g_j (g_j: weights of query point j), so
// the data-side right-hand side is b_j = W v_j, with W^T b_j = W^T W v_j and
// ||b_j||^2 = v_j . W^T W v_j; the factorized CG from x_0 = 0 returns
// W^T A^{-1} b_j, and
//   cov[i][j] = g_i . v_j - v_i . (W^T A^{-1} b_j).
// Everything is FP64 on the device; n enters only through W^T W.
// ---------------------------------------------------------------------------
constexpr int kCovMaxQ = 4096;  // query points per call
constexpr int kCovRhs = 64;     // right-hand sides per batched CG
constexpr int kCovTile = 64;    // query points per side of a pair tile
constexpr int kCovChunk = 16;
constexpr int kCovPairs = kCovTile * kCovTile / 256;  // pairs per thread

// For the tile (rows i0.., columns j0..) of the pair matrix: partial sums of
// g_i . v_j - v_i . x_j over the grid chunks of this block (chunk c goes to
// block c mod gridDim.x, in increasing order).
// partials[(tile * gridDim.x + block) * kCovTile^2 + a * kCovTile + b].
__global__ __launch_bounds__(256) void cov_partial(const double* __restrict__ G,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ X, int64_t M,
                                                   int nq, double* __restrict__ partials) {
    __shared__ double sG[kCovTile][kCovChunk + 1];
    __shared__ double sVi[kCovTile][kCovChunk + 1];
    __shared__ double sVj[kCovTile][kCovChunk + 1];
    __shared__ double sX[kCovTile][kCovChunk + 1];
    const int i0 = blockIdx.y * kCovTile, j0 = blockIdx.z * kCovTile;
    const int ni = min(kCovTile, nq - i0), nj = min(kCovTile, nq - j0);
    double acc[kCovPairs];
#pragma unroll
    for (int r = 0; r < kCovPairs; ++r) acc[r] = 0.0;
    const int64_t nchunk = (M + kCovChunk - 1) / kCovChunk;
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int64_t k0 = ch * kCovChunk;
        __syncthreads();
        for (int e = threadIdx.x; e < kCovTile * kCovChunk; e += 256) {
            const int a = e / kCovChunk, kk = e % kCovChunk;
            const int64_t k = k0 + kk;
            const bool oki = k < M && a < ni, okj = k < M && a < nj;
            const int64_t oi = (int64_t)(i0 + a) * M + k, oj = (int64_t)(j0 + a) * M + k;
            sG[a][kk] = oki ? G[oi] : 0.0;
            sVi[a][kk] = oki ? V[oi] : 0.0;
            sVj[a][kk] = okj ? V[oj] : 0.0;
            sX[a][kk] = okj ? X[oj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kCovPairs; ++r) {
            const int p = threadIdx.x + 256 * r;
            const int a = p / kCovTile, b = p % kCovTile;
            double t = 0.0;
#pragma unroll 8
            for (int kk = 0; kk < kCovChunk; ++kk)
                t = fma(sG[a][kk], sVj[b][kk], fma(-sVi[a][kk], sX[b][kk], t));
            acc[r] += t;
        }
    }
    const int tile = blockIdx.y * gridDim.z + blockIdx.z;
    double* out = partials + ((int64_t)tile * gridDim.x + blockIdx.x) * (kCovTile * kCovTile);
#pragma unroll
    for (int r = 0; r < kCovPairs; ++r) out[threadIdx.x + 256 * r] = acc[r];
}

// cov[i][j] = symmetric part of the summed partials (fixed order).
__global__ void cov_fin(const double* __restrict__ partials, int nb, int nq, int nt,
                        double* __restrict__ cov) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)nq * nq) return;
    const int i = (int)(p / nq), j = (int)(p % nq);
    auto sum = [&](int r, int c) {
        const int tile = (r / kCovTile) * nt + c / kCovTile;
        const double* q = partials + (int64_t)tile * nb * (kCovTile * kCovTile) +
                          (r % kCovTile) * kCovTile + c % kCovTile;
        double a = 0.0;
        for (int k = 0; k < nb; ++k) a += q[(int64_t)k * (kCovTile * kCovTile)];
        return a;
    };
    cov[p] = 0.5 * (sum(i, j) + sum(j, i));
}

fkgp_status posterior_cov_impl(const fkgp_handle* h, const fkgp_hypers* hyp,
                               const void* const* xq, int64_t nq64, fkgp_dtype in, double tol,
                               int maxiter, double* cov, fkgp_solve_info* info,
                               hipStream_t st) {
    Scratch sc(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, FKGP_F64, c, sc);
    if (rs != FKGP_OK) return rs;
    const int nq = (int)nq64;
    const int64_t M = h->M;
    const int64_t ldx = M + 2 * c.halo;
    double *G, *V, *WX;
    unsigned long long* bad;
    FKGP_HIP(sc.get(&G, M * nq));
    FKGP_HIP(sc.get(&V, M * nq));
    FKGP_HIP(sc.get(&WX, M * nq));
    FKGP_HIP(sc.get(&bad, 1));
    FKGP_HIP(hipMemsetAsync(G, 0, sizeof(double) * M * nq, st));
    FKGP_HIP(hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), st));
    rs = query_weights(h->g, xq, nq, in, G, bad, st);
    if (rs != FKGP_OK) return rs;
    unsigned long long hbad = ~0ull;
    FKGP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    if (hbad != ~0ull) {
        set_error("query point " + std::to_string(hbad) + " lies outside the interpolable region");
        return FKGP_EOUTOFGRID;
    }
    int iters_max = 0;
    double rel = 0.0;
    bool conv = true;
    for (int q0 = 0; q0 < nq; q0 += kCovRhs) {
        const int nr = std::min(kCovRhs, nq - q0);
        Scratch sj(st);
        double *Vpad, *BH, *bb, *alphas, *betas, *dotp;
        PState* ps;
        FKGP_HIP(sj.get(&Vpad, ldx * nr));
        FKGP_HIP(sj.get(&BH, M * nr));
        FKGP_HIP(sj.get(&bb, nr));
        FKGP_HIP(sj.get(&alphas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&betas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&dotp, (size_t)vec_blocks(M) * nr));
        FKGP_HIP(sj.get(&ps, nr));
        double* Vq = V + (int64_t)q0 * M;
        // v_j = K_G g_j, b_hat_j = W^T W v_j, ||b_j||^2 = v_j . b_hat_j
        rs = kg_apply(h->g, c.sp64, FKGP_F64, G + (int64_t)q0 * M, Vq, nr, c.so, nullptr, 0.0,
                      nullptr, st);
        if (rs != FKGP_OK) return rs;
        FKGP_HIP(hipMemsetAsync(Vpad, 0, sizeof(double) * ldx * nr, st));
        FKGP_HIP(hipMemcpy2DAsync(Vpad + c.halo, sizeof(double) * ldx, Vq, sizeof(double) * M,
                                  sizeof(double) * M, nr, hipMemcpyDeviceToDevice, st));
        rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, Vpad, BH, nr, c.halo, nullptr,
                          st);
        if (rs != FKGP_OK) return rs;
        rs = dots_dev(Vq, BH, M, nr, dotp, bb, st);
        if (rs != FKGP_OK) return rs;
        int it = 0;
        const fkgp_status cres = probe_cg(c, BH, nr, (double)h->n, tol, maxiter,
                                          WX + (int64_t)q0 * M, alphas, betas, ps, sj, st, it, bb,
                                          Vq);
        if (cres != FKGP_OK && cres != FKGP_ENOTCONV) return cres;
        conv &= cres == FKGP_OK;
        iters_max = std::max(iters_max, it);
        std::vector<PState> hs(nr);
        FKGP_HIP(hipMemcpyAsync(hs.data(), ps, sizeof(PState) * nr, hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < nr; ++j)
            if (hs[j].bb > 0) rel = std::max(rel, std::sqrt(std::max(hs[j].rho, 0.0) / hs[j].bb));
    }
    const int nt = (nq + kCovTile - 1) / kCovTile;
    const int64_t nchunk = (M + kCovChunk - 1) / kCovChunk;
    // about 2048 blocks in all, 8 to 256 per tile, at most one per chunk
    const int64_t per_tile = std::min<int64_t>(256, std::max<int64_t>(8, 2048 / ((int64_t)nt * nt)));
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(nchunk, per_tile));
    double* partials;
    FKGP_HIP(sc.get(&partials, (size_t)nt * nt * nb * kCovTile * kCovTile));
    cov_partial<<<dim3(nb, nt, nt), 256, 0, st>>>(G, V, WX, M, nq, partials);
    const int64_t P = (int64_t)nq * nq;
    cov_fin<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(partials, nb, nq, nt, cov);
    FKGP_HIP(hipGetLastError());
    FKGP_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iterations = iters_max;
        info->converged = conv ? 1 : 0;
        info->rel_residual = rel;
    }
    return conv ? FKGP_OK : FKGP_ENOTCONV;
}

// ---------------------------------------------------------------------------
// Rank-k posterior covariance (the low-rank covariance of Sec. 5) from the
// efficiently factorized Lanczos algorithm (Alg. 7) on A = W K_G W^T + s2 I
// started at y / ||y||.  The i-th Lanczos vector is Q_i = W qh_i + d_i y,
// kept as (qh_i, d_i) with p_i = W^T W qh_i and s_i = (K_G W^T W + s2 I) qh_i;
// A Q_i = W (s_i + d_i K_G W^T y) + s2 d_i y, and for two such vectors
//   <(a, ca), (e, ce)> = p_a . e + ca (W^T y . e) + ce (W^T y . a) + ca ce y^T y,
// so one operator B per step and only the statistics enter.  The new vector
// is orthogonalised against all earlier ones by two classical Gram-Schmidt
// passes (lambda_j = <Q_j, w>, with e_j = qh_j . W^T y kept per vector).
// The cache holds C = L^{-1} (K_G (P + W^T y d^T))^T with T = L L^T (L lower
// bidiagonal), so that for query weights w_x
//   cov(x, x') ~ w_x^T K_G w_x' - (C^T w_x) . (C^T w_x').
// ---------------------------------------------------------------------------
constexpr int kLoveMaxRank = 10000;
constexpr int kMdRows = 8;

// w = s_cur + d_i kb - beta_prev qprev (s_cur, qprev may be null: zero);
// state[0] = wc0 (the y-coefficient of the new vector).
__global__ void lz_start(double* __restrict__ wq, const double* __restrict__ s_cur,
                         const double* __restrict__ kb, const double* __restrict__ qprev,
                         double di, double bprev, int64_t M, double* state, double wc0) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) state[0] = wc0;
    if (r >= M) return;
    double v = di * kb[r];
    if (s_cur) v += s_cur[r];
    if (qprev) v = fma(-bprev, qprev[r], v);
    wq[r] = v;
}

// Partial dot products of x with rows 0..nr-1 of R (stride M) and with xb
// (row nr): partials[row][gridDim.x].
__global__ __launch_bounds__(kRedBlock) void mdot_kernel(const double* __restrict__ R, int nr,
                                                         const double* __restrict__ xb,
                                                         const double* __restrict__ x, int64_t M,
                                                         double* __restrict__ partials) {
    __shared__ double sh[kRedBlock];
    const int r0 = blockIdx.y * kMdRows;
    const int nrows = min(kMdRows, nr + 1 - r0);
    double acc[kMdRows];
#pragma unroll
    for (int q = 0; q < kMdRows; ++q) acc[q] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * kRedBlock) {
        const double xv = x[t];
#pragma unroll
        for (int q = 0; q < kMdRows; ++q) {
            if (q >= nrows) continue;
            const int row = r0 + q;
            const double* rp = row < nr ? R + (int64_t)row * M : xb;
            acc[q] = fma(rp[t], xv, acc[q]);
        }
    }
    for (int q = 0; q < nrows; ++q) {
        const double t = block_sum(acc[q], sh);
        if (threadIdx.x == 0) partials[(int64_t)(r0 + q) * gridDim.x + blockIdx.x] = t;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedBlock) void mdot_fin(const double* __restrict__ partials,
                                                      int nbk, double* __restrict__ raw) {
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nbk; i += kRedBlock)
        acc += partials[(int64_t)blockIdx.x * nbk + i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) raw[blockIdx.x] = t;
}

int mdot_blocks(int64_t M, int nrows) {
    const int ny = (nrows + kMdRows - 1) / kMdRows;
    const int64_t want = std::max<int64_t>(4, 4096 / ny);
    return (int)std::max<int64_t>(1, std::min<int64_t>(vec_blocks(M), want));
}

// raw[j] = R_j . x (j < nr), raw[nr] = xb . x
fkgp_status mdot(const double* R, int nr, const double* xb, const double* x, int64_t M,
                 double* partials, double* raw, hipStream_t st) {
    const int nbk = mdot_blocks(M, nr + 1);
    const int ny = (nr + 1 + kMdRows - 1) / kMdRows;
    mdot_kernel<<<dim3(nbk, ny), kRedBlock, 0, st>>>(R, nr, xb, x, M, partials);
    mdot_fin<<<nr + 1, kRedBlock, 0, st>>>(partials, nbk, raw);
    FKGP_HIP(hipGetLastError());
    return FKGP_OK;
}

// alpha_i = <Q_i, w> from raw = [p_i . w, yhat . w]; then wc -= alpha_i d_i.
__global__ void lz_alpha(const double* __restrict__ raw, double di, double ei, double bb,
                         double* state, double* alpha_i) {
    const double wc = state[0];
    const double al = raw[0] + di * raw[1] + wc * ei + di * wc * bb;
    *alpha_i = al;
    state[1] = al;
    state[0] = wc - al * di;
}

// w -= alpha_i qh_i
__global__ void lz_axpy(double* __restrict__ wq, const double* __restrict__ qi,
                        const double* __restrict__ state, int64_t M) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < M) wq[r] = fma(-state[1], qi[r], wq[r]);
}

// lambda_j = <Q_j, w> for j < nj from raw = [p_j . w (j < nj), yhat . w];
// wc -= sum_j lambda_j d_j (fixed-order block sum).
__global__ __launch_bounds__(kRedBlock) void lz_lambda(const double* __restrict__ raw,
                                                       const double* __restrict__ d,
                                                       const double* __restrict__ e, int nj,
                                                       double bb, double* state,
                                                       double* __restrict__ lam) {
    __shared__ double sh[kRedBlock];
    const double wc = state[0];
    const double rb = raw[nj];
    double acc = 0.0;
    for (int j = threadIdx.x; j < nj; j += kRedBlock) {
        const double l = raw[j] + d[j] * rb + wc * e[j] + d[j] * wc * bb;
        lam[j] = l;
        acc = fma(l, d[j], acc);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) state[0] = wc - t;
}

// w -= sum_j lambda_j qh_j (rows of Qh, j < nj), one thread per grid node.
constexpr int kLamChunk = 1024;
__global__ __launch_bounds__(256) void lz_update(double* __restrict__ wq,
                                                 const double* __restrict__ Qh,
                                                 const double* __restrict__ lam, int nj,
                                                 int64_t M) {
    __shared__ double sl[kLamChunk];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = r < M ? wq[r] : 0.0;
    for (int j0 = 0; j0 < nj; j0 += kLamChunk) {
        const int nc = min(kLamChunk, nj - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < nc; t += blockDim.x) sl[t] = lam[j0 + t];
        __syncthreads();
        if (r < M) {
            const double* q = Qh + (int64_t)j0 * M + r;
#pragma unroll 4
            for (int j = 0; j < nc; ++j) acc = fma(-sl[j], q[(int64_t)j * M], acc);
        }
    }
    if (r < M) wq[r] = acc;
}

__global__ void lz_beta(const double* __restrict__ raw, double bb, double* state) {
    const double wc = state[0];
    const double b2 = raw[0] + 2.0 * wc * raw[1] + wc * wc * bb;
    state[2] = sqrt(fmax(b2, 0.0));
    state[3] = raw[1];
}

// qh_{i+1} = w / beta, p_{i+1} /= beta, s_{i+1} = s_next / beta; d, e entries.
__global__ void lz_norm(const double* __restrict__ wq, double* __restrict__ qn,
                        double* __restrict__ pn, const double* __restrict__ s_next,
                        double* __restrict__ s_cur, double inv, int64_t M, double* d_slot,
                        double dv, double* e_slot, double ev) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) {
        *d_slot = dv;
        *e_slot = ev;
    }
    if (r >= M) return;
    qn[r] = wq[r] * inv;
    pn[r] *= inv;
    s_cur[r] = s_next[r] * inv;
}

// rows j < kk of P: P_j += d_j yhat
__global__ void lz_addb(double* __restrict__ P, const double* __restrict__ d,
                        const double* __restrict__ yhat, int kk, int64_t M) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    const double b = yhat[r];
    for (int j = 0; j < kk; ++j) P[(int64_t)j * M + r] = fma(d[j], b, P[(int64_t)j * M + r]);
}

// C_j = (K_j - lsub_j C_{j-1}) / ldiag_j  (forward substitution with the
// lower bidiagonal Cholesky factor of T), C stored [kk][M].
__global__ void lz_forward(const double* __restrict__ K, const double* __restrict__ ldiag,
                           const double* __restrict__ lsub, int kk, int64_t M,
                           double* __restrict__ C) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    double prev = 0.0;
    for (int j = 0; j < kk; ++j) {
        const double c = (K[(int64_t)j * M + r] - lsub[j] * prev) / ldiag[j];
        C[(int64_t)j * M + r] = c;
        prev = c;
    }
}

// out [cols][rows] = in [rows][cols]^T through 32 x 32 LDS tiles.
__global__ void transpose_kernel(const double* __restrict__ in, int64_t rows, int64_t cols,
                                 double* __restrict__ out) {
    __shared__ double t[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    for (int y = threadIdx.y; y < 32; y += 8) {
        const int64_t r = r0 + y, c = c0 + threadIdx.x;
        if (r < rows && c < cols) t[y][threadIdx.x] = in[r * cols + c];
    }
    __syncthreads();
    for (int y = threadIdx.y; y < 32; y += 8) {
        const int64_t c = c0 + y, r = r0 + threadIdx.x;
        if (c < cols && r < rows) out[c * rows + r] = t[threadIdx.x][y];
    }
}

fkgp_status love_build_impl(const fkgp_handle* h, const fkgp_hypers* hyp, int k, hipStream_t st,
                            fkgp_love* L) {
    Scratch sc(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, FKGP_F64, c, sc);
    if (rs != FKGP_OK) return rs;
    const int64_t M = h->M;
    const int64_t ldx = M + 2 * c.halo;
    const double bb = h->yty;
    const double* yhat = h->wty;
    double *Qh, *P, *s_cur, *s_next, *wq, *wpad, *kb, *raw, *lam, *partials, *d, *e, *alpha,
        *state;
    FKGP_HIP(sc.get(&Qh, (size_t)k * M));
    FKGP_HIP(sc.get(&P, (size_t)k * M));
    FKGP_HIP(sc.get(&s_cur, M));
    FKGP_HIP(sc.get(&s_next, M));
    FKGP_HIP(sc.get(&wq, M));
    FKGP_HIP(sc.get(&wpad, ldx));
    FKGP_HIP(sc.get(&kb, M));
    FKGP_HIP(sc.get(&raw, (size_t)k + 2));
    FKGP_HIP(sc.get(&lam, (size_t)k + 1));
    FKGP_HIP(sc.get(&partials, (size_t)(k + 8) * mdot_blocks(M, 1)));
    FKGP_HIP(sc.get(&d, k));
    FKGP_HIP(sc.get(&e, k));
    FKGP_HIP(sc.get(&alpha, k));
    FKGP_HIP(sc.get(&state, 4));
    FKGP_HIP(hipMemsetAsync(Qh, 0, sizeof(double) * M, st));
    FKGP_HIP(hipMemsetAsync(P, 0, sizeof(double) * M, st));
    FKGP_HIP(hipMemsetAsync(wpad, 0, sizeof(double) * ldx, st));
    rs = kg_apply(h->g, c.sp64, FKGP_F64, yhat, kb, 1, c.so, nullptr, 0.0, nullptr, st);
    if (rs != FKGP_OK) return rs;
    std::vector<double> hd(k, 0.0), he(k, 0.0), hal(k, 0.0), hbe(k, 0.0);
    hd[0] = 1.0 / std::sqrt(bb);
    FKGP_HIP(hipMemcpyAsync(d, hd.data(), sizeof(double), hipMemcpyHostToDevice, st));
    FKGP_HIP(hipMemcpyAsync(e, he.data(), sizeof(double), hipMemcpyHostToDevice, st));
    const unsigned ge = (unsigned)((M + 255) / 256);
    int kk = k;
    double maxal = 0.0;
    double hs[4];
    for (int i = 0; i < k; ++i) {
        const double* qi = Qh + (int64_t)i * M;
        const double wc0 = c.s2 * hd[i] - (i > 0 ? hbe[i - 1] * hd[i - 1] : 0.0);
        lz_start<<<ge, 256, 0, st>>>(wq, i > 0 ? s_cur : nullptr, kb,
                                     i > 0 ? Qh + (int64_t)(i - 1) * M : nullptr, hd[i],
                                     i > 0 ? hbe[i - 1] : 0.0, M, state, wc0);
        FKGP_HIP(hipGetLastError());
        rs = mdot(P + (int64_t)i * M, 1, yhat, wq, M, partials, raw, st);
        if (rs != FKGP_OK) return rs;
        lz_alpha<<<1, 1, 0, st>>>(raw, hd[i], he[i], bb, state, alpha + i);
        FKGP_HIP(hipGetLastError());
        if (i == k - 1) break;
        lz_axpy<<<ge, 256, 0, st>>>(wq, qi, state, M);
        FKGP_HIP(hipGetLastError());
        for (int pass = 0; pass < 2; ++pass) {
            rs = mdot(P, i + 1, yhat, wq, M, partials, raw, st);
            if (rs != FKGP_OK) return rs;
            lz_lambda<<<1, kRedBlock, 0, st>>>(raw, d, e, i + 1, bb, state, lam);
            lz_update<<<ge, 256, 0, st>>>(wq, Qh, lam, i + 1, M);
            FKGP_HIP(hipGetLastError());
        }
        double* pn = P + (int64_t)(i + 1) * M;
        FKGP_HIP(hipMemcpyAsync(wpad + c.halo, wq, sizeof(double) * M, hipMemcpyDeviceToDevice,
                                st));
        rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, wpad, pn, 1, c.halo, nullptr, st);
        if (rs != FKGP_OK) return rs;
        rs = kg_apply(h->g, c.sp64, FKGP_F64, pn, s_next, 1, c.so, wq, c.s2, nullptr, st);
        if (rs != FKGP_OK) return rs;
        rs = mdot(pn, 1, yhat, wq, M, partials, raw, st);
        if (rs != FKGP_OK) return rs;
        lz_beta<<<1, 1, 0, st>>>(raw, bb, state);
        FKGP_HIP(hipGetLastError());
        FKGP_HIP(hipMemcpyAsync(hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipStreamSynchronize(st));
        hal[i] = hs[1];
        maxal = std::max(maxal, std::fabs(hs[1]));
        const double beta = hs[2];
        if (!std::isfinite(beta) || !std::isfinite(hs[1])) {
            set_error("factorized Lanczos broke down (non-finite coefficient)");
            return FKGP_EDEVICE;
        }
        if (!(beta > 1e-10 * maxal)) {
            kk = i + 1;
            break;
        }
        hbe[i] = beta;
        hd[i + 1] = hs[0] / beta;
        he[i + 1] = hs[3] / beta;
        lz_norm<<<ge, 256, 0, st>>>(wq, Qh + (int64_t)(i + 1) * M, pn, s_next, s_cur, 1.0 / beta,
                                    M, d + i + 1, hd[i + 1], e + i + 1, he[i + 1]);
        FKGP_HIP(hipGetLastError());
    }
    FKGP_HIP(hipMemcpyAsync(hal.data(), alpha, sizeof(double) * kk, hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    // Cholesky of the tridiagonal T = L L^T (L lower bidiagonal)
    std::vector<double> ld(kk), ls(kk, 0.0);
    for (int j = 0; j < kk; ++j) {
        double t = hal[j];
        if (j > 0) {
            ls[j] = hbe[j - 1] / ld[j - 1];
            t -= ls[j] * ls[j];
        }
        if (!(t > 0.0) || !std::isfinite(t)) {
            set_error("Lanczos tridiagonal is not positive definite");
            return FKGP_EDEVICE;
        }
        ld[j] = std::sqrt(t);
    }
    double *dld, *dls;
    FKGP_HIP(sc.get(&dld, kk));
    FKGP_HIP(sc.get(&dls, kk));
    FKGP_HIP(hipMemcpyAsync(dld, ld.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
    FKGP_HIP(hipMemcpyAsync(dls, ls.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
    // rows P_j + d_j yhat, then K_G of them (into Qh), then C (into P)
    lz_addb<<<ge, 256, 0, st>>>(P, d, yhat, kk, M);
    FKGP_HIP(hipGetLastError());
    for (int j0 = 0; j0 < kk; j0 += 64) {
        const int nr = std::min(64, kk - j0);
        rs = kg_apply(h->g, c.sp64, FKGP_F64, P + (int64_t)j0 * M, Qh + (int64_t)j0 * M, nr, c.so,
                      nullptr, 0.0, nullptr, st);
        if (rs != FKGP_OK) return rs;
    }
    lz_forward<<<ge, 256, 0, st>>>(Qh, dld, dls, kk, M, P);
    FKGP_HIP(hipGetLastError());
    L->alloc = current_alloc();
    FKGP_HIP(dev_malloc(L->alloc, reinterpret_cast<void**>(&L->Ct), sizeof(double) * M * kk, st));
    transpose_kernel<<<dim3((unsigned)((M + 31) / 32), (unsigned)((kk + 31) / 32)), dim3(32, 8), 0,
                       st>>>(P, kk, M, L->Ct);
    FKGP_HIP(hipGetLastError());
    FKGP_HIP(hipStreamSynchronize(st));
    L->k = kk;
    L->alpha.assign(hal.begin(), hal.begin() + kk);
    L->beta.assign(hbe.begin(), hbe.begin() + std::max(kk - 1, 0));
    L->d.assign(hd.begin(), hd.begin() + kk);
    return FKGP_OK;
}

fkgp_status love_cov_impl(const fkgp_love* L, const void* const* xq, int nq, fkgp_dtype in,
                          double* cov, hipStream_t st) {
    Scratch sc(st);
    int* first;
    double *w, *U, *partials;
    unsigned long long* bad;
    FKGP_HIP(sc.get(&first, (size_t)nq * 3));
    FKGP_HIP(sc.get(&w, (size_t)nq * 12));
    FKGP_HIP(sc.get(&U, (size_t)nq * L->k));
    FKGP_HIP(sc.get(&partials, love_partials_doubles(nq, L->k, nullptr)));
    FKGP_HIP(sc.get(&bad, 1));
    FKGP_HIP(hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), st));
    fkgp_status rs = query_stencils(L->g, xq, nq, in, first, w, bad, st);
    if (rs != FKGP_OK) return rs;
    unsigned long long hbad = ~0ull;
    FKGP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, st));
    FKGP_HIP(hipStreamSynchronize(st));
    if (hbad != ~0ull) {
        set_error("query point " + std::to_string(hbad) + " lies outside the interpolable region");
        return FKGP_EOUTOFGRID;
    }
    rs = love_query(L->g, L->kind, L->ell, L->so, L->Ct, L->k, first, w, nq, U, partials, cov, st);
    if (rs != FKGP_OK) return rs;
    FKGP_HIP(hipStreamSynchronize(st));
    return FKGP_OK;
}

// k grid right-hand sides b_j = W rhs_j at once: out_j = W^T A^{-1} W rhs_j,
// batches of 64 through the batched factorized CG (FP64, started from
// r_hat = rhs_j; one W^T W read per iteration for the batch).
fkgp_status solve_multi_impl(const fkgp_handle* h, const fkgp_hypers* hyp, const double* rhs,
                             int k, double* out, double tol, int maxiter, fkgp_solve_info* info,
                             hipStream_t st) {
    Scratch sc(st);
    OpCtx c;
    fkgp_status rs = make_ctx(h, hyp, FKGP_F64, c, sc);
    if (rs != FKGP_OK) return rs;
    const int64_t M = h->M;
    const int64_t ldx = M + 2 * c.halo;
    int iters_max = 0;
    double rel = 0.0;
    bool conv = true;
    for (int q0 = 0; q0 < k; q0 += kCovRhs) {
        const int nr = std::min(kCovRhs, k - q0);
        Scratch sj(st);
        double *Vpad, *BH, *bb, *alphas, *betas, *dotp;
        PState* ps;
        FKGP_HIP(sj.get(&Vpad, ldx * nr));
        FKGP_HIP(sj.get(&BH, M * nr));
        FKGP_HIP(sj.get(&bb, nr));
        FKGP_HIP(sj.get(&alphas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&betas, (size_t)kMaxLanczos * nr));
        FKGP_HIP(sj.get(&dotp, (size_t)vec_blocks(M) * nr));
        FKGP_HIP(sj.get(&ps, nr));
        const double* R = rhs + (int64_t)q0 * M;
        FKGP_HIP(hipMemsetAsync(Vpad, 0, sizeof(double) * ldx * nr, st));
        FKGP_HIP(hipMemcpy2DAsync(Vpad + c.halo, sizeof(double) * ldx, R, sizeof(double) * M,
                                  sizeof(double) * M, nr, hipMemcpyDeviceToDevice, st));
        rs = spmv_dia_any(h->g, h->dt, FKGP_F64, h->A, h->bmask, Vpad, BH, nr, c.halo, nullptr,
                          st);
        if (rs != FKGP_OK) return rs;
        rs = dots_dev(R, BH, M, nr, dotp, bb, st);
        if (rs != FKGP_OK) return rs;
        int it = 0;
        const fkgp_status cres = probe_cg(c, BH, nr, (double)h->n, tol, maxiter,
                                          out + (int64_t)q0 * M, alphas, betas, ps, sj, st, it,
                                          bb, R);
        if (cres != FKGP_OK && cres != FKGP_ENOTCONV) return cres;
        conv &= cres == FKGP_OK;
        iters_max = std::max(iters_max, it);
        std::vector<PState> hs(nr);
        FKGP_HIP(hipMemcpyAsync(hs.data(), ps, sizeof(PState) * nr, hipMemcpyDeviceToHost, st));
        FKGP_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < nr; ++j)
            if (hs[j].bb > 0) rel = std::max(rel, std::sqrt(std::max(hs[j].rho, 0.0) / hs[j].bb));
    }
    if (info) {
        info->iterations = iters_max;
        info->converged = conv ? 1 : 0;
        info->rel_residual = rel;
    }
    return conv ? FKGP_OK : FKGP_ENOTCONV;
}

}  // namespace
}  // namespace fkgp

extern "C" fkgp_status fkgp_mll_and_grad(const fkgp_handle* h, const fkgp_hypers* hyp,
                                         const fkgp_mll_opts* opts, double* mll, double* grad,
                                         fkgp_mll_info* info, void* stream) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!h || !mll || !grad) {
            fkgp::set_error("handle, mll and grad must be non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = fkgp::check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        if (h->nprobe <= 0) {
            fkgp::set_error("the handle has no probe sketches (n_probes = 0 at precompute)");
            return FKGP_EINVAL;
        }
        if (h->n <= 0) {
            fkgp::set_error("the marginal likelihood needs n > 0");
            return FKGP_EINVAL;
        }
        fkgp_mll_opts o{30, 1e-6, 1000, 1, 0, 0, 0};
        if (opts) o = *opts;
        if (o.lanczos_steps < 1 || o.lanczos_steps > fkgp::kMaxLanczos || !(o.tol >= 0.0) ||
            o.maxiter < 1) {
            fkgp::set_error("lanczos_steps must be in [1, 64], tol >= 0, maxiter >= 1");
            return FKGP_EINVAL;
        }
        if (o.trace_mode < 0 || o.trace_mode > 2) {
            fkgp::set_error("trace_mode must be 0 (Hutchinson), 1 (exact) or 2 (gradient of "
                            "the Lanczos estimate)");
            return FKGP_EINVAL;
        }
        if (o.trace_mode == 1 && h->M > 4096) {
            fkgp::set_error("exact traces need m <= 4096 (one solve per grid node)");
            return FKGP_EINVAL;
        }
        return fkgp::mll_impl(h, hyp, o, mll, grad, info, static_cast<hipStream_t>(stream));
    });
}

extern "C" fkgp_status fkgp_posterior_cov(const fkgp_handle* h, const fkgp_hypers* hyp,
                                          const void* const* xq, int64_t nq, fkgp_dtype in,
                                          double tol, int maxiter, double* cov,
                                          fkgp_solve_info* info, void* stream) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!h || !xq || !cov) {
            fkgp::set_error("handle, xq and cov must be non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = fkgp::check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        if (nq < 1 || nq > fkgp::kCovMaxQ) {
            fkgp::set_error("nq must be in [1, 4096]");
            return FKGP_EINVAL;
        }
        if (in != FKGP_F32 && in != FKGP_F64) {
            fkgp::set_error("unknown point dtype");
            return FKGP_EINVAL;
        }
        for (int k = 0; k < h->g.d; ++k)
            if (!xq[k]) {
                fkgp::set_error("xq[k] is NULL");
                return FKGP_EINVAL;
            }
        if (!(tol >= 0.0) || maxiter < 1) {
            fkgp::set_error("tol must be >= 0 and maxiter >= 1");
            return FKGP_EINVAL;
        }
        return fkgp::posterior_cov_impl(h, hyp, xq, nq, in, tol, maxiter, cov, info,
                                        static_cast<hipStream_t>(stream));
    });
}

extern "C" fkgp_status fkgp_love_build(const fkgp_handle* h, const fkgp_hypers* hyp, int k,
                                       void* stream, fkgp_love** out) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!out) {
            fkgp::set_error("out must be non-NULL");
            return FKGP_EINVAL;
        }
        *out = nullptr;
        if (!h) {
            fkgp::set_error("handle must be non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = fkgp::check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        if (k < 1 || k > fkgp::kLoveMaxRank) {
            fkgp::set_error("k must be in [1, 10000]");
            return FKGP_EINVAL;
        }
        if (!(h->yty > 0.0)) {
            fkgp::set_error("the factorized Lanczos starts at y: needs y^T y > 0");
            return FKGP_EINVAL;
        }
        const int kc = (int)std::min<int64_t>(k, h->M + 1);
        auto* L = new fkgp_love();
        L->g = h->g;
        L->kind = hyp->kernel;
        for (int i = 0; i < 3; ++i) L->ell[i] = i < h->g.d ? hyp->lengthscale[i] : 1.0;
        L->so = hyp->outputscale;
        (void)hipGetDevice(&L->dev);
        st = fkgp::love_build_impl(h, hyp, kc, static_cast<hipStream_t>(stream), L);
        if (st != FKGP_OK) {
            (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
            fkgp::dev_free(L->alloc, L->Ct, static_cast<hipStream_t>(stream));
            (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
            delete L;
            return st;
        }
        *out = L;
        return FKGP_OK;
    });
}

extern "C" fkgp_status fkgp_love_tridiag(const fkgp_love* c, int* rank, double* alpha,
                                         double* beta, double* d) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!c || !rank) {
            fkgp::set_error("cache and rank must be non-NULL");
            return FKGP_EINVAL;
        }
        *rank = c->k;
        if (alpha) std::copy(c->alpha.begin(), c->alpha.end(), alpha);
        if (beta) std::copy(c->beta.begin(), c->beta.end(), beta);
        if (d) std::copy(c->d.begin(), c->d.end(), d);
        return FKGP_OK;
    });
}

extern "C" fkgp_status fkgp_love_cov(const fkgp_love* c, const void* const* xq, int64_t nq,
                                     fkgp_dtype in, double* cov, void* stream) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!c || !xq || !cov) {
            fkgp::set_error("cache, xq and cov must be non-NULL");
            return FKGP_EINVAL;
        }
        if (nq < 1 || nq > fkgp::kCovMaxQ) {
            fkgp::set_error("nq must be in [1, 4096]");
            return FKGP_EINVAL;
        }
        if (in != FKGP_F32 && in != FKGP_F64) {
            fkgp::set_error("unknown point dtype");
            return FKGP_EINVAL;
        }
        for (int k = 0; k < c->g.d; ++k)
            if (!xq[k]) {
                fkgp::set_error("xq[k] is NULL");
                return FKGP_EINVAL;
            }
        return fkgp::love_cov_impl(c, xq, (int)nq, in, cov, static_cast<hipStream_t>(stream));
    });
}

extern "C" void fkgp_love_destroy(fkgp_love* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    fkgp::dev_free(c->alloc, c->Ct, nullptr);
    (void)hipStreamSynchronize(nullptr);
    delete c;
}

extern "C" fkgp_status fkgp_solve_multi(const fkgp_handle* h, const fkgp_hypers* hyp,
                                        const double* rhs_grid, int k, double* out,
                                        const fkgp_solve_opts* opts, fkgp_solve_info* info,
                                        void* stream) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!h || (k > 0 && (!rhs_grid || !out)) || k < 0) {
            fkgp::set_error("handle must be non-NULL, k >= 0, rhs_grid and out non-NULL");
            return FKGP_EINVAL;
        }
        fkgp_status st = fkgp::check_hypers(h, hyp);
        if (st != FKGP_OK) return st;
        fkgp_solve_opts o{1e-6, 1000, FKGP_OP_F64};
        if (opts) o = *opts;
        if (!(o.tol >= 0.0) || o.maxiter < 1) {
            fkgp::set_error("tol must be >= 0 and maxiter >= 1");
            return FKGP_EINVAL;
        }
        if (o.op_precision != FKGP_OP_F64) {
            fkgp::set_error("fkgp_solve_multi runs with op_precision FKGP_OP_F64");
            return FKGP_EINVAL;
        }
        if (k == 0) {
            if (info) *info = fkgp_solve_info{0, 1, 0.0};
            return FKGP_OK;
        }
        return fkgp::solve_multi_impl(h, hyp, rhs_grid, k, out, o.tol, o.maxiter, info,
                                      static_cast<hipStream_t>(stream));
    });
}

extern "C" fkgp_status fkgp_batch_mll_and_grad(const fkgp_handle* const* hs, int nprob,
                                               const fkgp_hypers* hyps,
                                               const fkgp_mll_opts* opts, double* mll,
                                               double* grad, fkgp_mll_info* infos,
                                               void* stream) {
    return guarded([&]() -> fkgp_status {
        fkgp::set_error("");
        if (!hs || !hyps || !mll || !grad || nprob < 0) {
            fkgp::set_error("handles, hypers, mll and grad must be non-NULL, nprob >= 0");
            return FKGP_EINVAL;
        }
        for (int p = 0; p < nprob; ++p) {
            const fkgp_handle* h = hs[p];
            if (!h) {
                fkgp::set_error("handle " + std::to_string(p) + " is NULL");
                return FKGP_EINVAL;
            }
            fkgp_status st = fkgp::check_hypers(h, &hyps[p]);
            if (st != FKGP_OK) return st;
            if (h->nprobe <= 0 || h->n <= 0 || h->g.d > 2) {
                fkgp::set_error("problem " + std::to_string(p) +
                                ": needs probe sketches, n > 0 and d <= 2");
                return FKGP_EINVAL;
            }
        }
        fkgp_mll_opts o{30, 1e-6, 1000, 1, 0, 0, 0};
        if (opts) o = *opts;
        if (o.lanczos_steps < 1 || o.lanczos_steps > fkgp::kMaxLanczos || !(o.tol >= 0.0) ||
            o.maxiter < 1) {
            fkgp::set_error("lanczos_steps must be in [1, 64], tol >= 0, maxiter >= 1");
            return FKGP_EINVAL;
        }
        if (o.trace_mode != 0) {
            fkgp::set_error("the batched solver uses Hutchinson traces (trace_mode 0)");
            return FKGP_EINVAL;
        }
        if ((o.batch_rhs != 0 && o.batch_rhs != 2 && o.batch_rhs != 4 && o.batch_rhs != 8) ||
            (o.batch_block != 0 && o.batch_block != 256 && o.batch_block != 512)) {
            fkgp::set_error("batch_rhs must be 0 (autotune), 2, 4 or 8 and batch_block 0, 256 "
                            "or 512");
            return FKGP_EINVAL;
        }
        return fkgp::batch_mll_impl(hs, nprob, hyps, o, mll, grad, infos,
                                    static_cast<hipStream_t>(stream));
    });
}
