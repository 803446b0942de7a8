// C ABI of the library (declared in include/mpir.h): handle and workspace
// management, the blocked LU driver and the refinement-loop driver.  Every
// arithmetic step runs in the HIP kernels of this directory; this file only
// orders launches on the caller's stream and moves status words.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "mpir_internal.h"

using namespace mpir;

namespace mpir {
hipError_t launch_set_sigma(IrState *st, hipStream_t s);
int leaf_max_rows(int mode);
// layout shared with k_batched.hip
struct BatchSys {
    int64_t n, lda;
    const void *A;
    const void *b;
    void *x;
    float *W;
    int32_t *perm;
    int64_t pad;
};
struct BatchTerm {
    double tol_r, tol_e, rmax;
    int32_t litmax, residterm, wilk, pad;
};
}

// --------------------------------------------------------------------------
// Per-kernel timing (HIP events around launches on the library's stream)
// --------------------------------------------------------------------------
namespace {

struct ProfRec {
    hipEvent_t a, b;
    double work;
};
struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> recs[6];
    std::vector<hipEvent_t> pool;
};
Prof g_prof;

hipEvent_t prof_event() {
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Scoped timing of one launch of kernel kind `k` with algorithmic work `w`.
struct ProfScope {
    int kind;
    double work;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int k, double w, hipStream_t st) : kind(k), work(w), s(st) {
        if (!g_prof.on) return;
        std::lock_guard<std::mutex> g(g_prof.mu);
        a = prof_event();
        b = prof_event();
        if (a) hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a || !b) return;
        hipEventRecord(b, s);
        std::lock_guard<std::mutex> g(g_prof.mu);
        g_prof.recs[kind].push_back({a, b, work});
    }
};

}  // namespace

// --------------------------------------------------------------------------
// Handle
// --------------------------------------------------------------------------
struct mpir_fact_s {
    int64_t n = 0, lda = 0, ld = 0;
    int tw = 0, tf = 0, tr = 0, mode = 0;
    const void *A = nullptr;        // borrowed
    hipStream_t stream = nullptr;
    void *work = nullptr;           // row-major working array (ld x n)
    __half *lu16 = nullptr;         // F16: packed binary16 factors
    __half *hws[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // F16: binary16 update operands per stream
    int32_t *ipiv = nullptr, *perm = nullptr;
    int64_t *info_d = nullptr;
    uint32_t *flags_d = nullptr;
    uint64_t *anorm_bits_d = nullptr;
    PanelSync *ps = nullptr;        // leaf exchange area (uncached, pooled)
    int ps_dev = 0;
    uint32_t ps_base = 0;
    void *r = nullptr;              // residual (TR), n doubles of room
    void *rhat = nullptr;           // low-precision right side / solution (TS)
    double *partial = nullptr;      // residual partial sums
    int nchunks = 0;
    IrState *st = nullptr;
    TrsvSync *ts = nullptr;
    uint64_t *yw = nullptr;         // epoch-tagged solution words of the solves
    double anorm = 0.0;
    int64_t info = 0;
    // 1 once a factorization completed (OK or SINGULAR); a failed refactor
    // clears it, and every solve then refuses the handle
    int valid = 0;
    double t_factor_ms = 0.0;
    hipStream_t stream2 = nullptr;  // look-ahead: trailing updates
    hipEvent_t evA[2] = {nullptr, nullptr}, evB[2] = {nullptr, nullptr};
    // GMRES-IR workspace (first use): basis (km + 1) x n, work vectors,
    // coefficients, and the state the matrix-vector products report into
    int km = 0;
    double *kv = nullptr, *kw = nullptr, *kt = nullptr, *kzero = nullptr, *kd = nullptr;
    double *kc = nullptr;
    IrState *kst = nullptr;
    // several right-hand sides (first use): per-column states, residuals,
    // scaled residuals / solutions and solution words, residual partial sums
    int mcap = 0;
    IrState *mst = nullptr;
    void *mr = nullptr, *mrhat = nullptr;
    double *mpart = nullptr;
    uint64_t *myw = nullptr;
    // BiCGSTAB-IR (first use): nine n-vectors and eight scalars, and the
    // state the matrix-vector products report into
    double *bq = nullptr;
    IrState *bst = nullptr;
};

namespace {

size_t esize(int p) { return p == MPIR_F64 ? 8 : (p == MPIR_F32 ? 4 : 2); }

// 16-bit factorization precisions (factors packed for the solves).
bool is16(int tf) { return tf == MPIR_F16 || tf == MPIR_BF16; }

bool valid_triple(int tw, int tf, int tr) {
    if (tw != MPIR_F64 && tw != MPIR_F32) return false;
    if (tf != MPIR_F64 && tf != MPIR_F32 && tf != MPIR_F16 && tf != MPIR_BF16) return false;
    if (tr != MPIR_F64 && tr != MPIR_F32) return false;
    if (tw == MPIR_F32 && tf == MPIR_F64) return false;   // TF must not exceed TW
    if (tr == MPIR_F32 && tw == MPIR_F64) return false;   // TR >= TW
    return true;
}

int lu_mode_of(int tf) {
    return tf == MPIR_F64 ? LU_F64 : tf == MPIR_F32 ? LU_F32 : tf == MPIR_BF16 ? LU_BF16 : LU_F16;
}

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t _e = (x);                       \
        if (_e != hipSuccess) return MPIR_ERR_HIP; \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t bytes) {
    return hipMalloc((void **)p, bytes ? bytes : 16);
}

// Exchange areas of the multi-workgroup leaf, in uncached device memory:
// the leaf's epoch-tagged words then travel without the L2s, which the
// concurrent trailing update keeps busy (FP32 factorization at N = 32768
// about 2% faster, binary16 about 4%).  Memory of this kind that kernels
// have read is never handed back to the runtime -- a later allocation at
// its addresses could see stale contents -- so released areas go to a
// per-device free list and are reused by later handles.  Each area is
// cleared before every factorization that uses it.
struct SyncPool {
    std::mutex mu;
    std::vector<std::pair<int, PanelSync *>> free;   // (device, area)
};
SyncPool &sync_pool() {
    static SyncPool *p = new SyncPool();   // outlives every handle
    return *p;
}

hipError_t ps_acquire(PanelSync **out, int *dev) {
    *out = nullptr;
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return e;
    {
        SyncPool &p = sync_pool();
        std::lock_guard<std::mutex> g(p.mu);
        for (size_t i = 0; i < p.free.size(); ++i)
            if (p.free[i].first == *dev) {
                *out = p.free[i].second;
                p.free.erase(p.free.begin() + (std::ptrdiff_t)i);
                return hipSuccess;
            }
    }
    e = hipExtMallocWithFlags((void **)out, panel_sync_bytes(), hipDeviceMallocUncached);
    if (e == hipSuccess) return e;
    // a device without uncached allocations: ordinary memory (pooled the same way)
    (void)hipGetLastError();
    return hipMalloc((void **)out, panel_sync_bytes());
}

void ps_release(PanelSync *ps, int dev) {
    SyncPool &p = sync_pool();
    std::lock_guard<std::mutex> g(p.mu);
    p.free.emplace_back(dev, ps);
}

void free_handle(mpir_fact f) {
    if (!f) return;
    if (f->ps) {
        // no kernel of this handle may still use the area when it is reused
        hipStreamSynchronize(f->stream);
        if (f->stream2) hipStreamSynchronize(f->stream2);
        ps_release(f->ps, f->ps_dev);
        f->ps = nullptr;
    }
    hipFree(f->work);
    hipFree(f->lu16);
    for (auto &pr : f->hws)
        for (auto *q : pr) hipFree(q);
    hipFree(f->ipiv);
    hipFree(f->perm);
    hipFree(f->info_d);
    hipFree(f->flags_d);
    hipFree(f->anorm_bits_d);
    hipFree(f->r);
    hipFree(f->rhat);
    hipFree(f->partial);
    hipFree(f->st);
    hipFree(f->ts);
    hipFree(f->yw);
    for (int i = 0; i < 2; ++i) {
        if (f->evA[i]) hipEventDestroy(f->evA[i]);
        if (f->evB[i]) hipEventDestroy(f->evB[i]);
    }
    if (f->stream2) hipStreamDestroy(f->stream2);
    for (double *q : {f->kv, f->kw, f->kt, f->kzero, f->kd, f->kc}) hipFree(q);
    hipFree(f->kst);
    hipFree(f->mst);
    hipFree(f->mr);
    hipFree(f->mrhat);
    hipFree(f->mpart);
    hipFree(f->myw);
    hipFree(f->bq);
    hipFree(f->bst);
    delete f;
}

int panel_width(int mode);

mpir_status alloc_handle(mpir_fact f) {
    const int64_t n = f->n;
    const size_t wes = f->mode == LU_F64 ? 8 : 4;
    // Row pitch of the working array: a multiple of 32 elements (aligned
    // vector loads), never a multiple of 1024 (a power-of-two pitch would map
    // every row of a column block onto the same HBM channels).
    f->ld = (n + 31) / 32 * 32;
    if (f->ld % 1024 == 0) f->ld += 32;
    if (dalloc(&f->work, (size_t)f->ld * n * wes) != hipSuccess) return MPIR_ERR_ALLOC;
    // binary16 factors for the solves: the same padded pitch
    if (is16(f->tf) && dalloc(&f->lu16, (size_t)f->ld * n * 2) != hipSuccess) return MPIR_ERR_ALLOC;
    if (is16(f->tf)) {
        const size_t hw = gemm_h16_ws_halves(n, panel_width(f->mode)) * 2;
        for (auto &pr : f->hws)
            for (auto &q : pr)
                if (dalloc(&q, hw) != hipSuccess) return MPIR_ERR_ALLOC;
    }
    f->nchunks = residual_chunks(n);
    if (dalloc(&f->ipiv, n * 4) != hipSuccess || dalloc(&f->perm, n * 4) != hipSuccess ||
        dalloc(&f->info_d, 8) != hipSuccess || dalloc(&f->flags_d, 8) != hipSuccess ||
        dalloc(&f->anorm_bits_d, 8) != hipSuccess ||
        ps_acquire(&f->ps, &f->ps_dev) != hipSuccess || dalloc(&f->r, n * 8) != hipSuccess ||
        dalloc(&f->rhat, n * 8) != hipSuccess ||
        dalloc(&f->partial, (size_t)f->nchunks * n * 8) != hipSuccess ||
        dalloc(&f->st, sizeof(IrState)) != hipSuccess || dalloc(&f->ts, sizeof(TrsvSync)) != hipSuccess ||
        dalloc(&f->yw, (size_t)n * 16) != hipSuccess)
        return MPIR_ERR_ALLOC;
    if (hipMemset(f->ts, 0, sizeof(TrsvSync)) != hipSuccess || hipMemset(f->yw, 0, (size_t)n * 16) != hipSuccess)
        return MPIR_ERR_HIP;
    // second stream (default priority) and ordering events for the look-ahead
    if (hipStreamCreateWithFlags(&f->stream2, hipStreamNonBlocking) != hipSuccess) return MPIR_ERR_HIP;
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&f->evA[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&f->evB[i], hipEventDisableTiming) != hipSuccess)
            return MPIR_ERR_HIP;
    return MPIR_OK;
}

const int kIB = 32;    // leaf width inside the panel
const int kGmresMaxBasis = 64;   // largest GMRES basis of mpir_gmres_ir_solve

// Panel width (columns per trailing update): a larger width raises the
// arithmetic intensity of the trailing update (its C tile is read and written
// once per panel), a smaller one shortens the panel.  MPIR_NB overrides the
// per-precision default (a multiple of kIB).
int panel_width(int mode) {
    static int env = -1;
    if (env < 0) {
        const char *e = std::getenv("MPIR_NB");
        env = e ? std::atoi(e) : 0;
        if (env < 0 || env % kIB) env = 0;
    }
    if (env > 0) return env;
    return mode == LU_F16 ? 512 : 512;
}

// Row interchanges of ipiv[k0 .. k0+cnt), in chunks the kernel accepts.
hipError_t laswp_chunks(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int cnt, const int32_t *ipiv,
                        int64_t c0, int64_t c1, int64_t c2, int64_t c3, int32_t *perm, bool compact,
                        hipStream_t s) {
    for (int off = 0; off < cnt; off += 256) {
        const int c = cnt - off < 256 ? cnt - off : 256;
        hipError_t e = launch_laswp(mode, a, n, ld, k0 + off, c, ipiv, c0, c1, c2, c3, perm, compact, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Columns [c0, c1) of rows [K, K+w): U12 <- L11^{-1} U12, blocked by kIB
// (small triangular solve of each kIB-row block, then the update of the
// panel rows below it).
hipError_t upper_solve(mpir_fact f, int64_t K, int w, int64_t c0, int64_t c1, int cap, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    const int mode = f->mode;
    for (int64_t k = K; k < K + w; k += kIB) {
        const int wl = (int)((K + w - k) < kIB ? (K + w - k) : kIB);
        hipError_t e = launch_trsm(mode, f->work, f->ld, k, wl, c0, c1, s);
        if (e != hipSuccess) return e;
        if (k + wl < K + w) {
            e = launch_gemm_update(mode, f->work, f->ld, k + wl, K + w - k - wl, c0, c1 - c0, k, wl, cap, 1, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Panel factorization of columns [K, K+w), rows [K, n): leaves of kIB
// columns, each followed by its interchanges, triangular solve and update
// restricted to the other columns of the panel.
hipError_t factor_panel(mpir_fact f, int64_t K, int w, hipStream_t s) {
    const int64_t n = f->n, ld = f->ld;
    const int mode = f->mode;
    void *a = f->work;
    ProfScope ps_(1, 0.0, s);
    for (int64_t k = K; k < K + w; k += kIB) {
        const int wl = (int)((K + w - k) < kIB ? (K + w - k) : kIB);
        hipError_t e = launch_leaf(mode, a, n, ld, k, wl, f->ipiv, f->info_d, f->ps, &f->ps_base,
                                   f->flags_d, s);
        if (e != hipSuccess) return e;
        if (k > K || k + wl < K + w) {
            e = launch_laswp(mode, a, n, ld, k, wl, f->ipiv, K, k, k + wl, K + w, nullptr, true, s);
            if (e != hipSuccess) return e;
        }
        if (k + wl < K + w) {
            e = launch_trsm(mode, a, ld, k, wl, k + wl, K + w, s);
            if (e != hipSuccess) return e;
            e = launch_gemm_update(mode, a, ld, k + wl, n - k - wl, k + wl, K + w - k - wl, k, wl, 0, 1, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Step of panel [K, K+w) applied to the columns [c0, c1): interchanges,
// U12, trailing update of rows [K+w, n).
// Trailing update of rows [r0, r0+m) x columns [c0, c0+nc) by the panel
// [k, k+kk); F16: binary16 operands packed first (workspace slot ws).
hipError_t trailing_update(mpir_fact f, int64_t r0, int64_t m, int64_t c0, int64_t nc, int64_t k,
                           int64_t kk, int cap, int ws, hipStream_t s) {
    if (f->mode == LU_F16 || f->mode == LU_BF16)
        return launch_gemm_update_h16(f->mode, (float *)f->work, f->ld, r0, m, c0, nc, k, kk,
                                      f->hws[ws][0], f->hws[ws][1], cap, s);
    return launch_gemm_update(f->mode, f->work, f->ld, r0, m, c0, nc, k, kk, cap, 0, s);
}

hipError_t apply_step(mpir_fact f, int64_t K, int w, int64_t c0, int64_t c1, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    const int64_t n = f->n;
    hipError_t e;
    {
        ProfScope ps_(5, 0.0, s);
        e = laswp_chunks(f->mode, f->work, n, f->ld, K, w, f->ipiv, c0, c1, c1, c1, nullptr, true, s);
        if (e != hipSuccess) return e;
        e = w <= u12_max_rows() ? launch_u12(f->mode, f->work, f->ld, K, w, c0, c1, s)
                                : upper_solve(f, K, w, c0, c1, 0, s);
        if (e != hipSuccess) return e;
    }
    if (K + w < n) {
        ProfScope ps_(0, 2.0 * (double)(n - K - w) * (double)(c1 - c0) * w, s);
        e = trailing_update(f, K + w, n - K - w, c0, c1 - c0, K, w, 0, 0, s);
    }
    return e;
}

// Blocked right-looking LU with partial pivoting on the working array, with
// a look-ahead of one panel: while the trailing update of step p runs on the
// second stream, the main stream applies step p to panel p+1 only and
// factors panel p+1 (the latency-bound part), so the panel chain is hidden
// behind the matrix-core work.  The two streams touch disjoint columns; one
// event per stream and step parity orders them.
// MPIR_LOOKAHEAD=0 runs the whole factorization on the caller's stream.
bool lookahead_enabled() {
    static int env = -1;
    if (env < 0) {
        const char *e = std::getenv("MPIR_LOOKAHEAD");
        env = (e && e[0] == '0') ? 0 : 1;
    }
    return env == 1;
}

// Occupancy cap of the trailing update while the next panel is factored
// beside it (MPIR_GEMM_CAP overrides; 0 = no cap).
int trailing_cap(int mode) {
    static int env = -2;
    if (env == -2) {
        const char *e = std::getenv("MPIR_GEMM_CAP");
        env = e ? std::atoi(e) : -1;
    }
    if (env >= 0) return env;
    // measured at N = 32768 (factorization time against the cap, with the
    // binary32 / binary16 leaves held to 128 registers per lane): binary32
    // 6; the 16-bit update 2 (248 ms against 255 at 3 or 4); binary64 2
    // (680 ms against 708 at 4 or without a cap, although the update alone
    // then runs at 47 instead of 41 TFLOP/s: the leaves beside it slow down
    // more than it gains)
    return mode == LU_F32 ? 6 : 2;
}

mpir_status getrf(mpir_fact f) {
    const int64_t n = f->n;
    const bool la = lookahead_enabled();
    hipStream_t s = f->stream, s2 = la ? f->stream2 : f->stream;
    const int cap2 = la ? trailing_cap(f->mode) : 0;
    const int nb = panel_width(f->mode);
    if (n > leaf_max_rows(f->mode)) return MPIR_ERR_ARG;
    hipEvent_t *evA = f->evA, *evB = f->evB;
    // stream 2 starts after the work already queued on the main stream
    HIPCHK(hipEventRecord(evA[1], s));
    HIPCHK(hipStreamWaitEvent(s2, evA[1], 0));
    HIPCHK(hipEventRecord(evB[1], s2));
    const int w0 = (int)(n < nb ? n : nb);
    HIPCHK(factor_panel(f, 0, w0, s));
    HIPCHK(hipEventRecord(evA[1], s));
    int p = 0;
    for (int64_t K = 0; K < n; K += nb, ++p) {
        const int w = (int)((n - K) < nb ? (n - K) : nb);
        const int64_t K1 = K + w;
        const int w1 = (int)((n - K1) < nb ? (n - K1) : nb);
        const int64_t K2 = K1 + (w1 > 0 ? w1 : 0);
        const int cur = p & 1, prev = cur ^ 1;
        // ---- stream 2: everything of step p except panel p+1's columns ----
        HIPCHK(hipStreamWaitEvent(s2, evA[prev], 0));          // panel p factored
        {
            ProfScope ps_(5, 0.0, s2);
            HIPCHK(laswp_chunks(f->mode, f->work, n, f->ld, K, w, f->ipiv, 0, K, K2, n, f->perm, false, s2));
            HIPCHK(upper_solve(f, K, w, K2, n, cap2, s2));
        }
        if (K2 < n) {
            ProfScope ps_(0, 2.0 * (double)(n - K1) * (double)(n - K2) * w, s2);
            HIPCHK(trailing_update(f, K1, n - K1, K2, n - K2, K, w, cap2, 1, s2));
        }
        HIPCHK(hipEventRecord(evB[cur], s2));
        // ---- main stream: step p on panel p+1, then factor panel p+1 ----
        if (w1 > 0) {
            HIPCHK(hipStreamWaitEvent(s, evB[prev], 0));        // step p-1 done everywhere
            HIPCHK(apply_step(f, K, w, K1, K2, s));
            HIPCHK(factor_panel(f, K1, w1, s));
            HIPCHK(hipEventRecord(evA[cur], s));
        }
    }
    HIPCHK(hipStreamWaitEvent(s, evB[(p - 1) & 1], 0));
    return MPIR_OK;
}

// Identity permutation (perm[i] = i) and zeroed status words.
__global__ void k_init_perm(int64_t n, int32_t *perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int32_t)i;
}

mpir_status factor_impl(mpir_fact f, int64_t *info) {
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    f->valid = 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(hipMemsetAsync(f->info_d, 0, 8, s));
    HIPCHK(hipMemsetAsync(f->flags_d, 0, 8, s));
    HIPCHK(hipMemsetAsync(f->anorm_bits_d, 0, 8, s));
    HIPCHK(panel_sync_reset(f->ps, s));
    f->ps_base = 0;
    k_init_perm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, f->perm);
    HIPCHK(hipGetLastError());
    {
        ProfScope ps_(4, (double)n * n * (esize(f->tw) + (f->mode == LU_F64 ? 8 : 4)), s);
        HIPCHK(launch_downcast(n, f->A, f->lda, f->tw, f->tf, f->work, f->ld, f->anorm_bits_d, f->flags_d, s));
    }
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flags & DF_NONFINITE) return MPIR_ERR_NONFINITE;
    if (flags & DF_RANGE) return MPIR_ERR_RANGE;
    mpir_status st = getrf(f);
    if (st != MPIR_OK) return st;
    if (is16(f->tf)) HIPCHK(launch_pack_half(f->tf, n, (const float *)f->work, f->ld, f->lu16, f->ld, s));
    uint64_t abits = 0;
    int64_t inf = 0;
    HIPCHK(hipMemcpyAsync(&abits, f->anorm_bits_d, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&inf, f->info_d, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    f->t_factor_ms = ms;
    std::memcpy(&f->anorm, &abits, 8);
    f->info = inf;
    if (info) *info = inf;
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    f->valid = 1;
    return inf ? MPIR_ERR_SINGULAR : MPIR_OK;
}

const void *factors_ptr(mpir_fact f) { return is16(f->tf) ? (const void *)f->lu16 : f->work; }

}  // namespace

// --------------------------------------------------------------------------
// Public entry points
// --------------------------------------------------------------------------
extern "C" {

void mpir_term_default(mpir_term *t) {
    if (!t) return;
    t->Cr = 1.0;
    t->Ce = 1.0;
    t->Rmax = 0.5;
    t->litmax = 10;
    t->residterm = 1;
    t->tol_rel = 0.0;
    t->onthefly = 0;
    t->reserved = 0;
}

const char *mpir_status_str(mpir_status s) {
    switch (s) {
    case MPIR_OK: return "ok";
    case MPIR_ERR_SINGULAR: return "exactly singular factor (zero pivot)";
    case MPIR_ERR_ARG: return "invalid argument";
    case MPIR_ERR_ALLOC: return "device allocation failed";
    case MPIR_ERR_HIP: return "HIP runtime error";
    case MPIR_ERR_NONFINITE: return "non-finite input";
    case MPIR_ERR_RANGE: return "matrix entry overflows the factorization precision";
    case MPIR_ERR_STATE: return "handle holds no factorization (its last refactor failed)";
    case MPIR_ERR_DEVICE: return "device wait expired";
    }
    return "unknown status";
}

mpir_status mpir_factor(int64_t n, const void *dA, int64_t lda, mpir_prec tw, mpir_prec tf,
                        mpir_prec tr, void *hip_stream, mpir_fact *out, int64_t *info) {
    if (out) *out = nullptr;
    if (info) *info = 0;
    if (!out || n <= 0 || !dA || lda < n || !valid_triple(tw, tf, tr)) return MPIR_ERR_ARG;
    if (n > leaf_max_rows(lu_mode_of(tf))) return MPIR_ERR_ARG;
    mpir_fact f = new (std::nothrow) mpir_fact_s();
    if (!f) return MPIR_ERR_ALLOC;
    f->n = n;
    f->lda = lda;
    f->tw = tw;
    f->tf = tf;
    f->tr = tr;
    f->mode = lu_mode_of(tf);
    f->A = dA;
    f->stream = (hipStream_t)hip_stream;
    mpir_status st = alloc_handle(f);
    if (st != MPIR_OK) { free_handle(f); return st; }
    st = factor_impl(f, info);
    if (st != MPIR_OK && st != MPIR_ERR_SINGULAR) { free_handle(f); return st; }
    *out = f;
    return st;
}

mpir_status mpir_refactor(mpir_fact f, const void *dA, int64_t lda, int64_t *info) {
    if (info) *info = 0;
    if (!f || !dA || lda < f->n) return MPIR_ERR_ARG;
    f->A = dA;
    f->lda = lda;
    return factor_impl(f, info);
}

void mpir_destroy(mpir_fact f) {
    if (!f) return;
    hipStreamSynchronize(f->stream);
    free_handle(f);
}

mpir_status mpir_solve(mpir_fact f, const void *db, void *dx) {
    if (!f || !db || !dx) return MPIR_ERR_ARG;
    if (!f->valid) return MPIR_ERR_STATE;
    if (f->info) return MPIR_ERR_SINGULAR;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    IrState h{};
    h.it = -1;
    HIPCHK(hipMemcpyAsync(f->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(launch_ir_init(n, f->tw, f->tr, db, dx, f->r, f->st, s));
    HIPCHK(launch_set_sigma(f->st, s));
    HIPCHK(launch_scale_permute(n, f->tr, f->tf, f->r, f->perm, f->rhat, f->st, f->ts, 1, s));
    {
        ProfScope ps_(2, 2.0 * (double)n * n, s);
        HIPCHK(launch_trsv(f->tf, f->tf == MPIR_F64 ? MPIR_F64 : MPIR_F32, factors_ptr(f), n, f->ld, f->rhat, f->yw,
                           f->ts, f->flags_d, f->st, 1, s));
    }
    HIPCHK(launch_update(n, f->tw, f->tf, f->rhat, dx, f->st, 1, s));
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    return MPIR_OK;
}

mpir_status mpir_ir_solve(mpir_fact f, const void *db, void *dx, const mpir_term *t,
                          mpir_report *rep) {
    if (!f || !db || !dx) return MPIR_ERR_ARG;
    mpir_term term;
    if (t) term = *t;
    else mpir_term_default(&term);
    if (term.litmax < 1 || term.litmax > MPIR_HIST_MAX - 1 || !(term.Rmax > 0.0)) return MPIR_ERR_ARG;
    if ((term.onthefly != 0 && term.onthefly != 1) || term.reserved != 0) return MPIR_ERR_ARG;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->info = f->info;
        rep->t_factor_ms = f->t_factor_ms;
    }
    if (!f->valid) return MPIR_ERR_STATE;
    if (f->info) return MPIR_ERR_SINGULAR;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    const double uw = f->tw == MPIR_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    IrState h{};
    h.it = -1;
    h.anorm = f->anorm;
    h.wilk = (f->tr == MPIR_F64 && f->tw != MPIR_F64) ? 1 : 0;
    h.residterm = term.residterm ? 1 : 0;
    h.litmax = term.litmax;
    h.tol_r = term.tol_rel > 0 ? term.tol_rel : term.Cr * uw;
    h.tol_e = term.tol_rel > 0 ? term.tol_rel : term.Ce * uw;
    h.rmax = term.Rmax;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipMemcpyAsync(f->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(f->flags_d, 0, 4, s));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_ir_init(n, f->tw, f->tr, db, dx, f->r, f->st, s));
    HIPCHK(launch_terminate(f->st, s));
    const void *LU = factors_ptr(f);
    const int64_t lld = f->ld;
    const size_t twes = esize(f->tw);
    // LPS: the scaled residual rounded to TF, binary32 substitutions (binary64
    // for TF = F64).  MPS: the residual kept in TW, substitutions in TW
    // arithmetic on the promoted factors (the same solve when TF = TW).
    const bool mps = term.onthefly && f->tf != f->tw;
    const int rprec = mps ? f->tw : f->tf;                     // rounding of rhat
    const int yprec = mps ? f->tw : (f->tf == MPIR_F64 ? MPIR_F64 : MPIR_F32);
    for (int it = 0; it < term.litmax; ++it) {
        HIPCHK(launch_scale_permute(n, f->tr, rprec, f->r, f->perm, f->rhat, f->st, f->ts, 0, s));
        {
            ProfScope ps_(2, 2.0 * (double)n * n, s);
            HIPCHK(launch_trsv(f->tf, yprec, LU, n, lld, f->rhat, f->yw, f->ts, f->flags_d, f->st, 0, s));
        }
        HIPCHK(launch_update(n, f->tw, rprec, f->rhat, dx, f->st, 0, s));
        {
            ProfScope ps_(3, (double)n * n * twes, s);
            HIPCHK(launch_residual(n, f->A, f->lda, f->tw, f->tr, db, dx, f->r, f->partial, f->nchunks,
                                   f->st, 0, s));
        }
        HIPCHK(launch_terminate(f->st, s));
        int32_t done = 0;
        HIPCHK(hipMemcpyAsync(&done, &f->st->done, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (done) break;
    }
    HIPCHK(hipEventRecord(e1, s));
    IrState hs;
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(&hs, f->st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    if (hs.it == 0 && hs.stop == MPIR_STOP_NONFINITE) return MPIR_ERR_NONFINITE;
    double rnorm = hs.rnorm, xnorm = hs.xnorm;
    if (f->tr != MPIR_F64 && hs.it > 0) {
        // report the binary64 residual of the returned x
        IrState h2{};
        h2.it = 0;
        HIPCHK(hipMemcpyAsync(f->st, &h2, sizeof(h2), hipMemcpyHostToDevice, s));
        HIPCHK(launch_residual(n, f->A, f->lda, f->tw, MPIR_F64, db, dx, f->r, f->partial, f->nchunks,
                               f->st, 1, s));
        uint64_t bits[3];
        HIPCHK(hipMemcpyAsync(bits, &f->st->rnorm_bits, 24, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::memcpy(&rnorm, &bits[0], 8);
        std::memcpy(&xnorm, &bits[2], 8);
    }
    if (rep) {
        rep->n_iter = hs.it;
        rep->stop = hs.stop;
        rep->n_hist = hs.it + 1;
        for (int k = 0; k <= hs.it && k < MPIR_HIST_MAX; ++k) rep->rhist[k] = hs.rhist[k];
        for (int k = 0; k < hs.it && k < MPIR_HIST_MAX; ++k) rep->dhist[k] = hs.dhist[k];
        rep->bnorm_inf = hs.bnorm;
        rep->anorm_inf = f->anorm;
        rep->xnorm_inf = xnorm;
        rep->relres = hs.bnorm > 0 ? rnorm / hs.bnorm : rnorm;
        const double den = f->anorm * xnorm + hs.bnorm;
        rep->bwd_err = den > 0 ? rnorm / den : 0.0;
        rep->t_ir_ms = ms;
    }
    return MPIR_OK;
}

mpir_status mpir_gmres_ir_solve(mpir_fact f, const void *db, void *dx, const mpir_term *t,
                                int32_t basissize, double gmres_tol, mpir_report *rep,
                                int32_t *khist) {
    if (!f || !db || !dx) return MPIR_ERR_ARG;
    if (f->tr != MPIR_F64) return MPIR_ERR_ARG;         // TW = F64, or F32 with TR > TW
    if (basissize < 1 || basissize > kGmresMaxBasis) return MPIR_ERR_ARG;
    mpir_term term;
    if (t) term = *t;
    else mpir_term_default(&term);
    if (term.litmax < 1 || term.litmax > MPIR_HIST_MAX - 1 || !(term.Rmax > 0.0)) return MPIR_ERR_ARG;
    if ((term.onthefly != 0 && term.onthefly != 1) || term.reserved != 0) return MPIR_ERR_ARG;
    const double eta = gmres_tol > 0.0 ? gmres_tol : 1e-13;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->info = f->info;
        rep->t_factor_ms = f->t_factor_ms;
    }
    if (!f->valid) return MPIR_ERR_STATE;
    if (f->info) return MPIR_ERR_SINGULAR;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    const int m = basissize;
    if (f->km < m) {
        HIPCHK(hipStreamSynchronize(s));
        for (double **q : {&f->kv, &f->kw, &f->kt, &f->kzero, &f->kd, &f->kc}) {
            hipFree(*q);
            *q = nullptr;
        }
        hipFree(f->kst);
        f->kst = nullptr;
        f->km = 0;
        if (dalloc(&f->kv, (size_t)(m + 1) * n * 8) != hipSuccess || dalloc(&f->kw, n * 8) != hipSuccess ||
            dalloc(&f->kt, n * 8) != hipSuccess || dalloc(&f->kzero, n * 8) != hipSuccess ||
            dalloc(&f->kd, n * 8) != hipSuccess || dalloc(&f->kc, 4 * (kGmresMaxBasis + 1) * 8) != hipSuccess ||
            dalloc(&f->kst, sizeof(IrState)) != hipSuccess)
            return MPIR_ERR_ALLOC;
        HIPCHK(hipMemsetAsync(f->kzero, 0, n * 8, s));
        HIPCHK(hipMemsetAsync(f->kst, 0, sizeof(IrState), s));
        f->km = m;
    }
    double *V = f->kv, *w = f->kw, *c1 = f->kc, *c2 = f->kc + (kGmresMaxBasis + 1),
           *nrm = f->kc + 2 * (kGmresMaxBasis + 1), *yv = f->kc + 3 * (kGmresMaxBasis + 1);
    IrState h{};
    h.it = -1;
    h.anorm = f->anorm;
    h.wilk = f->tw != MPIR_F64 ? 1 : 0;                  // TR wider than TW: eq. wilkterm
    h.residterm = term.residterm ? 1 : 0;
    h.litmax = term.litmax;
    const double uw = f->tw == MPIR_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    h.tol_r = term.tol_rel > 0 ? term.tol_rel : term.Cr * uw;
    h.tol_e = term.tol_rel > 0 ? term.tol_rel : term.Ce * uw;
    h.rmax = term.Rmax;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipMemcpyAsync(f->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(f->flags_d, 0, 4, s));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_ir_init(n, f->tw, f->tr, db, dx, f->r, f->st, s));
    HIPCHK(launch_terminate(f->st, s));
    const void *LU = factors_ptr(f);
    const int64_t lld = f->ld;
    std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m), hh(2 * (m + 1) + 1);
    auto Hk = [&](int i, int k) -> double & { return H[(size_t)i * m + k]; };
    for (int it = 0; it < term.litmax; ++it) {
        int32_t done = 0;
        HIPCHK(hipMemcpyAsync(&done, &f->st->done, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (done) break;
        // right side P (r / sigma): the permutation, the exact power-of-two
        // scaling, then the binary64 substitutions on the TF factors
        HIPCHK(launch_scale_permute(n, MPIR_F64, MPIR_F64, f->r, f->perm, w, f->st, f->ts, 1, s));
        HIPCHK(launch_trsv(f->tf, MPIR_F64, LU, n, lld, w, f->yw, f->ts, f->flags_d, f->st, 1, s));
        HIPCHK(launch_dots(n, w, n, 1, w, nrm, s));
        double b2 = 0.0;
        HIPCHK(hipMemcpyAsync(&b2, nrm, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double beta = std::sqrt(b2);
        int kend = 0;
        if (beta > 0.0 && std::isfinite(beta)) {
            HIPCHK(launch_scale(n, w, beta, V, s));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            kend = m;
            for (int k = 0; k < m; ++k) {
                const double *vk = V + (size_t)k * n;
                // w = P A v_k (the residual kernel with b = 0 gives -A v_k)
                HIPCHK(launch_residual_x64(n, f->A, f->lda, f->tw, f->kzero, vk, f->kt, f->partial,
                                           f->nchunks, f->kst, s));
                HIPCHK(launch_gather_neg(n, f->kt, f->perm, w, f->ts, s));
                HIPCHK(launch_trsv(f->tf, MPIR_F64, LU, n, lld, w, f->yw, f->ts, f->flags_d, f->st, 1, s));
                // classical Gram-Schmidt, twice, then ||w||_2
                HIPCHK(launch_dots(n, V, n, k + 1, w, c1, s));
                HIPCHK(launch_sub_combo(n, V, n, k + 1, c1, w, s));
                HIPCHK(launch_dots(n, V, n, k + 1, w, c2, s));
                HIPCHK(launch_sub_combo(n, V, n, k + 1, c2, w, s));
                HIPCHK(launch_dots(n, w, n, 1, w, nrm, s));
                HIPCHK(hipMemcpyAsync(hh.data(), c1, (size_t)(k + 1) * 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(hh.data() + (m + 1), c2, (size_t)(k + 1) * 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(hh.data() + 2 * (m + 1), nrm, 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                for (int i = 0; i <= k; ++i) Hk(i, k) = hh[i] + hh[(m + 1) + i];
                const double hk1 = std::sqrt(hh[2 * (m + 1)]);
                Hk(k + 1, k) = hk1;
                if (hk1 > 0.0) HIPCHK(launch_scale(n, w, hk1, V + (size_t)(k + 1) * n, s));
                // earlier rotations, then the one that zeroes H(k+1, k)
                for (int i = 0; i < k; ++i) {
                    const double tt = cs[i] * Hk(i, k) + sn[i] * Hk(i + 1, k);
                    Hk(i + 1, k) = -sn[i] * Hk(i, k) + cs[i] * Hk(i + 1, k);
                    Hk(i, k) = tt;
                }
                const double a = Hk(k, k), bb = Hk(k + 1, k);
                if (bb == 0.0) { cs[k] = 1.0; sn[k] = 0.0; }
                else { const double r = std::hypot(a, bb); cs[k] = a / r; sn[k] = bb / r; }
                Hk(k, k) = cs[k] * a + sn[k] * bb;
                Hk(k + 1, k) = 0.0;
                g[k + 1] = -sn[k] * g[k];
                g[k] = cs[k] * g[k];
                if (std::fabs(g[k + 1]) <= eta * beta || hk1 == 0.0 || !std::isfinite(hk1)) {
                    kend = k + 1;
                    break;
                }
            }
            for (int i = kend - 1; i >= 0; --i) {
                double acc = 0.0;
                for (int j = i + 1; j < kend; ++j) acc += Hk(i, j) * y[j];
                y[i] = (g[i] - acc) / Hk(i, i);
            }
            HIPCHK(hipMemcpyAsync(yv, y.data(), (size_t)kend * 8, hipMemcpyHostToDevice, s));
            HIPCHK(launch_combo(n, V, n, kend, yv, f->kd, s));
        } else {
            HIPCHK(hipMemsetAsync(f->kd, 0, n * 8, s));
        }
        if (khist && it < term.litmax) khist[it] = kend;
        // x <- x + sigma d, the binary64 residual, the termination rules
        HIPCHK(launch_update(n, f->tw, MPIR_F64, f->kd, dx, f->st, 0, s));
        HIPCHK(launch_residual(n, f->A, f->lda, f->tw, f->tr, db, dx, f->r, f->partial, f->nchunks,
                               f->st, 0, s));
        HIPCHK(launch_terminate(f->st, s));
    }
    HIPCHK(hipEventRecord(e1, s));
    IrState hs;
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(&hs, f->st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    if (hs.it == 0 && hs.stop == MPIR_STOP_NONFINITE) return MPIR_ERR_NONFINITE;
    if (rep) {
        rep->n_iter = hs.it;
        rep->stop = hs.stop;
        rep->n_hist = hs.it + 1;
        for (int k = 0; k <= hs.it && k < MPIR_HIST_MAX; ++k) rep->rhist[k] = hs.rhist[k];
        for (int k = 0; k < hs.it && k < MPIR_HIST_MAX; ++k) rep->dhist[k] = hs.dhist[k];
        rep->bnorm_inf = hs.bnorm;
        rep->anorm_inf = f->anorm;
        rep->xnorm_inf = hs.xnorm;
        rep->relres = hs.bnorm > 0 ? hs.rnorm / hs.bnorm : hs.rnorm;
        const double den = f->anorm * hs.xnorm + hs.bnorm;
        rep->bwd_err = den > 0 ? hs.rnorm / den : 0.0;
        rep->t_ir_ms = ms;
    }
    return MPIR_OK;
}

mpir_status mpir_bicgstab_ir_solve(mpir_fact f, const void *db, void *dx, const mpir_term *t,
                                   int32_t maxit, double inner_tol, mpir_report *rep, int32_t *khist) {
    if (!f || !db || !dx) return MPIR_ERR_ARG;
    if (f->tr != MPIR_F64) return MPIR_ERR_ARG;         // TW = F64, or F32 with TR > TW
    if (maxit < 1 || maxit > 1000) return MPIR_ERR_ARG;
    mpir_term term;
    if (t) term = *t;
    else mpir_term_default(&term);
    if (term.litmax < 1 || term.litmax > MPIR_HIST_MAX - 1 || !(term.Rmax > 0.0)) return MPIR_ERR_ARG;
    if ((term.onthefly != 0 && term.onthefly != 1) || term.reserved != 0) return MPIR_ERR_ARG;
    const double eta = inner_tol > 0.0 ? inner_tol : 1e-13;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->info = f->info;
        rep->t_factor_ms = f->t_factor_ms;
    }
    if (!f->valid) return MPIR_ERR_STATE;
    if (f->info) return MPIR_ERR_SINGULAR;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    if (!f->bq) {
        if (dalloc(&f->bq, (size_t)(9 * n + 8) * 8) != hipSuccess || dalloc(&f->bst, sizeof(IrState)) != hipSuccess)
            return MPIR_ERR_ALLOC;
        HIPCHK(hipMemsetAsync(f->bq, 0, (size_t)(9 * n + 8) * 8, s));
        HIPCHK(hipMemsetAsync(f->bst, 0, sizeof(IrState), s));
    }
    double *vr = f->bq, *vrs = vr + n, *vp = vr + 2 * n, *vv = vr + 3 * n, *vs = vr + 4 * n, *vt = vr + 5 * n,
           *vd = vr + 6 * n, *vtmp = vr + 7 * n, *vzero = vr + 8 * n, *sc = vr + 9 * n;
    IrState h{};
    h.it = -1;
    h.anorm = f->anorm;
    h.wilk = f->tw != MPIR_F64 ? 1 : 0;                  // TR wider than TW: eq. wilkterm
    h.residterm = term.residterm ? 1 : 0;
    h.litmax = term.litmax;
    const double uw = f->tw == MPIR_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    h.tol_r = term.tol_rel > 0 ? term.tol_rel : term.Cr * uw;
    h.tol_e = term.tol_rel > 0 ? term.tol_rel : term.Ce * uw;
    h.rmax = term.Rmax;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipMemcpyAsync(f->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(f->flags_d, 0, 4, s));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_ir_init(n, f->tw, f->tr, db, dx, f->r, f->st, s));
    HIPCHK(launch_terminate(f->st, s));
    const void *LU = factors_ptr(f);
    // w = P A v: the residual kernel with b = 0 gives -A v, then the
    // permutation (negated) and the binary64 substitutions on the TF factors
    auto op = [&](const double *in, double *out) -> hipError_t {
        hipError_t e = launch_residual_x64(n, f->A, f->lda, f->tw, vzero, in, vtmp, f->partial,
                                           f->nchunks, f->bst, s);
        if (e == hipSuccess) e = launch_gather_neg(n, vtmp, f->perm, out, f->ts, s);
        if (e == hipSuccess) e = launch_trsv(f->tf, MPIR_F64, LU, n, f->ld, out, f->yw, f->ts, f->flags_d, f->st, 1, s);
        return e;
    };
    double hv = 0.0;
    auto dot = [&](const double *a, const double *b, double *out) -> hipError_t {
        hipError_t e = launch_dots(n, a, n, 1, b, sc, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hv, sc, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        *out = hv;
        return e;
    };
    for (int it = 0; it < term.litmax; ++it) {
        int32_t done = 0;
        HIPCHK(hipMemcpyAsync(&done, &f->st->done, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (done) break;
        // right side P (r / sigma)
        HIPCHK(launch_scale_permute(n, MPIR_F64, MPIR_F64, f->r, f->perm, vr, f->st, f->ts, 1, s));
        HIPCHK(launch_trsv(f->tf, MPIR_F64, LU, n, f->ld, vr, f->yw, f->ts, f->flags_d, f->st, 1, s));
        HIPCHK(hipMemsetAsync(vd, 0, n * 8, s));
        double b2 = 0.0;
        HIPCHK(dot(vr, vr, &b2));
        const double beta0 = std::sqrt(b2);
        int kend = 0;
        if (beta0 > 0.0 && std::isfinite(beta0)) {
            HIPCHK(launch_lin3(n, vr, 0.0, vr, 0.0, nullptr, vrs, s));     // shadow = P r / sigma
            HIPCHK(hipMemsetAsync(vp, 0, n * 8, s));
            HIPCHK(hipMemsetAsync(vv, 0, n * 8, s));
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            const double tol_in = eta * beta0;
            for (int k = 1; k <= maxit; ++k) {
                double rho = 0.0;
                HIPCHK(dot(vrs, vr, &rho));
                if (rho == 0.0) { kend = k - 1; break; }
                const double beta = (rho / rho_old) * (alpha / omega);
                HIPCHK(launch_lin3(n, vr, beta, vp, -beta * omega, vv, vp, s));   // p = r + beta (p - omega v)
                HIPCHK(op(vp, vv));
                double den = 0.0;
                HIPCHK(dot(vrs, vv, &den));
                if (den == 0.0) { kend = k - 1; break; }
                alpha = rho / den;
                HIPCHK(launch_lin3(n, vr, -alpha, vv, 0.0, nullptr, vs, s));      // s = r - alpha v
                double s2 = 0.0;
                HIPCHK(dot(vs, vs, &s2));
                kend = k;
                if (std::sqrt(s2) <= tol_in) {
                    HIPCHK(launch_lin3(n, vd, alpha, vp, 0.0, nullptr, vd, s));
                    break;
                }
                HIPCHK(op(vs, vt));
                double tt = 0.0, tsd = 0.0;
                HIPCHK(dot(vt, vt, &tt));
                if (tt == 0.0) {
                    HIPCHK(launch_lin3(n, vd, alpha, vp, 0.0, nullptr, vd, s));
                    break;
                }
                HIPCHK(dot(vt, vs, &tsd));
                omega = tsd / tt;
                HIPCHK(launch_lin3(n, vd, alpha, vp, omega, vs, vd, s));         // d += alpha p + omega s
                HIPCHK(launch_lin3(n, vs, -omega, vt, 0.0, nullptr, vr, s));      // r = s - omega t
                double r2 = 0.0;
                HIPCHK(dot(vr, vr, &r2));
                if (std::sqrt(r2) <= tol_in || omega == 0.0 || !std::isfinite(r2)) break;
                rho_old = rho;
            }
        }
        if (khist && it < term.litmax) khist[it] = kend;
        // x <- x + sigma d, the binary64 residual, the termination rules
        HIPCHK(launch_update(n, f->tw, MPIR_F64, vd, dx, f->st, 0, s));
        HIPCHK(launch_residual(n, f->A, f->lda, f->tw, f->tr, db, dx, f->r, f->partial, f->nchunks,
                               f->st, 0, s));
        HIPCHK(launch_terminate(f->st, s));
    }
    HIPCHK(hipEventRecord(e1, s));
    IrState hs;
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(&hs, f->st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    if (hs.it == 0 && hs.stop == MPIR_STOP_NONFINITE) return MPIR_ERR_NONFINITE;
    if (rep) {
        rep->n_iter = hs.it;
        rep->stop = hs.stop;
        rep->n_hist = hs.it + 1;
        for (int k = 0; k <= hs.it && k < MPIR_HIST_MAX; ++k) rep->rhist[k] = hs.rhist[k];
        for (int k = 0; k < hs.it && k < MPIR_HIST_MAX; ++k) rep->dhist[k] = hs.dhist[k];
        rep->bnorm_inf = hs.bnorm;
        rep->anorm_inf = f->anorm;
        rep->xnorm_inf = hs.xnorm;
        rep->relres = hs.bnorm > 0 ? hs.rnorm / hs.bnorm : hs.rnorm;
        const double den = f->anorm * hs.xnorm + hs.bnorm;
        rep->bwd_err = den > 0 ? hs.rnorm / den : 0.0;
        rep->t_ir_ms = ms;
    }
    return MPIR_OK;
}

mpir_status mpir_ir_solve_multi(mpir_fact f, int32_t nrhs, const void *dB, int64_t ldb, void *dX,
                                int64_t ldx, const mpir_term *t, mpir_report *reps) {
    if (!f || !dB || !dX || nrhs < 1 || ldb < f->n || ldx < f->n) return MPIR_ERR_ARG;
    mpir_term term;
    if (t) term = *t;
    else mpir_term_default(&term);
    if (term.litmax < 1 || term.litmax > MPIR_HIST_MAX - 1 || !(term.Rmax > 0.0)) return MPIR_ERR_ARG;
    if ((term.onthefly != 0 && term.onthefly != 1) || term.reserved != 0) return MPIR_ERR_ARG;
    if (reps) {
        for (int c = 0; c < nrhs; ++c) {
            std::memset(&reps[c], 0, sizeof(reps[c]));
            reps[c].info = f->info;
            reps[c].t_factor_ms = f->t_factor_ms;
        }
    }
    if (!f->valid) return MPIR_ERR_STATE;
    if (f->info) return MPIR_ERR_SINGULAR;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    const size_t es = esize(f->tw), rs = esize(f->tr);
    if (f->mcap < nrhs) {
        HIPCHK(hipStreamSynchronize(s));
        hipFree(f->mst);
        hipFree(f->mr);
        hipFree(f->mrhat);
        hipFree(f->mpart);
        hipFree(f->myw);
        f->mst = nullptr; f->mr = nullptr; f->mrhat = nullptr; f->mpart = nullptr; f->myw = nullptr;
        f->mcap = 0;
        if (dalloc(&f->mst, (size_t)nrhs * sizeof(IrState)) != hipSuccess ||
            dalloc(&f->mr, (size_t)nrhs * n * 8) != hipSuccess ||
            dalloc(&f->mrhat, (size_t)nrhs * n * 8) != hipSuccess ||
            dalloc(&f->mpart, (size_t)4 * f->nchunks * n * 8) != hipSuccess ||
            dalloc(&f->myw, (size_t)nrhs * n * 2 * 8) != hipSuccess)
            return MPIR_ERR_ALLOC;
        HIPCHK(hipMemsetAsync(f->mrhat, 0, (size_t)nrhs * n * 8, s));
        HIPCHK(hipMemsetAsync(f->myw, 0, (size_t)nrhs * n * 2 * 8, s));
        f->mcap = nrhs;
    }
    const double uw = f->tw == MPIR_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    IrState h{};
    h.it = -1;
    h.anorm = f->anorm;
    h.wilk = (f->tr == MPIR_F64 && f->tw != MPIR_F64) ? 1 : 0;
    h.residterm = term.residterm ? 1 : 0;
    h.litmax = term.litmax;
    h.tol_r = term.tol_rel > 0 ? term.tol_rel : term.Cr * uw;
    h.tol_e = term.tol_rel > 0 ? term.tol_rel : term.Ce * uw;
    h.rmax = term.Rmax;
    std::vector<IrState> hv((size_t)nrhs, h);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipMemcpyAsync(f->mst, hv.data(), (size_t)nrhs * sizeof(IrState), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(f->flags_d, 0, 4, s));
    HIPCHK(hipEventRecord(e0, s));
    const char *B = (const char *)dB;
    char *X = (char *)dX;
    char *R = (char *)f->mr, *RH = (char *)f->mrhat;
    IrState *S = f->mst;
    for (int c = 0; c < nrhs; ++c) {
        HIPCHK(launch_ir_init(n, f->tw, f->tr, B + c * ldb * es, X + c * ldx * es, R + c * n * rs, S + c, s));
        HIPCHK(launch_terminate(S + c, s));
    }
    const void *LU = factors_ptr(f);
    // the precisions of mpir_ir_solve: LPS (rhat in TF, binary32 solves;
    // binary64 for TF = F64) or the on-the-fly solve in TW
    const bool mps = term.onthefly && f->tf != f->tw;
    const int rprec = mps ? f->tw : f->tf;
    const int yprec = mps ? f->tw : (f->tf == MPIR_F64 ? MPIR_F64 : MPIR_F32);
    const size_t ys = yprec == MPIR_F64 ? 8 : 4;
    const int tnr = trsv_max_rhs(yprec);
    std::vector<int32_t> done((size_t)nrhs, 0);
    auto any_active = [&](int c0, int c1) {
        for (int c = c0; c < c1; ++c)
            if (!done[c]) return true;
        return false;
    };
    for (int it = 0; it < term.litmax; ++it) {
        HIPCHK(hipMemcpy2DAsync(done.data(), 4, &S->done, sizeof(IrState), 4, (size_t)nrhs,
                                hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!any_active(0, nrhs)) break;
        for (int c0 = 0, c1 = 0; c0 < nrhs; c0 = c1) {
            // chunks of 4, 2 or 1 columns (the solve's instantiations)
            int nr = nrhs - c0 < tnr ? nrhs - c0 : tnr;
            if (nr == 3) nr = 2;
            c1 = c0 + nr;
            if (!any_active(c0, c1)) continue;
            for (int c = c0; c < c1; ++c)
                HIPCHK(launch_scale_permute(n, f->tr, rprec, R + c * n * rs, f->perm, RH + c * n * ys, S + c,
                                            f->ts, 0, s));
            HIPCHK(launch_trsv_multi(f->tf, yprec, c1 - c0, LU, n, f->ld, RH + c0 * n * ys, n,
                                     f->myw, f->ts, f->flags_d, S + c0, 1, s));
            for (int c = c0; c < c1; ++c)
                HIPCHK(launch_update(n, f->tw, rprec, RH + c * n * ys, X + c * ldx * es, S + c, 0, s));
        }
        for (int c0 = 0; c0 < nrhs; c0 += 4) {
            const int c1 = c0 + 4 < nrhs ? c0 + 4 : nrhs;
            if (!any_active(c0, c1)) continue;
            HIPCHK(launch_residual_multi(n, f->A, f->lda, f->tw, f->tr, c1 - c0, B + c0 * ldb * es, ldb,
                                         X + c0 * ldx * es, ldx, R + c0 * n * rs, f->mpart, f->nchunks,
                                         S + c0, 0, s));
        }
        for (int c = 0; c < nrhs; ++c)
            if (!done[c]) HIPCHK(launch_terminate(S + c, s));
    }
    HIPCHK(hipEventRecord(e1, s));
    uint32_t flags = 0;
    HIPCHK(hipMemcpyAsync(hv.data(), S, (size_t)nrhs * sizeof(IrState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flags, f->flags_d, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (flags & DF_TIMEOUT) return MPIR_ERR_DEVICE;
    bool nonfinite_input = false;
    for (int c = 0; c < nrhs; ++c) {
        const IrState &hs = hv[c];
        if (hs.it == 0 && hs.stop == MPIR_STOP_NONFINITE) nonfinite_input = true;
        double rnorm = hs.rnorm, xnorm = hs.xnorm;
        if (f->tr != MPIR_F64 && hs.it > 0) {
            // report the binary64 residual of the returned x
            IrState h2{};
            h2.it = 0;
            HIPCHK(hipMemcpyAsync(f->st, &h2, sizeof(h2), hipMemcpyHostToDevice, s));
            HIPCHK(launch_residual(n, f->A, f->lda, f->tw, MPIR_F64, B + c * ldb * es, X + c * ldx * es, f->r,
                                   f->partial, f->nchunks, f->st, 1, s));
            uint64_t bits[3];
            HIPCHK(hipMemcpyAsync(bits, &f->st->rnorm_bits, 24, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            std::memcpy(&rnorm, &bits[0], 8);
            std::memcpy(&xnorm, &bits[2], 8);
        }
        if (reps) {
            mpir_report *rep = &reps[c];
            rep->n_iter = hs.it;
            rep->stop = hs.stop;
            rep->n_hist = hs.it + 1;
            for (int k = 0; k <= hs.it && k < MPIR_HIST_MAX; ++k) rep->rhist[k] = hs.rhist[k];
            for (int k = 0; k < hs.it && k < MPIR_HIST_MAX; ++k) rep->dhist[k] = hs.dhist[k];
            rep->bnorm_inf = hs.bnorm;
            rep->anorm_inf = f->anorm;
            rep->xnorm_inf = xnorm;
            rep->relres = hs.bnorm > 0 ? rnorm / hs.bnorm : rnorm;
            const double den = f->anorm * xnorm + hs.bnorm;
            rep->bwd_err = den > 0 ? rnorm / den : 0.0;
            rep->t_ir_ms = ms;
        }
    }
    return nonfinite_input ? MPIR_ERR_NONFINITE : MPIR_OK;
}

mpir_status mpir_downcast(int64_t n, const void *dA, int64_t lda, mpir_prec tw, mpir_prec tf,
                          void *dAF, double *anorm, void *hip_stream) {
    if (n <= 0 || !dA || !dAF || lda < n || !valid_triple(tw, tf, tw == MPIR_F64 ? MPIR_F64 : MPIR_F32))
        return MPIR_ERR_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    uint64_t *bits = nullptr;
    uint32_t *flags = nullptr;
    void *tmp = nullptr;
    mpir_status st = MPIR_OK;
    if (dalloc(&bits, 16) != hipSuccess || dalloc(&flags, 8) != hipSuccess) st = MPIR_ERR_ALLOC;
    if (st == MPIR_OK && is16(tf) && dalloc(&tmp, (size_t)n * n * 4) != hipSuccess) st = MPIR_ERR_ALLOC;
    if (st == MPIR_OK) {
        hipMemsetAsync(bits, 0, 8, s);
        hipMemsetAsync(flags, 0, 4, s);
        if (launch_downcast(n, dA, lda, tw, tf, is16(tf) ? tmp : dAF, n, bits, flags, s) != hipSuccess)
            st = MPIR_ERR_HIP;
        if (st == MPIR_OK && is16(tf) &&
            launch_pack_half(tf, n, (const float *)tmp, n, dAF, n, s) != hipSuccess)
            st = MPIR_ERR_HIP;
        uint64_t hb = 0;
        uint32_t hf = 0;
        if (st == MPIR_OK && (hipMemcpyAsync(&hb, bits, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                              hipMemcpyAsync(&hf, flags, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                              hipStreamSynchronize(s) != hipSuccess))
            st = MPIR_ERR_HIP;
        if (st == MPIR_OK) {
            if (anorm) std::memcpy(anorm, &hb, 8);
            if (hf & DF_NONFINITE) st = MPIR_ERR_NONFINITE;
            else if (hf & DF_RANGE) st = MPIR_ERR_RANGE;
        }
    }
    hipFree(bits);
    hipFree(flags);
    hipFree(tmp);
    return st;
}

mpir_status mpir_get_factors(mpir_fact f, void *dLU, int32_t *ipiv) {
    if (!f || (!dLU && !ipiv)) return MPIR_ERR_ARG;
    if (!f->valid) return MPIR_ERR_STATE;
    hipStream_t s = f->stream;
    const int64_t n = f->n;
    if (dLU) {
        const size_t es = esize(f->tf);
        const void *src = is16(f->tf) ? (const void *)f->lu16 : f->work;
        HIPCHK(hipMemcpy2DAsync(dLU, n * es, src, f->ld * es, n * es, n, hipMemcpyDeviceToDevice, s));
    }
    if (ipiv) HIPCHK(hipMemcpyAsync(ipiv, f->ipiv, n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MPIR_OK;
}

mpir_status mpir_residual(int64_t n, const void *dA, int64_t lda, mpir_prec tw, mpir_prec tr,
                          const void *db, const void *dx, void *dr, double *rnorm, void *hip_stream) {
    if (n <= 0 || !dA || !db || !dx || !dr || lda < n || !valid_triple(tw, tw, tr)) return MPIR_ERR_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    IrState *st = nullptr;
    double *partial = nullptr;
    const int nch = residual_chunks(n);
    mpir_status ret = MPIR_OK;
    if (dalloc(&st, sizeof(IrState)) != hipSuccess || dalloc(&partial, (size_t)nch * n * 8) != hipSuccess)
        ret = MPIR_ERR_ALLOC;
    if (ret == MPIR_OK) {
        IrState h{};
        uint64_t bits = 0;
        if (hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) ret = MPIR_ERR_HIP;
        {
            ProfScope ps_(3, (double)n * n * esize(tw), s);
            if (ret == MPIR_OK && launch_residual(n, dA, lda, tw, tr, db, dx, dr, partial, nch, st, 1, s) != hipSuccess)
                ret = MPIR_ERR_HIP;
        }
        if (ret == MPIR_OK && (hipMemcpyAsync(&bits, &st->rnorm_bits, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                               hipStreamSynchronize(s) != hipSuccess))
            ret = MPIR_ERR_HIP;
        if (ret == MPIR_OK && rnorm) std::memcpy(rnorm, &bits, 8);
    }
    hipFree(st);
    hipFree(partial);
    return ret;
}

}  // extern "C"

// --------------------------------------------------------------------------
// Batched refinement (a persistent launch over a queue of systems)
// --------------------------------------------------------------------------
struct mpir_batch_s {
    int32_t batch = 0;
    int tw = 0, tf = 0, tr = 0;
    hipStream_t stream = nullptr;
    BatchSys *sys_d = nullptr;
    int32_t *order_d = nullptr;
    uint32_t *queue_d = nullptr;
    float *work = nullptr;
    int32_t *perm = nullptr;
    mpir_report *reps_d = nullptr;
    std::vector<mpir_report> reps_h;   // host copy when the caller passes no reports
    BatchTerm term{};
    int nwg = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

__global__ void k_zero_u32(uint32_t *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

void free_batch(mpir_batch b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    hipFree(b->sys_d);
    hipFree(b->order_d);
    hipFree(b->queue_d);
    hipFree(b->work);
    hipFree(b->perm);
    hipFree(b->reps_d);
    delete b;
}

// Enqueue one solve of the whole batch: reset the queue with a kernel (no
// memset node, so the sequence can be captured), then the persistent launch.
hipError_t enqueue_batch(mpir_batch b, hipStream_t s) {
    k_zero_u32<<<1, 64, 0, s>>>(b->queue_d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_batched(b->tw, b->tf, b->sys_d, b->order_d, b->batch, b->queue_d, b->term,
                          b->reps_d, b->nwg, s);
}

int device_cus() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    return prop.multiProcessorCount;
}

}  // namespace

mpir_status batch_create_with(int32_t batch, const int64_t *n, const void *const *dA,
                              const int64_t *lda, const void *const *db, void *const *dx,
                              mpir_prec tw, mpir_prec tf, mpir_prec tr, const mpir_term *t,
                              int32_t use_graph, void *hip_stream, const mpir_batch_tuning *tab,
                              mpir_batch *out) {
    if (out) *out = nullptr;
    if (!out || batch <= 0 || !n || !dA || !lda || !db || !dx) return MPIR_ERR_ARG;
    if (!(tw == MPIR_F64 || tw == MPIR_F32) || !(tf == MPIR_F32 || tf == MPIR_F16 || tf == MPIR_BF16) ||
        tr != MPIR_F64)
        return MPIR_ERR_ARG;
    if (tw == MPIR_F32 && tf == MPIR_F32) {
        // TF = TW = F32 with TR = F64 (eq. wilkterm) is allowed
    }
    mpir_term term;
    if (t) term = *t;
    else mpir_term_default(&term);
    if (term.litmax < 1 || term.litmax > MPIR_HIST_MAX - 1 || !(term.Rmax > 0.0)) return MPIR_ERR_ARG;
    if (term.onthefly != 0 || term.reserved != 0) return MPIR_ERR_ARG;   // batched: LPS only
    int64_t total = 0, totn = 0;
    for (int32_t k = 0; k < batch; ++k) {
        if (n[k] <= 0 || n[k] > batched_max_n() || lda[k] < n[k] || !dA[k] || !db[k] || !dx[k])
            return MPIR_ERR_ARG;
        total += n[k] * n[k];
        totn += n[k];
    }
    mpir_batch b = new (std::nothrow) mpir_batch_s();
    if (!b) return MPIR_ERR_ALLOC;
    b->batch = batch;
    b->tw = tw;
    b->tf = tf;
    b->tr = tr;
    b->stream = (hipStream_t)hip_stream;
    const double uw = tw == MPIR_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    b->term.tol_r = term.tol_rel > 0 ? term.tol_rel : term.Cr * uw;
    b->term.tol_e = term.tol_rel > 0 ? term.tol_rel : term.Ce * uw;
    b->term.rmax = term.Rmax;
    b->term.litmax = term.litmax;
    b->term.residterm = term.residterm ? 1 : 0;
    b->term.wilk = tw != MPIR_F64 ? 1 : 0;
    if (dalloc(&b->sys_d, sizeof(BatchSys) * batch) != hipSuccess ||
        dalloc(&b->order_d, sizeof(int32_t) * batch) != hipSuccess ||
        dalloc(&b->queue_d, 16) != hipSuccess || dalloc(&b->work, sizeof(float) * total) != hipSuccess ||
        dalloc(&b->perm, sizeof(int32_t) * totn) != hipSuccess ||
        dalloc(&b->reps_d, sizeof(mpir_report) * batch) != hipSuccess) {
        free_batch(b);
        return MPIR_ERR_ALLOC;
    }
    b->reps_h.resize(batch);
    std::vector<BatchSys> sys(batch);
    int64_t wo = 0, po = 0;
    for (int32_t k = 0; k < batch; ++k) {
        sys[k] = BatchSys{n[k], lda[k], dA[k], db[k], dx[k], b->work + wo, b->perm + po,
                          batch_cfg(tw, tf, n[k], tab)};
        wo += n[k] * n[k];
        po += n[k];
    }
    // longest first (work ~ n^3): the largest systems start in the first wave
    std::vector<int32_t> order(batch);
    for (int32_t k = 0; k < batch; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return n[x] > n[y]; });
    if (hipMemcpy(b->sys_d, sys.data(), sizeof(BatchSys) * batch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->order_d, order.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) != hipSuccess) {
        free_batch(b);
        return MPIR_ERR_HIP;
    }
    const int cus = device_cus();
    b->nwg = cus > 0 ? (cus < batch ? cus : batch) : 1;
    if (use_graph) {
        // capture on a private stream (the caller's may be the legacy default
        // stream, which cannot be captured); replays go to the caller's stream
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            free_batch(b);
            return MPIR_ERR_HIP;
        }
        hipError_t e0 = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        const hipError_t e1 = e0 == hipSuccess ? enqueue_batch(b, cs) : e0;
        const hipError_t e2 = e0 == hipSuccess ? hipStreamEndCapture(cs, &b->graph) : e0;
        hipStreamDestroy(cs);
        if (e1 != hipSuccess || e2 != hipSuccess ||
            hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            free_batch(b);
            return MPIR_ERR_HIP;
        }
    }
    *out = b;
    return MPIR_OK;
}

extern "C" {

mpir_status mpir_batch_create(int32_t batch, const int64_t *n, const void *const *dA,
                              const int64_t *lda, const void *const *db, void *const *dx,
                              mpir_prec tw, mpir_prec tf, mpir_prec tr, const mpir_term *t,
                              int32_t use_graph, void *hip_stream, mpir_batch *out) {
    return batch_create_with(batch, n, dA, lda, db, dx, tw, tf, tr, t, use_graph, hip_stream, nullptr, out);
}

mpir_status mpir_batch_run(mpir_batch b, mpir_report *reps) {
    if (!b) return MPIR_ERR_ARG;
    if (b->exec) HIPCHK(hipGraphLaunch(b->exec, b->stream));
    else HIPCHK(enqueue_batch(b, b->stream));
    // the per-system statuses are read whether or not the caller wants the
    // reports: a failed system leaves its x unwritten, which must not pass
    // as MPIR_OK
    mpir_report *h = reps ? reps : b->reps_h.data();
    HIPCHK(hipMemcpyAsync(h, b->reps_d, sizeof(mpir_report) * b->batch, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int32_t k = 0; k < b->batch; ++k)
        if (h[k].reserved != MPIR_OK) return (mpir_status)h[k].reserved;
    return MPIR_OK;
}

void mpir_batch_destroy(mpir_batch b) {
    if (!b) return;
    hipStreamSynchronize(b->stream);
    free_batch(b);
}

mpir_status mpir_ir_solve_batched(int32_t batch, const int64_t *n, const void *const *dA,
                                  const int64_t *lda, const void *const *db, void *const *dx,
                                  mpir_prec tw, mpir_prec tf, mpir_prec tr, const mpir_term *t,
                                  mpir_report *reps, void *hip_stream) {
    mpir_batch b = nullptr;
    mpir_status st = mpir_batch_create(batch, n, dA, lda, db, dx, tw, tf, tr, t, 0, hip_stream, &b);
    if (st != MPIR_OK) return st;
    st = mpir_batch_run(b, reps);
    mpir_batch_destroy(b);
    return st;
}

void mpir_prof_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.on = on != 0;
}

void mpir_prof_reset(void) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (auto &v : g_prof.recs)
        for (auto &r : v) {
            g_prof.pool.push_back(r.a);
            g_prof.pool.push_back(r.b);
        }
    for (auto &v : g_prof.recs) v.clear();
}

mpir_status mpir_batch_phase_times(double *ms, int32_t reset) {
    static_assert(MPIR_BATCH_PHASES == mpir::kBatchPhases, "phase count of the batched kernel");
    if (!ms && !reset) return MPIR_ERR_ARG;
    int dev = 0, khz = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return MPIR_ERR_HIP;
    HIPCHK(hipDeviceSynchronize());
    unsigned long long t[mpir::kBatchPhases];
    HIPCHK(mpir::batched_phase_ticks(t, reset != 0));
    if (ms)
        for (int k = 0; k < mpir::kBatchPhases; ++k) ms[k] = (double)t[k] / (double)khz;
    return MPIR_OK;
}

mpir_status mpir_prof_get(int32_t kind, double *ms, int64_t *launches, double *work) {
    if (kind < 0 || kind >= 6) return MPIR_ERR_ARG;
    std::lock_guard<std::mutex> g(g_prof.mu);
    double tot = 0.0, wk = 0.0;
    for (auto &r : g_prof.recs[kind]) {
        if (hipEventSynchronize(r.b) != hipSuccess) return MPIR_ERR_HIP;
        float e = 0.f;
        if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return MPIR_ERR_HIP;
        tot += e;
        wk += r.work;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int64_t)g_prof.recs[kind].size();
    if (work) *work = wk;
    return MPIR_OK;
}

}  // extern "C"
