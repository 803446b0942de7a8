// Blocked right-looking LU with partial pivoting (the "Factor A = LU in
// precision TF" step of Algorithm IR; Julia lu! / LAPACK getrf semantics):
// the panel ("leaf") factorization with a wavefront argmax pivot search, the
// row interchanges, and the small unit-lower triangular solve that forms U12.
// The trailing-matrix update is in k_gemm.hip.
//
// Working array: row-major, leading dimension ld, binary32 (TF = F32, F16)
// or binary64 (TF = F64).  Row interchanges of a row-major matrix move
// contiguous memory, which is why this layout was chosen.
#include <climits>

#include "mpir_internal.h"

namespace mpir {

constexpr int kLeafMaxW = 32;     // columns per leaf
constexpr int kLeafT = 1024;      // threads per leaf workgroup = rows it owns
constexpr int kLeafMaxG = 64;     // workgroups per leaf (one wave reads all slots)

// Exchange area of the cooperative leaf.  Every value travels in 64-bit
// words (32-bit payload | 32-bit epoch), so a reader that sees the current
// epoch in a word also sees its payload: no separate barrier, no fences.
// Per column parity and workgroup: a header (|value| in 1-2 words, row
// index) and the candidate row (1-2 words per column); plus the old
// diagonal row posted by its owner.
constexpr int kHeadWords = 4;
constexpr int kRowWords = 2 * kLeafMaxW;
struct LeafSlot {
    uint64_t head[kHeadWords];
    uint64_t row[kRowWords];
};
struct PanelSync {
    LeafSlot slot[2][kLeafMaxG];
    uint64_t diag[2][kRowWords];
};

size_t panel_sync_bytes() { return sizeof(PanelSync); }

hipError_t panel_sync_reset(PanelSync *ps, hipStream_t s) {
    return hipMemsetAsync(ps, 0, sizeof(PanelSync), s);
}

namespace {

__device__ __forceinline__ void put_word(uint64_t *p, uint32_t payload, uint32_t epoch) {
    __hip_atomic_store(p, ((uint64_t)epoch << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get_word(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool word_ok(uint64_t w, uint32_t epoch) { return (uint32_t)(w >> 32) == epoch; }

// Values of type W split into 32-bit payloads (1 for float, 2 for double).
template <typename W> struct Words;
template <> struct Words<float> {
    static constexpr int K = 1;
    __device__ static uint32_t part(float v, int) { return __float_as_uint(v); }
    __device__ static float join(const uint32_t *p) { return __uint_as_float(p[0]); }
};
template <> struct Words<double> {
    static constexpr int K = 2;
    __device__ static uint32_t part(double v, int q) {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        return q == 0 ? (uint32_t)b : (uint32_t)(b >> 32);
    }
    __device__ static double join(const uint32_t *p) {
        return __longlong_as_double((long long)(((uint64_t)p[1] << 32) | p[0]));
    }
};

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// Leaf factorization of rows [k0, n) x columns [k0, k0+w) of the working
// array.  Workgroup g owns relative rows [g*1024, g*1024+1024), one row per
// thread, the w leaf entries of the row in registers.  For every column:
// local argmax (first maximum), candidate posted as epoch-tagged words,
// winner chosen identically by every workgroup, swap, scale, rank-1 update.
// F16: the pivot row is rounded to binary16 when it becomes the pivot row,
// each multiplier to binary16 when formed (products of binary16 numbers are
// exact in binary32).
template <typename W, bool F16>
__global__ __launch_bounds__(kLeafT) void k_leaf(W *__restrict__ a, int64_t n, int64_t ld,
                                                 int64_t k0, int w, int G,
                                                 int32_t *__restrict__ ipiv, int64_t *info,
                                                 PanelSync *ps, uint32_t base, uint32_t *flags) {
    using Wd = Words<W>;
    constexpr int K = Wd::K;
    __shared__ double red_v[kLeafT / 64];
    __shared__ int red_i[kLeafT / 64];
    __shared__ W crow[kLeafMaxW];      // this workgroup's candidate row
    __shared__ W jrow[kLeafMaxW];      // row j (if owned here)
    __shared__ W prow[kLeafMaxW];      // pivot row
    __shared__ W orow[kLeafMaxW];      // old row j
    __shared__ double s_bv;
    __shared__ int s_bi, s_p, s_bad;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t m = n - k0;
    const int64_t r0 = (int64_t)blockIdx.x * kLeafT;
    const int rows = (int)((m - r0) < kLeafT ? (m - r0) : kLeafT);
    // an earlier launch already timed out: every workgroup returns at once
    if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & DF_TIMEOUT) return;
    if (tid == 0) s_bad = 0;
    if (tid < kLeafMaxW) { prow[tid] = (W)0; orow[tid] = (W)0; crow[tid] = (W)0; jrow[tid] = (W)0; }
    __syncthreads();
    const bool mine = tid < rows;
    const int64_t rr = r0 + tid;               // relative row of this thread
    W v[kLeafMaxW];
#pragma unroll
    for (int c = 0; c < kLeafMaxW; ++c) v[c] = (W)0;
    if (mine) {
        const W *src = a + (k0 + rr) * ld + k0;
#pragma unroll
        for (int c = 0; c < kLeafMaxW; ++c)
            if (c < w) v[c] = src[c];
    }

#pragma unroll
    for (int j = 0; j < kLeafMaxW; ++j) {
        if (j >= w) break;
        const uint32_t epoch = base + (uint32_t)j + 1u;
        const int par = j & 1;
        // ---- local argmax of |a_rj| over owned rows r >= j ----
        double bv = (mine && rr >= j) ? fabs((double)v[j]) : -1.0;
        int bi = (mine && rr >= j) ? (int)rr : INT_MAX;
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
        __syncthreads();
        if (wv == 0) {
            bv = lane < kLeafT / 64 ? red_v[lane] : -1.0;
            bi = lane < kLeafT / 64 ? red_i[lane] : INT_MAX;
            for (int off = 8; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { s_bv = bv; s_bi = bi; }
        }
        __syncthreads();
        if (mine && rr == s_bi) {
#pragma unroll
            for (int c = 0; c < kLeafMaxW; ++c) crow[c] = v[c];
        }
        if (mine && rr == j) {
#pragma unroll
            for (int c = 0; c < kLeafMaxW; ++c) jrow[c] = v[c];
        }
        __syncthreads();

        if (G == 1) {
            if (tid < kLeafMaxW) { prow[tid] = crow[tid]; orow[tid] = jrow[tid]; }
            if (tid == 0) s_p = s_bi;
        } else if (wv == 0) {
            // ---- post this workgroup's candidate and (if owned) row j ----
            LeafSlot *my = &ps->slot[par][blockIdx.x];
            const bool own_j = j >= r0 && j < r0 + rows;
            if (lane < w) {
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    put_word(&my->row[lane * K + q], Wd::part(crow[lane], q), epoch);
                    if (own_j) put_word(&ps->diag[par][lane * K + q], Wd::part(jrow[lane], q), epoch);
                }
            }
            if (lane == 32) {
                const uint64_t b = (uint64_t)__double_as_longlong(s_bv);
                put_word(&my->head[0], (uint32_t)b, epoch);
                put_word(&my->head[1], (uint32_t)(b >> 32), epoch);
                put_word(&my->head[2], (uint32_t)s_bi, epoch);
            }
            // ---- read every workgroup's header (lane g <-> workgroup g) ----
            double gv = -1.0;
            int gi = INT_MAX, gw = 0;
            {
                uint64_t h0 = 0, h1 = 0, h2 = 0;
                bool ok = lane >= G;
                uint64_t spins = 0;
                for (;;) {
                    if (!ok) {
                        const LeafSlot *sl = &ps->slot[par][lane];
                        h0 = get_word(&sl->head[0]);
                        h1 = get_word(&sl->head[1]);
                        h2 = get_word(&sl->head[2]);
                        ok = word_ok(h0, epoch) && word_ok(h1, epoch) && word_ok(h2, epoch);
                    }
                    if (__all(ok)) break;
                    if (++spins > kSpinLimit) { if (lane == 0) s_bad = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (lane < G && ok) {
                    gv = __longlong_as_double((long long)((h1 << 32) | (uint32_t)h0));
                    gi = (int)(uint32_t)h2;
                    gw = lane;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(gv, off);
                const int oi = __shfl_xor(gi, off);
                const int og = __shfl_xor(gw, off);
                if (better(ov, oi, gv, gi)) { gv = ov; gi = oi; gw = og; }
            }
            // ---- winner's row and the old row j ----
            {
                uint32_t pw[K], ow[K];
                bool ok = lane >= w;
                uint64_t spins = 0;
                for (;;) {
                    if (!ok) {
                        ok = true;
#pragma unroll
                        for (int q = 0; q < K; ++q) {
                            const uint64_t x = get_word(&ps->slot[par][gw].row[lane * K + q]);
                            const uint64_t y = get_word(&ps->diag[par][lane * K + q]);
                            ok = ok && word_ok(x, epoch) && word_ok(y, epoch);
                            pw[q] = (uint32_t)x;
                            ow[q] = (uint32_t)y;
                        }
                    }
                    if (__all(ok)) break;
                    if (++spins > kSpinLimit) { if (lane == 0) s_bad = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (lane < w) { prow[lane] = Wd::join(pw); orow[lane] = Wd::join(ow); }
            }
            if (lane == 0) s_p = gi;
        }
        __syncthreads();
        const int p = s_p;
        if (s_bad || p == INT_MAX) {
            if (tid == 0) atomicOr(flags, (uint32_t)DF_TIMEOUT);
            break;
        }
        if (F16 && tid < kLeafMaxW && tid >= j) prow[tid] = (W)round_f16((float)prow[tid]);
        __syncthreads();
        // ---- swap rows j and p, record the pivot ----
        if (mine && p != j && rr == p) {
#pragma unroll
            for (int c = 0; c < kLeafMaxW; ++c) v[c] = orow[c];
        }
        if (mine && rr == j) {
#pragma unroll
            for (int c = 0; c < kLeafMaxW; ++c) v[c] = prow[c];
        }
        if (blockIdx.x == 0 && tid == 0) {
            ipiv[k0 + j] = (int32_t)(k0 + p);
            if (prow[j] == (W)0 && *info == 0) *info = k0 + j + 1;
        }
        // ---- scale and rank-1 update of the rows below the pivot ----
        const W piv = prow[j];
        if (mine && rr > j && piv != (W)0) {
            W l = v[j] / piv;
            if (F16) l = (W)round_f16((float)l);
            v[j] = l;
#pragma unroll
            for (int c = j + 1; c < kLeafMaxW; ++c) {
                const W prod = l * prow[c];
                v[c] = v[c] - prod;
            }
        }
        // prow/orow/crow are rewritten only after the next column's first
        // __syncthreads, which every thread reaches after this point.
    }
    if (mine) {
        W *dst = a + (k0 + rr) * ld + k0;
#pragma unroll
        for (int c = 0; c < kLeafMaxW; ++c)
            if (c < w) dst[c] = v[c];
    }
}

// Row interchanges ipiv[k0 .. k0+cnt) applied, in order, to the columns
// [c0,c1) U [c2,c3).  The composed permutation only moves the rows
// P = [k0, k0+cnt) U {ipiv targets}; the source of each destination row is
// found by applying the transpositions in reverse order, so every thread
// computes its own pair without a sequential pass.  The tile of moved rows
// is staged in LDS (all reads before any write).  The last workgroup also
// permutes `perm` (the row permutation used by the solves).
template <typename W, int CB>
__global__ __launch_bounds__(256) void k_laswp(W *__restrict__ a, int64_t ld, int64_t k0, int cnt,
                                               const int32_t *__restrict__ ipiv, int64_t c0,
                                               int64_t c1, int64_t c2, int64_t c3,
                                               int32_t *__restrict__ perm, int ncolblk) {
    __shared__ W tile[512 * CB];                        // [2*cnt][CB]
    __shared__ int32_t sp[256];
    __shared__ int32_t pdst[512], psrc[512];
    __shared__ int s_extra;
    const int tid = threadIdx.x;
    if (tid == 0) s_extra = 0;
    if (tid < cnt) sp[tid] = ipiv[k0 + tid];
    __syncthreads();
    auto src_of = [&](int64_t i) -> int64_t {
        for (int s = cnt - 1; s >= 0; --s) {
            const int64_t ks = k0 + s, ps = sp[s];
            if (i == ks) i = ps;
            else if (i == ps) i = ks;
        }
        return i;
    };
    if (tid < cnt) {
        pdst[tid] = (int32_t)(k0 + tid);
        psrc[tid] = (int32_t)src_of(k0 + tid);
        const int32_t p = sp[tid];
        if (p >= k0 + cnt) {
            bool first = true;
            for (int q = 0; q < tid; ++q) if (sp[q] == p) { first = false; break; }
            if (first) {
                const int slot = cnt + atomicAdd(&s_extra, 1);
                pdst[slot] = p;
                psrc[slot] = (int32_t)src_of(p);
            }
        }
    }
    __syncthreads();
    const int np = cnt + s_extra;
    if ((int)blockIdx.x == ncolblk) {   // the permutation vector
        __shared__ int32_t pv[512];
        if (perm) {
            for (int q = tid; q < np; q += 256) pv[q] = perm[psrc[q]];
            __syncthreads();
            for (int q = tid; q < np; q += 256) perm[pdst[q]] = pv[q];
        }
        return;
    }
    const int64_t w1 = c1 - c0, wtot = w1 + (c3 - c2);
    const int64_t v0 = (int64_t)blockIdx.x * CB;
    for (int e = tid; e < np * CB; e += 256) {
        const int q = e / CB, c = e - q * CB;
        const int64_t v = v0 + c;
        if (v < wtot) {
            const int64_t col = v < w1 ? c0 + v : c2 + (v - w1);
            tile[q * CB + c] = a[(int64_t)psrc[q] * ld + col];
        }
    }
    __syncthreads();
    for (int e = tid; e < np * CB; e += 256) {
        const int q = e / CB, c = e - q * CB;
        const int64_t v = v0 + c;
        if (v < wtot) {
            const int64_t col = v < w1 ? c0 + v : c2 + (v - w1);
            a[(int64_t)pdst[q] * ld + col] = tile[q * CB + c];
        }
    }
}

// U12 <- L11^{-1} U12 for rows [k, k+w), w <= 64, columns [c0, c1):
// right-looking substitution, row t final at step t (F16: rounded to
// binary16 then), rows below updated in parallel.
template <typename W, bool F16>
__global__ __launch_bounds__(256) void k_trsm(W *__restrict__ a, int64_t ld, int64_t k, int w,
                                              int64_t c0, int64_t c1) {
    __shared__ W L[64][65];
    __shared__ W X[64][65];
    const int tid = threadIdx.x;
    const int64_t cb = c0 + (int64_t)blockIdx.x * 64;
    const int ncol = (int)((c1 - cb) < 64 ? (c1 - cb) : 64);
    for (int e = tid; e < w * w; e += 256) {
        const int r = e / w, c = e - r * w;
        L[r][c] = a[(k + r) * ld + k + c];
    }
    for (int e = tid; e < w * 64; e += 256) {
        const int r = e / 64, c = e - r * 64;
        if (c < ncol) X[r][c] = a[(k + r) * ld + cb + c];
    }
    __syncthreads();
    const int c = tid & 63, g = tid >> 6;
    for (int t = 0; t < w; ++t) {
        if (F16 && tid < 64) X[t][tid] = (W)round_f16((float)X[t][tid]);
        __syncthreads();
        const W xt = X[t][c];
        for (int r = t + 1 + g; r < w; r += 4) {
            const W prod = L[r][t] * xt;
            X[r][c] = X[r][c] - prod;
        }
        __syncthreads();
    }
    for (int e = tid; e < w * 64; e += 256) {
        const int r = e / 64, cc = e - r * 64;
        if (cc < ncol) a[(k + r) * ld + cb + cc] = X[r][cc];
    }
}

int g_num_cus = 0;

int num_cus() {
    if (g_num_cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            g_num_cus = prop.multiProcessorCount;
        if (g_num_cus <= 0) g_num_cus = 64;
    }
    return g_num_cus;
}

template <typename W, bool F16>
hipError_t leaf_go(W *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv, int64_t *info,
                   PanelSync *ps, uint32_t *host_base, uint32_t *flags, hipStream_t s) {
    const int64_t m = n - k0;
    const int64_t G64 = (m + kLeafT - 1) / kLeafT;
    if (G64 > kLeafMaxG) return hipErrorInvalidValue;
    const int G = (int)G64;
    uint32_t base = *host_base;
    if (G == 1) {
        k_leaf<W, F16><<<1, kLeafT, 0, s>>>(a, n, ld, k0, w, G, ipiv, info, ps, base, flags);
        return hipGetLastError();
    }
    void *args[] = {&a, (void *)&n, (void *)&ld, (void *)&k0, (void *)&w, (void *)&G,
                    &ipiv, &info, &ps, &base, &flags};
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_leaf<W, F16>, dim3(G), dim3(kLeafT),
                                              args, 0, s);
    if (e == hipSuccess) *host_base = base + (uint32_t)w;
    return e;
}

}  // namespace

int leaf_max_rows(int mode) {
    (void)mode;
    const int gmax = num_cus() < kLeafMaxG ? num_cus() : kLeafMaxG;
    return gmax * kLeafT;
}

hipError_t launch_leaf(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv,
                       int64_t *info, PanelSync *ps, uint32_t *host_base, uint32_t *flags,
                       hipStream_t s) {
    if (w <= 0 || w > kLeafMaxW || k0 >= n) return hipErrorInvalidValue;
    if (mode == LU_F64)
        return leaf_go<double, false>((double *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    if (mode == LU_F32)
        return leaf_go<float, false>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    return leaf_go<float, true>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
}

hipError_t launch_laswp(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int cnt,
                        const int32_t *ipiv, int64_t c0, int64_t c1, int64_t c2, int64_t c3,
                        int32_t *perm, hipStream_t s) {
    (void)n;
    if (cnt <= 0 || cnt > 256) return hipErrorInvalidValue;
    const int64_t wtot = (c1 - c0) + (c3 - c2);
    if (mode == LU_F64) {
        constexpr int CB = 32;
        const int nb = (int)((wtot + CB - 1) / CB);
        k_laswp<double, CB><<<nb + 1, 256, 0, s>>>((double *)a, ld, k0, cnt, ipiv, c0, c1, c2, c3, perm, nb);
    } else {
        constexpr int CB = 64;
        const int nb = (int)((wtot + CB - 1) / CB);
        k_laswp<float, CB><<<nb + 1, 256, 0, s>>>((float *)a, ld, k0, cnt, ipiv, c0, c1, c2, c3, perm, nb);
    }
    return hipGetLastError();
}

hipError_t launch_trsm(int mode, void *a, int64_t ld, int64_t k, int w, int64_t c0, int64_t c1,
                       hipStream_t s) {
    if (w <= 0 || w > 64 || c1 <= c0) return w <= 0 || w > 64 ? hipErrorInvalidValue : hipSuccess;
    const unsigned nb = (unsigned)((c1 - c0 + 63) / 64);
    if (mode == LU_F64) k_trsm<double, false><<<nb, 256, 0, s>>>((double *)a, ld, k, w, c0, c1);
    else if (mode == LU_F32) k_trsm<float, false><<<nb, 256, 0, s>>>((float *)a, ld, k, w, c0, c1);
    else k_trsm<float, true><<<nb, 256, 0, s>>>((float *)a, ld, k, w, c0, c1);
    return hipGetLastError();
}

}  // namespace mpir
