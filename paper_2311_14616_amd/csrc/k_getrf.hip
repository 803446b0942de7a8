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
constexpr int kLeafMaxG = 256;    // workgroups per leaf (one per CU)

// Per-column exchange area of the cooperative leaf: every workgroup posts
// its local pivot candidate (|value|, row, and the candidate row), the owner
// of the diagonal row posts that row; double-buffered by column parity.
struct LeafSlot {
    double val;
    int32_t idx;
    int32_t pad;
    double row[kLeafMaxW];
};
struct PanelSync {
    uint32_t counter;             // monotonic arrival counter (grid barrier)
    uint32_t pad0[31];
    uint32_t base;                // host-maintained copy (unused on device)
    uint32_t pad1[31];
    LeafSlot slot[2][kLeafMaxG];
    double diag[2][kLeafMaxW];
};

size_t panel_sync_bytes() { return sizeof(PanelSync); }

hipError_t panel_sync_reset(PanelSync *ps, hipStream_t s) {
    return hipMemsetAsync(ps, 0, 256, s);
}

namespace {

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// Leaf factorization of rows [k0, n) x columns [k0, k0+w) of the working
// array.  Workgroup g owns relative rows [g*R, g*R+R) in LDS.  For every
// column: local argmax (first maximum), exchange through PanelSync with one
// grid barrier, swap, scale, rank-1 update of the remaining leaf columns.
// F16: the pivot row is rounded to binary16 when it becomes the pivot row,
// each multiplier to binary16 when formed (products of binary16 numbers are
// exact in binary32).
template <typename W, bool F16, int RMAX>
__global__ __launch_bounds__(256) void k_leaf(W *__restrict__ a, int64_t n, int64_t ld,
                                              int64_t k0, int w, int R, int G,
                                              int32_t *__restrict__ ipiv, int64_t *info,
                                              PanelSync *ps, uint32_t base, uint32_t *flags) {
    constexpr int LDW = kLeafMaxW + 1;
    __shared__ W blk[RMAX * LDW];
    __shared__ double red_v[4];
    __shared__ int red_i[4];
    __shared__ double prow[kLeafMaxW];
    __shared__ double orow[kLeafMaxW];
    __shared__ int s_p, s_win, s_bad;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t m = n - k0;
    const int64_t r0 = (int64_t)blockIdx.x * R;
    const int rows = (int)((m - r0) < R ? (m - r0) : R);
    // an earlier launch already timed out: the arrival counter is behind,
    // so every workgroup returns at once (the host reports the error)
    if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & DF_TIMEOUT) return;
    if (tid == 0) s_bad = 0;

    for (int e = tid; e < rows * w; e += 256) {
        const int r = e / w, c = e - r * w;
        blk[r * LDW + c] = a[(k0 + r0 + r) * ld + k0 + c];
    }
    __syncthreads();

    for (int j = 0; j < w; ++j) {
        const int par = j & 1;
        // ---- local argmax of |a_rj| over owned rows r >= j ----
        double bv = -1.0;
        int bi = INT_MAX;
        for (int r = tid; r < rows; r += 256) {
            const int64_t rr = r0 + r;
            if (rr < j) continue;
            const double v = fabs((double)blk[r * LDW + j]);
            if (v > bv) { bv = v; bi = (int)rr; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < 4; ++q)
                if (better(red_v[q], red_i[q], red_v[0], red_i[0])) { red_v[0] = red_v[q]; red_i[0] = red_i[q]; }
        }
        __syncthreads();
        const double lbv = red_v[0];
        const int lbi = red_i[0];

        if (G == 1) {
            if (tid < w) {
                prow[tid] = (double)blk[(lbi - r0) * LDW + tid];
                orow[tid] = (double)blk[(j - r0) * LDW + tid];
            }
            if (tid == 0) s_p = lbi;
            __syncthreads();
        } else {
            // ---- post candidate, diagonal row; grid barrier; pick winner ----
            LeafSlot *my = &ps->slot[par][blockIdx.x];
            if (tid < w) {
                const bool has = lbi != INT_MAX;
                st_agent(&my->row[tid], has ? (double)blk[(lbi - r0) * LDW + tid] : 0.0);
                if (j >= r0 && j < r0 + rows) st_agent(&ps->diag[par][tid], (double)blk[(j - r0) * LDW + tid]);
            }
            if (tid == 0) {
                st_agent(&my->val, lbv);
                st_agent(&my->idx, (int32_t)lbi);
            }
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_fetch_add(&ps->counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t target = base + (uint32_t)(j + 1) * (uint32_t)G;
                uint64_t spins = 0;
                while (__hip_atomic_load(&ps->counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (++spins > kSpinLimit) { s_bad = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (wv == 0) {
                double gv = -1.0;
                int gi = INT_MAX, gw = 0;
                for (int g = lane; g < G; g += 64) {
                    const double v = ld_agent(&ps->slot[par][g].val);
                    const int i = ld_agent(&ps->slot[par][g].idx);
                    if (better(v, i, gv, gi)) { gv = v; gi = i; gw = g; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(gv, off);
                    const int oi = __shfl_xor(gi, off);
                    const int og = __shfl_xor(gw, off);
                    if (better(ov, oi, gv, gi)) { gv = ov; gi = oi; gw = og; }
                }
                if (lane == 0) { s_p = gi; s_win = gw; }
            }
            __syncthreads();
            if (tid < w) {
                prow[tid] = ld_agent(&ps->slot[par][s_win].row[tid]);
                orow[tid] = ld_agent(&ps->diag[par][tid]);
            }
            __syncthreads();
        }

        const int p = s_p;
        if (s_bad || p == INT_MAX) {   // expired wait: leave the loop, report
            if (tid == 0) atomicOr(flags, (uint32_t)DF_TIMEOUT);
            break;
        }
        if (tid < w) {
            double v = prow[tid];
            if (F16 && tid >= j) v = (double)round_f16((float)v);
            prow[tid] = v;
        }
        __syncthreads();
        // ---- swap rows j and p inside the leaf ----
        if (p != j) {
            if (p >= r0 && p < r0 + rows && tid < w) blk[(p - r0) * LDW + tid] = (W)orow[tid];
        }
        if (j >= r0 && j < r0 + rows && tid < w) blk[(j - r0) * LDW + tid] = (W)prow[tid];
        if (blockIdx.x == 0 && tid == 0) {
            ipiv[k0 + j] = (int32_t)(k0 + p);
            if (prow[j] == 0.0 && *info == 0) *info = k0 + j + 1;
        }
        __syncthreads();
        // ---- scale and rank-1 update of the owned rows below the pivot ----
        const W piv = (W)prow[j];
        if (piv != (W)0) {
            for (int r = tid; r < rows; r += 256) {
                const int64_t rr = r0 + r;
                if (rr <= j) continue;
                W l = blk[r * LDW + j] / piv;
                if (F16) l = (W)round_f16((float)l);
                blk[r * LDW + j] = l;
                for (int c = j + 1; c < w; ++c) {
                    const W prod = l * (W)prow[c];
                    blk[r * LDW + c] = blk[r * LDW + c] - prod;
                }
            }
        }
        __syncthreads();
    }

    for (int e = tid; e < rows * w; e += 256) {
        const int r = e / w, c = e - r * w;
        a[(k0 + r0 + r) * ld + k0 + c] = blk[r * LDW + c];
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

constexpr int kLeafRowsF = 1024;   // rows per workgroup held in LDS (binary32)
constexpr int kLeafRowsD = 512;    // (binary64)

template <typename W, bool F16, int RMAX>
hipError_t leaf_go(W *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv, int64_t *info,
                   PanelSync *ps, uint32_t *host_base, uint32_t *flags, hipStream_t s) {
    const int64_t m = n - k0;
    int64_t G64 = (m + RMAX - 1) / RMAX;
    const int gmax = num_cus() < kLeafMaxG ? num_cus() : kLeafMaxG;
    if (G64 > gmax) return hipErrorInvalidValue;
    // fewer rows per workgroup than RMAX when that keeps G unchanged
    const int G = (int)G64;
    const int R = (int)((m + G - 1) / G);
    uint32_t base = *host_base;
    if (G == 1) {
        k_leaf<W, F16, RMAX><<<1, 256, 0, s>>>(a, n, ld, k0, w, R, G, ipiv, info, ps, base, flags);
        return hipGetLastError();
    }
    void *args[] = {&a, (void *)&n, (void *)&ld, (void *)&k0, (void *)&w, (void *)&R, (void *)&G,
                    &ipiv, &info, &ps, &base, &flags};
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_leaf<W, F16, RMAX>, dim3(G), dim3(256),
                                              args, 0, s);
    if (e == hipSuccess) *host_base = base + (uint32_t)G * (uint32_t)w;
    return e;
}

}  // namespace

int leaf_max_rows(int mode) {
    const int gmax = num_cus() < kLeafMaxG ? num_cus() : kLeafMaxG;
    return gmax * (mode == LU_F64 ? kLeafRowsD : kLeafRowsF);
}

hipError_t launch_leaf(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv,
                       int64_t *info, PanelSync *ps, uint32_t *host_base, uint32_t *flags,
                       hipStream_t s) {
    if (w <= 0 || w > kLeafMaxW || k0 >= n) return hipErrorInvalidValue;
    if (mode == LU_F64)
        return leaf_go<double, false, kLeafRowsD>((double *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    if (mode == LU_F32)
        return leaf_go<float, false, kLeafRowsF>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    return leaf_go<float, true, kLeafRowsF>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
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
