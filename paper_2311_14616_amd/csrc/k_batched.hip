// Batched iterative refinement: thousands of independent systems of uneven
// size (n <= 1024) solved in one persistent launch.  Each workgroup takes the
// next system from an atomic queue (systems ordered largest first, so the
// long ones start early) and runs the whole method on it: the interprecision
// copy and ||A||_inf, a blocked right-looking LU with partial pivoting (32
// column panels factored in LDS, interchanges, U12 solve, trailing update on
// the matrix cores), then Algorithm IR (low-precision triangular solves,
// update, FP64 residual, the termination rules) and a per-system report.
//
// Storage per system: the caller's A (column-major, TW), b and x (TW); a
// row-major binary32 working array W (n x n; binary16 / bfloat16 numbers for
// TF = F16 / BF16)
// and the row permutation, both in a workspace owned by the library.
#include "mpir_internal.h"

namespace mpir {

// Device time of each phase of the batched kernel, summed over its
// workgroups since the last reset (wall-clock ticks; see mpir_batch_phase_times).
__device__ unsigned long long g_batch_phase[kBatchPhases];

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

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The 16-bit operand type of the factorization's rounding RD (1 binary16,
// 2 bfloat16), its 8-element vector and the 32x32x16 MFMA on it.
template <int RD> struct Lo16 {
    using T = _Float16;
    using V8 = half8;
    __device__ static floatx16 mfma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Lo16<2> {
    using T = __bf16;
    using V8 = bf16x8;
    __device__ static floatx16 mfma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

constexpr int NT = 512;             // threads per workgroup
constexpr int NW = NT / 64;         // waves
constexpr int NMAX = 1024;          // largest system
constexpr int PB = 32;              // panel width
constexpr int PP = PB + 1;          // LDS pitch of the panel
constexpr int PANEL_FLOATS = NMAX * PP;

__device__ __forceinline__ double pow2_ceil(double m) {
    int e;
    const double f = frexp(m, &e);
    return f == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

// Global-memory pointers of the device pass (the host pass sees plain
// pointers).
#if defined(__HIP_DEVICE_COMPILE__)
#define GMEM __attribute__((address_space(1)))
#else
#define GMEM
#endif

// One 32 x 32 block of C in the matrix-core accumulator layout (lane l,
// entry v: row r0 + 8(v/4) + 4(l/32) + v%4, column bc).  Loads are issued
// unconditionally (out-of-range entries read an in-range word and are
// zeroed), so the compiler keeps them in flight across the products.
__device__ __forceinline__ void load_cblock(const GMEM float *W, int n, int r0, int bc, int lane,
                                            bool any, float (&c)[16]) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const bool ok = any && row < n && bc < n;
        const float x = W[(int64_t)(ok ? row : 0) * n + (ok ? bc : 0)];
        c[v] = ok ? x : 0.0f;
    }
}
__device__ __forceinline__ void store_cblock(GMEM float *W, int n, int r0, int bc, int lane,
                                             const float (&c)[16], const floatx16 &acc) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row < n && bc < n) W[(int64_t)row * n + bc] = c[v] - acc[v];
    }
}

// The same with the block's rows limited to < rlim and columns to < clim.
__device__ __forceinline__ void load_cblock_lim(const GMEM float *W, int n, int r0, int bc, int lane,
                                                int rlim, int clim, float (&c)[16]) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const bool ok = row < rlim && bc < clim;
        const float x = W[(int64_t)(ok ? row : 0) * n + (ok ? bc : 0)];
        c[v] = ok ? x : 0.0f;
    }
}
__device__ __forceinline__ void store_cblock_lim(GMEM float *W, int n, int r0, int bc, int lane,
                                                 int rlim, int clim, const float (&c)[16],
                                                 const floatx16 &acc) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row < rlim && bc < clim) W[(int64_t)row * n + bc] = c[v] - acc[v];
    }
}

// Rows of the rank-64 update's A panel staged in LDS at a time (pitch kWP).
constexpr int kWP = 65;
constexpr int kWideRows = 512;
static_assert(kWideRows * kWP <= PANEL_FLOATS, "wide update chunk fits the panel buffer");

// dst(e) = src(e) for e = tid, tid + NT, ... < N, with U loads in flight per
// thread (all U issued before the first is stored; src(e) must accept any
// e < N, and is called with e0 in place of an out-of-range e).
template <int U, typename LD, typename ST>
__device__ __forceinline__ void staged_copy(int N, LD src, ST dst) {
    for (int e0 = threadIdx.x; e0 < N; e0 += U * NT) {
        decltype(src(0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            v[u] = src(e < N ? e : e0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            if (e < N) dst(e, v[u]);
        }
    }
}

// Max of a non-negative double over the workgroup (NaN wins), via bits.
__device__ __forceinline__ double block_max(double v, uint64_t *red) {
    uint64_t b = (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)b, off);
        b = o > b ? o : b;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = b;
    __syncthreads();
    uint64_t m = red[0];
    for (int q = 1; q < NW; ++q) m = red[q] > m ? red[q] : m;
    return __longlong_as_double((long long)m);
}

template <typename TWt, int RD>
__global__ __launch_bounds__(NT) void k_batched(const BatchSys *__restrict__ sys,
                                                const int32_t *__restrict__ order, int nsys,
                                                uint32_t *queue, BatchTerm term,
                                                mpir_report *__restrict__ reps, double tick_ms) {
    __shared__ __align__(16) float panel[PANEL_FLOATS];   // LU: panel / staging tiles
    // refinement phase (the LU is finished): vectors carved from the panel
    double *const vr = reinterpret_cast<double *>(panel);  // residual (TR = FP64)
    double *const vx = vr + NMAX;                          // x as binary64 (exact copy of TW)
    float *const vy = reinterpret_cast<float *>(vx + NMAX); // low-precision rhs / solution
    __shared__ float L11[PB][PB + 1];
    __shared__ int32_t piv[PB];
    __shared__ int32_t pdst[2 * PB], psrc[2 * PB];
    __shared__ uint64_t redk[NW];
    __shared__ uint64_t redb[NW];
    __shared__ double tmp64[64];
    __shared__ double hist_r[MPIR_HIST_MAX], hist_d[MPIR_HIST_MAX];
    __shared__ int s_sys, s_extra, s_info, s_flags;
    (void)tmp64;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (;;) {
        if (tid == 0) {
            const uint32_t q = atomicAdd(queue, 1u);
            s_sys = q < (uint32_t)nsys ? order[q] : -1;
            s_info = 0;
            s_flags = 0;
        }
        __syncthreads();
        const int si = s_sys;
        if (si < 0) break;
        const long long t_start = wall_clock64();
        // phase timer: thread 0 adds the ticks since the previous mark.  (A
        // macro, not a lambda: with the lambda the compiler's allocation of
        // the binary32 kernel spilled 180 registers instead of 47, and the
        // batch ran 10% slower.)
        long long t_ph = t_start;
#define MARK(ph)                                                                        \
    do {                                                                                \
        if (tid == 0) {                                                                 \
            const long long t_ = wall_clock64();                                        \
            atomicAdd(&g_batch_phase[ph], (unsigned long long)(t_ - t_ph));             \
            t_ph = t_;                                                                  \
        }                                                                               \
    } while (0)
        const BatchSys S = sys[si];
        const int n = (int)S.n;
        const int64_t lda = S.lda;
        // every per-system pointer addresses global memory; typed so, the
        // compiler emits global (not flat) loads and stores, whose waits do
        // not also wait for LDS traffic
        const GMEM TWt *A = (const GMEM TWt *)S.A;
        const GMEM TWt *b = (const GMEM TWt *)S.b;
        GMEM TWt *x = (GMEM TWt *)S.x;
        GMEM float *W = (GMEM float *)S.W;
        GMEM int32_t *perm = (GMEM int32_t *)S.perm;
        // tuned per size class: panel width (16 or 32) and update form
        const int cfg = (int)S.pad;
        const int pb = (cfg & 0xff) == 16 ? 16 : PB;
        const int upd = (cfg >> 8) & 0xff;

        // ---------------- interchange-free copy A_F = fl_F(A), ||A||_inf ----
        // 256 x 64 tiles: coalesced column reads, LDS transpose, coalesced
        // row writes; row sums by one thread per row in increasing column
        // order (256 rows summed side by side).
        constexpr int TR = 256, TC = 64, TP = TR + 1;
        double *tile = reinterpret_cast<double *>(panel);   // [TC][TP] doubles
        static_assert(TC * TP * 2 <= PANEL_FLOATS, "tile fits the panel buffer");
        double amax = 0.0;                                  // max row sum seen by this thread
        for (int i0 = 0; i0 < n; i0 += TR) {
            double racc = 0.0;
            for (int j0 = 0; j0 < n; j0 += TC) {
                staged_copy<16>(TR * TC,
                    [&](int e) {
                        const int i = i0 + e % TR, j = j0 + e / TR;
                        const bool ok = i < n && j < n;
                        return A[(ok ? i : 0) + (int64_t)(ok ? j : 0) * lda];
                    },
                    [&](int e, TWt v) {
                        const int r = e % TR, c = e / TR;
                        tile[c * TP + r] = (i0 + r < n && j0 + c < n) ? (double)v : 0.0;
                    });
                __syncthreads();
                if (tid < TR && i0 + tid < n) {
                    // columns beyond n hold zeros: adding them changes nothing
#pragma unroll
                    for (int c0 = 0; c0 < TC; c0 += 16) {
                        double t[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) t[u] = tile[(c0 + u) * TP + tid];
#pragma unroll
                        for (int u = 0; u < 16; ++u) racc = racc + fabs(t[u]);
                    }
                }
                int fl = 0;
                for (int e = tid; e < TR * TC; e += NT) {
                    const int c = e % TC, r = e / TC;
                    const int i = i0 + r, j = j0 + c;
                    if (i < n && j < n) {
                        const double v = tile[c * TP + r];
                        const float f = RD == 1 ? d2h_as_float(v) : RD == 2 ? d2bf_as_float(v) : (float)v;
                        if (!isfinite(v)) fl |= DF_NONFINITE;
                        else if (isinf(f)) fl |= DF_RANGE;
                        W[(int64_t)i * n + j] = f;
                    }
                }
                if (fl) atomicOr(&s_flags, fl);
                __syncthreads();
            }
            if (tid < TR && i0 + tid < n) {
                amax = fmax(amax, racc);
                if (isnan(racc)) amax = racc;
            }
        }
        for (int i = tid; i < n; i += NT) perm[i] = i;
        __syncthreads();
        const double anorm = block_max(amax, redb);
        if (s_flags) {
            if (tid == 0) {
                mpir_report &R = reps[si];
                R.n_iter = 0;
                R.stop = 0;
                R.reserved = (s_flags & DF_NONFINITE) ? MPIR_ERR_NONFINITE : MPIR_ERR_RANGE;
                R.info = 0;
            }
            __syncthreads();
            continue;
        }

        // C[r0 .. r0+nr) x [c0 .. c0+nc) -= W[., kk0 .. kk0+kw) W[kk0 .. kk0+kw, .)
        // (kw <= 32), every 32 x 32 block on its own, both operands from
        // memory (unconditional loads: out-of-range entries read an in-range
        // word and are zeroed)
        auto upd_blocks = [&](int r0, int nr, int c0, int nc, int kk0, int kw) {
            const int nbr = (nr + 31) / 32, nbc = (nc + 31) / 32;
            const int rlim = r0 + nr, clim = c0 + nc;
            for (int blk = wv; blk < nbr * nbc; blk += NW) {
                const int bi = blk / nbc, bj = blk - bi * nbc;
                const int rb = r0 + bi * 32, cb = c0 + bj * 32;
                const int ar = rb + (lane & 31), bc = cb + (lane & 31);
                float cv[16];
                floatx16 acc = floatx16{0};
                if constexpr (RD != 0) {
                    using L16 = Lo16<RD>;
                    typename L16::V8 av[2], bvv[2];
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int kq = 16 * s2 + 8 * (lane >> 5) + q;
                            const bool oka = ar < rlim && kq < kw, okb = bc < clim && kq < kw;
                            const float xa = W[(int64_t)(oka ? ar : 0) * n + kk0 + (oka ? kq : 0)];
                            const float xb = W[(int64_t)(kk0 + (okb ? kq : 0)) * n + (okb ? bc : 0)];
                            av[s2][q] = (typename L16::T)(oka ? xa : 0.0f);
                            bvv[s2][q] = (typename L16::T)(okb ? xb : 0.0f);
                        }
                    load_cblock_lim(W, n, rb, bc, lane, rlim, clim, cv);
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) acc = L16::mfma(av[s2], bvv[s2], acc);
                } else {
                    float av[16], bvv[16];
#pragma unroll
                    for (int s1 = 0; s1 < 16; ++s1) {
                        const int kq = 2 * s1 + (lane >> 5);
                        const bool oka = ar < rlim && kq < kw, okb = bc < clim && kq < kw;
                        const float xa = W[(int64_t)(oka ? ar : 0) * n + kk0 + (oka ? kq : 0)];
                        const float xb = W[(int64_t)(kk0 + (okb ? kq : 0)) * n + (okb ? bc : 0)];
                        av[s1] = oka ? xa : 0.0f;
                        bvv[s1] = okb ? xb : 0.0f;
                    }
                    load_cblock_lim(W, n, rb, bc, lane, rlim, clim, cv);
#pragma unroll
                    for (int s1 = 0; s1 < 16; ++s1)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s1], bvv[s1], acc, 0, 0, 0);
                }
                store_cblock_lim(W, n, rb, bc, lane, rlim, clim, cv, acc);
            }
        };
        // rows and columns [r0, n) -= W[., kk0 .. kk0+kw) W[kk0 .. kk0+kw, .)
        // (kw <= 64): the A panel staged in LDS in chunks of up to kWideRows
        // rows; wave wv takes block columns bj = wv, wv + NW, ..., holds that
        // column's B block in registers and sweeps the chunk's block rows,
        // the next block row's C loads in flight
        auto upd_wide = [&](int r0, int kk0, int kw) {
            const int mm = n - r0;
            const int nbc = (mm + 31) / 32;
            for (int q0 = 0; q0 < mm; q0 += kWideRows) {
                const int cr = (mm - q0) < kWideRows ? (mm - q0) : kWideRows;
                const int nbr = (cr + 31) / 32;
                __syncthreads();
                staged_copy<8>(cr * 64,
                    [&](int e) {
                        const int r = e >> 6, c = e & 63;
                        return W[(int64_t)(r0 + q0 + r) * n + kk0 + (c < kw ? c : 0)];
                    },
                    [&](int e, float v) { panel[(e >> 6) * kWP + (e & 63)] = (e & 63) < kw ? v : 0.0f; });
                __syncthreads();
                for (int bj = wv; bj < nbc; bj += NW) {
                    const int cb = r0 + bj * 32, bc = cb + (lane & 31);
                    const int rb0 = r0 + q0;
                    if constexpr (RD != 0) {
                        using L16 = Lo16<RD>;
                        typename L16::V8 bh[4];
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const int kq = 16 * s2 + 8 * (lane >> 5) + q;
                                const bool ok = bc < n && kq < kw;
                                const float xb = W[(int64_t)(kk0 + (ok ? kq : 0)) * n + (ok ? bc : 0)];
                                bh[s2][q] = (typename L16::T)(ok ? xb : 0.0f);
                            }
                        float cv[16], cn[16];
                        load_cblock(W, n, rb0, bc, lane, true, cv);
                        for (int bi = 0; bi < nbr; ++bi) {
                            const int rb = rb0 + bi * 32, lr = bi * 32 + (lane & 31);
                            load_cblock(W, n, rb + 32, bc, lane, bi + 1 < nbr, cn);
                            floatx16 acc = floatx16{0};
#pragma unroll
                            for (int s2 = 0; s2 < 4; ++s2) {
                                typename L16::V8 av;
#pragma unroll
                                for (int q = 0; q < 8; ++q) {
                                    const float pv = panel[lr * kWP + 16 * s2 + 8 * (lane >> 5) + q];
                                    av[q] = (typename L16::T)(lr < cr ? pv : 0.0f);
                                }
                                acc = L16::mfma(av, bh[s2], acc);
                            }
                            store_cblock(W, n, rb, bc, lane, cv, acc);
#pragma unroll
                            for (int v = 0; v < 16; ++v) cv[v] = cn[v];
                        }
                    } else {
                        float bf[32];
#pragma unroll
                        for (int s1 = 0; s1 < 32; ++s1) {
                            const int kq = 2 * s1 + (lane >> 5);
                            bf[s1] = (bc < n && kq < kw) ? W[(int64_t)(kk0 + kq) * n + bc] : 0.0f;
                        }
                        float cv[16], cn[16];
                        load_cblock(W, n, rb0, bc, lane, true, cv);
                        for (int bi = 0; bi < nbr; ++bi) {
                            const int rb = rb0 + bi * 32, lr = bi * 32 + (lane & 31);
                            load_cblock(W, n, rb + 32, bc, lane, bi + 1 < nbr, cn);
                            floatx16 acc = floatx16{0};
#pragma unroll
                            for (int s1 = 0; s1 < 32; ++s1) {
                                const float pv = panel[lr * kWP + 2 * s1 + (lane >> 5)];
                                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(lr < cr ? pv : 0.0f, bf[s1], acc, 0, 0, 0);
                            }
                            store_cblock(W, n, rb, bc, lane, cv, acc);
#pragma unroll
                            for (int v = 0; v < 16; ++v) cv[v] = cn[v];
                        }
                    }
                }
            }
        };
        // update form 2: panels in pairs.  The first panel of a pair updates
        // only the second's columns (after its U rows for every column to
        // the right); the second panel, after its own interchanges, applies
        // the first's update to its 32 rows right of it, forms its U rows,
        // and one update of rank 64 (both panels' L columns) brings the rest
        // of the matrix up to date -- half the trailing matrix's memory
        // traffic of two rank-32 updates.  Row interchanges of the second
        // panel are applied to whole rows, so they meet the deferred update
        // consistently.
        const bool pairs = upd == 2 && pb == PB;

        MARK(0);
        // ---------------- blocked LU with partial pivoting ----------------
        for (int k = 0; k < n; k += pb) {
            if (k > 0) { __syncthreads(); MARK(4); }
            const int w = (n - k) < pb ? (n - k) : pb;
            const int m = n - k;
            __syncthreads();
            staged_copy<8>(m * w,
                [&](int e) { const int r = e / w, c = e - r * w; return W[(int64_t)(k + r) * n + k + c]; },
                [&](int e, float v) { const int r = e / w, c = e - r * w; panel[r * PP + c] = v; });
            __syncthreads();
            // first maximum of |a_rj|, r >= j: key = |v| bits above the
            // complemented row, maximised by DPP in each wave, then over the
            // waves by every thread.  Each thread forms its candidates for
            // column j+1 while it updates its rows for column j.
            auto cand = [&](float v, int r) {
                return ((uint64_t)__float_as_uint(fabsf(v)) << 32) | (uint64_t)(0xffffffffu - (uint32_t)r);
            };
            uint64_t key = 0;
            for (int r = tid; r < m; r += NT) {
                const uint64_t kk = cand(panel[r * PP], r);
                key = kk > key ? kk : key;
            }
            for (int j = 0; j < w; ++j) {
                key = wave_max_u64(key);
                if (lane == 0) redk[wv] = key;
                __syncthreads();
                uint64_t kb = redk[0];
#pragma unroll
                for (int q = 1; q < NW; ++q) kb = redk[q] > kb ? redk[q] : kb;
                const int p = (int)(0xffffffffu - (uint32_t)kb);
                if (tid == 0) piv[j] = p;
                if (tid < w) {
                    const int c = tid;
                    const float t = panel[j * PP + c];
                    float pv = panel[p * PP + c];
                    if (p != j) panel[p * PP + c] = t;
                    if (RD && c >= j) pv = round_lo<RD>(pv);
                    panel[j * PP + c] = pv;
                }
                __syncthreads();
                const float pj = panel[j * PP + j];
                if (pj == 0.0f && tid == 0 && s_info == 0) s_info = k + j + 1;
                key = 0;
                for (int r = j + 1 + tid; r < m; r += NT) {
                    if (pj != 0.0f) {
                        float l = panel[r * PP + j] / pj;
                        if (RD) l = round_lo<RD>(l);
                        panel[r * PP + j] = l;
                        // eight columns per step: their LDS reads in flight
                        // together (one column at a time waited for each read)
                        int c = j + 1;
                        for (; c + 8 <= w; c += 8) {
                            float pr[8], x[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                pr[u] = panel[j * PP + c + u];
                                x[u] = panel[r * PP + c + u];
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const float prod = l * pr[u];
                                panel[r * PP + c + u] = x[u] - prod;
                            }
                        }
                        for (; c < w; ++c) {
                            const float prod = l * panel[j * PP + c];
                            panel[r * PP + c] = panel[r * PP + c] - prod;
                        }
                    }
                    if (j + 1 < w) {
                        const uint64_t kk = cand(panel[r * PP + j + 1], r);
                        key = kk > key ? kk : key;
                    }
                }
                // redk and the pivot row are rewritten only after the next
                // barrier, which every thread reaches after its reads here
            }
            __syncthreads();
            for (int e = tid; e < m * w; e += NT) {
                const int r = e / w, c = e - r * w;
                W[(int64_t)(k + r) * n + k + c] = panel[r * PP + c];
            }
            MARK(1);
            // composed row permutation of this panel (positions >= k)
            if (tid == 0) s_extra = 0;
            __syncthreads();
            if (tid < w) {
                auto src_of = [&](int i) {
                    for (int s = w - 1; s >= 0; --s) {
                        const int ks = s, ps = piv[s];
                        if (i == ks) i = ps;
                        else if (i == ps) i = ks;
                    }
                    return i;
                };
                pdst[tid] = tid;
                psrc[tid] = src_of(tid);
                const int pp = piv[tid];
                if (pp >= w) {
                    bool first = true;
                    for (int q = 0; q < tid; ++q) if (piv[q] == pp) { first = false; break; }
                    if (first) {
                        const int slot = w + atomicAdd(&s_extra, 1);
                        pdst[slot] = pp;
                        psrc[slot] = src_of(pp);
                    }
                }
            }
            __syncthreads();
            const int np = w + s_extra;
            // apply it to the columns outside the panel and to perm (LDS staged)
            {
                constexpr int CH = 256;
                float *stage = panel;                       // [2*PB][CH]
                int32_t *pst = reinterpret_cast<int32_t *>(panel + 2 * PB * CH);
                for (int q = tid; q < np; q += NT) pst[q] = perm[k + psrc[q]];
                for (int c0 = 0; c0 < n; c0 += CH) {
                    __syncthreads();
                    staged_copy<8>(np * CH,
                        [&](int e) {
                            const int q = e / CH, c = c0 + (e - q * CH);
                            const bool ok = c < n && (c < k || c >= k + w);
                            return W[(int64_t)(k + psrc[q]) * n + (ok ? c : 0)];
                        },
                        [&](int e, float v) { stage[e] = v; });
                    __syncthreads();
                    for (int e = tid; e < np * CH; e += NT) {
                        const int q = e / CH, c = c0 + (e - q * CH);
                        if (c < n && (c < k || c >= k + w))
                            W[(int64_t)(k + pdst[q]) * n + c] = stage[e];
                    }
                }
                __syncthreads();
                for (int q = tid; q < np; q += NT) perm[k + pdst[q]] = pst[q];
            }
            MARK(2);
            if (k + w >= n) break;
            const bool second = pairs && ((k / PB) & 1);
            const bool first = pairs && !second;
            if (second) {
                // the first panel's update of this panel's rows right of it
                upd_blocks(k, w, k + w, n - k - w, k - PB, PB);
                __syncthreads();
            }
            // U12 = L11^{-1} A12 for rows [k, k+w), columns [k+w, n)
            for (int e = tid; e < w * w; e += NT) {
                const int r = e / w, c = e - r * w;
                L11[r][c] = W[(int64_t)(k + r) * n + k + c];
            }
            __syncthreads();
            // one thread per column, the column in registers (fully
            // unrolled over the panel width; a column kept in LDS made every
            // step an LDS read-modify-write on the dependence chain), L11
            // read from LDS by broadcast
            for (int c0 = k + w; c0 < n; c0 += NT) {
                const int c = c0 + tid;
                if (c < n) {
                    float xv[PB];
#pragma unroll
                    for (int t = 0; t < PB; ++t) xv[t] = W[(int64_t)(k + (t < w ? t : 0)) * n + c];
#pragma unroll
                    for (int t = 0; t < PB; ++t) {
                        if (t < w) {
                            float xt = xv[t];
                            if (RD) { xt = round_lo<RD>(xt); xv[t] = xt; }
#pragma unroll
                            for (int s2 = t + 1; s2 < PB; ++s2)
                                if (s2 < w) {
                                    const float prod = L11[s2][t] * xt;
                                    xv[s2] = xv[s2] - prod;
                                }
                        }
                        // keep column t's L11 reads in this step (hoisting
                        // all 496 of them spilled registers)
                        __asm__ volatile("" ::: "memory");
                    }
#pragma unroll
                    for (int t = 0; t < PB; ++t)
                        if (t < w) W[(int64_t)(k + t) * n + c] = xv[t];
                }
            }
            __syncthreads();
            MARK(3);
            if (first) {
                // only the next panel's columns
                const int w2 = (n - k - w) < PB ? (n - k - w) : PB;
                upd_blocks(k + w, n - k - w, k + w, w2, k, w);
            } else if (second) {
                upd_wide(k + w, k - PB, PB + w);
            } else
            // trailing update A22 -= L21 U12 (K = w <= 32) in 32 x 32 blocks
            if (upd == 1) {
                // L21 staged in LDS once; wave wv takes block columns bj =
                // wv, wv + NW, ..., holds that column's U12 block in
                // registers and sweeps the block rows.
                const int r0 = k + w, mm = n - r0;
                const int nbk = (mm + 31) / 32;
                staged_copy<8>(mm * PB,
                    [&](int e) {
                        const int r = e / PB, c = e - r * PB;
                        return W[(int64_t)(r0 + r) * n + k + (c < w ? c : 0)];
                    },
                    [&](int e, float v) { panel[(e / PB) * PP + e % PB] = e % PB < w ? v : 0.0f; });
                __syncthreads();
                for (int bj = wv; bj < nbk; bj += NW) {
                    const int cb = r0 + bj * 32, bc = cb + (lane & 31);
                    if constexpr (RD != 0) {
                        using L16 = Lo16<RD>;
                        typename L16::V8 bh[2];
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const int kq = 16 * s2 + 8 * (lane >> 5) + q;
                                bh[s2][q] = (typename L16::T)((bc < n && kq < w) ? W[(int64_t)(k + kq) * n + bc] : 0.0f);
                            }
                        // C of the next block row is loaded while this one
                        // is multiplied and stored
                        float cv[16], cn[16];
                        load_cblock(W, n, r0, bc, lane, true, cv);
                        for (int bi = 0; bi < nbk; ++bi) {
                            const int rb = r0 + bi * 32, lr = bi * 32 + (lane & 31);
                            load_cblock(W, n, rb + 32, bc, lane, bi + 1 < nbk, cn);
                            floatx16 acc = floatx16{0};
                            // entries beyond w are zero in both operands
#pragma unroll
                            for (int s2 = 0; s2 < 2; ++s2) {
                                typename L16::V8 av;
#pragma unroll
                                for (int q = 0; q < 8; ++q) {
                                    const float pv = panel[lr * PP + 16 * s2 + 8 * (lane >> 5) + q];
                                    av[q] = (typename L16::T)(lr < mm ? pv : 0.0f);
                                }
                                acc = L16::mfma(av, bh[s2], acc);
                            }
                            store_cblock(W, n, rb, bc, lane, cv, acc);
#pragma unroll
                            for (int v = 0; v < 16; ++v) cv[v] = cn[v];
                        }
                    } else {
                        float bf[16];
#pragma unroll
                        for (int s1 = 0; s1 < 16; ++s1) {
                            const int kq = 2 * s1 + (lane >> 5);
                            bf[s1] = (bc < n && kq < w) ? W[(int64_t)(k + kq) * n + bc] : 0.0f;
                        }
                        float cv[16], cn[16];
                        load_cblock(W, n, r0, bc, lane, true, cv);
                        for (int bi = 0; bi < nbk; ++bi) {
                            const int rb = r0 + bi * 32, lr = bi * 32 + (lane & 31);
                            load_cblock(W, n, rb + 32, bc, lane, bi + 1 < nbk, cn);
                            floatx16 acc = floatx16{0};
                            // entries beyond w are zero in both operands
#pragma unroll
                            for (int s1 = 0; s1 < 16; ++s1) {
                                const float pv = panel[lr * PP + 2 * s1 + (lane >> 5)];
                                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(lr < mm ? pv : 0.0f, bf[s1], acc, 0, 0, 0);
                            }
                            store_cblock(W, n, rb, bc, lane, cv, acc);
#pragma unroll
                            for (int v = 0; v < 16; ++v) cv[v] = cn[v];
                        }
                    }
                }
            } else {
                // every 32 x 32 block on its own: both operands from memory
                const int r0 = k + w, mm = n - r0;
                const int nbk = (mm + 31) / 32;
                for (int blk = wv; blk < nbk * nbk; blk += NW) {
                    const int bi = blk / nbk, bj = blk - bi * nbk;
                    const int rb = r0 + bi * 32, cb = r0 + bj * 32;
                    const int ar = rb + (lane & 31), bc = cb + (lane & 31);
                    // operands and C first (unconditional loads: out-of-range
                    // entries read an in-range word and are zeroed), then
                    // the products
                    float cv[16];
                    floatx16 acc = floatx16{0};
                    if constexpr (RD != 0) {
                        using L16 = Lo16<RD>;
                        typename L16::V8 av[2], bvv[2];
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const int kq = 16 * s2 + 8 * (lane >> 5) + q;
                                const bool oka = ar < n && kq < w, okb = bc < n && kq < w;
                                const float xa = W[(int64_t)(oka ? ar : 0) * n + k + (oka ? kq : 0)];
                                const float xb = W[(int64_t)(k + (okb ? kq : 0)) * n + (okb ? bc : 0)];
                                av[s2][q] = (typename L16::T)(oka ? xa : 0.0f);
                                bvv[s2][q] = (typename L16::T)(okb ? xb : 0.0f);
                            }
                        load_cblock(W, n, rb, bc, lane, true, cv);
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2)
                            acc = L16::mfma(av[s2], bvv[s2], acc);
                    } else {
                        float av[16], bvv[16];
#pragma unroll
                        for (int s1 = 0; s1 < 16; ++s1) {
                            const int kq = 2 * s1 + (lane >> 5);
                            const bool oka = ar < n && kq < w, okb = bc < n && kq < w;
                            const float xa = W[(int64_t)(oka ? ar : 0) * n + k + (oka ? kq : 0)];
                            const float xb = W[(int64_t)(k + (okb ? kq : 0)) * n + (okb ? bc : 0)];
                            av[s1] = oka ? xa : 0.0f;
                            bvv[s1] = okb ? xb : 0.0f;
                        }
                        load_cblock(W, n, rb, bc, lane, true, cv);
#pragma unroll
                        for (int s1 = 0; s1 < 16; ++s1)
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s1], bvv[s1], acc, 0, 0, 0);
                    }
                    store_cblock(W, n, rb, bc, lane, cv, acc);
                }
            }
        }
        __syncthreads();
        MARK(4);
        const int info = s_info;
        const long long t_lu = wall_clock64();

        // ---------------- Algorithm IR ----------------
        int it = 0, stop = MPIR_STOP_CONVERGED;
        double bnorm = 0.0, rnorm = 0.0, xnorm = 0.0;
        if (info == 0) {
            {
                double m = 0.0;
                for (int i = tid; i < n; i += NT) {
                    const double bi = (double)b[i];
                    vr[i] = bi;
                    vx[i] = 0.0;
                    x[i] = (TWt)0;
                    m = fmax(m, fabs(bi));
                    if (isnan(bi)) m = bi;
                }
                bnorm = block_max(m, redb);
            }
            rnorm = bnorm;
            if (tid == 0) hist_r[0] = bnorm;
            double prev_r = bnorm, prev_d = 0.0;
            bool done = false;
            if (!isfinite(bnorm)) { done = true; stop = MPIR_STOP_NONFINITE; }
            else if (bnorm == 0.0) done = true;
            else if (!term.wilk) {
                const bool conv = term.residterm ? (rnorm <= term.tol_r * bnorm)
                                                 : (rnorm <= term.tol_e * bnorm);
                done = conv;
            }
            while (!done) {
                const double sigma = pow2_ceil(rnorm);
                const double inv = 1.0 / sigma;
                for (int i = tid; i < n; i += NT) {
                    const double v = vr[perm[i]] * inv;
                    vy[i] = RD == 1 ? d2h_as_float(v) : RD == 2 ? d2bf_as_float(v) : (float)v;
                }
                __syncthreads();
                // 16-bit factors: the diagonal block of each substitution
                // step is staged in LDS by every wave, its loads in flight
                // with the off-diagonal block row's, so the 64-step chain
                // does not wait for them (solves 12.0 -> 10.7 ms per compute
                // unit for the binary16 batch).  The binary32 kernel keeps
                // wave 0's own loads: the staging's registers raised its
                // spills from 47 to 97 and slowed its trailing updates more
                // than the solves gained.
                constexpr int kDP = 65;
                float *const dtile = vy + NMAX;
                static_assert(5 * NMAX + 64 * kDP <= PANEL_FLOATS, "tile fits the panel buffer");
                static_assert(8 * NT == 64 * 64, "eight entries of the tile per thread");
                auto load_diag = [&](int i0, int rows, float (&dv)[8]) {
                    if constexpr (RD != 0) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int e = tid + q * NT, r = e >> 6, c = e & 63;
                            const bool ok = r < rows && c < rows;
                            const float v = W[(int64_t)(i0 + (ok ? r : 0)) * n + i0 + (ok ? c : 0)];
                            dv[q] = ok ? v : 0.0f;
                        }
                    }
                };
                auto store_diag = [&](const float (&dv)[8]) {
                    if constexpr (RD != 0) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int e = tid + q * NT;
                            dtile[(e >> 6) * kDP + (e & 63)] = dv[q];
                        }
                    }
                };
                // forward substitution with unit L, 64-row blocks
                for (int i0 = 0; i0 < n; i0 += 64) {
                    const int rows = (n - i0) < 64 ? (n - i0) : 64;
                    float dv[8];
                    load_diag(i0, rows, dv);
                    // off-diagonal: wave wv handles rows i0 + wv*8 .. +8
                    {
                        // the wave's 8 rows side by side: 8 loads in flight
                        float acc[8];
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) acc[rr] = 0.0f;
                        // four column strides per step: 32 loads in flight
                        for (int cb = lane; cb < i0; cb += 256) {
                            float yc[4], wr[8][4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) yc[u] = cb + 64 * u < i0 ? vy[cb + 64 * u] : 0.0f;
#pragma unroll
                            for (int rr = 0; rr < 8; ++rr)
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    wr[rr][u] = (wv * 8 + rr < rows && cb + 64 * u < i0)
                                                    ? W[(int64_t)(i0 + wv * 8 + rr) * n + cb + 64 * u] : 0.0f;
#pragma unroll
                            for (int u = 0; u < 4; ++u)
#pragma unroll
                                for (int rr = 0; rr < 8; ++rr)
                                    if (cb + 64 * u < i0) acc[rr] += wr[rr][u] * yc[u];
                        }
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) {
                            float a = acc[rr];
                            for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
                            if (lane == 0) tmp64[wv * 8 + rr] = a;
                        }
                    }
                    store_diag(dv);
                    __syncthreads();
                    if (wv == 0) {
                        float z = 0.0f;
                        float drow[64];
                        if (lane < rows) {
                            z = vy[i0 + lane] - (float)tmp64[lane];
#pragma unroll
                            for (int c = 0; c < 64; ++c)
                                if constexpr (RD != 0) drow[c] = dtile[lane * kDP + c];
                                else drow[c] = c < rows ? W[(int64_t)(i0 + lane) * n + i0 + c] : 0.0f;
                        } else {
#pragma unroll
                            for (int c = 0; c < 64; ++c) drow[c] = 0.0f;
                        }
#pragma unroll
                        for (int jj = 0; jj < 64; ++jj) {
                            const float yj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), jj));
                            if (lane > jj) z -= drow[jj] * yj;
                        }
                        if (lane < rows) vy[i0 + lane] = z;
                    }
                    __syncthreads();
                }
                // back substitution with U
                for (int i0 = ((n - 1) / 64) * 64; i0 >= 0; i0 -= 64) {
                    const int rows = (n - i0) < 64 ? (n - i0) : 64;
                    float dv[8];
                    load_diag(i0, rows, dv);
                    {
                        float acc[8];
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) acc[rr] = 0.0f;
                        for (int cb = i0 + 64 + lane; cb < n; cb += 256) {
                            float yc[4], wr[8][4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) yc[u] = cb + 64 * u < n ? vy[cb + 64 * u] : 0.0f;
#pragma unroll
                            for (int rr = 0; rr < 8; ++rr)
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    wr[rr][u] = (wv * 8 + rr < rows && cb + 64 * u < n)
                                                    ? W[(int64_t)(i0 + wv * 8 + rr) * n + cb + 64 * u] : 0.0f;
#pragma unroll
                            for (int u = 0; u < 4; ++u)
#pragma unroll
                                for (int rr = 0; rr < 8; ++rr)
                                    if (cb + 64 * u < n) acc[rr] += wr[rr][u] * yc[u];
                        }
#pragma unroll
                        for (int rr = 0; rr < 8; ++rr) {
                            float a = acc[rr];
                            for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
                            if (lane == 0) tmp64[wv * 8 + rr] = a;
                        }
                    }
                    store_diag(dv);
                    __syncthreads();
                    if (wv == 0) {
                        float z = 0.0f;
                        float drow[64];
                        if (lane < rows) {
                            z = vy[i0 + lane] - (float)tmp64[lane];
#pragma unroll
                            for (int c = 0; c < 64; ++c)
                                if constexpr (RD != 0) drow[c] = dtile[lane * kDP + c];
                                else drow[c] = c < rows ? W[(int64_t)(i0 + lane) * n + i0 + c] : 0.0f;
                        } else {
#pragma unroll
                            for (int c = 0; c < 64; ++c) drow[c] = 1.0f;
                        }
                        // the lane's own diagonal entry, inverted before
                        // the chain of 64 dependent steps (a division in
                        // each step would lengthen it several times)
                        float ul = drow[0];
#pragma unroll
                        for (int c = 1; c < 64; ++c)
                            if (lane == c) ul = drow[c];
                        const float rinv = 1.0f / ul;
#pragma unroll
                        for (int jj = 63; jj >= 0; --jj) {
                            if (lane == jj && lane < rows) z = z * rinv;
                            const float yj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), jj));
                            if (lane < jj) z -= drow[jj] * yj;
                        }
                        if (lane < rows) vy[i0 + lane] = z;
                    }
                    __syncthreads();
                }
                MARK(5);
                // d = sigma * y, x <- fl_W(x + d)
                double dm = 0.0;
                for (int i = tid; i < n; i += NT) {
                    const TWt d = (TWt)sigma * (TWt)vy[i];
                    const TWt xn = (TWt)vx[i] + d;
                    vx[i] = (double)xn;
                    x[i] = xn;
                    dm = fmax(dm, fabs((double)d));
                    if (isnan((double)d)) dm = (double)d;
                }
                const double dnorm = block_max(dm, redb);
                // r = b - A x in binary64 (thread per row, columns in order)
                double rm = 0.0, xm = 0.0;
                for (int i = tid; i < n; i += NT) {
                    double acc = 0.0;
                    const GMEM TWt *col = A + i;
                    // 16 loads in flight per thread, then the sums in order
                    int j = 0;
                    for (; j + 16 <= n; j += 16) {
                        TWt av[16];
#pragma unroll
                        for (int q = 0; q < 16; ++q) av[q] = col[(int64_t)(j + q) * lda];
#pragma unroll
                        for (int q = 0; q < 16; ++q) acc += (double)av[q] * vx[j + q];
                    }
                    for (; j < n; ++j) acc += (double)col[(int64_t)j * lda] * vx[j];
                    const double ri = (double)b[i] - acc;
                    vr[i] = ri;
                    rm = fmax(rm, fabs(ri));
                    if (isnan(ri)) rm = ri;
                    xm = fmax(xm, fabs(vx[i]));
                }
                rnorm = block_max(rm, redb);
                xnorm = block_max(xm, redb);
                MARK(6);
                ++it;
                if (tid == 0) { hist_r[it] = rnorm; hist_d[it - 1] = dnorm; }
                // every thread holds the same norms: the tests need no barrier
                const double pr = prev_r, pd = prev_d;
                prev_r = rnorm;
                prev_d = dnorm;
                if (!isfinite(rnorm) || !isfinite(dnorm)) { stop = MPIR_STOP_NONFINITE; break; }
                if (rnorm == 0.0) { stop = MPIR_STOP_CONVERGED; break; }
                if (!term.wilk) {
                    const bool conv = term.residterm ? (rnorm <= term.tol_r * bnorm)
                                                     : (rnorm <= term.tol_e * (bnorm + anorm * xnorm));
                    if (conv) { stop = MPIR_STOP_CONVERGED; break; }
                    if (it >= term.litmax) { stop = MPIR_STOP_LITMAX; break; }
                    if (rnorm >= term.rmax * pr) { stop = MPIR_STOP_STAGNATED; break; }
                } else {
                    if (it >= term.litmax) { stop = MPIR_STOP_LITMAX; break; }
                    if (it >= 2 && dnorm >= term.rmax * pd) { stop = MPIR_STOP_DSTAGNATED; break; }
                }
                __syncthreads();
            }
        }
        __syncthreads();
        MARK(6);
        // ---------------- report ----------------
        if (tid == 0) {
            mpir_report &R = reps[si];
            R.n_iter = it;
            R.stop = stop;
            R.n_hist = it + 1;
            R.reserved = info ? MPIR_ERR_SINGULAR : MPIR_OK;
            for (int q = 0; q <= it && q < MPIR_HIST_MAX; ++q) R.rhist[q] = hist_r[q];
            for (int q = 0; q < it && q < MPIR_HIST_MAX; ++q) R.dhist[q] = hist_d[q];
            R.anorm_inf = anorm;
            R.bnorm_inf = bnorm;
            R.xnorm_inf = xnorm;
            R.relres = bnorm > 0.0 ? rnorm / bnorm : rnorm;
            const double den = anorm * xnorm + bnorm;
            R.bwd_err = den > 0.0 ? rnorm / den : 0.0;
            R.info = info;
            R.t_factor_ms = (double)(t_lu - t_start) * tick_ms;
            R.t_ir_ms = (double)(wall_clock64() - t_lu) * tick_ms;
        }
        __syncthreads();
    }
}
#undef MARK

}  // namespace

int batched_max_n() { return NMAX; }

hipError_t batched_phase_ticks(unsigned long long *out, bool reset) {
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_batch_phase), sizeof(unsigned long long) * kBatchPhases);
    if (e != hipSuccess || !reset) return e;
    const unsigned long long zero[kBatchPhases] = {};
    return hipMemcpyToSymbol(HIP_SYMBOL(g_batch_phase), zero, sizeof zero);
}

hipError_t launch_batched(int tw, int tf, const BatchSys *sys, const int32_t *order, int nsys,
                          uint32_t *queue, const BatchTerm &term, mpir_report *reps, int nwg,
                          hipStream_t s) {
    // device wall clock (kHz) for the per-system timings in the reports
    static double tick_ms = -1.0;
    if (tick_ms < 0.0) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            tick_ms = 1.0 / (double)khz;
        else
            tick_ms = 0.0;
    }
    if (tw == MPIR_F64) {
        if (tf == MPIR_F16) k_batched<double, 1><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
        else if (tf == MPIR_BF16) k_batched<double, 2><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
        else k_batched<double, 0><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
    } else {
        if (tf == MPIR_F16) k_batched<float, 1><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
        else if (tf == MPIR_BF16) k_batched<float, 2><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
        else k_batched<float, 0><<<nwg, NT, 0, s>>>(sys, order, nsys, queue, term, reps, tick_ms);
    }
    return hipGetLastError();
}

}  // namespace mpir
