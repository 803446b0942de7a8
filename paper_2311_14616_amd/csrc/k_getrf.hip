// Blocked right-looking LU with partial pivoting (the "Factor A = LU in
// precision TF" step of Algorithm IR; Julia lu! / LAPACK getrf semantics):
// the panel ("leaf") factorization with a wavefront argmax pivot search, the
// row interchanges, and the small unit-lower triangular solve that forms U12.
// The trailing-matrix update is in k_gemm.hip.
//
// Working array: row-major, leading dimension ld, binary32 (TF = F32, F16, BF16)
// or binary64 (TF = F64).  Row interchanges of a row-major matrix move
// contiguous memory, which is why this layout was chosen.
#include <climits>
#include <cstdlib>
#include <type_traits>

#include "mpir_internal.h"

namespace mpir {

constexpr int kLeafMaxW = 32;     // columns per leaf
constexpr int kLeafNT = 512;      // threads per leaf workgroup
// Rows per thread: one, so that the local part of a column (argmax, swap,
// rank-1 update) is as short as it can be; binary32 panels that would need
// more than kLeafMaxG workgroups, or fit one workgroup at two rows per
// thread (no exchange at all), take two (register budget: binary64 one).
template <typename W> constexpr int leaf_rt_max() { return sizeof(W) == 4 ? 2 : 1; }
constexpr int kLeafMaxG = 64;     // workgroups per leaf (one wave reads every slot)

// Exchange area of the leaf.  Every value travels in 64-bit words (32-bit
// payload | 32-bit epoch), so a reader that sees the current epoch in a word
// also sees its payload: no barrier counter, no fences.  Per column parity
// each workgroup g posts its candidate header (|value| in 2 words, row) and
// its candidate row (1-2 words per column); workgroup 0 also posts the old
// row j.  Binary32 leaves use areas indexed [word][g]: lane g of the reading
// wave loads word q of every workgroup with one coalesced load, so a poll of
// all workgroups is a few dozen cache lines.  Binary64 leaves (two posting
// and reading waves) keep one contiguous slot per workgroup: measured with a
// concurrent binary64 update, the [word][g] form slowed them down many times
// over, while binary32 leaves gain from it with or without that load.
constexpr int kHeadWords = 4;
constexpr int kRowWords = 2 * kLeafMaxW;
struct XchgWordMajor {
    uint64_t head[2][kHeadWords][kLeafMaxG];
    uint64_t row[2][kRowWords][kLeafMaxG];
    uint64_t diag[2][kRowWords];
};
struct XchgSlot {
    uint64_t head[kHeadWords];
    uint64_t row[kRowWords];
    uint64_t diag[kRowWords];
};
struct PanelSync {
    XchgWordMajor wm;
    XchgSlot slot[2][kLeafMaxG];
};

// Word addresses in the exchange area for a leaf whose values take K words.
template <int K> struct Xchg;
template <> struct Xchg<1> {
    __device__ static uint64_t *head(PanelSync *ps, int par, int k, int g) { return &ps->wm.head[par][k][g]; }
    __device__ static uint64_t *row(PanelSync *ps, int par, int q, int g) { return &ps->wm.row[par][q][g]; }
    __device__ static uint64_t *diag(PanelSync *ps, int par, int q) { return &ps->wm.diag[par][q]; }
};
template <> struct Xchg<2> {
    __device__ static uint64_t *head(PanelSync *ps, int par, int k, int g) { return &ps->slot[par][g].head[k]; }
    __device__ static uint64_t *row(PanelSync *ps, int par, int q, int g) { return &ps->slot[par][g].row[q]; }
    __device__ static uint64_t *diag(PanelSync *ps, int par, int q) { return &ps->slot[par][0].diag[q]; }
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

// Values of type W as 32-bit parts (1 for float, 2 for double).
template <typename W> struct Words;
template <> struct Words<float> {
    static constexpr int K = 1;
    __device__ static uint32_t part(float v, int) { return __float_as_uint(v); }
    __device__ static float from(uint32_t lo, uint32_t) { return __uint_as_float(lo); }
    __device__ static float get(const uint32_t *w, int c) { return __uint_as_float(w[c]); }
    __device__ static void put(uint32_t *w, int c, float v) { w[c] = __float_as_uint(v); }
};
template <> struct Words<double> {
    static constexpr int K = 2;
    __device__ static uint32_t part(double v, int q) {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        return q == 0 ? (uint32_t)b : (uint32_t)(b >> 32);
    }
    __device__ static double from(uint32_t lo, uint32_t hi) {
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    }
    __device__ static double get(const uint32_t *w, int c) {
        const uint2 x = reinterpret_cast<const uint2 *>(w)[c];
        return from(x.x, x.y);
    }
    __device__ static void put(uint32_t *w, int c, double v) {
        reinterpret_cast<uint2 *>(w)[c] = make_uint2(part(v, 0), part(v, 1));
    }
};

// Pivot candidate: larger |value| wins, then the smaller row (the first
// maximum).  Binary32: one 64-bit key, |v| bits above the complemented row
// (|v| >= 0 orders as its bits).  Binary64: the |v| bits and the row.
template <typename W> struct Cand;
template <> struct Cand<float> {
    uint64_t key;
    __device__ static Cand none() { return {0ull}; }
    __device__ static Cand make(float v, int row) {
        return {((uint64_t)__float_as_uint(fabsf(v)) << 32) | (uint64_t)(0xffffffffu - (uint32_t)row)};
    }
    __device__ bool valid() const { return key != 0ull; }
    __device__ int row() const { return (int)(0xffffffffu - (uint32_t)key); }
    __device__ uint64_t vbits() const { return key >> 32; }
    __device__ static Cand from_words(uint64_t vb, int row) { return {(vb << 32) | (uint64_t)(0xffffffffu - (uint32_t)row)}; }
    __device__ void take_max(const Cand &o) { key = o.key > key ? o.key : key; }
};
template <> struct Cand<double> {
    uint64_t vb;
    int r;
    __device__ static Cand none() { return {0ull, 0x7fffffff}; }
    __device__ static Cand make(double v, int row) {
        return {(uint64_t)__double_as_longlong(fabs(v)), row};
    }
    __device__ bool valid() const { return r != 0x7fffffff; }
    __device__ int row() const { return r; }
    __device__ uint64_t vbits() const { return vb; }
    __device__ static Cand from_words(uint64_t b, int row) { return {b, row}; }
    __device__ void take_max(const Cand &o) {
        if (o.vb > vb || (o.vb == vb && o.r < r)) { vb = o.vb; r = o.r; }
    }
};

// Wave maximum of a pivot candidate by DPP: within rows of 16 lanes by
// shifts of 1, 2, 4, 8, then across rows by the row broadcasts of lanes 15
// and 31; lane 63 ends with the maximum, which readlane makes uniform.
// Lanes a shift moves no value into take the identity (old operand).
template <int CTRL, int RM>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ void dpp_max_step(Cand<float> &c) {
    const uint32_t lo = (uint32_t)c.key, hi = (uint32_t)(c.key >> 32);
    const uint32_t tlo = dpp_mov<CTRL, RM>(0u, lo), thi = dpp_mov<CTRL, RM>(0u, hi);
    const uint64_t t = ((uint64_t)thi << 32) | tlo;
    c.key = t > c.key ? t : c.key;
}
template <int CTRL, int RM>
__device__ __forceinline__ void dpp_max_step(Cand<double> &c) {
    const uint32_t lo = (uint32_t)c.vb, hi = (uint32_t)(c.vb >> 32);
    const uint32_t tlo = dpp_mov<CTRL, RM>(0u, lo), thi = dpp_mov<CTRL, RM>(0u, hi);
    const int tr = (int)dpp_mov<CTRL, RM>(0x7fffffffu, (uint32_t)c.r);
    c.take_max(Cand<double>{((uint64_t)thi << 32) | tlo, tr});
}
__device__ __forceinline__ Cand<float> lane63(const Cand<float> &c) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)c.key, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(c.key >> 32), 63);
    return {((uint64_t)hi << 32) | lo};
}
__device__ __forceinline__ Cand<double> lane63(const Cand<double> &c) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)c.vb, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(c.vb >> 32), 63);
    return {((uint64_t)hi << 32) | lo, __builtin_amdgcn_readlane(c.r, 63)};
}
template <typename Cd>
__device__ __forceinline__ Cd wave_max(Cd c) {
    dpp_max_step<0x111, 0xf>(c);   // row_shr:1
    dpp_max_step<0x112, 0xf>(c);   // row_shr:2
    dpp_max_step<0x114, 0xf>(c);   // row_shr:4
    dpp_max_step<0x118, 0xf>(c);   // row_shr:8
    dpp_max_step<0x142, 0xa>(c);   // row_bcast:15 into rows 1 and 3
    dpp_max_step<0x143, 0xc>(c);   // row_bcast:31 into rows 2 and 3
    return lane63(c);
}

// Leaf factorization of rows [k0, n) x columns [k0, k0+w) of the working
// array.  Workgroup g owns relative rows [g*R, g*R+R) (R = 512 RT, RT rows
// per thread), thread t rows g*R + t (+ 512), the 32 leaf entries of each in
// registers.
// The registers rotate: before column j, R[c] holds column j+c for
// c < 32-j and the finished column c-(32-j) above; each column shifts them
// left by one as it updates, so the column loop is not unrolled and every
// register index is static.  Per column: argmax (first maximum) in the
// wave, then over the waves; the best row of each workgroup is posted with
// the old row j in one slot of epoch-tagged words; every workgroup reads
// every slot in one round trip and picks the same winner; swap; scale;
// rank-1 update.  F16 / BF16: the pivot row is rounded to TF when it becomes
// the pivot row, each multiplier to binary16 when formed (products of
// binary16 numbers are exact in binary32).
// Binary32 leaves with one row per thread fit in 128 registers per lane,
// which leaves room on a compute unit for four workgroups of the capped
// trailing update beside the leaf's.
template <typename W, int RT> constexpr int leaf_min_waves() { return sizeof(W) == 4 && RT == 1 ? 4 : 2; }

template <typename W, int RD, int RT>
__global__ __launch_bounds__(kLeafNT, (leaf_min_waves<W, RT>())) void k_leaf(W *__restrict__ a, int64_t n, int64_t ld,
                                                  int64_t k0, int w, int G,
                                                  int32_t *__restrict__ ipiv, int64_t *info,
                                                  PanelSync *ps, uint32_t base, uint32_t *flags) {
    using Wd = Words<W>;
    using Cd = Cand<W>;
    constexpr int K = Wd::K;
    using Xc = Xchg<K>;
    constexpr int C = kLeafMaxW;
    constexpr int NWV = kLeafNT / 64;
    __shared__ Cd red[NWV];
    // rows in LDS as 32-bit words (value c in words K c .. K c + K-1)
    __shared__ __align__(16) uint32_t crow[C * K];   // this workgroup's candidate row (rotated)
    __shared__ __align__(16) uint32_t prow[C * K];   // pivot row (rotated; F16/BF16: current part rounded)
    __shared__ __align__(16) uint32_t pupd[C * K];   // pivot row with the finished part zeroed
    __shared__ __align__(16) uint32_t orow[C * K];   // old row j
    __shared__ int s_p, s_bad;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t m = n - k0;
    constexpr int kLeafRT = RT;
    const int64_t r0 = (int64_t)blockIdx.x * (kLeafNT * RT);
    // an earlier launch already timed out: every workgroup returns at once
    if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & DF_TIMEOUT) return;
    if (tid == 0) s_bad = 0;

    W v[kLeafRT][C];
    int rr[kLeafRT];
    bool mine[kLeafRT];
#pragma unroll
    for (int q = 0; q < kLeafRT; ++q) {
        rr[q] = (int)r0 + tid + q * kLeafNT;
        mine[q] = rr[q] < m;
#pragma unroll
        for (int c = 0; c < C; ++c) v[q][c] = (W)0;
        if (mine[q]) {
            const W *src = a + (k0 + rr[q]) * ld + k0;
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c < w) v[q][c] = src[c];
        }
    }
    __syncthreads();

#pragma unroll 1
    for (int j = 0; j < w; ++j) {
        const uint32_t epoch = base + (uint32_t)j + 1u;
        const int par = j & 1;
        const int cur = C - j;             // rotated positions [0, cur) are current
        // ---- argmax over the workgroup's rows r >= j ----
        Cd best = Cd::none();
#pragma unroll
        for (int q = 0; q < kLeafRT; ++q)
            if (mine[q] && rr[q] >= j) best.take_max(Cd::make(v[q][0], rr[q]));
        best = wave_max(best);
        if (lane == 0) red[wv] = best;
        __syncthreads();                                   // (A)
        best = red[0];
#pragma unroll
        for (int q = 1; q < NWV; ++q) best.take_max(red[q]);
        const int bi = best.row();
        if (G == 1) {
#pragma unroll
            for (int q = 0; q < kLeafRT; ++q) {
                if (mine[q] && rr[q] == bi) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const W x = (RD && c < cur) ? (W)round_lo<RD>((float)v[q][c]) : v[q][c];
                        Wd::put(prow, c, x);
                        Wd::put(pupd, c, c < cur ? x : (W)0);
                    }
                }
                if (mine[q] && rr[q] == j) {
#pragma unroll
                    for (int c = 0; c < C; ++c) Wd::put(orow, c, v[q][c]);
                }
            }
            if (tid == 0) s_p = bi;
            __syncthreads();                               // (B)
        } else {
#pragma unroll
            for (int q = 0; q < kLeafRT; ++q) {
                if (mine[q] && rr[q] == bi) {
#pragma unroll
                    for (int c = 0; c < C; ++c) Wd::put(crow, c, v[q][c]);
                }
                if (mine[q] && rr[q] == j) {
#pragma unroll
                    for (int c = 0; c < C; ++c) Wd::put(orow, c, v[q][c]);
                }
            }
            __syncthreads();                               // (B)
            // Waves 0 .. K-1 each move 32 of the 32*K words of a row: wave
            // wv posts and reads words [32 wv, 32 wv + 32) of every slot
            // (value c lives in words K c .. K c + K-1, low word first).
            if (wv < K) {
                const int g = blockIdx.x;
                const bool own_j = blockIdx.x == 0;        // relative row j < 32 <= R
                const int wb0 = __builtin_amdgcn_readfirstlane(wv) * 32;   // wave-uniform: scalar base addresses
                const uint32_t *cw = crow;
                const uint32_t *ow = orow;
                if (lane < 32) {
                    put_word(Xc::row(ps, par, wb0 + lane, g), cw[wb0 + lane], epoch);
                    if (own_j) put_word(Xc::diag(ps, par, wb0 + lane), ow[wb0 + lane], epoch);
                }
                if (wv == 0 && lane == 32) {
                    const uint64_t vb = best.vbits();
                    put_word(Xc::head(ps, par, 0, g), (uint32_t)vb, epoch);
                    put_word(Xc::head(ps, par, 1, g), (uint32_t)(vb >> 32), epoch);
                    put_word(Xc::head(ps, par, 2, g), (uint32_t)(best.valid() ? bi : 0x7fffffff), epoch);
                }
                // ---- every header (lane g <-> workgroup g) and the old row
                // j, polled with one round trip per poll; then the winner's
                // row only (word wb0 + q from lane q) ----
                uint32_t dw = 0;
                const int gl = lane < G ? lane : 0;
                bool okh = lane >= G, okd = own_j || lane >= 32;
                uint64_t h0 = 0, h1 = 0, h2 = 0, d = 0;
                uint64_t spins = 0;
                for (;;) {
                    if (!okh) {
                        h0 = get_word(Xc::head(ps, par, 0, gl));
                        h1 = get_word(Xc::head(ps, par, 1, gl));
                        h2 = get_word(Xc::head(ps, par, 2, gl));
                    }
                    if (!okd) d = get_word(Xc::diag(ps, par, wb0 + (lane & 31)));
                    okh = okh || (word_ok(h0, epoch) && word_ok(h1, epoch) && word_ok(h2, epoch));
                    okd = okd || word_ok(d, epoch);
                    if (__all(okh && okd)) break;
                    if (++spins > kSpinLimit) { if (lane == 0) s_bad = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
                dw = (uint32_t)d;
                Cd gbest = Cd::none();
                if (lane < G && okh) {
                    const int hr = (int)(uint32_t)h2;
                    if (hr != 0x7fffffff)
                        gbest = Cd::from_words(((uint64_t)(uint32_t)h1 << 32) | (uint32_t)h0, hr);
                }
                const Cd wbst = wave_max(gbest);
                const int p = wbst.row();
                const uint64_t wmask = __ballot(lane < G && gbest.valid() && gbest.row() == p);
                if (wmask != 0ull) {
                    const int gw = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)wmask) - 1);
                    uint64_t x = 0;
                    bool okx = lane >= 32;
                    for (;;) {
                        if (!okx) x = get_word(Xc::row(ps, par, wb0 + (lane & 31), gw));
                        okx = okx || word_ok(x, epoch);
                        if (__all(okx)) break;
                        if (++spins > kSpinLimit) { if (lane == 0) s_bad = 1; break; }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (lane < 32) {
                        const int c = (wb0 + lane) / K;
                        uint32_t xw = (uint32_t)x;
                        if (RD && c < cur) xw = __float_as_uint(round_lo<RD>(__uint_as_float(xw)));
                        prow[wb0 + lane] = xw;
                        pupd[wb0 + lane] = c < cur ? xw : 0u;
                    }
                }
                if (!own_j && lane < 32) orow[wb0 + lane] = dw;
                if (wv == 0 && lane == 0) s_p = p;
            }
            __syncthreads();                               // (C)
        }
        const int p = s_p;
        if (s_bad || p == 0x7fffffff) {
            if (tid == 0) atomicOr(flags, (uint32_t)DF_TIMEOUT);
            break;
        }
        // ---- swap rows j and p, record the pivot ----
#pragma unroll
        for (int q = 0; q < kLeafRT; ++q) {
            if (mine[q] && p != j && rr[q] == p) {
#pragma unroll
                for (int c = 0; c < C; ++c) v[q][c] = Wd::get(orow, c);
            }
            if (mine[q] && rr[q] == j) {
#pragma unroll
                for (int c = 0; c < C; ++c) v[q][c] = Wd::get(prow, c);
            }
        }
        const W piv = Wd::get(prow, 0);
        if (blockIdx.x == 0 && tid == 0) {
            ipiv[k0 + j] = (int32_t)(k0 + p);
            if (piv == (W)0 && *info == 0) *info = k0 + j + 1;
        }
        // ---- scale, rank-1 update and rotate by one ----
        // (with a zero pivot the column below it is zero: no update)
#pragma unroll
        for (int q = 0; q < kLeafRT; ++q) {
            if (rr[q] > j && piv != (W)0) {
                W l = v[q][0] / piv;
                if (RD) l = (W)round_lo<RD>((float)l);
#pragma unroll
                for (int c = 0; c < C - 1; ++c) {
                    const W prod = l * Wd::get(pupd, c + 1);
                    v[q][c] = v[q][c + 1] - prod;
                }
                v[q][C - 1] = l;
            } else {
                const W x0 = v[q][0];
#pragma unroll
                for (int c = 0; c < C - 1; ++c) v[q][c] = v[q][c + 1];
                v[q][C - 1] = x0;
            }
        }
        (void)cur;
        // red/crow/prow/pupd/orow are rewritten only after the next (A),
        // which every thread reaches after its reads here.
    }
    // w < 32: rotate the remaining 32 - w places so that v[c] is column c
#pragma unroll 1
    for (int t = w; t < C; ++t) {
#pragma unroll
        for (int q = 0; q < kLeafRT; ++q) {
            const W x0 = v[q][0];
#pragma unroll
            for (int c = 0; c < C - 1; ++c) v[q][c] = v[q][c + 1];
            v[q][C - 1] = x0;
        }
    }
#pragma unroll
    for (int q = 0; q < kLeafRT; ++q) {
        if (mine[q]) {
            W *dst = a + (k0 + rr[q]) * ld + k0;
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c < w) dst[c] = v[q][c];
        }
    }
}

// Row interchanges ipiv[k0 .. k0+cnt) applied, in order, to the columns
// [c0,c1) U [c2,c3).  The composed permutation only moves the rows
// P = [k0, k0+cnt) U {ipiv targets}; the source of each destination row is
// found by applying the transpositions in reverse order, so every thread
// computes its own pair without a sequential pass.  The tile of moved rows
// is staged in LDS (all reads before any write).  The last workgroup also
// permutes `perm` (the row permutation used by the solves).
template <typename W, int CB, int TR>
__global__ __launch_bounds__(256) void k_laswp(W *__restrict__ a, int64_t ld, int64_t k0, int cnt,
                                               const int32_t *__restrict__ ipiv, int64_t c0,
                                               int64_t c1, int64_t c2, int64_t c3,
                                               int32_t *__restrict__ perm, int ncolblk) {
    __shared__ W tile[TR * CB];                         // [2*cnt <= TR][CB]
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

// U12 <- L11^{-1} U12 for rows [k, k+w), w <= 32, columns [c0, c1): one
// thread per column, L11 in LDS, the w entries of the column in registers,
// no barrier inside the substitution.  Right-looking: row t is final at step
// t (F16 / BF16: rounded to TF then) and updates the rows below it.
template <typename W, int RD>
__global__ __launch_bounds__(256) void k_trsm_col(W *__restrict__ a, int64_t ld, int64_t k, int w,
                                                  int64_t c0, int64_t c1) {
    __shared__ W L[32][33];
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += 256) {
        const int r = e / w, c = e - r * w;
        L[r][c] = a[(k + r) * ld + k + c];
    }
    __syncthreads();
    const int64_t c = c0 + (int64_t)blockIdx.x * 256 + tid;
    if (c >= c1) return;
    W x[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) x[t] = t < w ? a[(k + t) * ld + c] : (W)0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        if (t < w) {
            if (RD) x[t] = (W)round_lo<RD>((float)x[t]);
#pragma unroll
            for (int s2 = t + 1; s2 < 32; ++s2) {
                const W prod = L[s2][t] * x[t];
                x[s2] = x[s2] - prod;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 32; ++t)
        if (t < w) a[(k + t) * ld + c] = x[t];
}

// U12 <- L11^{-1} U12 for a whole panel in one launch, for a narrow column
// range (the look-ahead panel): rows [k, k+w) (w <= kU12MaxW), columns
// [c0, c1).  A workgroup owns kU12CW columns and keeps their w rows in LDS
// for the whole solve.  Blocks of 32 rows, in increasing order: (a) the
// diagonal block by substitution in registers, one wave per two columns
// (lane = row; the final entry of row t is broadcast by readlane; F16 /
// BF16: rounded to TF when final, before it updates later rows); (b) every
// row below, by one thread, subtracting the block's 32 products in
// increasing order.  The L entries each phase needs are loaded while the
// other phase runs.  Each entry thus receives its updates in increasing k,
// as in the column-by-column substitution, with one launch instead of a
// triangular solve and an update per 32 rows.
constexpr int kU12MaxW = 512;
constexpr int kU12CW = 8;          // columns per workgroup (two per solving wave)
constexpr int kU12NT = 512;        // threads: one per row below a block

template <typename W> __device__ __forceinline__ W bcast_lane(W x, int l);
template <> __device__ __forceinline__ float bcast_lane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
template <> __device__ __forceinline__ double bcast_lane(double x, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <typename W, int RD>
__global__ __launch_bounds__(kU12NT) void k_u12(W *__restrict__ a, int64_t ld, int64_t k, int w,
                                                int64_t c0, int64_t c1) {
    __shared__ __align__(16) W X[kU12MaxW][kU12CW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t cb = c0 + (int64_t)blockIdx.x * kU12CW;
    const int ncol = (int)((c1 - cb) < kU12CW ? (c1 - cb) : kU12CW);
    for (int e = tid; e < w * kU12CW; e += kU12NT) {
        const int r = e / kU12CW, c = e - r * kU12CW;
        X[r][c] = c < ncol ? a[(k + r) * ld + cb + c] : (W)0;
    }
    // waves 0-3 solve the diagonal blocks: lane = (column half, row s); the
    // block's L row of each lane is loaded one block ahead
    const bool solver = wv < kU12CW / 2;
    const int s = lane & 31, cc = 2 * wv + (lane >> 5);
    W lr[32];
    auto load_lr = [&](int r0) {
        const int hb = (w - r0) < 32 ? (w - r0) : 32;
        const W *lp = a + (k + r0 + s) * ld + k + r0;
#pragma unroll
        for (int t = 0; t < 32; ++t) lr[t] = (solver && s < hb && t < s) ? lp[t] : (W)0;
    };
    load_lr(0);
    __syncthreads();
    for (int r0 = 0; r0 < w; r0 += 32) {
        const int hb = (w - r0) < 32 ? (w - r0) : 32;
        // (b)'s L row (thread = one row below the block), in flight during (a)
        const int r = r0 + 32 + tid;
        W lb[32];
        if (r < w) {
            const W *lp = a + (k + r) * ld + k + r0;
#pragma unroll
            for (int t = 0; t < 32; ++t) lb[t] = lp[t];
        }
        if (solver) {
            // (a) rows r0 + s of column cc
            W x = s < hb ? X[r0 + s][cc] : (W)0;
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                if (t < hb) {
                    if (RD && s == t) x = (W)round_lo<RD>((float)x);
                    const W xa = bcast_lane(x, t), xb = bcast_lane(x, 32 + t);
                    const W xt = (lane >> 5) ? xb : xa;
                    if (s > t) {
                        const W prod = lr[t] * xt;
                        x = x - prod;
                    }
                }
            }
            if (s < hb) X[r0 + s][cc] = x;
        }
        __syncthreads();
        if (r0 + 32 < w) load_lr(r0 + 32);
        // (b) the rows below (the block is full whenever rows follow it)
        if (r < w) {
            W acc[kU12CW];
#pragma unroll
            for (int c = 0; c < kU12CW; ++c) acc[c] = X[r][c];
#pragma unroll
            for (int t = 0; t < 32; ++t) {
#pragma unroll
                for (int c = 0; c < kU12CW; ++c) {
                    const W prod = lb[t] * X[r0 + t][c];
                    acc[c] = acc[c] - prod;
                }
            }
#pragma unroll
            for (int c = 0; c < kU12CW; ++c) X[r][c] = acc[c];
        }
        __syncthreads();
    }
    for (int e = tid; e < w * kU12CW; e += kU12NT) {
        const int r = e / kU12CW, c = e - r * kU12CW;
        if (c < ncol) a[(k + r) * ld + cb + c] = X[r][c];
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

// The leaf is launched as an ordinary kernel on the caller's queue: a
// cooperative launch goes through a queue of its own, which costs a queue
// switch before and after each leaf (about 10 ms per factorization at
// N = 32768).  Every workgroup still becomes resident: at most 64
// workgroups of one compute unit each, and whatever else runs on the device
// meanwhile (the trailing update on the second stream) finishes on its own
// and frees its units; the bounded waits turn anything else into
// MPIR_ERR_DEVICE.  MPIR_LEAF_COOP=1 restores the cooperative launch.
// (read at every launch, so that a process can switch it between calls)
bool leaf_cooperative() {
    const char *e = std::getenv("MPIR_LEAF_COOP");
    return e && e[0] == '1';
}

int leaf_gmax() { return num_cus() < kLeafMaxG ? num_cus() : kLeafMaxG; }

template <typename W, int RD, int RT>
hipError_t leaf_run(W *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv, int64_t *info,
                    PanelSync *ps, uint32_t *host_base, uint32_t *flags, hipStream_t s) {
    const int64_t m = n - k0;
    const int64_t G64 = (m + kLeafNT * RT - 1) / (kLeafNT * RT);
    if (G64 > leaf_gmax()) return hipErrorInvalidValue;
    const int G = (int)G64;
    uint32_t base = *host_base;
    if (G == 1) {
        k_leaf<W, RD, RT><<<1, kLeafNT, 0, s>>>(a, n, ld, k0, w, G, ipiv, info, ps, base, flags);
        return hipGetLastError();
    }
    if (!leaf_cooperative()) {
        k_leaf<W, RD, RT><<<G, kLeafNT, 0, s>>>(a, n, ld, k0, w, G, ipiv, info, ps, base, flags);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) *host_base = base + (uint32_t)w;
        return e;
    }
    void *args[] = {&a, (void *)&n, (void *)&ld, (void *)&k0, (void *)&w, (void *)&G,
                    &ipiv, &info, &ps, &base, &flags};
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_leaf<W, RD, RT>, dim3(G),
                                              dim3(kLeafNT), args, 0, s);
    if (e == hipSuccess) *host_base = base + (uint32_t)w;
    return e;
}

// One row per thread unless the panel fits one workgroup at two (then no
// exchange is needed) or needs more workgroups than may run at once.
template <typename W, int RD>
hipError_t leaf_go(W *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv, int64_t *info,
                   PanelSync *ps, uint32_t *host_base, uint32_t *flags, hipStream_t s) {
    if constexpr (leaf_rt_max<W>() == 2) {
        const int64_t m = n - k0;
        if (m <= 2 * kLeafNT || m > (int64_t)leaf_gmax() * kLeafNT)
            return leaf_run<W, RD, 2>(a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    }
    return leaf_run<W, RD, 1>(a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
}

}  // namespace

int leaf_max_rows(int mode) {
    return leaf_gmax() * kLeafNT * (mode == LU_F64 ? leaf_rt_max<double>() : leaf_rt_max<float>());
}

hipError_t launch_leaf(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int w, int32_t *ipiv,
                       int64_t *info, PanelSync *ps, uint32_t *host_base, uint32_t *flags,
                       hipStream_t s) {
    if (w <= 0 || w > kLeafMaxW || k0 >= n) return hipErrorInvalidValue;
    if (mode == LU_F64)
        return leaf_go<double, 0>((double *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    if (mode == LU_F32)
        return leaf_go<float, 0>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    if (mode == LU_BF16)
        return leaf_go<float, 2>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
    return leaf_go<float, 1>((float *)a, n, ld, k0, w, ipiv, info, ps, host_base, flags, s);
}

hipError_t launch_laswp(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int cnt,
                        const int32_t *ipiv, int64_t c0, int64_t c1, int64_t c2, int64_t c3,
                        int32_t *perm, bool compact, hipStream_t s) {
    (void)n;
    if (cnt <= 0 || cnt > 256) return hipErrorInvalidValue;
    const int64_t wtot = (c1 - c0) + (c3 - c2);
    // compact: 16 KB of LDS, so that the launch fits on a compute unit that
    // a concurrent trailing update already occupies; otherwise 128 KB tiles
    // of long row segments.
    auto go = [&](auto wtag, auto cbtag, auto trtag) {
        using W = decltype(wtag);
        constexpr int CB = decltype(cbtag)::value, TR = decltype(trtag)::value;
        const int nb = (int)((wtot + CB - 1) / CB);
        k_laswp<W, CB, TR><<<nb + 1, 256, 0, s>>>((W *)a, ld, k0, cnt, ipiv, c0, c1, c2, c3, perm, nb);
    };
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    using I512 = std::integral_constant<int, 512>;
    if (mode == LU_F64) {
        if (!compact) go(double(), I32(), I512());
        else if (cnt <= 32) go(double(), I32(), I64());
        else go(double(), I4(), I512());
    } else {
        if (!compact) go(float(), I64(), I512());
        else if (cnt <= 32) go(float(), I64(), I64());
        else go(float(), I8(), I512());
    }
    return hipGetLastError();
}

hipError_t launch_trsm(int mode, void *a, int64_t ld, int64_t k, int w, int64_t c0, int64_t c1,
                       hipStream_t s) {
    if (w <= 0 || w > 32 || c1 <= c0) return w <= 0 || w > 32 ? hipErrorInvalidValue : hipSuccess;
    const unsigned nb = (unsigned)((c1 - c0 + 255) / 256);
    if (mode == LU_F64) k_trsm_col<double, 0><<<nb, 256, 0, s>>>((double *)a, ld, k, w, c0, c1);
    else if (mode == LU_F32) k_trsm_col<float, 0><<<nb, 256, 0, s>>>((float *)a, ld, k, w, c0, c1);
    else if (mode == LU_BF16) k_trsm_col<float, 2><<<nb, 256, 0, s>>>((float *)a, ld, k, w, c0, c1);
    else k_trsm_col<float, 1><<<nb, 256, 0, s>>>((float *)a, ld, k, w, c0, c1);
    return hipGetLastError();
}

int u12_max_rows() { return kU12MaxW; }

hipError_t launch_u12(int mode, void *a, int64_t ld, int64_t k, int w, int64_t c0, int64_t c1,
                      hipStream_t s) {
    if (w <= 0 || w > kU12MaxW) return hipErrorInvalidValue;
    if (c1 <= c0) return hipSuccess;
    const unsigned nb = (unsigned)((c1 - c0 + kU12CW - 1) / kU12CW);
    if (mode == LU_F64) k_u12<double, 0><<<nb, kU12NT, 0, s>>>((double *)a, ld, k, w, c0, c1);
    else if (mode == LU_F32) k_u12<float, 0><<<nb, kU12NT, 0, s>>>((float *)a, ld, k, w, c0, c1);
    else if (mode == LU_BF16) k_u12<float, 2><<<nb, kU12NT, 0, s>>>((float *)a, ld, k, w, c0, c1);
    else k_u12<float, 1><<<nb, kU12NT, 0, s>>>((float *)a, ld, k, w, c0, c1);
    return hipGetLastError();
}

}  // namespace mpir
