// Trailing-matrix update of the blocked right-looking LU, A22 -= L21 * U12,
// on the MI355X matrix cores (MFMA).  One row-major working array holds all
// three operands: L21 = a[r0:r0+m, k:k+kk], U12 = a[k:k+kk, c0:c0+nc],
// A22 = a[r0:r0+m, c0:c0+nc].
//
//   TF = F32 : binary32 operands, v_mfma_f32_32x32x2_f32.
//   TF = F16 : L21 and U12 hold binary16 numbers (stored in the binary32
//              working array); they are staged to LDS as binary16 and
//              multiplied with v_mfma_f32_32x32x16_f16 into binary32
//              accumulators; A22 stays binary32.
//   TF = BF16: as F16 with bfloat16 operands and v_mfma_f32_32x32x16_bf16
//              in the trailing update; inside the panel the binary32 path
//              (products of two bfloat16 numbers are exact in binary32).
//   TF = F64 : binary64, v_mfma_f64_16x16x4_f64 (the FP64 comparator).
//
// Tiling: a workgroup of four wave64s computes a BM x BN tile of C,
// accumulators in registers (the sizes are in Cfg32 / Cfg64 below, chosen by
// timing the trailing update in the factorization: binary32 64 x 64, each
// wave one 32 x 32 block; binary16 operands inside the panel 128 x 64;
// binary64 64 x 64, each wave 2 x 2 blocks of 16 x 16; the packed 16-bit
// trailing update 128 x 128, each wave 2 x 2 blocks of 32 x 32).  K is walked in chunks staged through two LDS buffers: while the
// matrix cores work on chunk i, the global loads of chunk i+1 are in flight
// (16-byte vector loads when every offset is 4-element aligned), so the load
// latency hides behind the MFMA work of a chunk.  Workgroup ids are remapped
// so that each XCD (which has its own L2) receives a contiguous band of
// tiles sharing L21 rows and U12 columns.
#include <type_traits>

#include "mpir_internal.h"

namespace mpir {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 8-element operand vector of a 16-bit type and its 32x32x16 MFMA.
template <typename T16> struct Vec16;
template <> struct Vec16<_Float16> {
    using V8 = half8;
    __device__ static floatx16 mfma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Vec16<__bf16> {
    using V8 = bf16x8;
    __device__ static floatx16 mfma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
typedef double doublex4 __attribute__((ext_vector_type(4)));

// XCD-aware tile order: the dispatcher hands workgroup ids round-robin to
// the 8 XCDs; remap so that XCD x owns the contiguous tile range
// [x*per, (x+1)*per) (tiles ordered row-major over the tile grid).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int NX = 8;
    if (nblk < NX * 4) return bid;
    const int per = nblk / NX;
    const int full = per * NX;
    if (bid >= full) return bid;
    return (bid % NX) * per + bid / NX;
}

// Tile (row, column) of a remapped tile id: bands of GM tile rows, column by
// column inside a band, so the tiles in flight on one XCD (consecutive ids)
// form a GM x (in-flight / GM) block that shares GM row panels of A and a
// few column panels of B in that XCD's L2.
constexpr int kGroupM = 16;
__device__ __forceinline__ void tile_coords(int t, int tiles_m, int tiles_n, int &tr, int &tc) {
    const int band = kGroupM * tiles_n;
    const int g = t / band, r = t - g * band;
    const int rows = (tiles_m - g * kGroupM) < kGroupM ? (tiles_m - g * kGroupM) : kGroupM;
    tr = g * kGroupM + r % rows;
    tc = r / rows;
}

template <bool VEC, int NV>
__device__ __forceinline__ void load_row_f32(float (&dst)[NV], const float *src, bool rowok,
                                             int64_t k0, int64_t klim) {
    // NV consecutive floats from src[k0 ...], zero beyond klim or if !rowok
    if (VEC && rowok && k0 + NV <= klim) {
#pragma unroll
        for (int q = 0; q < NV; q += 4) {
            const floatx4 v = *reinterpret_cast<const floatx4 *>(src + k0 + q);
            dst[q] = v[0]; dst[q + 1] = v[1]; dst[q + 2] = v[2]; dst[q + 3] = v[3];
        }
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[q] = (rowok && k0 + q < klim) ? src[k0 + q] : 0.0f;
    }
}

// ------------------------------------------------- binary32 and binary16
// Workgroup tile BM x BN, K-chunk BK, NBUF LDS buffers, four waves in a 2 x 2
// grid, each wave (BM/2) x (BN/2) of C in 32 x 32 MFMA blocks.
// Global -> register split: A: TPR = 256/BM threads per row, each BK/TPR
// consecutive k; B: TPK = 256/BK threads per k-row, each BN/TPK consecutive
// columns.  Binary32 tiles are stored k-major in LDS (lanes read consecutive
// rows or columns of one k); binary16 tiles row-major for A and transposed
// for B (8 consecutive k per lane, one 16-byte LDS read per operand).
template <bool HALF, bool VEC, int BM, int BN, int BK, int NBUF, int ROLE>
__global__ __launch_bounds__(256) void k_gemm_32(float *__restrict__ a, int64_t ld, int64_t r0,
                                                 int64_t m, int64_t c0, int64_t nc, int64_t k,
                                                 int64_t kk, int tiles_n, int nblk) {
    constexpr int TPR = 256 / BM, AK = BK / TPR;      // A: threads per row, k's per thread
    constexpr int TPK = 256 / BK, BCOL = BN / TPK;    // B: threads per k-row, cols per thread
    constexpr int MI = BM / 64, NJ = BN / 64;         // 32x32 blocks per wave
    static_assert(TPR * BM == 256 && TPK * BK == 256 && AK % 4 == 0 && BCOL % 4 == 0, "split");
    static_assert(!HALF || BK % 16 == 0, "half k-step");
    using T = typename std::conditional<HALF, _Float16, float>::type;
    constexpr int AP = HALF ? BK + 8 : BM + 4;     // pitch of the fast dim
    constexpr int BP = HALF ? BK + 8 : BN + 4;
    constexpr int AS = HALF ? BM * AP : BK * AP;
    constexpr int BS = HALF ? BN * BP : BK * BP;
    __shared__ __align__(16) T As[NBUF][AS];
    __shared__ __align__(16) T Bs[NBUF][BS];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    int trow, tcol;
    tile_coords(bid, nblk / tiles_n, tiles_n, trow, tcol);
    const int64_t tm = (int64_t)trow * BM, tn = (int64_t)tcol * BN;
    const int wm = (wv >> 1) * (BM / 2), wn = (wv & 1) * (BN / 2);

    const int arow = tid / TPR, ak0 = (tid % TPR) * AK;
    const bool arow_ok = tm + arow < m;
    const float *ap = a + (r0 + tm + arow) * ld + k + ak0;
    const int bk = tid / TPK, bc0 = (tid % TPK) * BCOL;
    const float *bp = a + k * ld + c0 + tn + bc0;
    const int64_t bcol_lim = nc - (tn + bc0);     // valid columns from bc0

    float ra[AK], rb[BCOL];
    auto load = [&](int64_t kc) {
        load_row_f32<VEC, AK>(ra, ap, arow_ok, kc, kk - ak0);
        const int64_t kr = kc + bk;
        const bool kok = kr < kk;
        if (VEC && kok && bcol_lim >= BCOL) {
#pragma unroll
            for (int q = 0; q < BCOL; q += 4) {
                const floatx4 v = *reinterpret_cast<const floatx4 *>(bp + kr * ld + q);
                rb[q] = v[0]; rb[q + 1] = v[1]; rb[q + 2] = v[2]; rb[q + 3] = v[3];
            }
        } else {
#pragma unroll
            for (int q = 0; q < BCOL; ++q) rb[q] = (kok && q < bcol_lim) ? bp[kr * ld + q] : 0.0f;
        }
    };
    auto store = [&](int buf) {
        if constexpr (HALF) {
#pragma unroll
            for (int q = 0; q < AK; q += 4) {
                half4 h;
                h[0] = (_Float16)ra[q]; h[1] = (_Float16)ra[q + 1];
                h[2] = (_Float16)ra[q + 2]; h[3] = (_Float16)ra[q + 3];
                *reinterpret_cast<half4 *>(&As[buf][arow * AP + ak0 + q]) = h;
            }
#pragma unroll
            for (int q = 0; q < BCOL; ++q) Bs[buf][(bc0 + q) * BP + bk] = (_Float16)rb[q];
        } else {
#pragma unroll
            for (int q = 0; q < AK; ++q) As[buf][(ak0 + q) * AP + arow] = ra[q];
#pragma unroll
            for (int q = 0; q < BCOL; q += 4) {
                floatx4 v;
                v[0] = rb[q]; v[1] = rb[q + 1]; v[2] = rb[q + 2]; v[3] = rb[q + 3];
                *reinterpret_cast<floatx4 *>(&Bs[buf][bk * BP + bc0 + q]) = v;
            }
        }
    };

    floatx16 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = floatx16{0};

    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t kc = 0; kc < kk; kc += BK) {
        const bool more = kc + BK < kk;
        if (more) load(kc + BK);
        if constexpr (HALF) {
#pragma unroll
            for (int s = 0; s < BK; s += 16) {
                const int kb = s + 8 * (lane >> 5);
                half8 af[MI], bf[NJ];
#pragma unroll
                for (int i = 0; i < MI; ++i)
                    af[i] = *reinterpret_cast<const half8 *>(&As[buf][(wm + i * 32 + (lane & 31)) * AP + kb]);
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    bf[j] = *reinterpret_cast<const half8 *>(&Bs[buf][(wn + j * 32 + (lane & 31)) * BP + kb]);
#pragma unroll
                for (int i = 0; i < MI; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < BK; s += 2) {
                const int kr = s + (lane >> 5);
                float af[MI], bf[NJ];
#pragma unroll
                for (int i = 0; i < MI; ++i) af[i] = As[buf][kr * AP + wm + i * 32 + (lane & 31)];
#pragma unroll
                for (int j = 0; j < NJ; ++j) bf[j] = Bs[buf][kr * BP + wn + j * 32 + (lane & 31)];
#pragma unroll
                for (int i = 0; i < MI; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
        }
        if (more) {
            if constexpr (NBUF == 1) __syncthreads();
            store(NBUF == 1 ? 0 : buf ^ 1);
        }
        __syncthreads();
        if constexpr (NBUF == 2) buf ^= 1;
    }
    // epilogue: lane l, register v -> row 8*(v/4) + 4*(l/32) + v%4, col l%32.
    // Binary16 operands (the panel's updates of TF = F16): every C load of a
    // block is issued before the first store (FP16 factorization 258 ->
    // 248 ms at N = 32768).  Binary32 trailing update (role 0): c + (-acc)
    // by a no-return atomic add, carried out in the memory system beyond the
    // L2, which rounds as the subtraction does (IEEE, subnormals kept) and
    // leaves no load round trip in the wave (FP32 factorization about 1.5%
    // faster at N = 32768); every C element is added to once per launch,
    // and no other kernel touches those columns meanwhile.  Binary32
    // in-panel updates (role 1): one element at a time -- the batched form
    // raised the registers and cost the FP32 factorization 25% (350
    // against 443 ms), the atomic form slowed the panel stream.
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int64_t col = tn + wn + j * 32 + (lane & 31);
            if constexpr (HALF) {
                float cv[16];
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    cv[v] = (row < m && col < nc) ? a[(r0 + row) * ld + c0 + col] : 0.0f;
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    if (row < m && col < nc) a[(r0 + row) * ld + c0 + col] = cv[v] - acc[i][j][v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    if (row < m && col < nc) {
                        float *p = a + (r0 + row) * ld + c0 + col;
                        if constexpr (ROLE == 0)
                            __hip_atomic_fetch_add(p, -acc[i][j][v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else
                            *p = *p - acc[i][j][v];
                    }
                }
            }
        }
}

// --------------------------------------- 16-bit operands packed per step
// For TF = F16 (BF16), L21 and U12 hold binary16 (bfloat16) numbers in the
// binary32 working array.  They are packed once per update into 16-bit
// copies (the conversion is exact) with k
// contiguous (A as m x kp, B transposed as n x kp; kp = kk rounded up to 32,
// rows padded to 128, the padding zero), so the update reads half the bytes
// with 16-byte loads that land directly in the MFMA operand layout.
constexpr int kHT = 128;     // tile edge of the packed-operand update
constexpr int kHK = 32;      // k per LDS stage

template <typename T16>
__global__ __launch_bounds__(256) void k_pack_rows_h(const float *__restrict__ a, int64_t ld,
                                                     int64_t r0, int64_t m, int64_t mp, int64_t k,
                                                     int64_t kk, int64_t kp, T16 *__restrict__ out) {
    // out[i][t] = a[r0 + i][k + t] (i < m, t < kk), zero padding
    using V8 = typename Vec16<T16>::V8;
    const int64_t tot = mp * (kp / 8);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / (kp / 8), t0 = (e - i * (kp / 8)) * 8;
        V8 h;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            h[q] = (T16)((i < m && t0 + q < kk) ? a[(r0 + i) * ld + k + t0 + q] : 0.0f);
        *reinterpret_cast<V8 *>(out + i * kp + t0) = h;
    }
}

template <typename T16>
__global__ __launch_bounds__(256) void k_pack_cols_h(const float *__restrict__ a, int64_t ld,
                                                     int64_t k, int64_t kk, int64_t kp, int64_t c0,
                                                     int64_t nc, int64_t np_, T16 *__restrict__ out) {
    using V8 = typename Vec16<T16>::V8;
    // out[j][t] = a[k + t][c0 + j] (j < nc, t < kk), zero padding; 64 x 64
    // tiles transposed through LDS
    __shared__ float tl[64][65];
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64, t0 = (int64_t)blockIdx.y * 64;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int tt = e / 64, jj = e % 64;
        const int64_t t = t0 + tt, j = j0 + jj;
        tl[tt][jj] = (t < kk && j < nc) ? a[(k + t) * ld + c0 + j] : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 8; e += 256) {
        const int jj = e / 8, tq = (e % 8) * 8;
        const int64_t j = j0 + jj, t = t0 + tq;
        if (j < np_ && t < kp) {
            V8 h;
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] = (T16)tl[tq + q][jj];
            *reinterpret_cast<V8 *>(out + j * kp + t) = h;
        }
    }
}

// C[r0 + i][c0 + j] -= sum_t Ah[i][t] Bt[j][t]: four waves in a 2 x 2 grid,
// each (32 WM) x (32 WN) of C in WM x WN blocks of the 32x32x16 MFMA of T16
// (a wave reads WM + WN 16-byte operand vectors from LDS per WM * WN
// products), double-buffered LDS stages of BK k, binary32 accumulators.
// The C tile's read-modify-write issues every load of a block row before
// its first store (one C element at a time made each load wait for the
// previous store: 186 against 263 TFLOP/s in the factorization).  Measured
// at N = 32768: WM = WN = 2 with two workgroups per SIMD-set is fastest;
// 4 x 2 and 2 x 4 per wave (one workgroup) reach 165-177 TFLOP/s.
template <typename T16, int WM, int WN, int BK, int MINB>
__global__ __launch_bounds__(256, MINB) void k_gemm_h16(float *__restrict__ a, int64_t ld, int64_t r0,
                                                        int64_t m, int64_t c0, int64_t nc,
                                                        const T16 *__restrict__ Ah,
                                                        const T16 *__restrict__ Bt, int64_t kp,
                                                        int tiles_n, int nblk) {
    using V8 = typename Vec16<T16>::V8;
    constexpr int TM = 64 * WM, TN = 64 * WN;         // workgroup tile
    constexpr int P = BK + 8;                         // LDS pitch (16-bit elements)
    constexpr int TPA = 256 / TM, TPB = 256 / TN;     // threads per row of A / of B
    constexpr int NVA = BK / 8 / TPA, NVB = BK / 8 / TPB;   // 8-element vectors per thread
    static_assert(TPA >= 1 && TPB >= 1 && NVA >= 1 && NVB >= 1 && TPA * TM == 256 && TPB * TN == 256,
                  "load split");
    __shared__ __align__(16) T16 As[2][TM * P];
    __shared__ __align__(16) T16 Bs[2][TN * P];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    int trow, tcol;
    tile_coords(bid, nblk / tiles_n, tiles_n, trow, tcol);
    const int64_t tm = (int64_t)trow * TM, tn = (int64_t)tcol * TN;
    const int wm = (wv >> 1) * (32 * WM), wn = (wv & 1) * (32 * WN);
    const int la = tid / TPA, lka = (tid % TPA) * (BK / TPA);
    const int lb = tid / TPB, lkb = (tid % TPB) * (BK / TPB);
    const T16 *ap = Ah + (tm + la) * kp + lka;
    const T16 *bp = Bt + (tn + lb) * kp + lkb;
    V8 ra[NVA], rb[NVB];
    auto load = [&](int64_t kc) {
#pragma unroll
        for (int q = 0; q < NVA; ++q) ra[q] = *reinterpret_cast<const V8 *>(ap + kc + 8 * q);
#pragma unroll
        for (int q = 0; q < NVB; ++q) rb[q] = *reinterpret_cast<const V8 *>(bp + kc + 8 * q);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NVA; ++q) *reinterpret_cast<V8 *>(&As[buf][la * P + lka + 8 * q]) = ra[q];
#pragma unroll
        for (int q = 0; q < NVB; ++q) *reinterpret_cast<V8 *>(&Bs[buf][lb * P + lkb + 8 * q]) = rb[q];
    };
    floatx16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = floatx16{0};
    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t kc = 0; kc < kp; kc += BK) {
        const bool more = kc + BK < kp;
        if (more) load(kc + BK);
#pragma unroll
        for (int s2 = 0; s2 < BK; s2 += 16) {
            const int kb = s2 + 8 * (lane >> 5);
            V8 af[WM], bf[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                af[i] = *reinterpret_cast<const V8 *>(&As[buf][(wm + i * 32 + (lane & 31)) * P + kb]);
#pragma unroll
            for (int j = 0; j < WN; ++j)
                bf[j] = *reinterpret_cast<const V8 *>(&Bs[buf][(wn + j * 32 + (lane & 31)) * P + kb]);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = Vec16<T16>::mfma(af[i], bf[j], acc[i][j]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // epilogue: lane l, register v -> row 8*(v/4) + 4*(l/32) + v%4, col l%32;
    // per block row i all WN*16 loads first, then the subtractions and stores
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        float cv[WN][16];
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t col = tn + wn + j * 32 + (lane & 31);
                cv[j][v] = (row < m && col < nc) ? a[(r0 + row) * ld + c0 + col] : 0.0f;
            }
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t col = tn + wn + j * 32 + (lane & 31);
                if (row < m && col < nc) a[(r0 + row) * ld + c0 + col] = cv[j][v] - acc[i][j][v];
            }
    }
}

// ---------------------------------------------------------------- binary64
// Workgroup tile BM x BN, K-chunk BK, two LDS buffers, four waves in a 2 x 2
// grid, each wave (BM/2) x (BN/2) of C in 16 x 16 MFMA blocks.  A: TPR =
// 256/BM threads per row, each BK/TPR consecutive k; B: TPK = 256/BK threads
// per k-row, each BN/TPK consecutive columns.
template <bool VEC, int BM, int BN, int BK, int ROLE>
__global__ __launch_bounds__(256) void k_gemm_f64(double *__restrict__ a, int64_t ld, int64_t r0,
                                                  int64_t m, int64_t c0, int64_t nc, int64_t k,
                                                  int64_t kk, int tiles_n, int nblk) {
    constexpr int TPR = 256 / BM, AK = BK / TPR;
    constexpr int TPK = 256 / BK, BCOL = BN / TPK;
    constexpr int MI = BM / 32, NJ = BN / 32;
    static_assert(TPR * BM == 256 && TPK * BK == 256 && AK % 2 == 0 && BCOL % 2 == 0, "split");
    __shared__ __align__(16) double As[2][BK][BM + 2];
    __shared__ __align__(16) double Bs[2][BK][BN + 2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    int trow, tcol;
    tile_coords(bid, nblk / tiles_n, tiles_n, trow, tcol);
    const int64_t tm = (int64_t)trow * BM, tn = (int64_t)tcol * BN;
    const int wm = (wv >> 1) * (BM / 2), wn = (wv & 1) * (BN / 2);
    const int arow = tid / TPR, ak0 = (tid % TPR) * AK;
    const int bk = tid / TPK, bc0 = (tid % TPK) * BCOL;
    const bool aok = tm + arow < m;
    const double *ap = a + (r0 + tm + arow) * ld + k + ak0;
    const double *bp = a + k * ld + c0 + tn + bc0;
    const int64_t bcol_lim = nc - (tn + bc0);
    double ra[AK], rb[BCOL];
    auto load = [&](int64_t kc) {
        if (VEC && aok && kc + ak0 + AK <= kk) {
#pragma unroll
            for (int q = 0; q < AK; q += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(ap + kc + q);
                ra[q] = v.x; ra[q + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < AK; ++q) ra[q] = (aok && kc + ak0 + q < kk) ? ap[kc + q] : 0.0;
        }
        const int64_t kr = kc + bk;
        const bool kok = kr < kk;
        if (VEC && kok && bcol_lim >= BCOL) {
#pragma unroll
            for (int q = 0; q < BCOL; q += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(bp + kr * ld + q);
                rb[q] = v.x; rb[q + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < BCOL; ++q) rb[q] = (kok && q < bcol_lim) ? bp[kr * ld + q] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AK; ++q) As[buf][ak0 + q][arow] = ra[q];
#pragma unroll
        for (int q = 0; q < BCOL; q += 2)
            *reinterpret_cast<double2 *>(&Bs[buf][bk][bc0 + q]) = make_double2(rb[q], rb[q + 1]);
    };
    doublex4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = doublex4{0};
    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t kc = 0; kc < kk; kc += BK) {
        const bool more = kc + BK < kk;
        if (more) load(kc + BK);
#pragma unroll
        for (int s = 0; s < BK; s += 4) {
            const int kr = s + (lane >> 4);
            double af[MI], bf[NJ];
#pragma unroll
            for (int i = 0; i < MI; ++i) af[i] = As[buf][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NJ; ++j) bf[j] = Bs[buf][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // v_mfma_f64_16x16x4f64 output: lane l, register v -> row (l/16) + 4*v,
    // col l%16 (rows interleaved, unlike the binary32 16x16 layout).
    // Trailing update (role 0): c + (-acc) by a no-return atomic add, as in
    // the binary32 kernel (IEEE rounding, subnormals kept; FP64
    // factorization 677 -> 659 ms at N = 32768).  In-panel updates: every C load of the tile issued
    // before the first store (the atomic form slowed the panel stream).
    if constexpr (ROLE == 0) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = tm + wm + i * 16 + (lane >> 4) + 4 * v;
                    const int64_t col = tn + wn + j * 16 + (lane & 15);
                    if (row < m && col < nc)
                        __hip_atomic_fetch_add(a + (r0 + row) * ld + c0 + col, -acc[i][j][v], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                }
        return;
    }
    double cv[MI][NJ][4];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm + wm + i * 16 + (lane >> 4) + 4 * v;
                const int64_t col = tn + wn + j * 16 + (lane & 15);
                cv[i][j][v] = (row < m && col < nc) ? a[(r0 + row) * ld + c0 + col] : 0.0;
            }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm + wm + i * 16 + (lane >> 4) + 4 * v;
                const int64_t col = tn + wn + j * 16 + (lane & 15);
                if (row < m && col < nc) a[(r0 + row) * ld + c0 + col] = cv[i][j][v] - acc[i][j][v];
            }
}

// Tile configuration of the binary32 / binary16 kernels (chosen by timing
// the trailing update on MI355X).
template <bool HALF> struct Cfg32;
template <> struct Cfg32<false> { static constexpr int BM = 64, BN = 64, BK = 16, NBUF = 2; };
template <> struct Cfg32<true> { static constexpr int BM = 128, BN = 64, BK = 32, NBUF = 2; };
struct Cfg64 { static constexpr int BM = 64, BN = 64, BK = 16; };

// Dynamic LDS that limits a kernel with `stat` bytes of static LDS to at
// most `cap` workgroups per compute unit (160 KB of LDS each); 0 = no limit.
int cap_pad(const void *fn, int cap) {
    if (cap <= 0) return 0;
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) != hipSuccess) return 0;
    const int stat = (int)at.sharedSizeBytes, lds = 160 * 1024;
    const int want = lds / (cap + 1) + 1024;     // cap + 1 must not fit
    if (want <= stat || want * cap > lds) return 0;
    return want - stat;
}

template <bool HALF, int ROLE>
void go32(bool vec, float *a, int64_t ld, int64_t r0, int64_t m, int64_t c0, int64_t nc, int64_t k,
          int64_t kk, int cap, hipStream_t s) {
    using C = Cfg32<HALF>;
    const int64_t tiles_m = (m + C::BM - 1) / C::BM, tiles_n = (nc + C::BN - 1) / C::BN;
    const int64_t nblk = tiles_m * tiles_n;
    auto kv = k_gemm_32<HALF, true, C::BM, C::BN, C::BK, C::NBUF, ROLE>;
    auto ks = k_gemm_32<HALF, false, C::BM, C::BN, C::BK, C::NBUF, ROLE>;
    static int pad_v[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1}, pad_s[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    const int ci = cap < 0 ? 0 : cap > 8 ? 8 : cap;
    if (vec) {
        if (pad_v[ci] < 0) pad_v[ci] = cap_pad((const void *)kv, ci);
        kv<<<(unsigned)nblk, 256, pad_v[ci], s>>>(a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    } else {
        if (pad_s[ci] < 0) pad_s[ci] = cap_pad((const void *)ks, ci);
        ks<<<(unsigned)nblk, 256, pad_s[ci], s>>>(a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    }
}

template <int BM, int BN, int BK, int ROLE>
void go64(bool vec, double *a, int64_t ld, int64_t r0, int64_t m, int64_t c0, int64_t nc, int64_t k,
          int64_t kk, int cap, hipStream_t s) {
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (nc + BN - 1) / BN;
    const int64_t nblk = tiles_m * tiles_n;
    auto kv = k_gemm_f64<true, BM, BN, BK, ROLE>;
    auto ks = k_gemm_f64<false, BM, BN, BK, ROLE>;
    static int pad_v[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1}, pad_s[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    const int ci = cap < 0 ? 0 : cap > 8 ? 8 : cap;
    if (vec) {
        if (pad_v[ci] < 0) pad_v[ci] = cap_pad((const void *)kv, ci);
        kv<<<(unsigned)nblk, 256, pad_v[ci], s>>>(a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    } else {
        if (pad_s[ci] < 0) pad_s[ci] = cap_pad((const void *)ks, ci);
        ks<<<(unsigned)nblk, 256, pad_s[ci], s>>>(a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    }
}

template <int ROLE>
hipError_t gemm_go(int mode, void *a, int64_t ld, int64_t r0, int64_t m, int64_t c0,
                   int64_t nc, int64_t k, int64_t kk, int cap, hipStream_t s) {
    if (m <= 0 || nc <= 0 || kk <= 0) return hipSuccess;
    if ((m / 64 + 1) * (nc / 64 + 1) > 0x7fffffffll) return hipErrorInvalidValue;
    // 16-byte vector loads need every row start and offset 16-byte aligned
    const uintptr_t base = (uintptr_t)a;
    if (mode == LU_F64) {
        const bool vec = (ld % 2 == 0) && (k % 2 == 0) && (c0 % 2 == 0) && (base % 16 == 0);
        go64<Cfg64::BM, Cfg64::BN, Cfg64::BK, ROLE>(vec, (double *)a, ld, r0, m, c0, nc, k, kk, cap, s);
        return hipGetLastError();
    }
    const bool vec = (ld % 4 == 0) && (k % 4 == 0) && (c0 % 4 == 0) && (base % 16 == 0);
    if (mode == LU_F32 || mode == LU_BF16) go32<false, ROLE>(vec, (float *)a, ld, r0, m, c0, nc, k, kk, cap, s);
    else go32<true, ROLE>(vec, (float *)a, ld, r0, m, c0, nc, k, kk, cap, s);
    return hipGetLastError();
}

}  // namespace

size_t gemm_h16_ws_halves(int64_t rows, int64_t kk) {
    const int64_t rp = (rows + kHT - 1) / kHT * kHT, kp = (kk + kHK - 1) / kHK * kHK;
    return (size_t)(rp * kp);
}

template <typename T16>
hipError_t gemm_h16_go(float *a, int64_t ld, int64_t r0, int64_t m, int64_t c0, int64_t nc,
                       int64_t k, int64_t kk, void *wa, void *wb, int cap, hipStream_t s) {
    // operands packed with zero rows up to the next multiple of the tile
    // edge kHT, so every workgroup tile reads inside the workspace
    const int64_t mp = (m + kHT - 1) / kHT * kHT, np_ = (nc + kHT - 1) / kHT * kHT;
    const int64_t kp = (kk + kHK - 1) / kHK * kHK;
    const int64_t tiles_m = mp / kHT, tiles_n = np_ / kHT, nblk = tiles_m * tiles_n;
    if (nblk > 0x7fffffffll) return hipErrorInvalidValue;
    T16 *Ah = reinterpret_cast<T16 *>(wa), *Bt = reinterpret_cast<T16 *>(wb);
    {
        const int64_t work = mp * (kp / 8);
        const unsigned g = (unsigned)((work + 255) / 256 < 8192 ? (work + 255) / 256 : 8192);
        k_pack_rows_h<T16><<<g, 256, 0, s>>>(a, ld, r0, m, mp, k, kk, kp, Ah);
        dim3 gb((unsigned)(np_ / 64), (unsigned)((kp + 63) / 64));
        k_pack_cols_h<T16><<<gb, 256, 0, s>>>(a, ld, k, kk, kp, c0, nc, np_, Bt);
    }
    static_assert(64 * 2 == kHT, "the 16-bit update's tile edge");
    auto kv = k_gemm_h16<T16, 2, 2, kHK, 2>;
    static int pad[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
    const int ci = cap < 0 ? 0 : cap > 8 ? 8 : cap;
    if (pad[ci] < 0) pad[ci] = cap_pad((const void *)kv, ci);
    kv<<<(unsigned)nblk, 256, pad[ci], s>>>(a, ld, r0, m, c0, nc, Ah, Bt, kp, (int)tiles_n, (int)nblk);
    return hipGetLastError();
}

hipError_t launch_gemm_update_h16(int mode, float *a, int64_t ld, int64_t r0, int64_t m, int64_t c0,
                                  int64_t nc, int64_t k, int64_t kk, void *wa, void *wb, int cap,
                                  hipStream_t s) {
    if (m <= 0 || nc <= 0 || kk <= 0) return hipSuccess;
    if (mode == LU_BF16) return gemm_h16_go<__bf16>(a, ld, r0, m, c0, nc, k, kk, wa, wb, cap, s);
    return gemm_h16_go<_Float16>(a, ld, r0, m, c0, nc, k, kk, wa, wb, cap, s);
}

hipError_t launch_gemm_update(int mode, void *a, int64_t ld, int64_t r0, int64_t m, int64_t c0,
                              int64_t nc, int64_t k, int64_t kk, int cap, int role, hipStream_t s) {
    return role == 0 ? gemm_go<0>(mode, a, ld, r0, m, c0, nc, k, kk, cap, s)
                     : gemm_go<1>(mode, a, ld, r0, m, c0, nc, k, kk, cap, s);
}

}  // namespace mpir
