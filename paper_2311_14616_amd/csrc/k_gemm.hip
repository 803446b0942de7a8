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
//   TF = F64 : binary64, v_mfma_f64_16x16x4_f64 (the FP64 comparator).
//
// Tiling: 128 x 128 C tile per workgroup of four wave64s (2 x 2), each wave
// owning 64 x 64 of C in accumulator registers; operand tiles are staged in
// LDS with the next K-chunk prefetched into registers while the current one
// is multiplied.  The launch maps consecutive workgroup ids to tiles of one
// tile-row so that a tile-row's L21 block is shared in L2 by the workgroups
// that the dispatcher places on the same XCD.
#include "mpir_internal.h"

namespace mpir {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128;

// XCD-aware tile order: hardware dispatches workgroup ids round-robin over
// the 8 XCDs; remap so that XCD x receives a contiguous range of tiles
// (neighbouring tiles share operand rows/columns in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int NX = 8;
    if (nblk < NX * 4) return bid;
    const int per = nblk / NX;               // tiles per XCD (full part)
    const int full = per * NX;
    if (bid >= full) return bid;
    const int x = bid % NX, q = bid / NX;
    return x * per + q;
}

// ---------------------------------------------------------------- binary32
template <int BK>
__global__ __launch_bounds__(256) void k_gemm_f32(float *__restrict__ a, int64_t ld, int64_t r0,
                                                  int64_t m, int64_t c0, int64_t nc, int64_t k,
                                                  int64_t kk, int tiles_n, int nblk) {
    __shared__ float As[BK][BM + 4];   // k-major: lanes read consecutive rows
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    const int64_t tm = (int64_t)(bid / tiles_n) * BM, tn = (int64_t)(bid % tiles_n) * BN;
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;

    // global->register staging: A: row tid/2, 8 k's; B: k tid/16, 8 cols
    constexpr int AK = BK / 2;           // k's per thread for A (BK = 16 -> 8)
    const int arow = tid >> 1, ak0 = (tid & 1) * AK;
    constexpr int BCOLS = (BN * BK) / 256;   // cols per thread for B (8)
    const int bk = tid / (BN / BCOLS), bc0 = (tid % (BN / BCOLS)) * BCOLS;
    float ra[AK], rb[BCOLS];
    auto load = [&](int64_t kc) {
        const int64_t gi = r0 + tm + arow;
        const bool rok = (tm + arow) < m;
#pragma unroll
        for (int q = 0; q < AK; ++q) {
            const int64_t kq = kc + ak0 + q;
            ra[q] = (rok && kq < kk) ? a[gi * ld + k + kq] : 0.0f;
        }
        const int64_t kr = kc + bk;
#pragma unroll
        for (int q = 0; q < BCOLS; ++q) {
            const int64_t cj = tn + bc0 + q;
            rb[q] = (kr < kk && cj < nc) ? a[(k + kr) * ld + c0 + cj] : 0.0f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < AK; ++q) As[ak0 + q][arow] = ra[q];
#pragma unroll
        for (int q = 0; q < BCOLS; ++q) Bs[bk][bc0 + q] = rb[q];
    };

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};

    load(0);
    for (int64_t kc = 0; kc < kk; kc += BK) {
        store();
        __syncthreads();
        if (kc + BK < kk) load(kc + BK);
#pragma unroll
        for (int s = 0; s < BK; s += 2) {
            const int kr = s + (lane >> 5);
            float af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[kr][wm + i * 32 + (lane & 31)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][wn + j * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: lane l, register v -> row 8*(v/4) + 4*(l/32) + v%4, col l%32
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t col = tn + wn + j * 32 + (lane & 31);
                if (row < m && col < nc) {
                    float *p = a + (r0 + row) * ld + c0 + col;
                    *p = *p - acc[i][j][v];
                }
            }
}

// ------------------------------------------- binary16 operands, binary32 acc
constexpr int BK16 = 32;
__global__ __launch_bounds__(256) void k_gemm_f16(float *__restrict__ a, int64_t ld, int64_t r0,
                                                  int64_t m, int64_t c0, int64_t nc, int64_t k,
                                                  int64_t kk, int tiles_n, int nblk) {
    constexpr int KP = BK16 + 8;            // row pitch in halves (16-byte aligned)
    __shared__ __align__(16) _Float16 As[BM][KP];   // row-major: 8 consecutive k per lane
    __shared__ __align__(16) _Float16 Bs[BN][KP];   // transposed: [col][k]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    const int64_t tm = (int64_t)(bid / tiles_n) * BM, tn = (int64_t)(bid % tiles_n) * BN;
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;

    // A: 128 x 32 -> thread: row tid/2, 16 k's.  B: 32 x 128 -> thread: k tid/8, 16 cols
    const int arow = tid >> 1, ak0 = (tid & 1) * 16;
    const int bk = tid >> 3, bc0 = (tid & 7) * 16;
    float ra[16], rb[16];
    auto load = [&](int64_t kc) {
        const int64_t gi = r0 + tm + arow;
        const bool rok = (tm + arow) < m;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t kq = kc + ak0 + q;
            ra[q] = (rok && kq < kk) ? a[gi * ld + k + kq] : 0.0f;
        }
        const int64_t kr = kc + bk;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t cj = tn + bc0 + q;
            rb[q] = (kr < kk && cj < nc) ? a[(k + kr) * ld + c0 + cj] : 0.0f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < 16; ++q) As[arow][ak0 + q] = (_Float16)ra[q];
#pragma unroll
        for (int q = 0; q < 16; ++q) Bs[bc0 + q][bk] = (_Float16)rb[q];
    };

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};

    load(0);
    for (int64_t kc = 0; kc < kk; kc += BK16) {
        store();
        __syncthreads();
        if (kc + BK16 < kk) load(kc + BK16);
#pragma unroll
        for (int s = 0; s < BK16; s += 16) {
            const int kb = s + 8 * (lane >> 5);
            half8 af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const half8 *>(&As[wm + i * 32 + (lane & 31)][kb]);
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = *reinterpret_cast<const half8 *>(&Bs[wn + j * 32 + (lane & 31)][kb]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = tm + wm + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t col = tn + wn + j * 32 + (lane & 31);
                if (row < m && col < nc) {
                    float *p = a + (r0 + row) * ld + c0 + col;
                    *p = *p - acc[i][j][v];
                }
            }
}

// ---------------------------------------------------------------- binary64
constexpr int BK64 = 8;
__global__ __launch_bounds__(256) void k_gemm_f64(double *__restrict__ a, int64_t ld, int64_t r0,
                                                  int64_t m, int64_t c0, int64_t nc, int64_t k,
                                                  int64_t kk, int tiles_n, int nblk) {
    __shared__ double As[BK64][BM + 2];
    __shared__ double Bs[BK64][BN + 2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    const int64_t tm = (int64_t)(bid / tiles_n) * BM, tn = (int64_t)(bid % tiles_n) * BN;
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
    // A: 128 x 8 -> thread: row tid/2, 4 k's.  B: 8 x 128 -> thread: k tid/32, 4 cols
    const int arow = tid >> 1, ak0 = (tid & 1) * 4;
    const int bk = tid >> 5, bc0 = (tid & 31) * 4;
    double ra[4], rb[4];
    auto load = [&](int64_t kc) {
        const int64_t gi = r0 + tm + arow;
        const bool rok = (tm + arow) < m;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t kq = kc + ak0 + q;
            ra[q] = (rok && kq < kk) ? a[gi * ld + k + kq] : 0.0;
        }
        const int64_t kr = kc + bk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t cj = tn + bc0 + q;
            rb[q] = (kr < kk && cj < nc) ? a[(k + kr) * ld + c0 + cj] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) As[ak0 + q][arow] = ra[q];
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[bk][bc0 + q] = rb[q];
    };
    doublex4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0};
    load(0);
    for (int64_t kc = 0; kc < kk; kc += BK64) {
        store();
        __syncthreads();
        if (kc + BK64 < kk) load(kc + BK64);
#pragma unroll
        for (int s = 0; s < BK64; s += 4) {
            const int kr = s + (lane >> 4);
            double af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = Bs[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // v_mfma_f64_16x16x4f64 output: lane l, register v -> row (l/16) + 4*v,
    // col l%16 (rows interleaved, unlike the binary32 16x16 layout)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm + wm + i * 16 + (lane >> 4) + 4 * v;
                const int64_t col = tn + wn + j * 16 + (lane & 15);
                if (row < m && col < nc) {
                    double *p = a + (r0 + row) * ld + c0 + col;
                    *p = *p - acc[i][j][v];
                }
            }
}

}  // namespace

hipError_t launch_gemm_update(int mode, void *a, int64_t ld, int64_t r0, int64_t m, int64_t c0,
                              int64_t nc, int64_t k, int64_t kk, hipStream_t s) {
    if (m <= 0 || nc <= 0 || kk <= 0) return hipSuccess;
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (nc + BN - 1) / BN;
    const int64_t nblk = tiles_m * tiles_n;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(256);
    if (mode == LU_F64)
        k_gemm_f64<<<grid, block, 0, s>>>((double *)a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    else if (mode == LU_F32)
        k_gemm_f32<16><<<grid, block, 0, s>>>((float *)a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    else
        k_gemm_f16<<<grid, block, 0, s>>>((float *)a, ld, r0, m, c0, nc, k, kk, (int)tiles_n, (int)nblk);
    return hipGetLastError();
}

}  // namespace mpir
