// Interprecision copy A_F = I_W^F(A) (paper, notation following Algorithm IR)
// fused with ||A||_inf and the finiteness / range checks.
//
// Layout: A is column-major in TW (lda); A_F is the row-major working array
// of the factorization (binary32 for TF in {F32, F16, BF16}, binary64 for
// F64).
// One workgroup owns a strip of TR rows and walks the column tiles from left
// to right, so each row sum of |a_ij| is accumulated in increasing j (the
// same order as a plain loop, hence bit-identical to it).  Reads are
// coalesced along columns, the tile is transposed through LDS and written
// coalesced along rows.  The next tile's loads are issued into registers
// before the current tile's row sums and stores, so two tiles per workgroup
// are in flight (one tile at a time, with the loads issued a few at a time,
// reached 2.2 TB/s).
#include "mpir_internal.h"

namespace mpir {
namespace {

constexpr int TC = 64;   // columns per tile
// rows per strip (measured at N = 32768: 2.62 ms with 64, 2.69 with 32,
// 2.97 with 16)
constexpr int kStripRows = 64;

// TR rows per strip
template <typename TWt, typename Wt, int TF, int TR>
__global__ __launch_bounds__(256) void k_downcast(int64_t n, const TWt *__restrict__ A,
                                                  int64_t lda, Wt *__restrict__ AF, int64_t ldf,
                                                  uint64_t *anorm_bits, uint32_t *flags) {
    constexpr int LPT = TR * TC / 256;   // elements per thread and tile
    __shared__ double tile[TC][TR + 1];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * TR;
    // load mapping: thread -> row (t % TR), columns (t / TR) + (256 / TR) s
    const int lr = t % TR, lc = t / TR;
    constexpr int LCS = 256 / TR;
    const int64_t li = i0 + lr;
    double v[LPT];
    auto load = [&](int64_t j0) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int64_t j = j0 + lc + LCS * q;
            v[q] = (li < n && j < n) ? (double)A[li + j * lda] : 0.0;
        }
    };
    double rs = 0.0;
    uint32_t fl = 0;
    load(0);
    for (int64_t j0 = 0; j0 < n; j0 += TC) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) tile[lc + LCS * q][lr] = v[q];
        __syncthreads();
        if (j0 + TC < n) load(j0 + TC);
        if (t < TR) {
            // row sum in increasing column order (one thread per row)
            const int64_t i = i0 + t;
            if (i < n) {
                const int cmax = (int)((n - j0) < TC ? (n - j0) : TC);
                for (int c = 0; c < cmax; ++c) rs = rs + fabs(tile[c][t]);
            }
        }
        // store: thread -> column (t % TC), rows (t / TC) + 4 s
        {
            const int c = t % TC;
            const int64_t j = j0 + c;
#pragma unroll
            for (int s = 0; s < TR / 4; ++s) {
                const int r = t / TC + 4 * s;
                const int64_t i = i0 + r;
                if (i < n && j < n) {
                    const double x = tile[c][r];
                    Wt w;
                    if (TF == MPIR_F64) w = (Wt)x;
                    else if (TF == MPIR_F32) w = (Wt)(float)x;
                    else if (TF == MPIR_BF16) w = (Wt)d2bf_as_float(x);
                    else w = (Wt)d2h_as_float(x);
                    if (!isfinite(x)) fl |= DF_NONFINITE;
                    else if (isinf((double)w)) fl |= DF_RANGE;
                    AF[i * ldf + j] = w;
                }
            }
        }
        __syncthreads();
    }
    if (t < TR && i0 + t < n) {
        if (isfinite(rs)) atomic_max_nonneg(anorm_bits, rs);
        else fl |= DF_NONFINITE;
    }
    if (fl) atomicOr(flags, fl);
}

// dst (pitch ldd) = 16-bit copy of src (pitch lds): binary16 (BF = false)
// or bfloat16 (BF = true, the upper half of the binary32 pattern); the
// source holds such numbers already, so the conversion is exact.  One
// workgroup per row segment of kPackCols columns, four columns per thread
// (16-byte loads, 8-byte stores when both pitches and bases allow them).
constexpr int kPackCols = 1024;

template <bool BF>
__device__ __forceinline__ uint32_t pack2(float x, float y) {
    if (BF) return (__float_as_uint(x) >> 16) | (__float_as_uint(y) & 0xffff0000u);
    __half2 h = __floats2half2_rn(x, y);
    return *reinterpret_cast<uint32_t *>(&h);
}

template <bool BF>
__global__ __launch_bounds__(256) void k_pack_half(int64_t n, const float *__restrict__ src, int64_t lds,
                                                   uint16_t *__restrict__ dst, int64_t ldd, int segs, int vec) {
    const int64_t r = blockIdx.x / segs;
    const int64_t c = (int64_t)(blockIdx.x % segs) * kPackCols + threadIdx.x * 4;
    if (c >= n) return;
    const float *s = src + r * lds + c;
    uint16_t *d = dst + r * ldd + c;
    if (vec && c + 4 <= n) {
        const float4 v = *reinterpret_cast<const float4 *>(s);
        uint2 o;
        o.x = pack2<BF>(v.x, v.y);
        o.y = pack2<BF>(v.z, v.w);
        *reinterpret_cast<uint2 *>(d) = o;
    } else {
        for (int j = 0; j < 4 && c + j < n; ++j) d[j] = (uint16_t)(pack2<BF>(s[j], 0.0f) & 0xffffu);
    }
}

template <int TR>
void downcast_go(int64_t n, const void *A, int64_t lda, int tw, int tf, void *AF, int64_t ldf,
                 uint64_t *anorm_bits, uint32_t *flags, hipStream_t s) {
    dim3 grid((unsigned)((n + TR - 1) / TR)), block(256);
    if (tw == MPIR_F64) {
        const double *a = (const double *)A;
        if (tf == MPIR_F64) k_downcast<double, double, MPIR_F64, TR><<<grid, block, 0, s>>>(n, a, lda, (double *)AF, ldf, anorm_bits, flags);
        else if (tf == MPIR_F32) k_downcast<double, float, MPIR_F32, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
        else if (tf == MPIR_BF16) k_downcast<double, float, MPIR_BF16, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
        else k_downcast<double, float, MPIR_F16, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
    } else {
        const float *a = (const float *)A;
        if (tf == MPIR_F32) k_downcast<float, float, MPIR_F32, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
        else if (tf == MPIR_BF16) k_downcast<float, float, MPIR_BF16, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
        else k_downcast<float, float, MPIR_F16, TR><<<grid, block, 0, s>>>(n, a, lda, (float *)AF, ldf, anorm_bits, flags);
    }
}

}  // namespace

hipError_t launch_downcast(int64_t n, const void *A, int64_t lda, int tw, int tf, void *AF,
                           int64_t ldf, uint64_t *anorm_bits, uint32_t *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    downcast_go<kStripRows>(n, A, lda, tw, tf, AF, ldf, anorm_bits, flags, s);
    return hipGetLastError();
}

hipError_t launch_pack_half(int tf, int64_t n, const float *AF, int64_t ldf, void *LU, int64_t ldl,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int segs = (int)((n + kPackCols - 1) / kPackCols);
    const int vec = (ldf % 4 == 0 && ldl % 4 == 0 && ((uintptr_t)AF & 15) == 0 && ((uintptr_t)LU & 7) == 0);
    if (tf == MPIR_BF16)
        k_pack_half<true><<<(unsigned)(n * segs), 256, 0, s>>>(n, AF, ldf, (uint16_t *)LU, ldl, segs, vec);
    else
        k_pack_half<false><<<(unsigned)(n * segs), 256, 0, s>>>(n, AF, ldf, (uint16_t *)LU, ldl, segs, vec);
    return hipGetLastError();
}

hipError_t launch_copy_factors(int64_t n, const void *src, int tf, void *dst, hipStream_t s) {
    const size_t es = tf == MPIR_F64 ? 8 : (tf == MPIR_F32 ? 4 : 2);
    return hipMemcpyAsync(dst, src, (size_t)n * (size_t)n * es, hipMemcpyDeviceToDevice, s);
}

}  // namespace mpir
