// The O(N^2) and O(N) steps of the refinement loop (Algorithm IR):
//  - residual r = b - A x in precision TR (eq. xferrule: A, x, b promoted
//    exactly, then operated on in TR), as a coalesced column-major GEMV with
//    a deterministic two-pass column-chunk reduction;
//  - scale, permute and downcast of the residual for the low-precision solve
//    (eq. vdlow: rhat = I_W^F(P r / sigma));
//  - promote, unscale and update (eq. promotevd: d = sigma I_F^W(d_F);
//    x <- x + d in TW);
//  - the termination rules (eqs. residterm, term, stag, wilkterm, litmax),
//    evaluated on the device so that the loop needs no host round trip to
//    decide; every loop kernel returns at once after `done` is set.
#include "mpir_internal.h"

namespace mpir {
namespace {

constexpr int kRowsPerBlock = 256;   // one row per thread
constexpr int kChunkCols = 256;      // columns per partial sum

__device__ __forceinline__ double bits_to_d(uint64_t b) { return __longlong_as_double((long long)b); }

// Bit pattern of |v| for a max that keeps NaN (its pattern orders above +inf).
__device__ __forceinline__ uint64_t abs_bits(double v) {
    return (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
}
__device__ __forceinline__ uint64_t wave_max_bits(uint64_t b) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)b, off);
        b = o > b ? o : b;
    }
    return b;
}
__device__ __forceinline__ void atomic_max_bits(uint64_t *p, uint64_t b) {
    atomicMax((unsigned long long *)p, (unsigned long long)b);
}

// Power of two sigma with m / sigma in (1/2, 1] (m > 0, finite).
__device__ __forceinline__ double pow2_ceil(double m) {
    int e;
    const double f = frexp(m, &e);
    return f == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

// ---- residual, pass 1: partial[c][i] = sum_{j in chunk c} a_ij x_j --------
// Thread per RPT consecutive rows (one 8- or 16-byte load per column covers
// them; a wave reads 64*RPT consecutive entries of a column), 16 columns in
// flight per thread.
// (TXt: the type of x, binary64 for the Krylov products with a binary32 A)
template <typename TWt, typename TRt, int RPT, typename TXt = TWt>
__global__ __launch_bounds__(256) void k_resid_partial(int64_t n, const TWt *__restrict__ A, int64_t lda,
                                                       const TXt *__restrict__ x,
                                                       double *__restrict__ partial,
                                                       const IrState *st, int force) {
    if (!force && st->done) return;
    const int64_t i = ((int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x) * RPT;
    const int64_t j0 = (int64_t)blockIdx.y * kChunkCols;
    const int64_t j1 = (j0 + kChunkCols) < n ? (j0 + kChunkCols) : n;
    if (i >= n) return;
    TRt acc[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = 0;
    const TWt *col = A + i + j0 * lda;
    const bool full = i + RPT <= n;
    int64_t j = j0;
    if (full) {
        for (; j + 16 <= j1; j += 16) {
            TWt v[16][RPT];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const TWt *p = col + (j - j0 + q) * lda;
                if constexpr (RPT == 2 && sizeof(TWt) == 8) {
                    const double2 t = *reinterpret_cast<const double2 *>(p);
                    v[q][0] = t.x; v[q][1] = t.y;
                } else if constexpr (RPT == 2 && sizeof(TWt) == 4) {
                    const float2 t = *reinterpret_cast<const float2 *>(p);
                    v[q][0] = t.x; v[q][1] = t.y;
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) v[q][r] = p[r];
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const TRt xq = (TRt)x[j + q];
#pragma unroll
                for (int r = 0; r < RPT; ++r) acc[r] = fmadd((TRt)v[q][r], xq, acc[r]);
            }
        }
    }
    for (; j < j1; ++j) {
        const TRt xq = (TRt)x[j];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (i + r < n) acc[r] = fmadd((TRt)col[(j - j0) * lda + r], xq, acc[r]);
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
        if (i + r < n) partial[(int64_t)blockIdx.y * n + i + r] = (double)acc[r];
}

// ---- residual, pass 1 for NR right-hand sides (columns x + q * ldx):
// A is read once; column q's partial sums go to partial + q * nch * n and
// receive exactly the operations of the one-column pass, in its order.
template <typename TWt, typename TRt, int RPT, int NR>
__global__ __launch_bounds__(256) void k_resid_partial_multi(int64_t n, const TWt *__restrict__ A,
                                                             int64_t lda, const TWt *__restrict__ x,
                                                             int64_t ldx, double *__restrict__ partial,
                                                             int nch) {
    const int64_t i = ((int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x) * RPT;
    const int64_t j0 = (int64_t)blockIdx.y * kChunkCols;
    const int64_t j1 = (j0 + kChunkCols) < n ? (j0 + kChunkCols) : n;
    if (i >= n) return;
    TRt acc[NR][RPT];
#pragma unroll
    for (int c = 0; c < NR; ++c)
#pragma unroll
        for (int r = 0; r < RPT; ++r) acc[c][r] = 0;
    const TWt *col = A + i + j0 * lda;
    const bool full = i + RPT <= n;
    int64_t j = j0;
    if (full) {
        for (; j + 16 <= j1; j += 16) {
            TWt v[16][RPT];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const TWt *p = col + (j - j0 + q) * lda;
                if constexpr (RPT == 2 && sizeof(TWt) == 8) {
                    const double2 t = *reinterpret_cast<const double2 *>(p);
                    v[q][0] = t.x; v[q][1] = t.y;
                } else if constexpr (RPT == 2 && sizeof(TWt) == 4) {
                    const float2 t = *reinterpret_cast<const float2 *>(p);
                    v[q][0] = t.x; v[q][1] = t.y;
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) v[q][r] = p[r];
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q)
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const TRt xq = (TRt)x[c * ldx + j + q];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) acc[c][r] = fmadd((TRt)v[q][r], xq, acc[c][r]);
                }
        }
    }
    for (; j < j1; ++j)
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const TRt xq = (TRt)x[c * ldx + j];
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (i + r < n) acc[c][r] = fmadd((TRt)col[(j - j0) * lda + r], xq, acc[c][r]);
        }
#pragma unroll
    for (int c = 0; c < NR; ++c)
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (i + r < n) partial[((int64_t)c * nch + blockIdx.y) * n + i + r] = (double)acc[c][r];
}

// ---- residual, pass 2: r_i = b_i - sum_c partial[c][i] (c increasing) ----
template <typename TWt, typename TRt>
__global__ __launch_bounds__(256) void k_resid_reduce(int64_t n, const TWt *__restrict__ b,
                                                      const TWt *__restrict__ x,
                                                      const double *__restrict__ partial, int nch,
                                                      TRt *__restrict__ r, IrState *st, int force) {
    if (!force && st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t rm = 0, xm = 0;
    if (i < n) {
        TRt s = 0;
        for (int c = 0; c < nch; ++c) s += (TRt)partial[(int64_t)c * n + i];
        const TRt ri = (TRt)b[i] - s;
        r[i] = ri;
        rm = abs_bits((double)ri);
        xm = abs_bits((double)x[i]);
    }
    rm = wave_max_bits(rm);
    xm = wave_max_bits(xm);
    if ((threadIdx.x & 63) == 0) {
        atomic_max_bits(&st->rnorm_bits, rm);
        atomic_max_bits(&st->xnorm_bits, xm);
    }
}

// ---- x = 0, r = b (in TR), ||b|| into rnorm_bits ----
template <typename TWt, typename TRt>
__global__ void k_ir_init(int64_t n, const TWt *__restrict__ b, TWt *__restrict__ x,
                          TRt *__restrict__ r, IrState *st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t bm = 0;
    if (i < n) {
        const TWt bi = b[i];
        x[i] = (TWt)0;
        r[i] = (TRt)bi;
        bm = abs_bits((double)bi);
    }
    bm = wave_max_bits(bm);
    if ((threadIdx.x & 63) == 0) atomic_max_bits(&st->rnorm_bits, bm);
}

// ---- rhat_i = fl_F(r_{perm_i} / sigma) ----
template <typename TRt, typename Yt, int TF>
__global__ __launch_bounds__(256) void k_scale_permute(int64_t n, const TRt *__restrict__ r,
                                                       const int32_t *__restrict__ perm,
                                                       Yt *__restrict__ rhat, IrState *st,
                                                       TrsvSync *ts, int force) {
    if (!force && st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) { ts->ticket_l = 0; ts->done_l = 0; ts->ticket_u = 0; ts->done_u = 0; ts->epoch += 2u; }
    if (i >= n) return;
    const double inv = 1.0 / st->sigma;      // exact: sigma is a power of two
    const double v = (double)r[perm[i]] * inv;
    Yt o;
    if (TF == MPIR_F64) o = (Yt)v;
    else if (TF == MPIR_F32) o = (Yt)(float)v;
    else if (TF == MPIR_BF16) o = (Yt)d2bf_as_float(v);
    else o = (Yt)d2h_as_float(v);
    rhat[i] = o;
}

// ---- d = sigma * y (exact), x <- fl_W(x + d), ||d|| ----
template <typename TWt, typename Yt>
__global__ __launch_bounds__(256) void k_update(int64_t n, const Yt *__restrict__ y, TWt *__restrict__ x,
                                                IrState *st, int force) {
    if (!force && st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t dm = 0;
    if (i < n) {
        const TWt d = (TWt)st->sigma * (TWt)y[i];
        x[i] = x[i] + d;
        dm = abs_bits((double)d);
    }
    dm = wave_max_bits(dm);
    if ((threadIdx.x & 63) == 0) atomic_max_bits(&st->dnorm_bits, dm);
}

// ---- termination (one thread).  it < 0: the initial residual r = b. ----
__global__ void k_terminate(IrState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    const double rn = bits_to_d(st->rnorm_bits);
    st->rnorm_bits = 0;
    if (st->it < 0) {                       // r = b, x = 0
        st->it = 0;
        st->bnorm = rn;
        st->rnorm = rn;
        st->xnorm = 0.0;
        st->rhist[0] = rn;
        int conv = 0;
        if (!isfinite(rn)) { st->done = 1; st->stop = MPIR_STOP_NONFINITE; return; }
        if (rn == 0.0) conv = 1;
        else if (!st->wilk)
            conv = st->residterm ? (rn <= st->tol_r * st->bnorm)
                                 : (rn <= st->tol_e * (st->bnorm + st->anorm * 0.0));
        if (conv) { st->done = 1; st->stop = MPIR_STOP_CONVERGED; return; }
        st->sigma = pow2_ceil(rn);
        return;
    }
    const double dn = bits_to_d(st->dnorm_bits);
    const double xn = bits_to_d(st->xnorm_bits);
    st->dnorm_bits = 0;
    st->xnorm_bits = 0;
    const int it = st->it + 1;
    st->it = it;
    st->rnorm = rn;
    st->dnorm = dn;
    st->xnorm = xn;
    st->rhist[it] = rn;
    st->dhist[it - 1] = dn;
    int stop = -1;
    if (!isfinite(rn) || !isfinite(dn)) stop = MPIR_STOP_NONFINITE;
    else if (rn == 0.0) stop = MPIR_STOP_CONVERGED;
    else if (!st->wilk) {
        const int conv = st->residterm ? (rn <= st->tol_r * st->bnorm)
                                       : (rn <= st->tol_e * (st->bnorm + st->anorm * xn));
        if (conv) stop = MPIR_STOP_CONVERGED;
        else if (it >= st->litmax) stop = MPIR_STOP_LITMAX;
        else if (st->rhist[it] >= st->rmax * st->rhist[it - 1]) stop = MPIR_STOP_STAGNATED;
    } else {
        if (it >= st->litmax) stop = MPIR_STOP_LITMAX;
        else if (it >= 2 && st->dhist[it - 1] >= st->rmax * st->dhist[it - 2]) stop = MPIR_STOP_DSTAGNATED;
    }
    if (stop >= 0) { st->done = 1; st->stop = stop; return; }
    st->sigma = pow2_ceil(rn);
}

// sigma for a single solve (mpir_solve): from ||b|| in rnorm_bits.
__global__ void k_set_sigma(IrState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rn = bits_to_d(st->rnorm_bits);
    st->rnorm_bits = 0;
    st->bnorm = rn;
    st->sigma = (rn > 0.0 && isfinite(rn)) ? pow2_ceil(rn) : 1.0;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int residual_chunks(int64_t n) { return (int)((n + kChunkCols - 1) / kChunkCols); }

hipError_t launch_residual(int64_t n, const void *A, int64_t lda, int tw, int tr, const void *b,
                           const void *x, void *r, double *partial, int nch, IrState *st,
                           int force, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // two rows per thread with vector loads when every column start is aligned
    const size_t es = tw == MPIR_F64 ? 8 : 4;
    const bool vec = ((uintptr_t)A % (2 * es) == 0) && (lda % 2 == 0);
    const int rpt = vec ? 2 : 1;
    dim3 g1((unsigned)((n + (int64_t)kRowsPerBlock * rpt - 1) / ((int64_t)kRowsPerBlock * rpt)), (unsigned)nch);
    dim3 b1(kRowsPerBlock);
    dim3 g2(blocks_for(n, 256)), b2(256);
    if (tw == MPIR_F64) {
        if (vec) k_resid_partial<double, double, 2><<<g1, b1, 0, s>>>(n, (const double *)A, lda, (const double *)x, partial, st, force);
        else k_resid_partial<double, double, 1><<<g1, b1, 0, s>>>(n, (const double *)A, lda, (const double *)x, partial, st, force);
        k_resid_reduce<double, double><<<g2, b2, 0, s>>>(n, (const double *)b, (const double *)x, partial, nch, (double *)r, st, force);
    } else if (tr == MPIR_F64) {
        if (vec) k_resid_partial<float, double, 2><<<g1, b1, 0, s>>>(n, (const float *)A, lda, (const float *)x, partial, st, force);
        else k_resid_partial<float, double, 1><<<g1, b1, 0, s>>>(n, (const float *)A, lda, (const float *)x, partial, st, force);
        k_resid_reduce<float, double><<<g2, b2, 0, s>>>(n, (const float *)b, (const float *)x, partial, nch, (double *)r, st, force);
    } else {
        if (vec) k_resid_partial<float, float, 2><<<g1, b1, 0, s>>>(n, (const float *)A, lda, (const float *)x, partial, st, force);
        else k_resid_partial<float, float, 1><<<g1, b1, 0, s>>>(n, (const float *)A, lda, (const float *)x, partial, st, force);
        k_resid_reduce<float, float><<<g2, b2, 0, s>>>(n, (const float *)b, (const float *)x, partial, nch, (float *)r, st, force);
    }
    return hipGetLastError();
}

// r = b - A x with A in TW (binary64 or binary32) and b, x, r in binary64:
// the products of the Krylov corrections.
hipError_t launch_residual_x64(int64_t n, const void *A, int64_t lda, int tw, const double *b,
                               const double *x, double *r, double *partial, int nch, IrState *st,
                               hipStream_t s) {
    if (tw == MPIR_F64)
        return launch_residual(n, A, lda, MPIR_F64, MPIR_F64, b, x, r, partial, nch, st, 1, s);
    if (n <= 0) return hipSuccess;
    const bool vec = ((uintptr_t)A % 8 == 0) && (lda % 2 == 0);
    const int rpt = vec ? 2 : 1;
    dim3 g1((unsigned)((n + (int64_t)kRowsPerBlock * rpt - 1) / ((int64_t)kRowsPerBlock * rpt)), (unsigned)nch);
    dim3 g2(blocks_for(n, 256)), b2(256);
    if (vec) k_resid_partial<float, double, 2, double><<<g1, kRowsPerBlock, 0, s>>>(n, (const float *)A, lda, x, partial, st, 1);
    else k_resid_partial<float, double, 1, double><<<g1, kRowsPerBlock, 0, s>>>(n, (const float *)A, lda, x, partial, st, 1);
    k_resid_reduce<double, double><<<g2, b2, 0, s>>>(n, b, x, partial, nch, r, st, 1);
    return hipGetLastError();
}

template <typename TWt, typename TRt, int NR>
void resid_multi_go(bool vec, int64_t n, const TWt *A, int64_t lda, const TWt *x, int64_t ldx,
                    double *partial, int nch, hipStream_t s) {
    const int rpt = vec ? 2 : 1;
    dim3 g1((unsigned)((n + (int64_t)kRowsPerBlock * rpt - 1) / ((int64_t)kRowsPerBlock * rpt)), (unsigned)nch);
    if (vec) k_resid_partial_multi<TWt, TRt, 2, NR><<<g1, kRowsPerBlock, 0, s>>>(n, A, lda, x, ldx, partial, nch);
    else k_resid_partial_multi<TWt, TRt, 1, NR><<<g1, kRowsPerBlock, 0, s>>>(n, A, lda, x, ldx, partial, nch);
}

template <typename TWt, typename TRt>
void resid_multi_nr(int nr, bool vec, int64_t n, const TWt *A, int64_t lda, const TWt *x, int64_t ldx,
                    double *partial, int nch, hipStream_t s) {
    if (nr == 1) resid_multi_go<TWt, TRt, 1>(vec, n, A, lda, x, ldx, partial, nch, s);
    else if (nr == 2) resid_multi_go<TWt, TRt, 2>(vec, n, A, lda, x, ldx, partial, nch, s);
    else if (nr == 3) resid_multi_go<TWt, TRt, 3>(vec, n, A, lda, x, ldx, partial, nch, s);
    else resid_multi_go<TWt, TRt, 4>(vec, n, A, lda, x, ldx, partial, nch, s);
}

hipError_t launch_residual_multi(int64_t n, const void *A, int64_t lda, int tw, int tr, int nr,
                                 const void *b, int64_t ldb, const void *x, int64_t ldx, void *r,
                                 double *partial, int nch, IrState *st, int force, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nr < 1 || nr > 4) return hipErrorInvalidValue;
    const size_t es = tw == MPIR_F64 ? 8 : 4;
    const size_t rs = tr == MPIR_F64 ? 8 : 4;
    const bool vec = ((uintptr_t)A % (2 * es) == 0) && (lda % 2 == 0);
    dim3 g2(blocks_for(n, 256)), b2(256);
    if (tw == MPIR_F64)
        resid_multi_nr<double, double>(nr, vec, n, (const double *)A, lda, (const double *)x, ldx, partial, nch, s);
    else if (tr == MPIR_F64)
        resid_multi_nr<float, double>(nr, vec, n, (const float *)A, lda, (const float *)x, ldx, partial, nch, s);
    else
        resid_multi_nr<float, float>(nr, vec, n, (const float *)A, lda, (const float *)x, ldx, partial, nch, s);
    for (int c = 0; c < nr; ++c) {
        const char *bc = (const char *)b + c * ldb * es;
        const char *xc = (const char *)x + c * ldx * es;
        char *rc = (char *)r + c * n * rs;
        const double *pc = partial + (int64_t)c * nch * n;
        if (tw == MPIR_F64)
            k_resid_reduce<double, double><<<g2, b2, 0, s>>>(n, (const double *)bc, (const double *)xc, pc, nch, (double *)rc, st + c, force);
        else if (tr == MPIR_F64)
            k_resid_reduce<float, double><<<g2, b2, 0, s>>>(n, (const float *)bc, (const float *)xc, pc, nch, (double *)rc, st + c, force);
        else
            k_resid_reduce<float, float><<<g2, b2, 0, s>>>(n, (const float *)bc, (const float *)xc, pc, nch, (float *)rc, st + c, force);
    }
    return hipGetLastError();
}

hipError_t launch_ir_init(int64_t n, int tw, int tr, const void *b, void *x, void *r, IrState *st,
                          hipStream_t s) {
    dim3 g(blocks_for(n, 256)), bl(256);
    if (tw == MPIR_F64) k_ir_init<double, double><<<g, bl, 0, s>>>(n, (const double *)b, (double *)x, (double *)r, st);
    else if (tr == MPIR_F64) k_ir_init<float, double><<<g, bl, 0, s>>>(n, (const float *)b, (float *)x, (double *)r, st);
    else k_ir_init<float, float><<<g, bl, 0, s>>>(n, (const float *)b, (float *)x, (float *)r, st);
    return hipGetLastError();
}

hipError_t launch_scale_permute(int64_t n, int tr, int tf, const void *r, const int32_t *perm,
                                void *rhat, IrState *st, TrsvSync *ts, int force, hipStream_t s) {
    dim3 g(blocks_for(n, 256)), bl(256);
    if (tf == MPIR_F64) {
        k_scale_permute<double, double, MPIR_F64><<<g, bl, 0, s>>>(n, (const double *)r, perm, (double *)rhat, st, ts, force);
    } else if (tr == MPIR_F64) {
        if (tf == MPIR_F32) k_scale_permute<double, float, MPIR_F32><<<g, bl, 0, s>>>(n, (const double *)r, perm, (float *)rhat, st, ts, force);
        else if (tf == MPIR_BF16) k_scale_permute<double, float, MPIR_BF16><<<g, bl, 0, s>>>(n, (const double *)r, perm, (float *)rhat, st, ts, force);
        else k_scale_permute<double, float, MPIR_F16><<<g, bl, 0, s>>>(n, (const double *)r, perm, (float *)rhat, st, ts, force);
    } else {
        if (tf == MPIR_F32) k_scale_permute<float, float, MPIR_F32><<<g, bl, 0, s>>>(n, (const float *)r, perm, (float *)rhat, st, ts, force);
        else if (tf == MPIR_BF16) k_scale_permute<float, float, MPIR_BF16><<<g, bl, 0, s>>>(n, (const float *)r, perm, (float *)rhat, st, ts, force);
        else k_scale_permute<float, float, MPIR_F16><<<g, bl, 0, s>>>(n, (const float *)r, perm, (float *)rhat, st, ts, force);
    }
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, int tw, int tf, const void *y, void *x, IrState *st, int force,
                         hipStream_t s) {
    dim3 g(blocks_for(n, 256)), bl(256);
    if (tf == MPIR_F64 && tw == MPIR_F64) k_update<double, double><<<g, bl, 0, s>>>(n, (const double *)y, (double *)x, st, force);
    else if (tf == MPIR_F64) k_update<float, double><<<g, bl, 0, s>>>(n, (const double *)y, (float *)x, st, force);
    else if (tw == MPIR_F64) k_update<double, float><<<g, bl, 0, s>>>(n, (const float *)y, (double *)x, st, force);
    else k_update<float, float><<<g, bl, 0, s>>>(n, (const float *)y, (float *)x, st, force);
    return hipGetLastError();
}

hipError_t launch_terminate(IrState *st, hipStream_t s) {
    k_terminate<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_set_sigma(IrState *st, hipStream_t s) {
    k_set_sigma<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

}  // namespace mpir
