// Internal declarations of the MI355X implementation: device-side helpers
// shared by the kernels, launcher prototypes and the handle layout.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/mpir.h"

namespace mpir {

// ---------------------------------------------------------------------------
// Factorization modes (how "factor in precision TF" is carried out).
//   LU_F64   : binary64 everywhere (FP64 MFMA trailing update).
//   LU_F32   : binary32 everywhere (FP32 MFMA trailing update).
//   LU_F16   : binary16 L and U, binary32 trailing matrix, FP16 MFMA with
//              binary32 accumulation; a U row is rounded to binary16 when it
//              becomes final, a multiplier when it is formed.
//   LU_BF16  : the same with bfloat16 L and U (binary32 exponent range, an
//              8-bit significand); BF16 MFMA for the trailing update, FP32
//              MFMA (exact products of bfloat16 numbers) inside the panel.
// ---------------------------------------------------------------------------
enum LuMode { LU_F64 = 0, LU_F32 = 1, LU_F16 = 2, LU_BF16 = 3 };

// Rounding applied to the factors: 0 none, 1 binary16, 2 bfloat16.
constexpr int rd_of_mode(int mode) { return mode == LU_F16 ? 1 : mode == LU_BF16 ? 2 : 0; }

// Device status word bits (sticky, OR-ed by kernels).
enum DevFlag : uint32_t {
    DF_NONFINITE = 1u,   // NaN / Inf in an input
    DF_RANGE = 2u,       // overflow in the downcast
    DF_TIMEOUT = 4u,     // a bounded inter-workgroup wait expired
};

// Iteration state kept in device memory (termination decided on device).
struct IrState {
    double rnorm;        // ||r|| of the latest residual
    double dnorm;        // ||d|| of the latest correction
    double xnorm;        // ||x|| after the latest update
    double bnorm;        // ||b||
    double anorm;        // ||A||_inf (from the downcast)
    double sigma;        // scale of the current low-precision solve
    uint64_t rnorm_bits; // atomic max accumulators (bit patterns of |v| >= 0)
    uint64_t dnorm_bits;
    uint64_t xnorm_bits;
    int32_t it;          // corrections done
    int32_t done;        // 1 once a termination rule fired
    int32_t stop;        // mpir_stop
    int32_t wilk;        // 1: TR wider than TW (eq. wilkterm)
    int32_t residterm;
    int32_t litmax;
    double tol_r, tol_e, rmax;
    double rhist[MPIR_HIST_MAX];
    double dhist[MPIR_HIST_MAX];
};

// Ticket counters of the ordered triangular solves (zeroed per solve) and the
// epoch of the solution words (advanced by 2 per solve, never reset: a word
// written by an earlier solve can never carry the current epoch).
struct TrsvSync {
    uint32_t ticket_l, done_l, ticket_u, done_u;
    uint32_t epoch;
};

// Bounded spin: ~seconds at most; an expired wait raises DF_TIMEOUT and the
// kernel finishes its loop without the data (the host reports an error).
constexpr uint64_t kSpinLimit = 1ull << 26;

// ---------------------------------------------------------------------------
// Rounding helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float round_f16(float x) {
    return __half2float(__float2half_rn(x));
}

// binary64 -> binary32 rounded to odd (truncate, then set the last bit if
// inexact).  Rounding the result to binary16 with ties-to-even then equals
// the direct binary64 -> binary16 rounding (24 >= 11 + 2).
__device__ __forceinline__ float d2f_round_odd(double x) {
    float f = (float)x;
    double back = (double)f;
    if (back != x && !isinf(f)) {
        uint32_t u = __float_as_uint(f);
        if (fabs(back) > fabs(x)) u -= 1u;
        u |= 1u;
        f = __uint_as_float(u);
    } else if (isinf(f) && !isinf(x)) {
        // |x| beyond binary32: certainly beyond binary16 as well
        f = x > 0 ? INFINITY : -INFINITY;
    }
    return f;
}

__device__ __forceinline__ float d2h_as_float(double x) {
    return round_f16(d2f_round_odd(x));
}

// binary32 -> bfloat16 (round to nearest, ties to even, on the bit pattern:
// adding 0x7fff plus the lowest kept bit carries into the kept bits exactly
// when the dropped half is above the midpoint, or at it with the kept part
// odd; a carry out of the significand raises the exponent, up to infinity).
__device__ __forceinline__ float round_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return x;             // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// binary64 -> bfloat16 rounded once (round to odd to binary32 first:
// 24 >= 8 + 2).
__device__ __forceinline__ float d2bf_as_float(double x) {
    return round_bf16(d2f_round_odd(x));
}

template <int RD> __device__ __forceinline__ float round_lo(float x) {
    return RD == 1 ? round_f16(x) : RD == 2 ? round_bf16(x) : x;
}

// bfloat16 storage (the upper half of a binary32 pattern).
struct bf16_t { uint16_t u; };
__device__ __forceinline__ float bf16_to_f(bf16_t v) { return __uint_as_float((uint32_t)v.u << 16); }

// Fused multiply-add a*b + c, rounded once.  Written out where the same sum
// is computed by several kernels (or instantiations) that must agree bit for
// bit: left to the compiler, contraction depends on the surrounding code.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_d<__half>(__half v) { return (double)__half2float(v); }
template <> __device__ __forceinline__ double to_d<bf16_t>(bf16_t v) { return (double)bf16_to_f(v); }
template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }
template <> __device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float to_f<bf16_t>(bf16_t v) { return bf16_to_f(v); }

// Atomic max of a non-negative double through its bit pattern (IEEE order of
// non-negative doubles equals the unsigned order of their bits; NaN maps to a
// pattern above every finite value and infinity).
// Maximum of a 64-bit key over the wave: DPP row shifts by 1, 2, 4, 8 inside
// rows of 16 lanes, then the row broadcasts of lanes 15 and 31 (lanes that
// receive nothing keep 0, the identity for keys >= 0); lane 63 ends with the
// maximum, which readlane makes uniform.
template <int CTRL, int RM>
__device__ __forceinline__ uint64_t dpp_max_u64_step(uint64_t k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)k, CTRL, RM, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k >> 32), CTRL, RM, 0xf, false);
    const uint64_t t = ((uint64_t)hi << 32) | lo;
    return t > k ? t : k;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t k) {
    k = dpp_max_u64_step<0x111, 0xf>(k);
    k = dpp_max_u64_step<0x112, 0xf>(k);
    k = dpp_max_u64_step<0x114, 0xf>(k);
    k = dpp_max_u64_step<0x118, 0xf>(k);
    k = dpp_max_u64_step<0x142, 0xa>(k);
    k = dpp_max_u64_step<0x143, 0xc>(k);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void atomic_max_nonneg(uint64_t *p, double v) {
    uint64_t bits = __double_as_longlong(v);
    atomicMax((unsigned long long *)p, (unsigned long long)bits);
}

// ---------------------------------------------------------------------------
// Host-side launchers (each defined in the .hip file holding its kernel).
// All take the stream explicitly; none synchronises.
// ---------------------------------------------------------------------------

// A_F = I_W^F(A) into a row-major working array (float for TF in
// {F32, F16}; double for F64), ||A||_inf bits and status flags.
hipError_t launch_downcast(int64_t n, const void *A, int64_t lda, int tw, int tf,
                           void *AF, int64_t ldf, uint64_t *anorm_bits, uint32_t *flags,
                           hipStream_t s);
// Working array (row pitch ldf) -> n x n 16-bit factors (row pitch ldl):
// binary16 for tf = MPIR_F16, bfloat16 for MPIR_BF16.
hipError_t launch_pack_half(int tf, int64_t n, const float *AF, int64_t ldf, void *LU, int64_t ldl,
                            hipStream_t s);
// Working array -> TF storage with the given row-major layout (copy).
hipError_t launch_copy_factors(int64_t n, const void *src, int tf, void *dst, hipStream_t s);

// Leaf panel factorization: rows [k0, n), columns [k0, k0+w), w <= 32.
// ipiv receives 0-based global row indices.  host_base: host copy of the
// exchange epoch of ps (advanced per launch).
struct PanelSync;
hipError_t launch_leaf(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int w,
                       int32_t *ipiv, int64_t *info, PanelSync *ps, uint32_t *host_base,
                       uint32_t *flags, hipStream_t s);
int leaf_max_rows(int mode);
size_t panel_sync_bytes();
hipError_t panel_sync_reset(PanelSync *ps, hipStream_t s);

// Row interchanges ipiv[k0 .. k0+cnt) applied to the column ranges
// [c0, c1) and [c2, c3); perm (may be NULL) permuted alongside.  compact:
// small LDS tiles (fits beside a running trailing update).
hipError_t launch_laswp(int mode, void *a, int64_t n, int64_t ld, int64_t k0, int cnt,
                        const int32_t *ipiv, int64_t c0, int64_t c1, int64_t c2,
                        int64_t c3, int32_t *perm, bool compact, hipStream_t s);
// U12 <- L11^{-1} U12 for rows [k, k+w) (w <= 32), columns [c0, c1).
hipError_t launch_trsm(int mode, void *a, int64_t ld, int64_t k, int w, int64_t c0,
                       int64_t c1, hipStream_t s);
// a3 for a narrow column range: U12 <- L11^{-1} U12 for rows [k, k+w),
// w <= u12_max_rows(), columns [c0, c1), in one launch.
int u12_max_rows();
hipError_t launch_u12(int mode, void *a, int64_t ld, int64_t k, int w, int64_t c0, int64_t c1,
                      hipStream_t s);
// Trailing update C[r0:r0+m, c0:c0+nc] -= A[r0:, k:k+kk] * A[k:k+kk, c0:] on one
// row-major matrix (ld).  cap > 0: at most cap workgroups per compute unit
// (the rest of each unit stays free for work on another stream).  role: 0 =
// trailing update, 1 = update inside a panel or a U12 block (a separate
// kernel symbol, so that profiles tell them apart).
hipError_t launch_gemm_update(int mode, void *a, int64_t ld, int64_t r0, int64_t m,
                              int64_t c0, int64_t nc, int64_t k, int64_t kk, int cap,
                              int role, hipStream_t s);
// a4, TF = F16 or BF16 (mode): the same trailing update with L21 and U12
// first packed into 16-bit copies (k contiguous) in the workspaces wa
// (>= gemm_h16_ws_halves(m, kk) elements) and wb (>= gemm_h16_ws_halves(nc,
// kk) elements).
size_t gemm_h16_ws_halves(int64_t rows, int64_t kk);
hipError_t launch_gemm_update_h16(int mode, float *a, int64_t ld, int64_t r0, int64_t m, int64_t c0,
                                  int64_t nc, int64_t k, int64_t kk, void *wa, void *wb,
                                  int cap, hipStream_t s);

// Residual r = b - A x in TR, partial sums over column chunks then a
// fixed-order reduction; ||r|| and ||x|| bits into the state.
hipError_t launch_residual(int64_t n, const void *A, int64_t lda, int tw, int tr,
                           const void *b, const void *x, void *r, double *partial,
                           int nchunks, IrState *st, int force, hipStream_t s);
int residual_chunks(int64_t n);
// r = b - A x with A in TW and b, x, r in binary64 (force = 1).
hipError_t launch_residual_x64(int64_t n, const void *A, int64_t lda, int tw, const double *b,
                               const double *x, double *r, double *partial, int nch, IrState *st,
                               hipStream_t s);
// The residual of nr <= 4 right-hand sides (columns b + c * ldb, x + c * ldx,
// r + c * n; states st + c) with one pass over A; partial: nr * nch * n.
hipError_t launch_residual_multi(int64_t n, const void *A, int64_t lda, int tw, int tr, int nr,
                                 const void *b, int64_t ldb, const void *x, int64_t ldx, void *r,
                                 double *partial, int nch, IrState *st, int force, hipStream_t s);

// IR vector steps.
hipError_t launch_ir_init(int64_t n, int tw, int tr, const void *b, void *x, void *r,
                          IrState *st, hipStream_t s);
hipError_t launch_set_sigma(IrState *st, hipStream_t s);
hipError_t launch_scale_permute(int64_t n, int tr, int tf, const void *r,
                                const int32_t *perm, void *rhat, IrState *st,
                                TrsvSync *ts, int force, hipStream_t s);
hipError_t launch_update(int64_t n, int tw, int tf, const void *y, void *x,
                         IrState *st, int force, hipStream_t s);
hipError_t launch_terminate(IrState *st, hipStream_t s);

// Batched refinement of uneven systems in one persistent launch.
struct BatchSys;
struct BatchTerm;
int batched_max_n();
// Phases of the batched kernel with device timers: downcast, panel
// factorization, interchanges, U rows, trailing update, substitutions,
// residual and update of x.  batched_phase_ticks copies the accumulated
// wall-clock ticks (summed over workgroups) and optionally resets them.
constexpr int kBatchPhases = 7;
hipError_t batched_phase_ticks(unsigned long long *out, bool reset);
// Per-system configuration word of the batched kernel for a system of size n
// (panel width | update form << 8) from the tuning table tab, or from the
// process-wide table for (tw, tf) when tab is NULL.
int64_t batch_cfg(int tw, int tf, int64_t n, const mpir_batch_tuning *tab);
hipError_t launch_batched(int tw, int tf, const BatchSys *sys, const int32_t *order, int nsys,
                          uint32_t *queue, const BatchTerm &term, mpir_report *reps, int nwg,
                          hipStream_t s);

// Triangular solves with the packed factors (row-major, TF storage).
// y is float for TF in {F32, F16}, double for F64.
// yw: n * 2 epoch-tagged 64-bit words (zeroed once at allocation).
hipError_t launch_trsv(int tf, int ysol, const void *LU, int64_t n, int64_t ld, void *y, uint64_t *yw,
                       TrsvSync *ts, uint32_t *flags, const IrState *st, int force,
                       hipStream_t s);
// The same for nr right-hand sides at once (columns y + c * ldy, c < nr <=
// trsv_max_rhs(TS); solution words yw + c * n * 2): the factors are read once.
int trsv_max_rhs(int ysol);
hipError_t launch_trsv_multi(int tf, int ysol, int nr, const void *LU, int64_t n, int64_t ld, void *y,
                             int64_t ldy, uint64_t *yw, TrsvSync *ts, uint32_t *flags, const IrState *st,
                             int force, hipStream_t s);

// GMRES-IR vector kernels (binary64; V holds basis vectors in rows of ldv).
hipError_t launch_gather_neg(int64_t n, const double *t, const int32_t *perm, double *w,
                             TrsvSync *ts, hipStream_t s);
hipError_t launch_dots(int64_t n, const double *V, int64_t ldv, int nv, const double *w,
                       double *out, hipStream_t s);
hipError_t launch_sub_combo(int64_t n, const double *V, int64_t ldv, int nv, const double *c,
                            double *w, hipStream_t s);
hipError_t launch_scale(int64_t n, const double *w, double divisor, double *out, hipStream_t s);
hipError_t launch_combo(int64_t n, const double *V, int64_t ldv, int nv, const double *y, double *d,
                        hipStream_t s);
// out = (x + a y) + b z (z may be NULL); out may alias the inputs.
hipError_t launch_lin3(int64_t n, const double *x, double a, const double *y, double b, const double *z,
                       double *out, hipStream_t s);

}  // namespace mpir

// Batch creation with an explicit tuning table (NULL: the process-wide one).
mpir_status batch_create_with(int32_t batch, const int64_t *n, const void *const *dA,
                              const int64_t *lda, const void *const *db, void *const *dx,
                              mpir_prec tw, mpir_prec tf, mpir_prec tr, const mpir_term *t,
                              int32_t use_graph, void *hip_stream, const mpir_batch_tuning *tab,
                              mpir_batch *out);

