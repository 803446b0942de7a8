/*
 * mpir_oracle.c -- plain, slow CPU oracle for mixed-precision iterative
 * refinement (IR) with an LU factorization in a lower precision.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path links,
 * loads or calls this file: only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the GPU implementation.
 *
 * What it computes, and where the paper defines it (Kelley, "Using
 * MultiPrecisionArrays.jl: Iterative Refinement in Julia", arXiv:2311.14616):
 *
 *   - the interprecision copy A_F = I_W^F(A) and the rounding operator fl_p
 *     (section "Introduction", the notation paragraph after Algorithm IR);
 *   - LU with partial pivoting of A_F in precision TF (Algorithm IR, "Factor
 *     A = LU in precision TF"; Julia's lu!, i.e. LAPACK getrf semantics);
 *   - the IR loop of Algorithm IR with the low-precision solve of
 *     eqs. (vdlow)/(promotevd) (section "Interprecision Transfers: Part I"),
 *     the residual in precision TR by eq. (xferrule) (section "Evaluating the
 *     residual in extended precision") and the termination rules of eqs.
 *     (residterm), (term), (wilkterm), (stag) and litmax (section
 *     "Terminating the while loop").
 *
 * Every floating-point operation is written out and rounded once, in the
 * order the definition states: no FMA contraction (built with
 * -ffp-contract=off), no reassociation, no excess precision (SSE, not x87).
 * Rounding to binary16 is done by orc_fl_h below, written from the IEEE 754
 * definition (round to nearest, ties to even, gradual underflow, overflow to
 * infinity at 65520).  Binary32 rounding is the C conversion (double->float),
 * which is IEEE round-to-nearest-even.  Double rounding through binary32 or
 * binary64 before binary16 is innocuous for +,-,*,/ because 24 >= 2*11+2.
 * Rounding to bfloat16 (the 16-bit format of section "Half Precision": the
 * exponent range of binary32, an 8-bit significand) is done by orc_fl_b,
 * written from the same definition (round to nearest, ties to even, gradual
 * underflow at quantum 2^-133, overflow to infinity at (2 - 2^-8) 2^127);
 * the same double-rounding argument holds since 24 >= 2*8+2.
 *
 * LU modes (how "factor in precision TF" is read for each TF):
 *   ORC_LU_F64       all arithmetic in binary64.
 *   ORC_LU_F32       all arithmetic in binary32.
 *   ORC_LU_F16MIXED  binary16 factors, binary32 working array: when row k
 *                    becomes the pivot row its entries a_kj (j >= k) are
 *                    rounded to binary16; each multiplier is
 *                    fl_h(fl_s(a_ik / a_kk)); the update a_ij - l_ik*u_kj is
 *                    rounded to binary32 (the product of two binary16 values
 *                    is exact in binary32).
 *   ORC_LU_F16STRICT every operation rounded to binary16.
 *   ORC_LU_BF16MIXED as ORC_LU_F16MIXED with bfloat16 factors (fl_b in
 *                    place of fl_h; products of two bfloat16 values are
 *                    exact in binary32 too).
 *
 * Solve modes (precision TS of the triangular solves in the low-precision
 * solve): ORC_TS_F32 (binary32 arithmetic on the factors; the default for
 * TF = F32 and F16), ORC_TS_F64 (binary64; TF = F64), ORC_TS_F16 (every
 * operation rounded to binary16).
 *
 * Parallelism: OpenMP over the rows of one elimination step and over rows of
 * the residual.  Each element still receives its operations in exactly the
 * order above, so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_F64 = 0, ORC_F32 = 1, ORC_F16 = 2, ORC_BF16 = 3 };
enum { ORC_LU_F64 = 0, ORC_LU_F32 = 1, ORC_LU_F16MIXED = 2, ORC_LU_F16STRICT = 3,
       ORC_LU_BF16MIXED = 4 };
enum { ORC_TS_F64 = 0, ORC_TS_F32 = 1, ORC_TS_F16 = 2 };
enum { ORC_OK = 0, ORC_SINGULAR = 1, ORC_ERR_ARG = -1, ORC_ERR_ALLOC = -2,
       ORC_ERR_NONFINITE = -4, ORC_ERR_RANGE = -5 };
enum { ORC_STOP_CONVERGED = 0, ORC_STOP_STAGNATED = 1, ORC_STOP_DSTAGNATED = 2,
       ORC_STOP_LITMAX = 3, ORC_STOP_NONFINITE = 4 };

/* ------------------------------------------------------------------------ */
/* Rounding operators fl_p                                                   */
/* ------------------------------------------------------------------------ */

/* Round a binary64 value to the nearest binary16 value (ties to even). */
double orc_fl_h(double x)
{
    if (isnan(x)) return x;
    double ax = fabs(x);
    if (ax >= 65520.0) return copysign(INFINITY, x);
    if (ax == 0.0) return x;
    int e;
    frexp(ax, &e);                 /* ax = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;                /* floor(log2(ax)) */
    if (ex < -14) ex = -14;        /* subnormal range: fixed quantum 2^-24 */
    double q = ldexp(1.0, ex - 10);
    double m = ax / q;             /* exact: division by a power of two */
    double r = nearbyint(m);       /* round to nearest, ties to even */
    return copysign(r * q, x);
}

/* Round a binary64 value to the nearest bfloat16 value (ties to even). */
double orc_fl_b(double x)
{
    if (isnan(x)) return x;
    double ax = fabs(x);
    if (ax == 0.0) return x;
    int e;
    frexp(ax, &e);                 /* ax = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;                /* floor(log2(ax)) */
    if (ex < -126) ex = -126;      /* subnormal range: fixed quantum 2^-133 */
    double q = ldexp(1.0, ex - 7);
    double m = ax / q;             /* exact: division by a power of two */
    double r = nearbyint(m) * q;   /* round to nearest, ties to even */
    if (r >= ldexp(1.0, 128)) return copysign(INFINITY, x);
    return copysign(r, x);
}

static inline float fl_h(float x) { return (float)orc_fl_h((double)x); }
static inline float fl_b(float x) { return (float)orc_fl_b((double)x); }
static inline double fl_s(double x) { return (double)(float)x; }

void orc_fl_h_array(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_fl_h(in[i]);
}

void orc_fl_b_array(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_fl_b(in[i]);
}

static double unit_roundoff_eps(int p)
{
    /* Julia eps(T): the spacing of T at 1.0, used by the paper's termination. */
    if (p == ORC_F64) return ldexp(1.0, -52);
    if (p == ORC_F32) return ldexp(1.0, -23);
    if (p == ORC_BF16) return ldexp(1.0, -7);
    return ldexp(1.0, -10);
}

static inline double load_tw(const void *A, int tw, int64_t idx)
{
    return tw == ORC_F64 ? ((const double *)A)[idx] : (double)((const float *)A)[idx];
}

/* ------------------------------------------------------------------------ */
/* Interprecision copy A_F = I_W^F(A) and ||A||_inf                          */
/* ------------------------------------------------------------------------ */

/* A: column-major n x n in TW (lda >= n).  af: row-major n x n, receives
 * fl_F(A) as binary64 numbers.  anorm: max_i sum_j |a_ij| in binary64, each
 * row summed in increasing j.  Returns ORC_ERR_NONFINITE if A has a NaN or
 * infinity, ORC_ERR_RANGE if some fl_F(a_ij) overflows. */
int orc_downcast(int64_t n, const void *A, int64_t lda, int tw, int tf,
                 double *af, double *anorm)
{
    if (n < 0 || lda < (n > 0 ? n : 1) || (n > 0 && (!A || !af))) return ORC_ERR_ARG;
    int bad_nf = 0, bad_rg = 0;
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double a = load_tw(A, tw, i + j * lda);
            if (!isfinite(a)) bad_nf = 1;
            double f = a;
            if (tf == ORC_F32) f = fl_s(a);
            else if (tf == ORC_F16) f = orc_fl_h(a);
            else if (tf == ORC_BF16) f = orc_fl_b(a);
            if (isfinite(a) && !isfinite(f)) bad_rg = 1;
            af[i * n + j] = f;
            rs = rs + fabs(a);
        }
        if (rs > amax || isnan(rs)) amax = rs;
    }
    if (anorm) *anorm = amax;
    if (bad_nf) return ORC_ERR_NONFINITE;
    if (bad_rg) return ORC_ERR_RANGE;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting, right-looking (k, then rows i > k, then j > k) */
/* ------------------------------------------------------------------------ */

/* Pivot search: first index of the largest |a_ik|, i >= k (LAPACK i?amax). */
static int64_t pivot_f(const float *a, int64_t n, int64_t k)
{
    int64_t p = k;
    float best = fabsf(a[k * n + k]);
    for (int64_t i = k + 1; i < n; ++i) {
        float v = fabsf(a[i * n + k]);
        if (v > best) { best = v; p = i; }
    }
    return p;
}

static int64_t pivot_d(const double *a, int64_t n, int64_t k)
{
    int64_t p = k;
    double best = fabs(a[k * n + k]);
    for (int64_t i = k + 1; i < n; ++i) {
        double v = fabs(a[i * n + k]);
        if (v > best) { best = v; p = i; }
    }
    return p;
}

/* Progress lines on stderr every 1024 columns when ORC_PROGRESS is set (a
 * long factorization then shows that it is alive); no effect on results. */
static int progress_on(void)
{
    const char *e = getenv("ORC_PROGRESS");
    return e && e[0] == '1';
}

static void progress(int on, int64_t k, int64_t n)
{
    if (on && (k & 1023) == 0) {
        fprintf(stderr, "[oracle] lu column %lld of %lld\n", (long long)k, (long long)n);
        fflush(stderr);
    }
}

static void lu_f64(double *a, int64_t n, int32_t *ipiv, int64_t *info)
{
    const int prog = progress_on();
    for (int64_t k = 0; k < n; ++k) {
        progress(prog, k, n);
        int64_t p = pivot_d(a, n, k);
        ipiv[k] = (int32_t)p;
        if (a[p * n + k] == 0.0) {          /* exact zero pivot: record, skip */
            if (*info == 0) *info = k + 1;
            continue;
        }
        if (p != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
        const double akk = a[k * n + k];
        const double *rk = a + k * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            double *ri = a + i * n;
            double l = ri[k] / akk;
            ri[k] = l;
            for (int64_t j = k + 1; j < n; ++j) {
                double prod = l * rk[j];
                ri[j] = ri[j] - prod;
            }
        }
    }
}

/* mode: ORC_LU_F32, ORC_LU_F16MIXED, ORC_LU_F16STRICT or ORC_LU_BF16MIXED;
 * a holds binary32 numbers (binary16 / bfloat16 values for the half modes). */
static void lu_f32(float *a, int64_t n, int mode, int32_t *ipiv, int64_t *info)
{
    const int prog = progress_on();
    for (int64_t k = 0; k < n; ++k) {
        progress(prog, k, n);
        int64_t p = pivot_f(a, n, k);
        ipiv[k] = (int32_t)p;
        if (p != k && a[p * n + k] != 0.0f)
            for (int64_t j = 0; j < n; ++j) {
                float t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
        if (mode == ORC_LU_F16MIXED)       /* row k is now final: store U in binary16 */
            for (int64_t j = k; j < n; ++j) a[k * n + j] = fl_h(a[k * n + j]);
        if (mode == ORC_LU_BF16MIXED)      /* ... or in bfloat16 */
            for (int64_t j = k; j < n; ++j) a[k * n + j] = fl_b(a[k * n + j]);
        if (a[k * n + k] == 0.0f) {
            if (*info == 0) *info = k + 1;
            continue;
        }
        const float akk = a[k * n + k];
        const float *rk = a + k * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            float *ri = a + i * n;
            float l = ri[k] / akk;
            if (mode == ORC_LU_BF16MIXED) l = fl_b(l);
            else if (mode != ORC_LU_F32) l = fl_h(l);
            ri[k] = l;
            if (mode == ORC_LU_F16STRICT) {
                for (int64_t j = k + 1; j < n; ++j) {
                    float prod = fl_h(l * rk[j]);
                    ri[j] = fl_h(ri[j] - prod);
                }
            } else {
                for (int64_t j = k + 1; j < n; ++j) {
                    float prod = l * rk[j];
                    ri[j] = ri[j] - prod;
                }
            }
        }
    }
}

/* a: row-major n x n (binary64 container holding TF numbers), overwritten by
 * L (unit lower, multipliers below the diagonal) and U.  ipiv[k] = row swapped
 * with row k at step k (0-based).  info = first k+1 with a zero pivot. */
int orc_lu(int64_t n, double *a, int mode, int32_t *ipiv, int64_t *info)
{
    if (n < 0 || (n > 0 && (!a || !ipiv)) || !info) return ORC_ERR_ARG;
    *info = 0;
    if (mode == ORC_LU_F64) {
        lu_f64(a, n, ipiv, info);
    } else {
        float *w = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n * n : 1));
        if (!w) return ORC_ERR_ALLOC;
        for (int64_t t = 0; t < n * n; ++t) w[t] = (float)a[t];
        lu_f32(w, n, mode, ipiv, info);
        for (int64_t t = 0; t < n * n; ++t) a[t] = (double)w[t];
        free(w);
    }
    return *info ? ORC_SINGULAR : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Triangular solves with the factors: y <- U^{-1} L^{-1} P y                */
/* ------------------------------------------------------------------------ */

/* Apply the row interchanges of ipiv, in order, to a vector. */
void orc_apply_pivots(int64_t n, const int32_t *ipiv, double *y)
{
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = ipiv[k];
        if (p != k) { double t = y[k]; y[k] = y[p]; y[p] = t; }
    }
}

/* Column-oriented substitutions.  Forward, unit L: for j ascending,
 * y_i -= l_ij*y_j for i > j.  Backward, U: for j descending, y_j /= u_jj,
 * then y_i -= u_ij*y_j for i < j.  y is already permuted.  ts selects the
 * arithmetic precision. */
void orc_trsv_lu(int64_t n, const double *lu, int ts, double *y)
{
    if (ts == ORC_TS_F64) {
        for (int64_t j = 0; j < n; ++j) {
            double yj = y[j];
            for (int64_t i = j + 1; i < n; ++i) { double p = lu[i * n + j] * yj; y[i] = y[i] - p; }
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            y[j] = y[j] / lu[j * n + j];
            double yj = y[j];
            for (int64_t i = 0; i < j; ++i) { double p = lu[i * n + j] * yj; y[i] = y[i] - p; }
        }
        return;
    }
    float *w = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    if (!w) return;
    for (int64_t i = 0; i < n; ++i) w[i] = (float)y[i];
    if (ts == ORC_TS_F32) {
        for (int64_t j = 0; j < n; ++j) {
            float yj = w[j];
            for (int64_t i = j + 1; i < n; ++i) { float p = (float)lu[i * n + j] * yj; w[i] = w[i] - p; }
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            w[j] = w[j] / (float)lu[j * n + j];
            float yj = w[j];
            for (int64_t i = 0; i < j; ++i) { float p = (float)lu[i * n + j] * yj; w[i] = w[i] - p; }
        }
    } else { /* ORC_TS_F16 */
        for (int64_t j = 0; j < n; ++j) {
            float yj = w[j];
            for (int64_t i = j + 1; i < n; ++i) { float p = fl_h((float)lu[i * n + j] * yj); w[i] = fl_h(w[i] - p); }
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            w[j] = fl_h(w[j] / (float)lu[j * n + j]);
            float yj = w[j];
            for (int64_t i = 0; i < j; ++i) { float p = fl_h((float)lu[i * n + j] * yj); w[i] = fl_h(w[i] - p); }
        }
    }
    for (int64_t i = 0; i < n; ++i) y[i] = (double)w[i];
    free(w);
}

/* Plain solve with given factors: y <- U^{-1} L^{-1} P y. */
void orc_lu_solve(int64_t n, const double *lu, const int32_t *ipiv, int ts, double *y)
{
    orc_apply_pivots(n, ipiv, y);
    orc_trsv_lu(n, lu, ts, y);
}

/* ------------------------------------------------------------------------ */
/* Residual r = b - A x in precision TR (eq. xferrule: promote, then operate) */
/* ------------------------------------------------------------------------ */

/* A column-major in TW, x in TW, b in TW; r (binary64 container) receives
 * fl_R(b_i - sum_j a_ij x_j), the sum accumulated in increasing j in TR. */
void orc_residual(int64_t n, const void *A, int64_t lda, int tw, int tr,
                  const void *b, const void *x, double *r)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (tr == ORC_F64) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double p = load_tw(A, tw, i + j * lda) * load_tw(x, tw, j);
                acc = acc + p;
            }
            r[i] = load_tw(b, tw, i) - acc;
        } else {
            float acc = 0.0f;
            for (int64_t j = 0; j < n; ++j) {
                float p = (float)load_tw(A, tw, i + j * lda) * (float)load_tw(x, tw, j);
                acc = acc + p;
            }
            r[i] = (double)((float)load_tw(b, tw, i) - acc);
        }
    }
}

static double norm_inf(int64_t n, const double *v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a > m || isnan(a)) m = a;
    }
    return m;
}

/* sigma = 2^ceil(log2(m)) for m > 0: the power of two with m/sigma in (1/2, 1]. */
double orc_pow2_ceil(double m)
{
    int e;
    double f = frexp(m, &e);       /* m = f * 2^e, f in [0.5, 1) */
    return f == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

/* ------------------------------------------------------------------------ */
/* Iterative refinement (Algorithm IR with the low-precision solve)         */
/* ------------------------------------------------------------------------ */

/* Inputs: A column-major n x n in TW (lda), b (TW), precisions tw, tf, tr
 * (ORC_F64/F32/F16/BF16), lu_mode, ts, and the termination parameters
 * (Cr, Ce, Rmax, litmax, residterm, tol_rel; tol_rel > 0 replaces C*u_w).
 * Outputs: x (TW), n_iter (number of corrections), stop reason, rhist
 * (n_iter+1 entries: ||b||, then ||r|| after each correction), dhist
 * (n_iter entries, ||d||), out[0..4] = relres, backward error, ||A||,
 * ||b||, ||x|| (all infinity norms, backward error recomputed in binary64),
 * info (first zero pivot).  hist_cap bounds rhist/dhist (>= litmax+1).
 * Returns ORC_OK, ORC_SINGULAR (no refinement done), or a negative error. */
int orc_ir_solve(int64_t n, const void *A, int64_t lda, int tw, int tf, int tr,
                 int lu_mode, int ts, int rhat_prec, const void *b, void *x,
                 double Cr, double Ce, double Rmax, int litmax, int residterm,
                 double tol_rel, int hist_cap,
                 int32_t *n_iter, int32_t *stop, double *rhist, double *dhist,
                 double *out, int64_t *info)
{
    if (n <= 0 || lda < n || !A || !b || !x || !n_iter || !stop || !rhist || !dhist
        || !out || !info || litmax < 1 || hist_cap < litmax + 1)
        return ORC_ERR_ARG;
    *info = 0; *n_iter = 0; *stop = ORC_STOP_CONVERGED;
    double *af = (double *)malloc(sizeof(double) * (size_t)(n * n));
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *xd = (double *)malloc(sizeof(double) * (size_t)n);
    if (!af || !ipiv || !r || !y || !xd) {
        free(af); free(ipiv); free(r); free(y); free(xd); return ORC_ERR_ALLOC;
    }
    int status = ORC_OK;
    double anorm = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(load_tw(b, tw, i))) status = ORC_ERR_NONFINITE;
    if (status == ORC_OK) status = orc_downcast(n, A, lda, tw, tf, af, &anorm);
    if (status == ORC_OK) status = orc_lu(n, af, lu_mode, ipiv, info);
    if (status != ORC_OK) goto done;

    const int wilk = (tr == ORC_F64 && tw != ORC_F64);  /* TR wider than TW */
    const double uw = unit_roundoff_eps(tw);
    const double tol_r = tol_rel > 0.0 ? tol_rel : Cr * uw;
    const double tol_e = tol_rel > 0.0 ? tol_rel : Ce * uw;

    for (int64_t i = 0; i < n; ++i) {
        xd[i] = 0.0;                         /* x = 0 */
        r[i] = load_tw(b, tw, i);            /* r = b */
    }
    const double bnorm = norm_inf(n, r);
    double rnorm = bnorm, xnorm = 0.0;
    int it = 0;
    rhist[0] = rnorm;
    if (rnorm == 0.0) { *stop = ORC_STOP_CONVERGED; goto report; }
    if (!wilk) {
        int conv = residterm ? (rnorm <= tol_r * bnorm)
                             : (rnorm <= tol_e * (bnorm + anorm * xnorm));
        if (conv) { *stop = ORC_STOP_CONVERGED; goto report; }
    }
    for (;;) {
        /* d = sigma * I_F^W( (LU)^{-1} I_W^F(P r / sigma) ) */
        const double sigma = orc_pow2_ceil(rnorm);
        for (int64_t i = 0; i < n; ++i) y[i] = r[i];
        orc_apply_pivots(n, ipiv, y);
        /* the scaled residual in the precision the solve takes it in: TF
           for the low-precision solve, TW for the on-the-fly solve */
        for (int64_t i = 0; i < n; ++i) {
            double s = y[i] / sigma;
            if (rhat_prec == ORC_F32) s = fl_s(s);
            else if (rhat_prec == ORC_F16) s = orc_fl_h(s);
            else if (rhat_prec == ORC_BF16) s = orc_fl_b(s);
            y[i] = s;
        }
        orc_trsv_lu(n, af, ts, y);
        double dnorm = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double d, xn;
            if (tw == ORC_F64) {
                d = sigma * y[i];
                xn = xd[i] + d;
            } else {
                float df = (float)sigma * (float)y[i];
                d = (double)df;
                xn = (double)((float)xd[i] + df);
            }
            double ad = fabs(d);
            if (ad > dnorm || isnan(ad)) dnorm = ad;
            xd[i] = xn;
        }
        dhist[it] = dnorm;
        /* r = b - A x in TR */
        if (tw == ORC_F64) {
            orc_residual(n, A, lda, tw, tr, b, xd, r);
        } else {
            float *xf = (float *)malloc(sizeof(float) * (size_t)n);
            if (!xf) { status = ORC_ERR_ALLOC; goto done; }
            for (int64_t i = 0; i < n; ++i) xf[i] = (float)xd[i];
            orc_residual(n, A, lda, tw, tr, b, xf, r);
            free(xf);
        }
        rnorm = norm_inf(n, r);
        xnorm = norm_inf(n, xd);
        ++it;
        rhist[it] = rnorm;
        if (!isfinite(rnorm) || !isfinite(dnorm)) { *stop = ORC_STOP_NONFINITE; break; }
        if (rnorm == 0.0) { *stop = ORC_STOP_CONVERGED; break; }
        if (!wilk) {
            int conv = residterm ? (rnorm <= tol_r * bnorm)
                                 : (rnorm <= tol_e * (bnorm + anorm * xnorm));
            if (conv) { *stop = ORC_STOP_CONVERGED; break; }
            if (it >= litmax) { *stop = ORC_STOP_LITMAX; break; }
            if (rhist[it] >= Rmax * rhist[it - 1]) { *stop = ORC_STOP_STAGNATED; break; }
        } else {
            if (it >= litmax) { *stop = ORC_STOP_LITMAX; break; }
            if (it >= 2 && dhist[it - 1] >= Rmax * dhist[it - 2]) { *stop = ORC_STOP_DSTAGNATED; break; }
        }
    }
report:
    *n_iter = it;
    for (int64_t i = 0; i < n; ++i) {
        if (tw == ORC_F64) ((double *)x)[i] = xd[i];
        else ((float *)x)[i] = (float)xd[i];
    }
    {
        /* binary64 residual of the returned x for the report */
        if (tw == ORC_F64) orc_residual(n, A, lda, tw, ORC_F64, b, x, r);
        else orc_residual(n, A, lda, tw, ORC_F64, b, x, r);
        double rn = norm_inf(n, r);
        double xn = norm_inf(n, xd);
        out[0] = bnorm > 0.0 ? rn / bnorm : rn;
        out[1] = rn / (anorm * xn + bnorm);
        if (anorm * xn + bnorm == 0.0) out[1] = 0.0;
        out[2] = anorm;
        out[3] = bnorm;
        out[4] = xn;
    }
done:
    free(af); free(ipiv); free(r); free(y); free(xd);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Binary64 reference solve of the promoted problem (I_W^R A) x = I_W^R b    */
/* ------------------------------------------------------------------------ */

int orc_solve_f64(int64_t n, const void *A, int64_t lda, int tw, const void *b,
                  double *x, int64_t *info)
{
    if (n <= 0 || lda < n || !A || !b || !x || !info) return ORC_ERR_ARG;
    double *af = (double *)malloc(sizeof(double) * (size_t)(n * n));
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!af || !ipiv) { free(af); free(ipiv); return ORC_ERR_ALLOC; }
    double anorm;
    int st = orc_downcast(n, A, lda, tw, ORC_F64, af, &anorm);
    if (st == ORC_OK) st = orc_lu(n, af, ORC_LU_F64, ipiv, info);
    if (st == ORC_OK) {
        for (int64_t i = 0; i < n; ++i) x[i] = load_tw(b, tw, i);
        orc_lu_solve(n, af, ipiv, ORC_TS_F64, x);
    }
    free(af); free(ipiv);
    return st;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
