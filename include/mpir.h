/*
 * mpir.h -- C ABI of an MI355X (gfx950) library for mixed-precision
 * iterative refinement (IR) of dense linear systems A x = b.
 *
 * Method (Kelley, "Using MultiPrecisionArrays.jl: Iterative Refinement in
 * Julia", arXiv:2311.14616, Algorithm IR): copy A from the working precision
 * TW into the factorization precision TF (A_F = I_W^F(A)), factor
 * A_F = P^T L U with partial pivoting, then repeat  d = U^{-1} L^{-1} r,
 * x <- x + d,  r = b - A x  (residual in precision TR)  until a termination
 * rule of section "Terminating the while loop" fires.
 *
 * Conventions shared by every entry point:
 *  - Matrices and vectors passed as `d*` are DEVICE pointers owned by the
 *    caller.  A is column-major (LAPACK / Julia layout) with leading
 *    dimension lda >= n.  Host pointers are named without the `d` prefix.
 *  - Precisions: TW in {F64, F32}; TF in {F32, F16, BF16} below TW, or
 *    TF == TW; TR in {TW, F64} (section "Evaluating the residual in extended
 *    precision").  BF16 is the 16-bit format of section "Half Precision"
 *    (binary32 exponent range, 8-bit significand).
 *  - Every call is ordered on the HIP stream given to mpir_factor (a
 *    hipStream_t passed as void*, NULL = the default stream) and returns
 *    only when its results are in place (it synchronises that stream).
 *  - Errors are returned as mpir_status; nothing aborts.  A failed call
 *    leaves caller-owned outputs unspecified and owned handles valid, except
 *    a failed mpir_refactor, which empties its handle (MPIR_ERR_STATE).
 *  - One handle must not be used by two host threads at once.
 */
#ifndef MPIR_H
#define MPIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPIR_HIST_MAX 64

typedef enum { MPIR_F64 = 0, MPIR_F32 = 1, MPIR_F16 = 2, MPIR_BF16 = 3 } mpir_prec;

typedef enum {
    MPIR_OK = 0,
    MPIR_ERR_SINGULAR = 1,      /* exact zero pivot; *info = its 1-based column */
    MPIR_ERR_ARG = -1,          /* bad size, pointer or precision triple */
    MPIR_ERR_ALLOC = -2,        /* device allocation failed */
    MPIR_ERR_HIP = -3,          /* a HIP runtime call failed */
    MPIR_ERR_NONFINITE = -4,    /* NaN or infinity in A or b */
    MPIR_ERR_RANGE = -5,        /* an entry of A overflows in TF (e.g. |a| >= 65520 for F16) */
    MPIR_ERR_STATE = -6,        /* the handle holds no factorization: its last mpir_refactor failed */
    MPIR_ERR_DEVICE = -7        /* a kernel's bounded inter-workgroup wait expired */
} mpir_status;

typedef enum {
    MPIR_STOP_CONVERGED = 0,    /* eq. residterm or eq. term satisfied (or r == 0) */
    MPIR_STOP_STAGNATED = 1,    /* eq. stag: ||r_new|| >= Rmax ||r_old|| */
    MPIR_STOP_DSTAGNATED = 2,   /* eq. wilkterm: ||d_new|| >= Rmax ||d_old|| (TR wider than TW) */
    MPIR_STOP_LITMAX = 3,       /* litmax corrections done */
    MPIR_STOP_NONFINITE = 4     /* a residual or correction became NaN/Inf */
} mpir_stop;

/* Termination parameters: the paper's TERM structure (Cr, Ce, Rmax, litmax)
 * plus the choice between eq. residterm (residterm = 1) and eq. term
 * (residterm = 0).  tol_rel > 0 replaces the factor C*u_w of either test
 * (u_w = eps(TW): 2^-52 for F64, 2^-23 for F32).
 * onthefly selects the solve of each correction (section "Options and data
 * structures for mplu", the onthefly keyword): 0 = low-precision solve (LPS:
 * the scaled residual is rounded to TF and the substitutions run in binary32
 * on the stored factors); 1 = mixed-precision solve (MPS: the residual stays
 * in TW and the substitutions run in TW arithmetic, the stored TF factors
 * promoted as they are read).  Single-system calls only: the batched calls
 * take LPS and reject onthefly != 0 with MPIR_ERR_ARG. */
typedef struct {
    double Cr, Ce, Rmax;
    int32_t litmax;             /* 1 .. MPIR_HIST_MAX-1 */
    int32_t residterm;
    double tol_rel;
    int32_t onthefly;           /* 0 = LPS, 1 = MPS */
    int32_t reserved;           /* must be 0 */
} mpir_term;

/* Iteration statistics (the paper's reporting=true output: rhist, dhist).
 * n_iter = number of corrections; rhist[0] = ||b||, rhist[k] = ||r|| after
 * correction k; dhist[k-1] = ||d_k||.  All norms are infinity norms. */
typedef struct {
    int32_t n_iter, stop, n_hist, reserved;
    double rhist[MPIR_HIST_MAX], dhist[MPIR_HIST_MAX];
    double relres;              /* ||b - A x|| / ||b|| of the returned x, FP64 */
    double bwd_err;             /* ||b - A x|| / (||A|| ||x|| + ||b||), FP64 */
    double anorm_inf, bnorm_inf, xnorm_inf;
    int64_t info;
    double t_factor_ms, t_ir_ms;
} mpir_report;

typedef struct mpir_fact_s *mpir_fact;

/* Defaults of the paper's term_parms_default: Cr = Ce = 1, Rmax = .5,
 * litmax = 10, residterm = 1, tol_rel = 0; onthefly = 0. */
void mpir_term_default(mpir_term *t);

/* mplu (section "Options and data structures for mplu"): build the
 * multiprecision factorization of the n x n matrix dA (column-major, TW,
 * lda).  Computes A_F = I_W^F(A) and ||A||_inf (FP64), then the blocked
 * right-looking LU with partial pivoting of A_F in TF.
 *  - The handle BORROWS dA: it must stay allocated and unchanged until
 *    mpir_refactor or mpir_destroy (the residual reads it).
 *  - The handle OWNS the TF copy, the pivots and all workspace.  One part
 *    of it, the panel factorization's exchange area (about 205 KB), is
 *    uncached device memory taken from a per-device pool of the library:
 *    mpir_destroy returns it to the pool, not to the runtime, so the pool
 *    holds as many areas as handles were ever alive at once on that device,
 *    until the process ends.
 *  - F16 factorization: binary16 L and U, binary32 trailing matrix (each U
 *    row rounded to binary16 when it becomes final, each multiplier rounded
 *    to binary16 when formed; MFMA products of binary16 operands accumulate
 *    in binary32).  BF16: the same with bfloat16 L and U.
 *  - *out receives the handle also on MPIR_ERR_SINGULAR (*info = first zero
 *    pivot, 1-based, LAPACK semantics: the factorization is completed);
 *    on any other error *out is NULL.
 *  - Size limit: the panel factorization keeps every row of a 32-column
 *    leaf on chip, one or two rows per thread over at most 64 workgroups of
 *    512 threads (no more than the device's compute units), so n <= 65536 for TF in {F32, F16, BF16} and n <= 32768
 *    for TF = F64; a larger n returns MPIR_ERR_ARG.  (An n = 65536 system
 *    in binary64 is 32 GiB, well inside one GPU's memory: the limit is the
 *    leaf's, not the memory's.) */
mpir_status mpir_factor(int64_t n, const void *dA, int64_t lda, mpir_prec tw,
                        mpir_prec tf, mpir_prec tr, void *hip_stream,
                        mpir_fact *out, int64_t *info);

/* mplu!(MPF, B): refactor a matrix of the same size and precisions into an
 * existing handle, reusing its storage.  dA is borrowed as above.  On any
 * failure other than MPIR_ERR_SINGULAR (MPIR_ERR_RANGE, MPIR_ERR_NONFINITE,
 * MPIR_ERR_DEVICE, MPIR_ERR_HIP) the old factors are gone and the handle is
 * marked empty: mpir_solve, mpir_ir_solve, mpir_ir_solve_multi,
 * mpir_gmres_ir_solve, mpir_bicgstab_ir_solve and mpir_get_factors return
 * MPIR_ERR_STATE until a later mpir_refactor succeeds. */
mpir_status mpir_refactor(mpir_fact f, const void *dA, int64_t lda, int64_t *info);

/* One low-precision solve (eqs. vdlow / promotevd):
 * dx = sigma * I_F^W( U^{-1} L^{-1} I_W^F(P db / sigma) ), sigma the power
 * of two with ||db||/sigma in (1/2, 1].  db, dx: n entries in TW. */
mpir_status mpir_solve(mpir_fact f, const void *db, void *dx);

/* Algorithm IR from x = 0 on the factorization f.  db, dx: n entries in TW
 * (dx output only).  t = NULL uses mpir_term_default.  rep (host) may be
 * NULL.  Non-convergence is MPIR_OK with rep->stop != CONVERGED. */
mpir_status mpir_ir_solve(mpir_fact f, const void *db, void *dx,
                          const mpir_term *t, mpir_report *rep);

/* Several right-hand sides with one factorization (sections "Memory
 * Allocations: I", on reusing a factorization, and "Double-Single IR", on
 * solving for many right-hand sides with one factorization): column c of the
 * n x nrhs column-major matrices dB (ldb >= n) and dX (ldx >= n, TW) is
 * refined exactly as mpir_ir_solve refines it alone -- the same operations
 * in the same order, so each column's result and report equal that call's
 * -- but each residual pass reads A once for up to four columns and each
 * pair of triangular solves reads the factors once for up to four columns
 * (two with binary64 solves).  Every column keeps its own termination
 * state; columns that have stopped are not updated.  reps (host, may be
 * NULL): nrhs reports.  Returns MPIR_ERR_NONFINITE if some column of dB is
 * not finite (that column's report says so, the others are solved).
 * Workspace for nrhs columns is allocated in the handle on first use and
 * kept until mpir_destroy. */
mpir_status mpir_ir_solve_multi(mpir_fact f, int32_t nrhs, const void *dB, int64_t ldb, void *dX,
                                int64_t ldx, const mpir_term *t, mpir_report *reps);

/* GMRES-IR (sections "Krylov-IR" and "GMRES-IR"; the package's mpglu): the
 * refinement of mpir_ir_solve, each correction equation A d = r solved by
 * GMRES left-preconditioned with the factors, P = U^{-1} L^{-1} Pi applied
 * in binary64 arithmetic on the TF factors (the on-the-fly solve).  GMRES
 * starts from d = 0, runs at most `basissize` iterations (1..64, no restart;
 * the package's default is 10), orthogonalises by classical Gram-Schmidt
 * applied twice and stops once its estimated preconditioned residual is at
 * most gmres_tol * ||P r||_2 (gmres_tol <= 0: 1e-13).  Requires TR = F64
 * (MPIR_ERR_ARG otherwise); TW = F32 keeps x in binary32 (each correction
 * rounded to binary32 before it is added) and stops by eq. wilkterm, as
 * mpir_ir_solve does when TR is wider than TW.  khist (host, may be NULL): at least
 * t->litmax entries, the GMRES iterations of each correction; rep as for
 * mpir_ir_solve.  Krylov workspace ((basissize + 5) n binary64 numbers) is
 * allocated in the handle on first use and kept until mpir_destroy. */
mpir_status mpir_gmres_ir_solve(mpir_fact f, const void *db, void *dx, const mpir_term *t,
                                int32_t basissize, double gmres_tol, mpir_report *rep,
                                int32_t *khist);

/* BiCGSTAB-IR (section "Krylov-IR"; the package's mpblu): the refinement
 * of mpir_ir_solve, each correction equation A d = r solved by BiCGSTAB
 * preconditioned on the left with the factors, P = U^{-1} L^{-1} Pi applied
 * in binary64 arithmetic on the TF factors (as for mpir_gmres_ir_solve).
 * BiCGSTAB starts from d = 0 with the shadow vector P r, runs at most
 * `maxit` iterations (1..1000; two preconditioned products each) and stops
 * once the norm of its half-step or full-step residual is at most
 * inner_tol * ||P r||_2 (inner_tol <= 0: 1e-13), or on a zero denominator
 * (keeping the last iterate).  Requires TR = F64 (MPIR_ERR_ARG
 * otherwise); TW = F32 as for mpir_gmres_ir_solve.  khist (host, may be NULL): at least t->litmax entries, the
 * BiCGSTAB iterations of each correction; rep as for mpir_ir_solve.  Nine
 * binary64 n-vectors of workspace are allocated in the handle on first use
 * and kept until mpir_destroy. */
mpir_status mpir_bicgstab_ir_solve(mpir_fact f, const void *db, void *dx, const mpir_term *t,
                                   int32_t maxit, double inner_tol, mpir_report *rep,
                                   int32_t *khist);

/* Batched IR for `batch` independent systems of uneven sizes
 * 1 <= n[k] <= 1024 (host array).  dA[k], db[k], dx[k]: host arrays of
 * device pointers (A column-major, lda[k] >= n[k]); same precisions for
 * every system: TW in {F64, F32}, TF in {F32, F16, BF16}, TR = F64 (TW = F32 means
 * TR wider than TW: eq. wilkterm).  Every system is factored and refined on
 * the device in one persistent launch (workgroups take the systems from a
 * queue, largest first).  reps: host array of `batch` reports (may be NULL);
 * reps[k].reserved holds the per-system status (MPIR_OK, MPIR_ERR_SINGULAR
 * with reps[k].info, MPIR_ERR_NONFINITE, MPIR_ERR_RANGE).  Returns MPIR_OK,
 * an argument/runtime error, or the first failing per-system status.  The
 * workspace is allocated and freed by the call. */
mpir_status mpir_ir_solve_batched(int32_t batch, const int64_t *n,
                                  const void *const *dA, const int64_t *lda,
                                  const void *const *db, void *const *dx,
                                  mpir_prec tw, mpir_prec tf, mpir_prec tr,
                                  const mpir_term *t, mpir_report *reps,
                                  void *hip_stream);

/* The same batch as a reusable plan: mpir_batch_create validates, allocates
 * the workspace once and, if use_graph != 0, captures the launch sequence in
 * a hipGraph on hip_stream; mpir_batch_run replays it (or launches it) and
 * copies the reports to the host array reps (NULL: none); mpir_batch_destroy
 * releases it.  The device pointers are borrowed until destroy. */
typedef struct mpir_batch_s *mpir_batch;
mpir_status mpir_batch_create(int32_t batch, const int64_t *n, const void *const *dA,
                              const int64_t *lda, const void *const *db, void *const *dx,
                              mpir_prec tw, mpir_prec tf, mpir_prec tr, const mpir_term *t,
                              int32_t use_graph, void *hip_stream, mpir_batch *out);
mpir_status mpir_batch_run(mpir_batch b, mpir_report *reps);
void mpir_batch_destroy(mpir_batch b);

/* Tuning of the batched kernel.  Systems are grouped into size classes
 * (class k holds nmax[k-1] < n <= nmax[k], nmax increasing, the last one
 * 1024); each class has its own panel width and trailing-update form:
 *  - panel[k]: columns per panel of the blocked LU, 16 or 32 (a wider panel
 *    passes over the trailing matrix fewer times, a narrower one shortens
 *    the in-LDS panel factorization and the triangular solve per panel);
 *  - update[k]: 0 = every 32 x 32 block of A22 -= L21 U12 reads both of its
 *    operands from memory (good load balance on small trailing matrices),
 *    1 = L21 staged in LDS once per panel and each wave keeping one column
 *    block of U12 in registers while it sweeps the block rows;
 *    2 (panel 32 only) = panels in pairs: the first panel of a pair updates
 *    only the second's columns, and after the second one update of rank 64
 *    (form 1 with both panels' L21, staged 512 rows at a time) brings the
 *    rest of the trailing matrix up to date, passing over it half as often.
 * The library keeps one table per (TW, TF) pair for the whole process; it is
 * applied when a batch is created (mpir_batch_create, mpir_ir_solve_batched).
 * ms[k]: the measured time of the chosen configuration on the tuning batch
 * of the class (0 when not measured).  from_cache: 1 when mpir_batch_autotune
 * read the table from its cache file. */
#define MPIR_TUNE_CLASSES 8
typedef struct {
    int32_t nclass, from_cache;
    int32_t nmax[MPIR_TUNE_CLASSES];
    int32_t panel[MPIR_TUNE_CLASSES];
    int32_t update[MPIR_TUNE_CLASSES];
    double ms[MPIR_TUNE_CLASSES];
} mpir_batch_tuning;

/* The current table for (tw, tf) (TW in {F64, F32}, TF in {F32, F16, BF16}). */
mpir_status mpir_batch_get_tuning(mpir_prec tw, mpir_prec tf, mpir_batch_tuning *t);
/* Replace it (t = NULL restores the built-in defaults); MPIR_ERR_ARG if a
 * field is out of range.  Touches no device. */
mpir_status mpir_batch_set_tuning(mpir_prec tw, mpir_prec tf, const mpir_batch_tuning *t);
/* Autotuner: for each size class, time every (panel, update) candidate on a
 * synthetic batch of systems of the class's middle size (diagonally
 * dominant, seeded) on the current device, keep the fastest, install the
 * table and return it in *t (may be NULL).  cache_path (may be NULL): a text
 * file keyed by the device name, compute-unit count, TW and TF; a matching
 * file is read instead of measuring, otherwise it is (re)written after the
 * measurement.  Allocates and frees its own device memory; synchronises
 * hip_stream. */
mpir_status mpir_batch_autotune(mpir_prec tw, mpir_prec tf, const char *cache_path,
                                void *hip_stream, mpir_batch_tuning *t);

/* Release a handle (NULL is allowed). */
void mpir_destroy(mpir_fact f);

/* Text of a status code (static storage). */
const char *mpir_status_str(mpir_status s);

/* ---- Inspection entry points, for testing each step against a reference.
 * They run the same kernels as the calls above. ---- */

/* The interprecision copy A_F = I_W^F(A) (section "Introduction", notation
 * after Algorithm IR): dAF receives fl_F(a_ij) in ROW-major order (n*n
 * entries of TF: double, float or binary16), *anorm (host) = ||A||_inf in
 * FP64, each row summed in increasing column order. */
mpir_status mpir_downcast(int64_t n, const void *dA, int64_t lda, mpir_prec tw,
                          mpir_prec tf, void *dAF, double *anorm, void *hip_stream);

/* Copy the packed factors of f: dLU (device, n*n entries of TF, row-major,
 * unit-lower L below the diagonal, U on and above) and ipiv (host, n int32:
 * row swapped with row k at step k, 0-based). */
mpir_status mpir_get_factors(mpir_fact f, void *dLU, int32_t *ipiv);

/* The residual of eq. xferrule: dr[i] = fl_R(b_i - sum_j a_ij x_j) with A,
 * x, b in TW promoted exactly to TR.  dr: n entries of TR (double or float);
 * *rnorm (host) = ||r||_inf. */
mpir_status mpir_residual(int64_t n, const void *dA, int64_t lda, mpir_prec tw,
                          mpir_prec tr, const void *db, const void *dx, void *dr,
                          double *rnorm, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc):
 * mpir_residual with its scratch -- the norm accumulators and the binary64
 * partial sums of each 256-column chunk -- in a fixed device array of the
 * library (about 8 MiB, held on each GPU the library runs on until the
 * process ends) instead of memory allocated per call.  Same arguments,
 * results and rounding as mpir_residual; n <= MPIR_RESIDUAL_NOALLOC_MAX_N
 * (MPIR_ERR_ARG beyond).  It calls no hipMalloc or hipFree.  Every call on
 * one GPU uses the same array: calls that overlap on one GPU (two streams,
 * two host threads) race and must be serialised by the caller.  Synchronises
 * hip_stream before it returns. */
#define MPIR_RESIDUAL_NOALLOC_MAX_N 16384
mpir_status mpir_residual_noalloc(int64_t n, const void *dA, int64_t lda, mpir_prec tw,
                                  mpir_prec tr, const void *db, const void *dx, void *dr,
                                  double *rnorm, void *hip_stream);

/* Per-kernel timing with HIP events recorded around each launch, on the
 * stream that launch uses.  kind: 0 = trailing-update GEMM (A22 -= L21 U12),
 * 1 = panel factorization (leaves and in-panel updates), 2 = triangular
 * solves, 3 = residual GEMV, 4 = downcast, 5 = row interchanges outside the
 * panel and U12 = L11^{-1} A12.  mpir_prof_get returns the summed duration,
 * the number of timed intervals and the summed algorithmic work (flops for
 * kinds 0 and 2, bytes for 3 and 4, 0 otherwise) since the last reset.  With
 * the look-ahead, intervals of different kinds overlap in time. */
void mpir_prof_enable(int32_t on);
void mpir_prof_reset(void);
mpir_status mpir_prof_get(int32_t kind, double *ms, int64_t *launches, double *work);

/* Device-side phase times of the batched kernel (mpir_ir_solve_batched,
 * mpir_batch_run, the autotuner), summed over its workgroups and over every
 * launch on the current device since the last reset.  ms (host, 7 doubles)
 * receives milliseconds of workgroup time per phase: 0 = the copy
 * A_F = fl_F(A) and ||A||_inf, 1 = panel factorizations, 2 = row interchanges
 * outside the panels, 3 = U rows (U12 = L11^{-1} A12, and in update form 2
 * the first panel's update of the second's rows), 4 = trailing updates, 5 =
 * scaling of the residual and the two triangular solves, 6 = the update of
 * x, the binary64 residual and the termination tests.  Dividing a phase by
 * the number of workgroups (one per compute unit) gives its share of the
 * launch's duration.  reset != 0 clears the counters after reading them (ms
 * may then be NULL).  Synchronises the device. */
#define MPIR_BATCH_PHASES 7
mpir_status mpir_batch_phase_times(double *ms, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* MPIR_H */
