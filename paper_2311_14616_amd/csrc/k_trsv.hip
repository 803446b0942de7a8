// Triangular solves with the packed LU factors, d_F = U^{-1} L^{-1} rhat
// (the "d = U^{-1} L^{-1} r" step of Algorithm IR, done in the solve
// precision TS: binary32 arithmetic on binary32, binary16 or bfloat16
// factors, or
// binary64 for the FP64 comparator).
//
// One launch per triangle.  The factor is cut into 64-row block rows; each
// workgroup takes a ticket from an atomic counter (tickets follow dispatch
// order, so a workgroup only waits on workgroups that are already running)
// and owns block row t (from the top for L, from the bottom for U).  It
// streams its block row of the factor (row-major: contiguous, coalesced),
// multiplying each 64-column block by the matching solution block once that
// block is final, then solves its 64 x 64 diagonal block in one wave with
// register broadcasts and publishes its 64 solution entries.  Solution
// entries travel as 64-bit words (32-bit payload | 32-bit epoch, two words
// for binary64): a reader polls the words themselves, so seeing the epoch
// means seeing the value -- no counter, no fences.  Only the last dependency
// block is on the chain: the others are consumed while the previous block
// row is still being solved.  The bytes read are the factor entries of that
// triangle, once.
#include <type_traits>

#include "mpir_internal.h"

namespace mpir {
namespace {

constexpr int BS = 64;

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Yt> __device__ __forceinline__ Yt bcast(Yt v, int lane);
template <> __device__ __forceinline__ float bcast<float>(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <> __device__ __forceinline__ double bcast<double>(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <typename Yt> struct YWords;
template <> struct YWords<float> {
    static constexpr int K = 1;
    __device__ static uint32_t part(float v, int) { return __float_as_uint(v); }
    __device__ static float from(const uint32_t *p) { return __uint_as_float(p[0]); }
};
template <> struct YWords<double> {
    static constexpr int K = 2;
    __device__ static uint32_t part(double v, int q) {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        return q == 0 ? (uint32_t)b : (uint32_t)(b >> 32);
    }
    __device__ static double from(const uint32_t *p) {
        return __longlong_as_double((long long)(((uint64_t)p[1] << 32) | p[0]));
    }
};

// Entry `col` of NR solution columns (column c at yw + c * ystride words)
// once published with `epoch`: every lane of the wave polls its own words,
// the wave leaves when all have arrived.
template <typename Yt, int NR>
__device__ __forceinline__ void get_ys(const uint64_t *yw, int64_t ystride, int64_t col, bool valid,
                                       uint32_t epoch, bool &timed_out, Yt (&out)[NR]) {
    constexpr int K = YWords<Yt>::K;
    uint32_t p[NR][K];
    bool ok[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        ok[c] = !valid;
#pragma unroll
        for (int q = 0; q < K; ++q) p[c][q] = 0;
    }
    uint64_t spins = 0;
    for (;;) {
        bool all = true;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (!ok[c]) {
                bool o = true;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const uint64_t w = __hip_atomic_load(&yw[c * ystride + col * K + q], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    o = o && (uint32_t)(w >> 32) == epoch;
                    p[c][q] = (uint32_t)w;
                }
                ok[c] = o;
            }
            all = all && ok[c];
        }
        if (__all(all)) break;
        if (++spins > kSpinLimit) { timed_out = true; break; }
        __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) out[c] = valid ? YWords<Yt>::from(p[c]) : (Yt)0;
}

// NR right-hand sides at once (columns y + c * ldy, solution words at
// yw + c * n * K): the factor is read once for all of them; phase 1 keeps NR
// sums per row, and in phase 2 wave c solves the diagonal block of column c.
// Each column receives exactly the operations of the one-column solve, in
// the same order.
template <typename Ft, typename Yt, bool LOWER, int NR>
__global__ __launch_bounds__(256) void k_trsv(const Ft *__restrict__ LU, int64_t n, int64_t ld,
                                              Yt *__restrict__ y, int64_t ldy, uint64_t *__restrict__ yw,
                                              TrsvSync *ts, uint32_t *flags, const IrState *st,
                                              int force) {
    static_assert(NR >= 1 && NR <= 4, "one wave per right-hand side in phase 2");
    if (!force && st->done) return;
    constexpr int K = YWords<Yt>::K;
    const int64_t ystride = n * K;
    __shared__ Yt red[NR][BS][BS + 1];
    __shared__ int s_t;
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nblk = (int)((n + BS - 1) / BS);
    const uint32_t epoch = ts->epoch + (LOWER ? 0u : 1u);
    if (tid == 0) { s_t = (int)atomicAdd(LOWER ? &ts->ticket_l : &ts->ticket_u, 1u); s_bad = 0; }
    __syncthreads();
    const int t = s_t;
    if (t >= nblk) return;
    const int blk = LOWER ? t : nblk - 1 - t;
    const int64_t i0 = (int64_t)blk * BS;
    const int rows = (int)((n - i0) < BS ? (n - i0) : BS);
    bool timed_out = false;

    // waves 0 .. NR-1 preload their row of the diagonal block and of the last
    // dependency block (neither depends on the solution).  Every load below
    // reads a clamped, in-bounds index and the guard is applied to the value,
    // so the loads of a block are all in flight together.  Binary64 solves on
    // binary32 / 16-bit factors keep these rows in binary32 (exact).
    using St = typename std::conditional<(sizeof(Yt) == 8 && sizeof(Ft) < 8), float, Yt>::type;
    St drow[BS], lrow[BS];
    const int64_t lastc = t > 0 ? (int64_t)(LOWER ? t - 1 : nblk - t) * BS : 0;
    if (wv < NR) {
        const bool ok = lane < rows;
        const Ft *dr = LU + (i0 + (ok ? lane : rows - 1)) * ld;
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const Ft dv = dr[i0 + (c < rows ? c : rows - 1)];
            const int64_t lc = lastc + c < n ? lastc + c : n - 1;
            const Ft lv = dr[lc];
            drow[c] = (ok && c < rows) ? (St)to_d(dv) : (St)(LOWER ? 0 : 1);
            lrow[c] = (ok && t > 0 && lastc + c < n) ? (St)to_d(lv) : (St)0;
        }
    }

    // ---- phase 1 (all waves): dependency blocks 0 .. t-2 ----
    // rows past the end of the matrix read the last row (their sums are
    // never used); columns past the end read column n-1 and are masked
    Yt acc[NR][16];
#pragma unroll
    for (int c = 0; c < NR; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = (Yt)0;
    const Ft *base = LU + i0 * ld;
    const int wvs = __builtin_amdgcn_readfirstlane(wv);   // wave-uniform: row offsets stay scalar
    int rsel[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rsel[r] = wvs * 16 + r < rows ? wvs * 16 + r : rows - 1;
    // binary32 solves of one right-hand side take two dependency blocks per
    // step (both blocks' loads in flight together), so a workgroup that lags
    // behind the chain catches up faster; the operations and their order
    // are those of one block at a time
    int q = 0;
    if constexpr (sizeof(Yt) == 4 && NR == 1) {
        for (; q + 1 < t - 1 && !timed_out; q += 2) {
            const int cb0 = LOWER ? q : nblk - 1 - q;
            const int cb1 = LOWER ? q + 1 : nblk - 2 - q;
            const int64_t col0 = (int64_t)cb0 * BS + lane, col1 = (int64_t)cb1 * BS + lane;
            const bool cv0 = col0 < n, cv1 = col1 < n;
            const int64_t cc0 = cv0 ? col0 : n - 1, cc1 = cv1 ? col1 : n - 1;
            Ft lv0[16], lv1[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                lv0[r] = base[(int64_t)rsel[r] * ld + cc0];
                lv1[r] = base[(int64_t)rsel[r] * ld + cc1];
            }
            Yt y0[1], y1[1];
            get_ys<Yt, 1>(yw, ystride, col0, cv0, epoch, timed_out, y0);
            get_ys<Yt, 1>(yw, ystride, col1, cv1, epoch, timed_out, y1);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const Yt lvr = cv0 ? (Yt)to_d(lv0[r]) : (Yt)0;
                acc[0][r] = fmadd(lvr, y0[0], acc[0][r]);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const Yt lvr = cv1 ? (Yt)to_d(lv1[r]) : (Yt)0;
                acc[0][r] = fmadd(lvr, y1[0], acc[0][r]);
            }
        }
    }
    for (; q < t - 1 && !timed_out; ++q) {
        const int cb = LOWER ? q : nblk - 1 - q;
        const int64_t col = (int64_t)cb * BS + lane;
        const bool cv = col < n;
        const int64_t cc = cv ? col : n - 1;
        Ft lv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) lv[r] = base[(int64_t)rsel[r] * ld + cc];
        Yt yv[NR];
        get_ys<Yt, NR>(yw, ystride, col, cv, epoch, timed_out, yv);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const Yt lvr = cv ? (Yt)to_d(lv[r]) : (Yt)0;
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c][r] = fmadd(lvr, yv[c], acc[c][r]);
        }
    }
    if (timed_out) s_bad = 1;
#pragma unroll
    for (int c = 0; c < NR; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[c][wv * 16 + r][lane] = acc[c][r];
    __syncthreads();

    // ---- phase 2 (wave c, c < NR): last dependency block, then the
    // diagonal block of column c ----
    if (wv < NR) {
        const int c = wvs;
        Yt s = (Yt)0;
        if (lane < rows)
            for (int k = 0; k < BS; ++k) s += red[c][lane][k];
        bool to = s_bad != 0;
        if (t > 0 && !to) {
            Yt yl[1];
            get_ys<Yt, 1>(yw + c * ystride, ystride, lastc + lane, lastc + lane < n, epoch, to, yl);
#pragma unroll
            for (int k = 0; k < BS; ++k) s = fmadd((Yt)lrow[k], bcast(yl[0], k), s);
        }
        Yt *yc = y + c * ldy;
        Yt z = lane < rows ? yc[i0 + lane] - s : (Yt)0;
        if (LOWER) {
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                const Yt yj = bcast(z, j);
                if (lane > j) z = fmadd(-(Yt)drow[j], yj, z);
            }
        } else {
            // each lane's own diagonal entry u_ll, inverted before the chain
            // (a division on the chain of 64 dependent steps made the upper
            // solve 1.5x slower than the lower one); the entry is then
            // multiplied by it: one rounding more than a division
            St ul = drow[0];
#pragma unroll
            for (int j = 1; j < BS; ++j)
                if (lane == j) ul = drow[j];
            const Yt rinv = (Yt)1 / (Yt)ul;
#pragma unroll
            for (int j = BS - 1; j >= 0; --j) {
                if (lane == j) z = z * rinv;
                const Yt yj = bcast(z, j);
                if (lane < j) z = fmadd(-(Yt)drow[j], yj, z);
            }
        }
        if (lane < rows) {
            yc[i0 + lane] = z;
#pragma unroll
            for (int q = 0; q < K; ++q)
                __hip_atomic_store(&yw[c * ystride + (i0 + lane) * K + q],
                                   ((uint64_t)epoch << 32) | YWords<Yt>::part(z, q),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (to && lane == 0) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0 && s_bad) atomicOr(flags, (uint32_t)DF_TIMEOUT);
}

template <typename Ft, typename Yt, int NR>
hipError_t go(const Ft *LU, int64_t n, int64_t ld, Yt *y, int64_t ldy, uint64_t *yw, TrsvSync *ts,
              uint32_t *flags, const IrState *st, int force, hipStream_t s) {
    const unsigned nblk = (unsigned)((n + BS - 1) / BS);
    k_trsv<Ft, Yt, true, NR><<<nblk, 256, 0, s>>>(LU, n, ld, y, ldy, yw, ts, flags, st, force);
    k_trsv<Ft, Yt, false, NR><<<nblk, 256, 0, s>>>(LU, n, ld, y, ldy, yw, ts, flags, st, force);
    return hipGetLastError();
}

template <typename Ft, typename Yt>
hipError_t go_nr(int nr, const Ft *LU, int64_t n, int64_t ld, Yt *y, int64_t ldy, uint64_t *yw,
                 TrsvSync *ts, uint32_t *flags, const IrState *st, int force, hipStream_t s) {
    if (nr == 1) return go<Ft, Yt, 1>(LU, n, ld, y, ldy, yw, ts, flags, st, force, s);
    if (nr == 2) return go<Ft, Yt, 2>(LU, n, ld, y, ldy, yw, ts, flags, st, force, s);
    if constexpr (sizeof(Yt) == 4) {
        if (nr == 4) return go<Ft, Yt, 4>(LU, n, ld, y, ldy, yw, ts, flags, st, force, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_trsv(int tf, int ysol, const void *LU, int64_t n, int64_t ld, void *y, uint64_t *yw,
                       TrsvSync *ts, uint32_t *flags, const IrState *st, int force, hipStream_t s) {
    return launch_trsv_multi(tf, ysol, 1, LU, n, ld, y, n, yw, ts, flags, st, force, s);
}

int trsv_max_rhs(int ysol) { return ysol == MPIR_F64 ? 2 : 4; }

hipError_t launch_trsv_multi(int tf, int ysol, int nr, const void *LU, int64_t n, int64_t ld, void *y,
                             int64_t ldy, uint64_t *yw, TrsvSync *ts, uint32_t *flags, const IrState *st,
                             int force, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nr < 1 || nr > trsv_max_rhs(ysol == MPIR_F64 || tf == MPIR_F64 ? MPIR_F64 : MPIR_F32) || ldy < n)
        return hipErrorInvalidValue;
    if (tf == MPIR_F64) return go_nr<double, double>(nr, (const double *)LU, n, ld, (double *)y, ldy, yw, ts, flags, st, force, s);
    if (ysol == MPIR_F64) {
        // binary64 substitutions on binary32 / 16-bit factors (MPS)
        if (tf == MPIR_F32) return go_nr<float, double>(nr, (const float *)LU, n, ld, (double *)y, ldy, yw, ts, flags, st, force, s);
        if (tf == MPIR_BF16) return go_nr<bf16_t, double>(nr, (const bf16_t *)LU, n, ld, (double *)y, ldy, yw, ts, flags, st, force, s);
        return go_nr<__half, double>(nr, (const __half *)LU, n, ld, (double *)y, ldy, yw, ts, flags, st, force, s);
    }
    if (tf == MPIR_F32) return go_nr<float, float>(nr, (const float *)LU, n, ld, (float *)y, ldy, yw, ts, flags, st, force, s);
    if (tf == MPIR_BF16) return go_nr<bf16_t, float>(nr, (const bf16_t *)LU, n, ld, (float *)y, ldy, yw, ts, flags, st, force, s);
    return go_nr<__half, float>(nr, (const __half *)LU, n, ld, (float *)y, ldy, yw, ts, flags, st, force, s);
}

}  // namespace mpir
