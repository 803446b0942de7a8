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

// Entry `col` of the solution once published with `epoch` (every lane of
// the wave polls its own word; the wave leaves when all have arrived).
template <typename Yt>
__device__ __forceinline__ Yt get_y(const uint64_t *yw, int64_t col, bool valid, uint32_t epoch,
                                    bool &timed_out) {
    constexpr int K = YWords<Yt>::K;
    uint32_t p[K];
#pragma unroll
    for (int q = 0; q < K; ++q) p[q] = 0;
    bool ok = !valid;
    uint64_t spins = 0;
    for (;;) {
        if (!ok) {
            ok = true;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const uint64_t w = __hip_atomic_load(&yw[col * K + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = ok && (uint32_t)(w >> 32) == epoch;
                p[q] = (uint32_t)w;
            }
        }
        if (__all(ok)) break;
        if (++spins > kSpinLimit) { timed_out = true; break; }
        __builtin_amdgcn_s_sleep(1);
    }
    return valid ? YWords<Yt>::from(p) : (Yt)0;
}

template <typename Ft, typename Yt, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(const Ft *__restrict__ LU, int64_t n, int64_t ld,
                                              Yt *__restrict__ y, uint64_t *__restrict__ yw,
                                              TrsvSync *ts, uint32_t *flags, const IrState *st,
                                              int force) {
    if (!force && st->done) return;
    constexpr int K = YWords<Yt>::K;
    __shared__ Yt red[BS][BS + 1];
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

    // wave 0 preloads its row of the diagonal block and of the last
    // dependency block (neither depends on the solution).  Every load below
    // reads a clamped, in-bounds index and the guard is applied to the value,
    // so the loads of a block are all in flight together.  Binary64 solves on
    // binary32 / 16-bit factors keep these rows in binary32 (exact).
    using St = typename std::conditional<(sizeof(Yt) == 8 && sizeof(Ft) < 8), float, Yt>::type;
    St drow[BS], lrow[BS];
    const int64_t lastc = t > 0 ? (int64_t)(LOWER ? t - 1 : nblk - t) * BS : 0;
    if (wv == 0) {
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
    Yt acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = (Yt)0;
    const Ft *base = LU + i0 * ld;
    const int wvs = __builtin_amdgcn_readfirstlane(wv);   // wave-uniform: row offsets stay scalar
    int rsel[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rsel[r] = wvs * 16 + r < rows ? wvs * 16 + r : rows - 1;
    for (int q = 0; q < t - 1 && !timed_out; ++q) {
        const int cb = LOWER ? q : nblk - 1 - q;
        const int64_t col = (int64_t)cb * BS + lane;
        const bool cv = col < n;
        const int64_t cc = cv ? col : n - 1;
        Ft lv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) lv[r] = base[(int64_t)rsel[r] * ld + cc];
        const Yt yv = get_y<Yt>(yw, col, cv, epoch, timed_out);
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += (cv ? (Yt)to_d(lv[r]) : (Yt)0) * yv;
    }
    if (timed_out) s_bad = 1;
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv * 16 + r][lane] = acc[r];
    __syncthreads();

    // ---- phase 2 (wave 0): last dependency block, then the diagonal block ----
    if (wv == 0) {
        Yt s = (Yt)0;
        if (lane < rows)
            for (int c = 0; c < BS; ++c) s += red[lane][c];
        bool to = s_bad != 0;
        if (t > 0 && !to) {
            const Yt yl = get_y<Yt>(yw, lastc + lane, lastc + lane < n, epoch, to);
#pragma unroll
            for (int c = 0; c < BS; ++c) s += (Yt)lrow[c] * bcast(yl, c);
        }
        Yt z = lane < rows ? y[i0 + lane] - s : (Yt)0;
        if (LOWER) {
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                const Yt yj = bcast(z, j);
                if (lane > j) z -= (Yt)drow[j] * yj;
            }
        } else {
#pragma unroll
            for (int j = BS - 1; j >= 0; --j) {
                if (lane == j) z = z / (Yt)drow[j];
                const Yt yj = bcast(z, j);
                if (lane < j) z -= (Yt)drow[j] * yj;
            }
        }
        if (lane < rows) {
            y[i0 + lane] = z;
#pragma unroll
            for (int q = 0; q < K; ++q)
                __hip_atomic_store(&yw[(i0 + lane) * K + q],
                                   ((uint64_t)epoch << 32) | YWords<Yt>::part(z, q),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (to && lane == 0) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0 && s_bad) atomicOr(flags, (uint32_t)DF_TIMEOUT);
}

template <typename Ft, typename Yt>
hipError_t go(const Ft *LU, int64_t n, int64_t ld, Yt *y, uint64_t *yw, TrsvSync *ts, uint32_t *flags,
              const IrState *st, int force, hipStream_t s) {
    const unsigned nblk = (unsigned)((n + BS - 1) / BS);
    k_trsv<Ft, Yt, true><<<nblk, 256, 0, s>>>(LU, n, ld, y, yw, ts, flags, st, force);
    k_trsv<Ft, Yt, false><<<nblk, 256, 0, s>>>(LU, n, ld, y, yw, ts, flags, st, force);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_trsv(int tf, int ysol, const void *LU, int64_t n, int64_t ld, void *y, uint64_t *yw,
                       TrsvSync *ts, uint32_t *flags, const IrState *st, int force, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tf == MPIR_F64) return go<double, double>((const double *)LU, n, ld, (double *)y, yw, ts, flags, st, force, s);
    if (ysol == MPIR_F64) {
        // binary64 substitutions on binary32 / 16-bit factors (MPS)
        if (tf == MPIR_F32) return go<float, double>((const float *)LU, n, ld, (double *)y, yw, ts, flags, st, force, s);
        if (tf == MPIR_BF16) return go<bf16_t, double>((const bf16_t *)LU, n, ld, (double *)y, yw, ts, flags, st, force, s);
        return go<__half, double>((const __half *)LU, n, ld, (double *)y, yw, ts, flags, st, force, s);
    }
    if (tf == MPIR_F32) return go<float, float>((const float *)LU, n, ld, (float *)y, yw, ts, flags, st, force, s);
    if (tf == MPIR_BF16) return go<bf16_t, float>((const bf16_t *)LU, n, ld, (float *)y, yw, ts, flags, st, force, s);
    return go<__half, float>((const __half *)LU, n, ld, (float *)y, yw, ts, flags, st, force, s);
}

}  // namespace mpir
