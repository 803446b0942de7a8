// Triangular solves with the packed LU factors, d_F = U^{-1} L^{-1} rhat
// (the "d = U^{-1} L^{-1} r" step of Algorithm IR, done in the solve
// precision TS: binary32 arithmetic on binary32 or binary16 factors, or
// binary64 for the FP64 comparator).
//
// One launch per triangle.  The factor is cut into 64-row block rows; each
// workgroup takes a ticket from an atomic counter (tickets follow dispatch
// order, so a workgroup only waits on workgroups that are already running)
// and owns block row t (from the top for L, from the bottom for U).  It
// streams its block row of the factor (row-major: contiguous, coalesced),
// multiplying each 64-column block by the matching solution block as soon
// as the `done` counter says that block is final, then solves its 64 x 64
// diagonal block in one wave with register broadcasts, publishes its 64
// solution entries and advances `done`.  The bytes read are the factor
// entries of that triangle, once.
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

// Wait until `done` exceeds q (relaxed coherent polling, then one acquire
// fence); returns the observed count, or 0 after the spin limit.
__device__ __forceinline__ uint32_t wait_done(uint32_t *done, uint32_t q, int lane, bool &timed_out) {
    uint64_t spins = 0;
    for (;;) {
        uint32_t d = 0;
        if (lane == 0) d = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        d = (uint32_t)__shfl((int)d, 0);
        if (d > q) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return d;
        }
        if (++spins > kSpinLimit) { timed_out = true; return 0; }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <typename Ft, typename Yt, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(const Ft *__restrict__ LU, int64_t n, int64_t ld,
                                              Yt *__restrict__ y, uint32_t *ticket, uint32_t *done,
                                              uint32_t *flags, const IrState *st, int force) {
    if (!force && st->done) return;
    __shared__ Yt red[BS][BS + 1];
    __shared__ int s_t;
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nblk = (int)((n + BS - 1) / BS);
    if (tid == 0) { s_t = (int)atomicAdd(ticket, 1u); s_bad = 0; }
    __syncthreads();
    const int t = s_t;
    if (t >= nblk) return;
    const int blk = LOWER ? t : nblk - 1 - t;
    const int64_t i0 = (int64_t)blk * BS;
    const int rows = (int)((n - i0) < BS ? (n - i0) : BS);
    bool timed_out = false;

    // wave 0 preloads its row of the diagonal block and of the last
    // dependency block (neither depends on the solution)
    Yt drow[BS], lrow[BS];
    const int64_t lastc = t > 0 ? (int64_t)(LOWER ? t - 1 : nblk - t) * BS : 0;
    if (wv == 0) {
        const bool ok = lane < rows;
        const Ft *dr = LU + (i0 + (ok ? lane : 0)) * ld;
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            drow[c] = (ok && c < rows) ? (Yt)to_d(dr[i0 + c]) : (Yt)(LOWER ? 0 : 1);
            lrow[c] = (ok && t > 0 && lastc + c < n) ? (Yt)to_d(dr[lastc + c]) : (Yt)0;
        }
    }

    // ---- phase 1 (all waves): dependency blocks 0 .. t-2, as they become
    // final, streamed four at a time (16 factor rows x 4 blocks per lane) ----
    Yt acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = (Yt)0;
    const int qlast = t - 1;
    int q = 0;
    while (q < qlast) {
        const uint32_t avail = wait_done(done, (uint32_t)q, lane, timed_out);
        if (timed_out) break;
        const int qend = (int)avail < qlast ? (int)avail : qlast;
        const Ft *base = LU + (i0 + wv * 16) * ld;
        for (; q + 4 <= qend; q += 4) {
            Yt yv[4];
            int64_t col[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int cb = LOWER ? q + u : nblk - 1 - (q + u);
                col[u] = (int64_t)cb * BS + lane;
                yv[u] = col[u] < n ? ld_agent(&y[col[u]]) : (Yt)0;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (wv * 16 + r < rows) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (col[u] < n) acc[r] += (Yt)to_d(base[(int64_t)r * ld + col[u]]) * yv[u];
                }
            }
        }
        for (; q < qend; ++q) {
            const int cb = LOWER ? q : nblk - 1 - q;
            const int64_t col = (int64_t)cb * BS + lane;
            if (col < n) {
                const Yt yv = ld_agent(&y[col]);
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (wv * 16 + r < rows) acc[r] += (Yt)to_d(base[(int64_t)r * ld + col]) * yv;
            }
        }
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
            wait_done(done, (uint32_t)qlast, lane, to);
            const Yt yl = (lastc + lane < n && !to) ? ld_agent(&y[lastc + lane]) : (Yt)0;
#pragma unroll
            for (int c = 0; c < BS; ++c) s += lrow[c] * bcast(yl, c);
        }
        Yt z = lane < rows ? y[i0 + lane] - s : (Yt)0;
        if (LOWER) {
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                const Yt yj = bcast(z, j);
                if (lane > j) z -= drow[j] * yj;
            }
        } else {
#pragma unroll
            for (int j = BS - 1; j >= 0; --j) {
                if (lane == j) z = z / drow[j];
                const Yt yj = bcast(z, j);
                if (lane < j) z -= drow[j] * yj;
            }
        }
        if (lane < rows) st_agent(&y[i0 + lane], z);
        if (to && lane == 0) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0) {
        if (s_bad) atomicOr(flags, (uint32_t)DF_TIMEOUT);
        __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename Ft, typename Yt>
hipError_t go(const Ft *LU, int64_t n, int64_t ld, Yt *y, TrsvSync *ts, uint32_t *flags,
              const IrState *st, int force, hipStream_t s) {
    const unsigned nblk = (unsigned)((n + BS - 1) / BS);
    k_trsv<Ft, Yt, true><<<nblk, 256, 0, s>>>(LU, n, ld, y, &ts->ticket_l, &ts->done_l, flags, st, force);
    k_trsv<Ft, Yt, false><<<nblk, 256, 0, s>>>(LU, n, ld, y, &ts->ticket_u, &ts->done_u, flags, st, force);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_trsv(int tf, const void *LU, int64_t n, int64_t ld, void *y, TrsvSync *ts,
                       uint32_t *flags, const IrState *st, int force, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tf == MPIR_F64) return go<double, double>((const double *)LU, n, ld, (double *)y, ts, flags, st, force, s);
    if (tf == MPIR_F32) return go<float, float>((const float *)LU, n, ld, (float *)y, ts, flags, st, force, s);
    return go<__half, float>((const __half *)LU, n, ld, (float *)y, ts, flags, st, force, s);
}

}  // namespace mpir
