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

template <typename Ft, typename Yt, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(const Ft *__restrict__ LU, int64_t n, int64_t ld,
                                              Yt *__restrict__ y, uint32_t *ticket, uint32_t *done,
                                              uint32_t *flags, const IrState *st, int force) {
    if (!force && st->done) return;
    __shared__ Yt red[BS][BS + 1];
    __shared__ int s_t;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nblk = (int)((n + BS - 1) / BS);
    if (tid == 0) s_t = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int t = s_t;
    if (t >= nblk) return;
    const int blk = LOWER ? t : nblk - 1 - t;
    const int64_t i0 = (int64_t)blk * BS;
    const int rows = (int)((n - i0) < BS ? (n - i0) : BS);

    // ---- off-diagonal blocks, in the order they become final ----
    // Poll `done` with relaxed coherent loads; one acquire fence once new
    // blocks are seen.  All blocks already final are then streamed in groups
    // of four (16 factor rows x 4 blocks of loads in flight per lane).
    Yt acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = (Yt)0;
    bool timed_out = false;
    int q = 0;
    while (q < t) {
        uint32_t avail = 0;
        {
            uint64_t spins = 0;
            for (;;) {
                uint32_t d = 0;
                if (lane == 0) d = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                avail = (uint32_t)__shfl((int)d, 0);
                if (avail > (uint32_t)q) break;
                if (++spins > kSpinLimit) { timed_out = true; break; }
                __builtin_amdgcn_s_sleep(1);
            }
            if (timed_out) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const int qend = (int)avail < t ? (int)avail : t;
        for (; q + 4 <= qend; q += 4) {
            Yt yv[4];
            int64_t col[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int cb = LOWER ? q + u : nblk - 1 - (q + u);
                col[u] = (int64_t)cb * BS + lane;
                yv[u] = col[u] < n ? ld_agent(&y[col[u]]) : (Yt)0;
            }
            const Ft *base = LU + (i0 + wv * 16) * ld;
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
                const Ft *base = LU + (i0 + wv * 16) * ld + col;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (wv * 16 + r < rows) acc[r] += (Yt)to_d(base[(int64_t)r * ld]) * yv;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv * 16 + r][lane] = acc[r];
    __syncthreads();

    // ---- diagonal block in wave 0: lane i owns row i0 + i ----
    if (wv == 0) {
        Yt z = (Yt)0;
        Yt drow[BS];
        if (lane < rows) {
            Yt s = (Yt)0;
            for (int c = 0; c < BS; ++c) s += red[lane][c];
            z = y[i0 + lane] - s;
            const Ft *dr = LU + (i0 + lane) * ld + i0;
#pragma unroll
            for (int c = 0; c < BS; ++c) drow[c] = c < rows ? (Yt)to_d(dr[c]) : (Yt)0;
        } else {
#pragma unroll
            for (int c = 0; c < BS; ++c) drow[c] = (Yt)0;
        }
        if (LOWER) {
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                const Yt yj = __shfl(z, j);
                if (lane > j) z -= drow[j] * yj;
            }
        } else {
#pragma unroll
            for (int j = BS - 1; j >= 0; --j) {
                if (lane == j && lane < rows) z = z / drow[j];
                const Yt yj = __shfl(z, j);
                if (lane < j) z -= drow[j] * yj;
            }
        }
        if (lane < rows) st_agent(&y[i0 + lane], z);
    }
    __syncthreads();
    if (tid == 0) {
        if (timed_out) atomicOr(flags, (uint32_t)DF_TIMEOUT);
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
