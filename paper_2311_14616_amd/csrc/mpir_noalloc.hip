// Allocation-free variant of the residual entry point (mpir_residual_noalloc):
// the scratch the residual kernels need -- the iteration-state words the
// norms are reduced into and the per-chunk partial sums -- lives in one
// fixed device array of this library instead of memory allocated per call.
// For callers that cannot allocate device memory.
//
// The array below is a device symbol: in host code its name is a stand-in,
// not a device address.  Its address on each device is looked up once, with
// that device current, by hipGetSymbolAddress, and only that address is
// handed to kernels.
#include <cstring>
#include <mutex>

#include "mpir_internal.h"

using namespace mpir;

namespace {

constexpr int64_t kNoAllocMaxN = MPIR_RESIDUAL_NOALLOC_MAX_N;
constexpr size_t kStateBytes = (sizeof(IrState) + 255) / 256 * 256;
// one binary64 partial sum per row and 256-column chunk at the largest n
constexpr size_t kPartialBytes = (size_t)((kNoAllocMaxN + 255) / 256) * kNoAllocMaxN * 8;
constexpr size_t kScratchBytes = kStateBytes + kPartialBytes;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on first use).
hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

// The state words start at zero on every call (the array keeps the last
// call's contents).  A kernel, not a memset, so that the call can be
// captured in a graph.
__global__ void k_zero_state(unsigned char *p, int bytes) {
    for (int i = threadIdx.x; i < bytes; i += blockDim.x) p[i] = 0;
}

}  // namespace

extern "C" mpir_status mpir_residual_noalloc(int64_t n, const void *dA, int64_t lda, mpir_prec tw,
                                             mpir_prec tr, const void *db, const void *dx, void *dr,
                                             double *rnorm, void *hip_stream) {
    if (n <= 0 || n > kNoAllocMaxN || !dA || !db || !dx || !dr || lda < n) return MPIR_ERR_ARG;
    if (!(tw == MPIR_F64 || tw == MPIR_F32) || !(tr == MPIR_F64 || tr == MPIR_F32)) return MPIR_ERR_ARG;
    if (tw == MPIR_F64 && tr == MPIR_F32) return MPIR_ERR_ARG;              // TR >= TW
    const int nch = residual_chunks(n);
    if (kStateBytes + (size_t)nch * n * 8 > kScratchBytes) return MPIR_ERR_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    void *base = nullptr;
    if (scratch_ptr(&base) != hipSuccess) return MPIR_ERR_HIP;
    unsigned char *b8 = (unsigned char *)base;
    IrState *st = (IrState *)b8;
    double *partial = (double *)(b8 + kStateBytes);
    k_zero_state<<<1, 256, 0, s>>>(b8, (int)sizeof(IrState));
    if (hipGetLastError() != hipSuccess) return MPIR_ERR_HIP;
    if (launch_residual(n, dA, lda, tw, tr, db, dx, dr, partial, nch, st, 1, s) != hipSuccess)
        return MPIR_ERR_HIP;
    if (rnorm) {
        uint64_t bits = 0;
        if (hipMemcpyAsync(&bits, &st->rnorm_bits, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MPIR_ERR_HIP;
        std::memcpy(rnorm, &bits, 8);
    } else if (hipStreamSynchronize(s) != hipSuccess) {
        return MPIR_ERR_HIP;
    }
    return MPIR_OK;
}
