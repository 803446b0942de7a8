// Vector kernels of GMRES-IR (paper: sections "Krylov-IR" and "GMRES-IR"):
// the correction equation A d = r is solved by GMRES left-preconditioned
// with the low-precision factors, P = U^{-1} L^{-1} Pi, all in binary64.
// The Krylov basis V is (m+1) x n, row j = basis vector j.
//
//   k_gather_neg  w_i = -t_{perm_i} (t = -A v from the residual kernel with
//                 b = 0), and the ticket reset of the next substitutions
//   k_dots        out_j = sum_i V_j[i] w_i, j < nv: one workgroup per j,
//                 each thread sums its strided entries in order, then a
//                 fixed reduction tree (the result does not depend on timing)
//   k_sub_combo   w_i -= sum_j c_j V_j[i], j increasing
//   k_scale       out_i = w_i / s
//   k_combo       d_i = sum_j y_j V_j[i], j increasing
//   k_lin3        out_i = (x_i + a y_i) + b z_i (BiCGSTAB's vector updates;
//                 out may alias any input: each thread reads its entries
//                 before writing)
#include "mpir_internal.h"

namespace mpir {
namespace {

constexpr int kKT = 256;

__global__ __launch_bounds__(kKT) void k_gather_neg(int64_t n, const double *__restrict__ t,
                                                    const int32_t *__restrict__ perm,
                                                    double *__restrict__ w, TrsvSync *ts) {
    const int64_t i = (int64_t)blockIdx.x * kKT + threadIdx.x;
    if (i == 0) { ts->ticket_l = 0; ts->done_l = 0; ts->ticket_u = 0; ts->done_u = 0; ts->epoch += 2u; }
    if (i < n) w[i] = -t[perm[i]];
}

__global__ __launch_bounds__(kKT) void k_dots(int64_t n, const double *__restrict__ V, int64_t ldv,
                                              const double *__restrict__ w, double *__restrict__ out) {
    __shared__ double red[kKT];
    const double *v = V + (int64_t)blockIdx.x * ldv;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kKT) acc += v[i] * w[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kKT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kKT) void k_sub_combo(int64_t n, const double *__restrict__ V, int64_t ldv,
                                                   int nv, const double *__restrict__ c,
                                                   double *__restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * kKT + threadIdx.x;
    if (i >= n) return;
    double x = w[i];
    for (int j = 0; j < nv; ++j) x -= c[j] * V[(int64_t)j * ldv + i];
    w[i] = x;
}

__global__ __launch_bounds__(kKT) void k_scale(int64_t n, const double *__restrict__ w, double s,
                                               double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kKT + threadIdx.x;
    if (i < n) out[i] = w[i] / s;
}

__global__ __launch_bounds__(kKT) void k_combo(int64_t n, const double *__restrict__ V, int64_t ldv,
                                               int nv, const double *__restrict__ y,
                                               double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kKT + threadIdx.x;
    if (i >= n) return;
    double x = 0.0;
    for (int j = 0; j < nv; ++j) x += y[j] * V[(int64_t)j * ldv + i];
    d[i] = x;
}

__global__ __launch_bounds__(kKT) void k_lin3(int64_t n, const double *x, double a, const double *y,
                                              double b, const double *z, double *out) {
    const int64_t i = (int64_t)blockIdx.x * kKT + threadIdx.x;
    if (i >= n) return;
    double v = x[i] + a * y[i];
    if (z) v = v + b * z[i];
    out[i] = v;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kKT - 1) / kKT); }

}  // namespace

hipError_t launch_gather_neg(int64_t n, const double *t, const int32_t *perm, double *w,
                             TrsvSync *ts, hipStream_t s) {
    k_gather_neg<<<blocks(n), kKT, 0, s>>>(n, t, perm, w, ts);
    return hipGetLastError();
}

hipError_t launch_dots(int64_t n, const double *V, int64_t ldv, int nv, const double *w,
                       double *out, hipStream_t s) {
    if (nv <= 0) return hipSuccess;
    k_dots<<<(unsigned)nv, kKT, 0, s>>>(n, V, ldv, w, out);
    return hipGetLastError();
}

hipError_t launch_sub_combo(int64_t n, const double *V, int64_t ldv, int nv, const double *c,
                            double *w, hipStream_t s) {
    k_sub_combo<<<blocks(n), kKT, 0, s>>>(n, V, ldv, nv, c, w);
    return hipGetLastError();
}

hipError_t launch_scale(int64_t n, const double *w, double sc, double *out, hipStream_t s) {
    k_scale<<<blocks(n), kKT, 0, s>>>(n, w, sc, out);
    return hipGetLastError();
}

hipError_t launch_combo(int64_t n, const double *V, int64_t ldv, int nv, const double *y, double *d,
                        hipStream_t s) {
    k_combo<<<blocks(n), kKT, 0, s>>>(n, V, ldv, nv, y, d);
    return hipGetLastError();
}

hipError_t launch_lin3(int64_t n, const double *x, double a, const double *y, double b, const double *z,
                       double *out, hipStream_t s) {
    k_lin3<<<blocks(n), kKT, 0, s>>>(n, x, a, y, b, z, out);
    return hipGetLastError();
}

}  // namespace mpir
