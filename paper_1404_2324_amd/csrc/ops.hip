// Single-operation kernels exposing the device building blocks (Kepler drift,
// Hermite encounter minimum) through the C ABI for component checks.
#include "device_math.h"
#include "genga_impl.h"

namespace genga {
namespace {

// One lane per body: Kepler drift of Eq. (9) in universal variables.
__global__ __launch_bounds__(256) void k_op_kepler(double mu, int64_t n,
                                                   const double* __restrict__ x0,
                                                   const double* __restrict__ v0,
                                                   double dt, double* __restrict__ x,
                                                   double* __restrict__ v, int max_iter,
                                                   int* __restrict__ iters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = x0[3 * i], b = x0[3 * i + 1], c = x0[3 * i + 2];
  double d = v0[3 * i], e = v0[3 * i + 1], f = v0[3 * i + 2];
  const int it = kepler_drift(mu, dt, a, b, c, d, e, f, max_iter);
  x[3 * i] = a;
  x[3 * i + 1] = b;
  x[3 * i + 2] = c;
  v[3 * i] = d;
  v[3 * i + 1] = e;
  v[3 * i + 2] = f;
  if (iters) iters[i] = it;
}

// One lane per pair: minimum of the Hermite interpolant, Eqs. (10)-(12).
__global__ __launch_bounds__(256) void k_op_hermite(int64_t n, double dt,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* p = q + 12 * i;
  out[i] = hermite_dmin2(dt, p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8],
                         p[9], p[10], p[11]);
}

}  // namespace

hipError_t op_kepler(double mu, int64_t n, const double* x0, const double* v0,
                     double dt, double* x, double* v, int max_iter, int* iters,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_op_kepler, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mu, n,
                     x0, v0, dt, x, v, max_iter, iters);
  return hipGetLastError();
}

hipError_t op_hermite(int64_t n, double dt, const double* q, double* out,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_op_hermite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                     dt, q, out);
  return hipGetLastError();
}

}  // namespace genga
