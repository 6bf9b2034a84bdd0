// Layout kernels of the complex-tensor network (gfx950): split planes from
// and to interleaved (re, im) pairs, and the real embedding of a complex
// matrix that the polar update factors.
#include <hip/hip_runtime.h>

#include "complex.h"

namespace ttn {
namespace {

inline unsigned grid_of(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

__global__ void k_deinterleave(const double* __restrict__ z, double* __restrict__ re, double* __restrict__ im,
                               size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = reinterpret_cast<const double2*>(z)[i];
    re[i] = v.x;
    im[i] = v.y;
  }
}

__global__ void k_interleave(const double* __restrict__ re, const double* __restrict__ im, double* __restrict__ z,
                             size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    reinterpret_cast<double2*>(z)[i] = make_double2(re[i], im[i]);
}

// row r of the 2m x 2k embedding (blockIdx.y = r): [Re X | -Im X] for r < m,
// [Im X | Re X] below
__global__ void k_embed(const double* __restrict__ xr, const double* __restrict__ xi, double* __restrict__ y, int m,
                        long long k) {
  const int r = blockIdx.y;
  const bool top = r < m;
  const long long src = (long long)(top ? r : r - m) * k;
  const double* left = top ? xr + src : xi + src;
  const double* right = top ? xi + src : xr + src;
  const double sgn = top ? -1.0 : 1.0;
  double* row = y + (long long)r * 2 * k;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < k; i += (long long)gridDim.x * blockDim.x) {
    row[i] = left[i];
    row[k + i] = sgn * right[i];
  }
}

// row i of the complex m x k matrix nearest to the embedding y (2m x 2k) =
// [[P, Q], [R, S]] among embeddings: re = (P + S) / 2, im = (R - Q) / 2
// (blockIdx.y = i)
__global__ void k_unembed(const double* __restrict__ y, double* __restrict__ re, double* __restrict__ im, int m,
                          long long k) {
  const long long i = blockIdx.y;
  const double* top = y + i * 2 * k;
  const double* bot = y + (i + m) * 2 * k;
  double* r = re + i * k;
  double* c = im + i * k;
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < k; j += (long long)gridDim.x * blockDim.x) {
    r[j] = 0.5 * (top[j] + bot[k + j]);
    c[j] = 0.5 * (bot[j] - top[k + j]);
  }
}

}  // namespace

hipError_t unembed_complex_f64(const double* y, double* xr, double* xi, int m, long long k, hipStream_t s) {
  if (m < 1 || k < 1) return hipSuccess;
  if (m > 65535) return hipErrorInvalidValue;
  const unsigned gx = grid_of((size_t)k) < 64 ? grid_of((size_t)k) : 64;
  hipLaunchKernelGGL(k_unembed, dim3(gx, m), dim3(256), 0, s, y, xr, xi, m, k);
  return hipGetLastError();
}

hipError_t deinterleave_f64(const double* z, double* re, double* im, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_deinterleave, dim3(grid_of(n)), dim3(256), 0, s, z, re, im, n);
  return hipGetLastError();
}

hipError_t interleave_f64(const double* re, const double* im, double* z, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interleave, dim3(grid_of(n)), dim3(256), 0, s, re, im, z, n);
  return hipGetLastError();
}

hipError_t embed_complex_f64(const double* xr, const double* xi, double* y, int m, long long k, hipStream_t s) {
  if (m < 1 || k < 1) return hipSuccess;
  if (2 * m > 65535) return hipErrorInvalidValue;
  const unsigned gx = grid_of((size_t)k) < 64 ? grid_of((size_t)k) : 64;
  hipLaunchKernelGGL(k_embed, dim3(gx, 2 * m), dim3(256), 0, s, xr, xi, y, m, k);
  return hipGetLastError();
}

}  // namespace ttn
