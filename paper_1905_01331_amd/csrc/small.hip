// Element-wise kernels, deterministic reductions, the counter-based Gaussian
// generator and the float64 Jacobi eigensolver used by the polar update.
#include "common.h"
#include "jacobi.h"
#include <math.h>

namespace ttn {

GroupCtx& grp() {
  static thread_local GroupCtx g;
  return g;
}

namespace {

inline int grid_for(size_t n, int threads = 256, int cap = 8192) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (size_t)cap) b = cap;
  return (int)b;
}

__global__ void k_f64_to_f32(const double* __restrict__ x, float* __restrict__ y, size_t n, long long ms_) {
  x = mshift(x, ms_); y = mshift(y, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void k_f32_to_f64(const float* __restrict__ x, double* __restrict__ y, size_t n, long long ms_) {
  x = mshift(x, ms_); y = mshift(y, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}
template <typename T>
__global__ void k_fill(T* __restrict__ x, T v, size_t n, long long ms_) {
  x = mshift(x, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = v;
}
__global__ void k_copy(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, size_t n, long long ms_) {
  src = mshift(src, ms_); dst = mshift(dst, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_copy8(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, size_t n, long long ms_,
                        const int* sk = nullptr) {
  if (member_skipped(sk, ms_)) return;
  src = mshift(src, ms_); dst = mshift(dst, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_copy8_if(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, size_t n, const int* flag,
                           int want, long long ms_) {
  src = mshift(src, ms_); dst = mshift(dst, ms_); flag = mshift(flag, ms_);
  if (*flag != want) return;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) dst[i] = src[i];
}
__global__ void k_set_flag_le(int* flag, const int* info, int limit, long long ms_) {
  flag = mshift(flag, ms_); info = mshift(info, ms_);
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = info[0] <= limit ? 1 : 0;
}
__global__ void k_note_negative_info(const int* info, int nq, double* err, double* noconv, int limit, long long ms_) {
  info = mshift(info, ms_); err = mshift(err, ms_); noconv = mshift(noconv, ms_);
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < nq; ++q) {
    if (info[2 * q] < 0) err[0] = 1.0;
    if (noconv && info[2 * q] >= limit) noconv[0] = 1.0;
  }
}
__global__ void k_add_diag(double* X, int n, double v, long long ms_) {
  X = mshift(X, ms_);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) X[(size_t)i * n + i] += v;
}
template <typename T>
__global__ void k_axpby(const T* __restrict__ x, T* __restrict__ y, T alpha, T beta, size_t n, long long ms_) {
  x = mshift(x, ms_); y = mshift(y, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + (beta == T(0) ? T(0) : beta * y[i]);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__global__ void k_gaussian(double* __restrict__ x, size_t n, uint64_t seed, uint64_t stream_id, long long ms_) {
  x = mshift(x, ms_);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint64_t base = splitmix64(seed ^ splitmix64(stream_id + 0x632be59bd9b4e019ull));
    uint64_t r1 = splitmix64(base + 2 * (uint64_t)i);
    uint64_t r2 = splitmix64(base + 2 * (uint64_t)i + 1);
    // uniforms in (0, 1]
    double u1 = ((double)(r1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(r2 >> 11) * (1.0 / 9007199254740992.0);
    x[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);  // Box-Muller
  }
}

// Deterministic two-stage reductions: fixed grid, per-block partials, one
// final block summing the partials in order.
constexpr int RED_BLOCKS = 256;
constexpr int RED_THREADS = 256;

template <typename T>
__device__ double block_sum(double v, double* sh) {
  int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_pair_partial(const T* __restrict__ X, const T* __restrict__ Y,
                                                              long long n, double* __restrict__ part, long long ms_,
                                                              const int* sk) {
  if (member_skipped(sk, ms_)) return;
  X = mshift(X, ms_); Y = mshift(Y, ms_); part = mshift(part, ms_);
  __shared__ double sh[RED_THREADS];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    acc += (double)X[i] * (double)Y[i];
  double s = block_sum<T>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(RED_THREADS) void k_sum_partials(const double* __restrict__ part, int np,
                                                              double* __restrict__ out, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  part = mshift(part, ms_); out = mshift(out, ms_);
  __shared__ double sh[RED_THREADS];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  double s = block_sum<double>(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

// out[r os + oo] = beta out[r os + oo] + sum_i X[r sX + i] Y[r sY + i]: one
// work-group per row, a fixed summation order (no atomics)
__global__ __launch_bounds__(RED_THREADS) void k_pair_rows(const double* __restrict__ X, long long sX,
                                                           const double* __restrict__ Y, long long sY, long long len,
                                                           double* __restrict__ out, long long os, long long oo,
                                                           double beta) {
  const long long r = blockIdx.x;
  __shared__ double sh[RED_THREADS];
  const double* x = X + r * sX;
  const double* y = Y + r * sY;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < len; i += blockDim.x) acc += x[i] * y[i];
  double s = block_sum<double>(acc, sh);
  if (threadIdx.x == 0) {
    double* o = out + r * os + oo;
    *o = (beta == 0.0) ? s : beta * *o + s;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_ortho_err(const double* __restrict__ G, int n, double* out, long long ms_) {
  G = mshift(G, ms_); out = mshift(out, ms_);
  __shared__ double sh[RED_THREADS];
  double acc = 0.0;
  long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < nn; i += blockDim.x) {
    int r = (int)(i / n), c = (int)(i - (long long)r * n);
    double e = G[i] - (r == c ? 1.0 : 0.0);
    acc += e * e;
  }
  double s = block_sum<double>(acc, sh);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

__global__ __launch_bounds__(RED_THREADS) void k_row_normalize(const double* __restrict__ Y, double* __restrict__ Z,
                                                               double* __restrict__ nrm, long long k, long long ms_) {
  Y = mshift(Y, ms_); Z = mshift(Z, ms_); nrm = mshift(nrm, ms_);
  __shared__ double sh[RED_THREADS];
  const double* y = Y + (long long)blockIdx.x * k;
  double* z = Z + (long long)blockIdx.x * k;
  // scaled sum of squares: first the max magnitude, then sum (y/max)^2
  double mx = 0.0;
  for (long long i = threadIdx.x; i < k; i += blockDim.x) mx = fmax(mx, fabs(y[i]));
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  mx = sh[0];
  __syncthreads();
  double acc = 0.0;
  if (mx > 0.0) {
    double inv = 1.0 / mx;
    for (long long i = threadIdx.x; i < k; i += blockDim.x) {
      double t = y[i] * inv;
      acc += t * t;
    }
  }
  double ss = block_sum<double>(acc, sh);
  double norm = mx * sqrt(ss);
  if (threadIdx.x == 0) nrm[blockIdx.x] = norm;
  double inv = norm > 0.0 ? 1.0 / norm : 0.0;
  for (long long i = threadIdx.x; i < k; i += blockDim.x) z[i] = y[i] * inv;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver (parallel round-robin ordering), float64.
// Rotations from jacobi_rotation (common.h): G <- J^T G J, V <- V J,
// J = [[c, s], [-s, c]] on (p, q); the eigenvectors are returned as the ROWS
// of U = V^T.  All n/2 rotations of one round touch disjoint index pairs, so
// the 2x2 blocks of J^T G J are independent.
// ---------------------------------------------------------------------------
constexpr int JAC_THREADS = 1024;
constexpr int JAC_MAXN = 1024;

// MODE 0: G and U in global memory; 1: G copied into dynamic LDS; 2: G and U
// both in dynamic LDS (copied back at the end).  The rotations of a round
// (c, s, t and the index pair, n/2 of each) follow the matrices in the
// dynamic LDS, sized for n.
template <int MODE>
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(double* __restrict__ Gg, double* __restrict__ Vg, int n,
                                                        int max_sweeps, double tol, int* info, const int* skip, long long ms_) {
  Gg = mshift(Gg, ms_); Vg = mshift(Vg, ms_); info = mshift(info, ms_); skip = mshift(skip, ms_);
  if (skip && *skip) {
    if (threadIdx.x == 0 && info) { info[0] = 0; info[1] = 0; }
    return;
  }
  extern __shared__ double dyn[];
  constexpr bool LDS = MODE >= 1;
  const int N = n + (n & 1);   // even number of players; index n is a dummy when n is odd
  const int npair = N / 2;
  const long long mats = (long long)MODE * n * n;  // doubles of matrices in LDS
  double* V = (MODE == 2) ? dyn + (long long)n * n : Vg;
  double* cs = dyn + mats;
  double* sn = cs + npair;
  double* tn = sn + npair;
  int* pp = reinterpret_cast<int*>(tn + npair);
  int* qq = pp + npair;
  __shared__ int rot_count;
  const int tid = threadIdx.x;
  double* G = LDS ? dyn : Gg;
  for (long long i = tid; i < (long long)n * n; i += blockDim.x) {
    int r = (int)(i / n), c = (int)(i - (long long)r * n);
    V[i] = (r == c) ? 1.0 : 0.0;
    if (LDS) G[i] = Gg[i];
  }
  __syncthreads();
  int sweep = 0, first_rot = -1;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rot_count = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int k = tid; k < npair; k += blockDim.x) {
        int p, q;
        if (k == 0) { p = r; q = N - 1; }
        else { p = (r + k) % (N - 1); q = (r - k + (N - 1)) % (N - 1); }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
          double gpp = G[(long long)p * n + p], gqq = G[(long long)q * n + q], gpq = G[(long long)p * n + q];
          if (jacobi_rotation(gpp, gqq, gpq, tol, c, s, t)) atomicAdd(&rot_count, 1);
        }
        pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s; tn[k] = t;
      }
      __syncthreads();
      for (long long idx = tid; idx < (long long)npair * npair; idx += blockDim.x) {
        int k1 = (int)(idx / npair), k2 = (int)(idx - (long long)k1 * npair);
        double s1 = sn[k1], s2 = sn[k2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
        double c1 = cs[k1], c2 = cs[k2];
        bool hq1 = q1 < n, hq2 = q2 < n;
        double gpp = G[(long long)p1 * n + p2];
        double gpq = hq2 ? G[(long long)p1 * n + q2] : 0.0;
        double gqp = hq1 ? G[(long long)q1 * n + p2] : 0.0;
        double gqq = (hq1 && hq2) ? G[(long long)q1 * n + q2] : 0.0;
        // rows: (J1^T G)
        double rp_p = c1 * gpp - s1 * gqp, rp_q = c1 * gpq - s1 * gqq;
        double rq_p = s1 * gpp + c1 * gqp, rq_q = s1 * gpq + c1 * gqq;
        // columns: (. J2)
        double npp = c2 * rp_p - s2 * rp_q, npq = s2 * rp_p + c2 * rp_q;
        double nqp = c2 * rq_p - s2 * rq_q, nqq = s2 * rq_p + c2 * rq_q;
        if (k1 == k2 && s1 != 0.0) {
          // the rotated pair itself: exact annihilation, Rutishauser's diagonal update
          double t1 = tn[k1];
          npp = gpp - t1 * gpq;
          nqq = gqq + t1 * gpq;
          npq = 0.0;
          nqp = 0.0;
        }
        G[(long long)p1 * n + p2] = npp;
        if (hq2) G[(long long)p1 * n + q2] = npq;
        if (hq1) G[(long long)q1 * n + p2] = nqp;
        if (hq1 && hq2) G[(long long)q1 * n + q2] = nqq;
      }
      // rows p, q of U = V^T (eigenvectors as rows): coalesced along i
      for (long long idx = tid; idx < (long long)n * npair; idx += blockDim.x) {
        int k = (int)(idx / n), i = (int)(idx - (long long)k * n);
        double c = cs[k], s = sn[k];
        if (s == 0.0) continue;
        int p = pp[k], q = qq[k];
        double up = V[(long long)p * n + i], uq = V[(long long)q * n + i];
        V[(long long)p * n + i] = c * up - s * uq;
        V[(long long)q * n + i] = s * up + c * uq;
      }
      __syncthreads();
    }
    int rc = rot_count;
    if (first_rot < 0) first_rot = rc;
    __syncthreads();
    if (rc == 0) break;
  }
  if (LDS) {
    for (long long i = tid; i < (long long)n * n; i += blockDim.x) Gg[i] = G[i];
  }
  if (MODE == 2) {
    for (long long i = tid; i < (long long)n * n; i += blockDim.x) Vg[i] = V[i];
  }
  if (tid == 0 && info) {
    info[0] = sweep;
    info[1] = first_rot;
  }
}

}  // namespace

hipError_t convert_f64_to_f32(const double* x, float* y, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, y, n, grp().stride);
  return hipGetLastError();
}
hipError_t convert_f32_to_f64(const float* x, double* y, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, y, n, grp().stride);
  return hipGetLastError();
}
hipError_t fill_f64(double* x, double v, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, v, n, grp().stride);
  return hipGetLastError();
}
hipError_t fill_f32(float* x, float v, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, v, n, grp().stride);
  return hipGetLastError();
}
hipError_t copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  if ((bytes % 8 == 0) && ((uintptr_t)dst % 8 == 0) && ((uintptr_t)src % 8 == 0)) {
    size_t n = bytes / 8;
    hipLaunchKernelGGL(k_copy8, dim3(grid_for(n), grp().count), dim3(256), 0, s, (const uint64_t*)src, (uint64_t*)dst, n, grp().stride,
                       grp().skip);
  } else {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(bytes), grp().count), dim3(256), 0, s, (const uint8_t*)src, (uint8_t*)dst, bytes, grp().stride);
  }
  return hipGetLastError();
}
hipError_t copy_bytes_if(void* dst, const void* src, size_t bytes, const int* flag, int want, hipStream_t s) {
  if (!bytes) return hipSuccess;
  if ((bytes % 8) || ((uintptr_t)dst % 8) || ((uintptr_t)src % 8)) return hipErrorInvalidValue;
  const size_t n = bytes / 8;
  hipLaunchKernelGGL(k_copy8_if, dim3(grid_for(n), grp().count), dim3(256), 0, s, (const uint64_t*)src, (uint64_t*)dst, n, flag,
                     want, grp().stride);
  return hipGetLastError();
}
hipError_t set_flag_le(int* flag, const int* info, int limit, hipStream_t s) {
  hipLaunchKernelGGL(k_set_flag_le, dim3(1, grp().count), dim3(64), 0, s, flag, info, limit, grp().stride);
  return hipGetLastError();
}
hipError_t note_negative_info(const int* info, int nq, double* err, double* noconv, int limit, hipStream_t s) {
  hipLaunchKernelGGL(k_note_negative_info, dim3(1, grp().count), dim3(64), 0, s, info, nq, err, noconv, limit,
                     grp().stride);
  return hipGetLastError();
}
hipError_t add_diag_f64(double* X, int n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_diag, dim3(grid_for(n), grp().count), dim3(256), 0, s, X, n, v, grp().stride);
  return hipGetLastError();
}
hipError_t axpby_f64(const double* x, double* y, double alpha, double beta, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_axpby<double>, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, y, alpha, beta, n, grp().stride);
  return hipGetLastError();
}
hipError_t axpby_f32(const float* x, float* y, float alpha, float beta, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_axpby<float>, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, y, alpha, beta, n, grp().stride);
  return hipGetLastError();
}
hipError_t gaussian_f64(double* x, size_t n, unsigned long long seed, unsigned long long stream_id, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_gaussian, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, n, (uint64_t)seed, (uint64_t)stream_id, grp().stride);
  return hipGetLastError();
}
hipError_t pair_f64(const double* X, const double* Y, long long n, double* out, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_partial<double>, dim3(RED_BLOCKS, grp().count), dim3(RED_THREADS), 0, s, X, Y, n, part, grp().stride,
                     grp().skip);
  hipLaunchKernelGGL(k_sum_partials, dim3(1, grp().count), dim3(RED_THREADS), 0, s, part, RED_BLOCKS, out, grp().stride,
                     grp().skip);
  return hipGetLastError();
}
hipError_t pair_f32(const float* X, const float* Y, long long n, double* out, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_partial<float>, dim3(RED_BLOCKS, grp().count), dim3(RED_THREADS), 0, s, X, Y, n, part, grp().stride,
                     grp().skip);
  hipLaunchKernelGGL(k_sum_partials, dim3(1, grp().count), dim3(RED_THREADS), 0, s, part, RED_BLOCKS, out, grp().stride,
                     grp().skip);
  return hipGetLastError();
}
hipError_t pair_rows_f64(const double* X, long long sX, const double* Y, long long sY, long long len, int rows,
                         double* out, long long os, long long oo, double beta, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_rows, dim3(rows), dim3(RED_THREADS), 0, s, X, sX, Y, sY, len, out, os, oo, beta);
  return hipGetLastError();
}
hipError_t ortho_err_from_gram(const double* G, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ortho_err, dim3(1, grp().count), dim3(RED_THREADS), 0, s, G, n, out, grp().stride);
  return hipGetLastError();
}
hipError_t row_normalize_f64(const double* Y, double* Z, double* nrm, int m, long long k, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_normalize, dim3(m, grp().count), dim3(RED_THREADS), 0, s, Y, Z, nrm, k, grp().stride);
  return hipGetLastError();
}
hipError_t jacobi_eig_f64(double* G, double* V, int n, int max_sweeps, double tol, int* info, void* scratch,
                          hipStream_t s, const int* skip) {
  if (n > JAC_MAXN) return hipErrorInvalidValue;
  if (n > 64 && scratch) return jacobi_eig_blocked_f64(G, V, n, max_sweeps, tol, info, scratch, s, skip);
  // orders that fill their blocks of 16 (padding to an even block count
  // below 8): the blocked method inside one work-group
  if (jacobi_lds_preferred(n)) return jacobi_eig_lds_f64(G, V, n, max_sweeps, tol, info, s, skip);
  // the matrices go to LDS when they fit there with a round's rotations
  static int lds_limit = -1;
  if (lds_limit < 0) {
    int dev = 0, v = 0;
    lds_limit = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) lds_limit = v;
      int o = 0;
      if (hipDeviceGetAttribute(&o, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && o > lds_limit)
        lds_limit = o;
    }
    lds_limit -= 16;  // static: the rotation counter
    if (lds_limit > 0 &&
        (hipFuncSetAttribute((const void*)k_jacobi<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit) != hipSuccess ||
         hipFuncSetAttribute((const void*)k_jacobi<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit) != hipSuccess))
      lds_limit = 0;
    (void)hipGetLastError();
  }
  const size_t bytes = (size_t)n * n * sizeof(double);
  const size_t rot = (size_t)((n + 1) / 2) * (3 * sizeof(double) + 2 * sizeof(int));  // a round's rotations
  if (lds_limit > 0 && 2 * bytes + rot <= (size_t)lds_limit) {
    hipLaunchKernelGGL(k_jacobi<2>, dim3(1, grp().count), dim3(JAC_THREADS), 2 * bytes + rot, s, G, V, n, max_sweeps, tol, info, skip, grp().stride);
  } else if (lds_limit > 0 && bytes + rot <= (size_t)lds_limit) {
    hipLaunchKernelGGL(k_jacobi<1>, dim3(1, grp().count), dim3(JAC_THREADS), bytes + rot, s, G, V, n, max_sweeps, tol, info, skip, grp().stride);
  } else {
    hipLaunchKernelGGL(k_jacobi<0>, dim3(1, grp().count), dim3(JAC_THREADS), rot, s, G, V, n, max_sweeps, tol, info, skip, grp().stride);
  }
  return hipGetLastError();
}

namespace {
__global__ void k_copy_strided(const double* __restrict__ src, long long ss, double* __restrict__ dst, long long ds,
                               long long len) {
  const double* a = src + (long long)blockIdx.y * ss;
  double* b = dst + (long long)blockIdx.y * ds;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void k_flags_or(const double* __restrict__ x, long long stride, int count, int i0, int i1,
                           double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double f0 = out[0], f1 = out[1];
  for (int j = 0; j < count; ++j) {
    if (x[(long long)j * stride + i0] != 0.0) f0 = 1.0;
    if (x[(long long)j * stride + i1] != 0.0) f1 = 1.0;
  }
  out[0] = f0;
  out[1] = f1;
}
}  // namespace

hipError_t copy_strided_f64(double* dst, long long ds, const double* src, long long ss, long long len, int count,
                            hipStream_t s) {
  if (count < 1 || len < 1) return hipSuccess;
  hipLaunchKernelGGL(k_copy_strided, dim3(grid_for((size_t)len), count), dim3(256), 0, s, src, ss, dst, ds, len);
  return hipGetLastError();
}

hipError_t flags_or(const double* x, long long stride, int count, int i0, int i1, double* out, hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(k_flags_or, dim3(1), dim3(64), 0, s, x, stride, count, i0, i1, out);
  return hipGetLastError();
}

namespace {
// maximum of x[0..n), by the whole block (blockDim 256)
__device__ double block_max(const double* x, int n) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
// out[i] = sum_j Y[i, j]^2, one block per row, fixed order
__global__ void k_row_sumsq(const double* Y, long long k, double* out, long long ms_) {
  Y = mshift(Y, ms_); out = mshift(out, ms_);
  __shared__ double red[256];
  const double* y = Y + (long long)blockIdx.x * k;
  double acc = 0.0;
  for (long long j = threadIdx.x; j < k; j += blockDim.x) acc += y[j] * y[j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}
__global__ void k_no_null_rows(const double* nrm2, int m, double rel, int* flag, long long ms_) {
  nrm2 = mshift(nrm2, ms_); flag = mshift(flag, ms_);
  const double floor_ = rel * rel * block_max(nrm2, m);
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x)
    if (nrm2[i] < floor_) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) flag[0] = any ? 0 : 1;
}
__global__ void k_fill_null_rows(double* Y, const double* T, const double* nrm2, int m, long long k, double rel,
                                 const int* flag, long long ms_) {
  Y = mshift(Y, ms_); T = mshift(T, ms_); nrm2 = mshift(nrm2, ms_); flag = mshift(flag, ms_);
  if (flag[0]) return;
  const double nmax = block_max(nrm2, m);
  const int i = blockIdx.x;
  if (!(nrm2[i] < rel * rel * nmax)) return;
  const double scale = rel * sqrt(nmax);
  for (long long j = threadIdx.x; j < k; j += blockDim.x) Y[(long long)i * k + j] = scale * T[(long long)i * k + j];
}
}  // namespace

hipError_t no_null_rows(const double* Y, int m, long long k, double rel, double* nrm2, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_row_sumsq, dim3(m, grp().count), dim3(256), 0, s, Y, k, nrm2, grp().stride);
  hipLaunchKernelGGL(k_no_null_rows, dim3(1, grp().count), dim3(256), 0, s, nrm2, m, rel, flag, grp().stride);
  return hipGetLastError();
}

hipError_t fill_null_rows(double* Y, const double* T, const double* nrm2, int m, long long k, double rel,
                          const int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_null_rows, dim3(m, grp().count), dim3(256), 0, s, Y, T, nrm2, m, k, rel, flag,
                     grp().stride);
  return hipGetLastError();
}

}  // namespace ttn
