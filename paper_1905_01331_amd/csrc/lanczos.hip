// Device kernels of the float64 Lanczos solver for the top tensor and small
// helpers of the polar update.  All scalars of the recurrence live in device
// memory so the host never waits inside an iteration.
#include "common.h"
#include "lanczos.h"
#include <math.h>
#include <algorithm>

namespace ttn {
namespace {

inline int grid_for(size_t n, int threads = 256, int cap = 4096) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (size_t)cap) b = cap;
  return (int)b;
}

// Dense tridiagonal T (m x m) from alpha/beta; rows past m_eff are decoupled
// with a diagonal above every Ritz value so they never become the lowest.
__global__ void k_build_T(const double* __restrict__ alpha, const double* __restrict__ beta, int m,
                          const int* __restrict__ stop, const int* __restrict__ m_eff, double* __restrict__ T, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  alpha = mshift(alpha, ms_); beta = mshift(beta, ms_); stop = mshift(stop, ms_); m_eff = mshift(m_eff, ms_); T = mshift(T, ms_);
  int me = (*stop) ? *m_eff : m;
  double big = 0.0;
  for (int i = 0; i < me; ++i) big = fmax(big, fabs(alpha[i]) + 2.0 * fabs(beta[i]));
  big = 4.0 * big + 1.0;
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    int r = idx / m, c = idx - r * m;
    double v = 0.0;
    if (r < me && c < me) {
      if (r == c) v = alpha[r];
      else if (c == r + 1) v = beta[r];
      else if (r == c + 1) v = beta[c];
    } else if (r == c) {
      v = big;
    }
    T[idx] = v;
  }
}

// y = eigenvector of the smallest diagonal entry of the diagonalised T
// (rows of U).
__global__ void k_select_lowest(const double* __restrict__ Tdiag, const double* __restrict__ V, int m,
                                double* __restrict__ y, double* __restrict__ theta, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  Tdiag = mshift(Tdiag, ms_); V = mshift(V, ms_); y = mshift(y, ms_); theta = mshift(theta, ms_);
  __shared__ int best;
  if (threadIdx.x == 0) {
    int b = 0;
    for (int i = 1; i < m; ++i)
      if (Tdiag[(size_t)i * m + i] < Tdiag[(size_t)b * m + b]) b = i;
    best = b;
    theta[0] = Tdiag[(size_t)b * m + b];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) y[i] = V[(size_t)best * m + i];
}

// x *= 1 / sqrt(ss[0])
__global__ void k_scale_rsqrt(double* __restrict__ x, const double* __restrict__ ss, size_t n, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  x = mshift(x, ms_); ss = mshift(ss, ms_);
  double s = ss[0];
  double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] *= inv;
}

// r = Hv - lam v, lam = lamv[0]
__global__ void k_residual(const double* __restrict__ Hv, const double* __restrict__ v, const double* __restrict__ lamv,
                           double* __restrict__ r, size_t n, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  Hv = mshift(Hv, ms_); v = mshift(v, ms_); lamv = mshift(lamv, ms_); r = mshift(r, ms_);
  double lam = lamv[0];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    r[i] = Hv[i] - lam * v[i];
}

// Sign convention: the entry of largest magnitude (first on ties) positive.
__global__ void k_sign_fix(double* __restrict__ v, size_t n, long long ms_) {
  v = mshift(v, ms_);
  __shared__ double bv[256];
  __shared__ long long bi[256];
  double best = -1.0;
  long long idx = -1;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    double a = fabs(v[i]);
    if (a > best) { best = a; idx = (long long)i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double o = bv[threadIdx.x + s];
      long long oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi >= 0 && (bi[threadIdx.x] < 0 || oi < bi[threadIdx.x]))) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  long long im = bi[0];
  __syncthreads();
  if (im < 0) return;
  bool flip = v[im] < 0.0;
  __syncthreads();
  if (flip)
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) v[i] = -v[i];
}

// out = a*x + b*y with a, b read from device scalars (sa, sb may be null for 1)
__global__ void k_axpy_dev(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ scale,
                           double factor, size_t n, long long ms_) {
  y = mshift(y, ms_); x = mshift(x, ms_); scale = mshift(scale, ms_);
  double s = factor * (scale ? scale[0] : 1.0);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] += s * x[i];
}

__global__ void k_sqrt_inplace(double* x, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  x = mshift(x, ms_);
  if (threadIdx.x == 0 && blockIdx.x == 0) x[0] = sqrt(fmax(x[0], 0.0));
}

// energy bookkeeping: out[0] = lam, out[1] = (lam + c L) / (L ly)
// out[0] = lambda, out[1] = e = (lambda + c L) / (L ly); the energy it
// replaces goes to prev[0] (prev may be null)
__global__ void k_energy(const double* __restrict__ lam, const double* __restrict__ c, double L, double ly,
                         double* __restrict__ out, double* __restrict__ prev, long long ms_) {
  lam = mshift(lam, ms_); c = mshift(c, ms_); out = mshift(out, ms_); prev = mshift(prev, ms_);
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double l = lam[0];
    if (prev) prev[0] = out[1];
    out[0] = l;
    out[1] = (l + c[0] * L) / (L * ly);
  }
}

// min/max of nrm[0..m) -> out[0] = min/max ratio (0 if max == 0)
__global__ void k_ratio(const double* __restrict__ nrm, int m, double* __restrict__ out, double* __restrict__ run_min, long long ms_) {
  nrm = mshift(nrm, ms_); out = mshift(out, ms_); run_min = mshift(run_min, ms_);
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double mn = nrm[0], mx = nrm[0];
    for (int i = 1; i < m; ++i) { mn = fmin(mn, nrm[i]); mx = fmax(mx, nrm[i]); }
    double r = mx > 0.0 ? mn / mx : 0.0;
    out[0] = r;
    if (run_min) run_min[0] = fmin(run_min[0], r);
  }
}

__global__ void k_running_max(const double* __restrict__ x, double* __restrict__ run_max, long long ms_) {
  x = mshift(x, ms_); run_max = mshift(run_max, ms_);
  if (threadIdx.x == 0 && blockIdx.x == 0) run_max[0] = fmax(run_max[0], x[0]);
}

__global__ void k_identity(double* __restrict__ X, int n, long long ms_) {
  X = mshift(X, ms_);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x)
    X[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// X <- 1/2 (X + sign X^T) in place (n x n); one thread per unordered pair.
__global__ void k_symmetrize(double* __restrict__ X, int n, double sign, long long ms_) {
  X = mshift(X, ms_);
  long long total = (long long)n * (n + 1) / 2;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    // t -> (i, j) with i <= j
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
    while ((long long)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((long long)i * (i + 1) / 2 > t) --i;
    int j = (int)(t - (long long)i * (i + 1) / 2);  // j <= i
    double a = X[(long long)i * n + j], b = X[(long long)j * n + i];
    if (i == j) {
      X[(long long)i * n + i] = (sign > 0) ? a : 0.0;
    } else {
      double m = 0.5 * (a + sign * b);
      X[(long long)i * n + j] = m;
      X[(long long)j * n + i] = sign * m;
    }
  }
}

// Multi-dot for the full reorthogonalisation: part[b][i] = sum over block b's
// slice of Q[i] . w (i < nq), part[b][nq] = w . w.  Fixed grid, deterministic.
constexpr int MD_BLOCKS = 128, MD_THREADS = 256, MD_MAXQ = 64;
__global__ __launch_bounds__(MD_THREADS) void k_multidot(const double* __restrict__ Q, const double* __restrict__ w,
                                                         int nq, size_t n, double* __restrict__ part, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  Q = mshift(Q, ms_); w = mshift(w, ms_); part = mshift(part, ms_);
  __shared__ double red[MD_THREADS / 64][MD_MAXQ + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  size_t beg = blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  for (int i0 = 0; i0 <= nq; i0 += 16) {
    double acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.0;
    for (size_t e = beg + tid; e < end; e += MD_THREADS) {
      double we = w[e];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        int i = i0 + t;
        if (i < nq) acc[t] += Q[(size_t)i * n + e] * we;
        else if (i == nq) acc[t] += we * we;
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      double v = acc[t];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0 && i0 + t <= nq) red[wv][i0 + t] = v;
    }
  }
  __syncthreads();
  for (int i = tid; i <= nq; i += MD_THREADS) {
    double v = 0.0;
    for (int k = 0; k < MD_THREADS / 64; ++k) v += red[k][i];
    part[(size_t)blockIdx.x * (MD_MAXQ + 1) + i] = v;
  }
}
// The coefficients of a reorthogonalisation pass, summed from the per-block
// partials of k_multidot in a fixed order (wave i % 4 sums coefficient i:
// each lane two partials, then a fixed shuffle tree), so every work-group
// that calls this holds bitwise the same values.
__device__ void md_coefficients(const double* __restrict__ part, int nq, double* cs) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = wv; i <= nq; i += (int)(blockDim.x >> 6)) {
    double v = 0.0;
    for (int b = lane; b < MD_BLOCKS; b += 64) v += part[(size_t)b * (MD_MAXQ + 1) + i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) cs[i] = v;
  }
  __syncthreads();
}
// First pass: w -= sum_{i < nq} c[i] Q[i]; coef[0..nq] = c (coef[nq] = w.w
// before the pass).
__global__ __launch_bounds__(256) void k_reorth_apply(double* __restrict__ w, const double* __restrict__ Q,
                                                      const double* __restrict__ part, int nq, size_t n,
                                                      double* __restrict__ coef, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  w = mshift(w, ms_); Q = mshift(Q, ms_); part = mshift(part, ms_); coef = mshift(coef, ms_);
  __shared__ double cs[MD_MAXQ + 1];
  md_coefficients(part, nq, cs);
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= nq; i += blockDim.x) coef[i] = cs[i];
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double v = w[e];
    for (int i = 0; i < nq; ++i) v -= cs[i] * Q[(size_t)i * n + e];
    w[e] = v;
  }
}
// Second pass of step j (nq = j + 1): c2 from the partials, w -= sum c2[i]
// Q[i], the squares of the new w summed per work-group into nrm[blockIdx.x]
// (fixed order); work-group 0 stores c2 and alpha[j] = c1[j] + c2[j].
__global__ __launch_bounds__(256) void k_reorth_second(double* __restrict__ w, const double* __restrict__ Q,
                                                       const double* __restrict__ part, int nq, size_t n,
                                                       const double* __restrict__ c1, double* __restrict__ c2,
                                                       double* __restrict__ alpha, double* __restrict__ nrm,
                                                       long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  w = mshift(w, ms_); Q = mshift(Q, ms_); part = mshift(part, ms_); c1 = mshift(c1, ms_); c2 = mshift(c2, ms_);
  alpha = mshift(alpha, ms_); nrm = mshift(nrm, ms_);
  __shared__ double cs[MD_MAXQ + 1];
  __shared__ double red[4];
  md_coefficients(part, nq, cs);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i <= nq; ++i) c2[i] = cs[i];
    alpha[nq - 1] = c1[nq - 1] + cs[nq - 1];
  }
  double ss = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double v = w[e];
    for (int i = 0; i < nq; ++i) v -= cs[i] * Q[(size_t)i * n + e];
    w[e] = v;
    ss += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) nrm[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
// The recurrence step j: beta[j] = ||w|| from the nb per-work-group sums
// (each work-group adds them in the same fixed order), with the
// invariant-subspace test against ||H q_j|| = sqrt(c1[j + 1]) (stop and m_eff
// set, beta[j] = 0); q_{j+1} = w / beta[j] (zero after a stop), also into
// `stage` when given.  Work-group 0 stores the scalars.
__global__ __launch_bounds__(256) void k_lz_normalize(const double* __restrict__ w, const double* __restrict__ nrm,
                                                      int nb, int j, size_t n, const double* __restrict__ c1,
                                                      double* __restrict__ beta, double tol, int* __restrict__ stop,
                                                      int* __restrict__ m_eff, double* __restrict__ qn,
                                                      double* __restrict__ stage, long long ms_, const int* sk) {
  if (member_skipped(sk, ms_)) return;
  w = mshift(w, ms_); nrm = mshift(nrm, ms_); c1 = mshift(c1, ms_); beta = mshift(beta, ms_);
  stop = mshift(stop, ms_); m_eff = mshift(m_eff, ms_); qn = mshift(qn, ms_); stage = mshift(stage, ms_);
  __shared__ double sh[256];
  const bool stopped = *stop != 0;  // read before work-group 0 may set it
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += nrm[b];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double b = sqrt(fmax(sh[0], 0.0));
  const double hn = sqrt(fmax(c1[j + 1], 0.0));
  const bool now_stop = !stopped && (!(b > tol * hn) || b == 0.0);
  const double bj = (stopped || now_stop) ? 0.0 : b;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    beta[j] = bj;
    if (now_stop) {
      *stop = 1;
      *m_eff = j + 1;
    }
  }
  const double inv = bj > 0.0 ? 1.0 / bj : 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double q = w[e] * inv;
    qn[e] = q;
    if (stage) stage[e] = q;
  }
}

// Spectrum of a density matrix from the diagonal of its Jacobi-diagonalised
// form (n <= 1024): sorted (bitonic network over 1024 slots, the unused ones
// holding -inf), written in descending order, and the entropy
// S = -sum_{p > 0} p log2 p summed in a fixed order.
__global__ __launch_bounds__(512) void k_spectrum(const double* __restrict__ G, int n, double* __restrict__ p,
                                                  double* __restrict__ S) {
  constexpr int N = 1024;
  __shared__ double v[N];
  __shared__ double red[512];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += 512) v[i] = i < n ? G[(size_t)i * n + i] : -INFINITY;
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < N; i += 512) {
        const int l = i ^ j;
        if (l > i) {
          const double a = v[i], b = v[l];
          if (((i & k) == 0) ? (a > b) : (a < b)) {
            v[i] = b;
            v[l] = a;
          }
        }
      }
      __syncthreads();
    }
  double acc = 0.0;
  for (int i = tid; i < n; i += 512) {
    const double q = v[N - 1 - i];
    p[i] = q;
    if (q > 0.0) acc -= q * log2(q);
  }
  red[tid] = acc;
  __syncthreads();
  for (int st = 256; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) S[0] = red[0];
}

// After a restart: a restart that ran (done still 0 on entry) is counted in
// *runs; *done = 1 once ||r|| <= tol max(1, |lambda|) (never cleared here).
__global__ void k_lz_mark_done(const double* __restrict__ res, const double* __restrict__ lam, double tol,
                               int* __restrict__ done, int* __restrict__ runs, long long ms_) {
  res = mshift(res, ms_); lam = mshift(lam, ms_); done = mshift(done, ms_); runs = mshift(runs, ms_);
  if (threadIdx.x != 0 || blockIdx.x != 0 || *done) return;
  ++*runs;
  if (res[0] <= tol * fmax(1.0, fabs(lam[0]))) *done = 1;
}
__global__ void k_zero_int(int* x, int n, long long ms_) {
  x = mshift(x, ms_);
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0;
}

}  // namespace

hipError_t lz_build_T(const double* alpha, const double* beta, int m, const int* stop, const int* m_eff, double* T,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_build_T, dim3(1, grp().count), dim3(256), 0, s, alpha, beta, m, stop, m_eff, T, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t lz_select_lowest(const double* T, const double* V, int m, double* y, double* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_select_lowest, dim3(1, grp().count), dim3(64), 0, s, T, V, m, y, theta, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t scale_rsqrt(double* x, const double* ss, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rsqrt, dim3(grid_for(n), grp().count), dim3(256), 0, s, x, ss, n, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t residual_vec(const double* Hv, const double* v, const double* lam, double* r, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n), grp().count), dim3(256), 0, s, Hv, v, lam, r, n, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t sign_fix(double* v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_fix, dim3(1, grp().count), dim3(256), 0, s, v, n, grp().stride);
  return hipGetLastError();
}
hipError_t axpy_dev(double* y, const double* x, const double* scale, double factor, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(grid_for(n), grp().count), dim3(256), 0, s, y, x, scale, factor, n, grp().stride);
  return hipGetLastError();
}
hipError_t sqrt_inplace(double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_sqrt_inplace, dim3(1, grp().count), dim3(64), 0, s, x, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t energy_store(const double* lam, const double* c, double L, double ly, double* out, double* prev,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(1, grp().count), dim3(64), 0, s, lam, c, L, ly, out, prev, grp().stride);
  return hipGetLastError();
}
hipError_t ratio_minmax(const double* nrm, int m, double* out, double* run_min, hipStream_t s) {
  hipLaunchKernelGGL(k_ratio, dim3(1, grp().count), dim3(64), 0, s, nrm, m, out, run_min, grp().stride);
  return hipGetLastError();
}
hipError_t running_max(const double* x, double* run_max, hipStream_t s) {
  hipLaunchKernelGGL(k_running_max, dim3(1, grp().count), dim3(64), 0, s, x, run_max, grp().stride);
  return hipGetLastError();
}
hipError_t identity_f64(double* X, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_identity, dim3(grid_for((size_t)n * n), grp().count), dim3(256), 0, s, X, n, grp().stride);
  return hipGetLastError();
}
hipError_t symmetrize_f64(double* X, int n, double sign, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrize, dim3(grid_for((size_t)n * (n + 1) / 2), grp().count), dim3(256), 0, s, X, n, sign, grp().stride);
  return hipGetLastError();
}
size_t lz_reorth_part_doubles() { return (size_t)MD_BLOCKS * (MD_MAXQ + 1); }
hipError_t lz_reorth_first(double* w, const double* Q, int nq, size_t n, double* coef, double* part, hipStream_t s) {
  if (nq > MD_MAXQ) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multidot, dim3(MD_BLOCKS, grp().count), dim3(MD_THREADS), 0, s, Q, w, nq, n, part, grp().stride, grp().skip);
  hipLaunchKernelGGL(k_reorth_apply, dim3(grid_for(n), grp().count), dim3(256), 0, s, w, Q, part, nq, n, coef,
                     grp().stride, grp().skip);
  return hipGetLastError();
}
// work-groups of the fused passes: a fixed count for a given n
static int lz_groups(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 1024); }
size_t lz_norm_doubles() { return 1024; }
hipError_t lz_reorth_final(double* w, const double* Q, int nq, size_t n, const double* c1, double* c2, double* part,
                           double* nrm, double* alpha, double* beta, double tol, int* stop, int* m_eff, double* qn,
                           double* stage, hipStream_t s) {
  if (nq > MD_MAXQ) return hipErrorInvalidValue;
  const int nb = lz_groups(n);
  hipLaunchKernelGGL(k_multidot, dim3(MD_BLOCKS, grp().count), dim3(MD_THREADS), 0, s, Q, w, nq, n, part, grp().stride, grp().skip);
  hipLaunchKernelGGL(k_reorth_second, dim3(nb, grp().count), dim3(256), 0, s, w, Q, part, nq, n, c1, c2, alpha, nrm,
                     grp().stride, grp().skip);
  hipLaunchKernelGGL(k_lz_normalize, dim3(nb, grp().count), dim3(256), 0, s, w, nrm, nb, nq - 1, n, c1, beta, tol, stop,
                     m_eff, qn, stage, grp().stride, grp().skip);
  return hipGetLastError();
}
hipError_t lz_mark_done(const double* res, const double* lam, double tol, int* done, int* runs, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_mark_done, dim3(1, grp().count), dim3(64), 0, s, res, lam, tol, done, runs, grp().stride);
  return hipGetLastError();
}
hipError_t spectrum_sorted(const double* G, int n, double* p, double* S, hipStream_t s) {
  if (n < 1 || n > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_spectrum, dim3(1), dim3(512), 0, s, G, n, p, S);
  return hipGetLastError();
}
hipError_t zero_int(int* x, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1, grp().count), dim3(64), 0, s, x, n, grp().stride);
  return hipGetLastError();
}

}  // namespace ttn
