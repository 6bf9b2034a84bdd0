// Blocked two-sided Jacobi eigensolver for the float64 Gram matrices of the
// polar update when they are too large for one work-group's LDS (n > 128).
//
// The n indices are cut into blocks of 32 (the last one ragged; a dummy block
// makes the count even).  A round pairs the blocks by the circle method; for
// each block pair (I, J) the 64 x 64 sub-matrix G[I u J, I u J] is loaded
// into LDS and given one cyclic sweep of 2 x 2 Jacobi rotations (relative
// threshold, Rutishauser updates), which yields an orthogonal R (rows) and
// the rotated sub-matrix S' = R G_sub R^T; the same work-group then replaces
// rows I u J of G and of the eigenvector matrix U by R times themselves.  A
// second launch replaces columns I u J of G by themselves times R^T (the
// diagonal block takes S' directly), spread over row chunks.  A sweep with no rotation anywhere ends the iteration:
// every later launch returns at once.
#include "common.h"
#include <math.h>

namespace ttn {
namespace {

constexpr int BJ_K = 32, BJ_S = 64, BJ_T = 1024, BJ_U = 256;

__device__ __forceinline__ void bj_pair(int nb, int r, int j, int& I, int& J) {
  if (j == 0) { I = r; J = nb - 1; }
  else { I = (r + j) % (nb - 1); J = (r - j + (nb - 1)) % (nb - 1); }
}
__device__ __forceinline__ int bj_gidx(int I, int J, int i, int n) {
  int blk = i < BJ_K ? I : J;
  int g = blk * BJ_K + (i & (BJ_K - 1));
  return g < n ? g : -1;
}
// sweep s is skipped once some earlier sweep made no rotation
__device__ __forceinline__ bool bj_done(const int* cnt, int sweep) { return sweep > 0 && cnt[sweep - 1] == 0; }

// Solves the sub-problem of pair j (one sweep of 2 x 2 rotations), writes R
// and S', then replaces rows I u J of G and U by R times themselves.
__global__ __launch_bounds__(BJ_T) void k_bj_solve(double* __restrict__ G, double* __restrict__ U, int n, int nb,
                                                  int sweep, int r, double tol, int* __restrict__ cnt,
                                                  double* __restrict__ Rbuf, double* __restrict__ Sbuf) {
  if (bj_done(cnt, sweep)) return;
  __shared__ double S[BJ_S][BJ_S + 1];
  __shared__ double R[BJ_S][BJ_S + 1];
  __shared__ double T[BJ_S][BJ_S + 1];
  __shared__ double cs[BJ_S / 2], sn[BJ_S / 2], tn[BJ_S / 2];
  __shared__ int pp[BJ_S / 2], qq[BJ_S / 2], gid[BJ_S];
  __shared__ int rc;
  const int tid = threadIdx.x, j = blockIdx.x;
  int I, J;
  bj_pair(nb, r, j, I, J);
  if (tid < BJ_S) gid[tid] = bj_gidx(I, J, tid, n);
  if (tid == 0) rc = 0;
  __syncthreads();
  for (int e = tid; e < BJ_S * BJ_S; e += BJ_T) {
    int i = e / BJ_S, k = e % BJ_S;
    int gi = gid[i], gk = gid[k];
    S[i][k] = (gi >= 0 && gk >= 0) ? G[(long long)gi * n + gk] : 0.0;
    R[i][k] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int rr = 0; rr < BJ_S - 1; ++rr) {
    if (tid < BJ_S / 2) {
      int k = tid, p, q;
      if (k == 0) { p = rr; q = BJ_S - 1; }
      else { p = (rr + k) % (BJ_S - 1); q = (rr - k + (BJ_S - 1)) % (BJ_S - 1); }
      if (p > q) { int t = p; p = q; q = t; }
      double c = 1.0, s = 0.0, t = 0.0;
      if (gid[p] >= 0 && gid[q] >= 0) {
        double gpp = S[p][p], gqq = S[q][q], gpq = S[p][q];
        if (gpq != 0.0 && fabs(gpq) > tol * sqrt(fabs(gpp * gqq))) {
          double theta = (gqq - gpp) / (2.0 * gpq);
          t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          atomicAdd(&rc, 1);
        }
      }
      pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s; tn[k] = t;
    }
    __syncthreads();
    {  // one 2x2 block of S per thread
      const int k1 = tid >> 5, k2 = tid & 31;
      double s1 = sn[k1], s2 = sn[k2];
      if (s1 != 0.0 || s2 != 0.0) {
        int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
        double c1 = cs[k1], c2 = cs[k2];
        double gpp = S[p1][p2], gpq = S[p1][q2], gqp = S[q1][p2], gqq = S[q1][q2];
        double rp_p = c1 * gpp - s1 * gqp, rp_q = c1 * gpq - s1 * gqq;
        double rq_p = s1 * gpp + c1 * gqp, rq_q = s1 * gpq + c1 * gqq;
        double npp = c2 * rp_p - s2 * rp_q, npq = s2 * rp_p + c2 * rp_q;
        double nqp = c2 * rq_p - s2 * rq_q, nqq = s2 * rq_p + c2 * rq_q;
        if (k1 == k2) {
          double t1 = tn[k1];
          npp = gpp - t1 * gpq;
          nqq = gqq + t1 * gpq;
          npq = 0.0;
          nqp = 0.0;
        }
        S[p1][p2] = npp; S[p1][q2] = npq; S[q1][p2] = nqp; S[q1][q2] = nqq;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two entries of a rotated pair of R rows per thread
      int e = tid + h * BJ_T;
      int k = e / BJ_S, i = e % BJ_S;
      double s = sn[k];
      if (s != 0.0) {
        double c = cs[k];
        int p = pp[k], q = qq[k];
        double up = R[p][i], uq = R[q][i];
        R[p][i] = c * up - s * uq;
        R[q][i] = s * up + c * uq;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && rc) atomicAdd(&cnt[sweep], rc);
  double* Ro = Rbuf + (long long)j * BJ_S * BJ_S;
  double* So = Sbuf + (long long)j * BJ_S * BJ_S;
  for (int e = tid; e < BJ_S * BJ_S; e += BJ_T) {
    int i = e / BJ_S, k = e % BJ_S;
    Ro[e] = R[i][k];
    So[e] = S[i][k];
  }
  // rows I u J of G and U <- R times themselves, one 64-column chunk at a
  // time; quarter q of the work-group computes rows 16q .. 16q+15
  const int qtr = tid >> 8, t = tid & 255;
  const int nchunks = (n + BJ_S - 1) / BJ_S;
  for (int which = 0; which < 2; ++which) {
    double* X = which ? U : G;
    // chunk by chunk, all 1024 threads: load, then 4 quarters compute 16 rows each
    for (int ch = 0; ch < nchunks; ++ch) {
      const int c0 = ch * BJ_S;
      __syncthreads();
      for (int e = tid; e < BJ_S * BJ_S; e += BJ_T) {
        int i = e / BJ_S, col = e % BJ_S;
        int gi = gid[i], gc = c0 + col;
        T[i][col] = (gi >= 0 && gc < n) ? X[(long long)gi * n + gc] : 0.0;
      }
      __syncthreads();
      // quarter q computes output rows 16q .. 16q+15, thread t: row 16q + t/16, 4 columns
      const int row = 16 * qtr + (t >> 4), cg = (t & 15);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
      for (int m = 0; m < BJ_S; ++m) {
        double rv = R[row][m];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma(rv, T[m][cg + 16 * u], acc[u]);
      }
      const int gi = gid[row];
      if (gi >= 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int gc = c0 + cg + 16 * u;
          if (gc < n) X[(long long)gi * n + gc] = acc[u];
        }
      }
    }
  }
}

// columns I u J of G <- themselves times R^T, one 64-row chunk per
// work-group (256 threads, 4 x 4 register tiles); the diagonal block (rows in
// I u J) takes S' directly
__global__ __launch_bounds__(BJ_U) void k_bj_cols(double* __restrict__ G, int n, int nb, int sweep, int r,
                                                 const int* __restrict__ cnt, const double* __restrict__ Rbuf,
                                                 const double* __restrict__ Sbuf) {
  if (bj_done(cnt, sweep)) return;
  __shared__ double Rt[BJ_S][BJ_S + 1];  // Rt[m][i] = R[i][m]
  __shared__ double T[BJ_S][BJ_S + 1];   // T[row][m]
  __shared__ int gid[BJ_S];
  const int tid = threadIdx.x, j = blockIdx.x, r0 = blockIdx.y * BJ_S;
  int I, J;
  bj_pair(nb, r, j, I, J);
  if (tid < BJ_S) gid[tid] = bj_gidx(I, J, tid, n);
  const double* Rj = Rbuf + (long long)j * BJ_S * BJ_S;
  const double* Sj = Sbuf + (long long)j * BJ_S * BJ_S;
  for (int e = tid; e < BJ_S * BJ_S; e += BJ_U) Rt[e % BJ_S][e / BJ_S] = Rj[e];
  __syncthreads();
  for (int e = tid; e < BJ_S * BJ_S; e += BJ_U) {
    int row = e / BJ_S, i = e % BJ_S;
    int gr = r0 + row, gi = gid[i];
    T[row][i] = (gr < n && gi >= 0) ? G[(long long)gr * n + gi] : 0.0;
  }
  __syncthreads();
  // out[row][i] = sum_m T[row][m] Rt[m][i]
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
  for (int m = 0; m < BJ_S; ++m) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = T[ty + 16 * a][m];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Rt[m][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int row = ty + 16 * a, gr = r0 + row;
    if (gr >= n) continue;
    int blk = gr / BJ_K;
    bool diag = (blk == I || blk == J);
    int loc = (blk == I ? 0 : BJ_K) + (gr & (BJ_K - 1));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int i = tx + 16 * b, gi = gid[i];
      if (gi < 0) continue;
      G[(long long)gr * n + gi] = diag ? Sj[loc * BJ_S + i] : acc[a][b];
    }
  }
}

__global__ void k_bj_init(double* __restrict__ U, int n, int* __restrict__ cnt, int ncnt) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)n * n;
       e += (long long)gridDim.x * blockDim.x)
    U[e] = (e / n == e % n) ? 1.0 : 0.0;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < ncnt; i += blockDim.x) cnt[i] = 0;
}

// info[0] = sweeps that made rotations, info[1] = rotations of the first
__global__ void k_bj_info(const int* __restrict__ cnt, int ncnt, int* __restrict__ info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int s = 0;
  while (s < ncnt && cnt[s] != 0) ++s;
  info[0] = s;
  info[1] = cnt[0];
}

}  // namespace

size_t jacobi_blocked_scratch_bytes(int n) {
  int nb = (n + BJ_K - 1) / BJ_K;
  nb += nb & 1;
  return (size_t)2 * (nb / 2) * BJ_S * BJ_S * sizeof(double) + 256 * sizeof(int) + 256;
}

hipError_t jacobi_eig_blocked_f64(double* G, double* U, int n, int max_sweeps, double tol, int* info, void* scratch,
                                  hipStream_t s) {
  int nb = (n + BJ_K - 1) / BJ_K;
  nb += nb & 1;
  const int npairs = nb / 2;
  if (max_sweeps > 250) max_sweeps = 250;
  double* Rbuf = (double*)scratch;
  double* Sbuf = Rbuf + (size_t)npairs * BJ_S * BJ_S;
  int* cnt = (int*)(Sbuf + (size_t)npairs * BJ_S * BJ_S);
  hipLaunchKernelGGL(k_bj_init, dim3(64), dim3(256), 0, s, U, n, cnt, max_sweeps + 1);
  const int chunks = (n + BJ_S - 1) / BJ_S;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(k_bj_solve, dim3(npairs), dim3(BJ_T), 0, s, G, U, n, nb, sw, r, tol, cnt, Rbuf, Sbuf);
      hipLaunchKernelGGL(k_bj_cols, dim3(npairs, chunks), dim3(BJ_U), 0, s, G, n, nb, sw, r, cnt, Rbuf, Sbuf);
    }
    // every few sweeps ask whether the last sweep made any rotation
    if (sw % 3 == 2 && sw + 1 < max_sweeps) {
      int last = 1;
      hipError_t e = hipMemcpyAsync(&last, cnt + sw, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      if (last == 0) break;
    }
  }
  if (info) hipLaunchKernelGGL(k_bj_info, dim3(1), dim3(64), 0, s, cnt, max_sweeps + 1, info);
  return hipGetLastError();
}

}  // namespace ttn
