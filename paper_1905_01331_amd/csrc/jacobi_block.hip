// Blocked two-sided Jacobi eigensolver for the float64 Gram matrices of the
// polar update when they are too large for one work-group's LDS (n > 64).
//
// The n indices are cut into blocks of BK = BS/2 (the last one ragged; a
// dummy block makes the count even).  A round pairs the blocks by the circle
// method; for each block pair (I, J) the BS x BS sub-matrix G[I u J, I u J]
// gets one cyclic sweep of 2 x 2 Jacobi rotations (relative threshold,
// Rutishauser diagonal updates), which yields an orthogonal R and the
// rotated sub-matrix S' = R G_sub R^T (phase A).  Then every block of G
// between two index sets X, Y of the round is replaced by R_X G[X,Y] R_Y^T
// (S' on the diagonal) and the rows X of the eigenvector matrix U by
// R_X U[X,:] (phase B).  A sweep is nb - 1 rounds; a sweep with no rotation
// ends the iteration.
//
// The whole iteration is ONE launch of a persistent grid: its work-groups
// share phase A (one block pair each) and phase B (one block of G or one
// panel of U each) and meet at a grid barrier between phases.  The grid
// never exceeds the number of compute units and a work-group needs far less
// than one compute unit's resources, so every work-group of the grid is
// resident at once.  Each barrier wait is bounded: past the bound the
// kernel raises an abort flag, every work-group leaves at its next barrier,
// and info[0] = -1 reports the failure to the host.
#include "common.h"
#include <math.h>
#include <algorithm>

namespace ttn {
namespace {

constexpr int JC_MAX_WG = 128;
constexpr long long JC_SPIN_LIMIT = 1LL << 21;  // about a second of polling

struct JcCtl {
  unsigned bar;    // barrier arrivals
  int abort;       // set when a barrier wait exceeded its bound
  int pad[2];
  int cnt[256];    // rotations per sweep
  int rnd[64];     // rotations per round index, summed over sweeps
};

__device__ __forceinline__ void jc_pair(int nb, int r, int j, int& I, int& J) {
  if (j == 0) { I = r; J = nb - 1; }
  else { I = (r + j) % (nb - 1); J = (r - j + (nb - 1)) % (nb - 1); }
}

// Grid barrier: every thread publishes its stores at device scope, thread 0
// of each work-group counts in and polls; returns false after an abort.
__device__ bool jc_grid_sync(JcCtl* ctl, unsigned& target, int* ok_lds) {
  __threadfence();
  __syncthreads();
  target += gridDim.x;
  if (threadIdx.x == 0) {
    int ok = 1;
    atomicAdd(&ctl->bar, 1u);
    long long spins = 0;
    while (__hip_atomic_load(&ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (++spins > JC_SPIN_LIMIT) {
        atomicExch(&ctl->abort, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    *ok_lds = ok;
  }
  __syncthreads();
  __threadfence();
  return *ok_lds != 0;
}

template <int BS>
__global__ __launch_bounds__((BS / 2) * (BS / 2)) void k_jacobi_coop(double* __restrict__ G, double* __restrict__ U,
                                                                   int n, int nb, int max_sweeps, double tol,
                                                                   JcCtl* __restrict__ ctl, double* __restrict__ Rbuf,
                                                                   double* __restrict__ Sbuf, int* __restrict__ info) {
  constexpr int BK = BS / 2;   // block width
  constexpr int NT = BK * BK;  // threads: one 2 x 2 block of S each
  constexpr int LD = BS + 1;
  constexpr int RS = NT / BS;  // row stride of the four outputs per thread in phase B
  __shared__ double L0[BS * LD], L1[BS * LD], L2[BS * LD];
  __shared__ int gx[BS], gy[BS];
  __shared__ int ok_lds, rot_lds;
  __shared__ int seen[64];  // rnd[] as read at the previous visit of each round
  if (threadIdx.x < 64) seen[threadIdx.x] = 0;
  const int tid = threadIdx.x;
  const int npairs = nb / 2;
  const int ng = npairs * (npairs + 1) / 2;
  const int nchunks = (n + BS - 1) / BS;
  const int nitems = ng + npairs * nchunks;
  unsigned target = 0;
  int sweeps = max_sweeps;
  bool alive = true;

  auto gidx = [&](int I, int J, int i) {
    int g = i < BK ? I * BK + i : J * BK + (i - BK);
    return g < n ? g : -1;
  };

  for (int sw = 0; sw < max_sweeps && alive; ++sw) {
    for (int r = 0; r < nb - 1; ++r) {
      // ---------------- phase A: one block pair per work-group ----------------
      for (int j = blockIdx.x; j < npairs; j += gridDim.x) {
        int I, J;
        jc_pair(nb, r, j, I, J);
        __syncthreads();
        if (tid < BS) gx[tid] = gidx(I, J, tid);
        if (tid == 0) rot_lds = 0;
        __syncthreads();
        double* Sc = L0;
        double* Sn = L1;
        double* R = L2;
        for (int e = tid; e < BS * BS; e += NT) {
          int i = e / BS, k = e - i * BS;
          int gi = gx[i], gk = gx[k];
          Sc[i * LD + k] = (gi >= 0 && gk >= 0) ? G[(long long)gi * n + gk] : 0.0;
          R[i * LD + k] = (i == k) ? 1.0 : 0.0;
        }
        __syncthreads();
        const int k1 = tid / BK, k2 = tid - (tid / BK) * BK;
        int rot = 0;
        for (int rr = 0; rr < BS - 1; ++rr) {
          // rotation k of this step acts on the index pair (p, q), circle method
          int p1, q1, p2, q2;
          if (k1 == 0) { p1 = rr; q1 = BS - 1; }
          else { p1 = (rr + k1) % (BS - 1); q1 = (rr - k1 + (BS - 1)) % (BS - 1); }
          if (k2 == 0) { p2 = rr; q2 = BS - 1; }
          else { p2 = (rr + k2) % (BS - 1); q2 = (rr - k2 + (BS - 1)) % (BS - 1); }
          if (p1 > q1) { int t = p1; p1 = q1; q1 = t; }
          if (p2 > q2) { int t = p2; p2 = q2; q2 = t; }
          // both rotations, computed (identically) by every thread that needs them
          double c1, s1, t1, c2, s2, t2;
          c1 = 1.0; s1 = 0.0; t1 = 0.0;
          if (gx[p1] >= 0 && gx[q1] >= 0) jacobi_rotation(Sc[p1 * LD + p1], Sc[q1 * LD + q1], Sc[p1 * LD + q1], tol, c1, s1, t1);
          if (k2 == k1) {
            c2 = c1; s2 = s1; t2 = t1;
          } else {
            c2 = 1.0; s2 = 0.0; t2 = 0.0;
            if (gx[p2] >= 0 && gx[q2] >= 0) jacobi_rotation(Sc[p2 * LD + p2], Sc[q2 * LD + q2], Sc[p2 * LD + q2], tol, c2, s2, t2);
          }
          {  // the 2 x 2 block (rows p1, q1; columns p2, q2) of S' = R S R^T
            double gpp = Sc[p1 * LD + p2], gpq = Sc[p1 * LD + q2], gqp = Sc[q1 * LD + p2], gqq = Sc[q1 * LD + q2];
            double npp, npq, nqp, nqq;
            if (k1 == k2 && s1 != 0.0) {
              npp = gpp - t1 * gpq;
              nqq = gqq + t1 * gpq;
              npq = 0.0;
              nqp = 0.0;
              ++rot;
            } else {
              double rp_p = c1 * gpp - s1 * gqp, rp_q = c1 * gpq - s1 * gqq;
              double rq_p = s1 * gpp + c1 * gqp, rq_q = s1 * gpq + c1 * gqq;
              npp = c2 * rp_p - s2 * rp_q; npq = s2 * rp_p + c2 * rp_q;
              nqp = c2 * rq_p - s2 * rq_q; nqq = s2 * rq_p + c2 * rq_q;
            }
            Sn[p1 * LD + p2] = npp; Sn[p1 * LD + q2] = npq; Sn[q1 * LD + p2] = nqp; Sn[q1 * LD + q2] = nqq;
          }
          if (s1 != 0.0) {  // rows p1, q1 of R, columns 2 k2 and 2 k2 + 1
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              int c = 2 * k2 + h;
              double up = R[p1 * LD + c], uq = R[q1 * LD + c];
              R[p1 * LD + c] = c1 * up - s1 * uq;
              R[q1 * LD + c] = s1 * up + c1 * uq;
            }
          }
          __syncthreads();
          double* t = Sc; Sc = Sn; Sn = t;
        }
        if (rot) atomicAdd(&rot_lds, rot);
        __syncthreads();
        if (tid == 0 && rot_lds) {
          atomicAdd(&ctl->cnt[sw], rot_lds);
          atomicAdd(&ctl->rnd[r], rot_lds);
        }
        double* Ro = Rbuf + (long long)j * BS * BS;
        double* So = Sbuf + (long long)j * BS * BS;
        for (int e = tid; e < BS * BS; e += NT) {
          int i = e / BS, k = e - i * BS;
          Ro[e] = R[i * LD + k];
          So[e] = Sc[i * LD + k];
        }
      }
      if (!jc_grid_sync(ctl, target, &ok_lds)) { alive = false; break; }
      // a round without any rotation has R = I and S' = S: phase B would
      // rewrite G and U unchanged, so every work-group skips it (all read the
      // same count after the barrier)
      const int rv = __hip_atomic_load(&ctl->rnd[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool rotated = rv != seen[r];
      __syncthreads();
      if (tid == 0) seen[r] = rv;
      if (!rotated) continue;
      // ---------------- phase B: blocks of G and panels of U ----------------
      for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        __syncthreads();
        const int row = tid / BS, col = tid - (tid / BS) * BS;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (item < ng) {
          // (x, y) with x <= y from the packed upper-triangle index
          int x = 0, rem = item;
          while (rem >= npairs - x) { rem -= npairs - x; ++x; }
          const int y = x + rem;
          int Ix, Jx, Iy, Jy;
          jc_pair(nb, r, x, Ix, Jx);
          jc_pair(nb, r, y, Iy, Jy);
          if (tid < BS) { gx[tid] = gidx(Ix, Jx, tid); gy[tid] = gidx(Iy, Jy, tid); }
          __syncthreads();
          if (x == y) {
            const double* Sx = Sbuf + (long long)x * BS * BS;
            for (int e = tid; e < BS * BS; e += NT) {
              int i = e / BS, k = e - i * BS;
              int gi = gx[i], gk = gx[k];
              if (gi >= 0 && gk >= 0) G[(long long)gi * n + gk] = Sx[e];
            }
            continue;
          }
          const double* Rx = Rbuf + (long long)x * BS * BS;
          const double* Ry = Rbuf + (long long)y * BS * BS;
          for (int e = tid; e < BS * BS; e += NT) {
            int i = e / BS, k = e - i * BS;
            int gi = gx[i], gk = gy[k];
            L0[i * LD + k] = (gi >= 0 && gk >= 0) ? G[(long long)gi * n + gk] : 0.0;
            L1[i * LD + k] = Rx[e];
            L2[k * LD + i] = Ry[e];  // transposed: L2[m][k] = R_y[k][m]
          }
          __syncthreads();
          // T = G[X,Y] R_y^T, four outputs per thread (rows row + RS u, column col)
          for (int m = 0; m < BS; ++m) {
            double ry = L2[m * LD + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(L0[(row + u * RS) * LD + m], ry, acc[u]);
          }
          __syncthreads();
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            L0[(row + u * RS) * LD + col] = acc[u];
            acc[u] = 0.0;
          }
          __syncthreads();
          // out = R_x T
          for (int m = 0; m < BS; ++m) {
            double tv = L0[m * LD + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(L1[(row + u * RS) * LD + m], tv, acc[u]);
          }
          const int gk = gy[col];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int gi = gx[row + u * RS];
            if (gi >= 0 && gk >= 0) {
              G[(long long)gi * n + gk] = acc[u];
              G[(long long)gk * n + gi] = acc[u];
            }
          }
        } else {
          const int it = item - ng;
          const int x = it / nchunks, c0 = (it - x * nchunks) * BS;
          int Ix, Jx;
          jc_pair(nb, r, x, Ix, Jx);
          if (tid < BS) gx[tid] = gidx(Ix, Jx, tid);
          __syncthreads();
          const double* Rx = Rbuf + (long long)x * BS * BS;
          for (int e = tid; e < BS * BS; e += NT) {
            int i = e / BS, k = e - i * BS;
            int gi = gx[i], gc = c0 + k;
            L0[i * LD + k] = (gi >= 0 && gc < n) ? U[(long long)gi * n + gc] : 0.0;
            L1[i * LD + k] = Rx[e];
          }
          __syncthreads();
          for (int m = 0; m < BS; ++m) {
            double uv = L0[m * LD + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(L1[(row + u * RS) * LD + m], uv, acc[u]);
          }
          const int gc = c0 + col;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int gi = gx[row + u * RS];
            if (gi >= 0 && gc < n) U[(long long)gi * n + gc] = acc[u];
          }
        }
      }
      if (!jc_grid_sync(ctl, target, &ok_lds)) { alive = false; break; }
    }
    if (!alive) break;
    // every work-group reads the same final count after the barrier
    if (__hip_atomic_load(&ctl->cnt[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      sweeps = sw;
      break;
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    info[0] = alive ? sweeps : -1;
    info[1] = ctl->cnt[0];
  }
}

__global__ void k_jc_init(double* __restrict__ U, int n, JcCtl* __restrict__ ctl) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)n * n;
       e += (long long)gridDim.x * blockDim.x)
    U[e] = (e / n == e % n) ? 1.0 : 0.0;
  if (blockIdx.x == 0) {
    int* w = (int*)ctl;
    for (int i = threadIdx.x; i < (int)(sizeof(JcCtl) / sizeof(int)); i += blockDim.x) w[i] = 0;
  }
}

constexpr int JC_BS = 32;

int jc_compute_units() {
  static int cus = -1;
  if (cus < 0) {
    int dev = 0, v = 0;
    cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cus = v;
  }
  return cus;
}

}  // namespace

size_t jacobi_blocked_scratch_bytes(int n) {
  int nb = (n + JC_BS / 2 - 1) / (JC_BS / 2);
  nb += nb & 1;
  return (size_t)2 * (nb / 2) * JC_BS * JC_BS * sizeof(double) + sizeof(JcCtl) + 256;
}

hipError_t jacobi_eig_blocked_f64(double* G, double* U, int n, int max_sweeps, double tol, int* info, void* scratch,
                                  hipStream_t s) {
  constexpr int BS = JC_BS, BK = BS / 2;
  if (!info || !scratch || n < 1) return hipErrorInvalidValue;
  int nb = (n + BK - 1) / BK;
  nb += nb & 1;
  const int npairs = nb / 2;
  max_sweeps = std::min(std::max(max_sweeps, 1), 256);
  double* Rbuf = (double*)scratch;
  double* Sbuf = Rbuf + (size_t)npairs * BS * BS;
  JcCtl* ctl = (JcCtl*)(Sbuf + (size_t)npairs * BS * BS);
  const int nchunks = (n + BS - 1) / BS;
  const int nitems = npairs * (npairs + 1) / 2 + npairs * nchunks;
  const int cus = jc_compute_units();
  if (cus <= 0) return hipErrorInvalidDevice;
  const int grid = std::max(1, std::min({std::max(npairs, nitems), JC_MAX_WG, cus}));
  hipLaunchKernelGGL(k_jc_init, dim3(64), dim3(256), 0, s, U, n, ctl);
  hipLaunchKernelGGL(k_jacobi_coop<BS>, dim3(grid), dim3(BK * BK), 0, s, G, U, n, nb, max_sweeps, tol, ctl, Rbuf,
                     Sbuf, info);
  return hipGetLastError();
}

}  // namespace ttn
