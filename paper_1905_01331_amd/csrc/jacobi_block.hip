// Blocked two-sided Jacobi eigensolver for the float64 Gram matrices of the
// polar update when they are too large for one work-group's LDS (n > 64).
//
// The n indices are cut into nb blocks of BK = 16 (the last one ragged; a
// dummy block makes nb even).  A sweep is nb rounds.  In the first nb - 1
// rounds the blocks are paired by the circle method and each block pair
// (I, J) rotates exactly its cross pairs (i in I, j in J): 16 steps, step s
// rotating (I_i, J_(i+s) mod 16) for all i at once.  The last round pairs
// blocks (2j, 2j+1) and rotates the pairs inside each block (a 16-index
// circle method, 15 steps).  Every index pair is thus rotated once per
// sweep, as in the cyclic method.  A round (phase A) works on the 32 x 32
// sub-matrix G[I u J, I u J] with 2 x 2 rotations (relative threshold,
// Rutishauser diagonal updates), which yields an orthogonal R and the
// rotated sub-matrix S' = R G_sub R^T; phase B replaces every block of G
// between two index sets X, Y of the round by R_X G[X,Y] R_Y^T (S' on the
// diagonal) and the rows X of the eigenvector matrix U by R_X U[X,:].  The
// iteration ends when no pair meets the rotation test: every pair is tested
// before a sweep, so the sweep that would rotate nothing is not run.
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
constexpr long long JC_SPIN_LIMIT = 1LL << 21;  // about two seconds of polling
constexpr int JC_FLAG_STRIDE = 32;              // one 128-byte line per work-group flag

struct JcCtl {
  unsigned flag[JC_MAX_WG * JC_FLAG_STRIDE];  // barrier epoch reached by each work-group
  int abort;       // set when a barrier wait exceeded its bound
  int pad[3];
  int cnt[256];    // rotations per sweep
  int rnd[64];     // rotations per round index, summed over sweeps
  int need[256];   // set when some pair met the rotation test before a sweep
};

// Block pair j of round r (rounds 0 .. nb-2: circle method; round nb-1:
// neighbouring blocks, for the pairs inside each block).
__device__ __forceinline__ void jc_pair(int nb, int r, int j, int& I, int& J) {
  if (r == nb - 1) { I = 2 * j; J = 2 * j + 1; }
  else if (j == 0) { I = r; J = nb - 1; }
  else { I = (r + j) % (nb - 1); J = (r - j + (nb - 1)) % (nb - 1); }
}

// Grid barrier.  Every thread waits until its own global stores have been
// acknowledged (vmcnt(0)) and the work-group meets; thread 0 publishes at
// device scope (the agent-scope fence writes this compute unit's side of the
// L2 back for the other XCDs) and stores the barrier's epoch in the
// work-group's own flag.  Each flag has a cache line of its own and is
// written by one work-group only, so arrivals never queue on one address (a
// shared arrival counter serialises the grid's atomics: with it a sweep of
// order 256, 100 work-groups, took a fifth longer).  Thread i < grid then
// polls flag i, the work-group meets, and thread 0 acquires (the fence
// invalidates the stale lines of this compute unit) before the work-group
// meets again.
// Returns false after an abort.
__device__ bool jc_grid_sync(JcCtl* ctl, unsigned& epoch, int* ok_lds) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_store(&ctl->flag[blockIdx.x * JC_FLAG_STRIDE], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int ok = 1;
  if (threadIdx.x < gridDim.x) {
    const unsigned* f = &ctl->flag[threadIdx.x * JC_FLAG_STRIDE];
    long long spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (++spins > JC_SPIN_LIMIT) {
        atomicExch(&ctl->abort, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) {
    __threadfence();
    *ok_lds = ok;
  }
  __syncthreads();
  return *ok_lds != 0;
}

// Local index pair (p, q), p < q, of rotation k (0..15) at step st of a
// round on a 32-index sub-problem.  Cross round: p = k, q = 16 + (k + st) mod
// 16.  Intra round: rotations 0..7 run the circle method on indices 0..15
// (index 15 fixed), rotations 8..15 the same on indices 16..31.  Plain
// arithmetic (no tables), so that everything stays in registers.
template <bool CROSS>
__device__ __forceinline__ void jc_pq(int st, int k, int& p, int& q) {
  if constexpr (CROSS) {
    p = k;
    q = 16 + ((k + st) & 15);
  } else {
    const int kk = k & 7, off = k & 8 ? 16 : 0;
    int a, b;
    if (kk == 0) { a = st; b = 15; }
    else {
      a = st + kk; a = a >= 15 ? a - 15 : a;
      b = st - kk; b = b < 0 ? b + 15 : b;
    }
    p = off + (a < b ? a : b);
    q = off + (a < b ? b : a);
  }
}

constexpr int JC_BS = 32, JC_BK = 16, JC_LD = JC_BS + 1;
static_assert(JC_MAX_WG <= JC_BK * JC_BK, "every flag of the grid barrier needs a polling thread");

// Wave 0 of phase A: the sequential steps of one round on the 32 x 32
// sub-problem in Sc (double buffered with Sn).  Lane l computes rotation
// l % 16, the others read it by lane shuffles; each lane updates four 2 x 2
// blocks.  The rotations of step st go to rc[st][k], rs[st][k], and step_lds
// is raised to st once they are written.  Returns the lane's count of
// rotations made.
template <bool CROSS>
__device__ int jc_wave0(double* Sc, double* Sn, unsigned long long vmask, double tol, double (*rc)[JC_BK],
                        double (*rs)[JC_BK], int* step_lds, int lane) {
  constexpr int BK = JC_BK, LD = JC_LD, NB = BK * BK / 64, NS = CROSS ? BK : BK - 1;
  const int kr = lane % BK;         // rotation computed by this lane
  const int k1 = lane / (64 / BK);  // row pair of this lane's blocks
  const int k2b = lane % (64 / BK); // first column pair; then + 64/BK ...
  int rot = 0;
  for (int rr = 0; rr < NS; ++rr) {
    int pr, qr, p1, q1, p2[NB], q2[NB];
    jc_pq<CROSS>(rr, kr, pr, qr);
    jc_pq<CROSS>(rr, k1, p1, q1);
#pragma unroll
    for (int u = 0; u < NB; ++u) jc_pq<CROSS>(rr, k2b + u * (64 / BK), p2[u], q2[u]);
    // every LDS read of the step first, then the arithmetic
    const double app = Sc[pr * LD + pr], aqq = Sc[qr * LD + qr], apq = Sc[pr * LD + qr];
    double bpp[NB], bpq[NB], bqp[NB], bqq[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      bpp[u] = Sc[p1 * LD + p2[u]]; bpq[u] = Sc[p1 * LD + q2[u]];
      bqp[u] = Sc[q1 * LD + p2[u]]; bqq[u] = Sc[q1 * LD + q2[u]];
    }
    const bool real = (vmask >> pr) & (vmask >> qr) & 1ull;
    double c, sn, t;
    const bool did = jacobi_rotation(app, aqq, real ? apq : 0.0, tol, c, sn, t);
    if (lane < BK) {
      rc[rr][lane] = c;
      rs[rr][lane] = sn;
      rot += did ? 1 : 0;
    }
    const double c1 = __shfl(c, k1), s1 = __shfl(sn, k1), t1 = __shfl(t, k1);
    double c2[NB], s2[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      c2[u] = __shfl(c, k2b + u * (64 / BK));
      s2[u] = __shfl(sn, k2b + u * (64 / BK));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const double gpp = bpp[u], gpq = bpq[u], gqp = bqp[u], gqq = bqq[u];
      double npp, npq, nqp, nqq;
      if (k1 == k2b + u * (64 / BK) && s1 != 0.0) {
        npp = gpp - t1 * gpq;
        nqq = gqq + t1 * gpq;
        npq = 0.0;
        nqp = 0.0;
      } else {
        double rp_p = c1 * gpp - s1 * gqp, rp_q = c1 * gpq - s1 * gqq;
        double rq_p = s1 * gpp + c1 * gqp, rq_q = s1 * gpq + c1 * gqq;
        npp = c2[u] * rp_p - s2[u] * rp_q; npq = s2[u] * rp_p + c2[u] * rp_q;
        nqp = c2[u] * rq_p - s2[u] * rq_q; nqq = s2[u] * rq_p + c2[u] * rq_q;
      }
      Sn[p1 * LD + p2[u]] = npp; Sn[p1 * LD + q2[u]] = npq;
      Sn[q1 * LD + p2[u]] = nqp; Sn[q1 * LD + q2[u]] = nqq;
    }
    // publish the record of step rr to the waves that accumulate R
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(step_lds, rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // one wave: LDS operations complete in order; keep the compiler from
    // moving the next step's reads above these writes
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double* tp = Sc; Sc = Sn; Sn = tp;
  }
  return rot;
}

// Waves 1 and 2 of phase A: R = J_last ... J_0 (rows rotated), one step
// behind wave 0.  Wave w owns columns 16 (w - 1) .. 16 w - 1; lane l works on
// column 16 (w - 1) + l % 16 with rotations l / 16 + 4 u, u = 0..3 (the
// rotations of one step touch disjoint rows, and a column is one wave's).
template <bool CROSS>
__device__ void jc_build_r(double* R, const double (*rc)[JC_BK], const double (*rs)[JC_BK], const int* step_lds,
                           int wave, int lane) {
  constexpr int LD = JC_LD, NS = CROSS ? JC_BK : JC_BK - 1;
  const int col = (wave - 1) * 16 + (lane & 15);
  const int kb = lane >> 4;
  for (int rr = 0; rr < NS; ++rr) {
    // wave 0 always completes its steps, so this wait ends
    while (__hip_atomic_load(step_lds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < rr)
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = kb + 4 * u;
      int p, q;
      jc_pq<CROSS>(rr, k, p, q);
      const double c = rc[rr][k], sn = rs[rr][k];
      const double up = R[p * LD + col], uq = R[q * LD + col];
      R[p * LD + col] = c * up - sn * uq;
      R[q * LD + col] = sn * up + c * uq;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

template <int BS>
__global__ __launch_bounds__((BS / 2) * (BS / 2)) void k_jacobi_coop(double* __restrict__ G, double* __restrict__ U,
                                                                   int n, int nb, int max_sweeps, double tol,
                                                                   JcCtl* __restrict__ ctl, double* __restrict__ Rbuf,
                                                                   double* __restrict__ Sbuf, int* __restrict__ info,
                                                                   const int* __restrict__ skip) {
  if (skip && *skip) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { info[0] = 0; info[1] = 0; }
    return;
  }
  constexpr int BK = BS / 2;   // block width
  constexpr int NT = BK * BK;  // threads: one 2 x 2 block of S each
  constexpr int LD = BS + 1;
  constexpr int RS = NT / BS;  // row stride of the four outputs per thread in phase B
  __shared__ double L0[BS * LD], L1[BS * LD], L2[BS * LD];
  __shared__ int gx[BS], gy[BS];
  __shared__ int ok_lds, rot_lds;
  __shared__ int seen[64];  // rnd[] as read at the previous visit of each round
  __shared__ double rc_lds[BK][BK], rs_lds[BK][BK];  // rotations of one round, [step][rotation]
  __shared__ int step_lds;  // last step whose rotations wave 0 has recorded
  static_assert(BS == 32, "the wave split of phase A is written for 32 x 32 sub-problems (four waves)");
  if (threadIdx.x < 64) seen[threadIdx.x] = 0;
  const int tid = threadIdx.x;
  const int npairs = nb / 2;
  const int ng = npairs * (npairs + 1) / 2;
  const int nchunks = (n + BS - 1) / BS;
  const int nitems = ng + npairs * nchunks;
  unsigned epoch = 0;
  int sweeps = max_sweeps;
  bool alive = true;

  auto gidx = [&](int I, int J, int i) {
    int g = i < BK ? I * BK + i : J * BK + (i - BK);
    return g < n ? g : -1;
  };

  for (int sw = 0; sw < max_sweeps && alive; ++sw) {
    // A sweep rotates nothing exactly when no pair meets the rotation test
    // on the current matrix (which then stays as it is), so test every pair
    // first: the sweep that would only confirm convergence is not run, and
    // G, U and the sweep count come out as they would after it.  Both
    // triangles are tested, as a sub-problem may read either copy of an
    // off-diagonal entry (the two can differ by rounding).
    {
      int need = 0;
      const long long nn = (long long)n * n;
      for (long long e = (long long)blockIdx.x * NT + tid; e < nn; e += (long long)gridDim.x * NT) {
        const int i = (int)(e / n), j = (int)(e - (long long)i * n);
        if (j == i) continue;
        const double gpq = G[e];
        const double gpp = G[(long long)i * n + i], gqq = G[(long long)j * n + j];
        if (gpq != 0.0 && gpq * gpq > tol * tol * fabs(gpp * gqq)) need = 1;
      }
      need = __syncthreads_or(need);
      if (tid == 0 && need) atomicOr(&ctl->need[sw], 1);
    }
    if (!jc_grid_sync(ctl, epoch, &ok_lds)) { alive = false; break; }
    if (__hip_atomic_load(&ctl->need[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      sweeps = sw;
      break;
    }
    for (int r = 0; r < nb; ++r) {
      const bool cross = r < nb - 1;
      const int nsteps = cross ? BK : BK - 1;
      // ---------------- phase A: one block pair per work-group ----------------
      // wave 0 runs the round's steps (jc_wave0) while waves 1 and 2 build R
      // one step behind (jc_build_r): no work-group barrier inside a round
      for (int j = blockIdx.x; j < npairs; j += gridDim.x) {
        int I, J;
        jc_pair(nb, r, j, I, J);
        __syncthreads();
        if (tid < BS) gx[tid] = gidx(I, J, tid);
        if (tid == 0) { rot_lds = 0; step_lds = -1; }
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
        const int wave = tid >> 6, lane = tid & 63;
        if (wave == 0) {
          unsigned long long vmask = 0;  // bit i: index i of the sub-problem is real
          for (int i = 0; i < BS; ++i) vmask |= (unsigned long long)(gx[i] >= 0) << i;
          const int rot = cross ? jc_wave0<true>(Sc, Sn, vmask, tol, rc_lds, rs_lds, &step_lds, lane)
                                : jc_wave0<false>(Sc, Sn, vmask, tol, rc_lds, rs_lds, &step_lds, lane);
          if (rot) atomicAdd(&rot_lds, rot);
        } else if (wave <= 2) {
          if (cross) jc_build_r<true>(R, rc_lds, rs_lds, &step_lds, wave, lane);
          else jc_build_r<false>(R, rc_lds, rs_lds, &step_lds, wave, lane);
        }
        __syncthreads();
        // the final S is in the buffer written by the last step
        const double* Sf = (nsteps & 1) ? L1 : L0;
        if (tid == 0 && rot_lds) {
          atomicAdd(&ctl->cnt[sw], rot_lds);
          atomicAdd(&ctl->rnd[r], rot_lds);
        }
        double* Ro = Rbuf + (long long)j * BS * BS;
        double* So = Sbuf + (long long)j * BS * BS;
        for (int e = tid; e < BS * BS; e += NT) {
          int i = e / BS, k = e - i * BS;
          Ro[e] = R[i * LD + k];
          So[e] = Sf[i * LD + k];
        }
      }
      if (!jc_grid_sync(ctl, epoch, &ok_lds)) { alive = false; break; }
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
      if (!jc_grid_sync(ctl, epoch, &ok_lds)) { alive = false; break; }
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

__global__ void k_jc_init(double* __restrict__ U, int n, JcCtl* __restrict__ ctl, const int* __restrict__ skip) {
  if (skip && *skip) return;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)n * n;
       e += (long long)gridDim.x * blockDim.x)
    U[e] = (e / n == e % n) ? 1.0 : 0.0;
  if (blockIdx.x == 0) {
    int* w = (int*)ctl;
    for (int i = threadIdx.x; i < (int)(sizeof(JcCtl) / sizeof(int)); i += blockDim.x) w[i] = 0;
  }
}


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
                                  hipStream_t s, const int* skip) {
  constexpr int BS = JC_BS, BK = BS / 2;
  if (!info || !scratch || n < 1) return hipErrorInvalidValue;
  if (grp().count != 1) return hipErrorInvalidValue;  // the grid barrier needs one problem per launch
  int nb = (n + BK - 1) / BK;
  nb += nb & 1;
  if (nb > 64) return hipErrorInvalidValue;  // per-round counters hold 64 rounds (n <= 1024)
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
  hipLaunchKernelGGL(k_jc_init, dim3(64), dim3(256), 0, s, U, n, ctl, skip);
  hipLaunchKernelGGL(k_jacobi_coop<BS>, dim3(grid), dim3(BK * BK), 0, s, G, U, n, nb, max_sweeps, tol, ctl, Rbuf,
                     Sbuf, info, skip);
  return hipGetLastError();
}

}  // namespace ttn
