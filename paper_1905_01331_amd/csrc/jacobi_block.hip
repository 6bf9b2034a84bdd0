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
// The whole iteration is ONE launch of a persistent grid.  Phase B of a
// round and phase A of the next run side by side, between two grid
// barriers: phase B writes the next matrix into a second copy while phase
// A's work-groups (one block pair each) assemble their sub-problems from the
// current copy and the previous round's R and S records, with the same
// arithmetic as phase B's, so the two agree bit for bit and a round costs
// one barrier.  The grid never exceeds the number of compute units and a
// work-group needs far less than one compute unit's resources, so every
// work-group of the grid is resident at once.  Each barrier wait is bounded:
// past the bound the kernel raises an abort flag, every work-group leaves at
// its next barrier, and info[0] = -1 reports the failure to the host.
#include "common.h"
#include "jacobi.h"
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

// Scratch layout: the control block, two slots (round parity) of R and of S
// records (npairs 32 x 32 each), then the second copy of G.
constexpr size_t JC_CTL_BYTES = (sizeof(JcCtl) + 255) / 256 * 256;

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

// Phase A's steps of one round on the 32 x 32 sub-problem in Sc (double
// buffered with Sn), all four waves of the work-group in lockstep, one
// work-group barrier per step.  Every lane computes rotation lane % 16 of
// the step (its wave reads the others by lane shuffles); thread t updates
// the 2 x 2 block of row pair (t % 64) / 4 and column pair t % 4 + 4 (t / 64)
// of S, and rows p, q of R (R <- J R) for rotation t % 16 in columns t / 16
// and t / 16 + 16.  The rotations of one step touch disjoint index pairs, so
// these updates are independent.  Returns the rotations made (counted by
// lanes 0..15 of wave 0).
// lt: the thread's index among the 256 that share the sub-problem; threads
// with `active` false (a work-group running fewer sub-problems than it has
// thread groups) only meet the barriers.
template <bool CROSS>
__device__ int jc_round(double* Sc, double* Sn, double* R, unsigned long long vmask, double tol, int lt,
                        bool active) {
  constexpr int BK = JC_BK, LD = JC_LD, NS = CROSS ? BK : BK - 1;
  const int tid = lt, lane = tid & 63, wave = tid >> 6;
  const int kr = lane % BK;                      // rotation computed by this lane (and this thread's R rows)
  const int k1 = lane / (64 / BK);               // row pair of this thread's block of S
  const int k2 = lane % (64 / BK) + 4 * wave;    // its column pair
  const int col = tid / BK;                      // its columns of R: col, col + 16
  int rot = 0;
  for (int rr = 0; rr < NS; ++rr) {
    if (!active) {
      __syncthreads();
      continue;
    }
    int pr, qr, p1, q1, p2, q2;
    jc_pq<CROSS>(rr, kr, pr, qr);
    jc_pq<CROSS>(rr, k1, p1, q1);
    jc_pq<CROSS>(rr, k2, p2, q2);
    // every LDS read of the step first, then the arithmetic
    const double app = Sc[pr * LD + pr], aqq = Sc[qr * LD + qr], apq = Sc[pr * LD + qr];
    const double gpp = Sc[p1 * LD + p2], gpq = Sc[p1 * LD + q2];
    const double gqp = Sc[q1 * LD + p2], gqq = Sc[q1 * LD + q2];
    const double up0 = R[pr * LD + col], uq0 = R[qr * LD + col];
    const double up1 = R[pr * LD + col + BK], uq1 = R[qr * LD + col + BK];
    const bool real = (vmask >> pr) & (vmask >> qr) & 1ull;
    double c, sn, t;
    const bool did = jacobi_rotation(app, aqq, real ? apq : 0.0, tol, c, sn, t);
    if (wave == 0 && lane < BK) rot += did ? 1 : 0;
    const double c1 = __shfl(c, k1), s1 = __shfl(sn, k1), t1 = __shfl(t, k1);
    const double c2 = __shfl(c, k2), s2 = __shfl(sn, k2);
    double npp, npq, nqp, nqq;
    if (k1 == k2 && s1 != 0.0) {
      // the rotated pair itself: exact annihilation, Rutishauser's diagonal update
      npp = gpp - t1 * gpq;
      nqq = gqq + t1 * gpq;
      npq = 0.0;
      nqp = 0.0;
    } else {
      double rp_p = c1 * gpp - s1 * gqp, rp_q = c1 * gpq - s1 * gqq;
      double rq_p = s1 * gpp + c1 * gqp, rq_q = s1 * gpq + c1 * gqq;
      npp = c2 * rp_p - s2 * rp_q; npq = s2 * rp_p + c2 * rp_q;
      nqp = c2 * rq_p - s2 * rq_q; nqq = s2 * rq_p + c2 * rq_q;
    }
    Sn[p1 * LD + p2] = npp; Sn[p1 * LD + q2] = npq;
    Sn[q1 * LD + p2] = nqp; Sn[q1 * LD + q2] = nqq;
    R[pr * LD + col] = c * up0 - sn * uq0;
    R[qr * LD + col] = sn * up0 + c * uq0;
    R[pr * LD + col + BK] = c * up1 - sn * uq1;
    R[qr * LD + col + BK] = sn * up1 + c * uq1;
    __syncthreads();
    double* tp = Sc; Sc = Sn; Sn = tp;
  }
  return rot;
}

// Phase B's block product of round r for the block pair (x, y), x < y,
// restricted to rows r0 .. r0 + 15 of pair x and columns c0 .. c0 + 15 of
// pair y: out = (R_x G[X, Y] R_y^T)[rows, columns], each entry the same
// chain of fused multiply-adds as phase B's (so the same bits).  Uses L1, L2,
// L3; the 16 x 16 result is left in L1 at [r][c].
template <int BS>
__device__ void jc_cross_block(const double* __restrict__ Gc, int n, const double* __restrict__ Rx,
                               const double* __restrict__ Ry, const int* gxa, const int* gyb, int r0, int c0,
                               double* L1, double* L2, double* L3) {
  constexpr int BK = BS / 2, NT = BK * BK, LD = BS + 1;
  const int tid = threadIdx.x;
  for (int e = tid; e < BS * BS; e += NT) {
    const int i = e / BS, k = e - i * BS;
    const int gi = gxa[i], gk = gyb[k];
    L1[i * LD + k] = (gi >= 0 && gk >= 0) ? Gc[(long long)gi * n + gk] : 0.0;
  }
  for (int e = tid; e < BK * BS; e += NT) {
    const int i = e / BS, k = e - i * BS;
    L2[i * LD + k] = Ry[(c0 + i) * BS + k];  // row c of R_y restricted to the columns kept
    L3[i * LD + k] = Rx[(r0 + i) * BS + k];  // row r of R_x restricted to the rows kept
  }
  __syncthreads();
  // T[m][c] = sum_m' G[X_m, Y_m'] R_y[c0 + c][m'], m = 0..31, c = 0..15
  double t[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * NT, m = e / BK, c = e - m * BK;
    double acc = 0.0;
    for (int q = 0; q < BS; ++q) acc = fma(L1[m * LD + q], L2[c * LD + q], acc);
    t[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * NT, m = e / BK, c = e - m * BK;
    L2[m * LD + c] = t[u];  // T, 32 x 16
  }
  __syncthreads();
  {
    const int r = tid / BK, c = tid - r * BK;
    double acc = 0.0;
    for (int m = 0; m < BS; ++m) acc = fma(L3[r * LD + m], L2[m * LD + c], acc);
    L1[r * LD + c] = acc;
  }
  __syncthreads();
}

template <int BS>
__global__ __launch_bounds__((BS / 2) * (BS / 2)) void k_jacobi_coop(double* __restrict__ G, double* __restrict__ U,
                                                                   int n, int nb, int max_sweeps, double tol,
                                                                   JcCtl* __restrict__ ctl, double* __restrict__ Rbuf,
                                                                   double* __restrict__ Sbuf, double* __restrict__ Galt,
                                                                   int* __restrict__ info,
                                                                   const int* __restrict__ skip) {
  if (skip && *skip) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { info[0] = 0; info[1] = 0; }
    return;
  }
  constexpr int BK = BS / 2;   // block width
  constexpr int NT = BK * BK;  // threads: one 2 x 2 block of S each
  constexpr int LD = BS + 1;
  constexpr int RS = NT / BS;  // row stride of the four outputs per thread in phase B
  __shared__ double L0[BS * LD], L1[BS * LD], L2[BS * LD], L3[BS * LD];
  __shared__ int gx[BS], gy[BS], gz[BS];
  __shared__ int ok_lds, rot_lds;
  __shared__ int seen[64];  // rnd[] as read at the previous visit of each round
  __shared__ int inv[64];   // 2 * pair + half of every block in the previous round
  static_assert(BS == 32, "the wave split of phase A is written for 32 x 32 sub-problems (four waves)");
  if (threadIdx.x < 64) seen[threadIdx.x] = 0;
  const int tid = threadIdx.x;
  const int npairs = nb / 2;
  const int ng = npairs * (npairs + 1) / 2;
  const int nchunks = (n + BS - 1) / BS;
  const int nitems = ng + npairs * nchunks;
  const long long rec = (long long)npairs * BS * BS;  // one round's R (or S) records
  // phase A on work-groups 0 .. npairs - 1, phase B on the others (on all of
  // them, after phase A, when the grid has no others)
  const int b0 = (int)gridDim.x > npairs ? npairs : 0;
  const int bw = (int)blockIdx.x - b0, bstride = (int)gridDim.x - b0;
  double* Gc = G;     // the matrix as the current epoch starts
  double* Gn = Galt;  // the other copy, where phase B writes the next one
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
        const double gpq = Gc[e];
        const double gpp = Gc[(long long)i * n + i], gqq = Gc[(long long)j * n + j];
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
    // Epoch q runs phase A of round q and, beside it, phase B of round q - 1
    // (epoch nb: phase B of the last round alone).  Phase B reads the matrix
    // as round q - 1 found it (Gc) and writes the next one to Gn; phase A of
    // round q takes its sub-problem from Gc and the records of round q - 1,
    // computing exactly the entries phase B writes there, so both agree bit
    // for bit.  R and S records alternate between two slots by round parity.
    for (int q = 0; q <= nb; ++q) {
      // phase B of round q - 1 runs only if that round rotated (every
      // work-group reads the same count after the barrier)
      bool rot_b = false;
      if (q > 0) {
        const int rv = __hip_atomic_load(&ctl->rnd[q - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        rot_b = rv != seen[q - 1];
        __syncthreads();
        if (tid == 0) seen[q - 1] = rv;
      }
      const double* Rp = Rbuf + ((q - 1) & 1) * rec;  // records of round q - 1
      const double* Sp = Sbuf + ((q - 1) & 1) * rec;
      // ---------------- phase A of round q: one block pair per work-group ----------------
      // the four waves run the round's steps together (jc_round)
      if (q < nb) {
        const int r = q;
        const bool cross = r < nb - 1;
        const int nsteps = cross ? BK : BK - 1;
        for (int j = blockIdx.x; j < npairs; j += gridDim.x) {
          int I, J;
          jc_pair(nb, r, j, I, J);
          __syncthreads();
          if (tid < BS) gx[tid] = gidx(I, J, tid);
          if (tid == 0) rot_lds = 0;
          if (r > 0 && tid < npairs) {
            int Ip, Jp;
            jc_pair(nb, r - 1, tid, Ip, Jp);
            inv[Ip] = 2 * tid;
            inv[Jp] = 2 * tid + 1;
          }
          __syncthreads();
          double* Sc = L0;
          double* Sn = L1;
          double* R = L2;
          if (r == 0) {
            for (int e = tid; e < BS * BS; e += NT) {
              int i = e / BS, k = e - i * BS;
              int gi = gx[i], gk = gx[k];
              Sc[i * LD + k] = (gi >= 0 && gk >= 0) ? Gc[(long long)gi * n + gk] : 0.0;
            }
          } else {
            // G[I u J, I u J] after round r - 1: the blocks inside one pair
            // of that round from its S record, the cross block from its R
            // records and Gc
            const int c1 = inv[I], c2 = inv[J];
            const int x1 = c1 >> 1, h1 = c1 & 1, x2 = c2 >> 1, h2 = c2 & 1;
            const double* S1 = Sp + (long long)x1 * BS * BS;
            const double* S2 = Sp + (long long)x2 * BS * BS;
            for (int e = tid; e < BK * BK; e += NT) {
              const int i = e / BK, k = e - i * BK;
              Sc[i * LD + k] = S1[(h1 * BK + i) * BS + h1 * BK + k];
              Sc[(BK + i) * LD + BK + k] = S2[(h2 * BK + i) * BS + h2 * BK + k];
              if (x1 == x2) {
                Sc[i * LD + BK + k] = S1[(h1 * BK + i) * BS + h2 * BK + k];
                Sc[(BK + i) * LD + k] = S1[(h2 * BK + i) * BS + h1 * BK + k];
              }
            }
            if (x1 != x2) {
              // phase B computes the block of the pair with the lower index
              const int xa = x1 < x2 ? x1 : x2, xb = x1 < x2 ? x2 : x1;
              const int ha = x1 < x2 ? h1 : h2, hb = x1 < x2 ? h2 : h1;
              int Ia, Ja, Ib, Jb;
              jc_pair(nb, r - 1, xa, Ia, Ja);
              jc_pair(nb, r - 1, xb, Ib, Jb);
              if (tid < BS) { gy[tid] = gidx(Ia, Ja, tid); gz[tid] = gidx(Ib, Jb, tid); }
              __syncthreads();
              jc_cross_block<BS>(Gc, n, Rp + (long long)xa * BS * BS, Rp + (long long)xb * BS * BS, gy, gz,
                                 ha * BK, hb * BK, L1, L2, L3);
              for (int e = tid; e < BK * BK; e += NT) {
                const int i = e / BK, k = e - i * BK;
                const double v = L1[i * LD + k];
                if (x1 < x2) { Sc[i * LD + BK + k] = v; Sc[(BK + k) * LD + i] = v; }
                else { Sc[(BK + i) * LD + k] = v; Sc[k * LD + BK + i] = v; }
              }
            }
            __syncthreads();
            // entries of padding indices read as zero, as from G
            for (int e = tid; e < BS * BS; e += NT) {
              const int i = e / BS, k = e - i * BS;
              if (gx[i] < 0 || gx[k] < 0) Sc[i * LD + k] = 0.0;
            }
          }
          __syncthreads();
          for (int e = tid; e < BS * BS; e += NT) {
            int i = e / BS, k = e - i * BS;
            R[i * LD + k] = (i == k) ? 1.0 : 0.0;
          }
          __syncthreads();
          {
            unsigned long long vmask = 0;  // bit i: index i of the sub-problem is real
            for (int i = 0; i < BS; ++i) vmask |= (unsigned long long)(gx[i] >= 0) << i;
            const int rot = cross ? jc_round<true>(Sc, Sn, R, vmask, tol, tid, true)
                                  : jc_round<false>(Sc, Sn, R, vmask, tol, tid, true);
            if (rot) atomicAdd(&rot_lds, rot);
          }
          __syncthreads();
          // the final S is in the buffer written by the last step
          const double* Sf = (nsteps & 1) ? L1 : L0;
          if (tid == 0 && rot_lds) {
            atomicAdd(&ctl->cnt[sw], rot_lds);
            atomicAdd(&ctl->rnd[r], rot_lds);
          }
          double* Ro = Rbuf + (r & 1) * rec + (long long)j * BS * BS;
          double* So = Sbuf + (r & 1) * rec + (long long)j * BS * BS;
          for (int e = tid; e < BS * BS; e += NT) {
            int i = e / BS, k = e - i * BS;
            Ro[e] = R[i * LD + k];
            So[e] = Sf[i * LD + k];
          }
        }
      }
      // ---------------- phase B of round q - 1: blocks of G and panels of U ----------------
      if (rot_b && bw >= 0) {
        const int r = q - 1;
        for (int item = bw; item < nitems; item += bstride) {
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
              const double* Sx = Sp + (long long)x * BS * BS;
              for (int e = tid; e < BS * BS; e += NT) {
                int i = e / BS, k = e - i * BS;
                int gi = gx[i], gk = gx[k];
                if (gi >= 0 && gk >= 0) Gn[(long long)gi * n + gk] = Sx[e];
              }
              continue;
            }
            const double* Rx = Rp + (long long)x * BS * BS;
            const double* Ry = Rp + (long long)y * BS * BS;
            for (int e = tid; e < BS * BS; e += NT) {
              int i = e / BS, k = e - i * BS;
              int gi = gx[i], gk = gy[k];
              L0[i * LD + k] = (gi >= 0 && gk >= 0) ? Gc[(long long)gi * n + gk] : 0.0;
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
                Gn[(long long)gi * n + gk] = acc[u];
                Gn[(long long)gk * n + gi] = acc[u];
              }
            }
          } else {
            const int it = item - ng;
            const int x = it / nchunks, c0 = (it - x * nchunks) * BS;
            int Ix, Jx;
            jc_pair(nb, r, x, Ix, Jx);
            if (tid < BS) gx[tid] = gidx(Ix, Jx, tid);
            __syncthreads();
            const double* Rx = Rp + (long long)x * BS * BS;
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
      }
      if (q < nb || rot_b) {
        if (!jc_grid_sync(ctl, epoch, &ok_lds)) { alive = false; break; }
      }
      if (rot_b) { double* t = Gc; Gc = Gn; Gn = t; }
    }
    if (!alive) break;
    // every work-group reads the same final count after the barrier
    if (__hip_atomic_load(&ctl->cnt[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      sweeps = sw;
      break;
    }
  }
  // the result goes back to the caller's matrix (every write to Gc is behind
  // the last barrier)
  if (Gc != G) {
    for (long long e = (long long)blockIdx.x * NT + tid; e < (long long)n * n; e += (long long)gridDim.x * NT)
      G[e] = Gc[e];
  }
  if (blockIdx.x == 0 && tid == 0) {
    info[0] = alive ? sweeps : -1;
    info[1] = ctl->cnt[0];
  }
}


// ---------------------------------------------------------------------------
// The same blocked method inside ONE work-group (1024 threads), for orders
// 32 < n <= 96: G (padded to nb blocks of 16) in LDS, the eigenvector matrix
// in global memory.  Each of the round's block pairs (at most three) is
// rotated by a group of 256 threads (jc_round), then the whole work-group
// updates the blocks of G between two pairs and the rows of U in 32 x 32
// products, four at a time, with work-group barriers in place of the grid
// barriers.  One work-group per problem, so a launch group's members run side
// by side in one launch (blockIdx.y = member).
// ---------------------------------------------------------------------------
constexpr int JL_THREADS = 1024;
constexpr int JL_MAXP = 3;  // block pairs of one round (n <= 96)

__global__ __launch_bounds__(JL_THREADS) void k_jacobi_lds(double* __restrict__ Gg, double* __restrict__ Ug, int n,
                                                          int max_sweeps, double tol, int* __restrict__ info,
                                                          const int* __restrict__ skip, long long ms_) {
  Gg = mshift(Gg, ms_); Ug = mshift(Ug, ms_); info = mshift(info, ms_); skip = mshift(skip, ms_);
  if (skip && *skip) {
    if (threadIdx.x == 0 && info) { info[0] = 0; info[1] = 0; }
    return;
  }
  constexpr int BS = JC_BS, BK = JC_BK, LD = JC_LD, SUB = BS * LD, RS = 256 / BS;
  extern __shared__ double dyn[];
  __shared__ int gxs[4][BS], gys[4][BS];
  __shared__ int rot_l, cnt_l;
  int nb = (n + BK - 1) / BK;
  nb += nb & 1;
  const int np = nb * BK, LG = np + 1, npairs = nb / 2;
  double* G = dyn;                       // np x np, row stride LG; padding rows and columns stay zero
  double* P = G + (size_t)np * LG;       // pair p: S, S', R (SUB doubles each)
  const int tid = threadIdx.x, grp = tid >> 8, lt = tid & 255;
  for (int e = tid; e < np * np; e += JL_THREADS) {
    const int i = e / np, k = e - i * np;
    G[i * LG + k] = (i < n && k < n) ? Gg[(long long)i * n + k] : 0.0;
  }
  for (int e = tid; e < n * n; e += JL_THREADS) Ug[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  // phase B's thread groups each use a free S buffer of the pairs as scratch
  const int slots = 2 * npairs < 4 ? 2 * npairs : 4;
  const int ngi = npairs * (npairs - 1) / 2;  // blocks between two pairs (x < y)
  const int nch = (n + BS - 1) / BS;
  const int nitems = ngi + npairs * nch;
  int sweep = 0, first_rot = -1;
  for (; sweep < max_sweeps; ++sweep) {
    // the sweep that would rotate nothing is not run (as in the grid solver)
    int need = 0;
    for (int e = tid; e < n * n; e += JL_THREADS) {
      const int i = e / n, j = e - i * n;
      if (j == i) continue;
      const double gpq = G[i * LG + j], gpp = G[i * LG + i], gqq = G[j * LG + j];
      if (gpq != 0.0 && gpq * gpq > tol * tol * fabs(gpp * gqq)) need = 1;
    }
    if (!__syncthreads_or(need)) break;
    if (tid == 0) cnt_l = 0;
    for (int r = 0; r < nb; ++r) {
      const bool cross = r < nb - 1;
      const int nsteps = cross ? BK : BK - 1;
      // ---- phase A: thread group p rotates block pair p ----
      const bool act = grp < npairs;
      double* Sc = P + (size_t)(act ? grp : 0) * 3 * SUB;
      double* Sn = Sc + SUB;
      double* R = Sn + SUB;
      if (act && lt < BS) {
        int I, J;
        jc_pair(nb, r, grp, I, J);
        gxs[grp][lt] = lt < BK ? I * BK + lt : J * BK + (lt - BK);
      }
      if (tid == 0) rot_l = 0;
      __syncthreads();
      if (act) {
        for (int e = lt; e < BS * BS; e += 256) {
          const int i = e / BS, k = e - i * BS;
          Sc[i * LD + k] = G[gxs[grp][i] * LG + gxs[grp][k]];
          R[i * LD + k] = (i == k) ? 1.0 : 0.0;
        }
      }
      __syncthreads();
      unsigned long long vmask = 0;  // bit i: index i of the sub-problem is real
      if (act)
        for (int i = 0; i < BS; ++i) vmask |= (unsigned long long)(gxs[grp][i] < n) << i;
      const int rot = cross ? jc_round<true>(Sc, Sn, R, vmask, tol, lt, act)
                            : jc_round<false>(Sc, Sn, R, vmask, tol, lt, act);
      if (rot) atomicAdd(&rot_l, rot);
      __syncthreads();
      if (act) {
        // the rotated sub-problem back into its diagonal block of G
        const double* Sf = (nsteps & 1) ? Sn : Sc;
        for (int e = lt; e < BS * BS; e += 256) {
          const int i = e / BS, k = e - i * BS;
          G[gxs[grp][i] * LG + gxs[grp][k]] = Sf[i * LD + k];
        }
      }
      __syncthreads();
      const int rl = rot_l;
      if (tid == 0) cnt_l += rl;
      if (rl == 0) continue;  // R = I for every pair: nothing else changes
      // ---- phase B: G blocks between two pairs, then rows of U ----
      for (int it = 0; it * slots < nitems; ++it) {
        const int item = it * slots + grp;
        const bool valid = grp < slots && item < nitems;
        const bool gitem = valid && item < ngi;
        double* T = P + (size_t)(grp >> 1) * 3 * SUB + (grp & 1) * SUB;  // an S buffer, free now
        int x = 0, y = 0, c0 = 0;
        if (valid) {
          if (gitem) {
            int rem = item;
            while (rem >= npairs - 1 - x) { rem -= npairs - 1 - x; ++x; }
            y = x + 1 + rem;
          } else {
            x = (item - ngi) / nch;
            c0 = ((item - ngi) % nch) * BS;
          }
          if (lt < BS) {
            int I, J;
            jc_pair(nb, r, x, I, J);
            gxs[grp][lt] = lt < BK ? I * BK + lt : J * BK + (lt - BK);
            if (gitem) {
              jc_pair(nb, r, y, I, J);
              gys[grp][lt] = lt < BK ? I * BK + lt : J * BK + (lt - BK);
            }
          }
        }
        __syncthreads();
        const double* Rx = P + (size_t)x * 3 * SUB + 2 * SUB;
        const double* Ry = P + (size_t)y * 3 * SUB + 2 * SUB;
        const int row = lt / BS, col = lt - (lt / BS) * BS;
        if (valid) {
          for (int e = lt; e < BS * BS; e += 256) {
            const int i = e / BS, k = e - i * BS;
            if (gitem) {
              T[i * LD + k] = G[gxs[grp][i] * LG + gys[grp][k]];
            } else {
              const int gi = gxs[grp][i], gc = c0 + k;
              T[i * LD + k] = (gi < n && gc < n) ? Ug[(long long)gi * n + gc] : 0.0;
            }
          }
        }
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (gitem) {
          // G[X,Y] R_y^T
          for (int m = 0; m < BS; ++m) {
            const double ry = Ry[col * LD + m];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(T[(row + u * RS) * LD + m], ry, acc[u]);
          }
        } else if (valid) {
          // R_x U[X, c0 ..]
          for (int m = 0; m < BS; ++m) {
            const double uv = T[m * LD + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(Rx[(row + u * RS) * LD + m], uv, acc[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int gi = gxs[grp][row + u * RS], gc = c0 + col;
            if (gi < n && gc < n) Ug[(long long)gi * n + gc] = acc[u];
          }
        }
        __syncthreads();
        if (gitem) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            T[(row + u * RS) * LD + col] = acc[u];
            acc[u] = 0.0;
          }
        }
        __syncthreads();
        if (gitem) {
          // R_x (G[X,Y] R_y^T), into both triangles
          for (int m = 0; m < BS; ++m) {
            const double tv = T[m * LD + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(Rx[(row + u * RS) * LD + m], tv, acc[u]);
          }
          const int gk = gys[grp][col];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int gi = gxs[grp][row + u * RS];
            G[gi * LG + gk] = acc[u];
            G[gk * LG + gi] = acc[u];
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const int c = cnt_l;
    if (first_rot < 0) first_rot = c;
    __syncthreads();
    if (c == 0) break;
  }
  for (int e = tid; e < n * n; e += JL_THREADS) {
    const int i = e / n, k = e - i * n;
    Gg[e] = G[i * LG + k];
  }
  if (tid == 0 && info) {
    info[0] = sweep;
    info[1] = first_rot < 0 ? 0 : first_rot;
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
  return JC_CTL_BYTES + ((size_t)4 * (nb / 2) * JC_BS * JC_BS + (size_t)n * n) * sizeof(double);
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
  JcCtl* ctl = (JcCtl*)scratch;
  double* Rbuf = (double*)((char*)scratch + JC_CTL_BYTES);
  double* Sbuf = Rbuf + (size_t)2 * npairs * BS * BS;
  double* Galt = Sbuf + (size_t)2 * npairs * BS * BS;
  const int nchunks = (n + BS - 1) / BS;
  const int nitems = npairs * (npairs + 1) / 2 + npairs * nchunks;
  const int cus = jc_compute_units();
  if (cus <= 0) return hipErrorInvalidDevice;
  // phase A's work-groups beside phase B's, as far as the compute units go
  const int grid = std::max(1, std::min({npairs + nitems, JC_MAX_WG, cus}));
  hipLaunchKernelGGL(k_jc_init, dim3(64), dim3(256), 0, s, U, n, ctl, skip);
  hipLaunchKernelGGL(k_jacobi_coop<BS>, dim3(grid), dim3(BK * BK), 0, s, G, U, n, nb, max_sweeps, tol, ctl, Rbuf,
                     Sbuf, Galt, info, skip);
  return hipGetLastError();
}

size_t jacobi_lds_bytes(int n) {
  int nb = (n + JC_BK - 1) / JC_BK;
  nb += nb & 1;
  const size_t np = (size_t)nb * JC_BK;
  return (np * (np + 1) + (size_t)(nb / 2) * 3 * JC_BS * JC_LD) * sizeof(double);
}

hipError_t jacobi_eig_lds_f64(double* G, double* U, int n, int max_sweeps, double tol, int* info, hipStream_t s,
                              const int* skip) {
  if (n <= JC_BS || n > JC_LDS_MAXN) return hipErrorInvalidValue;
  static int lds_ok = -1;
  const size_t bytes = jacobi_lds_bytes(JC_LDS_MAXN);
  if (lds_ok < 0) {
    lds_ok = hipFuncSetAttribute((const void*)k_jacobi_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes) == hipSuccess ? 1 : 0;
    (void)hipGetLastError();
  }
  if (!lds_ok) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_jacobi_lds, dim3(1, grp().count), dim3(JL_THREADS), jacobi_lds_bytes(n), s, G, U, n,
                     std::min(std::max(max_sweeps, 1), 256), tol, info, skip, grp().stride);
  return hipGetLastError();
}

}  // namespace ttn
