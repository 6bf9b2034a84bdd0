// Position-resolved binary TTN: every node (tau, m) carries its own isometry
// w^(tau, m) (the labels of Sec. II.C; the paper equates them along a layer
// only for translation-invariant Hamiltonians, Sec. III).  Float64
// throughout.
//
// Per level tau the nodes sit side by side, so that one product launch covers
// every node of a level (or every node of one parity) through the batch
// strides of the product; the node index is the outer level of a two-level
// batch whose inner level runs over the product terms k or the output rows a.
//
//   W[t]   (t >= 1)  L_t isometries [a][b][b], a = chi_t, b = chi_{t-1}
//   OPS[t]           per node [h, A_1..A_D, B_1..B_D] (chi_t^2 each): h the sum
//                    of every term inside the node's block, A_k its right
//                    edge (site j of a bond leaving the block), B_k its left
//                    edge (site j+1 of a bond arriving); level 0 holds one
//                    block, h1 - c I, A_k, B_k, read with node stride 0
//   DX[t]            per node [rho, X_1..X_D, Y_1..Y_D]: the one-site density
//                    matrix of the node's upper index and the two-site
//                    information of its edges, X_k pairing with B_k (the bond
//                    arriving from the left) and Y_k with A_k (the bond
//                    leaving to the right), so that a bond energy is one
//                    pairing and the environment of w^(tau, m) is
//                    [rho | X | Y] o [S w | B_{L,k} .l w | A_{R,k} .r w]
//   PC[t]  (t >= 1)  rho^(t, m) o w^(t, m): the descent's cache
//
// Sweep (Sec. IV, with the layer's nodes split by parity): the density
// matrices of every level once (they depend only on the tensors above and on
// v, none of which change before their layer is reached); then layer by layer
// bottom-up, for the even and then the odd nodes: X and Y from the top down
// to the layer (they depend on operators below, which the previous group
// changed), the environments of the group, the polar updates (one launch
// group over the nodes, every node's scratch in a slab of its own), the new
// operators of the group and of every level above; last the top tensor.
// Nodes of one parity are never neighbours, so each group is one exact block
// step of the energy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ttn.h"
#include "common.h"
#include "lanczos.h"
#include "ttn_core.h"

using namespace ttn;
using namespace ttn::core;

namespace {

// staging of one launch chunk of nodes (bytes); a chunk holds at least one node
constexpr size_t POS_STAGE_BYTES = 8ull << 30;
// polar slabs of one launch group of nodes (bytes): a whole parity group of a
// bulk level at chi = 128 (128 nodes of 64 MB) in one launch, so that its
// one-work-group Jacobi solves run side by side
constexpr size_t POS_SLAB_BYTES = 16ull << 30;
// order above which a node's Jacobi solves take the blocked solver, one node
// per launch (below, one work-group per node, every node of a chunk at once)
constexpr int POS_GROUP_JACOBI_MAX = 128;
constexpr int POS_ERR = 0, POS_NOCONV = 1;  // slots of the handle's flag pair
constexpr double POS_REG = 1e-30;            // tie-breaker toward the current isometry

long long al32(long long x) { return (x + 31) & ~31LL; }  // doubles to a 256-byte boundary

struct SlabLayout {  // offsets in doubles within one node's polar slab
  long long env = 0, wold = 0, Y = 0, Y2 = 0, G = 0, V = 0, Q = 0, Q2 = 0, nrm = 0, jinfo = 0, skip3 = 0, scal = 0,
            part = 0, splitk = 0, size = 0;
};
SlabLayout slab_layout(int a, int b) {
  SlabLayout S;
  const long long cube = (long long)a * b * b, aa = (long long)a * a;
  long long o = 0;
  auto take = [&](long long k) { long long r = o; o = al32(o + k); return r; };
  S.env = take(cube);
  S.wold = take(cube);
  S.Y = take(cube);
  S.Y2 = take(cube);
  S.G = take(aa);
  S.V = take(aa);
  S.Q = take(aa);
  S.Q2 = take(aa);
  S.nrm = take(a);
  S.jinfo = take(32);  // 64 ints
  S.skip3 = take(32);
  S.scal = take(SCAL_N);
  S.part = take(256);
  // split-K partial sums of the polar update's products: the Gram matrix
  // (a x a) splits at most 128 ways
  S.splitk = take(128 * aa);
  S.size = o;
  return S;
}

}  // namespace

struct ttn_pos_ctx {
  Member M;  // top solver, product launchers, template of the per-node polar update
  hipStream_t s = nullptr;
  int L = 0, n = 0, d = 0, D = 0;
  std::vector<int> dims;
  std::vector<double*> W, OPS, DX, PC;
  std::vector<long long> chunk;   // nodes per staging chunk, per level
  std::vector<long long> pchunk;  // nodes per polar launch, per level
  double* stage = nullptr;
  double* slabs = nullptr;
  double* flags = nullptr;  // [error, no convergence] of the polar Jacobi solves
  double* topR = nullptr;   // float64 top operators of the right site (symmetrised)
  bool top_conv = true;
  double last_flops = 0.0, last_bytes = 0.0;  // products of the last sweep
  Profiler prof;
  KernelRecorder krec;
  ~ttn_pos_ctx() {
    if (kernel_timer() == &krec) kernel_timer() = nullptr;
  }

  long long nodes(int t) const { return (long long)L >> t; }
  long long x2(int t) const { return (long long)dims[t] * dims[t]; }
  long long cube(int t) const { return (long long)dims[t] * dims[t - 1] * dims[t - 1]; }
  long long ops_stride(int t) const { return t == 0 ? 0 : (1 + 2LL * D) * x2(t); }
  long long dx_stride(int t) const { return (1 + 2LL * D) * x2(t); }
};

namespace {

using Pos = ttn_pos_ctx;

// two-level batch (inner count `inner`, outer count `outer`) with the given strides
void batch2(GemmDesc& g, int inner, int outer, long long a1, long long a2, long long b1, long long b2, long long c1,
            long long c2) {
  g.batch1 = inner;
  g.batch = inner * outer;
  g.sAb = a1; g.sAb2 = a2;
  g.sBb = b1; g.sBb2 = b2;
  g.sCb = c1; g.sCb2 = c2;
}

// (O .r X)[a;l,r] = sum_r' O[r,r'] X[a;l,r'] over (k, node): X at X + k xk + j xn,
// O at O + k ok + j on, Y at Y + k yk + j yn
hipError_t pos_apply_r(Pos& P, const double* O, long long ok, long long on, const double* X, long long xk,
                       long long xn, double* Y, long long yk, long long yn, int a, int b, double beta, int nk, int nn) {
  if (nk < 1 || nn < 1) return hipSuccess;
  GemmDesc g = desc0();
  g.M = a * b; g.N = b; g.K = b;
  g.A = X; g.sAm = b; g.sAk = 1;
  g.B = O; g.sBk = 1; g.sBn = b;
  g.C = Y; g.sCm = b; g.sCn = 1;
  g.beta = beta;
  batch2(g, nk, nn, xk, xn, ok, on, yk, yn);
  return run(P.M, P_F64, g, P.s, OC_APPLY_R);
}
// (O .l X)[a;l,r] = sum_l' O[l,l'] X[a;l',r] over (row a, node), one operator per node
hipError_t pos_apply_l(Pos& P, const double* O, long long on, const double* X, long long xn, double* Y, long long yn,
                       int a, int b, double beta, int nn) {
  if (nn < 1) return hipSuccess;
  const long long bb = (long long)b * b;
  GemmDesc g = desc0();
  g.M = b; g.N = b; g.K = b;
  g.A = O; g.sAm = b; g.sAk = 1;
  g.B = X; g.sBk = b; g.sBn = 1;
  g.C = Y; g.sCm = b; g.sCn = 1;
  g.beta = beta;
  batch2(g, a, nn, 0, on, bb, xn, bb, yn);
  return run(P.M, P_F64, g, P.s, OC_APPLY_L);
}
// Y[a;l,r] (+)= sum_{k,l'} O_k[l,l'] X_k[a;l',r]: O_k at O + k ok, X_k at X + k xk
hipError_t pos_apply_l_sum(Pos& P, const double* O, long long ok, long long on, const double* X, long long xk,
                           long long xn, double* Y, long long yn, int a, int b, double beta, int nk, int nn) {
  if (nk < 1 || nn < 1) return hipSuccess;
  const long long bb = (long long)b * b;
  GemmDesc g = desc0();
  g.M = b; g.N = b; g.K = nk * b; g.K2 = b;
  g.A = O; g.sAm = b; g.sAk = 1; g.sAk1 = ok;
  g.B = X; g.sBk = b; g.sBk1 = xk; g.sBn = 1;
  g.C = Y; g.sCm = b; g.sCn = 1;
  g.beta = beta;
  batch2(g, a, nn, 0, on, bb, xn, bb, yn);
  return run(P.M, P_F64, g, P.s, OC_APPLY_L);
}
// C(P,Q)[a,a'] = sum_{l,r} P[a;l,r] Q[a';l,r] over (k, node); every use has
// P = w, Q = O w with O symmetric (antisymmetric for the bits of anti, by k),
// so C is computed on its upper triangle and mirrored
hipError_t pos_close(Pos& P, const double* Pm, long long pk, long long pn, const double* Qm, long long qk, long long qn,
                     double* C, long long ck, long long cn, int a, int b, int nk, int nn, unsigned long long anti) {
  if (nk < 1 || nn < 1) return hipSuccess;
  const long long bb = (long long)b * b;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  g.M = a; g.N = a; g.K = (int)bb;
  g.A = Pm; g.sAm = bb; g.sAk = 1;
  g.B = Qm; g.sBk = 1; g.sBn = bb;
  g.C = C; g.sCm = a; g.sCn = 1;
  batch2(g, nk, nn, pk, pn, qk, qn, ck, cn);
  return run(P.M, P_F64, g, P.s, OC_CLOSE);
}
// (X o Q)[a;l,r] = sum_a' X[a,a'] Q[a';l,r] over (k, node)
hipError_t pos_left_mul(Pos& P, const double* X, long long xk, long long xn, const double* Qm, long long qk,
                        long long qn, double* Y, long long yk, long long yn, int a, int b, int nk, int nn) {
  if (nk < 1 || nn < 1) return hipSuccess;
  const long long bb = (long long)b * b;
  GemmDesc g = desc0();
  g.M = a; g.N = (int)bb; g.K = a;
  g.A = X; g.sAm = a; g.sAk = 1;
  g.B = Qm; g.sBk = bb; g.sBn = 1;
  g.C = Y; g.sCm = bb; g.sCn = 1;
  batch2(g, nk, nn, xk, xn, qk, qn, yk, yn);
  return run(P.M, P_F64, g, P.s, OC_LEFT_MUL);
}
// C_R(P,Q)[r,r'] = sum_{a,l} P[a;l,r] Q[a;l,r'] over (k, node).  The child
// closes produce the children's rho (symmetric) and edge information of the
// parity of their product term (bit k of anti: antisymmetric), so a float64
// launch computes the block upper triangle and mirrors it.
hipError_t pos_close_r(Pos& P, const double* Pm, long long pk, long long pn, const double* Qm, long long qk,
                       long long qn, double* C, long long ck, long long cn, int a, int b, int nk, int nn,
                       unsigned long long anti) {
  if (nk < 1 || nn < 1) return hipSuccess;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  g.M = b; g.N = b; g.K = a * b;
  g.A = Pm; g.sAm = 1; g.sAk = b;
  g.B = Qm; g.sBk = b; g.sBn = 1;
  g.C = C; g.sCm = b; g.sCn = 1;
  batch2(g, nk, nn, pk, pn, qk, qn, ck, cn);
  return run(P.M, P_F64, g, P.s, OC_CLOSE_R);
}
// C_L(P,Q)[l,l'] = sum_{a,r} P[a;l,r] Q[a;l',r] over (k, node)
hipError_t pos_close_l(Pos& P, const double* Pm, long long pk, long long pn, const double* Qm, long long qk,
                       long long qn, double* C, long long ck, long long cn, int a, int b, int nk, int nn,
                       unsigned long long anti) {
  if (nk < 1 || nn < 1) return hipSuccess;
  const long long bb = (long long)b * b;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  g.M = b; g.N = b; g.K = a * b; g.K2 = b;
  g.A = Pm; g.sAm = b; g.sAk = 1; g.sAk1 = bb;
  g.B = Qm; g.sBk = 1; g.sBk1 = bb; g.sBn = b;
  g.C = C; g.sCm = b; g.sCn = 1;
  batch2(g, nk, nn, pk, pn, qk, qn, ck, cn);
  return run(P.M, P_F64, g, P.s, OC_CLOSE_L);
}

// S w = h_L .l w + h_R .r w + sum_k A_{L,k} .l (B_{R,k} .r w) for nodes
// m0, m0 + st, .. (nn of them) of level t, into Sw (node stride sws); S2
// (node stride sws, k stride cube) holds the D right applications.
ttn_status pos_s_apply(Pos& P, int t, long long m0, int st, int nn, double* Sw, double* S2, long long sws) {
  const int a = P.dims[t], b = P.dims[t - 1], D = P.D;
  const long long bb = (long long)b * b, cube = P.cube(t), so = P.ops_stride(t - 1);
  const double* w = P.W[t] + m0 * cube;
  const double* opL = P.OPS[t - 1] + 2 * m0 * so;  // left child of node m0
  const double* opR = opL + so;                    // right child (level 0: the same block)
  const long long cs = 2LL * st * so;              // children of consecutive nodes
  HIPCHK(pos_apply_l(P, opL, cs, w, st * cube, Sw, sws, a, b, 0.0, nn));
  HIPCHK(pos_apply_r(P, opR, 0, cs, w, 0, st * cube, Sw, 0, sws, a, b, 1.0, 1, nn));
  if (D == 0) return TTN_OK;
  HIPCHK(pos_apply_r(P, opR + (1 + D) * bb, bb, cs, w, 0, st * cube, S2, cube, sws, a, b, 0.0, D, nn));
  HIPCHK(pos_apply_l_sum(P, opL + bb, bb, cs, S2, cube, sws, Sw, sws, a, b, 1.0, D, nn));
  return TTN_OK;
}

// Operators of nodes m0, m0 + st, .. of level t from their children.
ttn_status pos_ascend_nodes(Pos& P, int t, long long m0, int st, long long count) {
  const int a = P.dims[t], b = P.dims[t - 1], D = P.D;
  const long long bb = (long long)b * b, aa = (long long)a * a, cube = P.cube(t);
  const long long so = P.ops_stride(t - 1), sp = P.ops_stride(t);
  const long long sws = (1 + (long long)D) * cube;
  for (long long j0 = 0; j0 < count; j0 += P.chunk[t]) {
    const int nn = (int)std::min<long long>(P.chunk[t], count - j0);
    const long long m = m0 + j0 * st;
    double* Sw = P.stage;
    double* S2 = P.stage + cube;
    ttn_status r = pos_s_apply(P, t, m, st, nn, Sw, S2, sws);
    if (r) return r;
    const double* w = P.W[t] + m * cube;
    const double* opL = P.OPS[t - 1] + 2 * m * so;
    const double* opR = opL + so;
    const long long cs = 2LL * st * so;
    double* out = P.OPS[t] + m * sp;
    HIPCHK(pos_close(P, w, 0, st * cube, Sw, 0, sws, out, 0, st * sp, a, b, 1, nn, 0));  // h
    if (D == 0) continue;
    // A'_k = C(w, A_{R,k} .r w)
    HIPCHK(pos_apply_r(P, opR + bb, bb, cs, w, 0, st * cube, S2, cube, sws, a, b, 0.0, D, nn));
    HIPCHK(pos_close(P, w, 0, st * cube, S2, cube, sws, out + aa, aa, st * sp, a, b, D, nn, P.M.anti_bits()));
    // B'_k = C(w, B_{L,k} .l w)
    for (int k = 0; k < D; ++k)
      HIPCHK(pos_apply_l(P, opL + (1 + D + k) * bb, cs, w, st * cube, S2 + k * cube, sws, a, b, 0.0, nn));
    HIPCHK(pos_close(P, w, 0, st * cube, S2, cube, sws, out + (1 + D) * aa, aa, st * sp, a, b, D, nn,
                     P.M.anti_bits()));
  }
  return TTN_OK;
}

ttn_status pos_ascend_all(Pos& P, int from) {
  for (int t = from; t < P.n; ++t) {
    ttn_status r = pos_ascend_nodes(P, t, 0, 1, P.nodes(t));
    if (r) return r;
  }
  return TTN_OK;
}

// rho at the top (v v^T, v^T v) and at every level below, with the cache
// PC[t] = rho^(t, m) o w^(t, m).
ttn_status pos_descend_rho(Pos& P) {
  const int n = P.n, x = P.dims[n - 1];
  const long long sdt = P.dx_stride(n - 1);
  HIPCHK(mm(P.M, P_F64, P.M.vtop, false, P.M.vtop, true, P.DX[n - 1], x, 1.0, 0.0, P.s));
  HIPCHK(mm(P.M, P_F64, P.M.vtop, true, P.M.vtop, false, P.DX[n - 1] + sdt, x, 1.0, 0.0, P.s));
  for (int t = n - 1; t >= 1; --t) {
    const int a = P.dims[t], b = P.dims[t - 1];
    const long long cube = P.cube(t), sd = P.dx_stride(t), sdc = P.dx_stride(t - 1);
    const int nn = (int)P.nodes(t);
    HIPCHK(pos_left_mul(P, P.DX[t], 0, sd, P.W[t], 0, cube, P.PC[t], 0, cube, a, b, 1, nn));
    HIPCHK(pos_close_l(P, P.W[t], 0, cube, P.PC[t], 0, cube, P.DX[t - 1], 0, 2 * sdc, a, b, 1, nn, 0));
    HIPCHK(pos_close_r(P, P.W[t], 0, cube, P.PC[t], 0, cube, P.DX[t - 1] + sdc, 0, 2 * sdc, a, b, 1, nn, 0));
  }
  return TTN_OK;
}

// X and Y at the top and at every level down to `lowest` (rho and PC current).
ttn_status pos_descend_xy(Pos& P, int lowest) {
  const int n = P.n, D = P.D, x = P.dims[n - 1];
  if (D == 0) return TTN_OK;
  const long long xx = (long long)x * x, sot = P.ops_stride(n - 1), sdt = P.dx_stride(n - 1);
  const double* v = P.M.vtop;
  const double* op0 = P.OPS[n - 1];
  const double* op1 = op0 + sot;
  double* dx0 = P.DX[n - 1];
  double* dx1 = dx0 + sdt;
  double* T = P.stage;
  const unsigned long long anti = P.M.anti_bits();
  // X^(0) = v A^(1) v^T, X^(1) = v^T A^(0) v, Y^(0) = v B^(1) v^T, Y^(1) = v^T B^(0) v
  HIPCHK(mm_k(P.M, P_F64, op1 + xx, xx, false, v, 0, true, T, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, v, 0, false, T, xx, false, dx0 + xx, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, op0 + xx, xx, false, v, 0, false, T, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, v, 0, true, T, xx, false, dx1 + xx, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, op1 + (1 + D) * xx, xx, false, v, 0, true, T, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, v, 0, false, T, xx, false, dx0 + (1 + D) * xx, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, op0 + (1 + D) * xx, xx, false, v, 0, false, T, xx, x, 1.0, 0.0, D, P.s));
  HIPCHK(mm_k(P.M, P_F64, v, 0, true, T, xx, false, dx1 + (1 + D) * xx, xx, x, 1.0, 0.0, D, P.s));
  for (int t = n - 1; t > lowest; --t) {
    const int a = P.dims[t], b = P.dims[t - 1];
    const long long bb = (long long)b * b, aa = (long long)a * a, cube = P.cube(t);
    const long long sd = P.dx_stride(t), sdc = P.dx_stride(t - 1), soc = P.ops_stride(t - 1);
    const long long ts = (long long)D * cube;  // staging per parent
    for (long long m0 = 0; m0 < P.nodes(t); m0 += P.chunk[t]) {
      const int nn = (int)std::min<long long>(P.chunk[t], P.nodes(t) - m0);
      const double* w = P.W[t] + m0 * cube;
      const double* pc = P.PC[t] + m0 * cube;
      const double* dx = P.DX[t] + m0 * sd;
      double* lo_l = P.DX[t - 1] + 2 * m0 * sdc;  // left child of parent m0
      double* lo_r = lo_l + sdc;
      const double* opl = P.OPS[t - 1] + 2 * m0 * soc;
      const double* opr = opl + soc;
      // outer edges from the parent's: X_L = C_L(w, X o w), Y_R = C_R(w, Y o w)
      HIPCHK(pos_left_mul(P, dx + aa, aa, sd, w, 0, cube, T, cube, ts, a, b, D, nn));
      HIPCHK(pos_close_l(P, w, 0, cube, T, cube, ts, lo_l + bb, bb, 2 * sdc, a, b, D, nn, anti));
      HIPCHK(pos_left_mul(P, dx + (1 + D) * aa, aa, sd, w, 0, cube, T, cube, ts, a, b, D, nn));
      HIPCHK(pos_close_r(P, w, 0, cube, T, cube, ts, lo_r + (1 + D) * bb, bb, 2 * sdc, a, b, D, nn, anti));
      // inner edges meet inside the parent: X_R = C_R(w, A_{L,k} .l (rho o w)),
      // Y_L = C_L(w, B_{R,k} .r (rho o w))
      for (int k = 0; k < D; ++k)
        HIPCHK(pos_apply_l(P, opl + (1 + k) * bb, 2 * soc, pc, cube, T + k * cube, ts, a, b, 0.0, nn));
      HIPCHK(pos_close_r(P, w, 0, cube, T, cube, ts, lo_r + bb, bb, 2 * sdc, a, b, D, nn, anti));
      HIPCHK(pos_apply_r(P, opr + (1 + D) * bb, bb, 2 * soc, pc, 0, cube, T, cube, ts, a, b, 0.0, D, nn));
      HIPCHK(pos_close_l(P, w, 0, cube, T, cube, ts, lo_l + (1 + D) * bb, bb, 2 * sdc, a, b, D, nn, anti));
    }
  }
  return TTN_OK;
}

// Environments of nodes m0, m0 + 2, .. (nn of them) of level t into the env
// areas of polar slabs slab0, slab0 + 1, ..
ttn_status pos_env_chunk(Pos& P, int t, long long m0, int nn, const SlabLayout& S, int slab0) {
  const int a = P.dims[t], b = P.dims[t - 1], D = P.D;
  const long long bb = (long long)b * b, aa = (long long)a * a, cube = P.cube(t);
  const long long so = P.ops_stride(t - 1), sd = P.dx_stride(t);
  const long long es = (1 + 3LL * D) * cube;  // staging per node: E (1 + 2D slices), then S2 (D)
  double* E = P.stage;
  double* S2 = P.stage + (1 + 2LL * D) * cube;
  ttn_status r = pos_s_apply(P, t, m0, 2, nn, E, S2, es);
  if (r) return r;
  const double* w = P.W[t] + m0 * cube;
  const double* opL = P.OPS[t - 1] + 2 * m0 * so;
  const double* opR = opL + so;
  const long long cs = 4 * so;
  for (int k = 0; k < D; ++k)
    HIPCHK(pos_apply_l(P, opL + (1 + D + k) * bb, cs, w, 2 * cube, E + (1 + k) * cube, es, a, b, 0.0, nn));
  HIPCHK(pos_apply_r(P, opR + bb, bb, cs, w, 0, 2 * cube, E + (1 + D) * cube, cube, es, a, b, 0.0, D, nn));
  GemmDesc g = desc0();  // Env = [rho | X | Y] . E, contraction over (slice, a')
  g.M = a; g.N = (int)bb; g.K = (1 + 2 * D) * a; g.K2 = a;
  g.A = P.DX[t] + m0 * sd; g.sAm = a; g.sAk = 1; g.sAk1 = aa; g.sAb = 2 * sd;
  g.B = E; g.sBk = bb; g.sBk1 = cube; g.sBn = 1; g.sBb = es;
  g.C = P.slabs + slab0 * S.size + S.env; g.sCm = bb; g.sCn = 1; g.sCb = S.size;
  g.batch = nn;
  HIPCHK(run(P.M, P_F64, g, P.s, OC_LEFT_MUL));
  return TTN_OK;
}

// w <- -polar(Env - eps ||Env|| w) for the nn nodes whose environments sit in
// the slabs (node m0 + 2j in slab j), written back to W[t].
ttn_status pos_polar_chunk(Pos& P, int t, long long m0, int nn, const SlabLayout& S) {
  const int a = P.dims[t], b = P.dims[t - 1];
  const long long K = (long long)b * b, aK = (long long)a * K, cube = P.cube(t);
  double* sl = P.slabs;
  HIPCHK(copy_strided_f64(sl + S.wold, S.size, P.W[t] + m0 * cube, 2 * cube, cube, nn, P.s));  // w_old
  Member Mn = P.M;  // the polar update's scratch: slab 0, the others S.size doubles apart
  Mn.flops_acc = Mn.traffic_acc = 0.0;
  Mn.Y = sl + S.Y;
  Mn.Y2 = sl + S.Y2;
  Mn.G = sl + S.G;
  Mn.V = sl + S.V;
  Mn.Q = sl + S.Q;
  Mn.Q2 = sl + S.Q2;
  Mn.nrm = sl + S.nrm;
  Mn.jinfo = (int*)(sl + S.jinfo);
  Mn.skip3 = (int*)(sl + S.skip3);
  Mn.scal = sl + S.scal;
  Mn.part = sl + S.part;
  Mn.splitk = sl + S.splitk;
  Mn.splitk_bytes = (size_t)(128LL * a * a * 8);
  Mn.solo = true;
  Mn.evd = false;
  // one work-group per node (up to POS_GROUP_JACOBI_MAX); a single node above
  // POLAR_ONE_WG_MAX takes the blocked solver with the handle's scratch, as
  // the uniform network does
  Mn.jscratch = (nn == 1 && a > POLAR_ONE_WG_MAX) ? P.M.jscratch : nullptr;
  {
    GroupScope grp_nodes(nn, S.size * 8);
    HIPCHK(zero_int(Mn.jinfo, 64, P.s));
    HIPCHK(fill_f64(Mn.scal, 0.0, SCAL_N, P.s));
    double* env = sl + S.env;
    HIPCHK(pair_f64(env, env, aK, Mn.scal + SCAL_TMP0, Mn.part, P.s));
    HIPCHK(sqrt_inplace(Mn.scal + SCAL_TMP0, P.s));
    HIPCHK(copy_bytes(Mn.Y2, env, (size_t)aK * 8, P.s));
    HIPCHK(axpy_dev(Mn.Y2, sl + S.wold, Mn.scal + SCAL_TMP0, -POS_REG, (size_t)aK, P.s));
    // the environment's area is free once Y2 holds it: scratch of the null-row
    // fill, then the output
    ttn_status r = polar_core(Mn, Mn.Y2, a, K, -1.0, env, P.s, nullptr, false, nullptr, sl + S.wold, env);
    if (r) return r;
  }
  P.M.flops_acc += Mn.flops_acc;
  P.M.traffic_acc += Mn.traffic_acc;
  HIPCHK(flags_or(sl + S.scal, S.size, nn, SCAL_ERR, SCAL_NOCONV, P.flags, P.s));
  HIPCHK(copy_strided_f64(P.W[t] + m0 * cube, 2 * cube, sl + S.env, S.size, cube, nn, P.s));
  return TTN_OK;
}

// Environments of one parity group, then its updates (or, with `host`, the
// environments copied to the host instead: nodes p, p + 2, .. in order).
ttn_status pos_group(Pos& P, int t, int p, double* host) {
  const int a = P.dims[t], b = P.dims[t - 1];
  const SlabLayout S = slab_layout(a, b);
  const long long count = P.nodes(t) / 2, cube = P.cube(t);
  // a polar launch group of pchunk nodes; their environments in staging
  // chunks of at most chunk nodes, each written into its nodes' slabs
  for (long long j0 = 0; j0 < count; j0 += P.pchunk[t]) {
    const int nn = (int)std::min<long long>(P.pchunk[t], count - j0);
    const long long m0 = p + 2 * j0;
    for (int e0 = 0; e0 < nn; e0 += (int)P.chunk[t]) {
      const int ne = (int)std::min<long long>(P.chunk[t], nn - e0);
      ttn_status r = pos_env_chunk(P, t, m0 + 2LL * e0, ne, S, e0);
      if (r) return r;
    }
    if (host) {
      for (int j = 0; j < nn; ++j)
        HIPCHK(hipMemcpyAsync(host + (j0 + j) * cube, P.slabs + j * S.size + S.env, cube * 8, hipMemcpyDeviceToHost,
                              P.s));
      HIPCHK(hipStreamSynchronize(P.s));
      continue;
    }
    ttn_status r = pos_polar_chunk(P, t, m0, nn, S);
    if (r) return r;
  }
  return TTN_OK;
}

ttn_status pos_top(Pos& P) {
  const int n = P.n, D = P.D;
  const long long xx = P.x2(n - 1);
  Member& M = P.M;
  M.opH[n - 1] = P.OPS[n - 1];
  M.opA[n - 1] = P.OPS[n - 1] + xx;
  M.opB[n - 1] = P.OPS[n - 1] + (1 + D) * xx;
  M.topR = P.OPS[n - 1] + P.ops_stride(n - 1);
  M.hopR64 = P.topR;
  ttn_status r;
  if ((r = top_prepare(M, P.s))) return r;
  bool conv = false;
  if ((r = top_restarts(M, P.s, M.restarts, true, &conv))) return r;
  P.top_conv = conv;
  return top_finish(M, P.s);
}

ttn_status pos_sweep_body(Pos& P) {
  ttn_status r;
  if ((r = pos_descend_rho(P))) return r;
  for (int t = 1; t < P.n; ++t)
    for (int p = 0; p < 2; ++p) {
      if ((r = pos_descend_xy(P, t))) return r;
      if ((r = pos_group(P, t, p, nullptr))) return r;
      if ((r = pos_ascend_nodes(P, t, p, 2, P.nodes(t) / 2))) return r;
      for (int u = t + 1; u < P.n; ++u)
        if ((r = pos_ascend_nodes(P, u, 0, 1, P.nodes(u)))) return r;
    }
  return pos_top(P);
}

ttn_status pos_sweep(Pos& P) {
  P.M.counting = true;
  P.M.flops_acc = P.M.traffic_acc = 0.0;
  const ttn_status r = pos_sweep_body(P);
  P.M.counting = false;
  P.last_flops = P.M.flops_acc;
  P.last_bytes = P.M.traffic_acc;
  return r;
}

// workspace: the member's layout, then the per-node arrays
struct PosSizes {
  std::vector<long long> W, OPS, DX, PC, chunk, pchunk;
  long long stage = 0, slabs = 0, topR = 0;
};
PosSizes pos_sizes(const Member& M, int chunk_nodes) {
  PosSizes z;
  const int n = M.n, D = M.D;
  z.W.assign(n, 0); z.OPS.assign(n, 0); z.DX.assign(n, 0); z.PC.assign(n, 0);
  z.chunk.assign(n, 1); z.pchunk.assign(n, 1);
  const long long x_top = (long long)M.dims[n - 1] * M.dims[n - 1];
  z.stage = std::max<long long>(1, D) * x_top;
  for (int t = 0; t < n; ++t) {
    const long long nodes = (long long)M.L >> t, q = (long long)M.dims[t] * M.dims[t];
    z.OPS[t] = t == 0 ? (1 + 2LL * D) * q : nodes * (1 + 2LL * D) * q;
    z.DX[t] = nodes * (1 + 2LL * D) * q;
    if (t == 0) continue;
    const int a = M.dims[t], b = M.dims[t - 1];
    const long long cube = (long long)a * b * b;
    z.W[t] = nodes * cube;
    z.PC[t] = nodes * cube;
    const long long per = (1 + 3LL * D) * cube;
    long long ch = std::min<long long>(nodes, (long long)(POS_STAGE_BYTES / 8) / per);
    // a launch's batch (rows a or terms D, times nodes) stays below the
    // 65535 work-group limit of a grid dimension
    ch = std::min<long long>(ch, 32768 / std::max(a, std::max(D, 1)));
    if (chunk_nodes > 0) ch = std::min<long long>(ch, chunk_nodes);
    z.chunk[t] = std::max<long long>(1, ch);
    z.stage = std::max(z.stage, z.chunk[t] * per);
    const long long sl = slab_layout(a, b).size;
    long long pc = a > POS_GROUP_JACOBI_MAX ? 1
                                            : std::max<long long>(1, (long long)(POS_SLAB_BYTES / 8) / sl);
    pc = std::min<long long>(pc, std::max<long long>(1, nodes / 2));
    if (chunk_nodes > 0) pc = std::min<long long>(pc, chunk_nodes);
    z.pchunk[t] = pc;
    z.slabs = std::max(z.slabs, pc * sl);
  }
  z.topR = (1 + 2LL * D) * x_top;
  return z;
}

ttn_status pos_member(const ttn_pos_config* cfg, Member& M) {
  if (!cfg) return fail(TTN_EINVAL, "bad arguments");
  ttn_config c;
  std::memset(&c, 0, sizeof c);
  c.L = cfg->L; c.d = cfg->d; c.chi = cfg->chi; c.D = cfg->D;
  c.h1 = cfg->h1; c.A = cfg->A; c.B = cfg->B; c.shift = cfg->shift; c.ly = cfg->ly;
  c.precision = TTN_FP64; c.seed = cfg->seed; c.w0 = nullptr; c.v0 = cfg->v0;
  c.krylov = cfg->krylov; c.restarts = cfg->restarts; c.lanczos_tol = cfg->lanczos_tol;
  c.keep_gauge = 1; c.evd_update = 0;
  ttn_status st = setup_member(c, M);
  if (st) return st;
  if (!cfg->w0) return fail(TTN_EINVAL, "w0 (the isometries of every node) is required");
  if (cfg->chunk_nodes < 0) return fail(TTN_EINVAL, "chunk_nodes=%d < 0", cfg->chunk_nodes);
  for (int t = 1; t < M.n; ++t)
    if (!cfg->w0[t - 1]) return fail(TTN_EINVAL, "w0[%d] is NULL", t - 1);
  return TTN_OK;
}

size_t pos_layout(Member& M, int chunk_nodes, Arena& ar, Pos* P) {
  layout_member(M, ar);
  const PosSizes z = pos_sizes(M, chunk_nodes);
  const int n = M.n;
  std::vector<double*> W(n, nullptr), OPS(n, nullptr), DX(n, nullptr), PC(n, nullptr);
  for (int t = 0; t < n; ++t) {
    OPS[t] = ar.take<double>(z.OPS[t]);
    DX[t] = ar.take<double>(z.DX[t]);
    if (t >= 1) {
      W[t] = ar.take<double>(z.W[t]);
      PC[t] = ar.take<double>(z.PC[t]);
    }
  }
  double* stage = ar.take<double>(z.stage);
  double* slabs = ar.take<double>(std::max<long long>(z.slabs, 1));
  double* flags = ar.take<double>(2);
  double* topR = ar.take<double>(z.topR);
  if (P) {
    P->W = W; P->OPS = OPS; P->DX = DX; P->PC = PC;
    P->chunk = z.chunk; P->pchunk = z.pchunk;
    P->stage = stage; P->slabs = slabs; P->flags = flags; P->topR = topR;
  }
  return ar.off + 256;
}

ttn_status pos_check(ttn_pos_handle h) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  return TTN_OK;
}

ttn_status pos_status(Pos& P, bool warn_top) {
  double f[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(f, P.flags, sizeof f, hipMemcpyDeviceToHost, P.s));
  HIPCHK(hipStreamSynchronize(P.s));
  if (f[POS_ERR] != 0.0) return fail(TTN_EHIP, "a Jacobi eigensolver aborted (grid barrier wait exceeded its bound)");
  if (f[POS_NOCONV] != 0.0) return fail(TTN_ENOCONV, "a polar Jacobi solve stopped at its sweep limit");
  return warn_top && !P.top_conv ? TTN_WNOCONV : TTN_OK;
}

}  // namespace

extern "C" {

ttn_status ttn_pos_workspace_bytes(const ttn_pos_config* cfg, size_t* bytes) {
  if (!bytes) return fail(TTN_EINVAL, "bad arguments");
  Member M;
  ttn_status st = pos_member(cfg, M);
  if (st) return st;
  Arena ar;
  *bytes = pos_layout(M, cfg->chunk_nodes, ar, nullptr);
  return TTN_OK;
}

ttn_status ttn_pos_init(const ttn_pos_config* cfg, void* workspace, size_t bytes, void* stream, ttn_pos_handle* out) {
  if (!out) return fail(TTN_EINVAL, "bad arguments");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(TTN_EINVAL, "workspace must be non-null and 256-byte aligned");
  size_t need = 0;
  ttn_status st = ttn_pos_workspace_bytes(cfg, &need);
  if (st) return st;
  if (bytes < need) return fail(TTN_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, need);
  Pos* P = new Pos;
  P->s = (hipStream_t)stream;
  pos_member(cfg, P->M);
  P->M.prof = &P->prof;
  Arena ar;
  ar.base = (char*)workspace;
  pos_layout(P->M, cfg->chunk_nodes, ar, P);
  Member& M = P->M;
  P->L = M.L; P->n = M.n; P->d = M.d; P->D = M.D; P->dims = M.dims;
  const int n = M.n, d = M.d, D = M.D;
  const size_t dd = (size_t)d * d;
  auto bail = [&](ttn_status e) { delete P; return e; };
  // level-0 operators [h1 - c I, A_1..A_D, B_1..B_D]
  std::vector<double> op0((1 + 2 * (size_t)D) * dd);
  std::copy(M.h1.begin(), M.h1.end(), op0.begin());
  for (int i = 0; i < d; ++i) op0[i * d + i] -= M.c;
  if (D) {
    std::copy(M.A.begin(), M.A.end(), op0.begin() + dd);
    std::copy(M.B.begin(), M.B.end(), op0.begin() + (1 + D) * dd);
  }
  double init_scal[SCAL_N] = {0};
  init_scal[SCAL_RATIO_MIN] = 1.0;
  init_scal[SCAL_SHIFT] = M.c;
  const double zero2[2] = {0.0, 0.0};
  hipError_t e = hipMemcpyAsync(P->OPS[0], op0.data(), op0.size() * 8, hipMemcpyHostToDevice, P->s);
  if (!e) e = hipMemcpyAsync(M.scal, init_scal, sizeof init_scal, hipMemcpyHostToDevice, P->s);
  if (!e) e = hipMemcpyAsync(P->flags, zero2, sizeof zero2, hipMemcpyHostToDevice, P->s);
  for (int t = 1; t < n && !e; ++t)
    e = hipMemcpyAsync(P->W[t], cfg->w0[t - 1], (size_t)P->nodes(t) * P->cube(t) * 8, hipMemcpyHostToDevice, P->s);
  const size_t xx = (size_t)P->x2(n - 1);
  if (!e) {
    if (cfg->v0) e = hipMemcpyAsync(M.vtop, cfg->v0, xx * 8, hipMemcpyHostToDevice, P->s);
    else e = gaussian_f64(M.vtop, xx, M.seed ^ 0x5bd1e995ull, 0xfffffffull, P->s);
  }
  if (!e) e = zero_int(M.jinfo, 64, P->s);
  if (!e) e = hipStreamSynchronize(P->s);
  if (e) return bail(fail(TTN_EHIP, "initialisation: %s", hipGetErrorString(e)));
  if ((st = pos_ascend_all(*P, 1))) return bail(st);
  if ((st = pos_top(*P))) return bail(st);
  if ((st = pos_status(*P, true)) < 0) return bail(st);
  *out = P;
  return st;
}

ttn_status ttn_pos_free(ttn_pos_handle h) {
  if (!h) return TTN_OK;
  hipStreamSynchronize(h->s);
  delete h;
  return TTN_OK;
}

ttn_status ttn_pos_energy(ttn_pos_handle h, double* e) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (!e) return fail(TTN_EINVAL, "bad arguments");
  double sc[2];
  HIPCHK(hipMemcpyAsync(sc, h->M.scal + SCAL_LAM, sizeof sc, hipMemcpyDeviceToHost, h->s));
  HIPCHK(hipStreamSynchronize(h->s));
  e[0] = sc[0];
  e[1] = sc[1];
  return pos_status(*h, true);
}

ttn_status ttn_pos_sweep(ttn_pos_handle h, int nsweeps) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (nsweeps < 0) return fail(TTN_EINVAL, "nsweeps=%d < 0", nsweeps);
  for (int i = 0; i < nsweeps; ++i) {
    if ((st = pos_sweep(*h))) return st;
    if ((st = pos_status(*h, true)) < 0) return st;
  }
  return pos_status(*h, true);
}

ttn_status ttn_pos_descend(ttn_pos_handle h) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if ((st = pos_descend_rho(*h))) return st;
  if ((st = pos_descend_xy(*h, 0))) return st;
  HIPCHK(hipStreamSynchronize(h->s));
  return TTN_OK;
}

ttn_status ttn_pos_env(ttn_pos_handle h, int tau, int parity, double* host) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (tau < 1 || tau >= h->n || (parity != 0 && parity != 1) || !host)
    return fail(TTN_EINVAL, "tau=%d parity=%d: need 1 <= tau < %d, parity 0 or 1, non-null host", tau, parity, h->n);
  if ((st = pos_descend_rho(*h))) return st;
  if ((st = pos_descend_xy(*h, tau))) return st;
  return pos_group(*h, tau, parity, host);
}

ttn_status ttn_pos_get(ttn_pos_handle h, int what, int level, double* host) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (!host) return fail(TTN_EINVAL, "null host pointer");
  const double* src = nullptr;
  size_t count = 0;
  if (what == TTN_POS_TOP) {
    src = h->M.vtop;
    count = (size_t)h->x2(h->n - 1);
  } else {
    if (level < 0 || level >= h->n) return fail(TTN_EINVAL, "level=%d outside [0, %d)", level, h->n);
    if (what == TTN_POS_W) {
      if (level < 1) return fail(TTN_EINVAL, "isometries live on levels >= 1");
      src = h->W[level];
      count = (size_t)(h->nodes(level) * h->cube(level));
    } else if (what == TTN_POS_OPS) {
      src = h->OPS[level];
      count = level == 0 ? (size_t)(1 + 2 * h->D) * h->x2(0) : (size_t)(h->nodes(level) * h->ops_stride(level));
    } else if (what == TTN_POS_DX) {
      src = h->DX[level];
      count = (size_t)(h->nodes(level) * h->dx_stride(level));
    } else {
      return fail(TTN_EINVAL, "unknown kind %d", what);
    }
  }
  HIPCHK(hipMemcpyAsync(host, src, count * 8, hipMemcpyDeviceToHost, h->s));
  HIPCHK(hipStreamSynchronize(h->s));
  return TTN_OK;
}

ttn_status ttn_pos_stats(ttn_pos_handle h, ttn_pos_stats_t* out) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (!out) return fail(TTN_EINVAL, "null output");
  double sc[SCAL_N];
  HIPCHK(hipMemcpyAsync(sc, h->M.scal, sizeof sc, hipMemcpyDeviceToHost, h->s));
  HIPCHK(hipStreamSynchronize(h->s));
  std::memset(out, 0, sizeof *out);
  out->lam = sc[SCAL_LAM];
  out->energy = sc[SCAL_E];
  out->lanczos_resid = sc[SCAL_RES];
  out->flops_sweep = h->last_flops;
  out->bytes_sweep = h->last_bytes;
  out->n_levels = h->n;
  out->top_converged = h->top_conv ? 1 : 0;
  return TTN_OK;
}

ttn_status ttn_pos_profile(ttn_pos_handle h, int enable) {
  ttn_status st = pos_check(h);
  if (st) return st;
  return profile_switch(h->prof, h->krec, enable);
}

ttn_status ttn_pos_profile_read(ttn_pos_handle h, ttn_profile_entry* out, int max_entries, int* n_out) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (!out || !n_out) return fail(TTN_EINVAL, "bad arguments");
  return profile_collect(h->prof, h->s, out, max_entries, n_out);
}

ttn_status ttn_pos_set(ttn_pos_handle h, int what, int level, const double* host) {
  ttn_status st = pos_check(h);
  if (st) return st;
  if (!host) return fail(TTN_EINVAL, "null host pointer");
  if (what == TTN_POS_TOP) {
    HIPCHK(hipMemcpyAsync(h->M.vtop, host, (size_t)h->x2(h->n - 1) * 8, hipMemcpyHostToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    return TTN_OK;
  }
  if (what != TTN_POS_W) return fail(TTN_EINVAL, "only isometries and the top tensor can be set (kind %d)", what);
  if (level < 1 || level >= h->n) return fail(TTN_EINVAL, "level=%d outside [1, %d)", level, h->n);
  HIPCHK(hipMemcpyAsync(h->W[level], host, (size_t)(h->nodes(level) * h->cube(level)) * 8, hipMemcpyHostToDevice,
                        h->s));
  if ((st = pos_ascend_all(*h, level))) return st;
  HIPCHK(hipStreamSynchronize(h->s));
  return TTN_OK;
}

}  // extern "C"
