// C ABI of the binary-TTN sweep: handle, workspace layout, the stages of the
// sweep (ascend, descend, environment, update, top), and their schedule.
//
// The arithmetic of every stage runs in device kernels (gemm_*.hip,
// small.hip, lanczos.hip); this file only decides shapes, strides and order.
// Host-side arithmetic is limited to validating inputs and the one-off shift
// constant (largest eigenvalue of the d^2 x d^2 bond term).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ttn.h"
#include "common.h"
#include "gemm_internal.h"
#include "lanczos.h"
#include "ttn_core.h"

using namespace ttn;

namespace ttn {
namespace core {

thread_local std::string g_err;

ttn_status fail(ttn_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}


// ---------------------------------------------------------------------------
// host: largest eigenvalue of a small symmetric matrix (cyclic Jacobi)
// ---------------------------------------------------------------------------
double host_lambda_max(std::vector<double> a, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) (p == q ? diag : off) += a[p * n + q] * a[p * n + q];
    if (off <= 1e-32 * (diag + off) || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // rows p, q
          double xp = a[p * n + k], xq = a[q * n + k];
          a[p * n + k] = c * xp - s * xq;
          a[q * n + k] = s * xp + c * xq;
        }
        for (int k = 0; k < n; ++k) {  // columns p, q
          double xp = a[k * n + p], xq = a[k * n + q];
          a[k * n + p] = c * xp - s * xq;
          a[k * n + q] = s * xp + c * xq;
        }
      }
  }
  double mx = -INFINITY;
  for (int i = 0; i < n; ++i) mx = std::max(mx, a[i * n + i]);
  return mx;
}

// Largest eigenvalue of a larger symmetric matrix (n > 64, e.g. the bond
// term of a column of 4 to 6 spins): restarted Lanczos with full
// reorthogonalisation (two Gram-Schmidt passes) from a fixed start vector,
// the tridiagonal matrix diagonalised by host_lambda_max's Jacobi method
// through its eigenvectors, until the Ritz residual is below 1e-14 of the
// matrix scale; returns the Rayleigh quotient of the Ritz vector.
double host_lambda_max_lanczos(const std::vector<double>& a, int n) {
  auto matvec = [&](const std::vector<double>& x, std::vector<double>& y) {
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      const double* row = a.data() + (size_t)i * n;
      for (int k = 0; k < n; ++k) acc += row[k] * x[k];
      y[i] = acc;
    }
  };
  auto dot = [&](const std::vector<double>& x, const std::vector<double>& y) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += x[i] * y[i];
    return acc;
  };
  double scale = 0.0;
  for (double v : a) scale += v * v;
  scale = std::sqrt(scale);
  const int m = std::min(n, 96);
  std::vector<double> x(n), w(n), r(n);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.5 * std::sin(1.0 + i);  // fixed, generic start
  double theta = 0.0;
  for (int rs = 0; rs < 40; ++rs) {
    double nx = std::sqrt(dot(x, x));
    for (double& v : x) v /= nx;
    std::vector<std::vector<double>> Q{x};
    std::vector<double> al, be;
    for (int j = 0; j < m; ++j) {
      matvec(Q[j], w);
      for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i <= j; ++i) {
          const double c = dot(Q[i], w);
          if (pass == 0 && i == j) al.push_back(c);
          if (pass == 1 && i == j) al.back() += c;
          for (int k = 0; k < n; ++k) w[k] -= c * Q[i][k];
        }
      const double b = std::sqrt(dot(w, w));
      if (j + 1 == m || b <= 1e-14 * scale) break;
      be.push_back(b);
      for (double& v : w) v /= b;
      Q.push_back(w);
    }
    const int k = (int)al.size();
    // eigenpairs of the k x k tridiagonal matrix: Jacobi on a copy that also
    // carries the eigenvectors (rows of the identity rotated alongside)
    std::vector<double> T((size_t)k * k, 0.0), V((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
      T[(size_t)i * k + i] = al[i];
      V[(size_t)i * k + i] = 1.0;
      if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = be[i];
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0.0, diag = 0.0;
      for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) (p == q ? diag : off) += T[(size_t)p * k + q] * T[(size_t)p * k + q];
      if (off <= 1e-32 * (diag + off) || off == 0.0) break;
      for (int p = 0; p < k - 1; ++p)
        for (int q = p + 1; q < k; ++q) {
          const double apq = T[(size_t)p * k + q];
          if (apq == 0.0) continue;
          const double th = (T[(size_t)q * k + q] - T[(size_t)p * k + p]) / (2.0 * apq);
          const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
          const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
          for (int u = 0; u < k; ++u) {
            const double xp = T[(size_t)p * k + u], xq = T[(size_t)q * k + u];
            T[(size_t)p * k + u] = c * xp - s * xq;
            T[(size_t)q * k + u] = s * xp + c * xq;
          }
          for (int u = 0; u < k; ++u) {
            const double xp = T[(size_t)u * k + p], xq = T[(size_t)u * k + q];
            T[(size_t)u * k + p] = c * xp - s * xq;
            T[(size_t)u * k + q] = s * xp + c * xq;
          }
          for (int u = 0; u < k; ++u) {  // eigenvectors as rows of V
            const double xp = V[(size_t)p * k + u], xq = V[(size_t)q * k + u];
            V[(size_t)p * k + u] = c * xp - s * xq;
            V[(size_t)q * k + u] = s * xp + c * xq;
          }
        }
    }
    int best = 0;
    for (int i = 1; i < k; ++i)
      if (T[(size_t)i * k + i] > T[(size_t)best * k + best]) best = i;
    std::fill(x.begin(), x.end(), 0.0);
    for (int i = 0; i < k; ++i)
      for (int u = 0; u < n; ++u) x[u] += V[(size_t)best * k + i] * Q[i][u];
    nx = std::sqrt(dot(x, x));
    for (double& v : x) v /= nx;
    matvec(x, w);
    theta = dot(x, w);
    for (int u = 0; u < n; ++u) r[u] = w[u] - theta * x[u];
    if (std::sqrt(dot(r, r)) <= 1e-14 * std::max(1.0, scale)) break;
  }
  return theta;
}

// ---------------------------------------------------------------------------
// workspace arena
// ---------------------------------------------------------------------------
// Streams over which the members of a batch run side by side in the layer
// part of a sweep (forked from and joined back into the caller's stream with
// events, so the fork is captured into the sweep graph as well).
constexpr int POOL_STREAMS = 8;

struct Ctx {
  std::vector<Member> m;
  hipStream_t s = nullptr;
  Profiler prof;
  KernelRecorder krec;
  // captured layer part of a sweep (descend(RHO) and every layer step of
  // every member), replayed by ttn_sweep(.., use_graph = 1)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // captured layer part of a grouped sweep, one per grouping (1 or 2 groups)
  hipGraph_t ggraph[2] = {nullptr, nullptr};
  hipGraphExec_t ggexec[2] = {nullptr, nullptr};
  std::vector<hipStream_t> pool;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // launch groups: members of identical configuration (all but the
  // Hamiltonian's values) laid out side by side at a uniform stride run
  // every kernel of a stage as one launch; members[0] is the lowest address
  struct Group {
    std::vector<int> members;
    long long stride = 0;
  };
  std::vector<Group> groups;
  // the layer part of a sweep runs over coarser groups: members of one
  // configuration but different lengths L (their per-level shapes agree),
  // laid out longest first at a uniform stride (shorter members padded to the
  // longest's depth), advanced level by level in lockstep; the members still
  // at a level are a prefix of the group, those whose top is at a level a
  // contiguous range
  std::vector<Group> coarse;
  hipStream_t grid_s = nullptr;          // serialises the persistent Jacobi solves of a batch
  hipStream_t cap_s = nullptr;           // stream the sweep graph is captured on
  // graphs of the planned top update, by the number of restarts they hold,
  // and the plan: the restarts the slowest member has needed so far
  std::map<int, hipGraphExec_t> top_exec;
  int top_plan = 1;
  std::vector<hipEvent_t> member_events;  // two per member, for grid_s
  ~Ctx() {
    if (kernel_timer() == &krec) kernel_timer() = nullptr;
    if (gexec) hipGraphExecDestroy(gexec);
    for (auto& kv : top_exec) hipGraphExecDestroy(kv.second);
    if (graph) hipGraphDestroy(graph);
    for (int i = 0; i < 2; ++i) {
      if (ggexec[i]) hipGraphExecDestroy(ggexec[i]);
      if (ggraph[i]) hipGraphDestroy(ggraph[i]);
    }
    for (auto e : join) hipEventDestroy(e);
    if (fork) hipEventDestroy(fork);
    for (auto e : member_events) hipEventDestroy(e);
    for (auto q : pool) hipStreamDestroy(q);
    if (grid_s) hipStreamDestroy(grid_s);
    if (cap_s) hipStreamDestroy(cap_s);
  }
};

// ---------------------------------------------------------------------------
// configuration
// ---------------------------------------------------------------------------
ttn_status setup_member(const ttn_config& c, Member& M) {
  if (c.L < 4 || (c.L & (c.L - 1))) return fail(TTN_EINVAL, "L=%d must be a power of two >= 4", c.L);
  if (c.d < 2 || c.d > 64) return fail(TTN_EINVAL, "d=%d out of range [2, 64]", c.d);
  if (c.chi < 1 || c.chi > 1024) return fail(TTN_EINVAL, "chi=%d out of range [1, 1024]", c.chi);
  if (c.D < 0 || c.D > 64) return fail(TTN_EINVAL, "D=%d out of range [0, 64]", c.D);
  if (!c.h1 || (c.D > 0 && (!c.A || !c.B))) return fail(TTN_EINVAL, "missing Hamiltonian arrays");
  if (c.ly < 1) return fail(TTN_EINVAL, "ly=%d must be >= 1", c.ly);
  if (c.precision < TTN_FP64 || c.precision > TTN_SPLIT_BF16) return fail(TTN_EINVAL, "unknown precision %d", c.precision);
  M.L = c.L;
  M.n = 0;
  while ((1 << M.n) < c.L) ++M.n;
  M.d = c.d;
  M.D = c.D;
  M.chi = c.chi;
  M.ly = c.ly;
  M.prec = c.precision;
  M.seed = c.seed;
  M.w0 = c.w0;
  M.v0 = c.v0;
  M.krylov = c.krylov > 0 ? c.krylov : 24;
  M.restarts = c.restarts > 0 ? c.restarts : 8;
  M.ltol = c.lanczos_tol > 0 ? c.lanczos_tol : 1e-12;
  M.gauge_fix = (c.keep_gauge == 0);
  if (c.evd_update != 0 && c.evd_update != 1) return fail(TTN_EINVAL, "evd_update=%d is neither 0 nor 1", c.evd_update);
  M.evd = (c.evd_update == 1);
  if (M.krylov > 63) return fail(TTN_EINVAL, "krylov=%d > 63", M.krylov);
  const int d = c.d, D = c.D;
  M.h1.assign(c.h1, c.h1 + d * d);
  M.A.assign(D ? c.A : nullptr, D ? c.A + (size_t)D * d * d : nullptr);
  M.B.assign(D ? c.B : nullptr, D ? c.B + (size_t)D * d * d : nullptr);
  for (double x : M.h1) if (!std::isfinite(x)) return fail(TTN_ENONFINITE, "h1 has a non-finite entry");
  for (double x : M.A) if (!std::isfinite(x)) return fail(TTN_ENONFINITE, "A has a non-finite entry");
  for (double x : M.B) if (!std::isfinite(x)) return fail(TTN_ENONFINITE, "B has a non-finite entry");
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(M.h1[i * d + j] - M.h1[j * d + i]) > 1e-12 * (1 + std::fabs(M.h1[i * d + j])))
        return fail(TTN_EINVAL, "h1 is not symmetric");
  for (int k = 0; k < D; ++k) {
    const double* a = &M.A[(size_t)k * d * d];
    const double* b = &M.B[(size_t)k * d * d];
    bool a_sym = true, a_anti = true, b_sym = true, b_anti = true;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double tol = 1e-12 * (1 + std::fabs(a[i * d + j]));
        if (std::fabs(a[i * d + j] - a[j * d + i]) > tol) a_sym = false;
        if (std::fabs(a[i * d + j] + a[j * d + i]) > tol) a_anti = false;
        double tolb = 1e-12 * (1 + std::fabs(b[i * d + j]));
        if (std::fabs(b[i * d + j] - b[j * d + i]) > tolb) b_sym = false;
        if (std::fabs(b[i * d + j] + b[j * d + i]) > tolb) b_anti = false;
      }
    if (!((a_sym && b_sym) || (a_anti && b_anti)))
      return fail(TTN_EINVAL, "product term %d: A and B must be both symmetric or both antisymmetric", k);
    M.anti.push_back(a_sym ? 0 : 1);
  }
  M.dims.resize(M.n);
  M.dims[0] = d;
  for (int t = 1; t < M.n; ++t) M.dims[t] = (int)std::min<long long>((long long)M.dims[t - 1] * M.dims[t - 1], c.chi);
  if (std::isnan(c.shift)) {
    // bond term 1/2 (h1 x I + I x h1) + sum_k A_k x B_k
    int dd = d * d;
    std::vector<double> b((size_t)dd * dd, 0.0);
    for (int i1 = 0; i1 < d; ++i1)
      for (int i2 = 0; i2 < d; ++i2)
        for (int j1 = 0; j1 < d; ++j1)
          for (int j2 = 0; j2 < d; ++j2) {
            double v = 0.0;
            if (i2 == j2) v += 0.5 * M.h1[i1 * d + j1];
            if (i1 == j1) v += 0.5 * M.h1[i2 * d + j2];
            for (int k = 0; k < D; ++k) v += M.A[(size_t)k * d * d + i1 * d + j1] * M.B[(size_t)k * d * d + i2 * d + j2];
            b[(size_t)(i1 * d + i2) * dd + (j1 * d + j2)] = v;
          }
    M.c = dd <= 64 ? host_lambda_max(b, dd) : host_lambda_max_lanczos(b, dd);
  } else {
    if (!std::isfinite(c.shift)) return fail(TTN_ENONFINITE, "shift is not finite");
    M.c = c.shift;
  }
  M.esz = (M.prec == TTN_FP64) ? 8 : 4;
  if (c.w0) {
    for (int t = 1; t < M.n; ++t)
      if (!c.w0[t - 1]) return fail(TTN_EINVAL, "w0[%d] is NULL", t - 1);
  }
  return TTN_OK;
}

void layout_member(Member& M, Arena& ar, int n_pad) {
  // n_pad > n: the per-level arrays of levels n .. n_pad - 1 are laid out too
  // (unused), so that members of one bond dimension and different lengths
  // share one layout and sit at a uniform stride
  const int n = std::max(M.n, n_pad), D = M.D;
  std::vector<int> dims = M.dims;
  while ((int)dims.size() < n) dims.push_back((int)std::min<long long>((long long)dims.back() * dims.back(), M.chi));
  int cmax = 0;
  size_t cube = 0;  // largest a*b*b
  for (int t = 0; t < n; ++t) cmax = std::max(cmax, dims[t]);
  for (int t = 1; t < n; ++t) cube = std::max(cube, (size_t)dims[t] * dims[t - 1] * dims[t - 1]);
  cube = std::max(cube, (size_t)(1 + 2 * D) * M.d * M.d);  // staging of the level-0 operators
  const int x = M.dims[M.n - 1];
  const size_t xx = (size_t)x * x;
  M.w64.assign(n, nullptr);
  M.wT.assign(n, nullptr);
  M.Qw.assign(n, nullptr);
  M.qw_valid.assign(n, 0);
  for (int t = 1; t < n; ++t) {
    size_t e = (size_t)dims[t] * dims[t - 1] * dims[t - 1];
    M.w64[t] = ar.take<double>(e);
    M.Qw[t] = ar.take<double>((size_t)dims[t] * dims[t]);
    M.wT[t] = (M.prec == TTN_FP64) ? (void*)M.w64[t] : ar.take_bytes(M.el(e));
  }
  M.opH.assign(n, nullptr);
  M.opA.assign(n, nullptr);
  M.opB.assign(n, nullptr);
  M.rho.assign(n, nullptr);
  M.Pc.assign(n, nullptr);
  M.At.assign(n, nullptr);
  M.Bt.assign(n, nullptr);
  for (int t = 0; t < n; ++t) {
    size_t q = (size_t)dims[t] * dims[t];
    M.opH[t] = ar.take_bytes(M.el(q));
    M.opA[t] = ar.take_bytes(M.el(q * std::max(D, 1)));
    M.opB[t] = ar.take_bytes(M.el(q * std::max(D, 1)));
    M.rho[t] = ar.take_bytes(M.el(q));
    M.At[t] = ar.take_bytes(M.el(q * std::max(D, 1)));
    M.Bt[t] = ar.take_bytes(M.el(q * std::max(D, 1)));
    if (t >= 2) M.Pc[t] = ar.take_bytes(M.el((size_t)dims[t] * dims[t - 1] * dims[t - 1]));
  }
  size_t cq = (size_t)cmax * cmax * std::max(D, 1);
  for (int i = 0; i < 2; ++i) {
    M.Rb[i] = ar.take_bytes(M.el(cq));
    M.Lb[i] = ar.take_bytes(M.el(cq));
  }
  // environment staging [S w | B_k .l w | A_k .r w], slice 0 doubles as S w;
  // S2, S3 hold one intermediate per product term
  const size_t nkk = (size_t)std::max(D, 1);
  M.Estage = ar.take_bytes(M.el((1 + 2 * (size_t)D) * cube));
  M.Sw = M.Estage;
  M.S2 = ar.take_bytes(M.el(nkk * cube));
  M.S3 = ar.take_bytes(M.el(nkk * cube));
  M.Xst = ar.take_bytes(M.el((1 + 2 * (size_t)D) * (size_t)cmax * cmax));
  M.envT = (M.prec == TTN_FP64) ? nullptr : ar.take_bytes(M.el(cube));
  M.env64 = ar.take<double>(cube);
  M.Y = ar.take<double>(cube);
  M.Y2 = ar.take<double>(cube);
  if (M.prec == TTN_FP64) M.envT = M.env64;
  size_t c2 = (size_t)cmax * cmax;
  M.G = ar.take<double>(c2);
  M.V = ar.take<double>(c2);
  M.Q = ar.take<double>(c2);
  M.Q2 = ar.take<double>(c2);
  M.nrm = ar.take<double>(cmax);
  M.jinfo = ar.take<int>(64);
  M.skip3 = ar.take<int>(64);
  M.jscratch = ar.take_bytes(jacobi_blocked_scratch_bytes(std::max(cmax, M.krylov)));
  M.vtop = ar.take<double>(xx);
  M.vT = (M.prec == TTN_FP64) ? (void*)M.vtop : ar.take_bytes(M.el(xx));
  M.tmpT = ar.take_bytes(M.el(xx * std::max(D, 1)));
  // float64 top operators, contiguous [h, A_1..A_D, B_1..B_D], and the
  // matvec staging [y, y B_1^T .. y B_D^T, y A_1^T .. y A_D^T]
  M.hop64 = ar.take<double>(xx * (1 + 2 * D));
  M.Aop64 = M.hop64 + xx;
  M.Bop64 = M.hop64 + (1 + D) * xx;
  M.lzStage = ar.take<double>(xx * (1 + 2 * D));
  int m = std::min<long long>(M.krylov, (long long)xx);
  M.lzQ = ar.take<double>((size_t)(m + 1) * xx);
  M.lzW = ar.take<double>(xx);
  M.lzT = ar.take<double>(xx);
  M.lzHv = ar.take<double>(xx);
  M.lzR = ar.take<double>(xx);
  M.alpha = ar.take<double>(m + 1);
  M.beta = ar.take<double>(m + 1);
  M.Tm = ar.take<double>((size_t)m * m);
  M.Vm = ar.take<double>((size_t)m * m);
  M.ycoef = ar.take<double>(m + 1);
  M.coef = ar.take<double>(2 * (m + 2));
  M.lzpart = ar.take<double>(lz_reorth_part_doubles());
  M.lznrm = ar.take<double>(lz_norm_doubles());
  M.lzint = ar.take<int>(16);
  M.scal = ar.take<double>(SCAL_N);
  M.part = ar.take<double>(256);
  // split-K partial sums: up to 64 slices of the largest output tile set
  size_t out_max = std::max<size_t>(c2, xx);
  M.splitk_bytes = 64 * out_max * 8;
  M.splitk = ar.take_bytes(M.splitk_bytes);
}

// ---------------------------------------------------------------------------
// contraction helpers (element strides; bulk arithmetic of the member)
// ---------------------------------------------------------------------------
CplxCtx& cplx() {
  static thread_local CplxCtx c;
  return c;
}

hipError_t run_real(const Member& M, Prec p, const GemmDesc& g, hipStream_t s, int cls);

hipError_t run(const Member& M, Prec p, const GemmDesc& g, hipStream_t s, int cls) {
  const CplxCtx cx = cplx();
  if (cx.delta == 0) return run_real(M, p, g, s, cls);
  // complex: four real products over the planes.  A result asked on its
  // triangle is Hermitian or anti-Hermitian when the caller allows it
  // (tri_ok): the real plane then has the parity of the anti bits and the
  // imaginary plane the opposite one, and each plane's two products run on
  // the triangle (the second accumulates into the first's upper triangle)
  const double sa = cx.conj_a ? -1.0 : 1.0;
  auto im = [&](const void* q) { return (const void*)((const char*)q + cx.delta); };
  const bool tri = g.tri != 0 && cx.tri_ok;
  GemmDesc q = g;
  q.tri = tri ? 1 : 0;
  q.anti = tri ? g.anti : 0;
  hipError_t e;
  if ((e = run_real(M, p, q, s, cls))) return e;  // Re C = alpha Re A Re B + beta Re C
  q.A = im(g.A); q.B = im(g.B); q.alpha = -sa * g.alpha; q.beta = 1.0;
  if ((e = run_real(M, p, q, s, cls))) return e;  //      - alpha (+-Im A) Im B
  q.anti = tri ? ~g.anti : 0;
  q.A = g.A; q.B = im(g.B); q.C = (void*)im(g.C); q.alpha = g.alpha; q.beta = g.beta;
  if ((e = run_real(M, p, q, s, cls))) return e;  // Im C = alpha Re A Im B + beta Im C
  q.A = im(g.A); q.B = g.B; q.alpha = sa * g.alpha; q.beta = 1.0;
  return run_real(M, p, q, s, cls);               //      + alpha (+-Im A) Re B
}

hipError_t run_real(const Member& M, Prec p, const GemmDesc& g, hipStream_t s, int cls) {
  size_t slot = 0;
  bool timed = false;
  GemmDesc gg = g;
  gg.mcount = grp().count;
  gg.mstride = grp().stride;
  if (!gg.skip) gg.skip = grp().skip;
  if (M.counting) {
    const double per = (p == P_F64 ? 8.0 : 4.0) * g.batch *
                       ((double)g.M * g.K + (double)g.K * g.N + (g.beta != 0.0 ? 2.0 : 1.0) * g.M * (double)g.N);
    const double members = gg.mcount > 1 ? gg.mcount : 1;
    M.bytes_acc += per;
    M.traffic_acc += per * members;
    M.flops_acc += 2.0 * g.M * (double)g.N * g.K * g.batch * members;
  }
  if (M.prof && M.prof->on) {
    double es = (p == P_F64) ? 8.0 : 4.0;
    double f = 2.0 * g.M * (double)g.N * g.K * g.batch * gg.mcount;
    double b = es * g.batch * gg.mcount *
               ((double)g.M * g.K + (double)g.K * g.N + (g.beta != 0.0 ? 2.0 : 1.0) * g.M * (double)g.N);
    timed = M.prof->begin(cls, f, b, s, &slot);
  }
  hipError_t e = gemm(p, gg, M.splitk, M.splitk_bytes, s);
  if (timed) M.prof->end(slot, s);
  return e;
}

// a copy of an array, and of its imaginary plane inside a CplxScope
hipError_t copy_planes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  hipError_t e = copy_bytes(dst, src, bytes, s);
  const long long d = cplx().delta;
  if (e || d == 0) return e;
  return copy_bytes((char*)dst + d, (const char*)src + d, bytes, s);
}

GemmDesc desc0() {
  GemmDesc g;
  std::memset(&g, 0, sizeof g);
  g.batch = 1;
  g.alpha = 1.0;
  g.beta = 0.0;
  return g;
}

// The building blocks over nk product terms at once: term k reads its
// operator at O + k sO, its tensor at X + k sX (sX = 0: one tensor for all)
// and writes Y + k sY; one launch for all terms.
// (O .r X)[a;l,r] = sum_r' O[r,r'] X[a;l,r']
hipError_t apply_r_k(const Member& M, Prec p, const void* O, long long sO, const void* X, long long sX, void* Y,
                     long long sY, int a, int b, double beta, int nk, hipStream_t s) {
  if (nk < 1) return hipSuccess;
  GemmDesc g = desc0();
  g.batch = nk;
  g.M = a * b; g.N = b; g.K = b; g.K2 = 0;
  g.A = X; g.sAm = b; g.sAk = 1; g.sAb = sX;
  g.B = O; g.sBk = 1; g.sBn = b; g.sBb = sO;
  g.C = Y; g.sCm = b; g.sCn = 1; g.sCb = sY;
  g.beta = beta;
  return run(M, p, g, s, OC_APPLY_R);
}
// (O .l X)[a;l,r] = sum_l' O[l,l'] X[a;l',r]   (batched over a, then over k)
hipError_t apply_l_k(const Member& M, Prec p, const void* O, long long sO, const void* X, long long sX, void* Y,
                     long long sY, int a, int b, double beta, int nk, hipStream_t s) {
  if (nk < 1) return hipSuccess;
  GemmDesc g = desc0();
  const long long bb = (long long)b * b;
  g.batch1 = a;
  g.batch = a * nk;
  g.M = b; g.N = b; g.K = b; g.K2 = 0;
  g.A = O; g.sAm = b; g.sAk = 1; g.sAb = 0; g.sAb2 = sO;
  g.B = X; g.sBk = b; g.sBn = 1; g.sBb = bb; g.sBb2 = sX;
  g.C = Y; g.sCm = b; g.sCn = 1; g.sCb = bb; g.sCb2 = sY;
  g.beta = beta;
  return run(M, p, g, s, OC_APPLY_L);
}
// C(P,Q)[a,a'] = sum_{l,r} P[a;l,r] Q[a';l,r]   (a x a, K = b*b).  Every
// use has Q = O w with P = w and O symmetric, or antisymmetric for the terms
// whose bit is set in anti, so C is symmetric (antisymmetric) and a float64
// launch computes its upper triangle only.  In the three closes P is the bra
// copy of a contraction (conjugated when the products are complex).
hipError_t close_aa_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                      long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                      unsigned long long anti) {
  if (nk < 1) return hipSuccess;
  BraScope bra;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  long long bb = (long long)b * b;
  g.batch = nk;
  g.M = a; g.N = a; g.K = (int)bb; g.K2 = 0;
  g.A = P; g.sAm = bb; g.sAk = 1; g.sAb = sP;
  g.B = Qm; g.sBk = 1; g.sBn = bb; g.sBb = sQ;
  g.C = C; g.sCm = a; g.sCn = 1; g.sCb = sC;
  g.alpha = alpha; g.beta = beta;
  return run(M, p, g, s, OC_CLOSE);
}
// (X o P)[a;l,r] = sum_a' X[a,a'] P[a';l,r]
hipError_t left_mul_k(const Member& M, Prec p, const void* X, long long sX, const void* P, long long sP, void* Y,
                      long long sY, int a, int b, double alpha, double beta, int nk, hipStream_t s) {
  if (nk < 1) return hipSuccess;
  GemmDesc g = desc0();
  long long bb = (long long)b * b;
  g.batch = nk;
  g.M = a; g.N = (int)bb; g.K = a; g.K2 = 0;
  g.A = X; g.sAm = a; g.sAk = 1; g.sAb = sX;
  g.B = P; g.sBk = bb; g.sBn = 1; g.sBb = sP;
  g.C = Y; g.sCm = bb; g.sCn = 1; g.sCb = sY;
  g.alpha = alpha; g.beta = beta;
  return run(M, p, g, s, OC_LEFT_MUL);
}
// C_R(P,Q)[r,r'] = sum_{a,l} P[a;l,r] Q[a;l,r']   (b x b, K = a*b).  Both
// child closes only ever produce symmetric matrices (density matrices:
// P = w, Q = rho o w, or Q = w and P = rho o w, with rho symmetric) or, in the
// dressed chains, matrices of their product term's parity (bit k of anti set:
// antisymmetric), so a float64 launch computes the block upper triangle and
// mirrors it; a beta != 0 accumulation reads the upper triangle of a C of the
// same parity.
hipError_t close_r_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                     long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                     unsigned long long anti) {
  if (nk < 1) return hipSuccess;
  BraScope bra;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  g.batch = nk;
  g.M = b; g.N = b; g.K = a * b; g.K2 = 0;
  g.A = P; g.sAm = 1; g.sAk = b; g.sAb = sP;
  g.B = Qm; g.sBk = b; g.sBn = 1; g.sBb = sQ;
  g.C = C; g.sCm = b; g.sCn = 1; g.sCb = sC;
  g.alpha = alpha; g.beta = beta;
  return run(M, p, g, s, OC_CLOSE_R);
}
// C_L(P,Q)[l,l'] = sum_{a,r} P[a;l,r] Q[a;l',r]   (b x b, K = (a, r))
hipError_t close_l_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                     long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                     unsigned long long anti) {
  if (nk < 1) return hipSuccess;
  BraScope bra;
  GemmDesc g = desc0();
  g.tri = 1;
  g.anti = anti;
  long long bb = (long long)b * b;
  g.batch = nk;
  g.M = b; g.N = b; g.K = a * b; g.K2 = b;
  g.A = P; g.sAm = b; g.sAk = 1; g.sAk1 = bb; g.sAb = sP;
  g.B = Qm; g.sBk = 1; g.sBk1 = bb; g.sBn = b; g.sBb = sQ;
  g.C = C; g.sCm = b; g.sCn = 1; g.sCb = sC;
  g.alpha = alpha; g.beta = beta;
  return run(M, p, g, s, OC_CLOSE_L);
}
hipError_t apply_r(const Member& M, Prec p, const void* O, const void* X, void* Y, int a, int b, double beta,
                   hipStream_t s) {
  return apply_r_k(M, p, O, 0, X, 0, Y, 0, a, b, beta, 1, s);
}
hipError_t apply_l(const Member& M, Prec p, const void* O, const void* X, void* Y, int a, int b, double beta,
                   hipStream_t s) {
  return apply_l_k(M, p, O, 0, X, 0, Y, 0, a, b, beta, 1, s);
}
hipError_t close_aa(const Member& M, Prec p, const void* P, const void* Qm, void* C, int a, int b, double alpha,
                    double beta, hipStream_t s, bool anti) {
  return close_aa_k(M, p, P, 0, Qm, 0, C, 0, a, b, alpha, beta, 1, s, anti ? 1ull : 0ull);
}
hipError_t left_mul(const Member& M, Prec p, const void* X, const void* P, void* Y, int a, int b, double alpha,
                    double beta, hipStream_t s) {
  return left_mul_k(M, p, X, 0, P, 0, Y, 0, a, b, alpha, beta, 1, s);
}
hipError_t close_r(const Member& M, Prec p, const void* P, const void* Qm, void* C, int a, int b, double alpha,
                   double beta, hipStream_t s) {
  return close_r_k(M, p, P, 0, Qm, 0, C, 0, a, b, alpha, beta, 1, s, 0);
}
hipError_t close_l(const Member& M, Prec p, const void* P, const void* Qm, void* C, int a, int b, double alpha,
                   double beta, hipStream_t s) {
  return close_l_k(M, p, P, 0, Qm, 0, C, 0, a, b, alpha, beta, 1, s, 0);
}
// dense square products of order x: C = alpha op(A) op(B) + beta C, for nk
// triples (A + k sA, B + k sB, C + k sC) in one launch
hipError_t mm_k(const Member& M, Prec p, const void* Am, long long sA, bool ta, const void* Bm, long long sB, bool tb,
                void* C, long long sC, int x, double alpha, double beta, int nk, hipStream_t s) {
  if (nk < 1) return hipSuccess;
  GemmDesc g = desc0();
  g.batch = nk;
  g.M = x; g.N = x; g.K = x; g.K2 = 0;
  g.A = Am; g.sAm = ta ? 1 : x; g.sAk = ta ? x : 1; g.sAb = sA;
  g.B = Bm; g.sBk = tb ? 1 : x; g.sBn = tb ? x : 1; g.sBb = sB;
  g.C = C; g.sCm = x; g.sCn = 1; g.sCb = sC;
  g.alpha = alpha; g.beta = beta;
  return run(M, p, g, s, OC_TOP_MM);
}
hipError_t mm(const Member& M, Prec p, const void* Am, bool ta, const void* Bm, bool tb, void* C, int x, double alpha,
              double beta, hipStream_t s) {
  return mm_k(M, p, Am, 0, ta, Bm, 0, tb, C, 0, x, alpha, beta, 1, s);
}

// S w = h .l w + h .r w + sum_k A_k .l (B_k .r w)   (into M.Sw, slice 0 of
// the environment staging).  The D right applications are one launch into
// S2 ([k][a][l][r]); the D left applications and their sum are one product
// whose contraction index runs over (k, l').
hipError_t s_apply(const Member& M, int lvl_below, const void* w, int a, int b, hipStream_t s) {
  Prec p = M.gp();
  const long long bb = (long long)b * b, cube = (long long)a * bb;
  hipError_t e;
  if ((e = apply_l(M, p, M.opH[lvl_below], w, M.Sw, a, b, 0.0, s))) return e;
  if ((e = apply_r(M, p, M.opH[lvl_below], w, M.Sw, a, b, 1.0, s))) return e;
  if (M.D == 0) return hipSuccess;
  if ((e = apply_r_k(M, p, M.opB[lvl_below], bb, w, 0, M.S2, cube, a, b, 0.0, M.D, s))) return e;
  GemmDesc g = desc0();  // Sw[a; l, r] += sum_{k, l'} A_k[l, l'] S2_k[a; l', r]
  g.batch = a;
  g.M = b; g.N = b; g.K = M.D * b; g.K2 = b;
  g.A = M.opA[lvl_below]; g.sAm = b; g.sAk = 1; g.sAk1 = bb; g.sAb = 0;
  g.B = M.S2; g.sBk = b; g.sBk1 = cube; g.sBn = 1; g.sBb = bb;
  g.C = M.Sw; g.sCm = b; g.sCn = 1; g.sCb = bb;
  g.beta = 1.0;
  return run(M, p, g, s, OC_APPLY_L);
}

// ---------------------------------------------------------------------------
// position-resolved density matrices and local energies (float64, from the
// master isometries and top tensor; the sweep's state is not touched)
// ---------------------------------------------------------------------------
// The caller's work buffer in doubles, every region on a 256-byte boundary:
// site and bond energies (L each), h1, the product operators of two adjacent
// levels ([A_1..A_D], [B_1..B_D], twice), the bond operator of every layer,
// the matrices of every level (level tau: L >> tau nodes of chi_tau^2), and
// scratch for the rest (at least two a*b*b slices; more lets more parents
// share one launch of the descent, up to 256 MB of them).
struct PosLayout {
  long long site = 0, bond = 0, h1 = 0, ops = 0, slot = 0, scratch = 0, scratch_min = 0, min_total = 0;
  std::vector<long long> bop, rho;
};
PosLayout pos_layout(const Member& M) {
  PosLayout P;
  const int n = M.n;
  long long o = 0, cmax = 0;
  for (int t = 0; t < n; ++t) cmax = std::max<long long>(cmax, M.dims[t]);
  auto take = [&](long long k) {
    long long r = o;
    o = (o + k + 31) & ~31LL;
    return r;
  };
  P.site = take(M.L);
  P.bond = take(M.L);
  P.h1 = take((long long)M.d * M.d);
  P.slot = (long long)std::max(M.D, 1) * cmax * cmax;
  P.ops = take(4 * P.slot);
  P.bop.assign(n, 0);
  for (int t = 1; t < n; ++t) P.bop[t] = take((long long)M.dims[t] * M.dims[t]);
  P.rho.assign(n, 0);
  for (int t = 0; t < n; ++t) P.rho[t] = take((long long)(M.L >> t) * M.dims[t] * M.dims[t]);
  long long sc = 2LL * M.dims[n - 1] * M.dims[n - 1];
  for (int t = 1; t < n; ++t) sc = std::max(sc, 2LL * M.dims[t] * M.dims[t - 1] * M.dims[t - 1]);
  P.scratch = o;
  P.scratch_min = sc;
  P.min_total = o + sc;
  return P;
}

// Bottom-up: the operators that A on the last and B on the first site of a
// block of each level become, and each layer's bond operator
// w (A x B) w^T summed over k.  Top: the two bonds between the halves of v.
// Top-down: the matrix of every node, node 2m (2m+1) of level tau-1 the left
// (right) child of node m of level tau, in batches of parents; each level's
// bonds pair its nodes with its layer's bond operator, level 0 its sites with
// h1.
ttn_status local_energies(Member& M, double* W, long long total, const PosLayout& P, hipStream_t s) {
  const int n = M.n, d = M.d, D = M.D, x = M.dims[n - 1];
  const long long L = M.L, dd = (long long)d * d, xx = (long long)x * x;
  double* S = W + P.scratch;
  const long long sc_len = total - P.scratch;
  double* site = W + P.site;
  double* bond = W + P.bond;
  HIPCHK(hipMemcpyAsync(W + P.h1, M.h1.data(), dd * 8, hipMemcpyHostToDevice, s));
  double* opA[2] = {W + P.ops, W + P.ops + 2 * P.slot};
  double* opB[2] = {W + P.ops + P.slot, W + P.ops + 3 * P.slot};
  int cur = 0;
  if (D) {
    HIPCHK(hipMemcpyAsync(opA[0], M.A.data(), D * dd * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(opB[0], M.B.data(), D * dd * 8, hipMemcpyHostToDevice, s));
    for (int t = 1; t < n; ++t) {
      const int a = M.dims[t], b = M.dims[t - 1];
      const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
      const double* w = M.w64[t];
      double* T1 = S;
      double* T2 = S + cube;
      for (int k = 0; k < D; ++k) {
        HIPCHK(apply_r(M, P_F64, opB[cur] + k * bb, w, T1, a, b, 0.0, s));
        HIPCHK(apply_l(M, P_F64, opA[cur] + k * bb, T1, T2, a, b, k ? 1.0 : 0.0, s));
      }
      HIPCHK(close_aa(M, P_F64, w, T2, W + P.bop[t], a, b, 1.0, 0.0, s, false));
      for (int k = 0; k < D; ++k) {
        HIPCHK(apply_r(M, P_F64, opA[cur] + k * bb, w, T1, a, b, 0.0, s));
        HIPCHK(close_aa(M, P_F64, w, T1, opA[cur ^ 1] + k * aa, a, b, 1.0, 0.0, s, M.anti[k] != 0));
        HIPCHK(apply_l(M, P_F64, opB[cur] + k * bb, w, T1, a, b, 0.0, s));
        HIPCHK(close_aa(M, P_F64, w, T1, opB[cur ^ 1] + k * aa, a, b, 1.0, 0.0, s, M.anti[k] != 0));
      }
      cur ^= 1;
    }
    double* X = S;
    double* Y = S + xx;
    for (int k = 0; k < D; ++k) {  // middle bond <v, A v B^T>, periodic bond <v, B v A^T>
      HIPCHK(mm(M, P_F64, opA[cur] + k * xx, false, M.vtop, false, X, x, 1.0, 0.0, s));
      HIPCHK(mm(M, P_F64, X, false, opB[cur] + k * xx, true, Y, x, 1.0, 0.0, s));
      HIPCHK(pair_rows_f64(M.vtop, 0, Y, 0, xx, 1, bond, 0, L / 2 - 1, k ? 1.0 : 0.0, s));
      HIPCHK(mm(M, P_F64, opB[cur] + k * xx, false, M.vtop, false, X, x, 1.0, 0.0, s));
      HIPCHK(mm(M, P_F64, X, false, opA[cur] + k * xx, true, Y, x, 1.0, 0.0, s));
      HIPCHK(pair_rows_f64(M.vtop, 0, Y, 0, xx, 1, bond, 0, L - 1, k ? 1.0 : 0.0, s));
    }
  } else {
    HIPCHK(fill_f64(bond, 0.0, (size_t)L, s));
  }
  double* rt = W + P.rho[n - 1];
  HIPCHK(mm(M, P_F64, M.vtop, false, M.vtop, true, rt, x, 1.0, 0.0, s));       // v v^T
  HIPCHK(mm(M, P_F64, M.vtop, true, M.vtop, false, rt + xx, x, 1.0, 0.0, s));  // v^T v
  for (int t = n - 1; t >= 1; --t) {
    const int a = M.dims[t], b = M.dims[t - 1];
    const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
    const long long parents = L >> t;
    double* up = W + P.rho[t];
    double* lo = W + P.rho[t - 1];
    const double* w = M.w64[t];
    if (D) HIPCHK(pair_rows_f64(up, aa, W + P.bop[t], 0, aa, (int)parents, bond, 1LL << t, (1LL << (t - 1)) - 1, 0.0, s));
    // parents per launch: their slabs rho o w (8 a b^2 bytes each) up to
    // 256 MB, the size of the last-level cache (at chi = 256, two parents:
    // measured faster than one, three or more)
    const long long slab_cap = std::max<long long>(1, (256LL << 20) / 8 / cube);
    const long long chunk = std::max<long long>(1, std::min<long long>({parents, sc_len / cube, slab_cap}));
    for (long long m0 = 0; m0 < parents; m0 += chunk) {
      const int c = (int)std::min<long long>(chunk, parents - m0);
      HIPCHK(left_mul_k(M, P_F64, up + m0 * aa, aa, w, 0, S, cube, a, b, 1.0, 0.0, c, s));
      HIPCHK(close_l_k(M, P_F64, w, 0, S, cube, lo + 2 * m0 * bb, 2 * bb, a, b, 1.0, 0.0, c, s, 0));
      HIPCHK(close_r_k(M, P_F64, w, 0, S, cube, lo + (2 * m0 + 1) * bb, 2 * bb, a, b, 1.0, 0.0, c, s, 0));
    }
  }
  HIPCHK(pair_rows_f64(W + P.rho[0], dd, W + P.h1, 0, dd, (int)L, site, 1, 0, 0.0, s));
  return TTN_OK;
}

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
ttn_status stage_ascend(Member& M, int tau, hipStream_t s) {
  Prec p = M.gp();
  const int a = M.dims[tau], b = M.dims[tau - 1], D = M.D;
  const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
  const void* w = M.wT[tau];
  HIPCHK(s_apply(M, tau - 1, w, a, b, s));
  HIPCHK(close_aa(M, p, w, M.Sw, M.opH[tau], a, b, 1.0, 0.0, s, false));
  // all product terms at once: A'_k = C(w, A_k .r w), B'_k = C(w, B_k .l w)
  HIPCHK(apply_r_k(M, p, M.opA[tau - 1], bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
  HIPCHK(close_aa_k(M, p, w, 0, M.S2, cube, M.opA[tau], aa, a, b, 1.0, 0.0, D, s, M.anti_bits()));
  HIPCHK(apply_l_k(M, p, M.opB[tau - 1], bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
  HIPCHK(close_aa_k(M, p, w, 0, M.S2, cube, M.opB[tau], aa, a, b, 1.0, 0.0, D, s, M.anti_bits()));
  return TTN_OK;
}

ttn_status stage_descend_rho(Member& M, hipStream_t s) {
  Prec p = M.gp();
  const int n = M.n, x = M.dims[n - 1];
  // rho^(n-1) = 1/2 (v v^T + v^T v) (the first factor is the bra copy)
  {
    BraScope bra;
    HIPCHK(mm(M, p, M.vT, false, M.vT, true, M.rho[n - 1], x, 0.5, 0.0, s));
    HIPCHK(mm(M, p, M.vT, true, M.vT, false, M.rho[n - 1], x, 0.5, 1.0, s));
  }
  for (int lv = n - 1; lv >= 2; --lv) {
    const int a = M.dims[lv], b = M.dims[lv - 1];
    HIPCHK(left_mul(M, p, M.rho[lv], M.wT[lv], M.Pc[lv], a, b, 1.0, 0.0, s));
    HIPCHK(close_l(M, p, M.wT[lv], M.Pc[lv], M.rho[lv - 1], a, b, 0.5, 0.0, s));
    HIPCHK(close_r(M, p, M.wT[lv], M.Pc[lv], M.rho[lv - 1], a, b, 0.5, 1.0, s));
  }
  M.rho_from = 1;
  M.pc_from = 2;
  return TTN_OK;
}

// Two-site information at the top from the carried operators At, Bt of level
// n-1: Rbar = 1/2 (v^T A v + v A v^T), Lbar = 1/2 (v B v^T + v^T B v), into
// slot rb_cur of the double buffer (set by the caller).
ttn_status dressed_top(Member& M, const void* At, const void* Bt, hipStream_t s) {
  Prec p = M.gp();
  const int n = M.n, D = M.D;
  const int x = M.dims[n - 1];
  const long long xx = (long long)x * x;
  void* R = M.Rb[M.rb_cur];
  void* Lq = M.Lb[M.rb_cur];
  // the left factor v (v^T) of each second product is the bra copy
  HIPCHK(mm_k(M, p, At, xx, false, M.vT, 0, false, M.tmpT, xx, x, 1.0, 0.0, D, s));  // A v
  {
    BraScope bra;
    HIPCHK(mm_k(M, p, M.vT, 0, true, M.tmpT, xx, false, R, xx, x, 0.5, 0.0, D, s));  // v^T A v
  }
  HIPCHK(mm_k(M, p, At, xx, false, M.vT, 0, true, M.tmpT, xx, x, 1.0, 0.0, D, s));   // A v^T
  {
    BraScope bra;
    HIPCHK(mm_k(M, p, M.vT, 0, false, M.tmpT, xx, false, R, xx, x, 0.5, 1.0, D, s));  // v A v^T
  }
  HIPCHK(mm_k(M, p, Bt, xx, false, M.vT, 0, true, M.tmpT, xx, x, 1.0, 0.0, D, s));   // B v^T
  {
    BraScope bra;
    HIPCHK(mm_k(M, p, M.vT, 0, false, M.tmpT, xx, false, Lq, xx, x, 0.5, 0.0, D, s));  // v B v^T
  }
  HIPCHK(mm_k(M, p, Bt, xx, false, M.vT, 0, false, M.tmpT, xx, x, 1.0, 0.0, D, s));  // B v
  {
    BraScope bra;
    HIPCHK(mm_k(M, p, M.vT, 0, true, M.tmpT, xx, false, Lq, xx, x, 0.5, 1.0, D, s));  // v^T B v
  }
  return TTN_OK;
}

// Rbar, Lbar one level down through layer sg (level sg -> sg-1), all k at
// once; Alow, Blow are the carried operators of level sg-1.  Needs the cached
// P = rho^(sg) o w_sg.
ttn_status dressed_down(Member& M, int sg, const void* Alow, const void* Blow, hipStream_t s) {
  Prec p = M.gp();
  const int D = M.D;
  const int a = M.dims[sg], b = M.dims[sg - 1];
  const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
  const void* w = M.wT[sg];
  const void* P = M.Pc[sg];
  const int cur = M.rb_cur, nx = 1 - cur;
  void* Rn = M.Rb[nx];
  void* Ln = M.Lb[nx];
  // inside a parent (A left child, B right child) + across parents
  HIPCHK(apply_l_k(M, p, Alow, bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
  HIPCHK(close_r_k(M, p, P, 0, M.S2, cube, Rn, bb, a, b, 0.5, 0.0, D, s, M.anti_bits()));
  HIPCHK(left_mul_k(M, p, M.Rb[cur], aa, w, 0, M.S3, cube, a, b, 1.0, 0.0, D, s));
  HIPCHK(close_l_k(M, p, w, 0, M.S3, cube, Rn, bb, a, b, 0.5, 1.0, D, s, M.anti_bits()));
  HIPCHK(apply_r_k(M, p, Blow, bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
  HIPCHK(close_l_k(M, p, P, 0, M.S2, cube, Ln, bb, a, b, 0.5, 0.0, D, s, M.anti_bits()));
  HIPCHK(left_mul_k(M, p, M.Lb[cur], aa, w, 0, M.S3, cube, a, b, 1.0, 0.0, D, s));
  HIPCHK(close_r_k(M, p, w, 0, M.S3, cube, Ln, bb, a, b, 0.5, 1.0, D, s, M.anti_bits()));
  M.rb_cur = nx;
  return TTN_OK;
}

ttn_status stage_descend_dressed(Member& M, int tau, hipStream_t s) {
  Prec p = M.gp();
  const int n = M.n, D = M.D;
  // carry A_k, B_k of level tau-1 up through layers tau..n-1 (all k at once)
  const void* prevA = M.opA[tau - 1];
  const void* prevB = M.opB[tau - 1];
  for (int sg = tau; sg < n; ++sg) {
    const int a = M.dims[sg], b = M.dims[sg - 1];
    const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
    const void* w = M.wT[sg];
    HIPCHK(apply_r_k(M, p, prevA, bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
    HIPCHK(close_aa_k(M, p, w, 0, M.S2, cube, M.At[sg], aa, a, b, 1.0, 0.0, D, s, M.anti_bits()));
    HIPCHK(apply_l_k(M, p, prevB, bb, w, 0, M.S2, cube, a, b, 0.0, D, s));
    HIPCHK(close_aa_k(M, p, w, 0, M.S2, cube, M.Bt[sg], aa, a, b, 1.0, 0.0, D, s, M.anti_bits()));
    prevA = M.At[sg];
    prevB = M.Bt[sg];
  }
  ttn_status st;
  M.rb_cur = 0;
  if ((st = dressed_top(M, M.At[n - 1], M.Bt[n - 1], s))) return st;
  // descend through layers n-1 .. tau+1
  for (int sg = n - 1; sg >= tau + 1; --sg)
    if ((st = dressed_down(M, sg, M.At[sg - 1], M.Bt[sg - 1], s))) return st;
  M.dressed_tau = tau;
  return TTN_OK;
}

// Env = [rho | Rbar_1..Rbar_D | Lbar_1..Lbar_D] o [S w ; B_k .l w ; A_k .r w]:
// the 1 + 2D tensors are staged side by side (slice s at s a b^2) and their
// left factors copied next to each other, so that the environment is one
// product whose contraction index runs over (slice, a'); it is written once.
ttn_status stage_env(Member& M, int tau, hipStream_t s) {
  Prec p = M.gp();
  const int a = M.dims[tau], b = M.dims[tau - 1], D = M.D;
  const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
  const void* w = M.wT[tau];
  HIPCHK(s_apply(M, tau - 1, w, a, b, s));                                        // slice 0
  HIPCHK(apply_l_k(M, p, M.opB[tau - 1], bb, w, 0, M.at(M.Estage, cube), cube, a, b, 0.0, D, s));
  HIPCHK(apply_r_k(M, p, M.opA[tau - 1], bb, w, 0, M.at(M.Estage, (1 + D) * cube), cube, a, b, 0.0, D, s));
  HIPCHK(copy_planes(M.Xst, M.rho[tau], M.el(aa), s));
  if (D > 0) {
    HIPCHK(copy_planes(M.at(M.Xst, aa), M.Rb[M.rb_cur], M.el(D * aa), s));
    HIPCHK(copy_planes(M.at(M.Xst, (1 + D) * aa), M.Lb[M.rb_cur], M.el(D * aa), s));
  }
  GemmDesc g = desc0();
  g.M = a; g.N = (int)bb; g.K = (1 + 2 * D) * a; g.K2 = a;
  g.A = M.Xst; g.sAm = a; g.sAk = 1; g.sAk1 = aa;
  g.B = M.Estage; g.sBk = bb; g.sBk1 = cube; g.sBn = 1;
  g.C = M.envT; g.sCm = bb; g.sCn = 1;
  HIPCHK(run(M, p, g, s, OC_LEFT_MUL));
  if (M.prec != TTN_FP64) HIPCHK(convert_f32_to_f64((const float*)M.envT, M.env64, (size_t)cube, s));
  M.env_tau = tau;
  return TTN_OK;
}

// The eigenproblem of the polar update's Gram matrix (M.G -> eigenvalues on
// its diagonal, eigenvectors as the rows of M.V).  The solver depends on the
// order a alone, so a member of a batch does the arithmetic it does alone:
// a <= POLAR_ONE_WG_MAX one work-group per matrix (the cyclic solver with G
// and its eigenvectors in LDS, or for the orders that fill whole blocks the
// blocked method with G in LDS; all members of a launch group in one
// launch), larger a the blocked solver with its persistent grid.  In a batch
// a blocked grid solve of a <= 128 (at most 30 work-groups) runs on the
// member's own stream, one launch per member of its launch group; larger ones (up to 128
// work-groups) go one at a time through the batch's shared stream, so the
// persistent grids that can run at once stay well below what the compute
// units hold.
hipError_t polar_jacobi(Member& M, int a, double jtol, int it, const int* skip, hipStream_t s) {
  int* info = M.jinfo + 2 * it;
  if (a <= POLAR_ONE_WG_MAX) return jacobi_eig_f64(M.G, M.V, a, POLAR_JACOBI_SWEEPS, jtol, info, nullptr, s, skip);
  if (M.solo) return jacobi_eig_f64(M.G, M.V, a, POLAR_JACOBI_SWEEPS, jtol, info, M.jscratch, s, skip);
  if (a <= 128) {
    const GroupCtx g = grp();
    GroupScope one(1, 0);
    for (int m = 0; m < g.count; ++m) {
      const long long off = (long long)m * g.stride;
      auto sh = [off](auto* p) { return p ? (decltype(p))((char*)p + off) : p; };
      hipError_t e = jacobi_eig_f64(sh(M.G), sh(M.V), a, POLAR_JACOBI_SWEEPS, jtol, sh(info), sh(M.jscratch), s,
                                    skip ? (const int*)((const char*)skip + off) : nullptr);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e;
  if ((e = hipEventRecord(M.grid_in, s))) return e;
  if ((e = hipStreamWaitEvent(M.grid_s, M.grid_in, 0))) return e;
  if ((e = jacobi_eig_f64(M.G, M.V, a, POLAR_JACOBI_SWEEPS, jtol, info, M.jscratch, M.grid_s, skip))) return e;
  if ((e = hipEventRecord(M.grid_out, M.grid_s))) return e;
  return hipStreamWaitEvent(s, M.grid_out, 0);
}

// out = sign * polar(src) for src (a x K), float64: Gram -> Jacobi eigenvectors
// -> rotate, repeated; rows of the rotated matrix end up mutually orthogonal
// with relative accuracy, then normalised and rotated back.
// With `warm` (a rotation kept from the previous update of this layer) the
// first Gram is taken of warm^T src, which is nearly diagonal once the sweep
// settles, so the Jacobi sweeps of the first refresh drop; the result is the
// same polar factor.  The final rotation is written back to `warm`.
// With `fill_from` (the current isometry, a x K) and `fill_tmp` (a x K
// scratch), rows of the first refresh's rotated matrix that are numerically
// null (norm below 4 eps sqrt(a) times the largest: rounding noise of the
// rotation, where the environment is rank deficient and the polar factor is
// not fixed) are replaced by the same rotation of the current isometry's
// rows at that scale, so that the
// completion leans toward the current isometry and the refreshes after it
// orthogonalise well-separated rows instead of rounding noise.  Nothing
// changes when no row is null (a device flag skips the fill).
ttn_status polar_core(Member& M, const double* src, int a, long long K, double sign, double* out, hipStream_t s,
                      double* warm, bool warm_valid, double** p_out, const double* fill_from, double* fill_tmp) {
  // Invariant: Y = P src with P orthogonal (P = Q^T, rows are the current
  // left singular vector estimates).  Each refresh diagonalises G = Y Y^T =
  // U^T diag U (Jacobi; rows of U are eigenvectors) and sets Y <- U Y,
  // P <- U P.  At the end the rows of Y are orthogonal to working accuracy,
  // Y = diag(nrm) Z, and polar(src) = P^T Z.
  const size_t aK = (size_t)a * K;
  double* Yc = M.Y;
  double* Yn = M.Y2;
  double* Pc = M.Q;
  double* Pn = M.Q2;
  const bool use_warm = warm && warm_valid;
  if (use_warm) {
    GemmDesc r = desc0();  // Y = P_warm src
    r.M = a; r.N = (int)K; r.K = a;
    r.A = warm; r.sAm = a; r.sAk = 1;
    r.B = src; r.sBk = K; r.sBn = 1;
    r.C = Yc; r.sCm = K; r.sCn = 1;
    HIPCHK(run(M, P_F64, r, s));
    HIPCHK(copy_bytes(Pc, warm, (size_t)a * a * 8, s));
  } else {
    HIPCHK(copy_bytes(Yc, src, aK * 8, s));
  }
  const double jtol = std::max(1e-15, 2.2e-16 * a);
  // POLAR_REFRESH refreshes, then one more whose need is decided on the
  // device (the previous Jacobi needed more than POLAR_THIRD_IF sweeps): its
  // kernels read the flag M.skip3 and return at once when it is set, so the
  // whole update has no host synchronisation and can be captured in a graph.
  // The eigenvalue-decomposition variant stops after the first refresh:
  // then P = U, Y = U src and polar(src) = U^T diag(1/|y_i|) U src.
  const int nref = M.evd ? 1 : POLAR_REFRESH;
  for (int it = 0; it <= nref; ++it) {
    const bool extra = it == nref;
    if (extra && M.evd) break;
    const int* skip = extra ? M.skip3 : nullptr;
    GemmDesc g = desc0();  // G = Y Y^T (symmetric: upper triangle and mirror)
    g.M = a; g.N = a; g.K = (int)K;
    g.tri = 1;
    g.A = Yc; g.sAm = K; g.sAk = 1;
    g.B = Yc; g.sBk = 1; g.sBn = K;
    g.C = M.G; g.sCm = a; g.sCn = 1;
    g.skip = skip;
    HIPCHK(run(M, P_F64, g, s));
    {
      size_t slot = 0;
      bool timed = M.prof && M.prof->begin(OC_JACOBI, 0.0, 0.0, s, &slot);
      HIPCHK(polar_jacobi(M, a, jtol, it, skip, s));
      if (timed) M.prof->end(slot, s);
    }
    GemmDesc r = desc0();  // Yn = U Y
    r.M = a; r.N = (int)K; r.K = a;
    r.A = M.V; r.sAm = a; r.sAk = 1;
    r.B = Yc; r.sBk = K; r.sBn = 1;
    r.C = Yn; r.sCm = K; r.sCn = 1;
    r.skip = skip;
    HIPCHK(run(M, P_F64, r, s));
    if (it == 0 && !use_warm && !M.evd && fill_from && fill_tmp) {
      // a row of U src whose norm is within a few roundings of the largest's
      // eps sqrt(a) is rounding noise of the rotation
      const double rel = 4.0 * 2.220446049250313e-16 * std::sqrt((double)a);
      int* none = M.skip3 + 1;  // 1: no null row, the fill is skipped
      HIPCHK(no_null_rows(Yn, a, K, rel, M.nrm, none, s));
      GemmDesc t = desc0();  // T = U w_cur
      t.M = a; t.N = (int)K; t.K = a;
      t.A = M.V; t.sAm = a; t.sAk = 1;
      t.B = fill_from; t.sBk = K; t.sBn = 1;
      t.C = fill_tmp; t.sCm = K; t.sCn = 1;
      t.skip = none;
      HIPCHK(run(M, P_F64, t, s));
      HIPCHK(fill_null_rows(Yn, fill_tmp, M.nrm, a, K, rel, none, s));
    }
    if (it == 0 && !use_warm) {
      HIPCHK(copy_bytes(Pc, M.V, (size_t)a * a * 8, s));
    } else {
      GemmDesc q = desc0();  // Pn = U P
      q.M = a; q.N = a; q.K = a;
      q.A = M.V; q.sAm = a; q.sAk = 1;
      q.B = Pc; q.sBk = a; q.sBn = 1;
      q.C = Pn; q.sCm = a; q.sCn = 1;
      q.skip = skip;
      HIPCHK(run(M, P_F64, q, s, OC_TOP_MM));
      if (!extra) std::swap(Pc, Pn);
    }
    if (extra) {
      // the extra refresh wrote Yn, Pn; bring them back only if it ran
      HIPCHK(copy_bytes_if(Yc, Yn, aK * 8, M.skip3, 0, s));
      HIPCHK(copy_bytes_if(Pc, Pn, (size_t)a * a * 8, M.skip3, 0, s));
    } else {
      std::swap(Yc, Yn);
    }
    if (it == nref - 1 && !M.evd) HIPCHK(set_flag_le(M.skip3, M.jinfo + 2 * it, POLAR_THIRD_IF, s));
  }
  HIPCHK(note_negative_info(M.jinfo, M.evd ? 1 : POLAR_REFRESH + 1, M.scal + SCAL_ERR, M.scal + SCAL_NOCONV,
                            POLAR_JACOBI_SWEEPS, s));
  HIPCHK(row_normalize_f64(Yc, Yn, M.nrm, a, K, s));
  if (p_out) {
    // gauge-fixed result: out = sign * Z, the rotation P is handed back
    HIPCHK(axpby_f64(Yn, out, sign, 0.0, aK, s));
    *p_out = Pc;
    return TTN_OK;
  }
  GemmDesc f = desc0();  // out = sign * P^T Z
  f.M = a; f.N = (int)K; f.K = a;
  f.A = Pc; f.sAm = 1; f.sAk = a;
  f.B = Yn; f.sBk = K; f.sBn = 1;
  f.C = out; f.sCm = K; f.sCn = 1;
  f.alpha = sign;
  HIPCHK(run(M, P_F64, f, s));
  if (warm) HIPCHK(copy_bytes(warm, Pc, (size_t)a * a * 8, s));
  return TTN_OK;
}

ttn_status refresh_shadow(Member& M, int tau, hipStream_t s) {
  if (M.prec == TTN_FP64) return TTN_OK;
  size_t e = (size_t)M.dims[tau] * M.dims[tau - 1] * M.dims[tau - 1];
  HIPCHK(convert_f64_to_f32(M.w64[tau], (float*)M.wT[tau], e, s));
  return TTN_OK;
}

ttn_status ortho_check(Member& M, int tau, hipStream_t s) {
  const int a = M.dims[tau];
  const long long K = (long long)M.dims[tau - 1] * M.dims[tau - 1];
  GemmDesc g = desc0();
  g.M = a; g.N = a; g.K = (int)K;
  g.tri = 1;
  g.A = M.w64[tau]; g.sAm = K; g.sAk = 1;
  g.B = M.w64[tau]; g.sBk = 1; g.sBn = K;
  g.C = M.G; g.sCm = a; g.sCn = 1;
  HIPCHK(run(M, P_F64, g, s));
  HIPCHK(ortho_err_from_gram(M.G, a, M.scal + SCAL_ORTHO, s));
  HIPCHK(running_max(M.scal + SCAL_ORTHO, M.scal + SCAL_ORTHO_MAX, s));
  return TTN_OK;
}

ttn_status stage_update_layer(Member& M, int tau, hipStream_t s) {
  const int a = M.dims[tau], b = M.dims[tau - 1];
  const long long K = (long long)b * b;
  const size_t aK = (size_t)a * K;
  // Env' = Env - eps ||Env|| w_old: a tie-breaker in directions where Env is
  // numerically zero; invisible elsewhere at float64 resolution.
  HIPCHK(pair_f64(M.env64, M.env64, (long long)aK, M.scal + SCAL_TMP0, M.part, s));
  HIPCHK(sqrt_inplace(M.scal + SCAL_TMP0, s));
  HIPCHK(copy_bytes(M.Y2, M.env64, aK * 8, s));
  HIPCHK(axpy_dev(M.Y2, M.w64[tau], M.scal + SCAL_TMP0, -POLAR_REG, aK, s));
  // polar_core consumes its source before it reuses M.Y2
  ttn_status st;
  if (M.gauge_fix) {
    double* P = nullptr;
    st = polar_core(M, M.Y2, a, K, -1.0, M.w64[tau], s, nullptr, false, &P, M.w64[tau], M.env64);
    if (st) return st;
    // absorb P^T on the input legs of the layer above: w' = P .l (P .r w),
    // or v' = P v P^T at the top
    if (tau < M.n - 1) {
      const int c2 = M.dims[tau + 1];
      HIPCHK(apply_r(M, P_F64, P, M.w64[tau + 1], M.Y2, c2, a, 0.0, s));
      HIPCHK(apply_l(M, P_F64, P, M.Y2, M.w64[tau + 1], c2, a, 0.0, s));
      if ((st = refresh_shadow(M, tau + 1, s))) return st;
      M.pc_from = std::max(M.pc_from, tau + 2);
    } else {
      HIPCHK(mm(M, P_F64, P, false, M.vtop, false, M.G, a, 1.0, 0.0, s));
      HIPCHK(mm(M, P_F64, M.G, false, P, true, M.vtop, a, 1.0, 0.0, s));
      if (M.prec != TTN_FP64) HIPCHK(convert_f64_to_f32(M.vtop, (float*)M.vT, (size_t)a * a, s));
      M.rho_from = M.pc_from = 1 << 20;
    }
  } else {
    st = polar_core(M, M.Y2, a, K, -1.0, M.w64[tau], s, M.Qw[tau], M.qw_valid[tau] != 0, nullptr, M.w64[tau],
                    M.env64);
    if (st) return st;
    M.qw_valid[tau] = 1;
  }
  HIPCHK(ratio_minmax(M.nrm, a, M.scal + SCAL_RATIO, M.scal + SCAL_RATIO_MIN, s));
  if ((st = ortho_check(M, tau, s))) return st;
  if ((st = refresh_shadow(M, tau, s))) return st;
  M.env_tau = -1;
  M.dressed_tau = -1;
  M.ops_upto = std::min(M.ops_upto, tau - 1);
  M.rho_from = std::max(M.rho_from, tau);
  M.pc_from = std::max(M.pc_from, tau + 1);
  return TTN_OK;
}

// H_top y for the two sites of level n-1 (float64 copies of the operators):
//   out = h y + y h^T + sum_k (A_k y B_k^T + B_k y A_k^T)
// as  stage = [y, y B_1^T, .., y B_D^T, y A_1^T, .., y A_D^T]  (one batched
// product), then out = [h, A_1..A_D, B_1..B_D] . stage (one product whose
// contraction index runs over the operator blocks), then out += y h^T.
// With right-site operators of their own (hopR64), the factors on the right
// of y (B_k^T, A_k^T, h^T) are the right site's.
// (staged: y is already in stage[0])
hipError_t top_matvec(Member& M, const double* y, double* out, hipStream_t s, bool staged) {
  if (M.matvec) return M.matvec(M, y, out, s);
  const int x = M.dims[M.n - 1], D = M.D;
  const long long xx = (long long)x * x;
  const double* hR = M.hopR64 ? M.hopR64 : M.hop64;
  const double* AR = hR + xx;
  const double* BR = hR + (1 + D) * xx;
  hipError_t e;
  if (!staged && (e = copy_bytes(M.lzStage, y, xx * 8, s))) return e;
  if (D > 0) {
    // stage[1 + half*D + k] = y . (half ? A_k : B_k)^T, both halves in one
    // launch: a two-level batch (k, half) whose outer step moves from the B
    // block to the A block below it and from slot 1 + k to slot 1 + D + k
    GemmDesc g = desc0();
    g.batch1 = D;
    g.batch = 2 * D;
    g.M = x; g.N = x; g.K = x;
    g.A = y; g.sAm = x; g.sAk = 1; g.sAb = 0; g.sAb2 = 0;
    g.B = BR; g.sBk = 1; g.sBn = x; g.sBb = xx; g.sBb2 = (long long)(AR - BR);
    g.C = M.lzStage + xx; g.sCm = x; g.sCn = 1; g.sCb = xx; g.sCb2 = D * xx;
    if ((e = run(M, P_F64, g, s, OC_TOP_MM))) return e;
  }
  GemmDesc g = desc0();  // out = sum_j op_j stage_j
  g.M = x; g.N = x; g.K = (int)((1 + 2 * D) * x); g.K2 = x;
  g.A = M.hop64; g.sAm = x; g.sAk = 1; g.sAk1 = xx;
  g.B = M.lzStage; g.sBk = x; g.sBn = 1; g.sBk1 = xx;
  g.C = out; g.sCm = x; g.sCn = 1;
  if ((e = run(M, P_F64, g, s, OC_TOP_MM))) return e;
  return mm(M, P_F64, y, false, hR, true, out, x, 1.0, 1.0, s);  // + y h^T
}

// The top update, in three parts.  top_prepare copies the top operators to
// float64, makes them exactly symmetric (or antisymmetric) and clears the
// convergence flag and the restart count; top_restarts runs Lanczos restarts;
// top_finish fixes the sign of v and stores the energy.  Restarts after the
// one whose residual met the target do nothing: a device flag (set by
// lz_mark_done) makes every kernel of a later restart return at once.  With
// `sync` the host reads the flags after every restart and stops launching once
// every member of the launch group has converged (*converged tells whether
// they did); without it `count` restarts are launched and nothing is read
// back, so they can be captured into a graph.  Both give the same arithmetic.
ttn_status top_prepare(Member& M, hipStream_t s) {
  const int n = M.n, x = M.dims[n - 1], D = M.D;
  const size_t xx = (size_t)x * x;
  if (M.prec == TTN_FP64) {
    HIPCHK(copy_bytes(M.hop64, M.opH[n - 1], xx * 8, s));
    if (D) {
      HIPCHK(copy_bytes(M.Aop64, M.opA[n - 1], D * xx * 8, s));
      HIPCHK(copy_bytes(M.Bop64, M.opB[n - 1], D * xx * 8, s));
    }
  } else {
    HIPCHK(convert_f32_to_f64((const float*)M.opH[n - 1], M.hop64, xx, s));
    if (D) {
      HIPCHK(convert_f32_to_f64((const float*)M.opA[n - 1], M.Aop64, D * xx, s));
      HIPCHK(convert_f32_to_f64((const float*)M.opB[n - 1], M.Bop64, D * xx, s));
    }
  }
  // the operators are symmetric (h) or of the parity of their level-0 term
  // in exact arithmetic; remove the rounding asymmetry so H_top is symmetric
  HIPCHK(symmetrize_f64(M.hop64, x, 1.0, s));
  for (int k = 0; k < D; ++k) {
    HIPCHK(symmetrize_f64(M.Aop64 + k * xx, x, M.anti[k] ? -1.0 : 1.0, s));
    HIPCHK(symmetrize_f64(M.Bop64 + k * xx, x, M.anti[k] ? -1.0 : 1.0, s));
  }
  if (M.hopR64) {
    HIPCHK(copy_bytes(M.hopR64, M.topR, (1 + 2 * D) * xx * 8, s));
    HIPCHK(symmetrize_f64(M.hopR64, x, 1.0, s));
    for (int k = 0; k < D; ++k) {
      HIPCHK(symmetrize_f64(M.hopR64 + (1 + k) * xx, x, M.anti[k] ? -1.0 : 1.0, s));
      HIPCHK(symmetrize_f64(M.hopR64 + (1 + D + k) * xx, x, M.anti[k] ? -1.0 : 1.0, s));
    }
  }
  HIPCHK(zero_int(M.lzint + LZ_DONE, 2, s));  // the flag and the count of restarts run
  return TTN_OK;
}

ttn_status top_restarts(Member& M, hipStream_t s, int count, bool sync, bool* converged) {
  const int n = M.n, x = M.dims[n - 1];
  const size_t xx = M.top_len ? (size_t)M.top_len : (size_t)x * x;
  const int m = (int)std::min<long long>(M.krylov, (long long)xx);
  *converged = false;
  // members of a launch group share the restart loop; a member whose
  // residual met the target sets its flag and every kernel of its later
  // restarts returns at once, so it ends with the vector it has alone
  int* done = M.lzint + LZ_DONE;
  const int* skip = done;
  for (int rs = 0; rs < count; ++rs) {
    SkipScope skip_done(skip);
    // q_0 = v / ||v||
    HIPCHK(pair_f64(M.vtop, M.vtop, (long long)xx, M.scal + SCAL_TMP0, M.part, s));
    HIPCHK(scale_rsqrt(M.vtop, M.scal + SCAL_TMP0, xx, s));
    HIPCHK(copy_bytes(M.lzQ, M.vtop, xx * 8, s));
    HIPCHK(zero_int(M.lzint, 2, s));  // stop, m_eff
    for (int j = 0; j < m; ++j) {
      double* qj = M.lzQ + (size_t)j * xx;
      // q_j is in stage[0] already from the previous step (j > 0)
      HIPCHK(top_matvec(M, qj, M.lzW, s, j > 0));
      // two passes of classical Gram-Schmidt against q_0..q_j: the first
      // also yields alpha_j and ||H q_j||^2, the second repairs round-off;
      // the second is fused with the recurrence step (alpha_j, beta_j, with
      // an invariant-subspace test well below the residual target so that a
      // start vector close to convergence still spans a useful Krylov space,
      // and q_{j+1}, also staged for the next product)
      double* c1 = M.coef;
      double* c2 = M.coef + (m + 2);
      HIPCHK(lz_reorth_first(M.lzW, M.lzQ, j + 1, xx, c1, M.lzpart, s));
      HIPCHK(lz_reorth_final(M.lzW, M.lzQ, j + 1, xx, c1, c2, M.lzpart, M.lznrm, M.alpha, M.beta, 1e-14, M.lzint,
                             M.lzint + 1, M.lzQ + (size_t)(j + 1) * xx, j + 1 < m && !M.matvec ? M.lzStage : nullptr,
                             s));
    }
    HIPCHK(lz_build_T(M.alpha, M.beta, m, M.lzint, M.lzint + 1, M.Tm, s));
    HIPCHK(jacobi_eig_f64(M.Tm, M.Vm, m, 80, std::max(1e-15, 2.2e-16 * m), M.jinfo + 16, M.jscratch, s, skip));
    HIPCHK(lz_select_lowest(M.Tm, M.Vm, m, M.ycoef, M.scal + SCAL_THETA, s));
    GemmDesc g = desc0();  // v = Q[0..m-1]^T y
    g.M = 1; g.N = (int)xx; g.K = m;
    g.A = M.ycoef; g.sAm = 0; g.sAk = 1;
    g.B = M.lzQ; g.sBk = (long long)xx; g.sBn = 1;
    g.C = M.vtop; g.sCm = 0; g.sCn = 1;
    HIPCHK(run(M, P_F64, g, s));
    HIPCHK(pair_f64(M.vtop, M.vtop, (long long)xx, M.scal + SCAL_TMP0, M.part, s));
    HIPCHK(scale_rsqrt(M.vtop, M.scal + SCAL_TMP0, xx, s));
    HIPCHK(top_matvec(M, M.vtop, M.lzHv, s));
    HIPCHK(pair_f64(M.vtop, M.lzHv, (long long)xx, M.scal + SCAL_LAM, M.part, s));
    HIPCHK(residual_vec(M.lzHv, M.vtop, M.scal + SCAL_LAM, M.lzR, xx, s));
    HIPCHK(pair_f64(M.lzR, M.lzR, (long long)xx, M.scal + SCAL_RES, M.part, s));
    HIPCHK(sqrt_inplace(M.scal + SCAL_RES, s));
    HIPCHK(lz_mark_done(M.scal + SCAL_RES, M.scal + SCAL_LAM, M.ltol, done, done + 1, s));
    if (!sync) continue;
    // every member of the launch group (they share the restarts)
    const int gc = grp().count;
    std::vector<double> hs((size_t)gc * (SCAL_ERR + 1));
    if (gc > 1)
      HIPCHK(hipMemcpy2DAsync(hs.data(), (SCAL_ERR + 1) * sizeof(double), M.scal, (size_t)grp().stride,
                              (SCAL_ERR + 1) * sizeof(double), gc, hipMemcpyDeviceToHost, s));
    else
      HIPCHK(hipMemcpyAsync(hs.data(), M.scal, (SCAL_ERR + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all_conv = true;
    for (int q = 0; q < gc; ++q) {
      const double* h = hs.data() + (size_t)q * (SCAL_ERR + 1);
      if (h[SCAL_ERR] != 0.0) return fail(TTN_EHIP, "a Jacobi eigensolver aborted (grid barrier wait exceeded its bound)");
      if (!(h[SCAL_RES] <= M.ltol * std::max(1.0, std::fabs(h[SCAL_LAM])))) all_conv = false;
    }
    if (all_conv) {
      *converged = true;
      break;
    }
  }
  if (!sync) *converged = true;  // not known here: read from the flag afterwards
  return TTN_OK;
}

// keep_prev: the energy replaced is not the previous update's (a top update
// continued after a first finish), so the stored previous energy stays
ttn_status top_finish(Member& M, hipStream_t s, bool keep_prev) {
  const int x = M.dims[M.n - 1];
  const size_t xx = M.top_len ? (size_t)M.top_len : (size_t)x * x;
  HIPCHK(sign_fix(M.vtop, xx, s));
  HIPCHK(energy_store(M.scal + SCAL_LAM, M.scal + SCAL_SHIFT, (double)M.L, (double)M.ly, M.scal + SCAL_LAM,
                      keep_prev ? nullptr : M.scal + SCAL_EPREV, s));
  if (M.prec != TTN_FP64) HIPCHK(convert_f64_to_f32(M.vtop, (float*)M.vT, xx, s));
  M.rho_from = M.pc_from = 1 << 20;
  return TTN_OK;
}

// The whole top update, eagerly: every restart of the budget until the
// launch group has converged.
ttn_status stage_update_top(Member& M, hipStream_t s, bool* converged) {
  ByteCount bc(M, M.bytes_top);
  ttn_status st;
  if ((st = top_prepare(M, s))) return st;
  if ((st = top_restarts(M, s, M.restarts, true, converged))) return st;
  return top_finish(M, s);
}

ttn_status init_member(Member& M, hipStream_t s, bool* conv) {
  const int n = M.n, d = M.d, D = M.D;
  HIPCHK(zero_int(M.jinfo, 64, s));  // solver reports read by ttn_stats
  const size_t dd = (size_t)d * d;
  // level-0 operators (host -> device through a float64 staging area)
  std::vector<double> h0 = M.h1;
  for (int i = 0; i < d; ++i) h0[i * d + i] -= M.c;
  double* stage = M.env64;  // scratch
  HIPCHK(hipMemcpyAsync(stage, h0.data(), dd * 8, hipMemcpyHostToDevice, s));
  if (D) {
    HIPCHK(hipMemcpyAsync(stage + dd, M.A.data(), D * dd * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(stage + (1 + D) * dd, M.B.data(), D * dd * 8, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (M.prec == TTN_FP64) {
    HIPCHK(copy_bytes(M.opH[0], stage, dd * 8, s));
    if (D) {
      HIPCHK(copy_bytes(M.opA[0], stage + dd, D * dd * 8, s));
      HIPCHK(copy_bytes(M.opB[0], stage + (1 + D) * dd, D * dd * 8, s));
    }
  } else {
    HIPCHK(convert_f64_to_f32(stage, (float*)M.opH[0], dd, s));
    if (D) {
      HIPCHK(convert_f64_to_f32(stage + dd, (float*)M.opA[0], D * dd, s));
      HIPCHK(convert_f64_to_f32(stage + (1 + D) * dd, (float*)M.opB[0], D * dd, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  // isometries
  for (int t = 1; t < n; ++t) {
    const int a = M.dims[t], b = M.dims[t - 1];
    const size_t e = (size_t)a * b * b;
    if (M.w0) {
      HIPCHK(hipMemcpyAsync(M.w64[t], M.w0[t - 1], e * 8, hipMemcpyHostToDevice, s));
    } else {
      HIPCHK(gaussian_f64(M.env64, e, M.seed, (unsigned long long)t, s));
      ttn_status st = polar_core(M, M.env64, a, (long long)b * b, 1.0, M.w64[t], s);
      if (st) return st;
    }
    ttn_status st = refresh_shadow(M, t, s);
    if (st) return st;
  }
  HIPCHK(hipStreamSynchronize(s));
  // scalars
  double init_scal[SCAL_N] = {0};
  init_scal[SCAL_RATIO_MIN] = 1.0;
  init_scal[SCAL_SHIFT] = M.c;
  HIPCHK(hipMemcpyAsync(M.scal, init_scal, sizeof init_scal, hipMemcpyHostToDevice, s));
  // top start vector
  const int x = M.dims[n - 1];
  const size_t xx = (size_t)x * x;
  if (M.v0) {
    HIPCHK(hipMemcpyAsync(M.vtop, M.v0, xx * 8, hipMemcpyHostToDevice, s));
  } else {
    HIPCHK(gaussian_f64(M.vtop, xx, M.seed ^ 0x5bd1e995ull, 0xfffffffull, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (int t = 1; t < n; ++t) {
    ttn_status st = stage_ascend(M, t, s);
    if (st) return st;
  }
  M.ops_upto = n - 1;
  ttn_status st = stage_update_top(M, s, conv);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(s));
  return TTN_OK;
}

void layer_flops(const Member& M, double* bulk, double* f64) {
  const int n = M.n, D = M.D;
  auto asc = [&](int t) { double a = M.dims[t], b = M.dims[t - 1]; return 2 * a * b * b * b + 2 * a * a * b * b; };
  double F = 0, G = 0;
  for (int t = 1; t < n; ++t) {
    double a = M.dims[t], b = M.dims[t - 1];
    double env = (4 + 8.0 * D) * a * b * b * b + (2 + 4.0 * D) * a * a * b * b;
    double reasc = (4 + 4.0 * D) * a * b * b * b + 2 * a * a * b * b + 2.0 * D * asc(t);
    double chain = 0;
    for (int sg = t; sg < n; ++sg) chain += 2.0 * D * asc(sg);
    double desc = 0;
    for (int sg = t + 1; sg < n; ++sg) {
      double aa = M.dims[sg], bb = M.dims[sg - 1];
      desc += D * (12 * aa * bb * bb * bb + 4 * aa * aa * bb * bb);
    }
    F += env + reasc + chain + desc;
    // float64: polar (POLAR_REFRESH Gram + rotate, gauge compensation or
    // final product) + orthonormality Gram
    G += (POLAR_REFRESH * 4.0 + 2.0 + 2.0) * a * a * b * b;
  }
  for (int sg = 2; sg < n; ++sg) {
    double a = M.dims[sg], b = M.dims[sg - 1];
    F += 2 * a * a * b * b + 4 * a * b * b * b;
  }
  *bulk = F;
  *f64 = G;
}

// Everything of a member's configuration that decides its layout and the
// host-side parameters of its launches (the Hamiltonian's values live on the
// device and may differ inside a group).
std::vector<double> group_key(const Member& M) {
  std::vector<double> k = {(double)M.L, (double)M.d, (double)M.D, (double)M.chi, (double)M.prec, (double)M.ly,
                           (double)M.krylov, (double)M.restarts, M.ltol, (double)M.gauge_fix, (double)M.evd};
  for (int a : M.anti) k.push_back((double)a);
  return k;
}

// Members that may share a coarse group: every configuration value but L,
// and the same top bond dimension (then their shapes agree level by level).
std::vector<double> coarse_key(const Member& M) {
  std::vector<double> k = group_key(M);
  k.erase(k.begin());
  k.push_back((double)M.dims[M.n - 1]);
  return k;
}

int member_cmax(const Member& M) {
  int cmax = 0;
  for (int t = 0; t < M.n; ++t) cmax = std::max(cmax, M.dims[t]);
  return cmax;
}

// Layout order and padded depth of a batch: sorted by coarse key, deepest
// first, then by the full key (so that members of identical configuration
// are adjacent); in a batch, the members of a coarse group with bond
// dimensions <= 128 are padded to the group's largest depth.
void plan_batch(const std::vector<Member>& ms, std::vector<int>& order, std::vector<int>& npad) {
  const int batch = (int)ms.size();
  order.resize(batch);
  npad.assign(batch, 0);
  std::vector<std::vector<double>> ck(batch), fk(batch);
  for (int i = 0; i < batch; ++i) {
    order[i] = i;
    ck[i] = coarse_key(ms[i]);
    fk[i] = group_key(ms[i]);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (ck[x] != ck[y]) return ck[x] < ck[y];
    if (ms[x].n != ms[y].n) return ms[x].n > ms[y].n;
    return fk[x] < fk[y];
  });
  if (batch < 2) return;
  for (int k = 0; k < batch;) {
    int j = k + 1;
    while (j < batch && ck[order[j]] == ck[order[k]]) ++j;
    if (member_cmax(ms[order[k]]) <= 128)
      for (int i = k; i < j; ++i) npad[order[i]] = ms[order[k]].n;
    k = j;
  }
}

// Host-side stage state of the leader, copied to the other members of its
// group after every group-wide call (they took the same path).
void sync_group_state(Ctx& c, const Ctx::Group& G) {
  const Member& L = c.m[G.members[0]];
  for (size_t i = 1; i < G.members.size(); ++i) {
    Member& M = c.m[G.members[i]];
    M.rho_from = L.rho_from; M.pc_from = L.pc_from; M.dressed_tau = L.dressed_tau; M.env_tau = L.env_tau;
    M.ops_upto = L.ops_upto; M.rb_cur = L.rb_cur; M.qw_valid = L.qw_valid;
    M.bytes_layers = L.bytes_layers; M.bytes_top = L.bytes_top;
  }
}

// f(leader, group) for every group, with the launch group set.
template <class F>
ttn_status for_groups(Ctx& c, F f) {
  for (auto& G : c.groups) {
    GroupScope gs((int)G.members.size(), G.stride);
    ttn_status st = f(c.m[G.members[0]], G);
    if (st) return st;
    sync_group_state(c, G);
  }
  return TTN_OK;
}

// The layer part of one sweep for one member on stream s.
ttn_status sweep_layers(Member& M, hipStream_t s) {
  ByteCount bc(M, M.bytes_layers);
  ttn_status st;
  if ((st = stage_descend_rho(M, s))) return st;
  for (int t = 1; t < M.n; ++t) {
    if ((st = stage_descend_dressed(M, t, s))) return st;
    if ((st = stage_env(M, t, s))) return st;
    if ((st = stage_update_layer(M, t, s))) return st;
    if ((st = stage_ascend(M, t, s))) return st;
    M.ops_upto = std::max(M.ops_upto, t);
  }
  return TTN_OK;
}

// The layer part of one grouped sweep (a schedule of our own, not the
// paper's): every layer of a group takes its environment from the same state,
// so the dressed chains of all of them come from one top-down pass over the
// ascended operators (the carried operators of a layer's own chain are those
// when nothing changes in between).  Groups: every layer (groups = 1), or the
// odd layers and then the even ones (groups = 2).  Per group: rho, then from
// the top down, for each level: the environment of its layer when the layer
// is in the group, the chains one level down (which still read the old
// isometry), the update; then every layer is ascended again.  A gauge-fixed
// update moves its rotation into the layer above (or v), already updated in
// this pass: the state is the same.
ttn_status sweep_layers_grouped(Member& M, int groups, hipStream_t s) {
  ByteCount bc(M, M.bytes_layers);
  const int n = M.n;
  ttn_status st;
  for (int gi = 0; gi < groups; ++gi) {
    const int parity = gi == 0 ? 1 : 0;
    bool any = false;
    for (int t = 1; t < n; ++t) any |= groups == 1 || t % 2 == parity;
    if (!any) continue;
    if ((st = stage_descend_rho(M, s))) return st;
    M.rb_cur = 0;
    if ((st = dressed_top(M, M.opA[n - 1], M.opB[n - 1], s))) return st;
    for (int sg = n - 1; sg >= 1; --sg) {
      const bool upd = groups == 1 || sg % 2 == parity;
      if (upd && (st = stage_env(M, sg, s))) return st;
      if (sg > 1 && (st = dressed_down(M, sg, M.opA[sg - 1], M.opB[sg - 1], s))) return st;
      if (upd && (st = stage_update_layer(M, sg, s))) return st;
    }
    for (int t = 1; t < n; ++t)
      if ((st = stage_ascend(M, t, s))) return st;
    M.ops_upto = n - 1;
  }
  M.dressed_tau = -1;
  return TTN_OK;
}

// The layer part of one sweep for a coarse group (members sorted by depth,
// deepest first, one layout at one stride): the stages of sweep_layers level
// by level over the members that have the level, each launch covering a
// contiguous range of members.  The two-site matrices sit in slot sg % 2 at
// level sg for every member, so that members whose chains started at
// different tops share each descent.  Every member does the arithmetic it
// does alone.  No host synchronisation: capturable.
ttn_status sweep_layers_coarse(Ctx& c, const Ctx::Group& G, hipStream_t s) {
  const int cnt = (int)G.members.size();
  auto nlev = [&](int i) { return c.m[G.members[i]].n; };
  const int nmax = nlev(0);
  // members [0, prefix(X)) have a level X; [first_top(X), prefix(X)) have their top there
  auto prefix = [&](int X) { int k = 0; while (k < cnt && nlev(k) - 1 >= X) ++k; return k; };
  auto first_top = [&](int X) { int k = 0; while (k < cnt && nlev(k) - 1 > X) ++k; return k; };
  // f(base member) on members [first, first + count) as one launch group;
  // the product bytes it issues are every member's
  std::vector<double> bytes(cnt, 0.0);
  auto on = [&](int first, int count, auto f) -> ttn_status {
    if (count <= 0) return TTN_OK;
    GroupScope gs(count, G.stride);
    Member& B = c.m[G.members[first]];
    B.bytes_acc = 0.0;
    B.counting = true;
    ttn_status st = f(B);
    B.counting = false;
    for (int i = first; i < first + count; ++i) bytes[i] += B.bytes_acc;
    return st;
  };
  ttn_status st;
  // rho of every level: top matrices where each member's top is, descents below
  for (int lv = nmax - 1; lv >= 1; --lv) {
    const int p = prefix(lv), f = first_top(lv);
    if ((st = on(f, p - f, [&](Member& B) -> ttn_status {
           const int x = B.dims[lv];
           BraScope bra;
           HIPCHK(mm(B, B.gp(), B.vT, false, B.vT, true, B.rho[lv], x, 0.5, 0.0, s));
           HIPCHK(mm(B, B.gp(), B.vT, true, B.vT, false, B.rho[lv], x, 0.5, 1.0, s));
           return TTN_OK;
         })))
      return st;
    if (lv < 2) continue;
    if ((st = on(0, p, [&](Member& B) -> ttn_status {
           const int a = B.dims[lv], b = B.dims[lv - 1];
           const Prec q = B.gp();
           HIPCHK(left_mul(B, q, B.rho[lv], B.wT[lv], B.Pc[lv], a, b, 1.0, 0.0, s));
           HIPCHK(close_l(B, q, B.wT[lv], B.Pc[lv], B.rho[lv - 1], a, b, 0.5, 0.0, s));
           HIPCHK(close_r(B, q, B.wT[lv], B.Pc[lv], B.rho[lv - 1], a, b, 0.5, 1.0, s));
           return TTN_OK;
         })))
      return st;
  }
  for (int t = 1; t < nmax; ++t) {
    const int pt = prefix(t);
    const int D = c.m[G.members[0]].D;
    // dressed chains: A^(t-1), B^(t-1) carried up through layers t .. (own top)
    for (int sg = t; sg < nmax; ++sg)
      if ((st = on(0, prefix(sg), [&](Member& B) -> ttn_status {
             const int a = B.dims[sg], b = B.dims[sg - 1];
             const long long bb = (long long)b * b, aa = (long long)a * a, cube = (long long)a * bb;
             const Prec q = B.gp();
             const void* pa = sg == t ? B.opA[t - 1] : B.At[sg - 1];
             const void* pb = sg == t ? B.opB[t - 1] : B.Bt[sg - 1];
             HIPCHK(apply_r_k(B, q, pa, bb, B.wT[sg], 0, B.S2, cube, a, b, 0.0, D, s));
             HIPCHK(close_aa_k(B, q, B.wT[sg], 0, B.S2, cube, B.At[sg], aa, a, b, 1.0, 0.0, D, s, B.anti_bits()));
             HIPCHK(apply_l_k(B, q, pb, bb, B.wT[sg], 0, B.S2, cube, a, b, 0.0, D, s));
             HIPCHK(close_aa_k(B, q, B.wT[sg], 0, B.S2, cube, B.Bt[sg], aa, a, b, 1.0, 0.0, D, s, B.anti_bits()));
             return TTN_OK;
           })))
        return st;
    // the top dressing of each member at its own top, the descents below it
    for (int sg = nmax - 1; sg >= t; --sg) {
      const int p = prefix(sg), f = first_top(sg);
      if ((st = on(f, p - f, [&](Member& B) -> ttn_status {
             B.rb_cur = sg % 2;
             return dressed_top(B, B.At[sg], B.Bt[sg], s);
           })))
        return st;
      if (sg == t) break;
      if ((st = on(0, p, [&](Member& B) -> ttn_status {
             B.rb_cur = sg % 2;
             return dressed_down(B, sg, B.At[sg - 1], B.Bt[sg - 1], s);
           })))
        return st;
    }
    if ((st = on(0, pt, [&](Member& B) -> ttn_status {
           B.rb_cur = t % 2;
           return stage_env(B, t, s);
         })))
      return st;
    // the update (its gauge rotation goes into the layer above, or into v
    // for the members whose top layer this is), then the new operators
    const int ft = first_top(t);
    if ((st = on(0, ft, [&](Member& B) -> ttn_status { return stage_update_layer(B, t, s); }))) return st;
    if ((st = on(ft, pt - ft, [&](Member& B) -> ttn_status { return stage_update_layer(B, t, s); }))) return st;
    if ((st = on(0, pt, [&](Member& B) -> ttn_status { return stage_ascend(B, t, s); }))) return st;
  }
  // host state as a member's own sweep_layers leaves it
  const Member& L0 = c.m[G.members[0]];
  for (int i = 0; i < cnt; ++i) {
    Member& M = c.m[G.members[i]];
    M.bytes_layers = bytes[i];
    M.rho_from = std::max(1, M.n - 1);
    M.pc_from = M.n;
    M.dressed_tau = -1;
    M.env_tau = -1;
    M.ops_upto = M.n - 1;
    for (int t = 1; t < M.n; ++t) M.qw_valid[t] = L0.qw_valid[t];
  }
  return TTN_OK;
}

// The layer part for the whole batch: one member runs on the caller's
// stream; a batch forks to the pool streams (member i on stream i mod P) and
// joins back.  No host synchronisation inside: capturable.
ttn_status sweep_layers_all(Ctx& c, hipStream_t s) {
  if (!c.coarse.empty()) {
    // coarse groups (one configuration, every length), side by side
    if (c.pool.empty()) {
      const int P = (int)std::min<size_t>(POOL_STREAMS, c.coarse.size());
      c.pool.resize(P, nullptr);
      c.join.resize(P, nullptr);
      for (int i = 0; i < P; ++i) {
        HIPCHK(hipStreamCreateWithFlags(&c.pool[i], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c.join[i], hipEventDisableTiming));
      }
      HIPCHK(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
    }
    const int P = (int)c.pool.size();
    HIPCHK(hipEventRecord(c.fork, s));
    for (int i = 0; i < P; ++i) HIPCHK(hipStreamWaitEvent(c.pool[i], c.fork, 0));
    for (size_t gi = 0; gi < c.coarse.size(); ++gi) {
      ttn_status st = sweep_layers_coarse(c, c.coarse[gi], c.pool[gi % P]);
      if (st) return st;
    }
    for (int i = 0; i < P; ++i) {
      HIPCHK(hipEventRecord(c.join[i], c.pool[i]));
      HIPCHK(hipStreamWaitEvent(s, c.join[i], 0));
    }
    return TTN_OK;
  }
  if (c.groups.size() == 1) {
    const Ctx::Group& G = c.groups[0];
    GroupScope gs((int)G.members.size(), G.stride);
    ttn_status st = sweep_layers(c.m[G.members[0]], s);
    if (!st) sync_group_state(c, G);
    return st;
  }
  if (c.pool.empty()) {
    const int P = (int)std::min<size_t>(POOL_STREAMS, c.groups.size());
    c.pool.resize(P, nullptr);
    c.join.resize(P, nullptr);
    for (int i = 0; i < P; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&c.pool[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&c.join[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
  }
  const int P = (int)c.pool.size();
  HIPCHK(hipEventRecord(c.fork, s));
  for (int i = 0; i < P; ++i) HIPCHK(hipStreamWaitEvent(c.pool[i], c.fork, 0));
  for (size_t gi = 0; gi < c.groups.size(); ++gi) {
    const Ctx::Group& G = c.groups[gi];
    GroupScope gs((int)G.members.size(), G.stride);
    ttn_status st = sweep_layers(c.m[G.members[0]], c.pool[gi % P]);
    if (st) return st;
    sync_group_state(c, G);
  }
  for (int i = 0; i < P; ++i) {
    HIPCHK(hipEventRecord(c.join[i], c.pool[i]));
    HIPCHK(hipStreamWaitEvent(s, c.join[i], 0));
  }
  return TTN_OK;
}

// The top update of a coarse group: the operators prepared and the result
// finished per length (a member's top operators sit at its own level, its
// energy divides by its own L), the restarts over the whole group (one top
// bond dimension, one layout): eagerly with a host check after each (all
// non-null), or `plan` of them without host reads (capturable).
ttn_status top_coarse(Ctx& c, const Ctx::Group& G, hipStream_t s, bool* all, int plan = 0) {
  const int cnt = (int)G.members.size();
  std::vector<std::pair<int, int>> runs;  // [first, end) of equal depth
  for (int k = 0; k < cnt;) {
    int j = k + 1;
    while (j < cnt && c.m[G.members[j]].n == c.m[G.members[k]].n) ++j;
    runs.push_back({k, j});
    k = j;
  }
  ttn_status st;
  for (auto& r : runs) {
    GroupScope gs(r.second - r.first, G.stride);
    if ((st = top_prepare(c.m[G.members[r.first]], s))) return st;
  }
  Member& B = c.m[G.members[0]];
  bool conv = false;
  {
    GroupScope gs(cnt, G.stride);
    B.bytes_acc = 0.0;
    B.counting = true;
    st = all ? top_restarts(B, s, B.restarts, true, &conv)
             : top_restarts(B, s, std::min(plan, B.restarts), false, &conv);
    B.counting = false;
    if (st) return st;
  }
  if (all && !conv) *all = false;
  for (auto& r : runs) {
    GroupScope gs(r.second - r.first, G.stride);
    if ((st = top_finish(c.m[G.members[r.first]], s))) return st;
  }
  for (int i = 0; i < cnt; ++i) {
    Member& M = c.m[G.members[i]];
    M.bytes_top = B.bytes_acc;
    M.rho_from = M.pc_from = 1 << 20;
  }
  return TTN_OK;
}

// The top update of every member, eagerly (launch group by launch group, or
// coarse group by coarse group); *all is cleared when a member stopped at its
// restart budget.
ttn_status top_all(Ctx& c, hipStream_t s, bool* all) {
  if (!c.coarse.empty()) {
    for (auto& G : c.coarse) {
      ttn_status st = top_coarse(c, G, s, all);
      if (st) return st;
    }
    return TTN_OK;
  }
  return for_groups(c, [&](Member& M, const Ctx::Group&) -> ttn_status {
    bool conv = false;
    ttn_status r = stage_update_top(M, s, &conv);
    if (!r && !conv) *all = false;
    return r;
  });
}

// The top update with `plan` restarts (at most each member's budget)
// launched without host reads, so that it can be captured into a graph
// (coarse group by coarse group when the batch has them).
ttn_status top_planned(Ctx& c, hipStream_t s, int plan) {
  if (!c.coarse.empty()) {
    for (auto& G : c.coarse) {
      ttn_status st = top_coarse(c, G, s, nullptr, plan);
      if (st) return st;
    }
    return TTN_OK;
  }
  return for_groups(c, [&](Member& M, const Ctx::Group&) -> ttn_status {
    ByteCount bc(M, M.bytes_top);
    bool conv = false;
    ttn_status st;
    if ((st = top_prepare(M, s))) return st;
    if ((st = top_restarts(M, s, std::min(plan, M.restarts), false, &conv))) return st;
    return top_finish(M, s);
  });
}

// Restarts run by the slowest member's last top update, and whether every
// member's flag is set (reads the device; synchronises the stream).
ttn_status top_status(Ctx& c, hipStream_t s, int* most, bool* all) {
  HIPCHK(hipStreamSynchronize(s));
  *most = 0;
  *all = true;
  for (auto& M : c.m) {
    int f[2] = {0, 0};
    HIPCHK(hipMemcpy(f, M.lzint + LZ_DONE, sizeof f, hipMemcpyDeviceToHost));
    *most = std::max(*most, f[1]);
    if (!f[0]) *all = false;
  }
  return TTN_OK;
}

// After a planned top update: the launch groups with a member whose flag is
// still clear get the rest of their restart budget eagerly (host reads after
// each restart), and v and the energy are finished again (the same
// arithmetic as one eager update: a finished v only had its sign fixed, and
// a restart normalises its start vector, so the sign carries through
// exactly).  *all is cleared when a member stopped at its budget; *most
// receives the restarts the slowest member ran.
ttn_status top_complete(Ctx& c, hipStream_t s, int plan, int* most, bool* all) {
  ttn_status st;
  if ((st = top_status(c, s, most, all))) return st;
  if (*all) return TTN_OK;
  for (auto& G : c.groups) {
    bool pending = false;
    for (int i : G.members) {
      int f = 0;
      HIPCHK(hipMemcpy(&f, c.m[i].lzint + LZ_DONE, sizeof f, hipMemcpyDeviceToHost));
      if (!f) pending = true;
    }
    Member& L = c.m[G.members[0]];
    const int rest = L.restarts - std::min(plan, L.restarts);
    if (!pending || rest <= 0) continue;
    GroupScope gs((int)G.members.size(), G.stride);
    bool conv = false;
    if ((st = top_restarts(L, s, rest, true, &conv))) return st;
    if ((st = top_finish(L, s, true))) return st;
    sync_group_state(c, G);
  }
  return top_status(c, s, most, all);
}

// Captures (once per restart plan) or replays the graph of a planned top update.
ttn_status top_graph_launch(Ctx& c, int plan) {
  auto it = c.top_exec.find(plan);
  if (it == c.top_exec.end()) {
    if (!c.cap_s) HIPCHK(hipStreamCreateWithFlags(&c.cap_s, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c.cap_s, hipStreamCaptureModeRelaxed));
    ttn_status st = top_planned(c, c.cap_s, plan);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c.cap_s, &g);
    if (st) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    HIPCHK(e);
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHK(e);
    it = c.top_exec.emplace(plan, ge).first;
  }
  HIPCHK(hipGraphLaunch(it->second, c.s));
  return TTN_OK;
}

// The top update after a replayed layer part.  use_graph == 2: every restart
// of the budget in the graph, no host read.  Otherwise the graph holds the
// restarts the slowest member needed in the previous update, one host read
// afterwards finishes any member that needs more (eagerly), and the plan
// follows what this update needed (a plan held at the largest need so far,
// that of the first solves from random isometries, kept launching restarts
// that return at once in every later sweep).
ttn_status top_after_graph(Ctx& c, int use_graph, ttn_status* warn) {
  int budget = 1;
  for (auto& M : c.m) budget = std::max(budget, M.restarts);
  if (use_graph == 2) return top_graph_launch(c, budget);
  const int plan = std::min(budget, std::max(1, c.top_plan));
  ttn_status st = top_graph_launch(c, plan);
  if (st) return st;
  int most = 0;
  bool all = true;
  if ((st = top_complete(c, c.s, plan, &most, &all))) return st;
  c.top_plan = std::max(1, most);
  if (!all) *warn = TTN_WNOCONV;
  return TTN_OK;
}

// ---------------------------------------------------------------------------
// event timing of a handle's launches (ttn_profile, ttn_pos_profile)
// ---------------------------------------------------------------------------
ttn_status profile_switch(Profiler& P, KernelRecorder& krec, int enable) {
  if (enable) {
    if (P.ev.empty()) {
      const size_t cap = 1 << 16;
      P.ev.resize(2 * cap);
      for (auto& e : P.ev) HIPCHK(hipEventCreate(&e));
      P.cls.resize(cap);
      P.flops.resize(cap);
      P.bytes.resize(cap);
    }
    P.used = 0;
    P.dropped = 0;
  }
  P.on = enable != 0;
  krec.P = &P;
  if (enable) kernel_timer() = &krec;
  else if (kernel_timer() == &krec) kernel_timer() = nullptr;
  return TTN_OK;
}

ttn_status profile_collect(Profiler& P, hipStream_t s, ttn_profile_entry* out, int max_entries, int* n_out) {
  HIPCHK(hipStreamSynchronize(s));
  std::vector<ttn_profile_entry> agg(OC_N + KID_N);
  for (int c = 0; c < OC_N + KID_N; ++c) {
    std::memset(&agg[c], 0, sizeof agg[c]);
    if (c < OC_N) std::snprintf(agg[c].name, sizeof agg[c].name, "%s", kOpNames[c]);
    else std::snprintf(agg[c].name, sizeof agg[c].name, "%s", kernel_name(c - OC_N));
  }
  for (size_t i = 0; i < P.used; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]));
    ttn_profile_entry& e = agg[P.cls[i]];
    e.launches += 1;
    e.ms += ms;
    e.flops += P.flops[i];
    e.bytes += P.bytes[i];
  }
  int n = 0;
  for (int c = 0; c < OC_N + KID_N && n < max_entries; ++c)
    if (agg[c].launches) out[n++] = agg[c];
  *n_out = n;
  P.used = 0;
  if (P.dropped) {
    const int d = P.dropped;
    P.dropped = 0;
    return fail(TTN_WPROF, "%d launches were not timed (event pool of %zu full): the record is incomplete", d,
                P.cls.size());
  }
  return TTN_OK;
}

}  // namespace core
}  // namespace ttn

using namespace ttn::core;

// ===========================================================================
// C ABI
// ===========================================================================
struct ttn_ctx {
  Ctx c;
};

namespace ttn {
// for the library's other sources: the stream a handle runs on, and the
// calling thread's error message (what ttn_last_error returns)
hipStream_t handle_stream(ttn_handle h) { return h ? h->c.s : nullptr; }
ttn_status set_error(ttn_status st, const char* msg) { return fail(st, "%s", msg); }
}  // namespace ttn

extern "C" {

const char* ttn_last_error(void) { return g_err.c_str(); }

ttn_status ttn_workspace_bytes(const ttn_config* cfgs, int batch, size_t* bytes) {
  if (!cfgs || batch < 1 || !bytes) return fail(TTN_EINVAL, "bad arguments");
  std::vector<Member> ms(batch);
  for (int i = 0; i < batch; ++i) {
    ttn_status st = setup_member(cfgs[i], ms[i]);
    if (st) return st;
  }
  std::vector<int> order, npad;
  plan_batch(ms, order, npad);
  Arena ar;
  for (int i : order) layout_member(ms[i], ar, npad[i]);
  *bytes = ar.off + 256;
  return TTN_OK;
}

ttn_status ttn_init(const ttn_config* cfgs, int batch, void* workspace, size_t bytes, void* stream, ttn_handle* out) {
  if (!cfgs || batch < 1 || !out) return fail(TTN_EINVAL, "bad arguments");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(TTN_EINVAL, "workspace must be non-null and 256-byte aligned");
  size_t need = 0;
  ttn_status st = ttn_workspace_bytes(cfgs, batch, &need);
  if (st) return st;
  if (bytes < need) return fail(TTN_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, need);
  ttn_ctx* h = new ttn_ctx;
  h->c.s = (hipStream_t)stream;
  h->c.m.resize(batch);
  Arena ar;
  ar.base = (char*)workspace;
  bool any_noconv = false;
  for (int i = 0; i < batch; ++i) {
    setup_member(cfgs[i], h->c.m[i]);
    h->c.m[i].prof = &h->c.prof;
  }
  // members of equal configuration are laid out next to each other, so that
  // they sit at a uniform stride and form one launch group; a group's bond
  // dimensions stay <= 128 (the larger polar solves need the whole GPU).
  // Members of one configuration but different lengths follow one another,
  // deepest first, padded to one layout: a coarse group for the layer part
  // of a sweep.
  {
    Ctx& c = h->c;
    std::vector<int> order, npad;
    plan_batch(c.m, order, npad);
    for (int i : order) layout_member(c.m[i], ar, npad[i]);
    // the next member is one stride after the previous (the whole layout moves)
    auto extends = [&](const Ctx::Group& G, int prev, int next) {
      const Member& A = c.m[prev];
      const Member& B2 = c.m[next];
      const long long st = (long long)((char*)B2.scal - (char*)A.scal);
      if (st <= 0 || (char*)B2.w64[1] - (char*)A.w64[1] != st || (char*)B2.jinfo - (char*)A.jinfo != st ||
          (G.members.size() > 1 && st != G.stride))
        return 0LL;
      return st;
    };
    auto build = [&](auto same, std::vector<Ctx::Group>& out) {
      for (size_t k = 0; k < order.size();) {
        Ctx::Group G;
        G.members.push_back(order[k]);
        size_t j = k + 1;
        if (member_cmax(c.m[order[k]]) <= 128) {
          for (; j < order.size() && same(order[j], order[k]); ++j) {
            const long long st = extends(G, order[j - 1], order[j]);
            if (!st) break;
            G.stride = st;
            G.members.push_back(order[j]);
          }
        }
        out.push_back(G);
        k = j;
      }
    };
    build([&](int x, int y) { return group_key(c.m[x]) == group_key(c.m[y]); }, c.groups);
    if (batch > 1) build([&](int x, int y) { return coarse_key(c.m[x]) == coarse_key(c.m[y]); }, c.coarse);
  }
  if (batch > 1) {
    Ctx& c = h->c;
    hipError_t e = hipStreamCreateWithFlags(&c.grid_s, hipStreamNonBlocking);
    c.member_events.resize(2 * batch, nullptr);
    for (int i = 0; i < 2 * batch && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&c.member_events[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      delete h;
      return fail(TTN_EHIP, "stream/event creation failed: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < batch; ++i) {
      Member& M = c.m[i];
      M.solo = false;
      M.grid_s = c.grid_s;
      M.grid_in = c.member_events[2 * i];
      M.grid_out = c.member_events[2 * i + 1];
    }
  }
  for (int i = 0; i < batch; ++i) {
    bool conv = false;
    st = init_member(h->c.m[i], h->c.s, &conv);
    if (st) {
      delete h;
      return st;
    }
    any_noconv |= !conv;
    h->c.m[i].w0 = nullptr;
    h->c.m[i].v0 = nullptr;
  }
  {  // the first restart plan of graph sweeps: what the initial top updates needed
    int most = 1;
    bool all = true;
    st = top_status(h->c, h->c.s, &most, &all);
    if (st) {
      delete h;
      return st;
    }
    h->c.top_plan = std::max(1, most);
  }
  *out = h;
  return any_noconv ? TTN_WNOCONV : TTN_OK;
}

ttn_status ttn_free(ttn_handle h) {
  delete h;
  return TTN_OK;
}

ttn_status ttn_ascend(ttn_handle h, int tau_from, int tau_to) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  for (auto& M : h->c.m) {
    if (tau_from < 1 || tau_to > M.n - 1 || tau_from > tau_to)
      return fail(TTN_EINVAL, "ascend range [%d, %d] outside [1, %d]", tau_from, tau_to, M.n - 1);
    if (M.ops_upto < tau_from - 1) return fail(TTN_ESTATE, "level %d operators are stale; ascend from a lower layer", tau_from - 1);
  }
  ttn_status st0 = for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status {
    for (int t = tau_from; t <= tau_to; ++t) {
      ttn_status st = stage_ascend(M, t, h->c.s);
      if (st) return st;
    }
    M.ops_upto = std::max(M.ops_upto, tau_to);
    return TTN_OK;
  });
  if (st0) return st0;
  return TTN_OK;
}

ttn_status ttn_descend(ttn_handle h, int tau, int what) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  if (what == TTN_DESCEND_RHO)
    return for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status { return stage_descend_rho(M, h->c.s); });
  if (what != TTN_DESCEND_DRESSED) return fail(TTN_EINVAL, "unknown descend kind %d", what);
  for (auto& M : h->c.m) {
    if (tau < 1 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [1, %d]", tau, M.n - 1);
    if (M.rho_from > tau || M.pc_from > tau + 1)
      return fail(TTN_ESTATE, "descend(DRESSED, %d) needs descend(RHO) after the last change of v or of a layer above %d", tau, tau);
    if (M.ops_upto < tau - 1) return fail(TTN_ESTATE, "level %d operators are stale", tau - 1);
  }
  return for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status { return stage_descend_dressed(M, tau, h->c.s); });
}

ttn_status ttn_env(ttn_handle h, int tau) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  for (auto& M : h->c.m) {
    if (tau < 1 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [1, %d]", tau, M.n - 1);
    if (M.dressed_tau != tau) return fail(TTN_ESTATE, "env(%d) needs descend(DRESSED, %d) first", tau, tau);
  }
  return for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status { return stage_env(M, tau, h->c.s); });
}

ttn_status ttn_update(ttn_handle h, int tau) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  if (tau == TTN_TOP) {
    for (auto& M : h->c.m)
      if (M.ops_upto < M.n - 1) return fail(TTN_ESTATE, "top update needs every layer ascended (ops up to %d of %d)", M.ops_upto, M.n - 1);
    bool all = true;
    ttn_status st = for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status {
      bool conv = false;
      ttn_status r = stage_update_top(M, h->c.s, &conv);
      all &= conv;
      return r;
    });
    if (st) return st;
    return all ? TTN_OK : TTN_WNOCONV;
  }
  for (auto& M : h->c.m) {
    if (tau < 1 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [1, %d]", tau, M.n - 1);
    if (M.env_tau != tau) return fail(TTN_ESTATE, "update(%d) needs env(%d) first", tau, tau);
  }
  return for_groups(h->c, [&](Member& M, const Ctx::Group&) -> ttn_status { return stage_update_layer(M, tau, h->c.s); });
}

ttn_status ttn_energy(ttn_handle h, double* e) {
  if (!h || !e) return fail(TTN_EINVAL, "bad arguments");
  HIPCHK(hipStreamSynchronize(h->c.s));
  bool bad = false, evd_loss = false, noconv = false;
  for (size_t i = 0; i < h->c.m.size(); ++i) {
    double sc[SCAL_N];
    HIPCHK(hipMemcpy(sc, h->c.m[i].scal, sizeof sc, hipMemcpyDeviceToHost));
    int done = 0;
    HIPCHK(hipMemcpy(&done, h->c.m[i].lzint + LZ_DONE, sizeof done, hipMemcpyDeviceToHost));
    noconv |= done == 0;
    e[i] = sc[SCAL_E];
    if (sc[SCAL_ERR] != 0.0) return fail(TTN_EHIP, "a Jacobi eigensolver aborted (grid barrier wait exceeded its bound)");
    if (sc[SCAL_NOCONV] != 0.0)
      return fail(TTN_ENOCONV, "a polar Jacobi solve used all %d of its sweeps without converging", POLAR_JACOBI_SWEEPS);
    // rounding of a x a rotations grows like eps a^(3/2) in the Frobenius norm
    const Member& M = h->c.m[i];
    const double amax = (double)*std::max_element(M.dims.begin(), M.dims.end());
    const double bound = std::max(1e-10, 64.0 * 2.220446049250313e-16 * amax * std::sqrt(amax));
    if (!(sc[SCAL_ORTHO_MAX] <= bound)) (M.evd ? evd_loss : bad) = true;
  }
  if (bad) return fail(TTN_EORTHO, "an updated isometry failed the orthonormality check");
  // the eigenvalue-decomposition update loses orthonormality on purpose where
  // the environment is ill conditioned: a warning, not an error
  if (evd_loss) return fail(TTN_WRANK, "an isometry from the eigenvalue-decomposition update is orthonormal only to "
                                       "the precision of the squared environment");
  if (noconv) return fail(TTN_WNOCONV, "the last top update stopped at its restart budget above its residual target");
  return TTN_OK;
}

ttn_status ttn_sweep(ttn_handle h, int nsweeps, int use_graph) {
  if (!h || nsweeps < 0) return fail(TTN_EINVAL, "bad arguments");
  Ctx& c = h->c;
  ttn_status warn = TTN_OK;
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (auto& M : c.m)
      if (M.ops_upto < M.n - 1) return fail(TTN_ESTATE, "sweep needs every layer ascended");
    ttn_status st;
    if (use_graph && !c.prof.on) {
      if (!c.gexec) {
        // captured on an internal stream (the caller's may be the legacy
        // default stream, which cannot capture); the host bookkeeping of the
        // stages runs once here, as in an eager sweep, and the graph holds
        // only device work, identical every sweep
        if (!c.cap_s) HIPCHK(hipStreamCreateWithFlags(&c.cap_s, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(c.cap_s, hipStreamCaptureModeRelaxed));
        st = sweep_layers_all(c, c.cap_s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c.cap_s, &g);
        if (st) {
          if (g) hipGraphDestroy(g);
          return st;
        }
        HIPCHK(e);
        c.graph = g;
        HIPCHK(hipGraphInstantiate(&c.gexec, c.graph, nullptr, nullptr, 0));
      }
      HIPCHK(hipGraphLaunch(c.gexec, c.s));
      if ((st = top_after_graph(c, use_graph, &warn))) return st;
    } else {
      if ((st = sweep_layers_all(c, c.s))) return st;
      bool all = true;
      if ((st = top_all(c, c.s, &all))) return st;
      if (!all) warn = TTN_WNOCONV;
    }
  }
  return warn;
}

// The layer part of a grouped sweep for the whole batch: launch groups one
// after another on stream s (no host synchronisation: capturable).
ttn_status grouped_layers_all(Ctx& c, int groups, hipStream_t s) {
  for (auto& G : c.groups) {
    GroupScope gs((int)G.members.size(), G.stride);
    ttn_status st = sweep_layers_grouped(c.m[G.members[0]], groups, s);
    if (st) return st;
    sync_group_state(c, G);
  }
  return TTN_OK;
}

ttn_status ttn_sweep_grouped(ttn_handle h, int nsweeps, int groups, int use_graph) {
  if (!h || nsweeps < 0) return fail(TTN_EINVAL, "bad arguments");
  if (groups != 1 && groups != 2) return fail(TTN_EINVAL, "groups = %d, must be 1 or 2", groups);
  Ctx& c = h->c;
  ttn_status warn = TTN_OK;
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (auto& M : c.m)
      if (M.ops_upto < M.n - 1) return fail(TTN_ESTATE, "sweep needs every layer ascended");
    ttn_status st;
    if (use_graph && !c.prof.on) {
      hipGraphExec_t& ge = c.ggexec[groups - 1];
      if (!ge) {
        // captured as for ttn_sweep: the host bookkeeping runs once here, the
        // graph holds only device work, identical every sweep
        if (!c.cap_s) HIPCHK(hipStreamCreateWithFlags(&c.cap_s, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(c.cap_s, hipStreamCaptureModeRelaxed));
        st = grouped_layers_all(c, groups, c.cap_s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c.cap_s, &g);
        if (st) {
          if (g) hipGraphDestroy(g);
          return st;
        }
        HIPCHK(e);
        c.ggraph[groups - 1] = g;
        HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      }
      HIPCHK(hipGraphLaunch(ge, c.s));
      if ((st = top_after_graph(c, use_graph, &warn))) return st;
    } else {
      if ((st = grouped_layers_all(c, groups, c.s))) return st;
      bool all = true;
      if ((st = top_all(c, c.s, &all))) return st;
      if (!all) warn = TTN_WNOCONV;
    }
  }
  return warn;
}

ttn_status ttn_get_tensor(ttn_handle h, int b, int tau, double* host) {
  if (!h || !host || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  Member& M = h->c.m[b];
  size_t e;
  const double* src;
  if (tau == TTN_TOP) {
    e = (size_t)M.dims[M.n - 1] * M.dims[M.n - 1];
    src = M.vtop;
  } else {
    if (tau < 1 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [1, %d]", tau, M.n - 1);
    e = (size_t)M.dims[tau] * M.dims[tau - 1] * M.dims[tau - 1];
    src = M.w64[tau];
  }
  HIPCHK(hipStreamSynchronize(h->c.s));
  HIPCHK(hipMemcpy(host, src, e * 8, hipMemcpyDeviceToHost));
  return TTN_OK;
}

ttn_status ttn_set_tensor(ttn_handle h, int b, int tau, const double* host) {
  if (!h || !host || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  Member& M = h->c.m[b];
  hipStream_t s = h->c.s;
  if (tau == TTN_TOP) {
    size_t e = (size_t)M.dims[M.n - 1] * M.dims[M.n - 1];
    for (size_t i = 0; i < e; ++i) if (!std::isfinite(host[i])) return fail(TTN_ENONFINITE, "v has a non-finite entry");
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(M.vtop, host, e * 8, hipMemcpyHostToDevice));
    if (M.prec != TTN_FP64) HIPCHK(convert_f64_to_f32(M.vtop, (float*)M.vT, e, s));
    M.rho_from = M.pc_from = 1 << 20;
    M.dressed_tau = -1;
    M.env_tau = -1;
    return TTN_OK;
  }
  if (tau < 1 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [1, %d]", tau, M.n - 1);
  size_t e = (size_t)M.dims[tau] * M.dims[tau - 1] * M.dims[tau - 1];
  for (size_t i = 0; i < e; ++i) if (!std::isfinite(host[i])) return fail(TTN_ENONFINITE, "w has a non-finite entry");
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(M.w64[tau], host, e * 8, hipMemcpyHostToDevice));
  ttn_status st = refresh_shadow(M, tau, s);
  if (st) return st;
  M.ops_upto = std::min(M.ops_upto, tau - 1);
  M.rho_from = std::max(M.rho_from, tau);
  M.pc_from = std::max(M.pc_from, tau + 1);
  M.dressed_tau = -1;
  M.env_tau = -1;
  return TTN_OK;
}

ttn_status ttn_get_operator(ttn_handle h, int b, int level, int kind, int k, double* host) {
  if (!h || !host || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  Member& M = h->c.m[b];
  if (level < 0 || level > M.n - 1) return fail(TTN_EINVAL, "level=%d outside [0, %d]", level, M.n - 1);
  if ((kind == TTN_OP_A || kind == TTN_OP_B || kind == TTN_OP_RBAR || kind == TTN_OP_LBAR) && (k < 0 || k >= M.D))
    return fail(TTN_EINVAL, "k=%d outside [0, %d)", k, M.D);
  const size_t q = (size_t)M.dims[level] * M.dims[level];
  const void* src = nullptr;
  size_t e = q;
  switch (kind) {
    case TTN_OP_H: src = M.opH[level]; break;
    case TTN_OP_A: src = M.at(M.opA[level], k * q); break;
    case TTN_OP_B: src = M.at(M.opB[level], k * q); break;
    case TTN_OP_RHO: src = M.rho[level]; break;
    case TTN_OP_RBAR:
      if (M.dressed_tau != level) return fail(TTN_ESTATE, "no dressed RDM at level %d", level);
      src = M.at(M.Rb[M.rb_cur], k * q);
      break;
    case TTN_OP_LBAR:
      if (M.dressed_tau != level) return fail(TTN_ESTATE, "no dressed RDM at level %d", level);
      src = M.at(M.Lb[M.rb_cur], k * q);
      break;
    case TTN_OP_ENV:
      if (M.env_tau != level || level < 1) return fail(TTN_ESTATE, "no environment of layer %d", level);
      e = (size_t)M.dims[level] * M.dims[level - 1] * M.dims[level - 1];
      HIPCHK(hipStreamSynchronize(h->c.s));
      HIPCHK(hipMemcpy(host, M.env64, e * 8, hipMemcpyDeviceToHost));
      return TTN_OK;
    default: return fail(TTN_EINVAL, "unknown operator kind %d", kind);
  }
  HIPCHK(hipStreamSynchronize(h->c.s));
  if (M.esz == 8) {
    HIPCHK(hipMemcpy(host, src, e * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(e);
    HIPCHK(hipMemcpy(tmp.data(), src, e * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < e; ++i) host[i] = tmp[i];
  }
  return TTN_OK;
}

ttn_status ttn_stats(ttn_handle h, int b, ttn_stats_t* out) {
  if (!h || !out || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  Member& M = h->c.m[b];
  HIPCHK(hipStreamSynchronize(h->c.s));
  double sc[SCAL_N];
  HIPCHK(hipMemcpy(sc, M.scal, sizeof sc, hipMemcpyDeviceToHost));
  out->energy = sc[SCAL_E];
  out->lambda = sc[SCAL_LAM];
  out->lanczos_resid = sc[SCAL_RES];
  out->ortho_err_max = sc[SCAL_ORTHO_MAX];
  out->sigma_ratio_min = sc[SCAL_RATIO_MIN];
  out->shift = M.c;
  layer_flops(M, &out->flops_bulk, &out->flops_fp64);
  out->n_levels = M.n;
  int lzi[2] = {0, 0};  // converged flag, restarts run
  HIPCHK(hipMemcpy(lzi, M.lzint + LZ_DONE, sizeof lzi, hipMemcpyDeviceToHost));
  out->lanczos_iters = lzi[1] * (int)std::min<long long>(M.krylov, (long long)M.dims[M.n - 1] * M.dims[M.n - 1]);
  out->e_prev = sc[SCAL_EPREV];
  out->bytes_hbm = M.bytes_layers + M.bytes_top;
  int ji[18];
  HIPCHK(hipMemcpy(ji, M.jinfo, sizeof ji, hipMemcpyDeviceToHost));
  out->jacobi_sweeps[0] = ji[0];
  out->jacobi_sweeps[1] = ji[2];
  out->jacobi_sweeps[2] = ji[4];
  out->jacobi_sweeps[3] = ji[16];
  return TTN_OK;
}

ttn_status ttn_autotune(int mode, int* entries) {
  if (mode < -1 || mode > 2) return fail(TTN_EINVAL, "autotune mode %d outside [-1, 2]", mode);
  if (mode >= 0) gemm_tune_set_mode(mode);
  if (entries) *entries = (int)gemm_tune_entries();
  return TTN_OK;
}

ttn_status ttn_autotune_save(const char* path) {
  if (!path) return fail(TTN_EINVAL, "null path");
  if (!gemm_tune_save(path)) return fail(TTN_EINVAL, "cannot write the launch table to %s", path);
  return TTN_OK;
}

ttn_status ttn_autotune_load(const char* path, int* entries) {
  if (!path) return fail(TTN_EINVAL, "null path");
  const int n = gemm_tune_load(path);
  if (n < 0) return fail(TTN_EINVAL, "cannot read a launch table from %s", path);
  if (entries) *entries = n;
  return TTN_OK;
}

ttn_status ttn_profile(ttn_handle h, int enable) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  return profile_switch(h->c.prof, h->c.krec, enable);
}

ttn_status ttn_profile_read(ttn_handle h, ttn_profile_entry* out, int max_entries, int* n_out) {
  if (!h || !out || !n_out) return fail(TTN_EINVAL, "bad arguments");
  return profile_collect(h->c.prof, h->c.s, out, max_entries, n_out);
}

// The spectrum and entropy of the matrix on the upper bond of a block of
// level tau: the position average (node < 0) or node `node` (its path from
// the top: at level sigma the node above it is node >> (sigma - tau), a left
// child when that index is even), float64 throughout (the master isometries),
// in scratch of the polar update: rho in G / V in turn, rho o w in Y.
ttn_status block_entanglement(Member& M, int tau, long long node, double* p, double* entropy, hipStream_t s) {
  const int n = M.n;
  const bool avg = node < 0;
  const int x = M.dims[n - 1];
  double* cur = M.G;
  double* nxt = M.V;
  const bool top_right = !avg && ((node >> (n - 1 - tau)) & 1);
  if (avg || !top_right) HIPCHK(mm(M, P_F64, M.vtop, false, M.vtop, true, cur, x, avg ? 0.5 : 1.0, 0.0, s));  // v v^T
  if (avg) HIPCHK(mm(M, P_F64, M.vtop, true, M.vtop, false, cur, x, 0.5, 1.0, s));                             // + v^T v
  if (top_right) HIPCHK(mm(M, P_F64, M.vtop, true, M.vtop, false, cur, x, 1.0, 0.0, s));                       // v^T v
  for (int lv = n - 1; lv > tau; --lv) {
    const int a = M.dims[lv], bd = M.dims[lv - 1];
    const bool right = !avg && ((node >> (lv - 1 - tau)) & 1);
    HIPCHK(left_mul(M, P_F64, cur, M.w64[lv], M.Y, a, bd, 1.0, 0.0, s));
    if (avg || !right) HIPCHK(close_l(M, P_F64, M.w64[lv], M.Y, nxt, a, bd, avg ? 0.5 : 1.0, 0.0, s));
    if (avg) HIPCHK(close_r(M, P_F64, M.w64[lv], M.Y, nxt, a, bd, 0.5, 1.0, s));
    if (right) HIPCHK(close_r(M, P_F64, M.w64[lv], M.Y, nxt, a, bd, 1.0, 0.0, s));
    std::swap(cur, nxt);
  }
  const int m = M.dims[tau];
  HIPCHK(symmetrize_f64(cur, m, 1.0, s));
  HIPCHK(jacobi_eig_f64(cur, nxt, m, 80, std::max(1e-15, 2.2e-16 * m), M.jinfo + 20, m > 64 ? M.jscratch : nullptr, s));
  HIPCHK(spectrum_sorted(cur, m, M.Y, M.scal + SCAL_TMP2, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(p, M.Y, (size_t)m * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(entropy, M.scal + SCAL_TMP2, sizeof(double), hipMemcpyDeviceToHost));
  int info[2] = {0, 0};
  HIPCHK(hipMemcpy(info, M.jinfo + 20, sizeof info, hipMemcpyDeviceToHost));
  if (info[0] < 0) return fail(TTN_EHIP, "the Jacobi eigensolver aborted (grid barrier wait exceeded its bound)");
  // the scratch held the polar update's temporaries only; the environment
  // (kept in its own buffers) stays valid
  return TTN_OK;
}

ttn_status ttn_entanglement(ttn_handle h, int b, int tau, int which, double* p, double* entropy) {
  if (!h || !p || !entropy || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  if (which != TTN_ENT_AVERAGE && which != TTN_ENT_LEFTMOST) return fail(TTN_EINVAL, "which=%d unknown", which);
  Member& M = h->c.m[b];
  if (tau < 0 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [0, %d]", tau, M.n - 1);
  GroupScope one(1, 0);
  return block_entanglement(M, tau, which == TTN_ENT_AVERAGE ? -1 : 0, p, entropy, h->c.s);
}

ttn_status ttn_entanglement_node(ttn_handle h, int b, int tau, long long node, double* p, double* entropy) {
  if (!h || !p || !entropy || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  Member& M = h->c.m[b];
  if (tau < 0 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [0, %d]", tau, M.n - 1);
  if (node < 0 || node >= (long long)(M.L >> tau)) return fail(TTN_EINVAL, "node=%lld outside [0, %d)", node, M.L >> tau);
  GroupScope one(1, 0);
  return block_entanglement(M, tau, node, p, entropy, h->c.s);
}

ttn_status ttn_positions_bytes(ttn_handle h, int b, size_t* bytes) {
  if (!h || !bytes || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  *bytes = (size_t)pos_layout(h->c.m[b]).min_total * 8;
  return TTN_OK;
}

ttn_status ttn_positions_offset(ttn_handle h, int b, int tau, size_t* offset) {
  if (!h || !offset || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  const Member& M = h->c.m[b];
  if (tau < 0 || tau > M.n - 1) return fail(TTN_EINVAL, "tau=%d outside [0, %d]", tau, M.n - 1);
  *offset = (size_t)pos_layout(M).rho[tau] * 8;
  return TTN_OK;
}

ttn_status ttn_local_energies(ttn_handle h, int b, void* work, size_t bytes, double* site, double* bond) {
  if (!h || !work || !site || !bond || b < 0 || b >= (int)h->c.m.size()) return fail(TTN_EINVAL, "bad arguments");
  if ((uintptr_t)work % 256) return fail(TTN_EINVAL, "work is not 256-byte aligned");
  Member& M = h->c.m[b];
  const PosLayout P = pos_layout(M);
  if ((long long)(bytes / 8) < P.min_total)
    return fail(TTN_ENOMEM, "work of %zu bytes is smaller than %lld", bytes, P.min_total * 8);
  hipStream_t s = h->c.s;
  GroupScope one(1, 0);
  ttn_status st = local_energies(M, (double*)work, (long long)(bytes / 8), P, s);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(site, (double*)work + P.site, (size_t)M.L * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bond, (double*)work + P.bond, (size_t)M.L * 8, hipMemcpyDeviceToHost));
  return TTN_OK;
}

int ttn_bond_dim(ttn_handle h, int b, int tau) {
  if (!h || b < 0 || b >= (int)h->c.m.size()) return -1;
  Member& M = h->c.m[b];
  if (tau < 0 || tau >= M.n) return -1;
  return M.dims[tau];
}

}  // extern "C"
