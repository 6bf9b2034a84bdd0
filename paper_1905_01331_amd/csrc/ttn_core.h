// Internal declarations shared by the host sources of libttn: the member
// state of a network (its workspace layout, solver scratch and top-solver
// buffers), the product launchers over that layout, the polar update and the
// top eigensolver.  ttn_api.cpp defines them; the position-resolved network
// (ttn_positional.cpp) reuses the launchers, the polar update and the top
// solver.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "ttn.h"
#include "common.h"

namespace ttn {
namespace core {

// records the calling thread's error message (ttn_last_error) and returns st
ttn_status fail(ttn_status st, const char* fmt, ...);
// largest eigenvalue of a small symmetric matrix (n x n, row-major), host:
// cyclic Jacobi (n <= 64) or restarted Lanczos
double host_lambda_max(std::vector<double> a, int n);
double host_lambda_max_lanczos(const std::vector<double>& a, int n);

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(TTN_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : reinterpret_cast<T*>(off + 256);
    off += n * sizeof(T);
    return p;
  }
  void* take_bytes(size_t n) { return take<char>(n); }
};

constexpr int SCAL_LAM = 0, SCAL_E = 1, SCAL_RES = 2, SCAL_ORTHO = 3, SCAL_ORTHO_MAX = 4, SCAL_RATIO = 5,
              SCAL_RATIO_MIN = 6, SCAL_TMP0 = 7, SCAL_TMP1 = 8, SCAL_TMP2 = 9, SCAL_THETA = 10,
              SCAL_ERR = 11,  // 1.0 once a Jacobi solve reported an abort
              SCAL_SHIFT = 12,  // the shift c (per member, read by the energy kernel)
              SCAL_EPREV = 13,  // the energy before the last top update
              SCAL_NOCONV = 14,  // 1.0 once a polar Jacobi solve used all its sweeps
              SCAL_N = 16;
// Gram refreshes of the polar update: two always, a third when the second
// Jacobi needed more than POLAR_THIRD_IF sweeps (its start was not nearly
// diagonal, so the rotated rows may not yet be orthogonal to working accuracy)
constexpr int LZ_DONE = 8;  // lzint slot of the top solver's per-member convergence flag
constexpr int POLAR_REFRESH = 2;
constexpr int POLAR_JACOBI_SWEEPS = 60;  // sweep limit of a polar Jacobi solve
// largest Gram order solved in one work-group (the cyclic solver's G and U,
// 2 * 96^2 doubles, and a round's rotation tables fit the 160 KB of LDS, as
// do the blocked one-work-group solver's padded G and sub-problems); above it
// the blocked grid solver
constexpr int POLAR_ONE_WG_MAX = 96;
constexpr int POLAR_THIRD_IF = 3;
constexpr double POLAR_REG = 1e-30;   // tie-breaker toward the current isometry in null directions

// Per-handle event timer of contraction classes (enabled by ttn_profile).
enum OpClass { OC_APPLY_R = 0, OC_APPLY_L, OC_CLOSE, OC_LEFT_MUL, OC_CLOSE_L, OC_CLOSE_R, OC_TOP_MM,
               OC_POLAR_GEMM, OC_JACOBI, OC_LANCZOS_GEMM, OC_N };
inline const char* const kOpNames[OC_N] = {"apply_r", "apply_l", "close", "left_mul", "close_l", "close_r",
                                    "top_mm", "polar_gemm", "jacobi", "lanczos_gemm"};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;      // pairs
  std::vector<int> cls;
  std::vector<double> flops, bytes;
  size_t used = 0;
  int dropped = 0;
  ~Profiler() {
    for (auto e : ev) hipEventDestroy(e);
  }
  bool begin(int c, double f, double b, hipStream_t s, size_t* slot) {
    if (!on) return false;
    if (used >= cls.size()) { ++dropped; return false; }
    *slot = used++;
    cls[*slot] = c;
    flops[*slot] = f;
    bytes[*slot] = b;
    return hipEventRecord(ev[2 * *slot], s) == hipSuccess;
  }
  void end(size_t slot, hipStream_t s) { (void)hipEventRecord(ev[2 * slot + 1], s); }
};

// Per-kernel records of the product kernels go into the same event pool,
// under class ids OC_N + kernel id.
struct KernelRecorder : KernelTimer {
  Profiler* P = nullptr;
  bool begin(int kid, double f, double b, hipStream_t s, size_t* slot) override {
    return P && P->begin(OC_N + kid, f, b, s, slot);
  }
  void end(size_t slot, hipStream_t s) override { P->end(slot, s); }
};

// Complex products over split planes: inside a CplxScope every product that
// run() issues is complex, each operand's imaginary plane lying `delta` bytes
// after its real plane (C = A B becomes four real products: Re C = Re A Re B
// - Im A Im B, Im C = Re A Im B + Im A Re B); inside a BraScope as well, the
// first operand is conjugated (the bra copy of a contraction).  delta = 0:
// real products.
// A product that asks for its block upper triangle (GemmDesc.tri: a
// symmetric real result, antisymmetric for the anti bits) keeps it in complex
// arithmetic when tri_ok: the caller's results are then Hermitian (anti bit
// clear: real part symmetric, imaginary part antisymmetric) or anti-Hermitian
// (the reverse), and each plane is computed on its triangle with its parity.
struct CplxCtx {
  long long delta = 0;
  bool conj_a = false;
  bool tri_ok = false;
};
CplxCtx& cplx();  // the calling thread's
struct CplxScope {
  CplxCtx saved;
  CplxScope(long long delta, bool tri_ok) : saved(cplx()) {
    cplx().delta = delta;
    cplx().conj_a = false;
    cplx().tri_ok = tri_ok;
  }
  ~CplxScope() { cplx() = saved; }
};
struct BraScope {
  bool saved;
  BraScope() : saved(cplx().conj_a) { cplx().conj_a = true; }
  ~BraScope() { cplx().conj_a = saved; }
};

struct Member {
  Profiler* prof = nullptr;
  // configuration
  int L = 0, n = 0, d = 0, D = 0, chi = 0, ly = 1, prec = TTN_FP64;
  double c = 0.0;
  unsigned long long seed = 0;
  std::vector<int> dims;
  std::vector<double> h1, A, B;
  std::vector<int> anti;  // product term k is antisymmetric
  const double* const* w0 = nullptr;
  const double* v0 = nullptr;
  int krylov = 24, restarts = 8;
  double ltol = 1e-12;
  bool gauge_fix = true;
  bool evd = false;  // one Gram refresh only (the eigenvalue-decomposition variant)
  // batch members run side by side: a Jacobi solve that needs its grid
  // co-resident (the persistent blocked solver) goes through one shared
  // stream, one at a time, and the smaller ones use the one-work-group solver
  bool solo = true;
  hipStream_t grid_s = nullptr;
  hipEvent_t grid_in = nullptr, grid_out = nullptr;
  // device
  size_t esz = 8;  // bulk element size
  std::vector<double*> w64;
  std::vector<double*> Qw;      // per layer: left rotation of the last polar update (warm start)
  std::vector<char> qw_valid;
  std::vector<void*> wT, opH, opA, opB, rho, Pc, At, Bt;
  void *Rb[2] = {nullptr, nullptr}, *Lb[2] = {nullptr, nullptr};
  int rb_cur = 0;
  void *Sw = nullptr, *S2 = nullptr, *S3 = nullptr, *envT = nullptr;
  void *Estage = nullptr, *Xst = nullptr;  // environment staging: tensors and their left factors
  double *env64 = nullptr, *Y = nullptr, *Y2 = nullptr, *G = nullptr, *V = nullptr, *Q = nullptr, *Q2 = nullptr,
         *nrm = nullptr;
  int* jinfo = nullptr;
  int* skip3 = nullptr;  // device flag: skip the extra polar refresh
  void* jscratch = nullptr;
  double* vtop = nullptr;
  void* vT = nullptr;
  void* tmpT = nullptr;  // D chi^2 bulk scratch for the top dressing
  double *hop64 = nullptr, *Aop64 = nullptr, *Bop64 = nullptr, *lzStage = nullptr;
  // top problem with different operators on its two sites (position-resolved
  // network): float64 [h, A_1..A_D, B_1..B_D] of the right site, and the
  // symmetrised copy the matvec reads; null: both sites carry hop64's
  const double* topR = nullptr;
  double* hopR64 = nullptr;
  // top problem of another form (complex tensors: a real vector of top_len
  // doubles and its own product y -> H y); null: the real top of dims[n-1]
  long long top_len = 0;
  hipError_t (*matvec)(Member& M, const double* y, double* out, hipStream_t s) = nullptr;
  void* owner = nullptr;
  double *lzQ = nullptr, *lzW = nullptr, *lzT = nullptr, *lzHv = nullptr, *lzR = nullptr;
  double *alpha = nullptr, *beta = nullptr, *Tm = nullptr, *Vm = nullptr, *ycoef = nullptr, *coef = nullptr,
         *lzpart = nullptr, *lznrm = nullptr;
  int* lzint = nullptr;
  double* scal = nullptr;
  double* part = nullptr;
  void* splitk = nullptr;
  size_t splitk_bytes = 0;
  // state of the sweep: rho^(l) is current for l >= rho_from, the cached
  // rho^(l) o w_l for l >= pc_from
  int rho_from = 1 << 20, pc_from = 1 << 20;
  int dressed_tau = -1, env_tau = -1, ops_upto = 0;
  bool ortho_fail = false;
  // algorithmic bytes of the products (operands read once, result written
  // once) of the last layer pass and of the last top update, counted while
  // the launches are issued (a graph replay repeats its capture's count)
  mutable double bytes_acc = 0.0;
  mutable bool counting = false;
  // every member of a launch group counted (flops and product bytes of the
  // position-resolved network's sweep)
  mutable double flops_acc = 0.0, traffic_acc = 0.0;
  double bytes_layers = 0.0, bytes_top = 0.0;

  Prec gp() const { return prec == TTN_FP64 ? P_F64 : (prec == TTN_FP32 ? P_F32 : P_BF16X3); }
  // bit k set: product term k is antisymmetric (its ascended operators are too)
  unsigned long long anti_bits() const {
    unsigned long long m = 0;
    for (size_t k = 0; k < anti.size() && k < 64; ++k)
      if (anti[k]) m |= 1ull << k;
    return m;
  }
  size_t el(size_t n_) const { return n_ * esz; }
  void* at(void* base, size_t elems) const { return (char*)base + elems * esz; }
  const void* at(const void* base, size_t elems) const { return (const char*)base + elems * esz; }
};

// Counts the product bytes of what runs in its scope into `into`.
struct ByteCount {
  Member& M;
  double& into;
  ByteCount(Member& m, double& dst) : M(m), into(dst) { M.bytes_acc = 0.0; M.counting = true; }
  ~ByteCount() { M.counting = false; into = M.bytes_acc; }
};

// ---------------------------------------------------------------------------
// shared entry points (defined in ttn_api.cpp)
// ---------------------------------------------------------------------------
// event timing of a handle's launches: switch on (allocating the event pool
// once) or off; collect per-class and per-kernel totals and reset
ttn_status profile_switch(Profiler& P, KernelRecorder& krec, int enable);
ttn_status profile_collect(Profiler& P, hipStream_t s, ttn_profile_entry* out, int max_entries, int* n_out);
ttn_status setup_member(const ttn_config& c, Member& M);
void layout_member(Member& M, Arena& ar, int n_pad = 0);
// one product in the member's arithmetic, timed and byte-counted
hipError_t run(const Member& M, Prec p, const GemmDesc& g, hipStream_t s, int cls = OC_POLAR_GEMM);
GemmDesc desc0();
// building blocks over nk product terms (see their definitions)
hipError_t apply_r_k(const Member& M, Prec p, const void* O, long long sO, const void* X, long long sX, void* Y,
                     long long sY, int a, int b, double beta, int nk, hipStream_t s);
hipError_t apply_l_k(const Member& M, Prec p, const void* O, long long sO, const void* X, long long sX, void* Y,
                     long long sY, int a, int b, double beta, int nk, hipStream_t s);
hipError_t close_aa_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                      long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                      unsigned long long anti);
hipError_t left_mul_k(const Member& M, Prec p, const void* X, long long sX, const void* P, long long sP, void* Y,
                      long long sY, int a, int b, double alpha, double beta, int nk, hipStream_t s);
hipError_t close_r_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                     long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                     unsigned long long anti);
hipError_t close_l_k(const Member& M, Prec p, const void* P, long long sP, const void* Qm, long long sQ, void* C,
                     long long sC, int a, int b, double alpha, double beta, int nk, hipStream_t s,
                     unsigned long long anti);
hipError_t mm_k(const Member& M, Prec p, const void* Am, long long sA, bool ta, const void* Bm, long long sB, bool tb,
                void* C, long long sC, int x, double alpha, double beta, int nk, hipStream_t s);
hipError_t mm(const Member& M, Prec p, const void* Am, bool ta, const void* Bm, bool tb, void* C, int x, double alpha,
              double beta, hipStream_t s);
// the stages of the uniform sweep over the member's arrays (the layer's S w
// into M.Sw; operators of level tau from level tau-1; rho of every level;
// the two-site matrices at the top, one level down, and for layer tau; the
// environment of layer tau into M.envT)
hipError_t s_apply(const Member& M, int lvl_below, const void* w, int a, int b, hipStream_t s);
ttn_status stage_ascend(Member& M, int tau, hipStream_t s);
ttn_status stage_descend_rho(Member& M, hipStream_t s);
ttn_status dressed_top(Member& M, const void* At, const void* Bt, hipStream_t s);
ttn_status dressed_down(Member& M, int sg, const void* Alow, const void* Blow, hipStream_t s);
ttn_status stage_descend_dressed(Member& M, int tau, hipStream_t s);
ttn_status stage_env(Member& M, int tau, hipStream_t s);
// a copy of an array, and of its imaginary plane inside a CplxScope
hipError_t copy_planes(void* dst, const void* src, size_t bytes, hipStream_t s);
// out = sign * polar(src), src a x K float64 (M.Y, M.Y2, M.G, M.V, M.Q,
// M.Q2, M.nrm, M.jinfo, M.skip3, M.scal as scratch)
ttn_status polar_core(Member& M, const double* src, int a, long long K, double sign, double* out, hipStream_t s,
                      double* warm = nullptr, bool warm_valid = false, double** p_out = nullptr,
                      const double* fill_from = nullptr, double* fill_tmp = nullptr);
// the top update: prepare (float64 operators, symmetrised), Lanczos restarts,
// finish (sign of v, energy)
hipError_t top_matvec(Member& M, const double* y, double* out, hipStream_t s, bool staged = false);
ttn_status top_prepare(Member& M, hipStream_t s);
ttn_status top_restarts(Member& M, hipStream_t s, int count, bool sync, bool* converged);
ttn_status top_finish(Member& M, hipStream_t s, bool keep_prev = false);

}  // namespace core
}  // namespace ttn
