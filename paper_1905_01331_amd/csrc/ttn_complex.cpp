// Uniform binary TTN with complex tensors, for Hamiltonians with complex
// matrix elements: the method of Secs. II.C and III with every transpose a
// conjugate transpose.  Float64 complex arithmetic throughout.
//
// Every complex array lives in two planes of one workspace region: the real
// plane at the array's address, the imaginary plane `delta` bytes after it
// (delta = the size of the region).  So a product of complex arrays is four
// real products on the same MFMA kernels, with the same strides and batch
// layout as the real network's (run() does the expansion inside a
// CplxScope), and the sweep's stages are the real network's stage
// functions: the closes contract their first operand as the bra copy, which
// a complex product conjugates.  The layer update factors the real
// embedding [[Re Env, -Im Env], [Im Env, Re Env]] of the environment with
// the real polar update (the embedding maps products and conjugate
// transposes to products and transposes, so the polar factor of the
// embedding is the embedding of the polar factor where Env has full rank);
// the top tensor is the lowest eigenvector of the real embedding of the
// Hermitian top Hamiltonian (each level doubled; any vector of the lowest
// pair is a complex ground vector), found by the real Lanczos solver with a
// complex product y -> H y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "ttn.h"
#include "common.h"
#include "complex.h"
#include "lanczos.h"
#include "ttn_core.h"

using namespace ttn;
using namespace ttn::core;

struct ttn_cplx_ctx {
  Member M;  // the stage functions' arrays (plane-paired), top solver, polar scratch
  hipStream_t s = nullptr;
  int L = 0, n = 0, d = 0, D = 0;
  std::vector<int> dims;
  long long delta = 0;  // bytes from a complex array's real plane to its imaginary plane
  // plane-paired: per level [h, A_1..A_D, B_1..B_D]; the symmetrised top
  // operators
  std::vector<double*> ops;
  double* tops = nullptr;
  // real: the embeddings [[Re O, -Im O], [Im O, Re O]] (2x x 2x) of the top
  // operators, and the top product's staging (1 + 2D blocks of [Re; Im])
  double *lhat = nullptr, *tstage = nullptr;
  // real: embedding of an environment (also the polar result), of the
  // current isometry, the polar update's fill scratch; host transfers
  double *emb = nullptr, *emb_w = nullptr, *emb_t = nullptr, *io = nullptr;
  std::vector<int> herm;  // per product term: 1 A_k, B_k Hermitian, -1 anti-Hermitian, 0 neither
  // every term Hermitian or anti-Hermitian: the ascended operators, the
  // descended matrices and the two-site matrices are too, and their products
  // run on the block upper triangle (M.anti: the anti-Hermitian terms)
  bool tri_ok = false;
  int env_tau = -1;
  long long repairs = 0;  // updates whose result was replaced by its nearest isometry
  bool top_conv = true;
  double last_flops = 0.0, last_bytes = 0.0;
  Profiler prof;
  KernelRecorder krec;
  ~ttn_cplx_ctx() {
    if (kernel_timer() == &krec) kernel_timer() = nullptr;
  }
  template <class T>
  T* im(T* p) const { return (T*)((char*)p + delta); }
  long long x2(int t) const { return (long long)dims[t] * dims[t]; }
  long long cube(int t) const { return (long long)dims[t] * dims[t - 1] * dims[t - 1]; }
};

namespace {

using Cx = ttn_cplx_ctx;
using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// configuration (host)
// ---------------------------------------------------------------------------
bool hermitian(const cd* m, int d, double sign) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const cd x = m[i * d + j], y = sign * std::conj(m[j * d + i]);
      if (std::abs(x - y) > 1e-12 * (1.0 + std::abs(x))) return false;
    }
  return true;
}

ttn_status cx_member(const ttn_cplx_config* cfg, Member& M, std::vector<int>* herm) {
  if (!cfg) return fail(TTN_EINVAL, "bad arguments");
  const ttn_cplx_config& c = *cfg;
  if (c.L < 4 || (c.L & (c.L - 1))) return fail(TTN_EINVAL, "L=%d must be a power of two >= 4", c.L);
  if (c.d < 2 || c.d > 64) return fail(TTN_EINVAL, "d=%d out of range [2, 64]", c.d);
  if (c.chi < 1 || c.chi > 1024) return fail(TTN_EINVAL, "chi=%d out of range [1, 1024]", c.chi);
  if (c.D < 0 || c.D > 64) return fail(TTN_EINVAL, "D=%d out of range [0, 64]", c.D);
  if (!c.h1 || (c.D > 0 && (!c.A || !c.B))) return fail(TTN_EINVAL, "missing Hamiltonian arrays");
  if (c.ly < 1) return fail(TTN_EINVAL, "ly=%d must be >= 1", c.ly);
  if (!c.w0) return fail(TTN_EINVAL, "w0 (the isometry of every layer) is required");
  M.L = c.L;
  M.n = 0;
  while ((1 << M.n) < c.L) ++M.n;
  M.d = c.d;
  M.D = c.D;
  M.chi = c.chi;
  M.ly = c.ly;
  M.prec = TTN_FP64;
  M.seed = c.seed;
  M.krylov = c.krylov > 0 ? c.krylov : 24;
  M.restarts = c.restarts > 0 ? c.restarts : 8;
  M.ltol = c.lanczos_tol > 0 ? c.lanczos_tol : 1e-12;
  if (M.krylov > 63) return fail(TTN_EINVAL, "krylov=%d > 63", M.krylov);
  M.gauge_fix = false;
  M.evd = false;
  M.solo = true;
  M.esz = 8;
  const int d = c.d, D = c.D, dd = d * d;
  const cd* h1 = reinterpret_cast<const cd*>(c.h1);
  const cd* A = reinterpret_cast<const cd*>(c.A);
  const cd* B = reinterpret_cast<const cd*>(c.B);
  for (int i = 0; i < 2 * dd; ++i)
    if (!std::isfinite(c.h1[i])) return fail(TTN_ENONFINITE, "h1 has a non-finite entry");
  for (long long i = 0; i < 2LL * D * dd; ++i)
    if (!std::isfinite(c.A[i]) || !std::isfinite(c.B[i])) return fail(TTN_ENONFINITE, "A or B has a non-finite entry");
  if (!hermitian(h1, d, 1.0)) return fail(TTN_EINVAL, "h1 is not Hermitian");
  std::vector<int> hm;
  for (int k = 0; k < D; ++k) {
    const cd* a = A + (size_t)k * dd;
    const cd* b = B + (size_t)k * dd;
    hm.push_back(hermitian(a, d, 1.0) && hermitian(b, d, 1.0) ? 1
                 : hermitian(a, d, -1.0) && hermitian(b, d, -1.0) ? -1 : 0);
  }
  // bond term 1/2 (h1 x I + I x h1) + sum_k A_k x B_k (dd x dd)
  std::vector<cd> bt((size_t)dd * dd, cd(0.0, 0.0));
  for (int i1 = 0; i1 < d; ++i1)
    for (int i2 = 0; i2 < d; ++i2)
      for (int j1 = 0; j1 < d; ++j1)
        for (int j2 = 0; j2 < d; ++j2) {
          cd v(0.0, 0.0);
          if (i2 == j2) v += 0.5 * h1[i1 * d + j1];
          if (i1 == j1) v += 0.5 * h1[i2 * d + j2];
          for (int k = 0; k < D; ++k) v += A[(size_t)k * dd + i1 * d + j1] * B[(size_t)k * dd + i2 * d + j2];
          bt[(size_t)(i1 * d + i2) * dd + (j1 * d + j2)] = v;
        }
  if (!hermitian(bt.data(), dd, 1.0)) return fail(TTN_EINVAL, "the bond term is not Hermitian");
  if (std::isnan(c.shift)) {
    // largest eigenvalue of the Hermitian bond term: that of its real
    // embedding [[Re, -Im], [Im, Re]] (each eigenvalue twice)
    const int e = 2 * dd;
    std::vector<double> r((size_t)e * e);
    for (int i = 0; i < dd; ++i)
      for (int j = 0; j < dd; ++j) {
        const cd x = bt[(size_t)i * dd + j];
        r[(size_t)i * e + j] = x.real();
        r[(size_t)i * e + dd + j] = -x.imag();
        r[(size_t)(dd + i) * e + j] = x.imag();
        r[(size_t)(dd + i) * e + dd + j] = x.real();
      }
    M.c = e <= 64 ? host_lambda_max(r, e) : host_lambda_max_lanczos(r, e);
  } else {
    if (!std::isfinite(c.shift)) return fail(TTN_ENONFINITE, "shift is not finite");
    M.c = c.shift;
  }
  M.dims.resize(M.n);
  M.dims[0] = d;
  for (int t = 1; t < M.n; ++t) M.dims[t] = (int)std::min<long long>((long long)M.dims[t - 1] * M.dims[t - 1], c.chi);
  for (int t = 1; t < M.n; ++t)
    if (!c.w0[t - 1]) return fail(TTN_EINVAL, "w0[%d] is NULL", t - 1);
  if (herm) *herm = hm;
  return TTN_OK;
}

// ---------------------------------------------------------------------------
// workspace: the plane region (twice: real and imaginary planes), then the
// real arrays.  Returns the bytes needed; with P, sets every pointer.
// ---------------------------------------------------------------------------
size_t cx_layout(Member& M, char* base, Cx* P) {
  const int n = M.n, D = M.D;
  const size_t nk = (size_t)std::max(D, 1);
  int cmax = 0;
  size_t cube = 0;
  for (int t = 0; t < n; ++t) cmax = std::max(cmax, M.dims[t]);
  for (int t = 1; t < n; ++t) cube = std::max(cube, (size_t)M.dims[t] * M.dims[t - 1] * M.dims[t - 1]);
  const int x = M.dims[n - 1];
  const size_t xx = (size_t)x * x, c2 = (size_t)cmax * cmax;
  Arena pl;
  pl.base = base;
  M.w64.assign(n, nullptr);
  M.wT.assign(n, nullptr);
  M.opH.assign(n, nullptr);
  M.opA.assign(n, nullptr);
  M.opB.assign(n, nullptr);
  M.rho.assign(n, nullptr);
  M.Pc.assign(n, nullptr);
  M.At.assign(n, nullptr);
  M.Bt.assign(n, nullptr);
  std::vector<double*> ops(n, nullptr);
  for (int t = 0; t < n; ++t) {
    const size_t q = (size_t)M.dims[t] * M.dims[t];
    ops[t] = pl.take<double>((1 + 2 * nk) * q);
    M.opH[t] = ops[t];
    M.opA[t] = ops[t] + q;
    M.opB[t] = ops[t] + (1 + nk) * q;
    M.rho[t] = pl.take<double>(q);
    M.At[t] = pl.take<double>(nk * q);
    M.Bt[t] = pl.take<double>(nk * q);
    if (t >= 1) {
      M.w64[t] = pl.take<double>((size_t)M.dims[t] * M.dims[t - 1] * M.dims[t - 1]);
      M.wT[t] = M.w64[t];
    }
    if (t >= 2) M.Pc[t] = pl.take<double>((size_t)M.dims[t] * M.dims[t - 1] * M.dims[t - 1]);
  }
  for (int i = 0; i < 2; ++i) {
    M.Rb[i] = pl.take<double>(nk * c2);
    M.Lb[i] = pl.take<double>(nk * c2);
  }
  M.Estage = pl.take<double>((1 + 2 * nk) * cube);
  M.Sw = M.Estage;
  M.S2 = pl.take<double>(nk * cube);
  M.S3 = pl.take<double>(nk * cube);
  M.Xst = pl.take<double>((1 + 2 * nk) * c2);
  M.env64 = pl.take<double>(cube);
  M.envT = M.env64;
  M.vtop = nullptr;
  M.vT = pl.take<double>(xx);
  M.tmpT = pl.take<double>(nk * xx);
  double* tops = pl.take<double>((1 + 2 * nk) * xx);
  const size_t plane = (pl.off + 255) & ~size_t(255);
  // real arrays after both planes
  Arena ar;
  ar.base = base ? base + 2 * plane : nullptr;
  const size_t big = 4 * cube;  // (2a) x (2 b^2)
  const int a2 = 2 * cmax;
  M.Y = ar.take<double>(big);
  M.Y2 = ar.take<double>(big);
  M.G = ar.take<double>((size_t)a2 * a2);
  M.V = ar.take<double>((size_t)a2 * a2);
  M.Q = ar.take<double>((size_t)a2 * a2);
  M.Q2 = ar.take<double>((size_t)a2 * a2);
  M.nrm = ar.take<double>(a2);
  M.jinfo = ar.take<int>(64);
  M.skip3 = ar.take<int>(64);
  M.jscratch = ar.take_bytes(jacobi_blocked_scratch_bytes(std::max(a2, M.krylov)));
  M.top_len = 2 * (long long)xx;
  const size_t tl = (size_t)M.top_len;
  M.vtop = ar.take<double>(tl);
  const int m = (int)std::min<long long>(M.krylov, M.top_len);
  M.lzStage = nullptr;
  M.lzQ = ar.take<double>((size_t)(m + 1) * tl);
  M.lzW = ar.take<double>(tl);
  M.lzT = ar.take<double>(tl);
  M.lzHv = ar.take<double>(tl);
  M.lzR = ar.take<double>(tl);
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
  M.splitk_bytes = 64 * std::max<size_t>((size_t)a2 * a2, xx) * 8;
  M.splitk = ar.take_bytes(M.splitk_bytes);
  double* lhat = ar.take<double>((1 + 2 * nk) * 4 * xx);
  double* tstage = ar.take<double>((1 + 2 * nk) * 2 * xx);
  double* emb = ar.take<double>(big);
  double* emb_w = ar.take<double>(big);
  double* emb_t = ar.take<double>(big);
  const size_t io_len = 2 * std::max({cube, (1 + 2 * nk) * c2, xx, (size_t)(1 + 2 * nk) * M.d * M.d});
  double* io = ar.take<double>(io_len);
  if (P) {
    P->delta = (long long)plane;
    P->ops = ops;
    P->tops = tops;
    P->lhat = lhat;
    P->tstage = tstage;
    P->emb = emb;
    P->emb_w = emb_w;
    P->emb_t = emb_t;
    P->io = io;
  }
  return 2 * plane + ar.off + 256;
}

// ---------------------------------------------------------------------------
// host transfers of complex arrays (interleaved on the host)
// ---------------------------------------------------------------------------
ttn_status to_planes(Cx& P, const double* host, double* dev_re, size_t count) {
  HIPCHK(hipMemcpyAsync(P.io, host, 2 * count * 8, hipMemcpyHostToDevice, P.s));
  HIPCHK(deinterleave_f64(P.io, dev_re, P.im(dev_re), count, P.s));
  return TTN_OK;
}

ttn_status from_planes(Cx& P, const double* dev_re, double* host, size_t count) {
  HIPCHK(interleave_f64(dev_re, P.im(dev_re), P.io, count, P.s));
  HIPCHK(hipMemcpyAsync(host, P.io, 2 * count * 8, hipMemcpyDeviceToHost, P.s));
  HIPCHK(hipStreamSynchronize(P.s));
  return TTN_OK;
}

// ---------------------------------------------------------------------------
// the top problem: y (real vector [Re y; Im y], two x x x planes) -> H_top y
// ---------------------------------------------------------------------------
// H_top y = h y + y h^T + sum_k (A_k y B_k^T + B_k y A_k^T) with complex
// operators, as real products against their embeddings
// Lhat = [[Re O, -Im O], [Im O, Re O]]: a left product O S is Lhat [Re S; Im S]
// (the planar layout of S read as a 2x x x matrix), a right product y O^T is
// [Re y | Im y] Lhat^T (y read as x x 2x through a two-level contraction
// index; each output plane one batch entry).  Staging as the real network's:
// stage = [y, y B_1^T .. y B_D^T, y A_1^T .. y A_D^T], then
// out = sum_j Lhat_j stage_j, then out += y h^T: five launches.
hipError_t cx_matvec(Member& M, const double* y, double* out, hipStream_t s) {
  Cx& P = *static_cast<Cx*>(M.owner);
  const int x = P.dims[P.n - 1], D = P.D;
  const long long xx = (long long)x * x, b2 = 2 * xx, b4 = 4 * xx;
  hipError_t e;
  if ((e = copy_bytes(P.tstage, y, b2 * 8, s))) return e;
  // y Op^T into plane q of the product's block; B[k][n] = Lhat[q x + n][k]
  auto right = [&](const double* lh, long long sb, long long sb2, double* C, long long sc, long long sc2, int inner,
                   int count, int q, double beta) {
    GemmDesc g = desc0();
    g.batch1 = count > 1 ? inner : 0;
    g.batch = count;
    g.M = x; g.N = x; g.K = 2 * x; g.K2 = x;
    g.A = y; g.sAm = x; g.sAk = 1; g.sAk1 = xx; g.sAb = 0; g.sAb2 = 0;
    g.B = lh + (long long)q * x * 2 * x; g.sBk = 1; g.sBk1 = x; g.sBn = 2 * x; g.sBb = sb; g.sBb2 = sb2;
    g.C = C + q * xx; g.sCm = x; g.sCn = 1; g.sCb = sc; g.sCb2 = sc2;
    g.beta = beta;
    return run(M, P_F64, g, s, OC_TOP_MM);
  };
  if (D > 0) {
    // stage[1 + half D + k] = y (half ? A_k : B_k)^T: a two-level batch (k,
    // half) whose outer step moves from the B block to the A block before it
    for (int q = 0; q < 2; ++q)
      if ((e = right(P.lhat + (1 + D) * b4, b4, -D * b4, P.tstage + b2, b2, D * b2, D, 2 * D, q, 0.0))) return e;
  }
  GemmDesc g = desc0();  // out = sum_j Lhat_j stage_j
  g.M = 2 * x; g.N = x; g.K = (1 + 2 * D) * 2 * x; g.K2 = 2 * x;
  g.A = P.lhat; g.sAm = 2 * x; g.sAk = 1; g.sAk1 = b4;
  g.B = P.tstage; g.sBk = x; g.sBn = 1; g.sBk1 = b2;
  g.C = out; g.sCm = x; g.sCn = 1;
  if ((e = run(M, P_F64, g, s, OC_TOP_MM))) return e;
  for (int q = 0; q < 2; ++q)  // + y h^T
    if ((e = right(P.lhat, 0, 0, out, 0, 0, 1, 1, q, 1.0))) return e;
  return hipSuccess;
}

ttn_status cx_top(Cx& P) {
  Member& M = P.M;
  const int n = P.n, x = P.dims[n - 1], D = P.D;
  const long long xx = (long long)x * x;
  {
    CplxScope cs(P.delta, P.tri_ok);
    HIPCHK(copy_planes(P.tops, P.ops[n - 1], (1 + 2 * D) * xx * 8, P.s));
  }
  // remove the rounding asymmetry: h Hermitian, A_k, B_k of their term's kind
  // (real part symmetric and imaginary part antisymmetric, or the reverse)
  HIPCHK(symmetrize_f64(P.tops, x, 1.0, P.s));
  HIPCHK(symmetrize_f64(P.im(P.tops), x, -1.0, P.s));
  for (int k = 0; k < D; ++k) {
    if (P.herm[k] == 0) continue;
    const double sg = P.herm[k];
    for (double* o : {P.tops + (1 + k) * xx, P.tops + (1 + D + k) * xx}) {
      HIPCHK(symmetrize_f64(o, x, sg, P.s));
      HIPCHK(symmetrize_f64(P.im(o), x, -sg, P.s));
    }
  }
  for (int j = 0; j < 1 + 2 * D; ++j)
    HIPCHK(embed_complex_f64(P.tops + j * xx, P.im(P.tops) + j * xx, P.lhat + 4 * j * xx, x, x, P.s));
  HIPCHK(zero_int(M.lzint + LZ_DONE, 2, P.s));
  ttn_status r;
  bool conv = false;
  if ((r = top_restarts(M, P.s, M.restarts, true, &conv))) return r;
  P.top_conv = conv;
  if ((r = top_finish(M, P.s))) return r;
  HIPCHK(copy_bytes(M.vT, M.vtop, xx * 8, P.s));
  HIPCHK(copy_bytes(P.im((double*)M.vT), M.vtop + xx, xx * 8, P.s));
  return TTN_OK;
}

// ---------------------------------------------------------------------------
// layer update: w = -polar(Env) through the real embedding
// ---------------------------------------------------------------------------
// ||W W^H - I||_F of the isometry w (a x K) into M.scal[SCAL_ORTHO], from the
// Gram matrix of its embedding (exactly sqrt 2 times it); emb: the embedding
ttn_status cx_ortho(Cx& P, const double* w, double* emb, int a, long long K) {
  Member& M = P.M;
  HIPCHK(embed_complex_f64(w, P.im(w), emb, a, K, P.s));
  GemmDesc g = desc0();
  g.M = 2 * a; g.N = 2 * a; g.K = (int)(2 * K);
  g.tri = 1;
  g.A = emb; g.sAm = 2 * K; g.sAk = 1;
  g.B = emb; g.sBk = 1; g.sBn = 2 * K;
  g.C = M.G; g.sCm = 2 * a; g.sCn = 1;
  HIPCHK(run(M, P_F64, g, P.s));
  HIPCHK(ortho_err_from_gram(M.G, 2 * a, M.scal + SCAL_ORTHO, P.s));
  return TTN_OK;
}

// W from the real polar factor emb of the embedding: the complex matrix whose
// embedding is nearest to it.  The computed factor is orthonormal but carries
// a deviation from the embedding's structure of the order of the polar
// factor's own error (eps / r for an environment of condition ratio r); the
// projection removes it to first order, since the structured part of that
// deviation is a first-order rotation that keeps W W^H = I, and the rest is
// of second order.
ttn_status cx_extract(Cx& P, const double* emb, double* w, int a, long long K) {
  HIPCHK(unembed_complex_f64(emb, w, P.im(w), a, K, P.s));
  return TTN_OK;
}

// Where Env has full rank, the polar factor of its embedding is the embedding
// of the complex polar factor.  Where Env is numerically rank deficient (the
// polar factor is not fixed there), the real solver completes the null
// directions of the embedding without its structure and the projected W is
// not an isometry in them: W W^H is then measured (from W's own embedding;
// one host read per update) and, when it is off the identity by more than
// CX_ORTHO_REPAIR, W is replaced by its polar factor, the nearest isometry
// (unchanged to rounding in the directions that were already orthonormal).
constexpr double CX_ORTHO_REPAIR = 1e-10;

ttn_status cx_update(Cx& P, int tau) {
  Member& M = P.M;
  const int a = P.dims[tau], b = P.dims[tau - 1];
  const long long K = (long long)b * b, aK = (long long)a * K;
  double* w = M.w64[tau];
  HIPCHK(embed_complex_f64(M.env64, P.im(M.env64), P.emb, a, K, P.s));
  HIPCHK(embed_complex_f64(w, P.im(w), P.emb_w, a, K, P.s));
  // Env' = Env - eps ||Env|| w_old (tie-breaker where Env is numerically zero)
  HIPCHK(pair_f64(P.emb, P.emb, 4 * aK, M.scal + SCAL_TMP0, M.part, P.s));
  HIPCHK(sqrt_inplace(M.scal + SCAL_TMP0, P.s));
  HIPCHK(axpy_dev(P.emb, P.emb_w, M.scal + SCAL_TMP0, -POLAR_REG, (size_t)(4 * aK), P.s));
  ttn_status st = polar_core(M, P.emb, 2 * a, 2 * K, -1.0, P.emb, P.s, nullptr, false, nullptr, P.emb_w, P.emb_t);
  if (st) return st;
  HIPCHK(ratio_minmax(M.nrm, 2 * a, M.scal + SCAL_RATIO, M.scal + SCAL_RATIO_MIN, P.s));
  if ((st = cx_extract(P, P.emb, w, a, K))) return st;
  if ((st = cx_ortho(P, w, P.emb_w, a, K))) return st;
  double err = 0.0;
  HIPCHK(hipMemcpyAsync(&err, M.scal + SCAL_ORTHO, sizeof err, hipMemcpyDeviceToHost, P.s));
  HIPCHK(hipStreamSynchronize(P.s));
  if (!(err <= CX_ORTHO_REPAIR * std::sqrt(2.0))) {
    // emb_w holds W's embedding: W <- polar(W)
    if ((st = polar_core(M, P.emb_w, 2 * a, 2 * K, 1.0, P.emb_w, P.s))) return st;
    if ((st = cx_extract(P, P.emb_w, w, a, K))) return st;
    if ((st = cx_ortho(P, w, P.emb_w, a, K))) return st;
    ++P.repairs;
  }
  HIPCHK(running_max(M.scal + SCAL_ORTHO, M.scal + SCAL_ORTHO_MAX, P.s));
  return TTN_OK;
}

ttn_status cx_ascend_from(Cx& P, int from) {
  CplxScope cs(P.delta, P.tri_ok);
  ttn_status r;
  for (int t = from; t < P.n; ++t)
    if ((r = stage_ascend(P.M, t, P.s))) return r;
  return TTN_OK;
}

ttn_status cx_sweep_body(Cx& P) {
  Member& M = P.M;
  ttn_status r;
  {
    CplxScope cs(P.delta, P.tri_ok);
    if ((r = stage_descend_rho(M, P.s))) return r;
  }
  for (int t = 1; t < P.n; ++t) {
    {
      CplxScope cs(P.delta, P.tri_ok);
      if ((r = stage_descend_dressed(M, t, P.s))) return r;
      if ((r = stage_env(M, t, P.s))) return r;
    }
    if ((r = cx_update(P, t))) return r;
    {
      CplxScope cs(P.delta, P.tri_ok);
      if ((r = stage_ascend(M, t, P.s))) return r;
    }
  }
  P.env_tau = -1;
  return cx_top(P);
}

ttn_status cx_sweep(Cx& P) {
  P.M.counting = true;
  P.M.flops_acc = P.M.traffic_acc = 0.0;
  const ttn_status r = cx_sweep_body(P);
  P.M.counting = false;
  P.last_flops = P.M.flops_acc;
  P.last_bytes = P.M.traffic_acc;
  return r;
}

ttn_status cx_check(ttn_cplx_handle h) {
  if (!h) return fail(TTN_EINVAL, "null handle");
  return TTN_OK;
}

ttn_status cx_status(Cx& P, bool warn_top) {
  double sc[SCAL_N];
  HIPCHK(hipMemcpyAsync(sc, P.M.scal, sizeof sc, hipMemcpyDeviceToHost, P.s));
  HIPCHK(hipStreamSynchronize(P.s));
  if (sc[SCAL_ERR] != 0.0) return fail(TTN_EHIP, "a Jacobi eigensolver aborted (grid barrier wait exceeded its bound)");
  if (sc[SCAL_NOCONV] != 0.0) return fail(TTN_ENOCONV, "a polar Jacobi solve stopped at its sweep limit");
  return warn_top && !P.top_conv ? TTN_WNOCONV : TTN_OK;
}

}  // namespace

extern "C" {

ttn_status ttn_cplx_workspace_bytes(const ttn_cplx_config* cfg, size_t* bytes) {
  if (!bytes) return fail(TTN_EINVAL, "bad arguments");
  Member M;
  ttn_status st = cx_member(cfg, M, nullptr);
  if (st) return st;
  *bytes = cx_layout(M, nullptr, nullptr);
  return TTN_OK;
}

ttn_status ttn_cplx_init(const ttn_cplx_config* cfg, void* workspace, size_t bytes, void* stream,
                         ttn_cplx_handle* out) {
  if (!out) return fail(TTN_EINVAL, "bad arguments");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(TTN_EINVAL, "workspace must be non-null and 256-byte aligned");
  size_t need = 0;
  ttn_status st = ttn_cplx_workspace_bytes(cfg, &need);
  if (st) return st;
  if (bytes < need) return fail(TTN_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, need);
  Cx* P = new Cx;
  auto bail = [&](ttn_status e) { delete P; return e; };
  P->s = (hipStream_t)stream;
  Member& M = P->M;
  if ((st = cx_member(cfg, M, &P->herm))) return bail(st);
  P->tri_ok = true;
  for (int hk : P->herm) {
    P->tri_ok = P->tri_ok && hk != 0;
    M.anti.push_back(hk < 0 ? 1 : 0);
  }
  cx_layout(M, (char*)workspace, P);
  M.prof = &P->prof;
  M.matvec = cx_matvec;
  M.owner = P;
  P->L = M.L; P->n = M.n; P->d = M.d; P->D = M.D; P->dims = M.dims;
  const int n = M.n, d = M.d, D = M.D;
  const size_t dd = (size_t)d * d;
  // level-0 operators [h1 - c I, A_1..A_D, B_1..B_D], interleaved
  std::vector<double> op0(2 * (1 + 2 * (size_t)D) * dd);
  std::copy(cfg->h1, cfg->h1 + 2 * dd, op0.begin());
  for (int i = 0; i < d; ++i) op0[2 * (i * d + i)] -= M.c;
  if (D) {
    std::copy(cfg->A, cfg->A + 2 * D * dd, op0.begin() + 2 * dd);
    std::copy(cfg->B, cfg->B + 2 * D * dd, op0.begin() + 2 * (1 + D) * dd);
  }
  double init_scal[SCAL_N] = {0};
  init_scal[SCAL_RATIO_MIN] = 1.0;
  init_scal[SCAL_SHIFT] = M.c;
  hipError_t e = hipMemcpyAsync(M.scal, init_scal, sizeof init_scal, hipMemcpyHostToDevice, P->s);
  if (!e) e = zero_int(M.jinfo, 64, P->s);
  if (e) return bail(fail(TTN_EHIP, "initialisation: %s", hipGetErrorString(e)));
  if ((st = to_planes(*P, op0.data(), P->ops[0], (1 + 2 * (size_t)D) * dd))) return bail(st);
  for (int t = 1; t < n; ++t)
    if ((st = to_planes(*P, cfg->w0[t - 1], M.w64[t], (size_t)P->cube(t)))) return bail(st);
  const size_t xx = (size_t)P->x2(n - 1);
  if (cfg->v0) {
    e = hipMemcpyAsync(P->io, cfg->v0, 2 * xx * 8, hipMemcpyHostToDevice, P->s);
    if (!e) e = deinterleave_f64(P->io, M.vtop, M.vtop + xx, xx, P->s);
  } else {
    e = gaussian_f64(M.vtop, 2 * xx, M.seed ^ 0x5bd1e995ull, 0xfffffffull, P->s);
  }
  if (!e) e = hipStreamSynchronize(P->s);
  if (e) return bail(fail(TTN_EHIP, "initialisation: %s", hipGetErrorString(e)));
  if ((st = cx_ascend_from(*P, 1))) return bail(st);
  if ((st = cx_top(*P))) return bail(st);
  if ((st = cx_status(*P, true)) < 0) return bail(st);
  *out = P;
  return st;
}

ttn_status ttn_cplx_free(ttn_cplx_handle h) {
  if (!h) return TTN_OK;
  hipStreamSynchronize(h->s);
  delete h;
  return TTN_OK;
}

ttn_status ttn_cplx_energy(ttn_cplx_handle h, double* e) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (!e) return fail(TTN_EINVAL, "bad arguments");
  double sc[2];
  HIPCHK(hipMemcpyAsync(sc, h->M.scal + SCAL_LAM, sizeof sc, hipMemcpyDeviceToHost, h->s));
  HIPCHK(hipStreamSynchronize(h->s));
  e[0] = sc[0];
  e[1] = sc[1];
  return cx_status(*h, true);
}

ttn_status ttn_cplx_sweep(ttn_cplx_handle h, int nsweeps) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (nsweeps < 0) return fail(TTN_EINVAL, "nsweeps=%d < 0", nsweeps);
  for (int i = 0; i < nsweeps; ++i) {
    if ((st = cx_sweep(*h))) return st;
    if ((st = cx_status(*h, true)) < 0) return st;
  }
  return cx_status(*h, true);
}

ttn_status ttn_cplx_descend(ttn_cplx_handle h) {
  ttn_status st = cx_check(h);
  if (st) return st;
  {
    CplxScope cs(h->delta, h->tri_ok);
    if ((st = stage_descend_rho(h->M, h->s))) return st;
  }
  HIPCHK(hipStreamSynchronize(h->s));
  return TTN_OK;
}

ttn_status ttn_cplx_env(ttn_cplx_handle h, int tau, double* host) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (tau < 1 || tau >= h->n || !host) return fail(TTN_EINVAL, "tau=%d: need 1 <= tau < %d, non-null host", tau, h->n);
  {
    CplxScope cs(h->delta, h->tri_ok);
    if ((st = stage_descend_rho(h->M, h->s))) return st;
    if ((st = stage_descend_dressed(h->M, tau, h->s))) return st;
    if ((st = stage_env(h->M, tau, h->s))) return st;
  }
  h->env_tau = tau;
  return from_planes(*h, h->M.env64, host, (size_t)h->cube(tau));
}

ttn_status ttn_cplx_get(ttn_cplx_handle h, int what, int level, double* host) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (!host) return fail(TTN_EINVAL, "null host pointer");
  const int D = h->D;
  const long long nk = std::max(D, 1);
  if (what == TTN_CPLX_TOP) return from_planes(*h, (const double*)h->M.vT, host, (size_t)h->x2(h->n - 1));
  if (what == TTN_CPLX_RBAR || what == TTN_CPLX_LBAR) {
    if (h->env_tau < 1) return fail(TTN_EINVAL, "no environment computed since the last change of state");
    const void* src = what == TTN_CPLX_RBAR ? h->M.Rb[h->M.rb_cur] : h->M.Lb[h->M.rb_cur];
    return from_planes(*h, (const double*)src, host, (size_t)(D * h->x2(h->env_tau)));
  }
  if (level < 0 || level >= h->n) return fail(TTN_EINVAL, "level=%d outside [0, %d)", level, h->n);
  if (what == TTN_CPLX_W) {
    if (level < 1) return fail(TTN_EINVAL, "isometries live on levels >= 1");
    return from_planes(*h, h->M.w64[level], host, (size_t)h->cube(level));
  }
  if (what == TTN_CPLX_OPS) {
    // [h, A_1..A_D, B_1..B_D]: the blocks are laid out with nk = max(D, 1)
    const long long q = h->x2(level);
    if ((st = from_planes(*h, h->ops[level], host, (size_t)q))) return st;
    if (D == 0) return TTN_OK;
    if ((st = from_planes(*h, h->ops[level] + q, host + 2 * q, (size_t)(D * q)))) return st;
    return from_planes(*h, h->ops[level] + (1 + nk) * q, host + 2 * (1 + D) * q, (size_t)(D * q));
  }
  if (what == TTN_CPLX_RHO) return from_planes(*h, (const double*)h->M.rho[level], host, (size_t)h->x2(level));
  return fail(TTN_EINVAL, "unknown kind %d", what);
}

ttn_status ttn_cplx_set(ttn_cplx_handle h, int what, int level, const double* host) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (!host) return fail(TTN_EINVAL, "null host pointer");
  if (what == TTN_CPLX_TOP) {
    const size_t xx = (size_t)h->x2(h->n - 1);
    HIPCHK(hipMemcpyAsync(h->io, host, 2 * xx * 8, hipMemcpyHostToDevice, h->s));
    HIPCHK(deinterleave_f64(h->io, h->M.vtop, h->M.vtop + xx, xx, h->s));
    HIPCHK(copy_bytes(h->M.vT, h->M.vtop, xx * 8, h->s));
    HIPCHK(copy_bytes(h->im((double*)h->M.vT), h->M.vtop + xx, xx * 8, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    h->env_tau = -1;
    return TTN_OK;
  }
  if (what != TTN_CPLX_W) return fail(TTN_EINVAL, "only isometries and the top tensor can be set (kind %d)", what);
  if (level < 1 || level >= h->n) return fail(TTN_EINVAL, "level=%d outside [1, %d)", level, h->n);
  if ((st = to_planes(*h, host, h->M.w64[level], (size_t)h->cube(level)))) return st;
  if ((st = cx_ascend_from(*h, level))) return st;
  HIPCHK(hipStreamSynchronize(h->s));
  h->env_tau = -1;
  return TTN_OK;
}

ttn_status ttn_cplx_stats(ttn_cplx_handle h, ttn_cplx_stats_t* out) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (!out) return fail(TTN_EINVAL, "null output");
  double sc[SCAL_N];
  HIPCHK(hipMemcpyAsync(sc, h->M.scal, sizeof sc, hipMemcpyDeviceToHost, h->s));
  HIPCHK(hipStreamSynchronize(h->s));
  std::memset(out, 0, sizeof *out);
  out->lam = sc[SCAL_LAM];
  out->energy = sc[SCAL_E];
  out->lanczos_resid = sc[SCAL_RES];
  out->ortho_err_max = sc[SCAL_ORTHO_MAX] / std::sqrt(2.0);
  out->sigma_ratio_min = sc[SCAL_RATIO_MIN];
  out->flops_sweep = h->last_flops;
  out->bytes_sweep = h->last_bytes;
  out->n_levels = h->n;
  out->top_converged = h->top_conv ? 1 : 0;
  out->repairs = h->repairs;
  return TTN_OK;
}

ttn_status ttn_cplx_profile(ttn_cplx_handle h, int enable) {
  ttn_status st = cx_check(h);
  if (st) return st;
  return profile_switch(h->prof, h->krec, enable);
}

ttn_status ttn_cplx_profile_read(ttn_cplx_handle h, ttn_profile_entry* out, int max_entries, int* n_out) {
  ttn_status st = cx_check(h);
  if (st) return st;
  if (!out || !n_out) return fail(TTN_EINVAL, "bad arguments");
  return profile_collect(h->prof, h->s, out, max_entries, n_out);
}

}  // extern "C"
