// Internal declarations shared by the HIP sources of libttn (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>
#include <stddef.h>

namespace ttn {

// Strided, batched matrix product  C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n).
// Element addresses:  A + b*sAb + m*sAm + koff_A(k),  B + b*sBb + koff_B(k) + n*sBn,
// C + b*sCb + m*sCm + n*sCn,  with a two-level contraction index k = k1*K2 + k2:
// koff_A(k) = k1*sAk1 + k2*sAk (likewise for B).  K2 == K means a single level.
struct GemmDesc {
  int M, N, K, K2;
  int batch;
  const void* A; long long sAm, sAk, sAk1, sAb;
  const void* B; long long sBk, sBn, sBk1, sBb;
  void* C;       long long sCm, sCn, sCb;
  double alpha, beta;
  // optional device flag: when non-null and nonzero at run time, every
  // kernel of the product returns at once (C untouched), so that a captured
  // graph can carry a product whose need is decided on the device
  const int* skip;
  // two-level batch: with batch1 > 0 the batch index b = b1 + batch1 * b2
  // (b1 < batch1) places operand X at b1 * sXb + b2 * sXb2; batch is the
  // total count.  batch1 == 0: one level, X at b * sXb.
  int batch1;
  long long sAb2, sBb2, sCb2;
  // launch group (see GroupCtx): mcount > 1 products of the same shape whose
  // operands, result, split-K scratch and skip flag all lie mstride bytes
  // apart, run as one launch (member index outermost)
  int mcount;
  long long mstride;
  // square outputs known to be symmetric (tri = 1) or, for the batch entries
  // whose bit is set in anti (inner batch index), antisymmetric: a float64
  // launch may compute the block upper triangle only and mirror the rest
  // (with beta != 0 the old C must have the same parity: only its upper
  // triangle is read); other launches ignore it.  The split count then
  // follows the tiles computed.
  int tri;
  unsigned long long anti;
};

__host__ __device__ __forceinline__ int gemm_members(const GemmDesc& g) { return g.mcount > 1 ? g.mcount : 1; }
template <class T>
__host__ __device__ __forceinline__ T* member_ptr(T* p, const GemmDesc& g, int m) {
  return p ? (T*)((uintptr_t)p + (long long)m * g.mstride) : p;
}

__host__ __device__ __forceinline__ long long batch_offset(const GemmDesc& g, int b, long long s1, long long s2) {
  if (g.batch1 <= 0) return (long long)b * s1;
  const int q = b / g.batch1;
  return (long long)(b - q * g.batch1) * s1 + (long long)q * s2;
}

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2 };

// Launch group: identical-layout batch members placed `stride` bytes apart in
// the workspace run as one launch per kernel; the member index is
// blockIdx.y (small kernels) or the outermost grid index (products), and
// every pointer argument (all of them point into a member's part of the
// workspace) moves by stride bytes per member.  count = 1: one member.
struct GroupCtx {
  int count = 1;
  long long stride = 0;
  // optional device flag (per member, shifted like every member pointer):
  // the kernels of the helpers that honour it return at once while it is set
  const int* skip = nullptr;
};
GroupCtx& grp();  // the calling thread's current launch group
// scoped setting of the launch group
struct GroupScope {
  GroupCtx saved;
  GroupScope(int count, long long stride) : saved(grp()) { grp().count = count; grp().stride = stride; }
  ~GroupScope() { grp() = saved; }
};
struct SkipScope {
  const int* saved;
  explicit SkipScope(const int* flag) : saved(grp().skip) { grp().skip = flag; }
  ~SkipScope() { grp().skip = saved; }
};

// Global-memory access through an address-space-qualified pointer.  Device
// pointers carried in structures are generic to the compiler, and generic
// (flat) accesses count against the LDS counter as well as the vector-memory
// counter, so a wait for LDS reads would also wait for every global load in
// flight; these helpers make the access a global one.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// (byte arithmetic on the pointer itself, not through an integer, so that the
// compiler keeps knowing a kernel argument points to global memory)
template <class T>
__device__ __forceinline__ T* mshift(T* p, long long ms) {
  typedef typename std::conditional<std::is_const<T>::value, const char, char>::type B;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long long)blockIdx.y * ms) : p;
}
// true when the member's skip flag is set (uniform over the work-group)
__device__ __forceinline__ bool member_skipped(const int* sk, long long ms) {
  return sk && *mshift(sk, ms);
}

// Optional per-kernel timing of the product kernels (set while a handle's
// profiling is on): begin/end bracket one kernel launch with HIP events;
// kernel ids name the instantiations (see kernel_name()).
struct KernelTimer {
  virtual bool begin(int kernel_id, double flops, double bytes, hipStream_t s, size_t* slot) = 0;
  virtual void end(size_t slot, hipStream_t s) = 0;
  virtual ~KernelTimer() {}
};
KernelTimer*& kernel_timer();
enum { KID_MFMA = 0,     // + 4 * (mode - 1) + 2 * akc + bkc  (mode 1: float32, 2: split-bf16)
       KID_F64 = 8,      // + 4 * tile + 2 * akc + bkc  (tile 0: 64 x 64, 1: 128 x 64, 2: 64 x 128)
       KID_PLAIN = 20,   // + precision
       KID_REDUCE = 23,  // split-K reductions: + 0 float, + 1 double
       KID_N = 25 };
const char* kernel_name(int kid);

// Launches one product in the given arithmetic.  F64: double operands and
// result.  F32 / BF16X3: float operands and result (BF16X3 splits every
// float operand into bf16 hi + lo on load).  `scratch` (float/double,
// `scratch_elems` elements) holds split-K partial sums when the launcher
// chooses to split the contraction; the reduction is deterministic.
hipError_t gemm(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);

// -------- small kernels (small.hip) -------------------------------------------
hipError_t convert_f64_to_f32(const double* x, float* y, size_t n, hipStream_t s);
hipError_t convert_f32_to_f64(const float* x, double* y, size_t n, hipStream_t s);
hipError_t fill_f64(double* x, double v, size_t n, hipStream_t s);
hipError_t fill_f32(float* x, float v, size_t n, hipStream_t s);
hipError_t copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
// copies when *flag == want (device flag read at run time)
hipError_t copy_bytes_if(void* dst, const void* src, size_t bytes, const int* flag, int want, hipStream_t s);
// flag[0] = (info[0] <= limit) ? 1 : 0; err[0] (a double) is set to 1 when
// any of info[0], info[2], .., info[2 (nq - 1)] is negative (an aborted
// solve), noconv[0] (may be null) when any of them is >= limit (a solve that
// used all its sweeps)
hipError_t set_flag_le(int* flag, const int* info, int limit, hipStream_t s);
hipError_t note_negative_info(const int* info, int nq, double* err, double* noconv, int limit, hipStream_t s);
hipError_t add_diag_f64(double* X, int n, double v, hipStream_t s);
// y = alpha*x + beta*y over n elements (float or double)
hipError_t axpby_f64(const double* x, double* y, double alpha, double beta, size_t n, hipStream_t s);
hipError_t axpby_f32(const float* x, float* y, float alpha, float beta, size_t n, hipStream_t s);
hipError_t gaussian_f64(double* x, size_t n, unsigned long long seed, unsigned long long stream_id, hipStream_t s);

// One 2 x 2 Jacobi rotation of the pair (p, q) of a symmetric matrix with
// diagonal gpp, gqq and off-diagonal gpq.  t = tan(phi) is the root of
// t^2 + 2 theta t - 1 = 0 of smaller magnitude, theta = (gqq - gpp) / (2 gpq),
// computed without forming theta:  t = sgn(x) y / (|x| + sqrt(x^2 + y^2)),
// x = gqq - gpp, y = 2 gpq;  c = 1/sqrt(1 + t^2), s = t c.  The square root,
// the reciprocal and c come from the hardware reciprocal (square root)
// estimates refined by two Newton steps each (a few ulps; c^2 + s^2 = 1 to
// working precision, which is what keeps the accumulated rotations
// orthogonal); x^2 + y^2 outside [1e-280, 1e280] takes hypot().  The pair is
// skipped (returns false, c = 1, s = t = 0) when |gpq| <= tol sqrt(|gpp gqq|):
// a relative threshold, so that small eigenvalues of a graded matrix keep
// their relative accuracy (Demmel and Veselic 1992).  Written without
// branches on the data so that a wave evaluates it in one pass.
__device__ __forceinline__ bool jacobi_rotation(double gpp, double gqq, double gpq, double tol, double& c, double& s,
                                                double& t) {
  const bool rotate = gpq != 0.0 && gpq * gpq > tol * tol * fabs(gpp * gqq);
  const double x = gqq - gpp, y = 2.0 * gpq;
  const double z = x * x + y * y;
  double h;
  if (z > 1e-280 && z < 1e280) {
    double r = __builtin_amdgcn_rsq(z);
    r = r * (1.5 - 0.5 * z * r * r);
    r = r * (1.5 - 0.5 * z * r * r);
    h = z * r;
  } else {
    h = hypot(x, y);
  }
  const double d = fabs(x) + h;
  double inv = __builtin_amdgcn_rcp(d);
  inv = inv * (2.0 - d * inv);
  inv = inv * (2.0 - d * inv);
  const double tt = (x >= 0.0 ? y : -y) * inv;
  const double w = 1.0 + tt * tt;
  double r = __builtin_amdgcn_rsq(w);
  r = r * (1.5 - 0.5 * w * r * r);
  r = r * (1.5 - 0.5 * w * r * r);
  t = rotate ? tt : 0.0;
  c = rotate ? r : 1.0;
  s = rotate ? tt * r : 0.0;
  return rotate;
}

// Jacobi eigensolver of a symmetric n x n float64 matrix G (in place; on
// return the diagonal holds the eigenvalues), eigenvectors in the ROWS of
// U (n x n), G_in = U^T diag U.  One work-group.  `info` (device int[4]): [0] sweeps used,
// [1] rotations in the first sweep.
// `scratch` (jacobi_blocked_scratch_bytes(n) bytes, may be null for n <= 128)
// serves the blocked variant taken for n > 128.
// `skip` (device flag, may be null): when nonzero at run time the kernels
// return at once and G, V and info are left untouched.
hipError_t jacobi_eig_f64(double* G, double* V, int n, int max_sweeps, double tol, int* info, void* scratch,
                          hipStream_t s, const int* skip = nullptr);
hipError_t jacobi_eig_blocked_f64(double* G, double* U, int n, int max_sweeps, double tol, int* info, void* scratch,
                                  hipStream_t s, const int* skip = nullptr);
size_t jacobi_blocked_scratch_bytes(int n);
// Z[i,:] = Y[i,:] / ||Y[i,:]||  for an m x k matrix (row norms into nrm[m]); rows
// with a zero norm are left zero.
hipError_t row_normalize_f64(const double* Y, double* Z, double* nrm, int m, long long k, hipStream_t s);
// Frobenius pairing sum X.*Y (float64 result into out[0]).
// `part` is device scratch of at least 256 doubles.
hipError_t pair_f64(const double* X, const double* Y, long long n, double* out, double* part, hipStream_t s);
hipError_t pair_f32(const float* X, const float* Y, long long n, double* out, double* part, hipStream_t s);
// Row-wise pairings: out[r os + oo] = beta out[r os + oo] + sum_{i < len}
// X[r sX + i] Y[r sY + i] for r < rows (sY = 0: one Y for every row).
hipError_t pair_rows_f64(const double* X, long long sX, const double* Y, long long sY, long long len, int rows,
                         double* out, long long os, long long oo, double beta, hipStream_t s);
// count blocks of len doubles: dst[j ds + i] = src[j ss + i] (not a launch
// group helper: the two strides differ)
hipError_t copy_strided_f64(double* dst, long long ds, const double* src, long long ss, long long len, int count,
                            hipStream_t s);
// out[0] = 1 when out[0] != 0 or any x[j stride + i0] != 0 (j < count); out[1]
// likewise with i1 (one work-item)
hipError_t flags_or(const double* x, long long stride, int count, int i0, int i1, double* out, hipStream_t s);
// nrm2[i] = squared norm of row i of Y (m x k); flag[0] = 1 when every row's
// norm is at least rel times the largest, else 0 (numerically null rows)
hipError_t no_null_rows(const double* Y, int m, long long k, double rel, double* nrm2, int* flag, hipStream_t s);
// unless *flag: the rows i of Y (m x k) whose squared norm nrm2[i] lies below
// rel^2 max_j nrm2[j] become rel sqrt(max_j nrm2[j]) T[i, :]
hipError_t fill_null_rows(double* Y, const double* T, const double* nrm2, int m, long long k, double rel,
                          const int* flag, hipStream_t s);
// ||W W^T - I||_F from the Gram G (n x n): out[0] = sqrt(sum (G - I)^2)
hipError_t ortho_err_from_gram(const double* G, int n, double* out, hipStream_t s);

}  // namespace ttn
