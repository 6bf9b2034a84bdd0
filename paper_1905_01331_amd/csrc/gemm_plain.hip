// Register-blocked, LDS-tiled strided GEMM for float64 and float32 (gfx950).
//
// Every contraction of the sweep (leg applications, closes, left
// multiplications, child closes; Fig. 4(b): matrix products after
// flattening) is one strided product; the index permutations of the
// rank-3 tensors are folded into the operand strides of the tile loaders,
// so no tensor is ever transposed in memory.
//
// This kernel is the general path: any strides, ragged edges, two-level
// contraction index.  The float32 / split-bf16 MFMA kernels take the large
// regular shapes.
#include "common.h"
#include "gemm_internal.h"

namespace ttn {

namespace {

constexpr int PT_M = 64, PT_N = 64, PT_K = 16, PT_THREADS = 256;

__device__ __forceinline__ long long koff(int k, int K2, long long s2, long long s1) {
  if (K2 <= 0) return (long long)k * s2;
  int k1 = k / K2;
  int k2 = k - k1 * K2;
  return (long long)k1 * s1 + (long long)k2 * s2;
}

// Round a float to the nearest bf16 value (ties to even), returned as float.
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  return __uint_as_float(u);
}

// MODE 0: plain (T = double or float).  MODE 1: split-bf16 emulation on the
// vector units (T = float): every operand is split into hi = bf16(x),
// lo = bf16(x - hi) and the product is hi*hi + hi*lo + lo*hi accumulated in
// float32.
template <typename T, int MODE>
__global__ __launch_bounds__(PT_THREADS) void gemm_plain_kernel(GemmDesc g, int splits, int kchunk,
                                                                T* __restrict__ partial) {
  __shared__ T As[PT_K][PT_M + 1];
  __shared__ T Bs[PT_K][PT_N + 1];
  __shared__ T Al[MODE ? PT_K : 1][MODE ? PT_M + 1 : 1];
  __shared__ T Bl[MODE ? PT_K : 1][MODE ? PT_N + 1 : 1];
  int bz = blockIdx.z;
  {  // launch-group member: outermost index
    const int per = g.batch * splits, mem = bz / per;
    bz -= mem * per;
    g.A = member_ptr(g.A, g, mem); g.B = member_ptr(g.B, g, mem); g.C = member_ptr(g.C, g, mem);
    g.skip = member_ptr(g.skip, g, mem);
    partial = member_ptr(partial, g, mem);
  }
  if (g.skip && gload(g.skip)) return;

  const int b = bz / splits;
  const int sp = bz - b * splits;
  const int m0 = blockIdx.y * PT_M;
  const int n0 = blockIdx.x * PT_N;
  const int kbeg = sp * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  const T* __restrict__ A = (const T*)g.A + batch_offset(g, b, g.sAb, g.sAb2);
  const T* __restrict__ B = (const T*)g.B + batch_offset(g, b, g.sBb, g.sBb2);

  const int tid = threadIdx.x;
  const int tx = tid & 15;  // columns n0 + tx + 16*j
  const int ty = tid >> 4;  // rows    m0 + ty + 16*i

  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);

  const bool a_kcontig = (g.sAk == 1);
  const bool b_ncontig = (g.sBn == 1);

  for (int k0 = kbeg; k0 < kend; k0 += PT_K) {
#pragma unroll
    for (int it = 0; it < (PT_M * PT_K) / PT_THREADS; ++it) {
      int idx = tid + it * PT_THREADS;
      int mm, kk;
      if (a_kcontig) { mm = idx / PT_K; kk = idx - mm * PT_K; }
      else           { kk = idx / PT_M; mm = idx - kk * PT_M; }
      int m = m0 + mm, k = k0 + kk;
      T v = T(0);
      if (m < g.M && k < kend) v = gload(A + (long long)m * g.sAm + koff(k, g.K2, g.sAk, g.sAk1));
      if constexpr (MODE == 1) {
        float hi = bf16_round((float)v);
        As[kk][mm] = hi;
        Al[kk][mm] = bf16_round((float)v - hi);
      } else {
        As[kk][mm] = v;
      }
    }
#pragma unroll
    for (int it = 0; it < (PT_N * PT_K) / PT_THREADS; ++it) {
      int idx = tid + it * PT_THREADS;
      int nn, kk;
      if (b_ncontig) { kk = idx / PT_N; nn = idx - kk * PT_N; }
      else           { nn = idx / PT_K; kk = idx - nn * PT_K; }
      int n = n0 + nn, k = k0 + kk;
      T v = T(0);
      if (n < g.N && k < kend) v = gload(B + (long long)n * g.sBn + koff(k, g.K2, g.sBk, g.sBk1));
      if constexpr (MODE == 1) {
        float hi = bf16_round((float)v);
        Bs[kk][nn] = hi;
        Bl[kk][nn] = bf16_round((float)v - hi);
      } else {
        Bs[kk][nn] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < PT_K; ++kk) {
      T a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
      if constexpr (MODE == 1) {
        T al[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) al[i] = Al[kk][ty + 16 * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) bl[j] = Bl[kk][tx + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i][j] = fmaf(al[i], bb[j], acc[i][j]);
            acc[i][j] = fmaf(a[i], bl[j], acc[i][j]);
            acc[i][j] = fmaf(a[i], bb[j], acc[i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bb[j];
      }
    }
    __syncthreads();
  }

  if (splits == 1) {
    T* C = (T*)g.C + batch_offset(g, b, g.sCb, g.sCb2);
    const T alpha = (T)g.alpha, beta = (T)g.beta;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m = m0 + ty + 16 * i;
      if (m >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int n = n0 + tx + 16 * j;
        if (n >= g.N) continue;
        T* c = C + (long long)m * g.sCm + (long long)n * g.sCn;
        T r = alpha * acc[i][j];
        if (g.beta != 0.0) r += beta * gload(c);
        gstore(c, r);
      }
    }
  } else {
    // partial sums, dense (M x N) per (split, batch) slice
    T* P = partial + ((long long)sp * g.batch + b) * (long long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m = m0 + ty + 16 * i;
      if (m >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int n = n0 + tx + 16 * j;
        if (n >= g.N) continue;
        gstore(P + (long long)m * g.N + n, acc[i][j]);
      }
    }
  }
}

}  // namespace

// Deterministic split-K reduction: C = alpha * sum_s P[s] + beta * C.  Eight
// independent partial sums over the splits s = 8q + u (u = 0..7) keep eight
// loads in flight per thread; they are combined in a fixed tree, so the
// result does not depend on timing.
template <typename T>
__global__ void splitk_reduce_kernel(GemmDesc g, int splits, const T* __restrict__ partial) {
  const long long MN = (long long)g.M * g.N;
  const long long stride = (long long)g.batch * MN;
  const long long total = stride * gemm_members(g);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int mem = (int)(i / stride);  // launch-group member
    const int* skip = member_ptr(g.skip, g, mem);
    if (skip && *skip) continue;
    const long long im = i - (long long)mem * stride;
    int b = (int)(im / MN);
    long long r = im - (long long)b * MN;
    int m = (int)(r / g.N);
    int n = (int)(r - (long long)m * g.N);
    const T* p = member_ptr(partial, g, mem) + (long long)b * MN + r;
    T s8[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    int sp = 0;
    for (; sp + 8 <= splits; sp += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s8[u] += gload(p + (long long)(sp + u) * stride);
    }
    for (int u = 0; sp + u < splits; ++u) s8[u] += gload(p + (long long)(sp + u) * stride);
    T s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    T* c = (T*)member_ptr(g.C, g, mem) + batch_offset(g, b, g.sCb, g.sCb2) + (long long)m * g.sCm +
           (long long)n * g.sCn;
    T out = (T)g.alpha * s;
    if (g.beta != 0.0) out += (T)g.beta * gload(c);
    gstore(c, out);
  }
}

template <typename T>
static hipError_t splitk_reduce(const GemmDesc& g, int splits, const T* partial, hipStream_t s) {
  const long long total = (long long)g.batch * g.M * g.N * gemm_members(g);
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  size_t slot = 0;
  KernelTimer* kt = kernel_timer();
  const bool timed =
      kt && kt->begin(KID_REDUCE + (sizeof(T) == 8 ? 1 : 0), 0.0, sizeof(T) * (double)total * (splits + 1), s, &slot);
  hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3(blocks), dim3(256), 0, s, g, splits, partial);
  if (timed) kt->end(slot, s);
  return hipGetLastError();
}

template <typename T>
static int choose_splits(const GemmDesc& g, size_t scratch_bytes) {
  long long tiles = (long long)((g.M + PT_M - 1) / PT_M) * ((g.N + PT_N - 1) / PT_N) * g.batch;
  if (tiles >= 512 || g.K < 8 * PT_K) return 1;
  long long want = (1024 + tiles - 1) / tiles;
  long long maxk = (g.K + 4 * PT_K - 1) / (4 * PT_K);  // at least 4 k-tiles per split
  long long s = want < maxk ? want : maxk;
  if (s > 64) s = 64;
  size_t slice = (size_t)g.batch * g.M * g.N * sizeof(T);
  if (slice == 0) return 1;
  long long fit = (long long)(scratch_bytes / slice);
  if (s > fit) s = fit;
  return s < 1 ? 1 : (int)s;
}

template <typename T, int MODE>
static hipError_t launch_plain(const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  int splits = (g.K > 0) ? choose_splits<T>(g, scratch_bytes) : 1;
  int kchunk = (g.K + splits - 1) / splits;
  kchunk = ((kchunk + PT_K - 1) / PT_K) * PT_K;
  if (kchunk == 0) kchunk = PT_K;
  splits = (g.K + kchunk - 1) / kchunk;
  if (splits < 1) splits = 1;
  dim3 grid((g.N + PT_N - 1) / PT_N, (g.M + PT_M - 1) / PT_M, g.batch * splits * gemm_members(g));
  size_t slot = 0;
  KernelTimer* kt = kernel_timer();
  const double work = (double)g.batch * gemm_members(g);
  const bool timed = kt && kt->begin(KID_PLAIN + (sizeof(T) == 8 ? 0 : 1 + MODE), 2.0 * g.M * (double)g.N * g.K * work,
                                     sizeof(T) * work * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N), s,
                                     &slot);
  hipLaunchKernelGGL((gemm_plain_kernel<T, MODE>), grid, dim3(PT_THREADS), 0, s, g, splits, kchunk,
                     (T*)scratch);
  if (timed) kt->end(slot, s);
  if (splits > 1) return splitk_reduce<T>(g, splits, (const T*)scratch, s);
  return hipGetLastError();
}

hipError_t gemm_plain(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s) {
  switch (prec) {
    case P_F64: return launch_plain<double, 0>(g, scratch, scratch_bytes, s);
    case P_F32: return launch_plain<float, 0>(g, scratch, scratch_bytes, s);
    case P_BF16X3: return launch_plain<float, 1>(g, scratch, scratch_bytes, s);
  }
  return hipErrorInvalidValue;
}

hipError_t splitk_reduce_f32(const GemmDesc& g, int splits, const float* partial, hipStream_t s) {
  return splitk_reduce<float>(g, splits, partial, s);
}

hipError_t splitk_reduce_f64(const GemmDesc& g, int splits, const double* partial, hipStream_t s) {
  return splitk_reduce<double>(g, splits, partial, s);
}

KernelTimer*& kernel_timer() {
  static KernelTimer* t = nullptr;
  return t;
}

const char* kernel_name(int kid) {
  static const char* const names[KID_N] = {
      "gemm_mfma_kernel<1, false, false>", "gemm_mfma_kernel<1, false, true>", "gemm_mfma_kernel<1, true, false>",
      "gemm_mfma_kernel<1, true, true>",   "gemm_mfma_kernel<2, false, false>", "gemm_mfma_kernel<2, false, true>",
      "gemm_mfma_kernel<2, true, false>",  "gemm_mfma_kernel<2, true, true>",
      "gemm_f64_kernel<false, false, 0>",  "gemm_f64_kernel<false, true, 0>",  "gemm_f64_kernel<true, false, 0>",
      "gemm_f64_kernel<true, true, 0>",    "gemm_f64_kernel<false, false, 1>", "gemm_f64_kernel<false, true, 1>",
      "gemm_f64_kernel<true, false, 1>",   "gemm_f64_kernel<true, true, 1>",   "gemm_f64_kernel<false, false, 2>",
      "gemm_f64_kernel<false, true, 2>",   "gemm_f64_kernel<true, false, 2>",  "gemm_f64_kernel<true, true, 2>",
      "gemm_plain_kernel<double, 0>",      "gemm_plain_kernel<float, 0>",      "gemm_plain_kernel<float, 1>",
      "splitk_reduce_kernel<float>",       "splitk_reduce_kernel<double>"};
  return (kid >= 0 && kid < KID_N) ? names[kid] : "?";
}

hipError_t gemm(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s) {
  if (gemm_path_mfma_enabled()) {
    GemmLaunch how;
    gemm_tuned_choice(prec, g, s, scratch, scratch_bytes, &how);
    hipError_t e = gemm_mfma(prec, g, scratch, scratch_bytes, s, how);
    if (e != hipErrorNotSupported) return e;
  }
  return gemm_plain(prec, g, scratch, scratch_bytes, s);
}

namespace {
bool g_mfma_enabled = true;
}
bool gemm_path_mfma_enabled() { return g_mfma_enabled; }
void gemm_set_mfma_enabled(bool on) { g_mfma_enabled = on; }

}  // namespace ttn
