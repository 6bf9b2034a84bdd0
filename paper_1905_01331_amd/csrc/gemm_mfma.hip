// MFMA strided GEMM for the float32 and split-bf16 bulk contractions (gfx950).
//
// One kernel serves every contraction shape of the sweep: the operand tile
// loaders take either a contraction-contiguous or an output-contiguous
// layout (the index permutations of the rank-3 tensors are folded into the
// strides, including the two-level contraction index of the left-child
// close), so no operand is transposed in memory.
//
// Tile 128 x 128 per 256-thread work-group, 2 x 2 waves, 64 x 64 per wave as
// 2 x 2 blocks of 32 x 32 MFMA accumulators.
//   float32:     v_mfma_f32_32x32x2_f32, BK = 16.
//   split-bf16:  every float32 operand x is split on load into hi = bf16(x),
//                lo = bf16(x - hi) (round to nearest even); each 32x32x16
//                step issues lo*hi, hi*lo, hi*hi with v_mfma_f32_32x32x16_bf16
//                into the same float32 accumulator, BK = 32.
// Operand tiles live in LDS as [k][mn] (float32) or [k/8][mn][8] (bf16 hi and
// lo planes), so that the 32 lanes of a half-wave read 32 consecutive
// entries (float32) or 32 consecutive 16-byte chunks (bf16).
// Long contractions are split over the grid's z dimension into partial
// float32 slices reduced in a fixed order; the split count depends on the
// product's shape alone, so a result never depends on how or where the
// product was launched (tile order, launch group, tuned choices).
#include "common.h"
#include "gemm_internal.h"
#include <algorithm>

namespace ttn {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, NT = 256;

template <int MODE> struct Cfg;
template <> struct Cfg<P_F32> { static constexpr int BK = 16; };
template <> struct Cfg<P_BF16X3> { static constexpr int BK = 32; };

// Operand view: element (mn, k) at base + mn*s_mn + koff(k), koff(k) =
// (k / K2)*s_k1 + (k % K2)*s_k.  KC: contraction-contiguous (s_k == 1),
// else output-contiguous (s_mn == 1).
struct OpView {
  const float* base;
  long long s_mn, s_k, s_k1;
  int MN, K2;
};

__device__ __forceinline__ long long k_offset(const OpView& v, int k) {
  if (v.K2 <= 0) return (long long)k * v.s_k;
  int k1 = k / v.K2;
  return (long long)k1 * v.s_k1 + (long long)(k - k1 * v.K2) * v.s_k;
}

// XCD-aware tile order.  Work-groups are handed to the 8 XCDs in turn
// (work-group id mod 8), and each XCD has its own L2.  The grid is launched
// 1-D with 8 * per work-groups; XCD c takes the contiguous range
// [c * per, (c + 1) * per) of a logical tile order in which the output-tile
// dimension with fewer tiles runs fastest, so that the tiles sharing an
// operand panel (the same rows of A, or the same columns of B, and the same
// K range) run at about the same time on one XCD and read that panel from
// HBM once.
struct TileMap {
  int gx, gy, gz, per, yfast;
};
constexpr int N_XCD = 8;
__device__ __forceinline__ bool map_tile(const TileMap& t, int& tx, int& ty, int& tz) {
  const int id = blockIdx.x;
  const long long L = (long long)(id % N_XCD) * t.per + id / N_XCD;
  if (L >= (long long)t.gx * t.gy * t.gz) return false;
  const int l = (int)L;
  if (t.yfast) { ty = l % t.gy; const int r = l / t.gy; tx = r % t.gx; tz = r / t.gx; }
  else { tx = l % t.gx; const int r = l / t.gx; ty = r % t.gy; tz = r / t.gy; }
  return true;
}
// orient: 0 the smaller tile dimension fastest, 1 x fastest, 2 y fastest
// (a launch-shape choice: the tiles compute the same values in any order)
TileMap make_map(int gx, int gy, int gz, int orient) {
  TileMap t;
  t.gx = gx; t.gy = gy; t.gz = gz;
  const long long total = (long long)gx * gy * gz;
  t.per = (int)((total + N_XCD - 1) / N_XCD);
  t.yfast = orient == 0 ? gy < gx : orient == 2;
  return t;
}

__device__ __forceinline__ f32x4 ld4(const float* p) { return gload(reinterpret_cast<const f32x4*>(p)); }

// Per-thread register staging of one operand tile (BMN x BK floats).
template <int MODE, bool KC>
struct Stage {
  static constexpr int BK = Cfg<MODE>::BK;
  static constexpr int NV = (BM * BK) / (4 * NT);  // float4 per thread
  f32x4 r[NV];

  // KC: float4 along k; index f -> (mn = f / (BK/4), kq = f % (BK/4)).
  // !KC (float32): float4 along mn; f -> (k = f / (BM/4), mq = f % (BM/4)).
  // !KC (bf16): a 4(mn) x 4(k) block per thread: t -> (mb = t % 32, kb = t / 32).
  __device__ __forceinline__ void load(const OpView& v, int mn0, int k0, int kend, int tid) {
    if constexpr (KC) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        int f = tid + i * NT;
        int mn = f / (BK / 4), k = (f % (BK / 4)) * 4;
        int gm = mn0 + mn, gk = k0 + k;
        if (gm < v.MN && gk < kend) r[i] = ld4(v.base + (long long)gm * v.s_mn + k_offset(v, gk));
        else r[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    } else if constexpr (MODE == P_F32) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        int f = tid + i * NT;
        int k = f / (BM / 4), mn = (f % (BM / 4)) * 4;
        int gm = mn0 + mn, gk = k0 + k;
        if (gm < v.MN && gk < kend) r[i] = ld4(v.base + gm + k_offset(v, gk));
        else r[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    } else {
      static_assert(NV == 4, "bf16 output-contiguous staging is a 4x4 block");
      int mn = (tid % 32) * 4, kb = (tid / 32) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gm = mn0 + mn, gk = k0 + kb + i;
        if (gm < v.MN && gk < kend) r[i] = ld4(v.base + gm + k_offset(v, gk));
        else r[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }

  // Whole tile in range and every BK chunk inside one block of the
  // two-level contraction index: the same elements as load(), addressed as
  // a work-group-uniform base (tile origin, k offset, load index) plus a
  // per-thread offset, with no range tests.
  __device__ __forceinline__ static long long fast_stride(const OpView& v) {
    if constexpr (KC) return (long long)(NT / (BK / 4)) * v.s_mn;
    else if constexpr (MODE == P_F32) return (long long)(NT / (BM / 4)) * v.s_k;
    else return v.s_k;
  }
  __device__ __forceinline__ static long long fast_voff(const OpView& v, int tid) {
    if constexpr (KC) return (long long)(tid / (BK / 4)) * v.s_mn + (tid % (BK / 4)) * 4;
    else if constexpr (MODE == P_F32) return (tid % (BM / 4)) * 4 + (long long)(tid / (BM / 4)) * v.s_k;
    else return (tid % 32) * 4 + (long long)(tid / 32) * 4 * v.s_k;
  }
  __device__ __forceinline__ void load_fast(const float* tile_base, long long s_i, long long voff) {
#pragma unroll
    for (int i = 0; i < NV; ++i) r[i] = ld4(tile_base + i * s_i + voff);
  }
};

// LDS planes
template <int MODE> struct Smem;
template <> struct Smem<P_F32> {
  float a[16][BM + 4];
  float b[16][BN + 4];
};
template <> struct Smem<P_BF16X3> {
  __bf16 ahi[4][BM][8], alo[4][BM][8];
  __bf16 bhi[4][BN][8], blo[4][BN][8];
};

// Row of the bf16 planes where operand row `row` of plane `plane` is kept:
// an XOR of the low three row bits with (row / 4) and (2 plane) that spreads
// the writes of one wave over the LDS banks (the planes are a multiple of
// the bank period apart, and an output-contiguous operand is written four
// rows per lane) while any 32 consecutive rows of one plane stay a
// permutation of one contiguous block for the MFMA operand reads.
__device__ __forceinline__ int swz(int row, int plane) {
  return row ^ (((row >> 2) ^ (plane << 1)) & 7);
}

// Two floats at once: hi = bf16(x), lo = bf16(x - hi), both rounded to
// nearest even (one packed conversion each); the float value of each hi is
// rebuilt from the packed pair by moving its 16 bits into place.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split2_bf16(float x0, float x1, bf16x2& hi, bf16x2& lo) {
  hi = __builtin_convertvector(f32x2{x0, x1}, bf16x2);
  const unsigned u = __builtin_bit_cast(unsigned, hi);
  const float h0 = __builtin_bit_cast(float, u << 16);
  const float h1 = __builtin_bit_cast(float, u & 0xffff0000u);
  const float l0 = x0 - h0, l1 = x1 - h1;
  lo = __builtin_convertvector(f32x2{l0, l1}, bf16x2);
}
__device__ __forceinline__ void split4_bf16(float x0, float x1, float x2, float x3, bf16x4& hi, bf16x4& lo) {
  bf16x2 h01, l01, h23, l23;
  split2_bf16(x0, x1, h01, l01);
  split2_bf16(x2, x3, h23, l23);
  hi = __builtin_shufflevector(h01, h23, 0, 1, 2, 3);
  lo = __builtin_shufflevector(l01, l23, 0, 1, 2, 3);
}

template <bool KC>
__device__ __forceinline__ void store_f32(const Stage<P_F32, KC>& st, float (*pl)[BM + 4], int tid) {
  constexpr int BK = 16;
  if constexpr (KC) {
#pragma unroll
    for (int i = 0; i < Stage<P_F32, KC>::NV; ++i) {
      int f = tid + i * NT;
      int mn = f / (BK / 4), k = (f % (BK / 4)) * 4;
      pl[k + 0][mn] = st.r[i][0];
      pl[k + 1][mn] = st.r[i][1];
      pl[k + 2][mn] = st.r[i][2];
      pl[k + 3][mn] = st.r[i][3];
    }
  } else {
#pragma unroll
    for (int i = 0; i < Stage<P_F32, KC>::NV; ++i) {
      int f = tid + i * NT;
      int k = f / (BM / 4), mn = (f % (BM / 4)) * 4;
      *reinterpret_cast<f32x4*>(&pl[k][mn]) = st.r[i];
    }
  }
}

template <bool KC>
__device__ __forceinline__ void store_bf16(const Stage<P_BF16X3, KC>& st, __bf16 (*hi)[BM][8], __bf16 (*lo)[BM][8],
                                           int tid) {
  constexpr int BK = 32;
  if constexpr (KC) {
#pragma unroll
    for (int i = 0; i < Stage<P_BF16X3, KC>::NV; ++i) {
      int f = tid + i * NT;
      int mn = f / (BK / 4), k = (f % (BK / 4)) * 4;
      bf16x4 h, l;
      split4_bf16(st.r[i][0], st.r[i][1], st.r[i][2], st.r[i][3], h, l);
      *reinterpret_cast<bf16x4*>(&hi[k >> 3][swz(mn, k >> 3)][k & 7]) = h;
      *reinterpret_cast<bf16x4*>(&lo[k >> 3][swz(mn, k >> 3)][k & 7]) = l;
    }
  } else {
    int mn = (tid % 32) * 4, kb = (tid / 32) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {  // row mn + e, k = kb .. kb+3
      bf16x4 h, l;
      split4_bf16(st.r[0][e], st.r[1][e], st.r[2][e], st.r[3][e], h, l);
      *reinterpret_cast<bf16x4*>(&hi[kb >> 3][swz(mn + e, kb >> 3)][kb & 7]) = h;
      *reinterpret_cast<bf16x4*>(&lo[kb >> 3][swz(mn + e, kb >> 3)][kb & 7]) = l;
    }
  }
}

// The contraction loop of one output tile: the next chunk of BK contraction
// indices of both operands is loaded into registers while the MFMAs consume
// the current one from LDS.
template <int MODE, bool AKC, bool BKC>
__device__ __forceinline__ void kloop(Smem<MODE>& sm, const OpView& va, const OpView& vb, int m0, int n0, int kbeg,
                                      int kend, f32x16 (&acc)[2][2], int tid, bool fast) {
  constexpr int BK = Cfg<MODE>::BK;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  Stage<MODE, AKC> sa;
  Stage<MODE, BKC> sb;
  const float* abase = va.base + (long long)m0 * (AKC ? va.s_mn : 1);
  const float* bbase = vb.base + (long long)n0 * (BKC ? vb.s_mn : 1);
  const long long as_i = Stage<MODE, AKC>::fast_stride(va), bs_i = Stage<MODE, BKC>::fast_stride(vb);
  const long long avo = Stage<MODE, AKC>::fast_voff(va, tid);
  const long long bvo = Stage<MODE, BKC>::fast_voff(vb, tid);
  auto load = [&](Stage<MODE, AKC>& xa, Stage<MODE, BKC>& xb, int k) {
    if (fast) {  // uniform over the work-group
      xa.load_fast(abase + k_offset(va, k), as_i, avo);
      xb.load_fast(bbase + k_offset(vb, k), bs_i, bvo);
    } else {
      xa.load(va, m0, k, kend, tid);
      xb.load(vb, n0, k, kend, tid);
    }
  };
  if (kbeg < kend) load(sa, sb, kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    if constexpr (MODE == P_F32) {
      store_f32<AKC>(sa, sm.a, tid);
      store_f32<BKC>(sb, sm.b, tid);
    } else {
      store_bf16<AKC>(sa, sm.ahi, sm.alo, tid);
      store_bf16<BKC>(sb, sm.bhi, sm.blo, tid);
    }
    __syncthreads();
    if (k0 + BK < kend) load(sa, sb, k0 + BK);
    if constexpr (MODE == P_F32) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        float a0 = sm.a[kk + (lane >> 5)][wm + (lane & 31)];
        float a1 = sm.a[kk + (lane >> 5)][wm + 32 + (lane & 31)];
        float b0 = sm.b[kk + (lane >> 5)][wn + (lane & 31)];
        float b1 = sm.b[kk + (lane >> 5)][wn + 32 + (lane & 31)];
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kc = 0; kc < BK / 8; kc += 2) {
        const int c = kc + (lane >> 5);
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ah[i] = *reinterpret_cast<const bf16x8*>(&sm.ahi[c][swz(wm + 32 * i + (lane & 31), c)][0]);
          al[i] = *reinterpret_cast<const bf16x8*>(&sm.alo[c][swz(wm + 32 * i + (lane & 31), c)][0]);
          bh[i] = *reinterpret_cast<const bf16x8*>(&sm.bhi[c][swz(wn + 32 * i + (lane & 31), c)][0]);
          bl[i] = *reinterpret_cast<const bf16x8*>(&sm.blo[c][swz(wn + 32 * i + (lane & 31), c)][0]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }
}

template <int MODE, bool AKC, bool BKC>
__global__ __launch_bounds__(NT) void gemm_mfma_kernel(GemmDesc g, int splits, int kchunk, float* __restrict__ partial,
                                                      TileMap tm, int fast_ok) {
  __shared__ Smem<MODE> sm;

  int tx, ty, bz;
  if (!map_tile(tm, tx, ty, bz)) return;
  {  // launch-group member: outermost index
    const int per = g.batch * splits, mem = bz / per;
    bz -= mem * per;
    g.A = member_ptr(g.A, g, mem); g.B = member_ptr(g.B, g, mem); g.C = member_ptr(g.C, g, mem);
    g.skip = member_ptr(g.skip, g, mem);
    partial = member_ptr(partial, g, mem);
  }
  if (g.skip && gload(g.skip)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  const int b = bz / splits, sp = bz - b * splits;
  const int m0 = ty * BM, n0 = tx * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  OpView va{(const float*)g.A + batch_offset(g, b, g.sAb, g.sAb2), g.sAm, g.sAk, g.sAk1, g.M, g.K2};
  OpView vb{(const float*)g.B + batch_offset(g, b, g.sBb, g.sBb2), g.sBn, g.sBk, g.sBk1, g.N, g.K2};

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const bool fast = fast_ok && m0 + BM <= g.M && n0 + BN <= g.N;
  kloop<MODE, AKC, BKC>(sm, va, vb, m0, n0, kbeg, kend, acc, tid, fast);

  // epilogue: lane l, register r of block (i, j) holds
  // row wm + 32 i + 8 (r / 4) + 4 (l / 32) + r % 4, column wn + 32 j + l % 32
  const int col_l = lane & 31, rowq = (lane >> 5) * 4;
  if (splits == 1) {
    float* C = (float*)g.C + batch_offset(g, b, g.sCb, g.sCb2);
    const float alpha = (float)g.alpha, beta = (float)g.beta;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int n = n0 + wn + 32 * j + col_l;
        if (n >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int m = m0 + wm + 32 * i + 8 * (r >> 2) + rowq + (r & 3);
          if (m >= g.M) continue;
          float* c = C + (long long)m * g.sCm + (long long)n * g.sCn;
          float v = alpha * acc[i][j][r];
          if (g.beta != 0.0) v += beta * gload(c);
          gstore(c, v);
        }
      }
  } else {
    float* P = partial + ((long long)sp * g.batch + b) * (long long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int n = n0 + wn + 32 * j + col_l;
        if (n >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int m = m0 + wm + 32 * i + 8 * (r >> 2) + rowq + (r & 3);
          if (m >= g.M) continue;
          gstore(P + (long long)m * g.N + n, acc[i][j][r]);
        }
      }
  }
}


// ---------------------------------------------------------------------------
// float64: v_mfma_f64_16x16x4_f64, 128 x 128 tile, BK = 16, 2 x 2 waves of
// 64 x 64 (4 x 4 blocks of 16 x 16).  Lane l of a block holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 r][l % 16].
// ---------------------------------------------------------------------------
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int BK64 = 16;

struct OpView64 {
  const double* base;
  long long s_mn, s_k, s_k1;
  int MN, K2;
};
__device__ __forceinline__ long long k_offset64(const OpView64& v, int k) {
  if (v.K2 <= 0) return (long long)k * v.s_k;
  int k1 = k / v.K2;
  return (long long)k1 * v.s_k1 + (long long)(k - k1 * v.K2) * v.s_k;
}

template <bool KC, int T>
struct Stage64 {
  static constexpr int NV = (T * BK64) / (2 * NT);  // double2 per thread (4 at T = 128, 2 at T = 64)
  f64x2 r[NV];
  __device__ __forceinline__ void load(const OpView64& v, int mn0, int k0, int kend, int tid) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int f = tid + i * NT;
      int mn, k;
      if constexpr (KC) { mn = f / (BK64 / 2); k = (f % (BK64 / 2)) * 2; }
      else              { k = f / (T / 2); mn = (f % (T / 2)) * 2; }
      int gm = mn0 + mn, gk = k0 + k;
      if (gm < v.MN && gk < kend) {
        const double* p = KC ? v.base + (long long)gm * v.s_mn + k_offset64(v, gk) : v.base + gm + k_offset64(v, gk);
        r[i] = gload(reinterpret_cast<const f64x2*>(p));
      } else {
        r[i] = f64x2{0.0, 0.0};
      }
    }
  }
  __device__ __forceinline__ void store(double (*pl)[T + 2], int tid) const {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int f = tid + i * NT;
      if constexpr (KC) {
        int mn = f / (BK64 / 2), k = (f % (BK64 / 2)) * 2;
        pl[k][mn] = r[i][0];
        pl[k + 1][mn] = r[i][1];
      } else {
        int k = f / (T / 2), mn = (f % (T / 2)) * 2;
        *reinterpret_cast<f64x2*>(&pl[k][mn]) = r[i];
      }
    }
  }
};

// T x T output tile per 256-thread work-group, 2 x 2 waves of T/2 x T/2 as
// (T/32) x (T/32) blocks of 16 x 16.  T = 128 for large products; T = 64
// gives small products four times the work-groups at a quarter of the
// registers per wave.
template <bool AKC, bool BKC, int T>
__global__ __launch_bounds__(NT) void gemm_mfma64_kernel(GemmDesc g, int splits, int kchunk, double* __restrict__ partial,
                                                        TileMap tm) {
  constexpr int NBK = T / 32;  // 16 x 16 blocks per wave and dimension
  __shared__ double sa_l[BK64][T + 2];
  __shared__ double sb_l[BK64][T + 2];
  int tx, ty, bz;
  if (!map_tile(tm, tx, ty, bz)) return;
  {  // launch-group member: outermost index
    const int per = g.batch * splits, mem = bz / per;
    bz -= mem * per;
    g.A = member_ptr(g.A, g, mem); g.B = member_ptr(g.B, g, mem); g.C = member_ptr(g.C, g, mem);
    g.skip = member_ptr(g.skip, g, mem);
    partial = member_ptr(partial, g, mem);
  }
  if (g.skip && gload(g.skip)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (T / 2), wn = (wave >> 1) * (T / 2);
  const int b = bz / splits, sp = bz - b * splits;
  const int m0 = ty * T, n0 = tx * T;
  const int kbeg = sp * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  OpView64 va{(const double*)g.A + batch_offset(g, b, g.sAb, g.sAb2), g.sAm, g.sAk, g.sAk1, g.M, g.K2};
  OpView64 vb{(const double*)g.B + batch_offset(g, b, g.sBb, g.sBb2), g.sBn, g.sBk, g.sBk1, g.N, g.K2};
  f64x4 acc[NBK][NBK];
#pragma unroll
  for (int i = 0; i < NBK; ++i)
#pragma unroll
    for (int j = 0; j < NBK; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  Stage64<AKC, T> sa;
  Stage64<BKC, T> sb;
  if (kbeg < kend) {
    sa.load(va, m0, kbeg, kend, tid);
    sb.load(vb, n0, kbeg, kend, tid);
  }
  for (int k0 = kbeg; k0 < kend; k0 += BK64) {
    sa.store(sa_l, tid);
    sb.store(sb_l, tid);
    __syncthreads();
    if (k0 + BK64 < kend) {
      sa.load(va, m0, k0 + BK64, kend, tid);
      sb.load(vb, n0, k0 + BK64, kend, tid);
    }
#pragma unroll
    for (int kk = 0; kk < BK64; kk += 4) {
      double a[NBK], bv[NBK];
#pragma unroll
      for (int i = 0; i < NBK; ++i) a[i] = sa_l[kk + (lane >> 4)][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NBK; ++j) bv[j] = sb_l[kk + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < NBK; ++i)
#pragma unroll
        for (int j = 0; j < NBK; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const int col_l = lane & 15, row_l = lane >> 4;
  if (splits == 1) {
    double* C = (double*)g.C + batch_offset(g, b, g.sCb, g.sCb2);
#pragma unroll
    for (int i = 0; i < NBK; ++i)
#pragma unroll
      for (int j = 0; j < NBK; ++j) {
        int n = n0 + wn + 16 * j + col_l;
        if (n >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int m = m0 + wm + 16 * i + row_l + 4 * r;
          if (m >= g.M) continue;
          double* c = C + (long long)m * g.sCm + (long long)n * g.sCn;
          double v = g.alpha * acc[i][j][r];
          if (g.beta != 0.0) v += g.beta * gload(c);
          gstore(c, v);
        }
      }
  } else {
    double* P = partial + ((long long)sp * g.batch + b) * (long long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < NBK; ++i)
#pragma unroll
      for (int j = 0; j < NBK; ++j) {
        int n = n0 + wn + 16 * j + col_l;
        if (n >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int m = m0 + wm + 16 * i + row_l + 4 * r;
          if (m >= g.M) continue;
          gstore(P + (long long)m * g.N + n, acc[i][j][r]);
        }
      }
  }
}

template <bool AKC, bool BKC, int T>
hipError_t launch64(const GemmDesc& g, int splits, int kchunk, double* partial, hipStream_t s, int orient) {
  const TileMap tm = make_map((g.N + T - 1) / T, (g.M + T - 1) / T, g.batch * splits * gemm_members(g), orient);
  size_t slot = 0;
  KernelTimer* kt = kernel_timer();
  const double work = (double)g.batch * gemm_members(g);
  const int kid = (T == 128 ? KID_MFMA64 : KID_MFMA64S) + 2 * AKC + BKC;
  const bool timed = kt && kt->begin(kid, 2.0 * g.M * (double)g.N * g.K * work,
                                     8.0 * work * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N), s, &slot);
  hipLaunchKernelGGL((gemm_mfma64_kernel<AKC, BKC, T>), dim3(N_XCD * tm.per), dim3(NT), 0, s, g, splits, kchunk,
                     partial, tm);
  if (timed) kt->end(slot, s);
  return hipGetLastError();
}

template <int MODE, bool AKC, bool BKC>
hipError_t launch(const GemmDesc& g, int splits, int kchunk, float* partial, hipStream_t s, int orient) {
  const TileMap tm = make_map((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch * splits * gemm_members(g), orient);
  size_t slot = 0;
  KernelTimer* kt = kernel_timer();
  const double work = (double)g.batch * gemm_members(g);
  const bool timed = kt && kt->begin(KID_MFMA + 4 * (MODE - 1) + 2 * AKC + BKC, 2.0 * g.M * (double)g.N * g.K * work,
                                     4.0 * work * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N), s, &slot);
  constexpr int BK = Cfg<MODE>::BK;
  // every chunk of BK contraction indices lies inside one block of the
  // two-level index (kchunk is a multiple of BK)
  const int fast_ok = (g.K % BK == 0) && (g.K2 <= 0 || g.K2 % BK == 0);
  hipLaunchKernelGGL((gemm_mfma_kernel<MODE, AKC, BKC>), dim3(N_XCD * tm.per), dim3(NT), 0, s, g, splits, kchunk,
                     partial, tm, fast_ok);
  if (timed) kt->end(slot, s);
  return hipGetLastError();
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

// Split-K count of a product: a function of its shape, batch and arithmetic
// only (never of a tuned choice, of the launch group or of timing), so that a
// product is summed in the same order wherever and however it is launched.
// Products with few output tiles (counted at the tile `tile`) and a long
// contraction are split for about 1024 work-groups, each slice at least
// 4 BK deep, at most 128 slices and what the scratch holds.
static int split_count(const GemmDesc& g, int tile, int bk, size_t elem, size_t scratch_bytes, int* kchunk) {
  const long long tiles = (long long)((g.M + tile - 1) / tile) * ((g.N + tile - 1) / tile) * g.batch;
  int splits = 1;
  if (tiles < 1024) {
    long long want = (1024 + tiles - 1) / tiles;
    long long maxk = g.K / (4 * bk);
    long long sps = want < maxk ? want : maxk;
    const size_t slice = (size_t)g.batch * g.M * g.N * elem;
    const long long fit = (long long)(scratch_bytes / slice);
    if (sps > fit) sps = fit;
    if (sps > 128) sps = 128;
    splits = sps < 1 ? 1 : (int)sps;
  }
  int kc = (g.K + splits - 1) / splits;
  kc = ((kc + bk - 1) / bk) * bk;
  splits = (g.K + kc - 1) / kc;
  *kchunk = kc;
  return splits < 1 ? 1 : splits;
}

// Returns hipErrorNotSupported when the shape/layout does not fit the MFMA
// loaders (caller falls back to the general kernel).
static hipError_t gemm_mfma64(const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s,
                              const GemmLaunch& how) {
  if (g.M < 32 || g.N < 32 || g.K < 16 || g.batch < 1) return hipErrorNotSupported;
  const bool akc = (g.sAk == 1), bkc = (g.sBk == 1);
  const bool amc = (g.sAm == 1), bmc = (g.sBn == 1);
  if (!(akc || amc) || !(bkc || bmc)) return hipErrorNotSupported;
  if (!aligned16(g.A) || !aligned16(g.B)) return hipErrorNotSupported;
  if (g.sAb % 2 || g.sBb % 2 || g.sAb2 % 2 || g.sBb2 % 2) return hipErrorNotSupported;
  if (akc) { if (g.K % 2 || g.sAm % 2 || (g.K2 > 0 && (g.K2 % 2 || g.sAk1 % 2))) return hipErrorNotSupported; }
  else     { if (g.M % 2 || g.sAk % 2 || (g.K2 > 0 && g.sAk1 % 2)) return hipErrorNotSupported; }
  if (bkc) { if (g.K % 2 || g.sBn % 2 || (g.K2 > 0 && (g.K2 % 2 || g.sBk1 % 2))) return hipErrorNotSupported; }
  else     { if (g.N % 2 || g.sBk % 2 || (g.K2 > 0 && g.sBk1 % 2)) return hipErrorNotSupported; }
  // small products (few 128 x 128 tiles) and short contractions (K <= 2048:
  // four work-groups per CU hide each tile's loads and stores, which a short
  // k loop cannot) take 64 x 64 tiles by default.  Both tiles issue the same
  // MFMA sequence for every output element, so the tile is a launch choice
  // only; the split count follows the default tile.
  const int T0 = ((long long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch < 64 || g.K <= 2048) ? 64 : 128;
  int kchunk = 0;
  const int splits = split_count(g, T0, BK64, sizeof(double), scratch_bytes, &kchunk);
  const int T = how.tile == 64 || how.tile == 128 ? how.tile : T0;
  double* partial = (double*)scratch;
  const int o = how.orient;
  hipError_t e;
  if (T == 64) {
    if (akc && bkc) e = launch64<true, true, 64>(g, splits, kchunk, partial, s, o);
    else if (akc) e = launch64<true, false, 64>(g, splits, kchunk, partial, s, o);
    else if (bkc) e = launch64<false, true, 64>(g, splits, kchunk, partial, s, o);
    else e = launch64<false, false, 64>(g, splits, kchunk, partial, s, o);
  } else {
    if (akc && bkc) e = launch64<true, true, 128>(g, splits, kchunk, partial, s, o);
    else if (akc) e = launch64<true, false, 128>(g, splits, kchunk, partial, s, o);
    else if (bkc) e = launch64<false, true, 128>(g, splits, kchunk, partial, s, o);
    else e = launch64<false, false, 128>(g, splits, kchunk, partial, s, o);
  }
  if (e != hipSuccess) return e;
  if (splits > 1) return splitk_reduce_f64(g, splits, partial, s);
  return hipSuccess;
}

hipError_t gemm_mfma(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s,
                     const GemmLaunch& how) {
  if (prec == P_F64) return gemm_mfma64(g, scratch, scratch_bytes, s, how);
  if (prec != P_F32 && prec != P_BF16X3) return hipErrorNotSupported;
  if (g.M < 32 || g.N < 32 || g.K < 16 || g.batch < 1) return hipErrorNotSupported;
  const int BK = (prec == P_F32) ? 16 : 32;
  const bool akc = (g.sAk == 1), bkc = (g.sBk == 1);
  const bool amc = (g.sAm == 1), bmc = (g.sBn == 1);
  if (!(akc || amc) || !(bkc || bmc)) return hipErrorNotSupported;
  if (!aligned16(g.A) || !aligned16(g.B)) return hipErrorNotSupported;
  if (g.sAb % 4 || g.sBb % 4 || g.sAb2 % 4 || g.sBb2 % 4) return hipErrorNotSupported;
  // contiguous extents and the other strides must keep float4 alignment
  if (akc) { if (g.K % 4 || g.sAm % 4 || (g.K2 > 0 && (g.K2 % 4 || g.sAk1 % 4))) return hipErrorNotSupported; }
  else     { if (g.M % 4 || g.sAk % 4 || (g.K2 > 0 && g.sAk1 % 4)) return hipErrorNotSupported; }
  if (bkc) { if (g.K % 4 || g.sBn % 4 || (g.K2 > 0 && (g.K2 % 4 || g.sBk1 % 4))) return hipErrorNotSupported; }
  else     { if (g.N % 4 || g.sBk % 4 || (g.K2 > 0 && g.sBk1 % 4)) return hipErrorNotSupported; }
  int kchunk = 0;
  const int splits = split_count(g, BM, BK, sizeof(float), scratch_bytes, &kchunk);
  float* partial = (float*)scratch;
  const int o = how.orient;
  hipError_t e;
  if (prec == P_F32) {
    if (akc && bkc) e = launch<P_F32, true, true>(g, splits, kchunk, partial, s, o);
    else if (akc) e = launch<P_F32, true, false>(g, splits, kchunk, partial, s, o);
    else if (bkc) e = launch<P_F32, false, true>(g, splits, kchunk, partial, s, o);
    else e = launch<P_F32, false, false>(g, splits, kchunk, partial, s, o);
  } else {
    if (akc && bkc) e = launch<P_BF16X3, true, true>(g, splits, kchunk, partial, s, o);
    else if (akc) e = launch<P_BF16X3, true, false>(g, splits, kchunk, partial, s, o);
    else if (bkc) e = launch<P_BF16X3, false, true>(g, splits, kchunk, partial, s, o);
    else e = launch<P_BF16X3, false, false>(g, splits, kchunk, partial, s, o);
  }
  if (e != hipSuccess) return e;
  if (splits > 1) return splitk_reduce_f32(g, splits, partial, s);
  return hipSuccess;
}

}  // namespace ttn
