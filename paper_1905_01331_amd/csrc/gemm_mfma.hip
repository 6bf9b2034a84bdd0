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
  int gx, gy, gz, per, yfast, tri;
};
constexpr int N_XCD = 8;
__device__ __forceinline__ bool map_tile(const TileMap& t, int& tx, int& ty, int& tz) {
  const int id = blockIdx.x;
  const long long L = (long long)(id % N_XCD) * t.per + id / N_XCD;
  if (t.tri) {
    // the block upper triangle (ty <= tx) of a gx x gx tile grid, row by row
    const int T = t.gx, ntri = T * (T + 1) / 2;
    if (L >= (long long)ntri * t.gz) return false;
    int r = (int)(L % ntri);
    tz = (int)(L / ntri);
    int row = 0;
    while (r >= T - row) { r -= T - row; ++row; }
    ty = row;
    tx = row + r;
    return true;
  }
  if (L >= (long long)t.gx * t.gy * t.gz) return false;
  const int l = (int)L;
  if (t.yfast) { ty = l % t.gy; const int r = l / t.gy; tx = r % t.gx; tz = r / t.gx; }
  else { tx = l % t.gx; const int r = l / t.gx; ty = r % t.gy; tz = r / t.gy; }
  return true;
}
// orient: 0 the smaller tile dimension fastest, 1 x fastest, 2 y fastest
// (a launch-shape choice: the tiles compute the same values in any order)
TileMap make_map(int gx, int gy, int gz, int orient, bool tri = false) {
  TileMap t;
  t.gx = gx; t.gy = gy; t.gz = gz;
  t.tri = tri ? 1 : 0;
  const long long total = tri ? (long long)gx * (gx + 1) / 2 * gz : (long long)gx * gy * gz;
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
// float64: v_mfma_f64_4x4x4_4b_f64, four independent 4 x 4 x 4 products per
// instruction.  On gfx950 this form runs at about 0.9 of the float64 peak in
// a loop of independent products, against about 0.6 for the 16 x 16 x 4
// form, so every float64 product uses it.  Lane layout (measured with
// one-hot operands): lane l holds A_b[l % 4][l / 16] and B_b[l / 16][l % 4]
// of block b = (l / 4) % 4 and receives D_b[l / 16][l % 4].  The four blocks
// are stacked along M, so one instruction multiplies a 16 x 4 slice of A by
// a 4 x 4 slice of B: lane l reads A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 4], and its result is C[4 ((l / 4) % 4) + l / 16][l % 4].
// A wave owns RI x RJ such units (16 RI rows, 4 RJ columns), 2 x 2 waves a
// work-group.  BK = 16 contraction indices per LDS chunk, two LDS buffers
// (one barrier per chunk).  Every tile issues the same instruction sequence
// for an output element, so the tile is a launch choice only.
// ---------------------------------------------------------------------------
typedef double f64x2 __attribute__((ext_vector_type(2)));
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

// tile t: 0 64 x 64 (RI 2, RJ 8), 1 128 x 64 (RI 4, RJ 8), 2 64 x 128 (RI 2, RJ 16)
template <int TILE> struct Tile64;
template <> struct Tile64<0> { static constexpr int RI = 2, RJ = 8; };
template <> struct Tile64<1> { static constexpr int RI = 4, RJ = 8; };
template <> struct Tile64<2> { static constexpr int RI = 2, RJ = 16; };

// Register staging of one operand tile (MN x BK64 doubles): float64 pairs
// along k (contraction-contiguous) or along mn (output-contiguous), written
// to LDS as [k][mn].
template <bool KC, int MN>
struct Stage64 {
  static constexpr int NV = (MN * BK64) / (2 * NT);
  f64x2 r[NV];
  __device__ __forceinline__ void load(const OpView64& v, int mn0, int k0, int kend, int tid) {
    // a two-level contraction index whose inner extent is a multiple of the
    // chunk: the chunk lies in one outer block, whose offset is computed once
    const bool blk = v.K2 > 0 && (v.K2 % BK64) == 0;
    long long kbase = 0;
    if (blk) {
      const int k1 = k0 / v.K2;
      kbase = (long long)k1 * v.s_k1 + (long long)(k0 - k1 * v.K2) * v.s_k;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int f = tid + i * NT;
      int mn, k;
      if constexpr (KC) { mn = f / (BK64 / 2); k = (f % (BK64 / 2)) * 2; }
      else              { k = f / (MN / 2); mn = (f % (MN / 2)) * 2; }
      int gm = mn0 + mn, gk = k0 + k;
      if (gm < v.MN && gk < kend) {
        const long long ko = blk ? kbase + (long long)k * v.s_k : k_offset64(v, gk);
        const double* p = KC ? v.base + (long long)gm * v.s_mn + ko : v.base + gm + ko;
        r[i] = gload(reinterpret_cast<const f64x2*>(p));
      } else {
        r[i] = f64x2{0.0, 0.0};
      }
    }
  }
  __device__ __forceinline__ void store(double (*pl)[MN + 2], int tid) const {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int f = tid + i * NT;
      if constexpr (KC) {
        int mn = f / (BK64 / 2), k = (f % (BK64 / 2)) * 2;
        pl[k][mn] = r[i][0];
        pl[k + 1][mn] = r[i][1];
      } else {
        int k = f / (MN / 2), mn = (f % (MN / 2)) * 2;
        *reinterpret_cast<f64x2*>(&pl[k][mn]) = r[i];
      }
    }
  }
};

template <bool AKC, bool BKC, int TILE>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(GemmDesc g, int splits, int kchunk, double* __restrict__ partial,
                                                     TileMap tm) {
  constexpr int RI = Tile64<TILE>::RI, RJ = Tile64<TILE>::RJ;
  constexpr int WM = 16 * RI, WN = 4 * RJ, TM = 2 * WM, TN = 2 * WN;
  __shared__ double sa_l[2][BK64][TM + 2];
  __shared__ double sb_l[2][BK64][TN + 2];
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
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const int b = bz / splits, sp = bz - b * splits;
  const int m0 = ty * TM, n0 = tx * TN;
  const int kbeg = sp * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  OpView64 va{(const double*)g.A + batch_offset(g, b, g.sAb, g.sAb2), g.sAm, g.sAk, g.sAk1, g.M, g.K2};
  OpView64 vb{(const double*)g.B + batch_offset(g, b, g.sBb, g.sBb2), g.sBn, g.sBk, g.sBk1, g.N, g.K2};
  double acc[RI][RJ];
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) acc[i][j] = 0.0;
  Stage64<AKC, TM> sa;
  Stage64<BKC, TN> sb;
  const int lk = lane >> 4, la = lane & 15, lbn = lane & 3;
  if (kbeg < kend) {
    sa.load(va, m0, kbeg, kend, tid);
    sb.load(vb, n0, kbeg, kend, tid);
    sa.store(sa_l[0], tid);
    sb.store(sb_l[0], tid);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK64) {
    const bool more = k0 + BK64 < kend;
    if (more) {
      sa.load(va, m0, k0 + BK64, kend, tid);
      sb.load(vb, n0, k0 + BK64, kend, tid);
    }
#pragma unroll
    for (int kk = 0; kk < BK64; kk += 4) {
      double av[RI], bv[RJ];
#pragma unroll
      for (int i = 0; i < RI; ++i) av[i] = sa_l[buf][kk + lk][wm + 16 * i + la];
#pragma unroll
      for (int j = 0; j < RJ; ++j) bv[j] = sb_l[buf][kk + lk][wn + 4 * j + lbn];
#pragma unroll
      for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      sa.store(sa_l[buf ^ 1], tid);
      sb.store(sb_l[buf ^ 1], tid);
    }
    __syncthreads();
    buf ^= 1;
  }
  // lane l's result of unit (i, j): row wm + 16 i + 4 ((l / 4) % 4) + l / 16,
  // column wn + 4 j + l % 4
  const int row_l = 4 * ((lane >> 2) & 3) + lk;
  if (splits == 1) {
    double* C = (double*)g.C + batch_offset(g, b, g.sCb, g.sCb2);
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int m = m0 + wm + 16 * i + row_l;
      if (m >= g.M) continue;
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const int n = n0 + wn + 4 * j + lbn;
        if (n >= g.N) continue;
        double* c = C + (long long)m * g.sCm + (long long)n * g.sCn;
        double v = g.alpha * acc[i][j];
        if (g.beta != 0.0) v += g.beta * gload(c);
        gstore(c, v);
      }
    }
  } else {
    double* P = partial + ((long long)sp * g.batch + b) * (long long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int m = m0 + wm + 16 * i + row_l;
      if (m >= g.M) continue;
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const int n = n0 + wn + 4 * j + lbn;
        if (n < g.N) gstore(P + (long long)m * g.N + n, acc[i][j]);
      }
    }
  }
}

template <bool AKC, bool BKC, int TILE>
hipError_t launch64(const GemmDesc& g, int splits, int kchunk, double* partial, hipStream_t s, int orient) {
  constexpr int TM = 32 * Tile64<TILE>::RI, TN = 8 * Tile64<TILE>::RJ;
  const bool tri = g.tri != 0 && TM == TN && g.M == g.N;
  const TileMap tm = make_map((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, g.batch * splits * gemm_members(g), orient,
                              tri);
  size_t slot = 0;
  KernelTimer* kt = kernel_timer();
  const int T = (g.N + TN - 1) / TN;
  // work of the tiles computed (a triangle counts its share of the square)
  const double work = (double)g.batch * gemm_members(g) * (tri ? (double)(T + 1) / (2.0 * T) : 1.0);
  const int kid = KID_F64 + 4 * TILE + 2 * AKC + BKC;
  const bool timed = kt && kt->begin(kid, 2.0 * g.M * (double)g.N * g.K * work,
                                     8.0 * work * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N), s, &slot);
  hipLaunchKernelGGL((gemm_f64_kernel<AKC, BKC, TILE>), dim3(N_XCD * tm.per), dim3(NT), 0, s, g, splits, kchunk,
                     partial, tm);
  if (timed) kt->end(slot, s);
  return hipGetLastError();
}

template <bool AKC, bool BKC>
hipError_t launch64_tile(int tile, const GemmDesc& g, int splits, int kchunk, double* partial, hipStream_t s,
                         int orient) {
  if (tile == 1) return launch64<AKC, BKC, 1>(g, splits, kchunk, partial, s, orient);
  if (tile == 2) return launch64<AKC, BKC, 2>(g, splits, kchunk, partial, s, orient);
  return launch64<AKC, BKC, 0>(g, splits, kchunk, partial, s, orient);
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

// C[i][j] = sign C[j][i] for the strictly lower tiles (i / tile > j / tile)
// of every batch entry and member of a product computed on its block upper
// triangle; sign -1 for the entries whose bit is set in g.anti.
__global__ void k_mirror_lower(GemmDesc g, int tile) {
  const int n = g.M;
  const long long nn = (long long)n * n;
  const int b = blockIdx.y % g.batch, mem = blockIdx.y / g.batch;
  if (g.skip && gload(member_ptr(g.skip, g, mem))) return;
  double* C = (double*)member_ptr(g.C, g, mem) + batch_offset(g, b, g.sCb, g.sCb2);
  const int bi = g.batch1 > 0 ? b % g.batch1 : b;
  const double sign = (bi < 64 && ((g.anti >> bi) & 1ull)) ? -1.0 : 1.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nn;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx - (long long)i * n);
    if (i / tile <= j / tile) continue;
    gstore(C + (long long)i * g.sCm + (long long)j * g.sCn, sign * gload(C + (long long)j * g.sCm + (long long)i * g.sCn));
  }
}

hipError_t mirror_lower_f64(const GemmDesc& g, int tile, hipStream_t s) {
  const long long nn = (long long)g.M * g.M;
  int blocks = (int)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(k_mirror_lower, dim3(blocks, g.batch * gemm_members(g)), dim3(256), 0, s, g, tile);
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
static int split_count(const GemmDesc& g, int tile, int bk, size_t elem, size_t scratch_bytes, int* kchunk,
                       bool tri = false) {
  const long long tm = (g.M + tile - 1) / tile, tn = (g.N + tile - 1) / tile;
  const long long tiles = (tri ? tm * (tm + 1) / 2 : tm * tn) * g.batch;
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
  // the split count follows the shape alone (counted at 64 x 64 tiles); the
  // tile (64 x 64 by default) is a launch choice
  // a symmetric (antisymmetric) square output: the 64 x 64 tiles of the
  // block upper triangle, then the mirror (with beta != 0 the old C is read
  // on the upper triangle only; the caller's C has the output's parity)
  const bool tri = g.tri != 0 && g.M == g.N;
  GemmDesc gt = g;
  gt.tri = tri ? 1 : 0;
  int kchunk = 0;
  const int splits = split_count(g, 64, BK64, sizeof(double), scratch_bytes, &kchunk, tri);
  const int tile = tri ? 0 : (how.tile >= 1 && how.tile <= 3 ? how.tile - 1 : 0);
  double* partial = (double*)scratch;
  const int o = how.orient;
  hipError_t e;
  if (akc && bkc) e = launch64_tile<true, true>(tile, gt, splits, kchunk, partial, s, o);
  else if (akc) e = launch64_tile<true, false>(tile, gt, splits, kchunk, partial, s, o);
  else if (bkc) e = launch64_tile<false, true>(tile, gt, splits, kchunk, partial, s, o);
  else e = launch64_tile<false, false>(tile, gt, splits, kchunk, partial, s, o);
  if (e != hipSuccess) return e;
  if (splits > 1 && (e = splitk_reduce_f64(gt, splits, partial, s)) != hipSuccess) return e;
  if (tri) return mirror_lower_f64(gt, 64, s);
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
