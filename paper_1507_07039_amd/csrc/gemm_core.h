// Device building blocks of the similarity GEMMs: operand tile loaders, the
// block-level MFMA main loops (FP32 and split-BF16), and the stream-K driver
// shared by every rectangular product.
//
// Every similarity of the method is T(X, Y)_ij = (XY)_ij / sqrt(|X_i.|^2 +
// |Y_.j|^2 - |(XY)_ij|) (Eq. 1), which Sec. II-C recasts as one matrix product
// followed by an element-wise step on row and column norms (Eq. 9).  The
// product runs on matrix cores; the element-wise step (and whatever update
// rule consumes the similarity) is the epilogue of the same kernel.
//
// Operands are zero-padded to tile multiples by the host, so main loops have
// no bounds checks; zero rows and columns add nothing to products.  The
// rectangular products share one tile schedule (whole tiles in full rounds,
// the remainder split stream-K style), described at k_rect_streamk.
#pragma once

#include <type_traits>

#include "panda_internal.h"

namespace panda {
namespace gemm {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Logical number for block b of an n-block grid: contiguous chunks per XCD.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t xcd = b & 7, slot = b >> 3;
  const int64_t q = n >> 3, r = n & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// (I, J) with I <= J for upper-triangular tile number u = J(J+1)/2 + I.
__device__ __forceinline__ void tri_tile(int64_t u, int64_t& I, int64_t& J) {
  int64_t j = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > u) --j;
  while ((j + 1) * (j + 2) / 2 <= u) ++j;
  J = j;
  I = u - j * (j + 1) / 2;
}

// Eq. 1 from the product and the two squared norms (FP64); T := 0 when the
// denominator vanishes (both vectors zero).
__device__ __forceinline__ double tanimoto(double dot, double xx, double yy) {
  const double den = xx + yy - fabs(dot);
  return den > 0.0 ? dot / sqrt(den) : 0.0;
}

// Deterministic sum of one double per thread over the block (at most 8
// waves); red holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// bf16 of x rounded to nearest even, as raw bits.
__device__ __forceinline__ bf16_t to_bf16(float x) {
  return __builtin_bit_cast(bf16_t, (__bf16)x);
}
__device__ __forceinline__ float from_bf16(bf16_t b) {
  return (float)__builtin_bit_cast(__bf16, b);
}
// x = hi + lo + O(2^-17 |x|): hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ void split_bf16(float x, bf16_t& hi, bf16_t& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - from_bf16(hi));
}

// ======================================================== FP32 main loop ==
// One operand's MN x BK tile: global -> registers -> LDS.  KC: the operand
// is contiguous along k in global memory (element (mn, k) at base[mn*ld+k]);
// otherwise along mn (element at base[k*ld + mn]).  The LDS copy is always
// [k][mn] with row length LD, the layout the MFMA operand reads want (32
// consecutive mn per half-wave).  LD is padded so that the transposing
// stores of the KC case hit every bank equally often.
template <int MN, bool KC, int BK>
struct TileLoad {
  static constexpr int NV = MN * BK / 4 / kThreads;  // float4 per thread
  static constexpr int KQ = BK / 4;                  // KC: threads per mn-row
  static constexpr int RP = kThreads / KQ;           // KC: mn-rows per pass
  static constexpr int TPR = MN / 4;                 // !KC: threads per k-row
  static constexpr int RPP = kThreads / TPR;         // !KC: k-rows per pass
  static constexpr int LD = KC ? MN + (BK == 32 ? 2 : 4) : MN + 4;
  static_assert(NV >= 1, "tile too small for one float4 per thread");
  static_assert(KC ? (RP * NV == MN) : (RPP * NV == BK), "loads must cover the tile");

  f4 v[NV];

  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int64_t mn0,
                                       int64_t k0, int t) {
    if constexpr (KC) {
      const int kq = (t % KQ) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = t / KQ + i * RP;
        v[i] = *reinterpret_cast<const f4*>(base + (mn0 + mn) * ld + k0 + kq);
      }
    } else {
      const int mnq = (t % TPR) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int k = t / TPR + i * RPP;
        v[i] = *reinterpret_cast<const f4*>(base + (k0 + k) * ld + mn0 + mnq);
      }
    }
  }

  __device__ __forceinline__ void store(float* lds, int t) const {
    if constexpr (KC) {
      const int kq = (t % KQ) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = t / KQ + i * RP;
        lds[(kq + 0) * LD + mn] = v[i].x;
        lds[(kq + 1) * LD + mn] = v[i].y;
        lds[(kq + 2) * LD + mn] = v[i].z;
        lds[(kq + 3) * LD + mn] = v[i].w;
      }
    } else {
      const int mnq = (t % TPR) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int k = t / TPR + i * RPP;
        *reinterpret_cast<f4*>(lds + k * LD + mnq) = v[i];
      }
    }
  }
};

// FP32 operands: X element (m, k) = XK ? X[m*ldx + k] : X[k*ldx + m];
// Y element (k, n) = YK ? Y[n*ldy + k] : Y[k*ldy + n].
struct OpsF32 {
  const float* X;
  int64_t ldx;
  const float* Y;
  int64_t ldy;
};

// Block-level FP32 GEMM over k in [kbeg, kend) for a BM x BN tile with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) sub-tile of 32 x 32 MFMA blocks
// (v_mfma_f32_32x32x2f32).
template <int BM_, int BN_, int WM, int WN, bool XK, bool YK, int BK_>
struct BlockGemm {
  using Ops = OpsF32;
  static constexpr int BM = BM_, BN = BN_, BK = BK_, NT = kThreads;
  static constexpr int WAVES_PER_EU = 1;  // occupancy asked of the compiler (1: no request)
  static_assert(WM * WN == 4, "four waves per block");
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static_assert(TM >= 1 && TN >= 1, "wave tile below one MFMA block");
  using LX = TileLoad<BM, XK, BK>;
  using LY = TileLoad<BN, YK, BK>;
  static constexpr int XS = BK * LX::LD;
  static constexpr int YS = BK * LY::LD;
  static constexpr int MAIN_BYTES = 2 * (XS + YS) * 4;

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  __device__ __forceinline__ void run(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg,
                                      int64_t kend, char* smem) {
    const int t = threadIdx.x;
    lane = t & 63;
    const int w = t >> 6;
    wm = w % WM;
    wn = w / WM;
    float* xs = reinterpret_cast<float*>(smem);
    float* ys = xs + 2 * XS;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    LX lx;
    LY ly;
    const int64_t nk = (kend - kbeg) / BK;
    if (nk > 0) {
      lx.load(o.X, o.ldx, m0, kbeg, t);
      ly.load(o.Y, o.ldy, n0, kbeg, t);
      lx.store(xs, t);
      ly.store(ys, t);
    }
    __syncthreads();
    const int mrow = wm * (BM / WM) + (lane & 31);
    const int ncol = wn * (BN / WN) + (lane & 31);
    const int khalf = lane >> 5;
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = (int)(kt & 1);
      const bool more = kt + 1 < nk;
      if (more) {
        lx.load(o.X, o.ldx, m0, kbeg + (kt + 1) * BK, t);
        ly.load(o.Y, o.ldy, n0, kbeg + (kt + 1) * BK, t);
      }
      const float* xc = xs + cur * XS;
      const float* yc = ys + cur * YS;
#pragma unroll
      for (int kk = 0; kk < BK / 2; ++kk) {
        const int kr = 2 * kk + khalf;
        float a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = xc[kr * LX::LD + mrow + i * 32];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = yc[kr * LY::LD + ncol + j * 32];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_iglp_opt(0);  // interleave LDS reads with the MFMAs
      }
      if (more) {
        lx.store(xs + (cur ^ 1) * XS, t);
        ly.store(ys + (cur ^ 1) * YS, t);
      }
      __syncthreads();
    }
  }

  // Local (row, col) in the block tile of accumulator register r of MFMA
  // block (i, j): the 32x32 result layout puts column lane%32 in each lane
  // and rows 8*(r/4) + 4*(lane/32) + r%4.
  __device__ __forceinline__ int row_of(int i, int r) const {
    return wm * (BM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
  __device__ __forceinline__ int col_of(int j) const {
    return wn * (BN / WN) + j * 32 + (lane & 31);
  }
  template <class F>
  __device__ __forceinline__ void for_each(F&& f) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = col_of(j);
#pragma unroll
        for (int r = 0; r < 16; ++r) f(row_of(i, r), c, acc[i][j][r]);
      }
  }
};

// ================================================== split-BF16 main loop ==
// Both operands are stored K-contiguous as two bf16 planes (hi, lo) with
// x = hi + lo: X_hi/X_lo[m][k] and Yt_hi/Yt_lo[n][k] (Yt = Y transposed).
// Each product is hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 with an
// FP32 accumulator; the dropped lo*lo term and the rounding of lo bound the
// relative error of each product term by about 2^-16.
struct OpsB3 {
  const bf16_t* Xh;
  const bf16_t* Xl;
  int64_t ldx;
  const bf16_t* Yh;
  const bf16_t* Yl;
  int64_t ldy;
};
// The same with Y an FP32 symmetric matrix (Yt = Y, rows read K-contiguous)
// that is split into hi/lo while it is staged.
struct OpsB3F {
  const bf16_t* Xh;
  const bf16_t* Xl;
  int64_t ldx;
  const float* Y;
  int64_t ldy;
};

// MN x BK tile of one K-contiguous operand, both planes, loaded by NT
// threads.  LDS rows are BK bf16 (chunks of 8 bf16 = 16 B) with the chunk
// index XOR-swizzled by the row's bank group, so the 16 rows one
// ds_read_b128 group touches land in distinct banks.
template <int MN, int NT, int BK_>
struct TileLoadB3 {
  static constexpr int BK = BK_;
  static constexpr int CPR = BK / 8;        // 16-byte chunks per row and plane
  static constexpr int RP = NT / CPR;       // rows per pass
  static constexpr int NV = MN >= RP ? MN / RP : 1;  // chunks per thread and plane
  static constexpr bool ALL = MN >= RP;     // every thread loads (else t < MN * CPR)
  static constexpr int PLANE = MN * BK;     // bf16 per plane in LDS
  static constexpr int RG = 64 / (BK / 2);  // rows sharing a bank offset
  static_assert(ALL ? RP * NV == MN : RP % MN == 0, "loads must cover the tile");

  u4 h[NV], l[NV];

  __device__ __forceinline__ static int swz(int row, int chunk) {
    return row * BK + ((chunk ^ ((row / RG) & (CPR - 1))) << 3);
  }
  __device__ __forceinline__ void load(const bf16_t* __restrict__ H, const bf16_t* __restrict__ L,
                                       int64_t ld, int64_t mn0, int64_t k0, int t) {
    if (!ALL && t >= MN * CPR) return;
    const int c = (t % CPR) * 8;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int r = t / CPR + i * RP;
      h[i] = *reinterpret_cast<const u4*>(H + (mn0 + r) * ld + k0 + c);
      l[i] = *reinterpret_cast<const u4*>(L + (mn0 + r) * ld + k0 + c);
    }
  }
  __device__ __forceinline__ void store(bf16_t* lds, int t) const {
    if (!ALL && t >= MN * CPR) return;
    const int c = t % CPR;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int r = t / CPR + i * RP;
      *reinterpret_cast<u4*>(lds + swz(r, c)) = h[i];
      *reinterpret_cast<u4*>(lds + PLANE + swz(r, c)) = l[i];
    }
  }
};

// MN x BK tile of a K-contiguous FP32 operand (row mn = mn0 + r holds k
// values k0..), split into the two planes of the TileLoadB3 layout when it is
// written to LDS.
template <int MN, int NT, int BK_>
struct TileLoadB3F {
  using Planes = TileLoadB3<MN, NT, BK_>;
  static constexpr int BK = BK_, CPR = Planes::CPR, RP = Planes::RP, NV = Planes::NV;
  static constexpr bool ALL = Planes::ALL;
  static constexpr int PLANE = Planes::PLANE;
  __device__ __forceinline__ static int swz(int row, int chunk) { return Planes::swz(row, chunk); }

  f4 a[NV], b[NV];
  int64_t mn0, k0;

  __device__ __forceinline__ void load(const float* __restrict__ M, int64_t ld, int64_t mn0_,
                                       int64_t k0_, int t) {
    mn0 = mn0_;
    k0 = k0_;
    if (!ALL && t >= MN * CPR) return;
    const int c = (t % CPR) * 8;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int r = t / CPR + i * RP;
      const float* p = M + (mn0 + r) * ld + k0 + c;
      a[i] = *reinterpret_cast<const f4*>(p);
      b[i] = *reinterpret_cast<const f4*>(p + 4);
    }
  }
  __device__ __forceinline__ void store(bf16_t* lds, int t) const {
    if (!ALL && t >= MN * CPR) return;
    const int c = t % CPR;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int r = t / CPR + i * RP;
      const float v[8] = {a[i].x, a[i].y, a[i].z, a[i].w, b[i].x, b[i].y, b[i].z, b[i].w};
      unsigned hw[4], lw[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bf16_t h0, l0, h1, l1;
        split_bf16(v[2 * e], h0, l0);
        split_bf16(v[2 * e + 1], h1, l1);
        hw[e] = (unsigned)h0 | ((unsigned)h1 << 16);
        lw[e] = (unsigned)l0 | ((unsigned)l1 << 16);
      }
      const int off = Planes::swz(r, c);
      *reinterpret_cast<u4*>(lds + off) = u4{hw[0], hw[1], hw[2], hw[3]};
      *reinterpret_cast<u4*>(lds + PLANE + off) = u4{lw[0], lw[1], lw[2], lw[3]};
    }
  }
};

// Block-level split-BF16 GEMM, WM x WN waves of (BM/WM) x (BN/WN) each.
// All fragments of a K-tile are read from LDS before its MFMAs are issued,
// so the LDS latency is paid once per tile rather than once per 16-k step.
template <int BM_, int BN_, int WM, int WN, int BK_ = 32, bool YF32 = false, int WPE = 1>
struct BlockGemmB3 {
  using Ops = typename std::conditional<YF32, OpsB3F, OpsB3>::type;
  static constexpr int BM = BM_, BN = BN_, BK = BK_, NT = 64 * WM * WN;
  static constexpr int WAVES_PER_EU = WPE;  // occupancy asked of the compiler (1: no request)
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int KS = BK / 16;  // MFMA k-steps per K-tile
  static_assert(TM >= 1 && TN >= 1, "wave tile below one MFMA block");
  using LX = TileLoadB3<BM, NT, BK>;
  using LY = typename std::conditional<YF32, TileLoadB3F<BN, NT, BK>, TileLoadB3<BN, NT, BK>>::type;
  static constexpr int XS = 2 * LX::PLANE;  // bf16 per stage
  static constexpr int YS = 2 * LY::PLANE;
  static constexpr int MAIN_BYTES = 2 * (XS + YS) * 2;

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  __device__ __forceinline__ static void load_y(LY& ly, const Ops& o, int64_t n0, int64_t k0,
                                                int t) {
    if constexpr (YF32)
      ly.load(o.Y, o.ldy, n0, k0, t);
    else
      ly.load(o.Yh, o.Yl, o.ldy, n0, k0, t);
  }

  __device__ __forceinline__ void run(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg,
                                      int64_t kend, char* smem) {
    const int t = threadIdx.x;
    lane = t & 63;
    const int w = t >> 6;
    wm = w % WM;
    wn = w / WM;
    bf16_t* xs = reinterpret_cast<bf16_t*>(smem);
    bf16_t* ys = xs + 2 * XS;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    LX lx;
    LY ly;
    const int64_t nk = (kend - kbeg) / BK;
    if (nk > 0) {
      lx.load(o.Xh, o.Xl, o.ldx, m0, kbeg, t);
      load_y(ly, o, n0, kbeg, t);
      lx.store(xs, t);
      ly.store(ys, t);
    }
    __syncthreads();
    const int mrow = wm * (BM / WM) + (lane & 31);
    const int ncol = wn * (BN / WN) + (lane & 31);
    const int khalf = lane >> 5;
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = (int)(kt & 1);
      const bool more = kt + 1 < nk;
      if (more) {
        lx.load(o.Xh, o.Xl, o.ldx, m0, kbeg + (kt + 1) * BK, t);
        load_y(ly, o, n0, kbeg + (kt + 1) * BK, t);
      }
      const bf16_t* xc = xs + cur * XS;
      const bf16_t* yc = ys + cur * YS;
      bf16x8 xh[KS][TM], xl[KS][TM], yh[KS][TN], yl[KS][TN];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int chunk = 2 * ks + khalf;  // this lane's 8 k-values of the 16-k step
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int off = LX::swz(mrow + i * 32, chunk);
          xh[ks][i] = *reinterpret_cast<const bf16x8*>(xc + off);
          xl[ks][i] = *reinterpret_cast<const bf16x8*>(xc + LX::PLANE + off);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int off = LY::swz(ncol + j * 32, chunk);
          yh[ks][j] = *reinterpret_cast<const bf16x8*>(yc + off);
          yl[ks][j] = *reinterpret_cast<const bf16x8*>(yc + LY::PLANE + off);
        }
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ks][i], yl[ks][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[ks][i], yh[ks][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ks][i], yh[ks][j], acc[i][j], 0, 0, 0);
          }
      if (more) {
        lx.store(xs + (cur ^ 1) * XS, t);
        ly.store(ys + (cur ^ 1) * YS, t);
      }
      __syncthreads();
    }
  }

  __device__ __forceinline__ int row_of(int i, int r) const {
    return wm * (BM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
  __device__ __forceinline__ int col_of(int j) const {
    return wn * (BN / WN) + j * 32 + (lane & 31);
  }
  template <class F>
  __device__ __forceinline__ void for_each(F&& f) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = col_of(j);
#pragma unroll
        for (int r = 0; r < 16; ++r) f(row_of(i, r), c, acc[i][j][r]);
      }
  }
};

// ============================================ pipelined split-BF16 loop ==
// The same products with the operand tiles moved by direct global -> LDS
// loads (global_load_lds_dwordx4: lane l of a wave writes its 16 bytes at
// LDS base + 16 l), so STAGES - 1 K-tiles are in flight without holding
// registers.  Which global chunk each lane fetches is chosen so that the LDS
// image is the swizzled layout the fragment reads want:
//   bf16 planes: rows of BK bf16, slot s of row r holds chunk s ^ f(r) (as
//     TileLoadB3);
//   FP32 rows (Y = a symmetric FP32 matrix, split at fragment-read time):
//     rows of BK floats = BK/4 chunks, slot s of row r holds chunk s ^ (r % 8).
typedef __attribute__((address_space(3))) void* lds_vptr;
typedef __attribute__((address_space(1))) void* gbl_vptr;

__device__ __forceinline__ void dma16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds((gbl_vptr)g, (lds_vptr)lds, 16, 0, 0);
}

// Wait until at most n vector-memory operations of this wave are pending
// (gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14; exp and lgkm counts left at
// their maxima, i.e. not waited for).
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <int BM_, int BN_, int WM, int WN, int STAGES, bool YF32>
struct BlockGemmB3D {
  using Ops = typename std::conditional<YF32, OpsB3F, OpsB3>::type;
  static constexpr int BM = BM_, BN = BN_, BK = 32, NT = 64 * WM * WN;
  static constexpr int WAVES = WM * WN;
  static constexpr int WAVES_PER_EU = 1;
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int KS = BK / 16;
  static_assert(TM >= 1 && TN >= 1 && STAGES >= 2, "shape");
  using PX = TileLoadB3<BM, NT, BK>;  // swizzle of the bf16 planes
  using PY = TileLoadB3<BN, NT, BK>;
  static constexpr int CPR = BK / 8;                        // 16-byte chunks per bf16 row
  static constexpr int XQ = BM * CPR;                       // chunks per X plane
  static constexpr int YQ = YF32 ? BN * (BK / 4) : BN * CPR;  // chunks per Y plane (1 or 2 planes)
  static constexpr int YPLANES = YF32 ? 1 : 2;
  static constexpr int STAGE_BYTES = (2 * XQ + YPLANES * YQ) * 16;
  static constexpr int MAIN_BYTES = 16;  // the stages are run()'s own LDS objects
  static constexpr int XI = 2 * XQ / 64, YI = YPLANES * YQ / 64;  // wave-instructions per stage
  static_assert((2 * XQ) % 64 == 0 && (YPLANES * YQ) % 64 == 0, "whole wave loads");
  static_assert((XI + YI) % WAVES == 0, "loads split evenly over the waves");
  static constexpr int IPW = (XI + YI) / WAVES;  // loads per wave and stage

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  // Issue the loads of K-tile k0 into stage buffer st (this wave's share).
  __device__ __forceinline__ void issue(const Ops& o, int64_t m0, int64_t n0, int64_t k0,
                                       char* st, int w) const {
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
      const int ins = w + q * WAVES;  // wave-instruction index within the stage
      const int pos = (ins % (XI + YI) < XI ? ins : ins - XI) * 64 + lane;
      if (ins < XI) {
        const int plane = pos / XQ, p = pos % XQ;
        const int r = p / CPR, slot = p % CPR;
        const int chunk = slot ^ ((r / PX::RG) & (CPR - 1));
        const bf16_t* src = (plane ? o.Xl : o.Xh) + (m0 + r) * o.ldx + k0 + chunk * 8;
        dma16(src, st + (size_t)ins * 1024);
      } else {
        char* dst = st + 2 * XQ * 16 + (size_t)(ins - XI) * 1024;
        if constexpr (YF32) {
          const int r = pos / (BK / 4), slot = pos % (BK / 4);
          const int chunk = slot ^ (r & 7);
          dma16(o.Y + (n0 + r) * o.ldy + k0 + chunk * 4, dst);
        } else {
          const int plane = pos / YQ, p = pos % YQ;
          const int r = p / CPR, slot = p % CPR;
          const int chunk = slot ^ ((r / PY::RG) & (CPR - 1));
          dma16((plane ? o.Yl : o.Yh) + (n0 + r) * o.ldy + k0 + chunk * 8, dst);
        }
      }
    }
  }

  template <int N>
  __device__ __forceinline__ static void wait_ahead(int ahead) {
    // pending loads allowed: `ahead` later stages of IPW loads each
    if constexpr (N <= 0) {
      wait_vmem<0>();
    } else {
      if (ahead >= N) {
        wait_vmem<N * IPW>();
      } else {
        wait_ahead<N - 1>(ahead);
      }
    }
  }

  // LDS byte address of a generic pointer into shared memory.
  __device__ __forceinline__ static unsigned lds_addr(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char*)p;
  }

  __device__ __forceinline__ void compute(const char* st, int64_t n0, int64_t k0) {
    static_assert(YF32 && KS == 2 && TM == 2 && (TN == 1 || TN == 2), "fragment reads written for these shapes");
    constexpr int PER = 2 * TM + 2 * TN;  // fragments per k-step
    constexpr int NR = KS * PER;
    const int mrow = wm * (BM / WM) + (lane & 31);
    const int khalf = lane >> 5;
    const unsigned base = lds_addr(st);
    const unsigned ybase = base + 2 * XQ * 16;
    unsigned ad[NR];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int chunk = 2 * ks + khalf;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const unsigned off = 2u * PX::swz(mrow + i * 32, chunk);
        ad[PER * ks + 2 * i] = base + off;
        ad[PER * ks + 2 * i + 1] = base + 2u * BM * BK + off;
      }
      const int c0 = 4 * ks + 2 * khalf;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * (BN / WN) + j * 32 + (lane & 31);
        ad[PER * ks + 2 * TM + 2 * j] = ybase + 4u * (n * BK + ((c0 ^ (n & 7)) << 2));
        ad[PER * ks + 2 * TM + 2 * j + 1] = ybase + 4u * (n * BK + (((c0 + 1) ^ (n & 7)) << 2));
      }
    }
    // All reads of the K-tile in one block that waits for them before it
    // ends, so no read is left in flight when its result is used.
    u4 r[NR];
    if constexpr (NR == 12) {
      asm volatile(
          "ds_read_b128 %0, %12\n\tds_read_b128 %1, %13\n\tds_read_b128 %2, %14\n\t"
          "ds_read_b128 %3, %15\n\tds_read_b128 %4, %16\n\tds_read_b128 %5, %17\n\t"
          "ds_read_b128 %6, %18\n\tds_read_b128 %7, %19\n\tds_read_b128 %8, %20\n\t"
          "ds_read_b128 %9, %21\n\tds_read_b128 %10, %22\n\tds_read_b128 %11, %23\n\t"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
            "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11])
          : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]), "v"(ad[6]),
            "v"(ad[7]), "v"(ad[8]), "v"(ad[9]), "v"(ad[10]), "v"(ad[11]));
    } else {
      asm volatile(
          "ds_read_b128 %0, %16\n\tds_read_b128 %1, %17\n\tds_read_b128 %2, %18\n\t"
          "ds_read_b128 %3, %19\n\tds_read_b128 %4, %20\n\tds_read_b128 %5, %21\n\t"
          "ds_read_b128 %6, %22\n\tds_read_b128 %7, %23\n\tds_read_b128 %8, %24\n\t"
          "ds_read_b128 %9, %25\n\tds_read_b128 %10, %26\n\tds_read_b128 %11, %27\n\t"
          "ds_read_b128 %12, %28\n\tds_read_b128 %13, %29\n\tds_read_b128 %14, %30\n\t"
          "ds_read_b128 %15, %31\n\ts_waitcnt lgkmcnt(0)"
          : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
            "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11]),
            "=&v"(r[12]), "=&v"(r[13]), "=&v"(r[14]), "=&v"(r[15])
          : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]), "v"(ad[6]),
            "v"(ad[7]), "v"(ad[8]), "v"(ad[9]), "v"(ad[10]), "v"(ad[11]), "v"(ad[12]),
            "v"(ad[13]), "v"(ad[14]), "v"(ad[15]));
    }
    bf16x8 xh[KS][TM], xl[KS][TM], yh[KS][TN], yl[KS][TN];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        xh[ks][i] = __builtin_bit_cast(bf16x8, r[PER * ks + 2 * i]);
        xl[ks][i] = __builtin_bit_cast(bf16x8, r[PER * ks + 2 * i + 1]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const f4 a = __builtin_bit_cast(f4, r[PER * ks + 2 * TM + 2 * j]);
        const f4 b = __builtin_bit_cast(f4, r[PER * ks + 2 * TM + 2 * j + 1]);
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const __bf16 h = (__bf16)v[e];
          yh[ks][j][e] = h;
          yl[ks][j][e] = (__bf16)(v[e] - (float)h);
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ks][i], yl[ks][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[ks][i], yh[ks][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ks][i], yh[ks][j], acc[i][j], 0, 0, 0);
        }
  }

  // One K-tile step: wait for stage `cur`, release stage `nxt`, start its
  // loads (tile kt + STAGES - 1), compute on `cur`.  Stages are distinct
  // LDS objects so that the compiler can tell the loads in flight from the
  // stage being read and does not wait for them.
  __device__ __forceinline__ void step(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg,
                                       int kt, int nk, char* cur, char* nxt, int w) {
    const int ahead = nk - 1 - kt < STAGES - 2 ? nk - 1 - kt : STAGES - 2;
    wait_ahead<STAGES - 2>(ahead);
    // Every wave has waited for its own loads of stage kt; the barrier alone
    // (no memory fence, which would wait for the later stages too) makes
    // stage kt complete for all and stage kt-1 free (its reads fed MFMAs).
    __builtin_amdgcn_s_barrier();
    if (kt + STAGES - 1 < nk) issue(o, m0, n0, kbeg + (int64_t)(kt + STAGES - 1) * BK, nxt, w);
    compute(cur, n0, kbeg + (int64_t)kt * BK);
  }

  __device__ __forceinline__ void run(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg,
                                      int64_t kend, char*) {
    static_assert(STAGES == 3, "three stage buffers");
    __shared__ __align__(16) char s0[STAGE_BYTES];
    __shared__ __align__(16) char s1[STAGE_BYTES];
    __shared__ __align__(16) char s2[STAGE_BYTES];
    const int t = threadIdx.x;
    lane = t & 63;
    const int w = t >> 6;
    wm = w % WM;
    wn = w / WM;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int nk = (int)((kend - kbeg) / BK);
    wait_vmem<0>();   // only this tile's loads are counted below
    __syncthreads();  // the previous tile's reads of every stage are done
    if (nk > 0) issue(o, m0, n0, kbeg, s0, w);
    if (nk > 1) issue(o, m0, n0, kbeg + BK, s1, w);
    int kt = 0;
    for (; kt + 3 <= nk; kt += 3) {
      step(o, m0, n0, kbeg, kt, nk, s0, s2, w);
      step(o, m0, n0, kbeg, kt + 1, nk, s1, s0, w);
      step(o, m0, n0, kbeg, kt + 2, nk, s2, s1, w);
    }
    if (kt < nk) step(o, m0, n0, kbeg, kt, nk, s0, s2, w);
    if (kt + 1 < nk) step(o, m0, n0, kbeg, kt + 1, nk, s1, s0, w);
  }

  __device__ __forceinline__ int row_of(int i, int r) const {
    return wm * (BM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
  __device__ __forceinline__ int col_of(int j) const {
    return wn * (BN / WN) + j * 32 + (lane & 31);
  }
  template <class F>
  __device__ __forceinline__ void for_each(F&& f) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = col_of(j);
#pragma unroll
        for (int r = 0; r < 16; ++r) f(row_of(i, r), c, acc[i][j][r]);
      }
  }
};

// ======================================================= tile schedule ==
// A grid of nb blocks (as many as the GPU runs at once) covers nTiles output
// tiles of U K-steps each in two parts:
//   full rounds: with R = nTiles / nb, block L computes tiles L, L + nb, ...,
//     L + (R-1) nb whole.  Consecutive tiles (M fastest, sharing a strip of
//     the Y operand) run on one XCD at the same time, so that strip is
//     fetched from memory about once per round.
//   tail: the remaining nTiles - R nb tiles are split stream-K style over the
//     first nbt <= nb blocks (at most kTailSplit blocks per tile, so the
//     fix-up sums few partials): block L < nbt owns items
//     [L*total/nbt, (L+1)*total/nbt) of their total = tail * U K-steps;
//     tiles finished inside one block get their epilogue at once, tiles
//     shared by blocks are summed in block order by the fix-up kernel
//     (deterministic; no block ever waits for another).
// Logical block numbers are assigned XCD by XCD (the hardware hands block b to
// XCD b % 8), so one XCD works on contiguous tiles.
__device__ __forceinline__ int64_t sk_begin(int64_t L, int64_t total, int64_t G) {
  return L * total / G;
}
// Logical block whose tail range holds item i (the largest L with begin <= i).
__device__ __forceinline__ int64_t sk_owner(int64_t i, int64_t total, int64_t G) {
  return ((i + 1) * G - 1) / total;
}

constexpr int64_t kTailSplit = 4;

template <class G, class Epi>
__global__ __launch_bounds__(G::NT) __attribute__((amdgpu_waves_per_eu(G::WAVES_PER_EU)))
void k_rect_streamk(typename G::Ops ops, int64_t nMT,
                                                        int64_t nTiles, int64_t U, int64_t nbt,
                                                        Epi epi, float* __restrict__ part,
                                                        const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[G::MAIN_BYTES];
  __shared__ double red[8];
  const int64_t nb = gridDim.x;
  const int64_t L = xcd_tile(blockIdx.x, nb);
  const int64_t R = nTiles / nb, nFull = R * nb;
  G g;
  for (int64_t r = 0; r < R; ++r) {
    const int64_t tile = r * nb + L;
    const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
    g.run(ops, m0, n0, 0, U * G::BK, smem);
    g.for_each([&](int rr, int c, float v) { epi.element(m0 + rr, n0 + c, v); });
    epi.end_tile(tile, red);
  }
  if (L >= nbt) return;
  const int64_t total = (nTiles - nFull) * U;
  const int64_t b = sk_begin(L, total, nbt), e = sk_begin(L + 1, total, nbt);
  int64_t it = b;
  while (it < e) {
    const int64_t tt = it / U;  // tail tile
    const int64_t k0 = it - tt * U;
    const int64_t k1 = (e - tt * U < U) ? e - tt * U : U;
    const int64_t tile = nFull + tt;
    const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
    g.run(ops, m0, n0, k0 * G::BK, k1 * G::BK, smem);
    if (k0 == 0 && k1 == U) {
      g.for_each([&](int rr, int c, float v) { epi.element(m0 + rr, n0 + c, v); });
      epi.end_tile(tile, red);
    } else {
      float* ps = part + (2 * L + (it == b ? 0 : 1)) * (int64_t)(G::BM * G::BN);
      g.for_each([&](int rr, int c, float v) { ps[rr * G::BN + c] = v; });
    }
    it = tt * U + k1;
  }
}

// Tail tiles whose K-steps were split between blocks: sum the partial
// products in block order (deterministic) and run the same epilogue.
template <class G, class Epi>
__global__ __launch_bounds__(kThreads) void k_rect_fixup(int64_t nMT, int64_t nTiles, int64_t U,
                                                         int64_t nb, int64_t nbt,
                                                         const float* __restrict__ part, Epi epi,
                                                         const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[8];
  const int64_t nFull = (nTiles / nb) * nb;
  const int64_t tile = nFull + blockIdx.x;
  if (tile >= nTiles) return;
  const int64_t tt = tile - nFull;
  const int64_t total = (nTiles - nFull) * U;
  const int64_t lo = sk_owner(tt * U, total, nbt), hi = sk_owner((tt + 1) * U - 1, total, nbt);
  if (lo == hi) return;  // finished inside one block
  const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
  constexpr int E = G::BM * G::BN;
  for (int e = threadIdx.x; e < E; e += kThreads) {
    float s = 0.0f;
    for (int64_t L = lo; L <= hi; ++L) {
      const int64_t bL = sk_begin(L, total, nbt);
      if (bL == sk_begin(L + 1, total, nbt)) continue;  // empty range
      const int64_t slot = 2 * L + ((L == lo && bL < tt * U) ? 1 : 0);
      s += part[slot * E + e];
    }
    epi.element(m0 + e / G::BN, n0 + e % G::BN, s);
  }
  epi.end_tile(tile, red);
}

// Blocks of kernel `fn` (nt threads each) the whole GPU runs at once.
inline int64_t resident_blocks(const void* fn, int nt = kThreads) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, nt, 0) != hipSuccess || occ <= 0)
    occ = 1;
  return (int64_t)cus * occ;
}

// Launch of a rectangular product over an Mp x Np output with K = Kp; part
// holds 2 * kMaxStreamKBlocks tiles of split-tile scratch.
template <class G, class Epi>
hipError_t launch_rect(const typename G::Ops& ops, int64_t Mp, int64_t Np, int64_t Kp, Epi epi,
                       float* part, const int32_t* gate, hipStream_t s) {
  static int64_t resident = 0;
  if (!resident)
    resident = resident_blocks(reinterpret_cast<const void*>(&k_rect_streamk<G, Epi>), G::NT);
  const int64_t nMT = Mp / G::BM, nNT = Np / G::BN;
  const int64_t nTiles = nMT * nNT, U = Kp / G::BK;
  int64_t nb = resident;
  if (nb > kMaxStreamKBlocks) nb = kMaxStreamKBlocks;
  if (nb > nTiles) nb = nTiles;
  const int64_t tail = nTiles - (nTiles / nb) * nb;
  const int64_t nbt = tail * kTailSplit < nb ? tail * kTailSplit : nb;
  k_rect_streamk<G, Epi><<<dim3((unsigned)nb), dim3(G::NT), 0, s>>>(ops, nMT, nTiles, U, nbt, epi,
                                                                     part, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tail == 0) return hipSuccess;
  k_rect_fixup<G, Epi><<<dim3((unsigned)tail), dim3(kThreads), 0, s>>>(nMT, nTiles, U, nb, nbt,
                                                                       part, epi, gate);
  return hipGetLastError();
}

}  // namespace gemm
}  // namespace panda
