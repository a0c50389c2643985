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
// The quotient is taken as dot times 1/sqrt(den): the hardware estimate
// (about 2^-23 relative) refined by one Newton step, which squares its error
// (about 1e-14 relative, far under the FP32 rounding of every result), for a
// few FMAs instead of a double divide and square root per entry.
// Computed without a branch (den <= 0 selects 0 after the fact), so that
// runs of entries compile to straight-line code.
__device__ __forceinline__ double tanimoto(double dot, double xx, double yy) {
  const double den = xx + yy - fabs(dot);
  const double y0 = __builtin_amdgcn_rsq(den);
  const double y1 = y0 * (1.5 - 0.5 * den * y0 * y0);
  return den > 0.0 ? dot * y1 : 0.0;
}

// Deterministic sum of one double per thread over the block; red holds one
// double per wave.
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
// The same with Y a packed symmetric matrix (packed_tile).
struct OpsF32P {
  const float* X;
  int64_t ldx;
  const float* Yp;
};

// Y tile (MN = kPT columns, BK rows) of a product whose Y is a packed
// symmetric matrix: element (k, n) = Y[k][n], n in column block J = n0 / kPT.
// For k in block Kb <= J, tile (Kb, J) holds it at row k, column n (n
// contiguous, TileLoad<MN, false>'s pattern); for Kb > J, tile (J, Kb) holds
// it at row n, column k (k contiguous, TileLoad<MN, true>'s pattern).  A
// K-tile lies inside one block (BK divides kPT), so the orientation is chosen
// per K-tile, the same for the whole block; both fill the same [k][mn] LDS
// layout.
template <int MN, int BK>
struct TileLoadPY {
  using LN = TileLoad<MN, false, BK>;
  using LT = TileLoad<MN, true, BK>;
  static_assert(MN == kPT && kPT % BK == 0, "one packed column block per tile");
  static_assert(LN::LD == LT::LD && LN::NV == LT::NV, "one LDS layout for both orientations");
  static constexpr int LD = LN::LD;
  static constexpr int NV = LN::NV;
  f4 v[NV];
  bool tr;

  __device__ __forceinline__ void load(const float* __restrict__ Yp, int64_t n0, int64_t k0, int t) {
    const int64_t J = n0 / kPT, Kb = k0 / kPT, kk = k0 % kPT;
    tr = Kb > J;
    if (!tr) {
      const float* base = Yp + packed_tile(Kb, J) * (kPT * kPT) + kk * kPT;
      const int mnq = (t % LN::TPR) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int k = t / LN::TPR + i * LN::RPP;
        v[i] = *reinterpret_cast<const f4*>(base + k * kPT + mnq);
      }
    } else {
      const float* base = Yp + packed_tile(J, Kb) * (kPT * kPT) + kk;
      const int kq = (t % LT::KQ) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = t / LT::KQ + i * LT::RP;
        v[i] = *reinterpret_cast<const f4*>(base + mn * kPT + kq);
      }
    }
  }

  __device__ __forceinline__ void store(float* lds, int t) const {
    if (!tr) {
      const int mnq = (t % LN::TPR) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int k = t / LN::TPR + i * LN::RPP;
        *reinterpret_cast<f4*>(lds + k * LD + mnq) = v[i];
      }
    } else {
      const int kq = (t % LT::KQ) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = t / LT::KQ + i * LT::RP;
        lds[(kq + 0) * LD + mn] = v[i].x;
        lds[(kq + 1) * LD + mn] = v[i].y;
        lds[(kq + 2) * LD + mn] = v[i].z;
        lds[(kq + 3) * LD + mn] = v[i].w;
      }
    }
  }
};

// Block-level FP32 GEMM over k in [kbeg, kend) for a BM x BN tile with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) sub-tile of 32 x 32 MFMA blocks
// (v_mfma_f32_32x32x2f32).  YP: Y is a packed symmetric matrix (OpsF32P).
template <int BM_, int BN_, int WM, int WN, bool XK, bool YK, int BK_, bool YP = false>
struct BlockGemm {
  using Ops = typename std::conditional<YP, OpsF32P, OpsF32>::type;
  static constexpr int BM = BM_, BN = BN_, BK = BK_, NT = kThreads;
  static constexpr int WAVES_PER_EU = 1;  // occupancy asked of the compiler (1: no request)
  static_assert(WM * WN == 4, "four waves per block");
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static_assert(TM >= 1 && TN >= 1, "wave tile below one MFMA block");
  using LX = TileLoad<BM, XK, BK>;
  using LY = typename std::conditional<YP, TileLoadPY<BN, BK>, TileLoad<BN, YK, BK>>::type;
  __device__ __forceinline__ static void load_y(LY& ly, const Ops& o, int64_t n0, int64_t k0,
                                                int t) {
    if constexpr (YP)
      ly.load(o.Yp, n0, k0, t);
    else
      ly.load(o.Y, o.ldy, n0, k0, t);
  }
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
        lx.load(o.X, o.ldx, m0, kbeg + (kt + 1) * BK, t);
        load_y(ly, o, n0, kbeg + (kt + 1) * BK, t);
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
  int64_t mrows = INT64_MAX;  // rows of X that exist (loaders may clamp to them)
};
// The same with Y an FP32 symmetric matrix (Yt = Y, rows read K-contiguous)
// that is split into hi/lo while it is staged.
struct OpsB3F {
  const bf16_t* Xh;
  const bf16_t* Xl;
  int64_t ldx;
  const float* Y;
  int64_t ldy;
  int64_t mrows = INT64_MAX;  // rows of X that exist (loaders may clamp to them)
};
// ... with Y stored packed (packed_tile).
struct OpsB3FP {
  const bf16_t* Xh;
  const bf16_t* Xl;
  int64_t ldx;
  const float* Yp;
  int64_t mrows = INT64_MAX;
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

// Block-level split-BF16 GEMM, WM x WN waves of (BM/WM) x (BN/WN) each.
// All fragments of a K-tile are read from LDS before its MFMAs are issued,
// so the LDS latency is paid once per tile rather than once per 16-k step.
template <int BM_, int BN_, int WM, int WN, int BK_ = 32, int WPE = 1>
struct BlockGemmB3 {
  using Ops = OpsB3;
  static constexpr bool kBlockEpi = true;  // epilogue entries in runs of 8
  static constexpr int BM = BM_, BN = BN_, BK = BK_, NT = 64 * WM * WN;
  static constexpr int WAVES_PER_EU = WPE;  // occupancy asked of the compiler (1: no request)
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int KS = BK / 16;  // MFMA k-steps per K-tile
  static_assert(TM >= 1 && TN >= 1, "wave tile below one MFMA block");
  using LX = TileLoadB3<BM, NT, BK>;
  using LY = TileLoadB3<BN, NT, BK>;
  static constexpr int XS = 2 * LX::PLANE;  // bf16 per stage
  static constexpr int YS = 2 * LY::PLANE;
  static constexpr int MAIN_BYTES = 2 * (XS + YS) * 2;

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  __device__ __forceinline__ static void load_y(LY& ly, const Ops& o, int64_t n0, int64_t k0,
                                                int t) {
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

// =============================== software-pipelined split-BF16 loop ==
// A x C with A given as bf16 hi/lo planes and C as FP32 (split into hi/lo
// as its fragments are read; C is symmetric, so its row n is the column the
// product needs).  Operand tiles move by direct global -> LDS loads
// (global_load_lds_dwordx4: lane l of a wave writes its 16 bytes at LDS base
// + 16 l) into STAGES (two or three) stages, so STAGES - 1 K-tiles are in
// flight without holding registers.  Which global chunk a lane fetches is chosen so that the LDS
// image is swizzled for conflict-free fragment reads:
//   bf16 planes: rows of BK bf16, slot s of row r holds chunk s ^ f(r) (as
//     TileLoadB3);
//   FP32 rows: BK floats = BK / 4 chunks, slot s of row r holds chunk
//     s ^ yswz(r), so the 16 rows one read touches at a time cover all 64
//     banks.
// The loop is also software-pipelined in registers: while the matrix cores
// work on K-tile k, the wave issues the loads of K-tile k + STAGES, reads
// the fragments of K-tile k + 1 from LDS and splits them.
//
// The direct loads are issued from inline assembly (no register results;
// the LDS base goes through M0), so the compiler's own LDS reads are not
// held back for them; ordering is explicit instead: every wave waits for its
// own loads of a stage (vmcnt), then a barrier that is also a compiler
// memory barrier makes the stage complete for all waves.  A stage is
// refilled only after the barrier that follows its last reads.
__device__ __forceinline__ void lds_dma16(unsigned voff, const void* sbase, unsigned ldsa) {
  // the base and the LDS address are wave-uniform; say so, so that they sit
  // in scalar registers whatever the compiler concluded about them
  // (the builtin returns a signed int: widen through unsigned, or a low half
  // with bit 31 set would be sign-extended into the high half)
  const uint64_t b = (uint64_t)sbase;
  const uint64_t lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const uint64_t hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  const uint64_t bs = lo | (hi << 32);
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(voff), "s"(bs), "s"(__builtin_amdgcn_readfirstlane(ldsa))
               : "memory", "m0");
}
// Barrier after this wave's LDS reads have completed (so no read of a stage
// can still be pending when another wave refills it); also a compiler
// memory barrier.
__device__ __forceinline__ void wave_barrier_mem() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Wait until at most n vector-memory operations of this wave are pending
// (gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14; exp and lgkm counts left at
// their maxima, i.e. not waited for).
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// hi = RNE(a), lo = RNE(a - hi) for two floats at once (packed bf16 pairs).
__device__ __forceinline__ void split_pair(float a, float b, unsigned& h, unsigned& l) {
  typedef float fl2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bh2 __attribute__((ext_vector_type(2)));
  h = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){a, b}, bh2));
  const float ha = __builtin_bit_cast(float, h << 16);
  const float hb = __builtin_bit_cast(float, h & 0xffff0000u);
  l = __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){a - ha, b - hb}, bh2));
}

// YF32: Y is the FP32 symmetric matrix split as its fragments are read;
// otherwise Y is given as bf16 hi/lo planes like X (no split arithmetic).
// The STAGES stage buffers are carved from the caller's shared memory.
// YP: Y (FP32) is stored packed (packed_tile).  The product needs row n of Y
// over the K-tile's k (Y symmetric: row n is column n).  Where the tile of
// (n, k) lies above the diagonal it holds that row directly; below it, the
// tile of (k, n) holds it as a column, so such a K-tile is loaded as it is
// stored, [k][n] rows of kPT floats, and its fragments are read with one
// 4-byte read per k.  Both rows of a fragment read's two half-waves differ
// by 8 in k, and their 16-byte chunks are XOR-swizzled by that bit, so the
// two half-waves use different banks.
template <int BM_, int BN_, int WM, int WN, bool YF32 = true, int STAGES = 3, int BK_ = 32,
          bool YP = false>
struct BlockGemmB3P {
  using Ops = typename std::conditional<
      YP, OpsB3FP, typename std::conditional<YF32, OpsB3F, OpsB3>::type>::type;
  static_assert(!YP || (YF32 && BN_ == (int)kPT && kPT % BK_ == 0 && BK_ == 32),
                "packed Y: FP32 rows of one packed column block, K-tiles inside a block");
  // one block per CU (its stages fill most of the LDS): the epilogue has
  // the registers to fetch its per-entry operands 16 at a time (see epi_tile)
  static constexpr bool kPrefetchEpi = true;
  static constexpr int BM = BM_, BN = BN_, BK = BK_, NT = 64 * WM * WN;
  static constexpr int WAVES = WM * WN;
  // the block's waves spread over the CU's four SIMDs: eight waves give each
  // SIMD two, so one wave's waits are covered by the other's matrix work
  static_assert(WAVES % 4 == 0, "whole waves per SIMD");
  static constexpr int WAVES_PER_EU = WAVES / 4;
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int KS = BK / 16;
  static_assert(TM >= 1 && TN >= 1 && (KS == 1 || KS == 2), "one or two 16-deep k-steps per K-tile");
  // Swizzle of FP32 Y rows (BK floats = BK / 4 chunks): chunk s of row r sits
  // in slot s ^ yswz(r), so the 16 rows a read touches at a time cover all
  // 64 banks (256 bytes hold 64 / BK rows).
  __device__ __forceinline__ static int yswz(int r) { return (r / (64 / BK)) % (BK / 4); }
  static_assert(STAGES == 2 || STAGES == 3, "two or three stages");
  using PX = TileLoadB3<BM, NT, BK>;  // swizzle of the bf16 planes
  using PY = TileLoadB3<BN, NT, BK>;
  static constexpr int CPR = BK / 8;  // 16-byte chunks per bf16 row
  static constexpr int XQ = BM * CPR; // chunks per X plane
  static constexpr int YQ = YF32 ? BN * (BK / 4) : 2 * BN * CPR;  // chunks of the Y tile
  static constexpr int STAGE_BYTES = (2 * XQ + YQ) * 16;
  static constexpr int MAIN_BYTES = STAGES * STAGE_BYTES;
  static constexpr int XI = 2 * XQ / 64, YI = YQ / 64;  // wave-instructions per stage
  static_assert((2 * XQ) % 64 == 0 && YQ % 64 == 0 && (XI + YI) % WAVES == 0, "load split");
  static constexpr int IPW = (XI + YI) / WAVES;  // loads per wave and stage
  static constexpr int PER = 2 * TM + 2 * TN;   // 16-byte fragment reads per k-step
  static constexpr int NR = KS * PER;
  // This wave's loads of one stage: wave-instruction q * WAVES + w of the
  // stage, so which operand (and plane) a load q reads is fixed at compile
  // time.
  static constexpr int XPW = XI / WAVES;  // X loads per wave (both planes)
  static constexpr int XPP = XPW / 2;     // ... per plane
  static constexpr int YPP = YI / WAVES / 2;  // Y loads per wave and plane (bf16 Y)
  static_assert(XI % (2 * WAVES) == 0, "X planes split evenly over the waves");
  static_assert(YF32 || YI % (2 * WAVES) == 0, "Y planes split evenly over the waves");

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  struct Frag {  // operands of one K-tile
    bf16x8 xh[KS][TM], xl[KS][TM], yh[KS][TN], yl[KS][TN];
  };
  struct Raw {
    u4 r[NR];
  };
  struct Dma {
    const char* xh;  // uniform bases at K-tile 0 of the range
    const char* xl;
    const char* yh;  // Y (FP32) or its hi plane
    const char* yl;
    unsigned voff[IPW];  // per lane
    unsigned wofs;       // this wave's LDS offset within a stage
    // packed Y: its base, the column block, the range start, and the per-lane
    // offsets of the K-tiles loaded as stored ([k][n])
    const char* yp;
    int64_t jb, kbeg;
    unsigned voffT[IPW];
  };
  // packed Y: whether K-tile kt of a range starting at kbeg is read as stored
  __device__ __forceinline__ static bool tr_at(const Dma& d, int kt) {
    if constexpr (!YP) return false;
    return d.jb > (d.kbeg + (int64_t)kt * BK) / kPT;
  }
  static constexpr int YSTEP = YF32 ? BK * 4 : BK * 2;  // bytes per K-tile along a Y row

  __device__ __forceinline__ static unsigned lds_addr(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char*)p;
  }

  __device__ __forceinline__ void setup(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg, int w,
                                        Dma& d) const {
    d.xh = reinterpret_cast<const char*>(o.Xh + m0 * o.ldx + kbeg);
    d.xl = reinterpret_cast<const char*>(o.Xl + m0 * o.ldx + kbeg);
    if constexpr (YP) {
      d.yh = d.yl = nullptr;  // per K-tile, from the packed tile (dma_at)
    } else if constexpr (YF32) {
      d.yh = reinterpret_cast<const char*>(o.Y + n0 * o.ldy + kbeg);
      d.yl = d.yh;
    } else {
      d.yh = reinterpret_cast<const char*>(o.Yh + n0 * o.ldy + kbeg);
      d.yl = reinterpret_cast<const char*>(o.Yl + n0 * o.ldy + kbeg);
    }
    d.wofs = (unsigned)w * 1024u;
    if constexpr (YP) {
      d.yp = reinterpret_cast<const char*>(o.Yp);
      d.jb = n0 / kPT;
      d.kbeg = kbeg;
    }
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
      if (q < XPW) {
        const int p = ((q % XPP) * WAVES + w) * 64 + lane;  // chunk within the plane
        const int r = p / CPR, slot = p % CPR;
        const int chunk = slot ^ ((r / PX::RG) & (CPR - 1));
        // rows past the operand's end (M padded to the tile) re-read its last
        // row; their outputs are never stored
        const int64_t rr = (m0 + r < o.mrows ? m0 + r : o.mrows - 1) - m0;
        d.voff[q] = (unsigned)((rr * o.ldx + chunk * 8) * 2);
      } else if constexpr (YP) {
        const int p = ((q - XPW) * WAVES + w) * 64 + lane;
        const int r = p / (BK / 4), slot = p % (BK / 4);
        const int chunk = slot ^ yswz(r);
        d.voff[q] = (unsigned)(((int64_t)r * kPT + chunk * 4) * 4);  // rows of a packed tile
        // as stored: row kr of kPT floats (32 chunks), chunk c in slot c ^ 8 (kr / 8 % 2)
        const int kr = p / (int)(kPT / 4), s2 = p % (int)(kPT / 4);
        const int c2 = s2 ^ (((kr >> 3) & 1) << 3);
        d.voffT[q] = (unsigned)((kr * kPT + c2 * 4) * 4);
      } else if constexpr (YF32) {
        const int p = ((q - XPW) * WAVES + w) * 64 + lane;
        const int r = p / (BK / 4), slot = p % (BK / 4);
        const int chunk = slot ^ yswz(r);
        d.voff[q] = (unsigned)(((int64_t)r * o.ldy + chunk * 4) * 4);
      } else {
        const int p = (((q - XPW) % YPP) * WAVES + w) * 64 + lane;
        const int r = p / CPR, slot = p % CPR;
        const int chunk = slot ^ ((r / PY::RG) & (CPR - 1));
        d.voff[q] = (unsigned)(((int64_t)r * o.ldy + chunk * 8) * 2);
      }
    }
  }

  // Direct load q of K-tile kt into the stage at LDS address sb (this wave's
  // part of it).
  __device__ __forceinline__ static void dma_at(const Dma& d, int q, int kt, unsigned sb) {
    const char* b;
    unsigned vo = d.voff[q];
    if (q < XPP) {
      b = d.xh + (size_t)kt * (BK * 2);
    } else if (q < XPW) {
      b = d.xl + (size_t)kt * (BK * 2);
    } else if constexpr (YP) {
      const int64_t k = d.kbeg + (int64_t)kt * BK, kb = k / kPT, kk = k % kPT;
      if (d.jb > kb) {  // tile (kb, jb): rows k, read as stored
        b = d.yp + (size_t)(packed_tile(kb, d.jb) * (kPT * kPT) + kk * kPT) * 4;
        vo = d.voffT[q];
      } else {          // tile (jb, kb): rows n, columns kk ..
        b = d.yp + (size_t)(packed_tile(d.jb, kb) * (kPT * kPT) + kk) * 4;
      }
    } else if (YF32 || q < XPW + YPP) {
      b = d.yh + (size_t)kt * YSTEP;
    } else {
      b = d.yl + (size_t)kt * YSTEP;
    }
    lds_dma16(vo, b, sb + d.wofs + (unsigned)(q * WAVES) * 1024u);
  }
  __device__ __forceinline__ static void issue(const Dma& d, int kt, const char* st) {
#pragma unroll
    for (int q = 0; q < IPW; ++q) dma_at(d, q, kt, lds_addr(st));
  }

  // Packed Y read as stored: byte offset (within a stage) of this lane's
  // column n of fragment j, at the first of its 8 k (the rest at + kPT * 4 per k).
  __device__ __forceinline__ void read_offsets_t(unsigned (&adT)[TN]) const {
    const int khalf = lane >> 5;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = wn * (BN / WN) + j * 32 + (lane & 31);
      adT[j] = 2u * XQ * 16 + (unsigned)(8 * khalf) * (unsigned)(kPT * 4) +
               (((unsigned)(n >> 2) ^ (unsigned)(8 * khalf)) << 4) + 4u * (n & 3);
    }
  }
  // Read r of a K-tile's fragment reads: X and row-stored Y reads are 16
  // bytes at ad[r]; a packed Y K-tile read as stored takes four 4-byte reads
  // of consecutive k.
  template <bool TR>
  __device__ __forceinline__ static u4 read_r(const char* st, const unsigned (&ad)[NR],
                                              const unsigned (&adT)[TN], int r) {
    if constexpr (TR) {
      const int ks = r / PER, q = r % PER;
      if (q >= 2 * TM) {
        const int j = (q - 2 * TM) / 2, h = (q - 2 * TM) % 2;
        const char* b = st + adT[j] + (unsigned)((16 * ks + 4 * h) * kPT * 4);
        return (u4){*reinterpret_cast<const unsigned*>(b),
                    *reinterpret_cast<const unsigned*>(b + kPT * 4),
                    *reinterpret_cast<const unsigned*>(b + 2 * kPT * 4),
                    *reinterpret_cast<const unsigned*>(b + 3 * kPT * 4)};
      }
    }
    return *reinterpret_cast<const u4*>(st + ad[r]);
  }

  // Byte offsets (within a stage) of this lane's fragment reads.
  __device__ __forceinline__ void read_offsets(unsigned (&ad)[NR]) const {
    const int mrow = wm * (BM / WM) + (lane & 31);
    const int khalf = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int chunk = 2 * ks + khalf;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const unsigned off = 2u * PX::swz(mrow + i * 32, chunk);
        ad[PER * ks + 2 * i] = off;
        ad[PER * ks + 2 * i + 1] = 2u * BM * BK + off;
      }
      const int c0 = 4 * ks + 2 * khalf;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * (BN / WN) + j * 32 + (lane & 31);
        if constexpr (YF32) {
          const unsigned yb = 2u * XQ * 16 + 4u * n * BK;
          const int f = yswz(n);
          ad[PER * ks + 2 * TM + 2 * j] = yb + 4u * ((c0 ^ f) << 2);
          ad[PER * ks + 2 * TM + 2 * j + 1] = yb + 4u * (((c0 + 1) ^ f) << 2);
        } else {
          const unsigned off = 2u * XQ * 16 + 2u * PY::swz(n, chunk);
          ad[PER * ks + 2 * TM + 2 * j] = off;                     // hi plane
          ad[PER * ks + 2 * TM + 2 * j + 1] = off + 2u * BN * BK;  // lo plane
        }
      }
    }
  }

  template <bool TR>
  __device__ __forceinline__ static void read(const char* st, const unsigned (&ad)[NR],
                                              const unsigned (&adT)[TN], Raw& rw) {
#pragma unroll
    for (int i = 0; i < NR; ++i) rw.r[i] = read_r<TR>(st, ad, adT, i);
  }

  // Split pair sp of the next tile's FP32 Y fragments (4 pairs per fragment).
  __device__ __forceinline__ static void split_at(const Raw& rw, unsigned (&h)[KS][TN][4],
                                                  unsigned (&l)[KS][TN][4], int sp) {
    const int fi = sp / 4, pr = sp % 4, ks = fi / TN, j = fi % TN;
    const f4 v = __builtin_bit_cast(f4, rw.r[PER * ks + 2 * TM + 2 * j + pr / 2]);
    if (pr % 2 == 0)
      split_pair(v.x, v.y, h[ks][j][pr], l[ks][j][pr]);
    else
      split_pair(v.z, v.w, h[ks][j][pr], l[ks][j][pr]);
    // keep the pair here, between its MFMAs (the compiler would otherwise sink
    // it to the end of the K-tile, next to its first use)
    asm volatile("" : "+v"(h[ks][j][pr]), "+v"(l[ks][j][pr]));
  }
  static constexpr int NSP = YF32 ? KS * TN * 4 : 0;  // split pairs per K-tile

  // Fragments of a K-tile from its LDS reads (and split pairs).
  __device__ __forceinline__ static void assemble(const Raw& rw, const unsigned (&h)[KS][TN][4],
                                                  const unsigned (&l)[KS][TN][4], Frag& f) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        f.xh[ks][i] = __builtin_bit_cast(bf16x8, rw.r[PER * ks + 2 * i]);
        f.xl[ks][i] = __builtin_bit_cast(bf16x8, rw.r[PER * ks + 2 * i + 1]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if constexpr (YF32) {
          f.yh[ks][j] = __builtin_bit_cast(bf16x8, (u4){h[ks][j][0], h[ks][j][1], h[ks][j][2], h[ks][j][3]});
          f.yl[ks][j] = __builtin_bit_cast(bf16x8, (u4){l[ks][j][0], l[ks][j][1], l[ks][j][2], l[ks][j][3]});
        } else {
          f.yh[ks][j] = __builtin_bit_cast(bf16x8, rw.r[PER * ks + 2 * TM + 2 * j]);
          f.yl[ks][j] = __builtin_bit_cast(bf16x8, rw.r[PER * ks + 2 * TM + 2 * j + 1]);
        }
      }
    }
  }
  __device__ __forceinline__ static void split(const Raw& rw, Frag& f) {
    unsigned h[KS][TN][4], l[KS][TN][4];
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp) split_at(rw, h, l, sp);
    assemble(rw, h, l, f);
  }

  __device__ __forceinline__ void mfma(const Frag& f) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[ks][i], f.yl[ks][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xl[ks][i], f.yh[ks][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[ks][i], f.yh[ks][j], acc[i][j], 0, 0, 0);
        }
  }
  // One MFMA of a K-tile: m = ((ks * 3 + product) * TM + i) * TN + j.  Each
  // accumulator sees its products in the order of mfma() (so results are
  // the same bit for bit), while consecutive MFMAs go to different
  // accumulators and never wait for each other.
  __device__ __forceinline__ void mfma_at(const Frag& f, int m) {
    const int j = m % TN, i = (m / TN) % TM, p = (m / TN / TM) % 3, ks = m / TN / TM / 3;
    if (p == 0)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[ks][i], f.yl[ks][j], acc[i][j], 0, 0, 0);
    else if (p == 1)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xl[ks][i], f.yh[ks][j], acc[i][j], 0, 0, 0);
    else
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.xh[ks][i], f.yh[ks][j], acc[i][j], 0, 0, 0);
  }

  // K-tile kt whose STAGES successors exist: stage `rd` holds tile kt + 1,
  // stage `fr` held tile kt (already in registers) and takes tile
  // kt + STAGES.  The MFMAs of tile kt are issued one by one, each followed
  // by work of the next tile that does not depend on them: first the direct
  // loads of tile kt + STAGES and the LDS reads of tile kt + 1, then the
  // split of tile kt + 1's C fragments.  Scheduling barriers keep this order
  // (the matrix core runs each MFMA while the wave issues what follows it).
  template <bool TR>
  __device__ __forceinline__ void full_step(const Dma& d, const unsigned (&ad)[NR],
                                            const unsigned (&adT)[TN], int kt, const char* rd,
                                            const char* fr, Frag& cur) {
    constexpr int NM = KS * TM * TN * 3;  // MFMAs per K-tile
    constexpr int NRM = (NR + 1) / 2;     // MFMAs followed by reads
    static_assert(IPW <= NM, "one direct load per MFMA slot at most");
    wait_vmem<(STAGES - 2) * IPW>();  // tile kt + 1 landed (later ones may be in flight)
    wave_barrier_mem();
    __builtin_amdgcn_sched_barrier(0);
    const unsigned sb = lds_addr(fr);
    Raw rw;
    unsigned h[KS][TN][4], l[KS][TN][4];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      mfma_at(cur, m);
      if (m < IPW) dma_at(d, m, kt + STAGES, sb);
      if (m < NRM) {
#pragma unroll
        for (int r = 2 * m; r < 2 * m + 2 && r < NR; ++r) rw.r[r] = read_r<TR>(rd, ad, adT, r);
      } else if (m - NRM < NSP) {
        split_at(rw, h, l, m - NRM);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = NM; m < NRM + NSP; ++m) split_at(rw, h, l, m - NRM);  // left over
    assemble(rw, h, l, cur);
  }

  // Packed Y: K-tiles [0, ksplit) of the range lie below the diagonal.
  __device__ __forceinline__ static int ksplit_of(const Dma& d, int nk) {
    const int64_t ks = (d.jb * kPT - d.kbeg + BK - 1) / BK;
    return ks <= 0 ? 0 : ks >= nk ? nk : (int)ks;
  }

  // Any K-tile (near the end of the range): the same with bounds.
  __device__ __forceinline__ void tail_step(const Dma& d, const unsigned (&ad)[NR],
                                            const unsigned (&adT)[TN], int kt, int nk,
                                            const char* rd, const char* fr, Frag& cur) {
    if (kt + 1 < nk) {
      if (STAGES == 3 && kt + 2 < nk) wait_vmem<IPW>(); else wait_vmem<0>();
      wave_barrier_mem();
      if (kt + STAGES < nk) issue(d, kt + STAGES, fr);
      Raw rw;
      if (tr_at(d, kt + 1))
        read<true>(rd, ad, adT, rw);
      else
        read<false>(rd, ad, adT, rw);
      mfma(cur);
      split(rw, cur);
    } else {
      mfma(cur);
    }
  }

  __device__ __forceinline__ void run(const Ops& o, int64_t m0, int64_t n0, int64_t kbeg,
                                      int64_t kend, char* smem) {
    char* const s0 = smem;
    char* const s1 = smem + STAGE_BYTES;
    char* const s2 = smem + (STAGES == 3 ? 2 * STAGE_BYTES : 0);
    lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    wm = w % WM;
    wn = w / WM;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int nk = (int)((kend - kbeg) / BK);
    // Every wave of the block is done with the stages (and with whatever the
    // caller kept in the same shared memory).
    wait_vmem<0>();
    wave_barrier_mem();
    if (nk <= 0) return;
    Dma d;
    setup(o, m0, n0, kbeg, w, d);
    unsigned ad[NR];
    read_offsets(ad);
    unsigned adT[TN];
    if constexpr (YP) read_offsets_t(adT);
    issue(d, 0, s0);
    if (nk > 1) {
      issue(d, 1, s1);
      wait_vmem<IPW>();
    } else {
      wait_vmem<0>();
    }
    wave_barrier_mem();
    if (STAGES == 3 && nk > 2) issue(d, 2, s2);
    // A wave whose rows all lie past the operand's end (M padded to the tile)
    // only takes its share of the loads and barriers: no reads, no MFMAs.
    // (Only the A product pads M.)
    if (YF32 && m0 + wm * (BM / WM) >= o.mrows) {
      for (int kt = 0; kt + 1 < nk; ++kt) {
        if (STAGES == 3 && kt + 2 < nk) wait_vmem<IPW>(); else wait_vmem<0>();
        wave_barrier_mem();
        if (kt + STAGES < nk) issue(d, kt + STAGES, kt % STAGES == 0 ? s0 : kt % STAGES == 1 ? s1 : s2);
      }
      wave_barrier_mem();
      return;
    }
    Frag cur;
    {
      Raw rw;
      if (tr_at(d, 0))
        read<true>(s0, ad, adT, rw);
      else
        read<false>(s0, ad, adT, rw);
      split(rw, cur);
    }
    int kt = 0;
    if constexpr (STAGES == 3) {
      // Packed Y: the K-tiles below the diagonal (k < jb kPT, read as stored)
      // come first, then the others; each run of one orientation gets its own
      // loop (a choice between the two inside one loop costs the register
      // allocator hundreds of spilled registers).  Reads of tile kt + 1.
      const int ksplit = YP ? ksplit_of(d, nk) : 0;
      auto stg = [&](int k) { const int m = k % 3; return m == 0 ? s0 : m == 1 ? s1 : s2; };
      for (; kt + 5 < nk && kt + 3 < ksplit; kt += 3) {
        full_step<true>(d, ad, adT, kt, s1, s0, cur);
        full_step<true>(d, ad, adT, kt + 1, s2, s1, cur);
        full_step<true>(d, ad, adT, kt + 2, s0, s2, cur);
      }
      for (; kt + 5 < nk && kt + 1 < ksplit; ++kt)
        full_step<true>(d, ad, adT, kt, stg(kt + 1), stg(kt), cur);
      for (; kt + 5 < nk && kt % 3 != 0; ++kt)
        full_step<false>(d, ad, adT, kt, stg(kt + 1), stg(kt), cur);
      for (; kt + 5 < nk; kt += 3) {
        full_step<false>(d, ad, adT, kt, s1, s0, cur);
        full_step<false>(d, ad, adT, kt + 1, s2, s1, cur);
        full_step<false>(d, ad, adT, kt + 2, s0, s2, cur);
      }
      for (; kt < nk; ++kt) tail_step(d, ad, adT, kt, nk, stg(kt + 1), stg(kt), cur);
    } else {
      static_assert(!YP, "packed Y takes three stages");
      for (; kt + 3 < nk; kt += 2) {
        full_step<false>(d, ad, adT, kt, s1, s0, cur);
        full_step<false>(d, ad, adT, kt + 1, s0, s1, cur);
      }
      for (; kt < nk; ++kt) {
        const bool ph = kt % 2;
        tail_step(d, ad, adT, kt, nk, ph ? s0 : s1, ph ? s1 : s0, cur);
      }
    }
    // the caller may reuse the shared memory once every wave has read its last stage
    wave_barrier_mem();
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
//     the Y operand) run on one XCD at the same time, so that strip and the
//     X tiles they need are fetched from memory about once per round.
//   tail: the T = nTiles - R nb remaining tiles are cut into S equal K-chunks
//     each, and item i = c T + t (chunk c of tail tile t) goes to block i mod
//     nb.  Items are numbered chunk first, so the blocks of one XCD work on
//     the same K-chunk of neighbouring tiles at the same time and keep
//     sharing operand strips in L2, as in a full round.  With S = 1 a block
//     finishes the tile itself; otherwise it stores its partial product and
//     the fix-up kernel adds the S partials of each tile in chunk order
//     (deterministic; no block ever waits for another).  The host picks S
//     to minimise the largest tail load of a block.
// Logical block numbers are assigned XCD by XCD (the hardware hands block b to
// XCD b % 8), so one XCD works on contiguous tiles.
// The epilogue of a finished tile.  Where the block GEMM allows it
// (kPrefetchEpi) and the epilogue reads operands of its own per entry
// (fetch), those are loaded for the 16 entries of one accumulator block
// before any is used, so the loads are in flight together instead of one
// dependent load per entry.  Same arithmetic, same order, either way.
template <class E, class = void>
struct has_fetch : std::false_type {};
template <class E>
struct has_fetch<E, std::void_t<decltype(&E::fetch)>> : std::true_type {};
// Epi::Pre where the epilogue fetches its operands ahead, else a placeholder.
template <class E, class = void>
struct fetch_t {
  struct type {};
};
template <class E>
struct fetch_t<E, std::void_t<typename E::Pre>> {
  using type = typename E::Pre;
};
template <class G, class = void>
struct prefetch_epi : std::false_type {};
template <class G>
struct prefetch_epi<G, std::void_t<decltype(G::kPrefetchEpi)>>
    : std::integral_constant<bool, G::kPrefetchEpi> {};

// Epilogues with a block<N>(rows, cols, acc) member take N entries at once:
// every operand of the N entries is loaded before the first result is
// stored (a store may alias an operand buffer, so entry by entry each
// entry's loads would wait for the store before them).
template <class E, class = void>
struct has_block : std::false_type {};
template <class E>
struct has_block<E, std::void_t<decltype(&E::template block<16>)>> : std::true_type {};
// Block GEMMs whose epilogue takes entries in runs (kBlockEpi); the others
// keep their registers for occupancy (measured: the FP32 products run
// slower with the extra live operands).
template <class G, class = void>
struct block_epi : std::false_type {};
template <class G>
struct block_epi<G, std::void_t<decltype(G::kBlockEpi)>>
    : std::integral_constant<bool, G::kBlockEpi> {};

// The epilogue of a tile in runs of NB entries of one column (Epi::block):
// all operands of a run are loaded before any of its results is stored.
template <int NB, class G, class Epi>
__device__ __forceinline__ void epi_tile_runs(const G& g, Epi& epi, int64_t m0, int64_t n0) {
  static_assert(16 % NB == 0, "whole runs per accumulator column");
#pragma unroll
  for (int i = 0; i < G::TM; ++i)
#pragma unroll
    for (int j = 0; j < G::TN; ++j)
#pragma unroll
      for (int r0 = 0; r0 < 16; r0 += NB) {
        int64_t rs[NB], cs[NB];
        float a[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          rs[r] = m0 + g.row_of(i, r0 + r);
          cs[r] = n0 + g.col_of(j);
          a[r] = g.acc[i][j][r0 + r];
        }
        epi.template block<NB>(rs, cs, a);
      }
}

template <class G, class Epi>
__device__ __forceinline__ void epi_tile(const G& g, Epi& epi, int64_t m0, int64_t n0) {
  if constexpr (has_fetch<Epi>::value && prefetch_epi<G>::value) {
#pragma unroll
    for (int i = 0; i < G::TM; ++i)
#pragma unroll
      for (int j = 0; j < G::TN; ++j) {
        const int64_t c = n0 + g.col_of(j);
        typename Epi::Pre pre[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) pre[r] = epi.fetch(m0 + g.row_of(i, r), c);
#pragma unroll
        for (int r = 0; r < 16; ++r) epi.element_pre(m0 + g.row_of(i, r), c, g.acc[i][j][r], pre[r]);
      }
  } else if constexpr (has_block<Epi>::value && block_epi<G>::value) {
    epi_tile_runs<8>(g, epi, m0, n0);
  } else {
    g.for_each([&](int rr, int c, float v) { epi.element(m0 + rr, n0 + c, v); });
  }
}

template <class G, class Epi>
__global__ __launch_bounds__(G::NT) __attribute__((amdgpu_waves_per_eu(G::WAVES_PER_EU)))
void k_rect_streamk(typename G::Ops ops, int64_t nMT, int64_t nTiles, int64_t U, int64_t S,
                    Epi epi, float* __restrict__ part, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[G::MAIN_BYTES];
  __shared__ double red[G::NT / 64];
  const int64_t nb = gridDim.x;
  const int64_t L = xcd_tile(blockIdx.x, nb);
  const int64_t R = nTiles / nb, nFull = R * nb, T = nTiles - nFull;
  G g;
  for (int64_t r = 0; r < R; ++r) {
    const int64_t tile = r * nb + L;
    const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
    g.run(ops, m0, n0, 0, U * G::BK, smem);
    epi_tile(g, epi, m0, n0);
    epi.end_tile(tile, red);
  }
  for (int64_t i = L; i < T * S; i += nb) {
    const int64_t c = i / T, tile = nFull + i % T;
    const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
    g.run(ops, m0, n0, c * U / S * G::BK, (c + 1) * U / S * G::BK, smem);
    if (S == 1) {
      epi_tile(g, epi, m0, n0);
      epi.end_tile(tile, red);
    } else {
      float* ps = part + i * (int64_t)(G::BM * G::BN);
      g.for_each([&](int rr, int c2, float v) { ps[rr * G::BN + c2] = v; });
    }
  }
}

// Tail tiles computed in S > 1 K-chunks: add the partial products in chunk
// order (deterministic) and run the epilogue.  1024 threads per block: the
// epilogue's loads form a dependent chain per element, so the fix-up runs as
// many waves per tile as a block holds, and a tile of more than 8 entries per
// thread is shared by kFixParts(G) blocks of 8 entries per thread each (one
// round of loads per thread instead of several in a row).  Block part q > 0
// of tile `tile` leaves its share of the h sum in slot q * nTiles + tile of
// the epilogue's per-tile partials, part 0 in slot `tile`.
constexpr int kFixThreads = 1024;
template <class G>
constexpr int kFixParts = (G::BM * G::BN) / kFixThreads > 8 ? (G::BM * G::BN) / kFixThreads / 8 : 1;
template <class G, class Epi>
__global__ __launch_bounds__(kFixThreads) void k_rect_fixup(int64_t nMT, int64_t nTiles, int64_t nb,
                                                            int64_t S,
                                                            const float* __restrict__ part, Epi epi,
                                                            const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[kFixThreads / 64];
  constexpr int Q = kFixParts<G>;
  const int64_t nFull = (nTiles / nb) * nb, T = nTiles - nFull;
  const int64_t t = blockIdx.x / Q, tile = nFull + t;
  const int qb = (int)(blockIdx.x % Q);
  const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
  constexpr int E = G::BM * G::BN;
  static_assert(E % (kFixThreads * Q) == 0, "whole passes");
  // entries e = threadIdx.x + q kFixThreads, q in this block's share [q_lo,
  // q_lo + PER), taken GRP at a time: their partials (and the epilogue's own
  // operands) are loaded together, then summed in chunk order and finished
  // in the order of q
  constexpr int PER = E / kFixThreads / Q, GRP = PER < 8 ? PER : 8;
  static_assert(PER % GRP == 0, "whole groups");
  const int q_lo = qb * PER;
  for (int q0 = q_lo; q0 < q_lo + PER; q0 += GRP) {
    // the epilogue's own operands first, then the partials of up to two
    // chunks at a time, all in flight before they are added in chunk order
    typename fetch_t<Epi>::type pre[GRP];
    if constexpr (has_fetch<Epi>::value) {
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = threadIdx.x + (q0 + q) * kFixThreads;
        pre[q] = epi.fetch(m0 + e / G::BN, n0 + e % G::BN);
      }
    }
    float s[GRP];
#pragma unroll
    for (int q = 0; q < GRP; ++q) s[q] = part[t * E + threadIdx.x + (q0 + q) * kFixThreads];
    for (int64_t c = 1; c < S; c += 2) {
      float v[2][GRP];
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (c + k < S)
#pragma unroll
          for (int q = 0; q < GRP; ++q)
            v[k][q] = part[((c + k) * T + t) * E + threadIdx.x + (q0 + q) * kFixThreads];
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (c + k < S)
#pragma unroll
          for (int q = 0; q < GRP; ++q) s[q] += v[k][q];
    }
    if constexpr (has_block<Epi>::value && !has_fetch<Epi>::value) {
      int64_t rs[GRP], cs[GRP];
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = threadIdx.x + (q0 + q) * kFixThreads;
        rs[q] = m0 + e / G::BN;
        cs[q] = n0 + e % G::BN;
      }
      epi.template block<GRP>(rs, cs, s);
    } else if constexpr (has_fetch<Epi>::value) {
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = threadIdx.x + (q0 + q) * kFixThreads;
        epi.element_pre(m0 + e / G::BN, n0 + e % G::BN, s[q], pre[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = threadIdx.x + (q0 + q) * kFixThreads;
        epi.element(m0 + e / G::BN, n0 + e % G::BN, s[q]);
      }
    }
  }
  epi.end_tile(qb * nTiles + tile, red);
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
  // computed once per kernel (a function-local static: thread-safe initialisation)
  static const int64_t resident =
      resident_blocks(reinterpret_cast<const void*>(&k_rect_streamk<G, Epi>), G::NT);
  const int64_t nMT = Mp / G::BM, nNT = Np / G::BN;
  const int64_t nTiles = nMT * nNT, U = Kp / G::BK;
  int64_t nb = resident;
  if (nb > nTiles) nb = nTiles;
  const int64_t T = nTiles - (nTiles / nb) * nb;
  // K-chunks per tail tile: the smallest S with the least cost, counted in
  // K-steps: the largest block load (with start-up per item) plus the fix-up,
  // which reads S partials per entry; the partials must fit the scratch
  // (2 * kMaxStreamKBlocks tiles of 64 x 128)
  const int64_t cap = 2 * kMaxStreamKBlocks * 64 * 128 / (G::BM * G::BN);
  constexpr int64_t kItemCost = 8;
  int64_t S = 1, best = T ? ((T + nb - 1) / nb) * (U + kItemCost) : 0;
  for (int64_t c = 2; T && c <= 64 && c <= U && T * c <= cap; ++c) {
    const int64_t load = ((T * c + nb - 1) / nb) * ((U + c - 1) / c + kItemCost) + c;
    if (load < best) {
      best = load;
      S = c;
    }
  }
  k_rect_streamk<G, Epi><<<dim3((unsigned)nb), dim3(G::NT), 0, s>>>(ops, nMT, nTiles, U, S, epi,
                                                                     part, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (T == 0 || S == 1) return hipSuccess;
  k_rect_fixup<G, Epi><<<dim3((unsigned)(T * kFixParts<G>)), dim3(kFixThreads), 0, s>>>(
      nMT, nTiles, nb, S, part, epi, gate);
  return hipGetLastError();
}

}  // namespace gemm
}  // namespace panda
