// Similarity GEMMs of the PANDA iteration on gfx950 FP32 matrix cores.
//
// Every similarity of the method is T(X, Y)_ij = (XY)_ij / sqrt(|X_i.|^2 +
// |Y_.j|^2 - |(XY)_ij|) (Eq. 1), which Sec. II-C recasts as one matrix product
// followed by an element-wise step on row and column norms (Eq. 9).  Here the
// product runs on v_mfma_f32_32x32x2f32 tiles, the two norm vectors are
// accumulated in FP64 from the same K-tiles the block stages through LDS (so
// no norm pass and no N_e x N_a norm matrices exist), and each kernel fuses
// the update rule that consumes its similarity into the epilogue:
//   k_tanimoto_store   T(X, Y) written out (the Tfunction; R = T(P, W), Eq. 3)
//   k_avail_wupdate    A = T(W, C) (Eq. 4) + W update (Eq. 2) + h partials (Eq. 7)
//   k_coreg_update     C off-diagonal update (Eq. 5) on upper tiles of
//                      T(W^T, W), mirror write, row sums for Eq. 6's sigma
//   k_coop_partial     split-K partial products of W W^T for the P update
//
// Operands are zero-padded to tile multiples by the host, so the main loop
// has no bounds checks; zero rows and columns add nothing to products or
// norms.  Blocks are mapped to tiles XCD by XCD: the hardware hands block b
// to XCD b % 8, and consecutive tiles (which share operand strips) are given
// to the same XCD so its L2 serves the reuse.
#include "panda_internal.h"

namespace panda {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Tile index for block b of an n-block grid, contiguous chunks per XCD.
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

__device__ __forceinline__ double tanimoto(double dot, double xx, double yy) {
  const double den = xx + yy - fabs(dot);
  return den > 0.0 ? dot / sqrt(den) : 0.0;
}

// One operand's MN x kBK tile: global -> registers -> LDS, with the squared
// norms of its MN vectors accumulated in FP64 along the way.  KC: the
// operand is contiguous along k in global memory (element (mn, k) at
// base[mn*ld + k]); otherwise along mn (element at base[k*ld + mn]).  The
// LDS copy is always [k][mn] with row length LD, the layout the MFMA
// operand reads want (32 consecutive mn per half-wave).
template <int MN, bool KC>
struct TileLoad {
  static constexpr int NV = MN * kBK / 4 / kThreads;  // float4 per thread
  static constexpr int LD = MN + 4;
  static constexpr int NSQ = KC ? NV : 4;
  static constexpr int TPR = MN / 4;          // !KC: threads per k-row
  static constexpr int RPP = kThreads / TPR;  // !KC: k-rows per pass
  static constexpr int SCRATCH = KC ? 0 : RPP * MN;  // doubles for the norm reduction
  static_assert(NV >= 1, "tile too small for one float4 per thread");
  static_assert(KC || RPP * NV == kBK, "k-rows must cover the tile");

  float4 v[NV];
  double sq[NSQ];

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < NSQ; ++i) sq[i] = 0.0;
  }

  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int64_t mn0,
                                       int64_t k0, int t) {
    if constexpr (KC) {
      const int kq = (t & 3) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = (t >> 2) + i * 64;
        v[i] = *reinterpret_cast<const float4*>(base + (mn0 + mn) * ld + k0 + kq);
      }
    } else {
      const int mnq = (t % TPR) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int k = t / TPR + i * RPP;
        v[i] = *reinterpret_cast<const float4*>(base + (k0 + k) * ld + mn0 + mnq);
      }
    }
  }

  __device__ __forceinline__ void accumulate() {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double a = v[i].x, b = v[i].y, c = v[i].z, d = v[i].w;
      if constexpr (KC) {
        sq[i] += a * a + b * b + c * c + d * d;
      } else {
        sq[0] += a * a;
        sq[1] += b * b;
        sq[2] += c * c;
        sq[3] += d * d;
      }
    }
  }

  __device__ __forceinline__ void store(float* lds, int t) const {
    if constexpr (KC) {
      const int kq = (t & 3) * 4;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int mn = (t >> 2) + i * 64;
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
        *reinterpret_cast<float4*>(lds + k * LD + mnq) = v[i];
      }
    }
  }

  // Norms of the MN vectors into nrm[MN].  Needs a barrier before nrm or
  // scratch is read by other threads; !KC calls one itself.
  __device__ __forceinline__ void finish(double* nrm, double* scratch, int t) {
    if constexpr (KC) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double s = sq[i];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        if ((t & 3) == 0) nrm[(t >> 2) + i * 64] = s;
      }
    } else {
      const int mnq = (t % TPR) * 4, r = t / TPR;
#pragma unroll
      for (int e = 0; e < 4; ++e) scratch[r * MN + mnq + e] = sq[e];
      __syncthreads();
      for (int c = t; c < MN; c += kThreads) {
        double s = 0.0;
        for (int q = 0; q < RPP; ++q) s += scratch[q * MN + c];
        nrm[c] = s;
      }
    }
  }
};

// Block-level GEMM over k in [kbeg, kend) for a BM x BN tile with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) sub-tile of 32 x 32 MFMA blocks.
// X element (m, k): XK ? X[m*ldx + k] : X[k*ldx + m].
// Y element (k, n): YK ? Y[n*ldy + k] : Y[k*ldy + n].
template <int BM, int BN, int WM, int WN, bool XK, bool YK>
struct BlockGemm {
  static_assert(WM * WN == 4, "four waves per block");
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static_assert(TM >= 1 && TN >= 1, "wave tile below one MFMA block");
  using LX = TileLoad<BM, XK>;
  using LY = TileLoad<BN, YK>;
  static constexpr int XS = kBK * LX::LD;
  static constexpr int YS = kBK * LY::LD;
  static constexpr int MAIN_BYTES = 2 * (XS + YS) * 4;
  static constexpr int SCRATCH_BYTES = (LX::SCRATCH + LY::SCRATCH) * 8;
  static_assert(SCRATCH_BYTES <= MAIN_BYTES, "norm scratch must fit the stage buffers");

  floatx16 acc[TM][TN];
  int lane, wm, wn;

  // smem: MAIN_BYTES of stage buffers; nrmX[BM], nrmY[BN] separate.
  __device__ __forceinline__ void run(const float* __restrict__ X, int64_t ldx,
                                      const float* __restrict__ Y, int64_t ldy, int64_t m0,
                                      int64_t n0, int64_t kbeg, int64_t kend, char* smem,
                                      double* nrmX, double* nrmY) {
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
    lx.init();
    ly.init();
    const int64_t nk = (kend - kbeg) / kBK;
    if (nk > 0) {
      lx.load(X, ldx, m0, kbeg, t);
      ly.load(Y, ldy, n0, kbeg, t);
      lx.accumulate();
      ly.accumulate();
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
        lx.load(X, ldx, m0, kbeg + (kt + 1) * kBK, t);
        ly.load(Y, ldy, n0, kbeg + (kt + 1) * kBK, t);
      }
      const float* xc = xs + cur * XS;
      const float* yc = ys + cur * YS;
#pragma unroll
      for (int kk = 0; kk < kBK / 2; ++kk) {
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
      }
      if (more) {
        lx.accumulate();
        ly.accumulate();
        lx.store(xs + (cur ^ 1) * XS, t);
        ly.store(ys + (cur ^ 1) * YS, t);
      }
      __syncthreads();
    }
    double* scr = reinterpret_cast<double*>(smem);
    lx.finish(nrmX, scr, t);
    ly.finish(nrmY, scr + LX::SCRATCH, t);
    __syncthreads();
  }

  // Local (row, col) in the block tile of accumulator register r of MFMA
  // block (i, j): the 32x32x2 f32 result layout puts column lane%32 in each
  // lane and rows 8*(r/4) + 4*(lane/32) + r%4.
  __device__ __forceinline__ int row_of(int i, int r) const {
    return wm * (BM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
  __device__ __forceinline__ int col_of(int j) const {
    return wn * (BN / WN) + j * 32 + (lane & 31);
  }
};

template <int BM, int BN>
struct SmemNorms {
  double x[BM];
  double y[BN];
  double red[8];
};

// ------------------------------------------------------------------------
// T(X, Y) stored: Sec. II-C Tfunction; used for R = T(P, W) (Eq. 3).
constexpr int kRB_M = 64, kRB_N = 256;
using RectGemm = BlockGemm<kRB_M, kRB_N, 1, 4, true, false>;

__global__ __launch_bounds__(kThreads) void k_tanimoto_store(
    const float* __restrict__ X, int64_t ldx, const float* __restrict__ Y, int64_t ldy,
    int64_t nMT, int64_t Kp, int64_t M, int64_t N, float* __restrict__ Out, int64_t ldo,
    const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[RectGemm::MAIN_BYTES];
  __shared__ SmemNorms<kRB_M, kRB_N> nr;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t m0 = (tile % nMT) * kRB_M, n0 = (tile / nMT) * kRB_N;
  RectGemm g;
  g.run(X, ldx, Y, ldy, m0, n0, 0, Kp, smem, nr.x, nr.y);
#pragma unroll
  for (int i = 0; i < RectGemm::TM; ++i)
#pragma unroll
    for (int j = 0; j < RectGemm::TN; ++j) {
      const int c = g.col_of(j);
      const int64_t gc = n0 + c;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = g.row_of(i, r);
        const int64_t gr = m0 + rr;
        if (gr < M && gc < N)
          Out[gr * ldo + gc] = (float)tanimoto((double)g.acc[i][j][r], nr.x[rr], nr.y[c]);
      }
    }
}

// ------------------------------------------------------------------------
// A = T(W, C) with the W update of Eq. 2 and the h partial sum of Eq. 7 in
// the epilogue.  W (old) and R are read at the output positions, the new W
// goes to a second buffer (the old one is still an operand of other blocks).
__global__ __launch_bounds__(kThreads) void k_avail_wupdate(
    const float* __restrict__ Wold, const float* __restrict__ C, const float* __restrict__ R,
    float* __restrict__ Wnew, int64_t ld, int64_t nMT, int64_t Nap, int64_t Ne, int64_t Na,
    double alpha, int32_t h_undamped, double* __restrict__ hpart, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[RectGemm::MAIN_BYTES];
  __shared__ SmemNorms<kRB_M, kRB_N> nr;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t m0 = (tile % nMT) * kRB_M, n0 = (tile / nMT) * kRB_N;
  RectGemm g;
  g.run(Wold, ld, C, ld, m0, n0, 0, Nap, smem, nr.x, nr.y);
  double hsum = 0.0;
  const double keep = 1.0 - alpha;
#pragma unroll
  for (int i = 0; i < RectGemm::TM; ++i)
#pragma unroll
    for (int j = 0; j < RectGemm::TN; ++j) {
      const int c = g.col_of(j);
      const int64_t gc = n0 + c;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = g.row_of(i, r);
        const int64_t gr = m0 + rr;
        if (gr < Ne && gc < Na) {
          const int64_t o = gr * ld + gc;
          const double a = tanimoto((double)g.acc[i][j][r], nr.x[rr], nr.y[c]);
          const double w = Wold[o];
          const double pred = 0.5 * (a + (double)R[o]);
          const float wn = (float)(keep * w + alpha * pred);
          Wnew[o] = wn;
          hsum += h_undamped ? fabs(pred - w) : fabs((double)wn - w);
        }
      }
    }
  // deterministic block sum: wave shuffle tree, then waves in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) hsum += __shfl_xor(hsum, off);
  if ((threadIdx.x & 63) == 0) nr.red[threadIdx.x >> 6] = hsum;
  __syncthreads();
  if (threadIdx.x == 0) hpart[tile] = ((nr.red[0] + nr.red[1]) + nr.red[2]) + nr.red[3];
}

// ------------------------------------------------------------------------
// C update of Eq. 5 on the upper tiles of T(W^T, W).  Within a tile only the
// strictly-upper entries (global row < col) are updated, each written at
// (i, j) and mirrored at (j, i), so C stays exactly symmetric and no entry
// is read after another thread wrote it.  The updated tile is staged in LDS
// for the coalesced mirror write and for the per-row sums (sum, sum of
// squares) that give the sigma of Eq. 6: slot J of row i gets the sum over
// the row part, slot I of row j the sum over the column part.
constexpr int kCB = 128;
using SymGemm = BlockGemm<kCB, kCB, 2, 2, false, false>;
constexpr int kSymLD = kCB + 1;

template <bool SIGT>
__global__ __launch_bounds__(kThreads) void k_coreg_update(
    const float* __restrict__ W, int64_t ldw, int64_t Nep, float* __restrict__ C, int64_t ldc,
    int64_t nT, int64_t Na, double alpha, double2* __restrict__ cstat, int64_t ldstat,
    const int32_t* gate) {
  if (gate && *gate == 0) return;
  constexpr int TILE_BYTES = kCB * kSymLD * 4 * (SIGT ? 2 : 1);
  constexpr int SMEM = SymGemm::MAIN_BYTES > TILE_BYTES ? SymGemm::MAIN_BYTES : TILE_BYTES;
  __shared__ __align__(16) char smem[SMEM];
  __shared__ SmemNorms<kCB, kCB> nr;
  const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
  int64_t I, J;
  tri_tile(u, I, J);
  const int64_t m0 = I * kCB, n0 = J * kCB;
  SymGemm g;
  // X = W^T (gene m, tf k) = W[k][m]; Y = W (tf k, gene n) = W[k][n].
  g.run(W, ldw, W, ldw, m0, n0, 0, Nep, smem, nr.x, nr.y);
  float* ts = reinterpret_cast<float*>(smem);  // updated values
  float* tt = ts + kCB * kSymLD;               // fresh T (SIGT only)
  const double keep = 1.0 - alpha;
#pragma unroll
  for (int i = 0; i < SymGemm::TM; ++i)
#pragma unroll
    for (int j = 0; j < SymGemm::TN; ++j) {
      const int c = g.col_of(j);
      const int64_t gc = n0 + c;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = g.row_of(i, r);
        const int64_t gr = m0 + rr;
        float v = 0.0f, tv = 0.0f;
        if (gr < gc && gc < Na) {
          const double tsim = tanimoto((double)g.acc[i][j][r], nr.x[rr], nr.y[c]);
          const int64_t o = gr * ldc + gc;
          v = (float)(keep * (double)C[o] + alpha * tsim);
          C[o] = v;
          tv = (float)tsim;
        }
        ts[rr * kSymLD + c] = v;
        if constexpr (SIGT) tt[rr * kSymLD + c] = tv;
      }
    }
  __syncthreads();
  const int t = threadIdx.x;
  // mirror write: C[n0 + q][m0 + p] = ts[p][q] for global m0+p < n0+q
  for (int e = t; e < kCB * kCB; e += kThreads) {
    const int q = e / kCB, p = e % kCB;
    const int64_t gi = m0 + p, gj = n0 + q;
    if (gi < gj && gj < Na) C[gj * ldc + gi] = ts[p * kSymLD + q];
  }
  // per-row partial sums of the updated off-diagonal entries
  const float* sv = SIGT ? tt : ts;
  if (I == J) {
    if (t < kCB) {
      double s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < kCB; ++q) {  // row part (entries right of the diagonal)
        const double x = sv[t * kSymLD + q];
        s1 += x;
        s2 += x * x;
      }
      for (int p = 0; p < kCB; ++p) {  // column part (entries above the diagonal)
        const double x = sv[p * kSymLD + t];
        s1 += x;
        s2 += x * x;
      }
      cstat[I * ldstat + m0 + t] = make_double2(s1, s2);
    }
  } else {
    const int q = t & (kCB - 1);
    double s1 = 0.0, s2 = 0.0;
    if (t < kCB) {
      for (int p = 0; p < kCB; ++p) {
        const double x = sv[q * kSymLD + p];
        s1 += x;
        s2 += x * x;
      }
      cstat[J * ldstat + m0 + q] = make_double2(s1, s2);
    } else {
      for (int p = 0; p < kCB; ++p) {
        const double x = sv[p * kSymLD + q];
        s1 += x;
        s2 += x * x;
      }
      cstat[I * ldstat + n0 + q] = make_double2(s1, s2);
    }
  }
}

// ------------------------------------------------------------------------
// P update, first half: W W^T is only N_e x N_e but has K = N_a, so the
// upper tiles are split over K; each block writes its partial product and,
// on diagonal tiles, the partial squared row norms of its K chunk.
constexpr int kPB = 64;
using CoopGemm = BlockGemm<kPB, kPB, 2, 2, true, true>;

__global__ __launch_bounds__(kThreads) void k_coop_partial(
    const float* __restrict__ W, int64_t ldw, int64_t Nep, int64_t nU, int64_t chunk,
    int64_t Nap, float* __restrict__ part, double* __restrict__ pnrm, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[CoopGemm::MAIN_BYTES];
  __shared__ SmemNorms<kPB, kPB> nr;
  const int64_t idx = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t u = idx % nU, s = idx / nU;
  int64_t I, J;
  tri_tile(u, I, J);
  const int64_t m0 = I * kPB, n0 = J * kPB;
  int64_t kb = s * chunk, ke = kb + chunk;
  if (kb > Nap) kb = Nap;
  if (ke > Nap) ke = Nap;
  CoopGemm g;
  g.run(W, ldw, W, ldw, m0, n0, kb, ke, smem, nr.x, nr.y);
  float* ps = part + s * Nep * Nep;
#pragma unroll
  for (int i = 0; i < CoopGemm::TM; ++i)
#pragma unroll
    for (int j = 0; j < CoopGemm::TN; ++j) {
      const int c = g.col_of(j);
#pragma unroll
      for (int r = 0; r < 16; ++r) ps[(m0 + g.row_of(i, r)) * Nep + n0 + c] = g.acc[i][j][r];
    }
  if (I == J && threadIdx.x < kPB) pnrm[s * Nep + m0 + threadIdx.x] = nr.x[threadIdx.x];
}

}  // namespace

// ---------------------------------------------------------------- launch --

hipError_t launch_tanimoto_store(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                 int64_t Mp, int64_t Np, int64_t Kp, int64_t M, int64_t N,
                                 float* Out, int64_t ldo, const int32_t* gate, hipStream_t s) {
  const int64_t nMT = Mp / kRB_M, nNT = Np / kRB_N;
  k_tanimoto_store<<<dim3((unsigned)(nMT * nNT)), dim3(kThreads), 0, s>>>(
      X, ldx, Y, ldy, nMT, Kp, M, N, Out, ldo, gate);
  return hipGetLastError();
}

int64_t avail_wupdate_blocks(int64_t Nep, int64_t Nap) { return (Nep / kRB_M) * (Nap / kRB_N); }

hipError_t launch_avail_wupdate(const float* Wold, const float* C, const float* R, float* Wnew,
                                int64_t ld, int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na,
                                Rule rule, double* hpart, const int32_t* gate, hipStream_t s) {
  const int64_t nMT = Nep / kRB_M;
  k_avail_wupdate<<<dim3((unsigned)avail_wupdate_blocks(Nep, Nap)), dim3(kThreads), 0, s>>>(
      Wold, C, R, Wnew, ld, nMT, Nap, Ne, Na, rule.alpha, rule.h_undamped, hpart, gate);
  return hipGetLastError();
}

int64_t coreg_slots(int64_t Nap) { return Nap / kCB; }

hipError_t launch_coreg_update(const float* W, int64_t ldw, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, Rule rule, double2* cstat,
                               const int32_t* gate, hipStream_t s) {
  const int64_t nT = Nap / kCB;
  const unsigned nb = (unsigned)(nT * (nT + 1) / 2);
  if (rule.sigma_from_T)
    k_coreg_update<true><<<dim3(nb), dim3(kThreads), 0, s>>>(W, ldw, Nep, C, ldc, nT, Na,
                                                             rule.alpha, cstat, Nap, gate);
  else
    k_coreg_update<false><<<dim3(nb), dim3(kThreads), 0, s>>>(W, ldw, Nep, C, ldc, nT, Na,
                                                              rule.alpha, cstat, Nap, gate);
  return hipGetLastError();
}

int coop_splits(int64_t Nep, int64_t Nap) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  int64_t s = (512 + nU - 1) / nU;       // aim at a few hundred blocks
  const int64_t maxs = Nap / (4 * kBK);  // at least 4 K-steps per block
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t launch_coop_partial(const float* W, int64_t ldw, int64_t Nep, int64_t Nap, int splits,
                               float* part, double* pnrm, const int32_t* gate, hipStream_t s) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  const int64_t chunk = round_up((Nap + splits - 1) / splits, kBK);
  k_coop_partial<<<dim3((unsigned)(nU * splits)), dim3(kThreads), 0, s>>>(W, ldw, Nep, nU, chunk,
                                                                          Nap, part, pnrm, gate);
  return hipGetLastError();
}

}  // namespace panda
