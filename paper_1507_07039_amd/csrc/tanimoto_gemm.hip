// Similarity GEMMs of the PANDA iteration on gfx950 FP32 matrix cores.
//
// Every similarity of the method is T(X, Y)_ij = (XY)_ij / sqrt(|X_i.|^2 +
// |Y_.j|^2 - |(XY)_ij|) (Eq. 1), which Sec. II-C recasts as one matrix product
// followed by an element-wise step on row and column norms (Eq. 9).  Here the
// product runs on v_mfma_f32_32x32x2f32 tiles and the element-wise step is the
// epilogue of the same kernel, which also applies the update rule that
// consumes the similarity:
//   k_rect_streamk<EpiStoreT>   T(X, Y) written out (Tfunction; R = T(P, W), Eq. 3)
//   k_rect_streamk<EpiWUpdate>  A = T(W, C) (Eq. 4) + W update (Eq. 2) + h partials (Eq. 7)
//   k_coreg_update              C off-diagonal update (Eq. 5) on upper tiles of
//                               T(W^T, W), mirror write, row sums for Eq. 6's sigma
//   k_coop_partial              split-K partial products of W W^T for the P update
// The squared-norm vectors are FP64 inputs produced by the kernels that write
// the matrices (never N_e x N_a norm matrices), so the main loops are pure
// MFMA work.
//
// Operands are zero-padded to tile multiples by the host, so the main loop
// has no bounds checks; zero rows and columns add nothing to products.
// The rectangular products use a stream-K schedule: the grid holds as many
// blocks as the GPU runs at once, each takes an equal share of all
// (tile, K-step) work, tiles finished inside one block get their epilogue at
// once, and tiles shared by two blocks are summed and finished by a small
// fix-up kernel -- no block ever waits for another.  Logical block numbers
// are assigned XCD by XCD (the hardware hands block b to XCD b % 8), so the
// tiles one XCD works on are contiguous and share operand strips in its L2.
#include "panda_internal.h"

namespace panda {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ double tanimoto(double dot, double xx, double yy) {
  const double den = xx + yy - fabs(dot);
  return den > 0.0 ? dot / sqrt(den) : 0.0;
}

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

// Block-level GEMM over k in [kbeg, kend) for a BM x BN tile with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) sub-tile of 32 x 32 MFMA blocks.
// X element (m, k): XK ? X[m*ldx + k] : X[k*ldx + m].
// Y element (k, n): YK ? Y[n*ldy + k] : Y[k*ldy + n].
template <int BM_, int BN_, int WM, int WN, bool XK, bool YK, int BK_>
struct BlockGemm {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
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

  __device__ __forceinline__ void run(const float* __restrict__ X, int64_t ldx,
                                      const float* __restrict__ Y, int64_t ldy, int64_t m0,
                                      int64_t n0, int64_t kbeg, int64_t kend, char* smem) {
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
      lx.load(X, ldx, m0, kbeg, t);
      ly.load(Y, ldy, n0, kbeg, t);
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
        lx.load(X, ldx, m0, kbeg + (kt + 1) * BK, t);
        ly.load(Y, ldy, n0, kbeg + (kt + 1) * BK, t);
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
      }
      if (more) {
        lx.store(xs + (cur ^ 1) * XS, t);
        ly.store(ys + (cur ^ 1) * YS, t);
      }
      __syncthreads();
    }
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

// Deterministic sum of one double per thread over the 256-thread block.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// ------------------------------------------------------------ epilogues --
// T(X, Y) stored for i < M, j < N (Sec. II-C Tfunction; R of Eq. 3).
struct EpiStoreT {
  float* out;
  int64_t ldo, M, N;
  const double* nx;
  const double* ny;
  __device__ __forceinline__ void element(int64_t r, int64_t c, float acc) {
    if (r < M && c < N) out[r * ldo + c] = (float)tanimoto((double)acc, nx[r], ny[c]);
  }
  __device__ __forceinline__ void end_tile(int64_t, double*) {}
};

// A = T(W, C) (Eq. 4) folded into the W update of Eq. 2, with the tile's
// share of the h sum of Eq. 7.  The new W goes to a second buffer because
// the old one is still an operand of other blocks.
struct EpiWUpdate {
  const float* Wold;
  const float* R;
  float* Wnew;
  int64_t ld, Ne, Na;
  const double* nx;  // |W_i.|^2
  const double* ny;  // |C_.j|^2
  double alpha;
  int32_t h_undamped;
  double* hpart;
  double hsum;
  __device__ __forceinline__ void element(int64_t r, int64_t c, float acc) {
    if (r < Ne && c < Na) {
      const int64_t o = r * ld + c;
      const double a = tanimoto((double)acc, nx[r], ny[c]);
      const double w = Wold[o];
      const double pred = 0.5 * (a + (double)R[o]);
      const float wn = (float)((1.0 - alpha) * w + alpha * pred);
      Wnew[o] = wn;
      hsum += h_undamped ? fabs(pred - w) : fabs((double)wn - w);
    }
  }
  __device__ __forceinline__ void end_tile(int64_t tile, double* red) {
    const double s = block_sum(hsum, red);
    if (threadIdx.x == 0) hpart[tile] = s;
    hsum = 0.0;
  }
};

// ----------------------------------------------------- stream-K kernels --
using RectGemm = BlockGemm<64, 128, 1, 4, true, false, 16>;

// Block L (logical) owns work items [L*total/G, (L+1)*total/G) of the
// total = tiles * U items (U = K-steps per tile), tile-major, M fastest.
__device__ __forceinline__ int64_t sk_begin(int64_t L, int64_t total, int64_t G) {
  return L * total / G;
}
// Logical block whose range holds item i (the largest L with begin <= i).
__device__ __forceinline__ int64_t sk_owner(int64_t i, int64_t total, int64_t G) {
  return ((i + 1) * G - 1) / total;
}

template <class G, class Epi>
__global__ __launch_bounds__(kThreads) void k_rect_streamk(
    const float* __restrict__ X, int64_t ldx, const float* __restrict__ Y, int64_t ldy,
    int64_t nMT, int64_t nTiles, int64_t U, Epi epi, float* __restrict__ part,
    const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[G::MAIN_BYTES];
  __shared__ double red[4];
  const int64_t nb = gridDim.x;
  const int64_t L = xcd_tile(blockIdx.x, nb);
  const int64_t total = nTiles * U;
  const int64_t b = sk_begin(L, total, nb), e = sk_begin(L + 1, total, nb);
  G g;
  int64_t it = b;
  while (it < e) {
    const int64_t tile = it / U;
    const int64_t k0 = it - tile * U;
    const int64_t k1 = (e - tile * U < U) ? e - tile * U : U;
    const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
    g.run(X, ldx, Y, ldy, m0, n0, k0 * G::BK, k1 * G::BK, smem);
    if (k0 == 0 && k1 == U) {
      g.for_each([&](int r, int c, float v) { epi.element(m0 + r, n0 + c, v); });
      epi.end_tile(tile, red);
    } else {
      float* ps = part + (2 * L + (it == b ? 0 : 1)) * (int64_t)(G::BM * G::BN);
      g.for_each([&](int r, int c, float v) { ps[r * G::BN + c] = v; });
    }
    it = tile * U + k1;
  }
}

// Tiles whose K-steps were split between blocks: sum the partial products in
// block order (deterministic) and run the same epilogue.
template <class G, class Epi>
__global__ __launch_bounds__(kThreads) void k_rect_fixup(int64_t nMT, int64_t nTiles, int64_t U,
                                                         int64_t nb, const float* __restrict__ part,
                                                         Epi epi, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[4];
  const int64_t tile = blockIdx.x;
  const int64_t total = nTiles * U;
  const int64_t lo = sk_owner(tile * U, total, nb), hi = sk_owner((tile + 1) * U - 1, total, nb);
  if (lo == hi) return;  // finished inside one block
  const int64_t m0 = (tile % nMT) * G::BM, n0 = (tile / nMT) * G::BN;
  constexpr int E = G::BM * G::BN;
  for (int e = threadIdx.x; e < E; e += kThreads) {
    float s = 0.0f;
    for (int64_t L = lo; L <= hi; ++L) {
      const int64_t bL = sk_begin(L, total, nb);
      if (bL == sk_begin(L + 1, total, nb)) continue;  // empty range
      const int64_t slot = 2 * L + ((L == lo && bL < tile * U) ? 1 : 0);
      s += part[slot * E + e];
    }
    epi.element(m0 + e / G::BN, n0 + e % G::BN, s);
  }
  epi.end_tile(tile, red);
}

// ------------------------------------------------------------------------
// C update of Eq. 5 on the upper tiles of T(W^T, W).  Within a tile only the
// strictly-upper entries (global row < col) are updated, each written at
// (i, j) and mirrored at (j, i), so C stays exactly symmetric and no entry
// is read after another thread wrote it.  The updated tile is staged in LDS
// for the coalesced mirror write and for the per-row sums (sum, sum of
// squares) that give the sigma of Eq. 6: slot J of row i gets the sum over
// the row part, slot I of row j the sum over the column part.  With SIGT the
// sums are taken over the fresh similarities instead, and the sums of
// squares of the updated entries (for |C_.j|^2) go to csq.
constexpr int kCB = 128;
using SymGemm = BlockGemm<kCB, kCB, 2, 2, false, false, 16>;
constexpr int kSymLD = kCB + 1;

template <bool SIGT>
__global__ __launch_bounds__(kThreads) void k_coreg_update(
    const float* __restrict__ W, int64_t ldw, int64_t Nep, float* __restrict__ C, int64_t ldc,
    int64_t Na, const double* __restrict__ ncol, double alpha, double2* __restrict__ cstat,
    double* __restrict__ csq, int64_t ldstat, const int32_t* gate) {
  if (gate && *gate == 0) return;
  constexpr int TILE_BYTES = kCB * kSymLD * 4 * (SIGT ? 2 : 1);
  constexpr int SMEM = SymGemm::MAIN_BYTES > TILE_BYTES ? SymGemm::MAIN_BYTES : TILE_BYTES;
  __shared__ __align__(16) char smem[SMEM];
  const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
  int64_t I, J;
  tri_tile(u, I, J);
  const int64_t m0 = I * kCB, n0 = J * kCB;
  SymGemm g;
  // X = W^T (gene m, tf k) = W[k][m]; Y = W (tf k, gene n) = W[k][n].
  g.run(W, ldw, W, ldw, m0, n0, 0, Nep, smem);
  float* ts = reinterpret_cast<float*>(smem);  // updated values
  float* tt = ts + kCB * kSymLD;               // fresh T (SIGT only)
  // The denominator here is built from column norms of W alone (no growing
  // diagonal), so it is formed in FP64 and the rest runs in FP32:
  // T = acc * rsqrt(den), C <- (1 - alpha) C + alpha T (about 2 ulp).
  const float keep = (float)(1.0 - alpha), alf = (float)alpha;
  g.for_each([&](int rr, int c, float acc) {
    const int64_t gr = m0 + rr, gc = n0 + c;
    float v = 0.0f, tv = 0.0f;
    if (gr < gc && gc < Na) {
      const float den = (float)(ncol[gr] + ncol[gc] - fabs((double)acc));
      const float tsim = den > 0.0f ? acc * __frsqrt_rn(den) : 0.0f;
      const int64_t o = gr * ldc + gc;
      v = keep * C[o] + alf * tsim;
      C[o] = v;
      tv = tsim;
    }
    ts[rr * kSymLD + c] = v;
    if constexpr (SIGT) tt[rr * kSymLD + c] = tv;
  });
  __syncthreads();
  const int t = threadIdx.x;
  // mirror write: C[n0 + q][m0 + p] = ts[p][q] for global m0+p < n0+q
  for (int e = t; e < kCB * kCB; e += kThreads) {
    const int q = e / kCB, p = e % kCB;
    const int64_t gi = m0 + p, gj = n0 + q;
    if (gi < gj && gj < Na) C[gj * ldc + gi] = ts[p * kSymLD + q];
  }
  // per-row partial sums of the off-diagonal entries
  const float* sv = SIGT ? tt : ts;
  if (I == J) {
    if (t < kCB) {
      double s1 = 0.0, s2 = 0.0, c2 = 0.0;
      for (int q = 0; q < kCB; ++q) {  // row part (entries right of the diagonal)
        const double x = sv[t * kSymLD + q];
        s1 += x;
        s2 += x * x;
        if constexpr (SIGT) c2 += (double)ts[t * kSymLD + q] * (double)ts[t * kSymLD + q];
      }
      for (int p = 0; p < kCB; ++p) {  // column part (entries above the diagonal)
        const double x = sv[p * kSymLD + t];
        s1 += x;
        s2 += x * x;
        if constexpr (SIGT) c2 += (double)ts[p * kSymLD + t] * (double)ts[p * kSymLD + t];
      }
      cstat[I * ldstat + m0 + t] = make_double2(s1, s2);
      if constexpr (SIGT) csq[I * ldstat + m0 + t] = c2;
    }
  } else {
    const int q = t & (kCB - 1);
    double s1 = 0.0, s2 = 0.0, c2 = 0.0;
    if (t < kCB) {
      for (int p = 0; p < kCB; ++p) {
        const double x = sv[q * kSymLD + p];
        s1 += x;
        s2 += x * x;
        if constexpr (SIGT) c2 += (double)ts[q * kSymLD + p] * (double)ts[q * kSymLD + p];
      }
      cstat[J * ldstat + m0 + q] = make_double2(s1, s2);
      if constexpr (SIGT) csq[J * ldstat + m0 + q] = c2;
    } else {
      for (int p = 0; p < kCB; ++p) {
        const double x = sv[p * kSymLD + q];
        s1 += x;
        s2 += x * x;
        if constexpr (SIGT) c2 += (double)ts[p * kSymLD + q] * (double)ts[p * kSymLD + q];
      }
      cstat[I * ldstat + n0 + q] = make_double2(s1, s2);
      if constexpr (SIGT) csq[I * ldstat + n0 + q] = c2;
    }
  }
}

// ------------------------------------------------------------------------
// P update, first half: W W^T is only N_e x N_e but has K = N_a, so the
// upper tiles are split over K; each block writes its partial product.
constexpr int kPB = 64;
using CoopGemm = BlockGemm<kPB, kPB, 2, 2, true, true, 32>;

__global__ __launch_bounds__(kThreads) void k_coop_partial(
    const float* __restrict__ W, int64_t ldw, int64_t Nep, int64_t nU, int64_t chunk,
    int64_t Nap, float* __restrict__ part, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[CoopGemm::MAIN_BYTES];
  const int64_t idx = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t u = idx % nU, s = idx / nU;
  int64_t I, J;
  tri_tile(u, I, J);
  const int64_t m0 = I * kPB, n0 = J * kPB;
  int64_t kb = s * chunk, ke = kb + chunk;
  if (kb > Nap) kb = Nap;
  if (ke > Nap) ke = Nap;
  CoopGemm g;
  g.run(W, ldw, W, ldw, m0, n0, kb, ke, smem);
  float* ps = part + s * Nep * Nep;
  g.for_each([&](int r, int c, float v) { ps[(m0 + r) * Nep + n0 + c] = v; });
}

// ------------------------------------------------------------------------
// Blocks of kernel `fn` the whole GPU runs at once (CUs x occupancy).
int64_t resident_blocks(const void* fn) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, 0) != hipSuccess || occ <= 0)
    occ = 1;
  return (int64_t)cus * occ;
}

// Stream-K launch of a rectangular product; nb_max caps the grid (0: one
// block per resident slot, at most kMaxStreamKBlocks).
template <class G, class Epi>
hipError_t launch_rect(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t Mp,
                       int64_t Np, int64_t Kp, Epi epi, float* part, const int32_t* gate,
                       hipStream_t s, int64_t nb_max = 0) {
  static int64_t resident = 0;
  if (!resident) resident = resident_blocks(reinterpret_cast<const void*>(&k_rect_streamk<G, Epi>));
  const int64_t nMT = Mp / G::BM, nNT = Np / G::BN;
  const int64_t nTiles = nMT * nNT, U = Kp / G::BK;
  int64_t nb = nb_max > 0 ? nb_max : resident;
  if (nb > kMaxStreamKBlocks) nb = kMaxStreamKBlocks;
  if (nb > nTiles) nb = nTiles;
  k_rect_streamk<G, Epi><<<dim3((unsigned)nb), dim3(kThreads), 0, s>>>(X, ldx, Y, ldy, nMT, nTiles,
                                                                       U, epi, part, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_rect_fixup<G, Epi><<<dim3((unsigned)nTiles), dim3(kThreads), 0, s>>>(nMT, nTiles, U, nb, part,
                                                                         epi, gate);
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- launch --

int64_t rect_tiles(int64_t Mp, int64_t Np) { return (Mp / RectGemm::BM) * (Np / RectGemm::BN); }
size_t rect_partial_floats() {
  return (size_t)2 * (size_t)kMaxStreamKBlocks * RectGemm::BM * RectGemm::BN;
}

hipError_t launch_tanimoto_store(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                 int64_t Mp, int64_t Np, int64_t Kp, int64_t M, int64_t N,
                                 const double* nx, const double* ny, float* Out, int64_t ldo,
                                 float* part, const int32_t* gate, hipStream_t s) {
  EpiStoreT epi{Out, ldo, M, N, nx, ny};
  return launch_rect<RectGemm>(X, ldx, Y, ldy, Mp, Np, Kp, epi, part, gate, s);
}

hipError_t launch_avail_wupdate(const float* Wold, const float* C, const float* R, float* Wnew,
                                int64_t ld, int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na,
                                const double* nWrow, const double* nC, Rule rule, double* hpart,
                                float* part, const int32_t* gate, hipStream_t s) {
  EpiWUpdate epi{Wold, R, Wnew, ld, Ne, Na, nWrow, nC, rule.alpha, rule.h_undamped, hpart, 0.0};
  return launch_rect<RectGemm>(Wold, ld, C, ld, Nep, Nap, Nap, epi, part, gate, s);
}

int64_t coreg_slots(int64_t Nap) { return Nap / kCB; }

hipError_t launch_coreg_update(const float* W, int64_t ldw, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, const double* nWcol, Rule rule,
                               double2* cstat, double* csq, const int32_t* gate, hipStream_t s) {
  const int64_t nT = Nap / kCB;
  const unsigned nb = (unsigned)(nT * (nT + 1) / 2);
  if (rule.sigma_from_T)
    k_coreg_update<true><<<dim3(nb), dim3(kThreads), 0, s>>>(W, ldw, Nep, C, ldc, Na, nWcol,
                                                             rule.alpha, cstat, csq, Nap, gate);
  else
    k_coreg_update<false><<<dim3(nb), dim3(kThreads), 0, s>>>(W, ldw, Nep, C, ldc, Na, nWcol,
                                                              rule.alpha, cstat, csq, Nap, gate);
  return hipGetLastError();
}

int coop_splits(int64_t Nep, int64_t Nap) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  int64_t s = (512 + nU - 1) / nU;                  // aim at a few hundred blocks
  const int64_t maxs = Nap / (4 * CoopGemm::BK);   // at least 4 K-steps per block
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t launch_coop_partial(const float* W, int64_t ldw, int64_t Nep, int64_t Nap, int splits,
                               float* part, const int32_t* gate, hipStream_t s) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  const int64_t chunk = round_up((Nap + splits - 1) / splits, CoopGemm::BK);
  k_coop_partial<<<dim3((unsigned)(nU * splits)), dim3(kThreads), 0, s>>>(W, ldw, Nep, nU, chunk,
                                                                          Nap, part, gate);
  return hipGetLastError();
}

}  // namespace panda
