// Epilogues of the similarity products and the C-tile update rule, shared
// by the single-network kernels and the grouped (batched) kernels, so both
// forms run the same arithmetic on every tile.
#pragma once

#include "gemm_core.h"

namespace panda {
namespace gemm {

// ------------------------------------------------------------ epilogues --
// The diagonals of P and C grow like exp(2 alpha t) (Eq. 6).  They are kept
// outside the matrices, as FP64 vectors (the matrices hold zeros there), so
// the products see only off-diagonal entries and the diagonal term of each
// dot product is added here in FP64: an FP32 or bf16 accumulator holding
// P_ii W_ij or W_ij C_jj would lose every other term late in a run.
//
// T(X, Y) stored for i < M, j < N (Sec. II-C Tfunction; R of Eq. 3).  With
// xd set, X's diagonal term xd[i] * yv[i][j] is added to the product (R =
// T(P, W): xd = diagonal of P, yv = W); with yd set, Y's diagonal term
// xv[i][j] * yd[j] (T(W, C): xv = W, yd = diagonal of C).
struct EpiStoreT {
  float* out;
  int64_t ldo, M, N;
  const double* nx;
  const double* ny;
  const double* xd = nullptr;
  const float* yv = nullptr;
  int64_t ldyv = 0;
  const double* yd = nullptr;
  const float* xv = nullptr;
  int64_t ldxv = 0;
  __device__ __forceinline__ void element(int64_t r, int64_t c, float acc) {
    if (r < M && c < N) {
      double dot = (double)acc;
      if (xd) dot += xd[r] * (double)yv[r * ldyv + c];
      if (yd) dot += (double)xv[r * ldxv + c] * yd[c];
      out[r * ldo + c] = (float)tanimoto(dot, nx[r], ny[c]);
    }
  }
  // NE entries at once, the same arithmetic as element(); entries past
  // M x N read a clamped in-range entry and store nothing.
  template <int NE>
  __device__ __forceinline__ void block(const int64_t (&r)[NE], const int64_t (&c)[NE],
                                        const float (&acc)[NE]) {
    float v[NE];
    if (xd) {
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int64_t rr = r[k] < M ? r[k] : M - 1, cc = c[k] < N ? c[k] : N - 1;
        double dot = (double)acc[k];
        dot += xd[rr] * (double)yv[rr * ldyv + cc];
        v[k] = (float)tanimoto(dot, nx[rr], ny[cc]);
      }
    } else if (yd) {
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int64_t rr = r[k] < M ? r[k] : M - 1, cc = c[k] < N ? c[k] : N - 1;
        double dot = (double)acc[k];
        dot += (double)xv[rr * ldxv + cc] * yd[cc];
        v[k] = (float)tanimoto(dot, nx[rr], ny[cc]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int64_t rr = r[k] < M ? r[k] : M - 1, cc = c[k] < N ? c[k] : N - 1;
        v[k] = (float)tanimoto((double)acc[k], nx[rr], ny[cc]);
      }
    }
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (r[k] < M && c[k] < N) out[r[k] * ldo + c[k]] = v[k];
  }
  __device__ __forceinline__ void end_tile(int64_t, double*) {}
};

// A = T(W, C) (Eq. 4) folded into the W update of Eq. 2, with the tile's
// share of the h sum of Eq. 7.  The new W goes to a second buffer because
// the old one is still an operand of other blocks.  C's diagonal term
// W_ij * C_jj is added to the product from the FP64 vector cd.
struct EpiWUpdate {
  const float* Wold;
  const float* R;
  float* Wnew;
  int64_t ld, Ne, Na;
  const double* nx;  // |W_i.|^2
  const double* ny;  // |C_.j|^2
  const double* cd;  // diagonal of C
  double alpha;
  int32_t h_undamped;
  double* hpart;
  double hsum;
  // the entry's old W and R, fetched ahead by epi_tile where it can
  using Pre = float2;
  __device__ __forceinline__ Pre fetch(int64_t r, int64_t c) const {
    if (r < Ne && c < Na) {
      const int64_t o = r * ld + c;
      return make_float2(Wold[o], R[o]);
    }
    return make_float2(0.0f, 0.0f);
  }
  __device__ __forceinline__ void element_pre(int64_t r, int64_t c, float acc, Pre pre) {
    if (r < Ne && c < Na) {
      const double w = pre.x;
      double dot = (double)acc;
      dot += w * cd[c];
      const double a = tanimoto(dot, nx[r], ny[c]);
      const double pred = 0.5 * (a + (double)pre.y);
      const float wn = (float)((1.0 - alpha) * w + alpha * pred);
      Wnew[r * ld + c] = wn;
      hsum += h_undamped ? fabs(pred - w) : fabs((double)wn - w);
    }
  }
  __device__ __forceinline__ void element(int64_t r, int64_t c, float acc) {
    element_pre(r, c, acc, fetch(r, c));
  }
  // NE entries at once, the same arithmetic as element_pre and the same
  // order of the h sum; entries past Ne x Na read a clamped in-range entry
  // and neither store nor count.
  template <int NE>
  __device__ __forceinline__ void block(const int64_t (&r)[NE], const int64_t (&c)[NE],
                                        const float (&acc)[NE]) {
    float wn[NE];
    double dh[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int64_t rr = r[k] < Ne ? r[k] : Ne - 1, cc = c[k] < Na ? c[k] : Na - 1;
      const int64_t o = rr * ld + cc;
      const double w = Wold[o];
      double dot = (double)acc[k];
      dot += w * cd[cc];
      const double a = tanimoto(dot, nx[rr], ny[cc]);
      const double pred = 0.5 * (a + (double)R[o]);
      wn[k] = (float)((1.0 - alpha) * w + alpha * pred);
      dh[k] = h_undamped ? fabs(pred - w) : fabs((double)wn[k] - w);
    }
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (r[k] < Ne && c[k] < Na) {
        Wnew[r[k] * ld + c[k]] = wn[k];
        hsum += dh[k];
      }
  }
  __device__ __forceinline__ void end_tile(int64_t tile, double* red) {
    const double s = block_sum(hsum, red);
    if (threadIdx.x == 0) hpart[tile] = s;
    hsum = 0.0;
  }
};

// Tile configurations.  Rectangular products: 64 x 128 tiles (N_e = 700 pads
// to 704 = 11 x 64), 4 waves side by side.  Symmetric C product: 128 x 128.
using RectF32 = BlockGemm<64, 128, 1, 4, true, false, 16>;
using RectF32P = BlockGemm<64, 128, 1, 4, true, false, 16, true>;  // A product, packed C
using RectB3 = BlockGemmB3<64, 128, 1, 4>;  // R: K = N_e is short, register staging wins
static_assert(RectF32::BM == RectB3::BM && RectF32::BN == RectB3::BN, "one tile grid");
// The split-BF16 A product moves its operands by direct loads into LDS, and
// the memory side bounds it: 256 x 128 tiles move half the bytes per MFMA of
// 64 x 128 ones.  Eight waves of 64 x 64, two per SIMD, so that one wave's
// waits (loads landing, barriers) are covered by the other's MFMAs: 6-8 %
// faster than four waves of 64 x 128 at T=700, G=18000 (same products in the
// same order per entry).  N_e is padded to the tile (704 -> 768) by clamped
// reads; waves whose rows all lie in the padding skip their MFMAs.  (A block
// spanning all of N_e with a 64-gene strip of C reads C once but re-reads
// W's planes per block: 2.6 ms against 1.46 ms.)
using RectB3D = BlockGemmB3P<256, 128, 4, 2>;
using RectB3DP = BlockGemmB3P<256, 128, 4, 2, true, 3, 32, true>;  // the same on packed C
using SymF32 = BlockGemm<128, 128, 2, 2, false, false, 16>;
using SymB3 = BlockGemmB3P<128, 128, 2, 2, false, 2>;  // direct-to-LDS, two stages (two blocks per CU)
using CoopF32 = BlockGemm<64, 64, 2, 2, true, true, 32>;
using CoopB3 = BlockGemmB3<64, 64, 2, 2>;
// The single-network W W^T partials: each block's K chunk is ~70 K-tiles, long
// enough for the direct-to-LDS pipeline with three stages (two K-tiles in
// flight while one is multiplied); same products in the same order.
using CoopB3P = BlockGemmB3P<64, 64, 2, 2, false, 3>;
static_assert(CoopF32::BK == CoopB3::BK, "one K split");

// ------------------------------------------------------------------------
// C update of Eq. 5 on the upper tiles of T(W^T, W).  Within a tile only the
// strictly-upper entries (global row < col) are updated, each written at
// (i, j) and mirrored at (j, i), so C stays exactly symmetric and no entry
// is read after another thread wrote it.  The updated tile is staged in LDS
// for the coalesced mirror write and for the per-row sums (sum, sum of
// squares) that give the sigma of Eq. 6: slot J of row i gets the sum over
// the row part, slot I of row j the sum over the column part.  With SIGT the
// sums are taken over the fresh similarities instead, and the sums of
// squares of the updated entries (for |C_.j|^2) go to csq.  With shadows
// (split-BF16 form) the hi/lo planes of the new entries are written too; the
// diagonal of the planes stays zero.
// With PK, C is packed (packed_tile): the tile is read and written in its own
// slot, row length kPT, and an off-diagonal tile has no mirror image to
// write; a diagonal tile gets its lower triangle as well.
constexpr int kCB = 128;
static_assert(kCB == kPT, "C-update tiles are the packed tiles");
constexpr int kSymLD = kCB + 1;

// EpiStoreT with X's diagonal term (xd set: R = T(P, W)) on a 128 x 128 tile
// of a block GEMM of 256 threads: the tile's per-row values (xd, nx) and
// per-column norms (ny) are staged in LDS once, then every entry takes the
// arithmetic of EpiStoreT::block (the same results bit for bit), the W
// entries of NB rows of a column loaded together.
template <int NB, class G>
__device__ __forceinline__ void store_t_tile_xd(const G& g, char* smem, const EpiStoreT& e,
                                                int64_t m0, int64_t n0) {
  static_assert(G::BM == kCB && G::BN == kCB && G::NT == 2 * kCB, "128 x 128 tiles, 256 threads");
  static_assert(16 % NB == 0, "whole runs per accumulator column");
  double* sxd = reinterpret_cast<double*>(smem);  // after the product's last LDS reads
  double* snx = sxd + kCB;
  double* sny = snx + kCB;
  const int t = threadIdx.x;
  __syncthreads();
  if (t < kCB) {
    const int64_t r = m0 + t < e.M ? m0 + t : e.M - 1;
    sxd[t] = e.xd[r];
    snx[t] = e.nx[r];
  } else {
    const int64_t c = n0 + (t - kCB) < e.N ? n0 + (t - kCB) : e.N - 1;
    sny[t - kCB] = e.ny[c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < G::TM; ++i)
#pragma unroll
    for (int j = 0; j < G::TN; ++j) {
      const int c = g.col_of(j);
      const int64_t gc = n0 + c, cc = gc < e.N ? gc : e.N - 1;
      const double ny = sny[c];
#pragma unroll
      for (int r0 = 0; r0 < 16; r0 += NB) {
        float yv[NB], v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int64_t gr = m0 + g.row_of(i, r0 + k), rr = gr < e.M ? gr : e.M - 1;
          yv[k] = e.yv[rr * e.ldyv + cc];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int rl = g.row_of(i, r0 + k);
          double dot = (double)g.acc[i][j][r0 + k];
          dot += sxd[rl] * (double)yv[k];
          v[k] = (float)tanimoto(dot, snx[rl], ny);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int64_t gr = m0 + g.row_of(i, r0 + k);
          if (gr < e.M && gc < e.N) e.out[gr * e.ldo + gc] = v[k];
        }
      }
    }
}

// Fresh similarity of one C-tile entry from its product and the squared
// norms nr = |W_.gr|^2, nc = |W_.gc|^2 (FP32 math, see above); 0 outside the
// strictly-upper real part.
// Computed without branches (the entries outside, or with den <= 0, select
// 0 after the fact), so a wave's entries need no divergent paths.
__device__ __forceinline__ float coreg_sim(float acc, int64_t gr, int64_t gc, int64_t Na,
                                           double nr, double nc) {
  const float den = (float)(nr + nc - fabs((double)acc));
  const float v = acc * __frsqrt_rn(den);
  return (gr < gc && gc < Na && den > 0.0f) ? v : 0.0f;
}

// The squared norm this thread stages for tile (I, J): threads 0-127 the
// tile's rows, 128-255 its columns.  Loaded before the tile's product (the
// load is then long complete when the epilogue needs it).
__device__ __forceinline__ double coreg_norm_load(const double* __restrict__ ncol, int64_t I,
                                                  int64_t J, int64_t Na) {
  const int t = threadIdx.x;
  const int64_t k = t < kCB ? I * kCB + t : J * kCB + (t - kCB);
  return k < Na ? ncol[k] : 0.0;
}

// Everything of the C update after the similarities of tile (I, J) are
// known; fv(f) calls f(rr, c, tsim) for every entry the thread holds.  The
// similarities are staged in LDS first, so that the read-modify-write of C
// and its mirror image go to memory 16 bytes per lane, row-contiguous.
constexpr int kC4 = kCB / 4;                     // float4 per tile row
constexpr int kChunks = kCB * kC4 / kThreads;    // float4 per thread

template <bool SIGT, bool PK, class FV>
__device__ __forceinline__ void coreg_tile_update(FV&& fv, char* smem, int64_t I, int64_t J,
                                                  float* __restrict__ C, int64_t ldc, int64_t Na,
                                                  double alpha, double2* __restrict__ cstat,
                                                  double* __restrict__ csq, int64_t ldstat) {
  static_assert(kChunks * kThreads == kCB * kC4, "whole chunks");
  const int64_t m0 = I * kCB, n0 = J * kCB;
  // address of entry (rr, c) of the tile: in C, or in the tile's packed slot
  float* const Ct = PK ? C + packed_tile(I, J) * (kCB * kCB) : C;
  const int64_t ldt = PK ? kCB : ldc;
  const int64_t r0 = PK ? 0 : m0, c0 = PK ? 0 : n0;
  float* ts = reinterpret_cast<float*>(smem);  // fresh T, then the updated values
  float* tt = ts + kCB * kSymLD;               // fresh T (SIGT only)
  const int t = threadIdx.x;
  fv([&](int rr, int c, float tsim) {
    ts[rr * kSymLD + c] = tsim;
    if constexpr (SIGT) tt[rr * kSymLD + c] = tsim;
  });
  __syncthreads();
  const float keep = (float)(1.0 - alpha), alf = (float)alpha;
  // C (N_a^2 entries, far beyond the last-level cache) is read and written
  // with non-temporal hints: no block reads it again before it is evicted.
  f4 old[kChunks];
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {  // all old values in flight together
    const int id = t + k * kThreads, rr = id / kC4, c = (id % kC4) * 4;
    old[k] = __builtin_nontemporal_load(
        reinterpret_cast<const f4*>(Ct + (r0 + rr) * ldt + c0 + c));
  }
  // this thread's fresh similarities, all read before the first write-back
  // below (a read after a write to the staged tile would wait for it)
  float fresh[kChunks][4];
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int id = t + k * kThreads, rr = id / kC4, c = (id % kC4) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) fresh[k][e] = ts[rr * kSymLD + c + e];
  }
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int id = t + k * kThreads, rr = id / kC4, c = (id % kC4) * 4;
    const int64_t gr = m0 + rr, gc = n0 + c;
    f4 nv;
    bool upper[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      upper[e] = gr < gc + e && gc + e < Na;  // strictly upper and real
      const float v = upper[e] ? keep * old[k][e] + alf * fresh[k][e] : 0.0f;
      nv[e] = upper[e] ? v : old[k][e];
      ts[rr * kSymLD + c + e] = v;
    }
    float* dst = Ct + (r0 + rr) * ldt + c0 + c;
    if (I != J) {
      // every entry of an upper off-diagonal tile is strictly upper; padding
      // columns keep their zeros
      __builtin_nontemporal_store(nv, reinterpret_cast<f4*>(dst));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (upper[e]) dst[e] = nv[e];
    }
  }
  __syncthreads();
  // mirror: C[n0 + q][m0 + p] = ts[p][q] for the strictly-upper entries (a
  // packed off-diagonal tile has no mirror image to write)
#pragma unroll 4
  for (int k = 0; k < kChunks; ++k) {
    if (PK && I != J) break;
    const int id = t + k * kThreads, q = id / kC4, p = (id % kC4) * 4;
    const int64_t gj = n0 + q, gi = m0 + p;
    if (gj >= Na) continue;
    f4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = ts[(p + e) * kSymLD + q];
    float* dst = PK ? Ct + q * ldt + p : C + gj * ldc + gi;
    if (gi + 3 < gj) {
      __builtin_nontemporal_store(v, reinterpret_cast<f4*>(dst));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (gi + e < gj) dst[e] = v[e];
    }
  }
  // per-row partial sums of the off-diagonal entries, each over four
  // interleaved partial sums (four independent FP64 chains instead of one)
  const float* sv = SIGT ? tt : ts;
  double a1[4] = {0.0, 0.0, 0.0, 0.0}, a2[4] = {0.0, 0.0, 0.0, 0.0}, a3[4] = {0.0, 0.0, 0.0, 0.0};
  // entries base + e * step, e = 0 .. kCB - 1
  auto walk = [&](int base, int step) {
#pragma unroll 8
    for (int e = 0; e < kCB; e += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int at = base + (e + u) * step;
        const double x = sv[at];
        a1[u] += x;
        a2[u] += x * x;
        if constexpr (SIGT) a3[u] += (double)ts[at] * (double)ts[at];
      }
    }
  };
  auto fold = [](const double (&a)[4]) { return (a[0] + a[1]) + (a[2] + a[3]); };
  if (I == J) {
    if (t < kCB) {
      walk(t * kSymLD, 1);  // row part (entries right of the diagonal)
      walk(t, kSymLD);      // column part (entries above the diagonal)
      cstat[I * ldstat + m0 + t] = make_double2(fold(a1), fold(a2));
      if constexpr (SIGT) csq[I * ldstat + m0 + t] = fold(a3);
    }
  } else {
    const int q = t & (kCB - 1);
    if (t < kCB) {
      walk(q * kSymLD, 1);
      cstat[J * ldstat + m0 + q] = make_double2(fold(a1), fold(a2));
      if constexpr (SIGT) csq[J * ldstat + m0 + q] = fold(a3);
    } else {
      walk(q, kSymLD);
      cstat[I * ldstat + n0 + q] = make_double2(fold(a1), fold(a2));
      if constexpr (SIGT) csq[I * ldstat + n0 + q] = fold(a3);
    }
  }
}

// The C update of tile (I, J) from the accumulators of block GEMM g; nval
// is this thread's coreg_norm_load, staged in LDS beside the tile.
template <bool SIGT>
constexpr int coreg_tile_bytes() {
  return kCB * kSymLD * 4 * (SIGT ? 2 : 1);
}
template <bool SIGT, bool PK, class G>
__device__ __forceinline__ void coreg_epilogue(const G& g, char* smem, int64_t I, int64_t J,
                                               float* __restrict__ C, int64_t ldc, int64_t Na,
                                               double nval, double alpha,
                                               double2* __restrict__ cstat,
                                               double* __restrict__ csq, int64_t ldstat) {
  static_assert(G::BM == kCB && G::BN == kCB && kThreads == 2 * kCB, "square tiles");
  const int64_t m0 = I * kCB, n0 = J * kCB;
  double* nsh = reinterpret_cast<double*>(smem + coreg_tile_bytes<SIGT>());
  nsh[threadIdx.x] = nval;
  __syncthreads();
  // the norms of this lane's rows and columns, all read before the first
  // store of the staged tile (reads after a store to the same shared array
  // would each wait for the one before)
  double nr[G::TM][16], nc[G::TN];
#pragma unroll
  for (int i = 0; i < G::TM; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) nr[i][r] = nsh[g.row_of(i, r)];
#pragma unroll
  for (int j = 0; j < G::TN; ++j) nc[j] = nsh[kCB + g.col_of(j)];
  coreg_tile_update<SIGT, PK>(
      [&](auto&& f) {
#pragma unroll
        for (int i = 0; i < G::TM; ++i)
#pragma unroll
          for (int j = 0; j < G::TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int rr = g.row_of(i, r), c = g.col_of(j);
              f(rr, c, coreg_sim(g.acc[i][j][r], m0 + rr, n0 + c, Na, nr[i][r], nc[j]));
            }
      },
      smem, I, J, C, ldc, Na, alpha, cstat, csq, ldstat);
}

// Shared memory of the C update with block GEMM G: the larger of the main
// loop's stages and the staged tile (two tiles with SIGT) with the 256
// staged norms.
template <class G, bool SIGT>
constexpr int coreg_smem_bytes() {
  constexpr int TILE = coreg_tile_bytes<SIGT>() + 2 * kCB * 8;
  return G::MAIN_BYTES > TILE ? G::MAIN_BYTES : TILE;
}

// Co-expression prior (Sec. II-A): upper tile (I, J) of Z Z^T, Z the
// centred rows of the expression matrix scaled to unit norm, holds Pearson
// correlations.  The tile goes through LDS so that both its own rows and,
// off the diagonal, its mirror image at (J, I) are stored row-contiguous.
// Only entries inside the G x G result are written; the diagonal is 1.
template <class G>
__device__ __forceinline__ void corr_sym_epilogue(const G& g, char* smem, int64_t I, int64_t J,
                                                  float* __restrict__ C, int64_t ldc, int64_t n) {
  static_assert(G::BM == kCB && G::BN == kCB, "square tiles");
  constexpr int kRows = kThreads / kCB;  // tile rows stored per pass
  float* ts = reinterpret_cast<float*>(smem);
  g.for_each([&](int rr, int c, float v) { ts[rr * kSymLD + c] = v; });
  __syncthreads();
  const int64_t m0 = I * kCB, n0 = J * kCB;
  const int c = threadIdx.x % kCB, r0 = threadIdx.x / kCB;
  for (int rr = r0; rr < kCB; rr += kRows) {
    const int64_t gr = m0 + rr, gc = n0 + c;
    if (gr < n && gc < n)
      __builtin_nontemporal_store(gr == gc ? 1.0f : ts[rr * kSymLD + c], C + gr * ldc + gc);
  }
  if (I == J) return;  // a diagonal tile holds both triangles itself
  for (int q = r0; q < kCB; q += kRows) {
    const int64_t gr = n0 + q, gc = m0 + c;
    if (gr < n && gc < n) __builtin_nontemporal_store(ts[c * kSymLD + q], C + gr * ldc + gc);
  }
}

template <class G>
constexpr int corr_smem_bytes() {
  constexpr int TILE = kCB * kSymLD * 4;
  return G::MAIN_BYTES > TILE ? G::MAIN_BYTES : TILE;
}

// P update, first half: W W^T is only N_e x N_e but has K = N_a, so its
// upper tiles are split over K into partial products.
constexpr int kPB = (int)kCoopTile;

}  // namespace gemm
}  // namespace panda
