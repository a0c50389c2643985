// The similarity products of one PANDA iteration, in the two arithmetic
// forms the library offers, with the update rules fused into the epilogues:
//   R = T(P, W)                 Eq. 3, stored (also the stand-alone Tfunction)
//   A = T(W, C) + W update      Eq. 4 folded into Eq. 2, h partials of Eq. 7
//   C update                    Eq. 5 on upper tiles of T(W^T, W), mirrored,
//                               with the per-row sums for the sigma of Eq. 6
//   W W^T partial products      first half of the P update (Eq. 5), split-K
// FP32 form: v_mfma_f32_32x32x2f32 on FP32 operands.  Split-BF16 form: the
// same products as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 with an
// FP32 accumulator; the diagonals of P and C (which grow like exp(2 alpha t),
// Eq. 6) are kept out of the bf16 operands and added back in FP64 in the
// epilogue (P_ii W_ij in R, W_ij C_jj in A).  Norms, denominators and h stay
// FP64 in both forms.
#include "epilogues.h"

namespace panda {
namespace {

using namespace gemm;

// R = T(P, W) (Eq. 3) on 128 x 128 tiles of the symmetric product's block,
// the same K = N_e as the C update: X = P (split-BF16: P's planes with rows
// past N_e clamped; FP32: P read k-major, rows past N_e read into slack),
// Y = W^T (its planes) or W; rows past N_e are never stored.  Both forms
// compute the next iteration's R inside the C update's launch, as soon as P,
// its diagonal and W's norms (and planes) are new: its tiles fill the
// launch's last wave of C tiles.
template <class G>
struct NextR {
  typename G::Ops ops;
  EpiStoreT epi;
};
// An entry of the tile order with this bit set is R tile (entry & 0xffff,
// (entry >> 16) & 0x7fff) (row tile of P, column tile of W); the others are
// C tiles (I, J) = (entry & 0xffff, entry >> 16).
constexpr uint32_t kNextRTile = 0x80000000u;
// R's epilogue: W entries of runs of 16 rows of a column loaded together.
constexpr int kNextRRun = 16;

// The product of the tile, then the update in its epilogue (two blocks per
// CU, so one block's epilogue overlaps the other's products).  With NR the
// order also holds R tiles (kNextRTile).
template <class G, bool SIGT, bool PK, bool NR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_coreg_update(
    typename G::Ops ops, int64_t Kp, float* __restrict__ C, int64_t ldc, int64_t Na,
    const double* __restrict__ ncol, double alpha, double2* __restrict__ cstat,
    double* __restrict__ csq, int64_t ldstat, const uint32_t* __restrict__ order,
    const int32_t* gate, NextR<G> nr) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[coreg_smem_bytes<G, SIGT>()];
  const uint32_t ij = order[xcd_tile(blockIdx.x, gridDim.x)];
  if constexpr (NR) {
    if (ij & kNextRTile) {
      const int64_t m0 = (int64_t)(ij & 0xffff) * kCB, n0 = (int64_t)((ij >> 16) & 0x7fff) * kCB;
      G g;
      g.run(nr.ops, m0, n0, 0, Kp, smem);
      store_t_tile_xd<kNextRRun>(g, smem, nr.epi, m0, n0);
      return;
    }
  }
  const int64_t I = ij & 0xffff, J = ij >> 16;
  const int64_t m0 = I * kCB, n0 = J * kCB;
  const double nval = coreg_norm_load(ncol, I, J, Na);
  G g;
  g.run(ops, m0, n0, 0, Kp, smem);
  coreg_epilogue<SIGT, PK>(g, smem, I, J, C, ldc, Na, nval, alpha, cstat, csq, ldstat);
}

// R alone on the same tiles (same arithmetic, so R is the same bit for bit
// whichever launch computed it): block b is tile (b % nRT, b / nRT).
template <class G>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_resp_tiles(
    NextR<G> nr, int64_t Kp, int64_t nRT, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ __align__(16) char smem[G::MAIN_BYTES];
  const int64_t b = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t m0 = (b % nRT) * kCB, n0 = (b / nRT) * kCB;
  G g;
  g.run(nr.ops, m0, n0, 0, Kp, smem);
  store_t_tile_xd<kNextRRun>(g, smem, nr.epi, m0, n0);
}

// Pearson correlations: one upper 128 x 128 tile of Z Z^T per block, both
// operands read from Z^T (samples x genes), stored at the tile and mirrored.
template <class G>
__global__ __launch_bounds__(kThreads) void k_corr_sym(typename G::Ops ops, int64_t Kp,
                                                       float* __restrict__ C, int64_t ldc,
                                                       int64_t n) {
  __shared__ __align__(16) char smem[corr_smem_bytes<G>()];
  int64_t I, J;
  tri_tile(xcd_tile(blockIdx.x, gridDim.x), I, J);
  G g;
  g.run(ops, I * kCB, J * kCB, 0, Kp, smem);
  corr_sym_epilogue(g, smem, I, J, C, ldc, n);
}

// ------------------------------------------------------------------------
// P update, first half: each block writes the partial product of one upper
// tile over one K chunk.

template <class G>
__global__ __launch_bounds__(kThreads) void k_coop_partial(typename G::Ops ops, int64_t Nep,
                                                           int64_t nU, int64_t chunk, int64_t Nap,
                                                           float* __restrict__ part,
                                                           const int32_t* gate) {
  if (gate && *gate == 0) return;
  static_assert(G::BM == kPB && G::BN == kPB, "square tiles");
  __shared__ __align__(16) char smem[G::MAIN_BYTES];
  const int64_t idx = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t u = idx % nU, s = idx / nU;
  int64_t I, J;
  tri_tile(u, I, J);
  const int64_t m0 = I * kPB, n0 = J * kPB;
  int64_t kb = s * chunk, ke = kb + chunk;
  if (kb > Nap) kb = Nap;
  if (ke > Nap) ke = Nap;
  G g;
  g.run(ops, m0, n0, kb, ke, smem);
  float* ps = part + s * Nep * Nep;
  g.for_each([&](int r, int c, float v) { ps[(m0 + r) * Nep + n0 + c] = v; });
}

}  // namespace

// ---------------------------------------------------------------- launch --

int64_t rect_tiles(int64_t Mp, int64_t Np) { return (Mp / RectF32::BM) * (Np / RectF32::BN); }
int64_t rect_tiles_b3(int64_t Mp, int64_t Np) {
  return ((Mp + RectB3D::BM - 1) / RectB3D::BM) * (Np / RectB3D::BN);
}
static_assert(kFixParts<RectB3D> == kFixParts<RectB3DP>, "one slot layout for both C layouts");
int64_t rect_hpart_slots_b3(int64_t Mp, int64_t Np) {
  return rect_tiles_b3(Mp, Np) * kFixParts<RectB3D>;
}
size_t rect_partial_floats() {
  return (size_t)2 * (size_t)kMaxStreamKBlocks * RectF32::BM * RectF32::BN;
}

hipError_t launch_tanimoto_store(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                 int64_t Mp, int64_t Np, int64_t Kp, int64_t M, int64_t N,
                                 const double* nx, const double* ny, float* Out, int64_t ldo,
                                 float* part, const int32_t* gate, hipStream_t s,
                                 const double* yd) {
  EpiStoreT epi{Out, ldo, M, N, nx, ny};
  if (yd) {  // Y's diagonal held apart: its term X_ij Y_jj (X square with Y)
    epi.yd = yd;
    epi.xv = X;
    epi.ldxv = ldx;
  }
  return launch_rect<RectF32>(OpsF32{X, ldx, Y, ldy}, Mp, Np, Kp, epi, part, gate, s);
}

hipError_t launch_corr(const float* Zt, int64_t Gp, int64_t Sp, int64_t G, float* C, int64_t ldc,
                       hipStream_t s) {
  // X = Z stored sample-major (Z^T), as W^T is read from W in the C update.
  if (Gp % kCB || Sp % SymF32::BK || G > Gp) return hipErrorInvalidValue;
  const int64_t nT = Gp / kCB;
  k_corr_sym<SymF32><<<dim3((unsigned)(nT * (nT + 1) / 2)), dim3(kThreads), 0, s>>>(
      OpsF32{Zt, Gp, Zt, Gp}, Sp, C, ldc, G);
  return hipGetLastError();
}

hipError_t launch_resp(const float* P, int64_t ldp, const double* dP, const float* W, int64_t ldw,
                       int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na, const double* nP,
                       const double* nWc, float* R, float* part, const int32_t* gate,
                       hipStream_t s) {
  EpiStoreT epi{R, ldw, Ne, Na, nP, nWc, dP, W, ldw};
  return launch_rect<RectF32>(OpsF32{P, ldp, W, ldw}, Nep, Nap, Nep, epi, part, gate, s);
}

hipError_t launch_resp_b3(const bf16_t* Ph, const bf16_t* Pl, int64_t ldp, const double* dP,
                          const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nep,
                          int64_t Nap, int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                          const double* nP, const double* nWc, float* R, float* part,
                          const int32_t* gate, hipStream_t s) {
  EpiStoreT epi{R, ldw, Ne, Na, nP, nWc, dP, W, ldw};
  return launch_rect<RectB3>(OpsB3{Ph, Pl, ldp, Wth, Wtl, ldwt}, Nep, Nap, Nep, epi, part, gate, s);
}

hipError_t launch_avail_wupdate(const float* Wold, const float* C, const double* dC,
                                const float* R, float* Wnew, int64_t ld, int64_t Nep, int64_t Nap,
                                int64_t Ne, int64_t Na, const double* nWrow, const double* nC,
                                Rule rule, double* hpart, float* part, const int32_t* gate,
                                hipStream_t s, bool packed) {
  EpiWUpdate epi{Wold, R, Wnew, ld, Ne, Na, nWrow, nC, dC, rule.alpha, rule.h_undamped, hpart, 0.0};
  if (packed)
    return launch_rect<RectF32P>(OpsF32P{Wold, ld, C}, Nep, Nap, Nap, epi, part, gate, s);
  return launch_rect<RectF32>(OpsF32{Wold, ld, C, ld}, Nep, Nap, Nap, epi, part, gate, s);
}

hipError_t launch_avail_wupdate_b3(const bf16_t* Wh, const bf16_t* Wl, const float* Wold,
                                   const float* C, const double* dC, const float* R, float* Wnew,
                                   int64_t ld, int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na,
                                   const double* nWrow, const double* nC, Rule rule,
                                   double* hpart, float* part, const int32_t* gate,
                                   hipStream_t s, bool packed) {
  EpiWUpdate epi{Wold, R, Wnew, ld, Ne, Na, nWrow, nC, dC, rule.alpha, rule.h_undamped, hpart, 0.0};
  // C is symmetric: its row n is the column n the product needs
  const int64_t Mp = (Nep + RectB3D::BM - 1) / RectB3D::BM * RectB3D::BM;
  if (packed)
    return launch_rect<RectB3DP>(OpsB3FP{Wh, Wl, ld, C, Nep}, Mp, Nap, Nap, epi, part, gate, s);
  return launch_rect<RectB3D>(OpsB3F{Wh, Wl, ld, C, ld, Nep}, Mp, Nap, Nap, epi, part, gate, s);
}

int64_t coreg_slots(int64_t Nap) { return Nap / kCB; }
int64_t coreg_tiles(int64_t Nap) { return (Nap / kCB) * (Nap / kCB + 1) / 2; }

void coreg_order_fill(int64_t Nap, int group, uint32_t* out) {
  const int64_t nT = Nap / kCB, nG = (nT + group - 1) / group;
  int64_t k = 0;
  for (int64_t bj = 0; bj < nG; ++bj)
    for (int64_t bi = 0; bi <= bj; ++bi)
      for (int64_t J = bj * group; J < (bj + 1) * group && J < nT; ++J)
        for (int64_t I = bi * group; I < (bi + 1) * group && I <= J; ++I)
          out[k++] = (uint32_t)(I | (J << 16));
}

template <class G, bool PK, bool NR>
static hipError_t coreg_launch_pk(const typename G::Ops& ops, int64_t Nep, float* C, int64_t ldc,
                                  int64_t Nap, int64_t Na, const double* nWcol, Rule rule,
                                  double2* cstat, double* csq, const uint32_t* order,
                                  const int32_t* gate, hipStream_t s, const NextR<G>& nr,
                                  int64_t extra) {
  const unsigned nb = (unsigned)(coreg_tiles(Nap) + extra);
  if (rule.sigma_from_T)
    k_coreg_update<G, true, PK, NR><<<dim3(nb), dim3(kThreads), 0, s>>>(
        ops, Nep, C, ldc, Na, nWcol, rule.alpha, cstat, csq, Nap, order, gate, nr);
  else
    k_coreg_update<G, false, PK, NR><<<dim3(nb), dim3(kThreads), 0, s>>>(
        ops, Nep, C, ldc, Na, nWcol, rule.alpha, cstat, csq, Nap, order, gate, nr);
  return hipGetLastError();
}

template <class G, bool NR = false>
static hipError_t coreg_launch(const typename G::Ops& ops, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, const double* nWcol, Rule rule,
                               double2* cstat, double* csq, const uint32_t* order,
                               const int32_t* gate, hipStream_t s, bool packed,
                               const NextR<G>& nr = NextR<G>{}, int64_t extra = 0) {
  return packed ? coreg_launch_pk<G, true, NR>(ops, Nep, C, ldc, Nap, Na, nWcol, rule, cstat,
                                               csq, order, gate, s, nr, extra)
                : coreg_launch_pk<G, false, NR>(ops, Nep, C, ldc, Nap, Na, nWcol, rule, cstat,
                                                csq, order, gate, s, nr, extra);
}

hipError_t launch_coreg_update(const float* W, int64_t ldw, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, const double* nWcol, Rule rule,
                               double2* cstat, double* csq, const uint32_t* order,
                               const int32_t* gate, hipStream_t s, bool packed) {
  // X = W^T (gene m, tf k) = W[k][m]; Y = W (tf k, gene n) = W[k][n].
  return coreg_launch<SymF32>(OpsF32{W, ldw, W, ldw}, Nep, C, ldc, Nap, Na, nWcol, rule, cstat,
                              csq, order, gate, s, packed);
}

hipError_t launch_coreg_update_b3(const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nep,
                                  float* C, int64_t ldc, int64_t Nap, int64_t Na,
                                  const double* nWcol, Rule rule, double2* cstat, double* csq,
                                  const uint32_t* order, const int32_t* gate, hipStream_t s,
                                  bool packed) {
  // X = Yt = W^T stored gene-major: row m of W^T is column m of W.  Only the
  // FP32 C is written; the next A product splits it while staging.
  return coreg_launch<SymB3>(OpsB3{Wth, Wtl, ldwt, Wth, Wtl, ldwt}, Nep, C, ldc, Nap, Na, nWcol,
                             rule, cstat, csq, order, gate, s, packed);
}

int64_t next_r_row_tiles(int64_t Nep) { return (Nep + kCB - 1) / kCB; }
int64_t next_r_tiles(int64_t Nep, int64_t Nap) { return next_r_row_tiles(Nep) * (Nap / kCB); }

void coreg_next_r_order_fill(int64_t Nep, int64_t Nap, const uint32_t* corder, uint32_t* out) {
  // each XCD's share of the launch (the ranges xcd_tile maps block indices
  // to) takes its share of the C tiles in their order, then its share of the
  // R tiles, column tile by column tile (R tiles of one column share W's
  // strip): the R tiles fill the end of every XCD's work
  const int64_t nC = coreg_tiles(Nap), nRT = next_r_row_tiles(Nep), nR = next_r_tiles(Nep, Nap);
  const int64_t n = nC + nR;
  int64_t ci = 0, ri = 0, pos = 0;
  for (int64_t x = 0; x < 8; ++x) {
    const int64_t size = n / 8 + (x < n % 8 ? 1 : 0);
    const int64_t nr = nR / 8 + (x < nR % 8 ? 1 : 0);
    for (int64_t k = 0; k < size - nr; ++k) out[pos++] = corder[ci++];
    for (int64_t k = 0; k < nr; ++k, ++ri)
      out[pos++] = kNextRTile | (uint32_t)(ri % nRT) | ((uint32_t)(ri / nRT) << 16);
  }
}

// FP32 form: X = P read k-major (P[k][i] = P[i][k]); the rows of the last
// row tile past N_e read past row N_e - 1 into the slack P is allocated with
// (next_r_p_slack floats), and their outputs are never stored.
static NextR<SymF32> next_r_args_f32(const float* P, int64_t ldp, const double* dP,
                                     const double* nP, const float* W, int64_t ldw, int64_t Ne,
                                     int64_t Na, const double* nWc, float* R) {
  NextR<SymF32> nr;
  nr.ops = OpsF32{P, ldp, W, ldw};
  nr.epi = EpiStoreT{R, ldw, Ne, Na, nP, nWc, dP, W, ldw};
  return nr;
}
int64_t next_r_p_slack(int64_t Nep) { return next_r_row_tiles(Nep) * kCB - Nep; }

hipError_t launch_resp_tiles(const float* P, int64_t ldp, const double* dP, int64_t Nap,
                             int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                             const double* nP, const double* nWc, float* R, const int32_t* gate,
                             hipStream_t s) {
  if (ldp % SymF32::BK || Nap % kCB) return hipErrorInvalidValue;
  k_resp_tiles<SymF32><<<dim3((unsigned)next_r_tiles(ldp, Nap)), dim3(kThreads), 0, s>>>(
      next_r_args_f32(P, ldp, dP, nP, W, ldw, Ne, Na, nWc, R), ldp, next_r_row_tiles(ldp), gate);
  return hipGetLastError();
}

hipError_t launch_coreg_update_next_r(const float* W, int64_t ldw, int64_t Nep, float* C,
                                      int64_t ldc, int64_t Nap, int64_t Na, const double* nWcol,
                                      Rule rule, double2* cstat, double* csq,
                                      const uint32_t* order_r, const int32_t* gate, hipStream_t s,
                                      bool packed, const float* P, const double* dP,
                                      const double* nP, int64_t Ne, float* R) {
  if (Nep % SymF32::BK || Nap % kCB) return hipErrorInvalidValue;
  return coreg_launch<SymF32, true>(
      OpsF32{W, ldw, W, ldw}, Nep, C, ldc, Nap, Na, nWcol, rule, cstat, csq, order_r, gate, s,
      packed, next_r_args_f32(P, Nep, dP, nP, W, ldw, Ne, Na, nWcol, R), next_r_tiles(Nep, Nap));
}

static NextR<SymB3> next_r_args(const bf16_t* Ph, const bf16_t* Pl, int64_t ldp, const double* dP,
                                const double* nP, const bf16_t* Wth, const bf16_t* Wtl,
                                int64_t ldwt, const float* W, int64_t ldw, int64_t Ne, int64_t Na,
                                const double* nWc, float* R) {
  NextR<SymB3> nr;
  nr.ops = OpsB3{Ph, Pl, ldp, Wth, Wtl, ldwt, ldp};  // P has ldp (= N_e padded) rows
  nr.epi = EpiStoreT{R, ldw, Ne, Na, nP, nWc, dP, W, ldw};
  return nr;
}

hipError_t launch_resp_tiles_b3(const bf16_t* Ph, const bf16_t* Pl, int64_t ldp, const double* dP,
                                const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nap,
                                int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                                const double* nP, const double* nWc, float* R,
                                const int32_t* gate, hipStream_t s) {
  if (ldp % SymB3::BK || Nap % kCB) return hipErrorInvalidValue;
  const int64_t nRT = next_r_row_tiles(ldp);
  k_resp_tiles<SymB3><<<dim3((unsigned)next_r_tiles(ldp, Nap)), dim3(kThreads), 0, s>>>(
      next_r_args(Ph, Pl, ldp, dP, nP, Wth, Wtl, ldwt, W, ldw, Ne, Na, nWc, R), ldp, nRT, gate);
  return hipGetLastError();
}

hipError_t launch_coreg_update_next_r_b3(const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt,
                                         int64_t Nep, float* C, int64_t ldc, int64_t Nap,
                                         int64_t Na, const double* nWcol, Rule rule,
                                         double2* cstat, double* csq, const uint32_t* order_r,
                                         const int32_t* gate, hipStream_t s, bool packed,
                                         const bf16_t* Ph, const bf16_t* Pl, const double* dP,
                                         const double* nP, const float* W, int64_t ldw,
                                         int64_t Ne, float* R) {
  if (Nep % SymB3::BK || Nap % kCB) return hipErrorInvalidValue;
  return coreg_launch<SymB3, true>(
      OpsB3{Wth, Wtl, ldwt, Wth, Wtl, ldwt}, Nep, C, ldc, Nap, Na, nWcol, rule, cstat, csq,
      order_r, gate, s, packed,
      next_r_args(Ph, Pl, Nep, dP, nP, Wth, Wtl, ldwt, W, ldw, Ne, Na, nWcol, R),
      next_r_tiles(Nep, Nap));
}

int coop_splits(int64_t Nep, int64_t Nap, int64_t blocks) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  int64_t s = (blocks + nU - 1) / nU;
  const int64_t maxs = Nap / (4 * CoopF32::BK);  // at least 4 K-steps per block
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return (int)s;
}

static int64_t coop_chunk(int64_t Nap, int splits) {
  return round_up((Nap + splits - 1) / splits, CoopF32::BK);
}

hipError_t launch_coop_partial(const float* W, int64_t ldw, int64_t Nep, int64_t Nap, int splits,
                               float* part, const int32_t* gate, hipStream_t s) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  k_coop_partial<CoopF32><<<dim3((unsigned)(nU * splits)), dim3(kThreads), 0, s>>>(
      OpsF32{W, ldw, W, ldw}, Nep, nU, coop_chunk(Nap, splits), Nap, part, gate);
  return hipGetLastError();
}

hipError_t launch_coop_partial_b3(const bf16_t* Wh, const bf16_t* Wl, int64_t ldw, int64_t Nep,
                                  int64_t Nap, int splits, float* part, const int32_t* gate,
                                  hipStream_t s) {
  const int64_t nT = Nep / kPB, nU = nT * (nT + 1) / 2;
  k_coop_partial<CoopB3P><<<dim3((unsigned)(nU * splits)), dim3(kThreads), 0, s>>>(
      OpsB3{Wh, Wl, ldw, Wh, Wl, ldw}, Nep, nU, coop_chunk(Nap, splits), Nap, part, gate);
  return hipGetLastError();
}

}  // namespace panda
