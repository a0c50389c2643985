// Internal declarations shared by the HIP sources of libpanda.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace panda {

// Device-resident iteration state.  Kernels read the gates and skip their
// work once the run has converged, so the host can enqueue iterations ahead
// of reading h back.
struct DevState {
  double h;        // h of the last completed iteration (Eq. 7)
  int32_t t;       // number of completed iterations (t of Eq. 6 during the P/C phase)
  int32_t active;  // 1 while h >= tol: gates R, A, W and h
  int32_t run_pc;  // 1 when the current iteration updates P and C: gates Eq. 5-6
  int32_t conv;    // 1 once h < tol
  int32_t wsel;    // index (0/1) of the buffer holding the current W; flipped with t
  int32_t pad;
};

// Scalars of the update rules.
struct Rule {
  double alpha;
  double tol;
  int32_t diag_alpha;
  int32_t sigma_from_T;
  int32_t n_own;
  int32_t h_undamped;
  int32_t update_last;
  int32_t sigma_ddof;
};

typedef unsigned short bf16_t;           // raw bits of a bfloat16

constexpr int kThreads = 256;            // threads per block (4 waves of 64)
constexpr int64_t kMaxStreamKBlocks = 1024;
constexpr int kColChunks = 64;           // row chunks of the column-norm kernel

// Padding of the internal state: TF dimension to 64, gene dimension to 128.
constexpr int64_t kPadE = 64;
constexpr int64_t kPadA = 128;
constexpr int64_t kPadK = 32;            // K of a stand-alone similarity product
constexpr int64_t kCoopTile = 64;        // tile side of the W W^T partial products
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Packed-symmetric storage of C (an option of the single-network context):
// only the upper kPT x kPT tiles (a <= b) of the padded N_a x N_a matrix,
// tile (a, b) at index b (b + 1) / 2 + a, each tile row-major with its own
// row length kPT.  An upper tile serves both triangles: C[i][j] for i in
// block a, j in block b is tile (a, b) entry (i mod kPT, j mod kPT), and
// C[j][i] is the same entry.  Diagonal tiles hold both of their triangles
// (they are symmetric), so any row of them can be read directly.
constexpr int64_t kPT = 128;
__host__ __device__ inline int64_t packed_tile(int64_t a, int64_t b) { return b * (b + 1) / 2 + a; }
inline int64_t packed_floats(int64_t Nap) {
  const int64_t nT = Nap / kPT;
  return nT * (nT + 1) / 2 * kPT * kPT;
}

// ------------------------------------------------------------ launchers --
// Rectangular similarity products (stream-K).  X is Mp x Kp (k contiguous),
// Y is Kp x Np (n contiguous); Mp % 64 == 0, Np % 128 == 0, Kp % 32 == 0.
// nx / ny are the FP64 squared norms of the rows of X / columns of Y.
// part: rect_partial_floats() floats of split-tile scratch.
int64_t rect_tiles(int64_t Mp, int64_t Np);
int64_t rect_tiles_b3(int64_t Mp, int64_t Np);  // tiles of the split-BF16 A + W product
// h partial slots of the split-BF16 A + W product: one per tile and fix-up
// block part (slots of tiles the fix-up never splits stay zero)
int64_t rect_hpart_slots_b3(int64_t Mp, int64_t Np);
size_t rect_partial_floats();

// Out[i][j] = T(X, Y)_ij for i < M, j < N.  yd (optional): Y is square with
// its diagonal held apart in this FP64 vector (and zero in Y).
hipError_t launch_tanimoto_store(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                 int64_t Mp, int64_t Np, int64_t Kp, int64_t M, int64_t N,
                                 const double* nx, const double* ny, float* Out, int64_t ldo,
                                 float* part, const int32_t* gate, hipStream_t s,
                                 const double* yd = nullptr);

// The diagonals of P and C are held apart in FP64 vectors dP, dC (the
// matrices hold zero there); the products add their terms in the epilogues.
// R = T(P, W) of the iteration (Eq. 3).
hipError_t launch_resp(const float* P, int64_t ldp, const double* dP, const float* W, int64_t ldw,
                       int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na, const double* nP,
                       const double* nWc, float* R, float* part, const int32_t* gate,
                       hipStream_t s);

// A = T(W, C) fused with the W update of Eq. 2 and per-tile h partials (Eq. 7).
hipError_t launch_avail_wupdate(const float* Wold, const float* C, const double* dC,
                                const float* R, float* Wnew, int64_t ld, int64_t Nep, int64_t Nap,
                                int64_t Ne, int64_t Na, const double* nWrow, const double* nC,
                                Rule rule, double* hpart, float* part, const int32_t* gate,
                                hipStream_t s, bool packed = false);

// C update (Eq. 5) on the upper tiles of T(W^T, W) with mirror writes and
// per-row partial sums for the sigma of Eq. 6 (and |C_.j|^2).  order holds
// the upper tiles (I | J << 16) in launch order, see coreg_order_fill.
hipError_t launch_coreg_update(const float* W, int64_t ldw, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, const double* nWcol, Rule rule,
                               double2* cstat, double* csq, const uint32_t* order,
                               const int32_t* gate, hipStream_t s, bool packed = false);
int64_t coreg_slots(int64_t Nap);
// Upper tiles of the C product (Nap / 128 per side) and their launch order:
// group x group super-tiles, so the tiles running together on one XCD share
// 2 * group operand strips in its L2.
int64_t coreg_tiles(int64_t Nap);
void coreg_order_fill(int64_t Nap, int group, uint32_t* out);
#ifndef PANDA_COREG_GROUP
#define PANDA_COREG_GROUP 6
#endif
constexpr int kCoregGroup = PANDA_COREG_GROUP;

// P update, split over K: partial products of W W^T on upper tiles.
hipError_t launch_coop_partial(const float* W, int64_t ldw, int64_t Nep, int64_t Nap, int splits,
                               float* part, const int32_t* gate, hipStream_t s);
// K chunks of the partial products, for about `blocks` blocks in all (at
// T=700, G=18000 the FP32 products run best at 1024, the split-BF16 ones at
// 512: their partial sums then cost the finalise more than they save).
int coop_splits(int64_t Nep, int64_t Nap, int64_t blocks);

// Split-BF16 forms of the same products.  Operands are K-contiguous hi/lo
// planes: P (diagonal zero), W row-major, W^T (gene-major); C stays FP32.
hipError_t launch_resp_b3(const bf16_t* Ph, const bf16_t* Pl, int64_t ldp, const double* dP,
                          const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nep,
                          int64_t Nap, int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                          const double* nP, const double* nWc, float* R, float* part,
                          const int32_t* gate, hipStream_t s);
// A = T(W, C) + W update with X = the W planes and Y = the FP32 C itself
// (symmetric; split into hi/lo while staged).
hipError_t launch_avail_wupdate_b3(const bf16_t* Wh, const bf16_t* Wl, const float* Wold,
                                   const float* C, const double* dC, const float* R, float* Wnew,
                                   int64_t ld, int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na,
                                   const double* nWrow, const double* nC, Rule rule,
                                   double* hpart, float* part, const int32_t* gate,
                                   hipStream_t s, bool packed = false);
hipError_t launch_coreg_update_b3(const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nep,
                                  float* C, int64_t ldc, int64_t Nap, int64_t Na,
                                  const double* nWcol, Rule rule, double2* cstat, double* csq,
                                  const uint32_t* order, const int32_t* gate, hipStream_t s,
                                  bool packed = false);
// R = T(P, W) (Eq. 3) on 128 x 128 tiles (next_r_tiles of them), alone or
// inside the C update's launch: that launch runs the C tiles and the R tiles
// of the order coreg_next_r_order_fill builds, so the next iteration's R is
// ready when the C update ends (P, its diagonal dP and norms nP, and W's
// planes and column norms must be the new ones).  Both compute R the same
// way, bit for bit.  W, R: leading dimension ldw; P's planes Nep x Nep.
int64_t next_r_row_tiles(int64_t Nep);
int64_t next_r_tiles(int64_t Nep, int64_t Nap);
void coreg_next_r_order_fill(int64_t Nep, int64_t Nap, const uint32_t* corder, uint32_t* out);
// FP32 form: P is read k-major and needs next_r_p_slack(Nep) floats of
// readable memory after its Nep x Nep entries.
int64_t next_r_p_slack(int64_t Nep);
hipError_t launch_resp_tiles(const float* P, int64_t ldp, const double* dP, int64_t Nap,
                             int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                             const double* nP, const double* nWc, float* R, const int32_t* gate,
                             hipStream_t s);
hipError_t launch_coreg_update_next_r(const float* W, int64_t ldw, int64_t Nep, float* C,
                                      int64_t ldc, int64_t Nap, int64_t Na, const double* nWcol,
                                      Rule rule, double2* cstat, double* csq,
                                      const uint32_t* order_r, const int32_t* gate, hipStream_t s,
                                      bool packed, const float* P, const double* dP,
                                      const double* nP, int64_t Ne, float* R);
hipError_t launch_resp_tiles_b3(const bf16_t* Ph, const bf16_t* Pl, int64_t ldp, const double* dP,
                                const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt, int64_t Nap,
                                int64_t Ne, int64_t Na, const float* W, int64_t ldw,
                                const double* nP, const double* nWc, float* R,
                                const int32_t* gate, hipStream_t s);
hipError_t launch_coreg_update_next_r_b3(const bf16_t* Wth, const bf16_t* Wtl, int64_t ldwt,
                                         int64_t Nep, float* C, int64_t ldc, int64_t Nap,
                                         int64_t Na, const double* nWcol, Rule rule,
                                         double2* cstat, double* csq, const uint32_t* order_r,
                                         const int32_t* gate, hipStream_t s, bool packed,
                                         const bf16_t* Ph, const bf16_t* Pl, const double* dP,
                                         const double* nP, const float* W, int64_t ldw,
                                         int64_t Ne, float* R);
hipError_t launch_coop_partial_b3(const bf16_t* Wh, const bf16_t* Wl, int64_t ldw, int64_t Nep,
                                  int64_t Nap, int splits, float* part, const int32_t* gate,
                                  hipStream_t s);
// hi/lo planes of W (Ne x Na, leading dimension ldw) row-major (ld ldw) and
// hi/lo planes of an n x n matrix with its diagonal left zero.
hipError_t launch_split_offdiag(const float* M, int64_t n, int64_t ld, bf16_t* Mh, bf16_t* Ml,
                                hipStream_t s);

// Packed C (see packed_tile).  pack: the upper tiles of the n x n symmetric
// matrix src (leading dimension lds; the upper triangle is read, and
// mirrored inside diagonal tiles), zero past n.  unpack: the full n x n
// matrix into dst (leading dimension ldd).  identity: dval on the diagonal,
// oval off it (within n), zero past n.  take_diag: the diagonal moves to d
// and reads zero.  col_sqnorms: out[j] = sum_i C[i][j]^2 (j < Nap, FP64),
// through slots (nT x Nap doubles, nT = Nap / kPT).
hipError_t launch_pack_sym(const float* src, int64_t n, int64_t lds, float* dst, int64_t Nap,
                           hipStream_t s);
hipError_t launch_unpack_sym(const float* src, int64_t n, int64_t Nap, float* dst, int64_t ldd,
                             hipStream_t s);
hipError_t launch_identity_packed(float* dst, int64_t n, int64_t Nap, double dval, double oval,
                                  hipStream_t s);
hipError_t launch_take_diag_packed(float* C, int64_t n, double* d, hipStream_t s);
hipError_t launch_col_sqnorms_packed(const float* C, int64_t Nap, double* slots, double* out,
                                     hipStream_t s);

// Rest of the iteration: h, P finalisation, both diagonals, norm vectors.
hipError_t launch_finish_h(const double* hpart, int64_t n, int64_t count, DevState* st,
                           Rule rule, hipStream_t s);
hipError_t launch_coop_finalize(const float* part, int splits, int64_t Nep, const double* nWrow,
                                float* P, int64_t ldp, int64_t Ne, Rule rule, float* Tside,
                                bf16_t* Ph, bf16_t* Pl, const int32_t* gate, hipStream_t s);
// part: kDiagBoth, or kDiagP / kDiagC for P's rows (dP, nP: they need only
// the new P) or C's rows (dC, nC: they need the C update's row sums) alone.
constexpr int kDiagBoth = 0, kDiagP = 1, kDiagC = 2;
hipError_t launch_diagonals(const float* P, int64_t ldp, double* dP, int64_t Ne,
                            const float* Tside, double* nP, double* dC, int64_t ldc, int64_t Na,
                            const double2* cstat, const double* csq, int64_t nslots, double* nC,
                            Rule rule, const DevState* st, hipStream_t s, int part = kDiagBoth);
// The same with the diagonal rule new = keep * old + f * N * sigma * g given
// (closed form of several steps of Eq. 6).
hipError_t launch_diagonals_schedule(const float* P, int64_t ldp, double* dP, int64_t Ne,
                                     const float* Tside, double* nP, double* dC, int64_t ldc,
                                     int64_t Na, const double2* cstat, const double* csq,
                                     int64_t nslots, double* nC, Rule rule, double keep, double g,
                                     const DevState* st, hipStream_t s);
// The diagonal of an n x n matrix into / out of its FP64 vector (take also
// sets the matrix diagonal to zero).
hipError_t launch_take_diag(float* M, int64_t n, int64_t ld, double* d, hipStream_t s);
hipError_t launch_put_diag(float* M, int64_t n, int64_t ld, const double* d, hipStream_t s);
// t, the gates, and the current-W selector back to buffer 0.
hipError_t launch_state_set(DevState* st, int32_t t, int32_t active, int32_t run_pc,
                            hipStream_t s);
// Squared norms of the rows / columns of a rows x cols matrix with leading
// Row and column squared norms of W (padded Nep x ldw, real Ne x Na) in one
// pass over it, plus its bf16 planes (row-major and gene-major, leading
// dimension ldt) when Wh is given.  scr holds w_norm_scratch_doubles().
size_t w_norm_scratch_doubles(int64_t Nep, int64_t Nap);
hipError_t launch_w_norms(const float* W, int64_t Ne, int64_t Na, int64_t ldw, int64_t Nep,
                          double* nr, double* nc, double* scr, bf16_t* Wh, bf16_t* Wl, bf16_t* Wth,
                          bf16_t* Wtl, int64_t ldt, const int32_t* gate, hipStream_t s);
// dimension ld.  The column version needs kColChunks * cols doubles of scratch.
hipError_t launch_row_sqnorms(const float* M, int64_t rows, int64_t cols, int64_t ld, double* out,
                              const int32_t* gate, hipStream_t s);
hipError_t launch_col_sqnorms(const float* M, int64_t rows, int64_t cols, int64_t ld, double* out,
                              double* scratch, const int32_t* gate, hipStream_t s);

// Z-score (Sec. II-A) on a strided matrix; scratch holds kZsBlocks + 8 doubles.
constexpr int kZsBlocks = 1024;
hipError_t launch_zscore_stats(const float* M, int64_t rows, int64_t cols, int64_t ld,
                               double* scratch, hipStream_t s, int ddof = 0);
// Per-row moments (rs, one per row) and, when cs is given, per-column
// moments (cs, one per column) as (mean, std); flags[0] / flags[1] are set
// for a NaN/Inf entry / a row or column of zero spread.  apply: per-row
// z-score, or (row z + column z) / sqrt 2 when cs is given.
hipError_t launch_zscore_rc_stats(const float* M, int64_t rows, int64_t cols, int64_t ld, int ddof,
                                  double* flags, double2* rs, double2* cs, hipStream_t s);
hipError_t launch_zscore_rc_apply(float* M, int64_t rows, int64_t cols, int64_t ld,
                                  const double2* rs, const double2* cs, hipStream_t s);
hipError_t launch_zscore_apply(float* M, int64_t rows, int64_t cols, int64_t ld,
                               const double* scratch, hipStream_t s);
hipError_t launch_fill_identity(float* M, int64_t n, int64_t ld, hipStream_t s);
// Pearson correlation of the G rows of E (G x S, leading dimension lde):
// row statistics, then the centred rows scaled to unit norm, stored
// sample-major as Zt (Sp x Gp, zero-padded; Gp a multiple of 128, Sp of 16);
// then C = Z Z^T on the upper 128 x 128 tiles, mirrored, 1 on the diagonal.
hipError_t launch_pearson_z(const float* E, int64_t G, int64_t S, int64_t lde, double2* stat,
                            float* Zt, int64_t Gp, int64_t Sp, hipStream_t s);
hipError_t launch_corr(const float* Zt, int64_t Gp, int64_t Sp, int64_t G, float* C, int64_t ldc,
                       hipStream_t s);

hipError_t launch_state_init(DevState* st, int32_t t0, hipStream_t s);

}  // namespace panda
