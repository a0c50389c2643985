/*
 * panda.h -- C ABI of libpanda.so, the MI355X (gfx950) implementation of the
 * PANDA message-passing iteration in matrix form (Glass, Quackenbush & Kepner,
 * arXiv 1507.07039).
 *
 * Problem (Sec. II-A, II-B).  Three networks: the regulatory network W
 * (N_e x N_a, transcription factors x genes), the cooperativity network P
 * (N_e x N_e, symmetric) and the co-regulatory network C (N_a x N_a,
 * symmetric).  Each iteration t = 1, 2, ... computes
 *     R = T(P, W), A = T(W, C)                              (Eq. 3, Eq. 4)
 *     W <- (1 - alpha) W + alpha/2 (A + R)                  (Eq. 2)
 *     h = mean |W(t) - W(t-1)|, stop when h < tol           (Eq. 7)
 *     P_im <- (1 - alpha) P_im + alpha T(W_i., W_m.), i != m (Eq. 5)
 *     C_kj <- (1 - alpha) C_kj + alpha T(W_.k, W_.j), k != j (Eq. 5)
 *     P_ii, C_jj from the off-diagonal spread of their row   (Eq. 6)
 * where T(X, Y)_ij = X_i.Y_.j / sqrt(|X_i.|^2 + |Y_.j|^2 - |X_i.Y_.j|)
 * is the similarity of Eq. 1 in the matrix form of Sec. II-C (Eq. 9).
 *
 * Conventions for every entry point:
 *   - Matrix pointers are DEVICE pointers to row-major, contiguous FP32
 *     arrays, owned by the caller.  The library never frees them.
 *   - Work is enqueued on the given HIP stream (NULL = the default stream).
 *     Calls that return a value computed on the device (h, t, status of a
 *     normalisation) synchronise that stream before returning.
 *   - Arguments are validated on the host before any device work; a failed
 *     validation returns PANDA_ERR_ARG and enqueues nothing.
 *   - Network sizes: 1 <= N_e <= 65536 TFs and 1 <= N_a <= 262144 genes (so
 *     every grid and tile index stays in range); outside them the calls
 *     return PANDA_ERR_ARG and the *_workspace_bytes() calls return 0.
 *   - Errors are returned as panda_status; no exception or abort crosses the
 *     ABI.  panda_last_error() gives a thread-local message for the last
 *     failure on the calling thread.
 *   - The workspace is caller-owned device memory of at least the size the
 *     matching *_workspace_bytes() call returns, aligned to 256 bytes.  The
 *     library allocates no device memory of its own; a context allocates one
 *     small pinned host buffer for reading the convergence state.
 */
#ifndef PANDA_H
#define PANDA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PANDA_OK = 0,              /* converged (h < tol) or call succeeded         */
  PANDA_NOT_CONVERGED = 1,   /* max_iter reached; outputs hold the last state */
  PANDA_ERR_ARG = -1,        /* invalid argument; nothing was enqueued         */
  PANDA_ERR_DEGENERATE = -2, /* z-score of a constant network (std = 0)        */
  PANDA_ERR_NONFINITE = -3,  /* NaN or Inf in an input network                 */
  PANDA_ERR_HIP = -4,        /* a HIP runtime call failed                      */
  PANDA_ERR_WORKSPACE = -5,  /* workspace missing, too small or misaligned     */
  PANDA_STATUS_MAX_ENUM = 0x7fffffff /* not a status: makes every 32-bit value a
                                        valid panda_status (so an unknown code can
                                        be passed to panda_status_string)      */
} panda_status;

/* Arithmetic of the similarity products (norms, denominators, h and the
 * diagonal rule are FP64 in both forms; the state W, P, C is FP32):
 *   PANDA_PREC_FP32    FP32 matrix-core products, FP32 accumulation.
 *   PANDA_PREC_BF16X3  every operand split as x = hi + lo (bf16, round to
 *                      nearest even) and each product formed as
 *                      hi*hi + hi*lo + lo*hi on bf16 matrix cores with FP32
 *                      accumulation; the diagonals of P and C are kept out
 *                      of the split operands and their terms added in FP64.
 *                      C stays FP32 (split while it is staged for the
 *                      products); the extra workspace is the hi/lo planes of
 *                      W (two layouts) and P, about 4 * Ne * Na * 2 bytes. */
enum { PANDA_PREC_FP32 = 0, PANDA_PREC_BF16X3 = 1 };

/* Scope of the z-score of Sec. II-A (the paper says only that each network
 * is z-score normalised):
 *   PANDA_ZSCORE_GLOBAL  one mean and standard deviation over all entries
 *   PANDA_ZSCORE_ROW     each row by its own mean and standard deviation
 *                        (for W: per transcription factor; it does not keep
 *                        a symmetric network symmetric, so it is not meant
 *                        for P and C, which the iteration takes symmetric)
 *   PANDA_ZSCORE_ROWCOL  (Zr + Zc) / sqrt(2), Zr the per-row and Zc the
 *                        per-column z-score of the same input (symmetric in,
 *                        symmetric out) */
enum { PANDA_ZSCORE_GLOBAL = 0, PANDA_ZSCORE_ROW = 1, PANDA_ZSCORE_ROWCOL = 2 };

/* Run parameters and the readings of the paper where it is ambiguous.
 * panda_default_options() fills the defaults given in brackets. */
typedef struct {
  double alpha;         /* [0.1]  update rate of Eq. 2, 5 and 6, 0 < alpha <= 1   */
  double tol;           /* [1e-3] stop when h < tol (Sec. II-B)                   */
  int32_t max_iter;     /* [200]  iteration cap                                   */
  int32_t diag_alpha;   /* [1]    Eq. 6 increment multiplied by alpha; 0: literal */
  int32_t sigma_from_T; /* [0]    sigma of Eq. 6 from the damped off-diagonal row;
                                  1: from the fresh similarity row               */
  int32_t n_own;        /* [0]    Eq. 6 multiplier N_a for P, N_e for C as printed;
                                  1: the network's own dimension                 */
  int32_t h_undamped;   /* [0]    h of Eq. 7 from W(t) - W(t-1); 1: mean |(A+R)/2 - W| */
  int32_t update_last;  /* [0]    skip the P/C update on the converging iteration */
  int32_t poll_every;   /* [1]    panda_run reads h back every poll_every iterations */
  int32_t precision;    /* [PANDA_PREC_FP32]                                      */
  int32_t sigma_ddof;   /* [0]    standard deviations (sigma of Eq. 6, and the
                                  z-score of an identity default) divide by n;
                                  1: by n - 1 (sample)                           */
  int32_t zscore_mode;  /* [PANDA_ZSCORE_GLOBAL] scope of the z-score that the
                                  library applies itself (identity defaults)     */
  int32_t packed_c;     /* [0]    1: a context stores C as its upper 128 x 128 tiles
                                  only (C is symmetric, and Eq. 5 keeps it so):
                                  about half the workspace of C, no mirror writes
                                  in the C update; the A product reads each
                                  stored tile for both triangles.  Results are the
                                  same as with 0.  Contexts and panda_run only (a
                                  batch stores C whole); panda_ws_features needs 0 */
} panda_options;

typedef struct panda_ctx panda_ctx;

/* Fill *opt with the defaults listed above. */
void panda_default_options(panda_options* opt);

/* Z-score normalisation of one network in place (Sec. II-A; NormalizeNetwork
 * in Sec. II-C): mean and population standard deviation over all rows*cols
 * entries, then M <- (M - mean) / std.  Reductions in FP64, two passes.
 * Needs panda_normalize_workspace_bytes() bytes of workspace (a few KB).
 * Synchronises the stream.  Returns PANDA_ERR_NONFINITE (M untouched) if an
 * entry is NaN/Inf, PANDA_ERR_DEGENERATE (M untouched) if the standard
 * deviation is 0. */
size_t panda_normalize_workspace_bytes(void);
panda_status panda_normalize(float* M, int64_t rows, int64_t cols, void* workspace,
                             size_t ws_bytes, hipStream_t stream);

/* The same z-score with a choice of scope (PANDA_ZSCORE_*) and normaliser
 * (ddof 0: divide the sum of squared deviations by the count n; ddof 1: by
 * n - 1).  M is rows x cols, row-major, contiguous, device memory, changed in
 * place.  Moments in FP64, two passes.  Returns PANDA_ERR_NONFINITE (M
 * untouched) for a NaN/Inf entry; PANDA_ERR_DEGENERATE (M untouched) if the
 * network, or under the row / row + column scopes any row / column, has zero
 * spread (or fewer than ddof + 1 entries).  Needs
 * panda_normalize_ex_workspace_bytes(rows, cols, zscore_mode) bytes of
 * workspace (0 for invalid arguments; about 16 (rows + cols) bytes).
 * Synchronises the stream.  panda_normalize is zscore_mode GLOBAL, ddof 0. */
size_t panda_normalize_ex_workspace_bytes(int64_t rows, int64_t cols, int32_t zscore_mode);
panda_status panda_normalize_ex(float* M, int64_t rows, int64_t cols, int32_t zscore_mode,
                                int32_t ddof, void* workspace, size_t ws_bytes,
                                hipStream_t stream);

/* Similarity matrix of Eq. 1 in the matrix form of Sec. II-C (the paper's
 * Tfunction): Out[i][j] = T(row i of X, column j of Y) for X (M x K) and
 * Y (K x N); Out is M x N.  FP32 MFMA products, FP64 norms and denominator,
 * T := 0 where the denominator is 0 (both vectors zero).  M, K, N >= 1.
 * Needs panda_tanimoto_workspace_bytes(M, K, N) bytes of workspace. */
size_t panda_tanimoto_workspace_bytes(int64_t M, int64_t K, int64_t N);
panda_status panda_tanimoto(const float* X, const float* Y, int64_t M, int64_t K, int64_t N,
                            float* Out, void* workspace, size_t ws_bytes, hipStream_t stream);

/* Co-expression prior of Sec. II-A: C[i][j] = Pearson correlation between
 * rows i and j of the expression matrix E (G genes x S samples, row-major,
 * leading dimension lde >= S, device memory); C is G x G with leading
 * dimension ldc >= G (device memory, written; E is not modified; columns past
 * G of each row are left alone).  Row means and centred sums of squares in
 * FP64; the correlations as one FP32 MFMA product of the centred rows scaled
 * to unit norm, computed on the upper triangle of 128 x 128 tiles and
 * mirrored, so C is exactly symmetric.  C[i][i] = 1, and a constant row gets
 * correlation 0 with every other row.  G >= 1, S >= 2.  Needs
 * panda_pearson_workspace_bytes(G, S) bytes of workspace (256-byte aligned;
 * 4 S G bytes plus padding).  The result is not z-scored: call
 * panda_normalize on it, as on any prior.  Enqueued on the stream; returns
 * without synchronising. */
size_t panda_pearson_workspace_bytes(int64_t G, int64_t S);
panda_status panda_pearson(const float* E, int64_t G, int64_t S, int64_t lde, float* C,
                           int64_t ldc, void* workspace, size_t ws_bytes, hipStream_t stream);

/* The same prior without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
 * panda_pearson; its scratch is an array of PANDA_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that the library holds in the memory of every GPU it runs on
 * until the process ends, found once per device on the first call there.
 * The call itself allocates nothing and does not synchronise.  Sizes whose
 * panda_pearson_workspace_bytes(G, S) exceeds PANDA_NOALLOC_SCRATCH_BYTES
 * (for example G = 30000 genes with S up to about 550 samples fit) return
 * PANDA_ERR_ARG with the sizes in panda_last_error() and enqueue nothing.
 * The stream must belong to the current device.  All calls on one GPU share
 * its array: calls that overlap in time on one GPU (different streams, or
 * threads without ordering) race and must not be made; calls ordered on one
 * stream are safe, since every byte of scratch a call reads it writes first. */
#define PANDA_NOALLOC_SCRATCH_BYTES (64u << 20)
panda_status panda_pearson_noalloc(const float* E, int64_t G, int64_t S, int64_t lde, float* C,
                                   int64_t ldc, hipStream_t stream);

/* Workspace for a context or panda_run on an N_e x N_a problem. */
size_t panda_workspace_bytes(int64_t Ne, int64_t Na, const panda_options* opt);

/* Create a context holding the message-passing state (W, P, C, t) inside the
 * workspace (Sec. II-B, PANDA()).  opt NULL = defaults.  Ne, Na >= 1. */
panda_status panda_ctx_create(int64_t Ne, int64_t Na, const panda_options* opt, void* workspace,
                              size_t ws_bytes, hipStream_t stream, panda_ctx** out);

/* Load the state: W (Ne x Na), P (Ne x Ne), C (Na x Na), already normalised,
 * and the number t of iterations already done (0 for a fresh start; the
 * diagonal rule of Eq. 6 depends on t).  P or C NULL means the identity
 * network, z-scored like any other (Sec. II-A; fails with
 * PANDA_ERR_DEGENERATE for a 1 x 1 identity). */
panda_status panda_ctx_load(panda_ctx* ctx, const float* W, const float* P, const float* C,
                            int32_t t);

/* One message-passing iteration (Eq. 2-7).  Synchronises the stream and
 * returns h and the iteration number t.  Once h < tol the state is frozen:
 * further calls change nothing and return PANDA_OK with the same h and t. */
panda_status panda_iterate(panda_ctx* ctx, double* h, int32_t* t);

/* Copy the current state out (any pointer may be NULL to skip it).  The
 * diagonals of P and C (Eq. 6) grow like exp(2 alpha t); the library keeps
 * them in FP64, rounded to FP32 after each step while they fit in FP32 (so a
 * stored state loads and resumes exactly), unrounded beyond.  A diagonal
 * past the FP32 range (about alpha t > 40) is stored as +inf; W and the
 * off-diagonal entries are unaffected and the iteration itself goes on. */
panda_status panda_ctx_store(panda_ctx* ctx, float* W, float* P, float* C, double* h, int32_t* t);

void panda_ctx_destroy(panda_ctx* ctx);

/* The whole message-passing procedure (PANDA() of Sec. II-C): from the
 * normalised priors (W0, P0, C0; P0/C0 NULL = identity) iterate until h < tol
 * or max_iter iterations, then write the final networks to W, P, C (may alias
 * the inputs).  alpha, tol and max_iter override the same fields of opt.
 * Returns PANDA_OK (converged) or PANDA_NOT_CONVERGED; *iters = final t,
 * *h = final h.  Blocks only to read h back every poll_every iterations. */
panda_status panda_run(const float* W0, const float* P0, const float* C0, int64_t Ne, int64_t Na,
                       double alpha, double tol, int32_t max_iter, float* W, float* P, float* C,
                       void* workspace, size_t ws_bytes, const panda_options* opt,
                       int32_t* iters, double* h, hipStream_t stream);

/* ---- Permutation null ----------------------------------------------------
 * Node-label randomisation on input (an option of the paper's C
 * implementation, Sec. III) as a null model for the edges of W.
 *
 * panda_permute_sym: out[i][j] = M[perm[i]][perm[j]] for an n x n matrix M
 * (leading dimension ldm >= n; out ldo >= n; device memory, out must not
 * alias M).  perm: n int32 in device memory, a permutation of 0 .. n-1
 * (checked on the host: PANDA_ERR_ARG otherwise; the check synchronises the
 * stream).  A z-scored network stays z-scored (same entries).
 *
 * panda_null: K null instances.  Instance k relabels the genes of C0 by row k
 * of gene_perm (K x Na, device) and the TFs of P0 by row k of tf_perm (K x Ne,
 * device); either may be NULL (no relabelling of that prior; an identity prior,
 * P0 or C0 NULL, is unchanged by any relabelling), and W0 keeps its labels.  Each
 * instance runs PANDA() from its normalised priors to convergence with the
 * options opt (alpha, tol, max_iter, precision ...; NULL = defaults); the
 * converged W of all K are folded into mean[i][j] and sd[i][j] (population
 * standard deviation over the K instances; FP64 running sums, Welford's
 * update; outputs FP32, Ne x Na, device).  iters (host, K entries, may be NULL)
 * receives each instance's final t.  Returns PANDA_NOT_CONVERGED if any
 * instance stopped at max_iter (its W is still counted).  Needs
 * panda_null_workspace_bytes(Ne, Na, opt) bytes of workspace (256-byte
 * aligned): a context's workspace, the relabelled priors and the FP64 sums.
 * Blocks until the last instance has converged; mean and sd are enqueued on
 * the stream after it.
 *
 * panda_null_zscore: z[i][j] = (W[i][j] - mean[i][j]) / sd[i][j], 0 where
 * sd = 0 (all Ne x Na, device; z may alias W).  Enqueued on the stream. */
panda_status panda_permute_sym(const float* M, int64_t n, int64_t ldm, const int32_t* perm,
                               float* out, int64_t ldo, hipStream_t stream);
size_t panda_null_workspace_bytes(int64_t Ne, int64_t Na, const panda_options* opt);
panda_status panda_null(const float* W0, const float* P0, const float* C0, int64_t Ne,
                        int64_t Na, int32_t K, const int32_t* gene_perm, const int32_t* tf_perm,
                        const panda_options* opt, void* workspace, size_t ws_bytes, float* mean,
                        float* sd, int32_t* iters, hipStream_t stream);
panda_status panda_null_zscore(const float* W, const float* mean, const float* sd, int64_t Ne,
                               int64_t Na, float* z, hipStream_t stream);

/* Per-phase timing of a context (the paper times the message-passing
 * procedure alone, Sec. II-D; this splits that time by step).  When enabled,
 * each phase of each iteration is bracketed by HIP events on the context's
 * stream; elapsed times are summed whenever the state is read back.  Phases
 * are indexed by the enum below.  phase_times fills total_ms[PANDA_NPHASE]
 * and count[PANDA_NPHASE] (iterations timed); either may be NULL. */
enum {
  PANDA_PHASE_R = 0,      /* R = T(P, W)                          (Eq. 3)       */
  PANDA_PHASE_AW = 1,     /* A = T(W, C), W update, h partials    (Eq. 4, 2, 7) */
  PANDA_PHASE_H = 2,      /* h and the convergence test           (Eq. 7)       */
  PANDA_PHASE_PPART = 3,  /* W W^T split-K partial products       (Eq. 5, P)    */
  PANDA_PHASE_PFIN = 4,   /* P off-diagonal update                (Eq. 5, P)    */
  PANDA_PHASE_C = 5,      /* C off-diagonal update, row sums      (Eq. 5, C)    */
  PANDA_PHASE_DIAG = 6,   /* diagonals of P and C                 (Eq. 6)       */
  PANDA_NPHASE = 7
};
panda_status panda_ctx_set_timing(panda_ctx* ctx, int32_t enable);
panda_status panda_ctx_phase_times(panda_ctx* ctx, double* total_ms, int64_t* count);

/* ---- Batched form ---------------------------------------------------------
 * n independent networks of arbitrary sizes iterate together (the paper runs
 * PANDA on sets of networks, Sec. I; each network follows Eq. 2-7 exactly as
 * a context does).  Every phase of an iteration is one grouped launch over
 * all networks (persistent kernels over per-XCD work queues for the four
 * similarity products); a network stops being updated once its own h < tol
 * (its convergence mask), while the others go on.  One iteration can be
 * captured in a HIP graph and replayed.  precision PANDA_PREC_FP32 or
 * PANDA_PREC_BF16X3 (the split-BF16 products of a context with the same
 * option; such a batch has one tiling for R, A + W and the C update, tile
 * choice 0, and the autotuner varies only the W W^T K chunk).  All matrices
 * are device pointers, row-major FP32.
 *
 * Workspace: panda_batch_workspace_bytes(n, Ne, Na, opt) bytes, 256-byte
 * aligned, owned by the caller; it holds each network's state (about what a
 * context of the same size needs) plus the work lists.  n >= 1, every
 * Ne[i], Na[i] >= 1. */
typedef struct panda_batch panda_batch;

size_t panda_batch_workspace_bytes(int32_t n, const int64_t* Ne, const int64_t* Na,
                                   const panda_options* opt);
panda_status panda_batch_create(int32_t n, const int64_t* Ne, const int64_t* Na,
                                const panda_options* opt, void* workspace, size_t ws_bytes,
                                hipStream_t stream, panda_batch** out);
void panda_batch_destroy(panda_batch* b);

/* Tile choices of the grouped products, one per entry of the enum below;
 * panda_batch_tile_candidates(phase) gives how many exist for an FP32 batch
 * (choice in [0, count); a split-BF16 batch accepts only choice 0 for R, A + W
 * and the C update).  set_tiles validates every entry and rebuilds the work lists
 * (synchronises the stream).  autotune times every candidate of every phase
 * on the batch's own shapes (reps timed launches each, best time wins) and
 * keeps the fastest; it overwrites the whole state, so it must precede
 * panda_batch_load (loaded networks are marked unloaded).  Timing does not
 * depend on the values, so the state is zero while it runs. */
enum {
  PANDA_BATCH_TILE_R = 0,     /* R = T(P, W) tile                    */
  PANDA_BATCH_TILE_AW = 1,    /* A = T(W, C) + W update tile         */
  PANDA_BATCH_TILE_PPART = 2, /* K chunk of the W W^T partials       */
  PANDA_BATCH_TILE_C = 3,     /* C update tile shape                 */
  PANDA_BATCH_NTILE = 4
};
int32_t panda_batch_tile_candidates(int32_t phase);
panda_status panda_batch_get_tiles(const panda_batch* b, int32_t* choice);
panda_status panda_batch_set_tiles(panda_batch* b, const int32_t* choice);
panda_status panda_batch_autotune(panda_batch* b, int32_t reps, float* best_ms);

/* Load network i (0 <= i < n) as panda_ctx_load does, including the identity
 * default for a NULL P or C. */
panda_status panda_batch_load(panda_batch* b, int32_t i, const float* W, const float* P,
                              const float* C, int32_t t);

/* steps iterations of every network whose h is still >= tol (use_graph: by
 * replaying the captured iteration; the graph is captured on first use and
 * again after the tiles change).  Then reads the states back (synchronises
 * the stream) and returns in *active how many networks are still iterating.
 * Every network must be loaded. */
panda_status panda_batch_iterate(panda_batch* b, int32_t steps, int32_t use_graph,
                                 int32_t* active);
/* Iterate until every network has converged or opt.max_iter iterations have
 * run, reading the states back every opt.poll_every iterations.  Returns
 * PANDA_OK when all converged, else PANDA_NOT_CONVERGED; *steps = iterations
 * run by the batch. */
panda_status panda_batch_run(panda_batch* b, int32_t use_graph, int32_t* steps);
/* State of network i as of the last read-back: h, t and whether it is still
 * iterating (any pointer may be NULL). */
panda_status panda_batch_state(const panda_batch* b, int32_t i, double* h, int32_t* t,
                               int32_t* active);
/* Copy network i out, as panda_ctx_store does. */
panda_status panda_batch_store(panda_batch* b, int32_t i, float* W, float* P, float* C,
                               double* h, int32_t* t);

/* ---- Learned warm start ---------------------------------------------------
 * Not part of the paper's method: a small network predicts the converged W
 * of a run from features of the priors, and the message passing of Eq. 2-7
 * is then polished from a state rebuilt around that prediction.  The plain
 * run from the priors remains the reference and the fallback.
 *
 * Features (16 per edge (i, j), row i*Na + j of F, FP32, each column z-scored
 * over the Ne*Na edges with the population std; a constant column is 0):
 *   W0_ij; sum_j W0_ij; sum_i W0_ij; for k < 6: a_k[i] b_k[j] and c_k[i] d_k[j];
 *   (R0_ij + A0_ij) / 2.  a = orthonormal basis (Cholesky QR; a rank-deficient
 *   sketch ends the basis and zeroes the rest) of P0 (P0 omegaP), b = W0^T P0 a;
 *   d = basis of C0 (C0 omegaC), c = W0 C0 d; R0 = T(P0, W0), A0 = T(W0, C0)
 *   (Eq. 1, 3, 4).  omegaP (Ne x 6) and omegaC (Na x 6) are the caller's
 *   random sketch matrices (device, FP32, row-major).  The features are taken
 *   from a context just loaded with the normalised priors (a context of a
 *   batch is rejected); *tau = population std of (R0 + A0) / 2 - W0, the unit
 *   of the network's output.  Synchronises the context's stream. */
enum { PANDA_WS_FEATURES = 16, PANDA_WS_SKETCH = 6, PANDA_MLP_PARAMS = 5313 };
size_t panda_ws_features_workspace_bytes(int64_t Ne, int64_t Na);
panda_status panda_ws_features(panda_ctx* ctx, const float* omegaP, const float* omegaC, float* F,
                               double* tau, void* workspace, size_t ws_bytes);

/* The network: 16 -> 64 -> 64 -> 1, ReLU, parameters (FP32 master copy,
 * PANDA_MLP_PARAMS floats, device) packed as W1[64][16], b1[64], W2[64][64]
 * (out, in), b2[64], w3[64], b3.  Products take bf16-rounded weights and
 * activations on matrix cores with FP32 accumulation.  forward: y[e] for the
 * n rows of F (n x 16).  grad: gradient (PANDA_MLP_PARAMS floats, device) of
 * the mean squared error of y against target over a batch of n rows (rows
 * idx[e] of F / target when idx is given, indices outside [0, nrows) are
 * skipped; rows 0..n-1 otherwise) and the loss (device double, may be NULL);
 * in the backward pass dz2 and dz1 enter the products bf16-rounded.  adam: one
 * Adam update at step >= 1 (m, v: FP32 moments, zero before step 1).
 * train_step: grad then adam with beta1 0.9, beta2 0.999, eps 1e-8.  All
 * enqueue on `stream` without synchronising. */
panda_status panda_mlp_forward(const float* params, const float* F, int64_t n, float* y,
                               hipStream_t stream);
size_t panda_mlp_grad_workspace_bytes(int64_t n);
panda_status panda_mlp_grad(const float* params, const float* F, int64_t nrows,
                            const float* target, const int64_t* idx, int64_t n, float* grad,
                            double* loss, void* workspace, size_t ws_bytes, hipStream_t stream);
panda_status panda_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                            float lr, float beta1, float beta2, float eps, hipStream_t stream);
panda_status panda_mlp_train_step(float* params, float* m, float* v, int32_t step, float lr,
                                  const float* F, int64_t nrows, const float* target,
                                  const int64_t* idx, int64_t n, float* grad, double* loss,
                                  void* workspace, size_t ws_bytes, hipStream_t stream);

/* Target and prediction in the units above (rows x cols, row-major, device):
 * out = (Wstar - W0) / tau and Wpred = W0 + tau * y. */
panda_status panda_ws_target(const float* W0, const float* Wstar, int64_t rows, int64_t cols,
                             double tau, float* out, hipStream_t stream);
panda_status panda_ws_predict(const float* W0, const float* y, int64_t rows, int64_t cols,
                              double tau, float* Wpred, hipStream_t stream);

/* Warm state of a loaded context (its P and C diagonals are the priors'):
 * W = Wpred (Ne x Na, device); P and C off-diagonals = T of the rows /
 * columns of Wpred (the fixed point of Eq. 5 for this W); diagonals = t0
 * steps of Eq. 6 in closed form with sigma held at the std of the rebuilt
 * off-diagonal row, (1-a)^t0 d0 + f N sigma sum_{s<=t0} (1-a)^(t0-s) e^(2as);
 * t = t0.  panda_iterate then continues from iteration t0 + 1.  Synchronises
 * the stream. */
panda_status panda_ws_init(panda_ctx* ctx, const float* Wpred, int32_t t0);

const char* panda_status_string(panda_status s);
const char* panda_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PANDA_H */
