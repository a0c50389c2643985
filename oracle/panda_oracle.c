/*
 * panda_oracle.c -- plain FP64 CPU oracle for the PANDA message-passing
 * iteration (Glass, Quackenbush & Kepner, "High Performance Computing of Gene
 * Regulatory Networks using a Message-Passing Model", arXiv 1507.07039).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * Every similarity value is evaluated one entry at a time from its plain
 * element-wise definition (Eq. 1, as in the nested-loop form of Eq. 8): a dot
 * product and the two squared norms accumulated in one sequential pass over
 * the shared index, in FP64, IEEE round-to-nearest, no fast-math and no FMA
 * contraction (built with -ffp-contract=off).  Each output entry is owned by
 * one thread, so the results do not depend on the thread count.
 *
 * Readings of the paper that this file takes (each switchable by a flag):
 *   - R and A are both formed from the previous iterate (Eq. 3, Eq. 4).
 *   - the P update of Eq. 5 compares rows i and m of the new W; the C update
 *     compares columns k and j of the new W.
 *   - Eq. 6 diagonal: increment multiplied by alpha (D1) by default; the
 *     literal form without alpha (D0) behind diag_alpha = 0.
 *   - sigma: population standard deviation of the off-diagonal entries of the
 *     damped row (Sec. II-B text after Eq. 6); fresh T row behind sigma_from_T;
 *     the sample standard deviation (divisor n - 1) behind sigma_ddof = 1.
 *   - z-score (Sec. II-A): mean and standard deviation over all entries of a
 *     network; per row, or the sum of the row and the column z-scores over
 *     sqrt 2, behind the zscore mode of oracle_normalize_ex.
 *   - multiplier: N_a for P and N_e for C as printed in Eq. 6; own dimension
 *     behind n_own.
 *   - h: Eq. 7 literal (damped difference); undamped "predicted" form behind
 *     h_undamped.
 *   - once h < tol the P and C updates of that iteration are skipped;
 *     update_last = 1 performs them anyway.
 *   - t = 1 on the first iteration.
 *   - T(0,0) := 0 (zero denominator only when both vectors are zero).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_NOT_CONVERGED 1
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_DEGENERATE (-2)
#define ORACLE_ERR_NONFINITE (-3)
#define ORACLE_ERR_NOMEM (-5)

typedef struct {
  double alpha;
  double tol;
  int32_t max_iter;
  int32_t diag_alpha;
  int32_t sigma_from_T;
  int32_t n_own;
  int32_t h_undamped;
  int32_t update_last;
  int32_t sigma_ddof; /* 0: population std in Eq. 6; 1: sample std */
} oracle_opts;

/* Number of OpenMP threads for the calls that follow (n >= 1); returns the
 * previous maximum.  Results do not depend on it (each output entry is owned
 * by one thread); only timing does. */
int oracle_set_threads(int n) {
  int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
}

/* Eq. 1: T(x, y) = x.y / sqrt(|x|^2 + |y|^2 - |x.y|), x and y given with
 * element strides incx and incy.  One pass, three accumulators. */
double oracle_T(const double* x, int64_t incx, const double* y, int64_t incy,
                int64_t n) {
  double dot = 0.0, xx = 0.0, yy = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double a = x[k * incx];
    double b = y[k * incy];
    dot += a * b;
    xx += a * a;
    yy += b * b;
  }
  double den = xx + yy - fabs(dot);
  if (den == 0.0) return 0.0;
  return dot / sqrt(den);
}

/* Out[i][j] = T(row i of X, column j of Y).  X is M x K, Y is K x N, both
 * row-major FP64; Out is M x N.  This is the Tfunction of Sec. II-C computed
 * entry by entry.  Column j of Y is gathered once per j (a copy, no
 * arithmetic) so that the inner loop runs over contiguous memory. */
int oracle_tanimoto(const double* X, const double* Y, int64_t M, int64_t K,
                    int64_t N, double* Out) {
  if (M < 0 || K < 0 || N < 0) return ORACLE_ERR_ARG;
  int fail = 0;
#pragma omp parallel
  {
    double* col = (double*)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    if (!col) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t j = 0; j < N; ++j) {
      if (!col) continue;
      for (int64_t k = 0; k < K; ++k) col[k] = Y[k * N + j];
      for (int64_t i = 0; i < M; ++i) Out[i * N + j] = oracle_T(X + i * K, 1, col, 1, K);
    }
    free(col);
  }
  return fail ? ORACLE_ERR_NOMEM : ORACLE_OK;
}

/* Sampled entries of the same matrix: Out[s] = T(row rows[s] of X, column
 * cols[s] of Y). */
int oracle_tanimoto_entries(const double* X, const double* Y, int64_t M,
                            int64_t K, int64_t N, const int64_t* rows,
                            const int64_t* cols, int64_t n, double* Out) {
  for (int64_t s = 0; s < n; ++s)
    if (rows[s] < 0 || rows[s] >= M || cols[s] < 0 || cols[s] >= N) return ORACLE_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < n; ++s)
    Out[s] = oracle_T(X + rows[s] * K, 1, Y + cols[s], N, K);
  return ORACLE_OK;
}

/* Z-score of one network (Sec. II-A, NormalizeNetwork): mean and population
 * standard deviation over all entries, then M <- (M - mean) / std. */
int oracle_normalize(double* Mat, int64_t n) {
  if (n < 1 || !Mat) return ORACLE_ERR_ARG;
  for (int64_t k = 0; k < n; ++k)
    if (!isfinite(Mat[k])) return ORACLE_ERR_NONFINITE;
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += Mat[k];
  double mean = s / (double)n;
  double q = 0.0;
  for (int64_t k = 0; k < n; ++k) q += (Mat[k] - mean) * (Mat[k] - mean);
  double sd = sqrt(q / (double)n);
  if (!(sd > 0.0)) return ORACLE_ERR_DEGENERATE;
  for (int64_t k = 0; k < n; ++k) Mat[k] = (Mat[k] - mean) / sd;
  return ORACLE_OK;
}

/* Z-score with a choice of scope and normaliser (readings of the single
 * sentence of Sec. II-A): mode 0 = mean and standard deviation over all
 * entries (what oracle_normalize does); mode 1 = each row by its own mean
 * and standard deviation; mode 2 = (Zr + Zc) / sqrt(2), Zr the per-row and
 * Zc the per-column z-score of the same input.  ddof 0 divides the sum of
 * squared deviations by the count n (population), ddof 1 by n - 1 (sample).
 * A set with zero spread, or with n - ddof < 1, is ORACLE_ERR_DEGENERATE;
 * NaN/Inf is ORACLE_ERR_NONFINITE; on an error M is left untouched. */
static int mean_sd(const double* x, int64_t n, int64_t stride, int32_t ddof, double* mean,
                   double* sd) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += x[k * stride];
  *mean = s / (double)n;
  double q = 0.0;
  for (int64_t k = 0; k < n; ++k) q += (x[k * stride] - *mean) * (x[k * stride] - *mean);
  if (n - ddof < 1) return ORACLE_ERR_DEGENERATE;
  *sd = sqrt(q / (double)(n - ddof));
  return *sd > 0.0 ? ORACLE_OK : ORACLE_ERR_DEGENERATE;
}

int oracle_normalize_ex(double* Mat, int64_t rows, int64_t cols, int32_t mode, int32_t ddof) {
  if (!Mat || rows < 1 || cols < 1 || mode < 0 || mode > 2 || ddof < 0 || ddof > 1)
    return ORACLE_ERR_ARG;
  const int64_t n = rows * cols;
  for (int64_t k = 0; k < n; ++k)
    if (!isfinite(Mat[k])) return ORACLE_ERR_NONFINITE;
  if (mode == 0) {
    double mean, sd;
    int st = mean_sd(Mat, n, 1, ddof, &mean, &sd);
    if (st != ORACLE_OK) return st;
    for (int64_t k = 0; k < n; ++k) Mat[k] = (Mat[k] - mean) / sd;
    return ORACLE_OK;
  }
  double* rm = (double*)malloc(sizeof(double) * (size_t)rows * 2);
  double* cm = (double*)malloc(sizeof(double) * (size_t)cols * 2);
  if (!rm || !cm) {
    free(rm);
    free(cm);
    return ORACLE_ERR_NOMEM;
  }
  int st = ORACLE_OK;
  for (int64_t i = 0; i < rows && st == ORACLE_OK; ++i)
    st = mean_sd(Mat + i * cols, cols, 1, ddof, &rm[2 * i], &rm[2 * i + 1]);
  if (mode == 2)
    for (int64_t j = 0; j < cols && st == ORACLE_OK; ++j)
      st = mean_sd(Mat + j, rows, cols, ddof, &cm[2 * j], &cm[2 * j + 1]);
  if (st == ORACLE_OK) {
    for (int64_t i = 0; i < rows; ++i)
      for (int64_t j = 0; j < cols; ++j) {
        double x = Mat[i * cols + j];
        double zr = (x - rm[2 * i]) / rm[2 * i + 1];
        Mat[i * cols + j] = mode == 1 ? zr : (zr + (x - cm[2 * j]) / cm[2 * j + 1]) / sqrt(2.0);
      }
  }
  free(rm);
  free(cm);
  return st;
}

/* Standard deviation of the off-diagonal entries of row i of the n x n
 * matrix S (Eq. 6 and the sentence after it): population (ddof 0) or sample
 * (ddof 1).  Fewer than ddof + 1 entries give 0. */
static double offdiag_row_std(const double* S, int64_t n, int64_t i, int32_t ddof) {
  if (n - 1 - ddof < 1) return 0.0;
  double s = 0.0;
  for (int64_t m = 0; m < n; ++m)
    if (m != i) s += S[i * n + m];
  double mean = s / (double)(n - 1);
  double q = 0.0;
  for (int64_t m = 0; m < n; ++m)
    if (m != i) q += (S[i * n + m] - mean) * (S[i * n + m] - mean);
  return sqrt(q / (double)(n - 1 - ddof));
}

/* W-side of one iteration: Wn = (1-alpha) W + alpha/2 (A + R) with
 * R = T(P, W) (Eq. 3) and A = T(W, C) (Eq. 4), both from the previous
 * iterate; hp receives h (Eq. 7, or the undamped variant). */
static int w_half_step(const double* W, const double* P, const double* C,
                       int64_t Ne, int64_t Na, const oracle_opts* o,
                       double* Wn, double* hp) {
  size_t nw = (size_t)Ne * (size_t)Na;
  double* R = (double*)malloc(sizeof(double) * nw);
  double* A = (double*)malloc(sizeof(double) * nw);
  if (!R || !A) {
    free(R);
    free(A);
    return ORACLE_ERR_NOMEM;
  }
  int st = oracle_tanimoto(P, W, Ne, Ne, Na, R); /* R_ij = T(P_i., W_.j) */
  if (st == ORACLE_OK) st = oracle_tanimoto(W, C, Ne, Na, Na, A); /* A_ij = T(W_i., C_.j) */
  if (st != ORACLE_OK) {
    free(R);
    free(A);
    return st;
  }
  const double a = o->alpha;
  double hsum = 0.0;
  for (size_t k = 0; k < nw; ++k) {
    double pred = 0.5 * (A[k] + R[k]);
    Wn[k] = (1.0 - a) * W[k] + a * pred;
    hsum += o->h_undamped ? fabs(pred - W[k]) : fabs(Wn[k] - W[k]);
  }
  *hp = hsum / (double)nw;
  free(R);
  free(A);
  return ORACLE_OK;
}

/* Eq. 5 and Eq. 6 for one symmetric network S (n x n): Tm is the fresh
 * similarity matrix, mult the Eq. 6 multiplier, t the iteration number.
 * Off-diagonal entries are damped towards Tm; the diagonal follows Eq. 6. */
static void sym_update(double* S, const double* Tm, int64_t n, double mult,
                       int32_t t, const oracle_opts* o) {
  const double a = o->alpha;
  double* Sn = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* sig = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t m = 0; m < n; ++m)
      Sn[i * n + m] = (i == m) ? S[i * n + m] : (1.0 - a) * S[i * n + m] + a * Tm[i * n + m];
  for (int64_t i = 0; i < n; ++i)
    sig[i] = offdiag_row_std(o->sigma_from_T ? Tm : Sn, n, i, o->sigma_ddof);
  double g = exp(2.0 * a * (double)t);
  for (int64_t i = 0; i < n; ++i) {
    double inc = mult * sig[i] * g;
    if (o->diag_alpha) inc = a * inc;
    Sn[i * n + i] = (1.0 - a) * S[i * n + i] + inc;
  }
  memcpy(S, Sn, sizeof(double) * (size_t)n * (size_t)n);
  free(Sn);
  free(sig);
}

/* One message-passing iteration (Sec. II-B) in place on (W, P, C), t >= 1.
 * On return *h holds Eq. 7 and *conv is 1 when h < tol (then P and C are left
 * untouched unless update_last is set). */
int oracle_step(double* W, double* P, double* C, int64_t Ne, int64_t Na,
                int32_t t, const oracle_opts* o, double* h, int32_t* conv) {
  if (!W || !P || !C || !o || Ne < 1 || Na < 1 || t < 1) return ORACLE_ERR_ARG;
  size_t nw = (size_t)Ne * (size_t)Na;
  double* Wn = (double*)malloc(sizeof(double) * nw);
  if (!Wn) return ORACLE_ERR_NOMEM;
  double hv = 0.0;
  int st = w_half_step(W, P, C, Ne, Na, o, Wn, &hv);
  if (st != ORACLE_OK) {
    free(Wn);
    return st;
  }
  memcpy(W, Wn, sizeof(double) * nw);
  free(Wn);
  *h = hv;
  *conv = (hv < o->tol) ? 1 : 0;
  if (*conv && !o->update_last) return ORACLE_OK;

  /* Eq. 5, P: T(W_i., W_m.) -- rows of the new W.  As a matrix this is
   * T(W, W^T), so build W^T once (a copy) and reuse the Tfunction. */
  double* Wt = (double*)malloc(sizeof(double) * nw);
  double* TP = (double*)malloc(sizeof(double) * (size_t)Ne * (size_t)Ne);
  double* TC = (double*)malloc(sizeof(double) * (size_t)Na * (size_t)Na);
  if (!Wt || !TP || !TC) {
    free(Wt);
    free(TP);
    free(TC);
    return ORACLE_ERR_NOMEM;
  }
  for (int64_t i = 0; i < Ne; ++i)
    for (int64_t j = 0; j < Na; ++j) Wt[j * Ne + i] = W[i * Na + j];
  st = oracle_tanimoto(W, Wt, Ne, Na, Ne, TP); /* TP_im = T(W_i., W_m.) */
  /* Eq. 5, C: T(W_.k, W_.j) -- columns of the new W, i.e. T(W^T, W). */
  if (st == ORACLE_OK) st = oracle_tanimoto(Wt, W, Na, Ne, Na, TC);
  free(Wt);
  if (st != ORACLE_OK) {
    free(TP);
    free(TC);
    return st;
  }
  double multP = o->n_own ? (double)Ne : (double)Na;
  double multC = o->n_own ? (double)Na : (double)Ne;
  sym_update(P, TP, Ne, multP, t, o);
  sym_update(C, TC, Na, multC, t, o);
  free(TP);
  free(TC);
  return ORACLE_OK;
}

/* Whole message-passing procedure from t = t0 + 1 until h < tol or max_iter
 * iterations have run.  h_trace (optional, length max_iter) receives h per
 * iteration.  Returns OK or NOT_CONVERGED; *iters is the last t reached. */
int oracle_run(double* W, double* P, double* C, int64_t Ne, int64_t Na,
               int32_t t0, const oracle_opts* o, int32_t* iters, double* h,
               double* h_trace) {
  if (!o || o->max_iter < 1 || !(o->alpha > 0.0) || o->alpha > 1.0 || !(o->tol >= 0.0) || t0 < 0 ||
      o->sigma_ddof < 0 || o->sigma_ddof > 1)
    return ORACLE_ERR_ARG;
  double hv = 0.0;
  int32_t conv = 0, t = t0;
  for (int32_t it = 0; it < o->max_iter; ++it) {
    ++t;
    int st = oracle_step(W, P, C, Ne, Na, t, o, &hv, &conv);
    if (st != ORACLE_OK) return st;
    if (h_trace) h_trace[it] = hv;
    if (conv) break;
  }
  *iters = t;
  *h = hv;
  return conv ? ORACLE_OK : ORACLE_NOT_CONVERGED;
}

/* Sampled entries of the W produced by one iteration from (W, P, C):
 * Out[s] = (1-alpha) W_ij + alpha/2 (T(P_i., W_.j) + T(W_i., C_.j)) with
 * (i, j) = (rows[s], cols[s]).  Used at sizes where the full step is too slow. */
int oracle_step_w_entries(const double* W, const double* P, const double* C,
                          int64_t Ne, int64_t Na, double alpha,
                          const int64_t* rows, const int64_t* cols, int64_t n,
                          double* Out) {
  for (int64_t s = 0; s < n; ++s)
    if (rows[s] < 0 || rows[s] >= Ne || cols[s] < 0 || cols[s] >= Na) return ORACLE_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = rows[s], j = cols[s];
    double r = oracle_T(P + i * Ne, 1, W + j, Na, Ne);
    double a = oracle_T(W + i * Na, 1, C + j, Na, Na);
    Out[s] = (1.0 - alpha) * W[i * Na + j] + alpha * 0.5 * (a + r);
  }
  return ORACLE_OK;
}

/* Pearson correlation between rows i and j of the expression matrix E
 * (G genes x S samples, row-major): the co-expression prior of Sec. II-A,
 * a correlation of two genes across all samples.  Straight from its
 * definition: the two row means, then the sum of products of the centred
 * entries over the square root of the product of the two centred sums of
 * squares.  A constant row (centred sum of squares 0) has no defined
 * correlation: it gets 0 with every other row.  The diagonal is 1. */
static double pearson_pair(const double* E, int64_t S, int64_t i, int64_t j) {
  if (i == j) return 1.0;
  const double* x = E + i * S;
  const double* y = E + j * S;
  double sx = 0.0, sy = 0.0;
  for (int64_t k = 0; k < S; ++k) {
    sx += x[k];
    sy += y[k];
  }
  double mx = sx / (double)S, my = sy / (double)S;
  double sxy = 0.0, sxx = 0.0, syy = 0.0;
  for (int64_t k = 0; k < S; ++k) {
    double a = x[k] - mx, b = y[k] - my;
    sxy += a * b;
    sxx += a * a;
    syy += b * b;
  }
  if (sxx == 0.0 || syy == 0.0) return 0.0;
  return sxy / sqrt(sxx * syy);
}

/* C[i][j] = Pearson correlation of rows i and j of E, G x G. */
int oracle_pearson(const double* E, int64_t G, int64_t S, double* C) {
  if (G < 1 || S < 2 || !E || !C) return ORACLE_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < G; ++i)
    for (int64_t j = 0; j < G; ++j) C[i * G + j] = pearson_pair(E, S, i, j);
  return ORACLE_OK;
}

/* Sampled entries of the same matrix: Out[s] = C[rows[s]][cols[s]]. */
int oracle_pearson_entries(const double* E, int64_t G, int64_t S, const int64_t* rows,
                           const int64_t* cols, int64_t n, double* Out) {
  if (G < 1 || S < 2 || !E) return ORACLE_ERR_ARG;
  for (int64_t s = 0; s < n; ++s)
    if (rows[s] < 0 || rows[s] >= G || cols[s] < 0 || cols[s] >= G) return ORACLE_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < n; ++s) Out[s] = pearson_pair(E, S, rows[s], cols[s]);
  return ORACLE_OK;
}
