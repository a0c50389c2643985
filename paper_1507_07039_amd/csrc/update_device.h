// Device bodies of the element-wise and reduction steps of one PANDA
// iteration: the h of Eq. 7, the second half of the P update (Eq. 5), the
// diagonal rule of Eq. 6 and the squared-norm vectors the similarity
// epilogues read.  The single-network kernels and the grouped (batched)
// kernels both call these, so the two forms share their arithmetic.  All
// reductions are FP64 and run in a fixed order, so results do not depend on
// scheduling.  Every body expects a block of kUT threads.
#pragma once

#include "panda_internal.h"

namespace panda {
namespace upd {

constexpr int kUT = 256;  // threads per block of every body in this file

// Sum of one double per thread over a kUT-thread block, fixed order.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

__device__ __forceinline__ bf16_t to_bf16(float x) {
  return __builtin_bit_cast(bf16_t, (__bf16)x);
}
// hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even.
__device__ __forceinline__ void split_bf16(float x, bf16_t& hi, bf16_t& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - (float)__builtin_bit_cast(__bf16, hi));
}

// h = (1 / count) * sum of the n per-tile partials (Eq. 7); advance t, flip
// the current-W selector and set the gates of the rest of this iteration and
// of the next one.  One block.
__device__ __forceinline__ void finish_h(const double* __restrict__ hpart, int64_t n,
                                         int64_t count, DevState* st, double tol,
                                         int32_t update_last, double* red) {
  if (st->active == 0) {  // converged earlier: this iteration is a no-op
    if (threadIdx.x == 0) st->run_pc = 0;
    return;
  }
  // this thread's partials i, i + kUT, ... added in that order, eight loads
  // in flight before the first of them is added
  double s = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 7 * kUT < n; i += 8 * kUT) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = hpart[i + k * kUT];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; i < n; i += kUT) s += hpart[i];
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double h = tot / (double)count;
    st->h = h;
    st->t = st->t + 1;
    st->wsel ^= 1;
    const int conv = h < tol;
    st->conv = conv;
    st->run_pc = (!conv || update_last) ? 1 : 0;
    if (conv) st->active = 0;
  }
}

// P update, second half (Eq. 5), entry e of the row-major Ne x Ne matrix:
// for i < j sum the split-K partial products, form T(W_i., W_j.) with the
// row norms of the new W and write the damped value at (i, j) and (j, i)
// (and the hi/lo planes, and the fresh similarity when Tside is set).
__device__ __forceinline__ void coop_finalize_entry(
    int64_t e, const float* __restrict__ part, int splits, int64_t Nep,
    const double* __restrict__ nW, float* __restrict__ P, int64_t ldp, int64_t Ne, double alpha,
    float* __restrict__ Tside, bf16_t* __restrict__ Ph, bf16_t* __restrict__ Pl) {
  if (e >= Ne * Ne) return;
  const int64_t i = e / Ne, j = e % Ne;
  if (i >= j) return;
  // the partials in split order, eight loads in flight before the first of
  // them is added
  double dot = 0.0;
  const float* pe = part + i * Nep + j;
  const int64_t ps = Nep * Nep;
  int s = 0;
  for (; s + 8 <= splits; s += 8) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = pe[(int64_t)(s + k) * ps];
#pragma unroll
    for (int k = 0; k < 8; ++k) dot += (double)v[k];
  }
  for (; s < splits; ++s) dot += (double)pe[(int64_t)s * ps];
  const double den = nW[i] + nW[j] - fabs(dot);
  const double tv = den > 0.0 ? dot / sqrt(den) : 0.0;
  const float v = (float)((1.0 - alpha) * (double)P[i * ldp + j] + alpha * tv);
  P[i * ldp + j] = v;
  P[j * ldp + i] = v;
  if (Ph) {
    bf16_t h, l;
    split_bf16(v, h, l);
    Ph[i * ldp + j] = Ph[j * ldp + i] = h;
    Pl[i * ldp + j] = Pl[j * ldp + i] = l;
  }
  if (Tside) {
    Tside[i * ldp + j] = (float)tv;
    Tside[j * ldp + i] = (float)tv;
  }
}

// Scalars of the diagonal rule: new = keep * old + f * N * sigma * g.  One
// step of Eq. 6 at iteration t: keep = 1 - alpha, g = exp(2 alpha t); f =
// alpha (default reading) or 1 (literal).  The warm state uses the closed
// form of t0 such steps with sigma held fixed (diag_schedule_host).
struct DiagRule {
  double keep, g, f;
  int32_t n_own;
  int32_t ddof;  // sigma: population (0) or sample (1) standard deviation
};
__device__ __forceinline__ DiagRule diag_rule(double alpha, int32_t diag_alpha, int32_t n_own,
                                              int32_t ddof, int32_t t) {
  return DiagRule{1.0 - alpha, exp(2.0 * alpha * (double)t), diag_alpha ? alpha : 1.0, n_own,
                  ddof};
}

// A new diagonal is rounded to FP32 like every stored entry, so that a state
// stored to FP32 matrices and loaded again resumes exactly; past the FP32
// range (exp(2 alpha t) overflows it near alpha t ~ 40) it stays FP64, the
// run goes on as in FP64, and only a stored copy of that diagonal reads inf.
__device__ __forceinline__ double diag_round(double x) {
  const float f = (float)x;
  return __builtin_isinf(f) ? x : (double)f;
}

// Eq. 6 for row i of P (one block): standard deviation (population, or
// sample under ddof = 1) of the off-diagonal entries by two passes over the row (of the fresh similarities when Tside is
// set), the new diagonal dP[i] (an FP32 value held in FP64 beside P, which
// holds zero there), and |P_i.|^2 for the next iteration.
__device__ __forceinline__ void diag_p_row(int64_t i, const float* __restrict__ P, int64_t ldp,
                                           double* __restrict__ dP, int64_t Ne, int64_t Na,
                                           const float* __restrict__ Tside,
                                           double* __restrict__ nP, const DiagRule& dr,
                                           double* red) {
  const float* prow = P + i * ldp;
  const float* row = Tside ? Tside + i * ldp : prow;
  double s = 0.0, q2 = 0.0;
  for (int64_t m = threadIdx.x; m < Ne; m += kUT)
    if (m != i) {
      s += row[m];
      q2 += (double)prow[m] * (double)prow[m];
    }
  const double n = (double)(Ne - 1);
  const double mean = Ne > 1 ? block_sum(s, red) / n : 0.0;
  const double off2 = block_sum(q2, red);
  double q = 0.0;
  for (int64_t m = threadIdx.x; m < Ne; m += kUT)
    if (m != i) q += ((double)row[m] - mean) * ((double)row[m] - mean);
  const double qs = block_sum(q, red);
  const double var = n - dr.ddof >= 1.0 ? qs / (n - dr.ddof) : 0.0;
  if (threadIdx.x == 0) {
    const double mult = dr.n_own ? (double)Ne : (double)Na;
    const double dn = diag_round(dr.keep * dP[i] + dr.f * mult * sqrt(var) * dr.g);
    dP[i] = dn;
    nP[i] = off2 + dn * dn;
  }
}

// Eq. 6 for row r of C (one thread), from the per-slot (sum, sum of squares)
// written by the C update (slot stride = ldc, the padded N_a): the new
// Eq. 6 for C_rr from the sum s1 and the sum of squares s2 of the
// off-diagonal entries of row r, and the sum of squares c2 of the updated
// entries (the squared column norm without the diagonal).
__device__ __forceinline__ void diag_c_finish(int64_t r, double s1, double s2, double c2,
                                              double* __restrict__ dC, int64_t Ne, int64_t Na,
                                              double* __restrict__ nC, const DiagRule& dr) {
  // one-pass FP64 variance; the off-diagonal entries of C are O(1) with a
  // mean well below their spread, so the cancellation costs a few FP64 ulps
  double var = 0.0;
  const double n = (double)(Na - 1);
  if (n - dr.ddof >= 1.0) {
    const double mean = s1 / n;
    var = s2 / n - mean * mean;
    if (var < 0.0) var = 0.0;
    if (dr.ddof) var *= n / (n - 1.0);
  }
  const double mult = dr.n_own ? (double)Na : (double)Ne;
  const double dn = diag_round(dr.keep * dC[r] + dr.f * mult * sqrt(var) * dr.g);
  dC[r] = dn;
  nC[r] = c2 + dn * dn;
}

// diagonal dC[r] (FP64) and |C_.r|^2 for the next iteration.
__device__ __forceinline__ void diag_c_row(int64_t r, double* __restrict__ dC, int64_t ldc,
                                           int64_t Ne, int64_t Na,
                                           const double2* __restrict__ cstat,
                                           const double* __restrict__ csq, int64_t nslots,
                                           double* __restrict__ nC, const DiagRule& dr) {
  double s1 = 0.0, s2 = 0.0, c2 = 0.0;
  for (int64_t sl = 0; sl < nslots; ++sl) {
    const double2 v = cstat[sl * ldc + r];
    s1 += v.x;
    s2 += v.y;
    if (csq) c2 += csq[sl * ldc + r];
  }
  if (!csq) c2 = s2;
  diag_c_finish(r, s1, s2, c2, dC, Ne, Na, nC, dr);
}

// |M_r.|^2 of one row (one block).
__device__ __forceinline__ double row_sqnorm(const float* __restrict__ row, int64_t cols,
                                             double* red) {
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < cols; j += kUT) s += (double)row[j] * (double)row[j];
  return block_sum(s, red);
}

// Column sums of squares over rows [r0, r1) for column j (one thread).
__device__ __forceinline__ double col_sqnorm_part(const float* __restrict__ M, int64_t ld,
                                                  int64_t j, int64_t r0, int64_t r1) {
  double s = 0.0;
  for (int64_t i = r0; i < r1; ++i) s += (double)M[i * ld + j] * (double)M[i * ld + j];
  return s;
}

// Row chunks of the column-norm reduction: about 64 rows each, at most
// kColChunks.  The single-network and grouped forms use the same chunking.
__host__ __device__ __forceinline__ int col_chunks(int64_t rows) {
  int nch = (int)((rows + 63) / 64);
  if (nch > kColChunks) nch = kColChunks;
  if (nch < 1) nch = 1;
  return nch;
}

}  // namespace upd
}  // namespace panda
