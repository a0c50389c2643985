// Element-wise and reduction kernels of the PANDA iteration: the h of Eq. 7,
// the second half of the P update (Eq. 5), the diagonal rule of Eq. 6, the
// squared-norm vectors the similarity epilogues read, and the z-score
// normalisation of Sec. II-A.  All reductions are FP64 and run in a fixed
// order, so results do not depend on scheduling.
#include "update_device.h"

namespace panda {
namespace {

using upd::block_sum;
using upd::split_bf16;
constexpr int kRT = upd::kUT;  // threads per block for the kernels in this file

__global__ __launch_bounds__(kRT) void k_finish_h(const double* __restrict__ hpart, int64_t n,
                                                  int64_t count, DevState* st, double tol,
                                                  int32_t update_last) {
  __shared__ double red[4];
  upd::finish_h(hpart, n, count, st, tol, update_last, red);
}

__global__ __launch_bounds__(kRT) void k_coop_finalize(
    const float* __restrict__ part, int splits, int64_t Nep, const double* __restrict__ nW,
    float* __restrict__ P, int64_t ldp, int64_t Ne, double alpha, float* __restrict__ Tside,
    bf16_t* __restrict__ Ph, bf16_t* __restrict__ Pl, const int32_t* gate) {
  if (*gate == 0) return;
  upd::coop_finalize_entry((int64_t)blockIdx.x * kRT + threadIdx.x, part, splits, Nep, nW, P, ldp,
                           Ne, alpha, Tside, Ph, Pl);
}

// Eq. 6 for both networks.  Blocks [0, Ne): row i of P; remaining blocks:
// one thread per row of C.  The diagonals live in the FP64 vectors dP, dC.
__global__ __launch_bounds__(kRT) void k_diagonals(
    const float* __restrict__ P, int64_t ldp, double* __restrict__ dP, int64_t Ne,
    const float* __restrict__ Tside, double* __restrict__ nP, double* __restrict__ dC,
    int64_t ldc, int64_t Na, const double2* __restrict__ cstat, const double* __restrict__ csq,
    int64_t nslots, double* __restrict__ nC, double alpha, int32_t diag_alpha, int32_t n_own,
    int32_t ddof, const DevState* st, int32_t sched, double keep, double g, int64_t b0) {
  __shared__ double red[4];
  if (st->run_pc == 0) return;
  upd::DiagRule dr = upd::diag_rule(alpha, diag_alpha, n_own, ddof, st->t);
  if (sched) {  // closed form of several steps (warm state)
    dr.keep = keep;
    dr.g = g;
  }
  const int64_t blk = (int64_t)blockIdx.x + b0;  // launches of one part start at b0
  if (blk < Ne) {
    upd::diag_p_row(blk, P, ldp, dP, Ne, Na, Tside, nP, dr, red);
    return;
  }
  // C: 64 rows per block; wave w adds slots w, w + 4, ... and wave 0 adds
  // the four partial sums in wave order
  __shared__ double3 part[kRT / 64][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (blk - Ne) * 64 + lane;
  double s1 = 0.0, s2 = 0.0, c2 = 0.0;
  if (r < Na) {
    // slots w, w + 4, ..., added in that order; eight slots' loads are in
    // flight before the first of them is added
    constexpr int64_t kStep = kRT / 64, kU = 8;
    int64_t sl = w;
    for (; sl + (kU - 1) * kStep < nslots; sl += kU * kStep) {
      double2 v[kU];
      double q[kU];
#pragma unroll
      for (int k = 0; k < kU; ++k) {
        v[k] = cstat[(sl + k * kStep) * ldc + r];
        q[k] = csq ? csq[(sl + k * kStep) * ldc + r] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kU; ++k) {
        s1 += v[k].x;
        s2 += v[k].y;
        if (csq) c2 += q[k];
      }
    }
    for (; sl < nslots; sl += kStep) {
      const double2 v = cstat[sl * ldc + r];
      s1 += v.x;
      s2 += v.y;
      if (csq) c2 += csq[sl * ldc + r];
    }
  }
  part[w][lane] = make_double3(s1, s2, c2);
  __syncthreads();
  if (w == 0 && r < Na) {
    double3 t = part[0][lane];
    for (int k = 1; k < kRT / 64; ++k) {
      t.x += part[k][lane].x;
      t.y += part[k][lane].y;
      t.z += part[k][lane].z;
    }
    upd::diag_c_finish(r, t.x, t.y, csq ? t.z : t.y, dC, Ne, Na, nC, dr);
  }
}

// d[i] = M[i][i] and M[i][i] = 0: the diagonal moves to its FP64 vector.
__global__ __launch_bounds__(kRT) void k_take_diag(float* __restrict__ M, int64_t n, int64_t ld,
                                                   double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (i >= n) return;
  d[i] = (double)M[i * ld + i];
  M[i * ld + i] = 0.0f;
}

// M[i][i] = d[i] (rounded to FP32): the diagonal back into a stored matrix.
__global__ __launch_bounds__(kRT) void k_put_diag(float* __restrict__ M, int64_t n, int64_t ld,
                                                  const double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (i < n) M[i * ld + i] = (float)d[i];
}

// ---- co-expression prior (Sec. II-A) ---------------------------------------
// Pearson correlation between genes across samples.  Per row: mean and
// centred sum of squares in FP64 (two passes), one wave per row.
__global__ __launch_bounds__(kRT) void k_pearson_stats(const float* __restrict__ E, int64_t G,
                                                       int64_t S, int64_t lde,
                                                       double2* __restrict__ stat) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (kRT / 64) + (threadIdx.x >> 6);
  if (i >= G) return;
  const float* e = E + i * lde;
  double s = 0.0;
  for (int64_t k = lane; k < S; k += 64) s += (double)e[k];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  const double mean = s / (double)S;
  double q = 0.0;
  for (int64_t k = lane; k < S; k += 64) q += ((double)e[k] - mean) * ((double)e[k] - mean);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off);
  // a constant row gets scale 0: its normalised entries are 0
  if (lane == 0) stat[i] = make_double2(mean, q > 0.0 ? 1.0 / sqrt(q) : 0.0);
}

// Zt[k][i] = (E[i][k] - mean_i) / sqrt(ss_i), zero-padded, through a 64 x 64
// tile in LDS so that E is read and Zt written along their rows.
__global__ __launch_bounds__(kRT) void k_pearson_z(const float* __restrict__ E, int64_t G,
                                                   int64_t S, int64_t lde,
                                                   const double2* __restrict__ stat,
                                                   float* __restrict__ Zt, int64_t Gp,
                                                   int64_t Sp) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr, c = c0 + tx;
    float v = 0.0f;
    if (r < G && c < S) {
      const double2 st = stat[r];
      v = (float)(((double)E[r * lde + c] - st.x) * st.y);
    }
    tile[rr][tx] = v;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t c = c0 + cc, r = r0 + tx;
    if (r < Gp && c < Sp) Zt[c * Gp + r] = tile[tx][cc];
  }
}

// ---- split-BF16 operand planes ----------------------------------------------
// Planes of P without its diagonal (which lives in its FP64 vector).
__global__ __launch_bounds__(kRT) void k_split_offdiag(const float* __restrict__ M, int64_t n,
                                                       int64_t ld, bf16_t* __restrict__ Mh,
                                                       bf16_t* __restrict__ Ml) {
  const int64_t tot = n * n;
  for (int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * kRT) {
    const int64_t i = e / n, j = e % n;
    bf16_t h = 0, l = 0;
    if (i != j) split_bf16(M[i * ld + j], h, l);
    Mh[i * ld + j] = h;
    Ml[i * ld + j] = l;
  }
}

// ---- squared norms --------------------------------------------------------
// Squared norms of the rows and columns of W in one pass (Eq. 9 needs
// |W_i.|^2 and |W_.j|^2), and with SHADOW also its bf16 hi/lo planes,
// row-major and gene-major.  Block (bx, by) takes the 64 x 64 tile at rows
// 64 by, columns 64 bx and writes FP64 partial sums: rowpart[bx][r] over its
// 64 columns, colpart[by][c] over its 64 rows; k_w_norms_sum adds them up in
// block order (deterministic).  The tile is staged in LDS: a column's sum is
// the thread's own (its 16 rows, then the four waves in order), a row's the
// sum of four threads' quarters (16 columns each, in order) combined within
// the quad of lanes.  The planes are written whole tiles at a time from the
// staged tile, 8 entries (16 bytes) per store; entries past Ne x Na are zero
// in the tile, so the padding of the planes stays zero.
template <bool SHADOW>
__global__ __launch_bounds__(kRT) void k_w_norms(const float* __restrict__ W, int64_t Ne,
                                                 int64_t Na, int64_t ldw, int64_t Nep,
                                                 double* __restrict__ rowpart,
                                                 double* __restrict__ colpart,
                                                 bf16_t* __restrict__ Wh, bf16_t* __restrict__ Wl,
                                                 bf16_t* __restrict__ Wth,
                                                 bf16_t* __restrict__ Wtl, int64_t ldt,
                                                 const int32_t* gate) {
  __shared__ float tile[64][65];
  __shared__ double cred[4][64];
  if (gate && *gate == 0) return;
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  double cs = 0.0;
  // this thread's 16 entries, all loads in flight before the first is used
  float vals[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t r = r0 + ty + 4 * k, c = c0 + tx;
    vals[k] = (r < Ne && c < Na) ? W[r * ldw + c] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float v = vals[k];
    tile[ty + 4 * k][tx] = v;
    cs += (double)v * (double)v;
  }
  cred[ty][tx] = cs;
  __syncthreads();
  {
    // row rr, quarter q: entries 16 q .. 16 q + 15 (pitch 65: the 64 lanes of
    // a read hit 64 distinct banks)
    const int rr = threadIdx.x >> 2, q = threadIdx.x & 3;
    double rs = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double v = tile[rr][16 * q + i];
      rs += v * v;
    }
    rs += __shfl_xor(rs, 1);  // (q0 + q1) and (q2 + q3) ..
    rs += __shfl_xor(rs, 2);  // .. then their sum, the same in all four lanes
    if (q == 0) rowpart[(int64_t)blockIdx.x * Nep + r0 + rr] = rs;
  }
  if (ty == 0)
    colpart[(int64_t)blockIdx.y * gridDim.x * 64 + c0 + tx] =
        ((cred[0][tx] + cred[1][tx]) + cred[2][tx]) + cred[3][tx];
  if constexpr (SHADOW) {
    // thread t: line t / 8 (+ 32 in the second pass), entries 8 (t % 8) .. +7
    const int q = threadIdx.x & 7;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int line = (int)(threadIdx.x >> 3) + 32 * pass;
      unsigned rh[4], rl[4], th[4], tl[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bf16_t h0, l0, h1, l1;
        split_bf16(tile[line][8 * q + 2 * e], h0, l0);  // row line, along the columns
        split_bf16(tile[line][8 * q + 2 * e + 1], h1, l1);
        rh[e] = (unsigned)h0 | ((unsigned)h1 << 16);
        rl[e] = (unsigned)l0 | ((unsigned)l1 << 16);
        split_bf16(tile[8 * q + 2 * e][line], h0, l0);  // column line, along the rows
        split_bf16(tile[8 * q + 2 * e + 1][line], h1, l1);
        th[e] = (unsigned)h0 | ((unsigned)h1 << 16);
        tl[e] = (unsigned)l0 | ((unsigned)l1 << 16);
      }
      const int64_t ro = (r0 + line) * ldw + c0 + 8 * q;  // rows < Nep, columns < ldw
      const int64_t to = (c0 + line) * ldt + r0 + 8 * q;  // columns < ldw, rows < ldt
      *reinterpret_cast<uint4*>(Wh + ro) = make_uint4(rh[0], rh[1], rh[2], rh[3]);
      *reinterpret_cast<uint4*>(Wl + ro) = make_uint4(rl[0], rl[1], rl[2], rl[3]);
      *reinterpret_cast<uint4*>(Wth + to) = make_uint4(th[0], th[1], th[2], th[3]);
      *reinterpret_cast<uint4*>(Wtl + to) = make_uint4(tl[0], tl[1], tl[2], tl[3]);
    }
  }
}

// Sums of the partials of k_w_norms: blocks [0, Nep) one row each, then
// the columns, kRT per block.
__global__ __launch_bounds__(kRT) void k_w_norms_sum(const double* __restrict__ rowpart,
                                                     const double* __restrict__ colpart,
                                                     int64_t Nep, int64_t Nap,
                                                     double* __restrict__ nr,
                                                     double* __restrict__ nc,
                                                     const int32_t* gate) {
  __shared__ double red[kRT / 64];
  if (gate && *gate == 0) return;
  const int64_t ncb = Nap / 64, nrb = Nep / 64;
  if ((int64_t)blockIdx.x < Nep) {
    const int64_t r = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < ncb; b += kRT) s += rowpart[b * Nep + r];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) nr[r] = tot;
    return;
  }
  const int64_t c = ((int64_t)blockIdx.x - Nep) * kRT + threadIdx.x;
  if (c >= Nap) return;
  // blocks in order; eight blocks' loads in flight before the first is added
  double s = 0.0;
  int64_t b = 0;
  for (; b + 8 <= nrb; b += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = colpart[(b + k) * Nap + c];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; b < nrb; ++b) s += colpart[b * Nap + c];
  nc[c] = s;
}

__global__ __launch_bounds__(kRT) void k_row_sqnorms(const float* __restrict__ M, int64_t cols,
                                                     int64_t ld, double* __restrict__ out,
                                                     const int32_t* gate) {
  __shared__ double red[4];
  if (gate && *gate == 0) return;
  const double tot = upd::row_sqnorm(M + (int64_t)blockIdx.x * ld, cols, red);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// Column sums of squares over row chunk blockIdx.y, into scratch[chunk][col].
__global__ __launch_bounds__(kRT) void k_col_sqnorms_part(const float* __restrict__ M,
                                                          int64_t rows, int64_t cols, int64_t ld,
                                                          int64_t chunk, double* __restrict__ scr,
                                                          const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int64_t j = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (j >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  scr[(int64_t)blockIdx.y * cols + j] = upd::col_sqnorm_part(M, ld, j, r0, r1);
}

__global__ __launch_bounds__(kRT) void k_col_sqnorms_sum(const double* __restrict__ scr,
                                                         int64_t cols, int nchunks,
                                                         double* __restrict__ out,
                                                         const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int64_t j = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += scr[(int64_t)c * cols + j];
  out[j] = s;
}

// ---- z-score --------------------------------------------------------------
// scratch layout: [0, kZsBlocks) block partials, then
// [kZsBlocks + 0] mean, [+1] std, [+2] 1.0 if any entry is NaN or Inf.
__global__ __launch_bounds__(kRT) void k_zs_sum(const float* __restrict__ M, int64_t rows,
                                                int64_t cols, int64_t ld, double* scratch,
                                                int pass) {
  __shared__ double red[4];
  const int64_t n = rows * cols;
  const double mean = pass ? scratch[kZsBlocks] : 0.0;
  double s = 0.0, bad = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRT) {
    const double x = (double)M[(e / cols) * ld + e % cols];
    if (!isfinite(x)) bad += 1.0;
    s += pass ? (x - mean) * (x - mean) : x;
  }
  const double tot = block_sum(s, red);
  double nb = 0.0;
  if (!pass) nb = block_sum(bad, red);
  if (threadIdx.x == 0) {
    scratch[blockIdx.x] = tot;
    if (!pass && nb > 0.0) scratch[kZsBlocks + 2] = 1.0;  // every writer stores the same 1.0
  }
}

__global__ __launch_bounds__(kRT) void k_zs_finish(double* scratch, int64_t n, int pass,
                                                   int ddof) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < kZsBlocks; i += kRT) s += scratch[i];
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) {
    if (!pass) {
      scratch[kZsBlocks] = tot / (double)n;
    } else {
      // std = 0 (a constant network, or no degree of freedom) is reported
      scratch[kZsBlocks + 1] = n - ddof >= 1 ? sqrt(tot / (double)(n - ddof)) : 0.0;
    }
  }
}

__global__ __launch_bounds__(kRT) void k_zs_clear(double* scratch) {
  for (int i = threadIdx.x; i < kZsBlocks + 8; i += kRT) scratch[i] = 0.0;
}

__global__ __launch_bounds__(kRT) void k_zs_apply(float* __restrict__ M, int64_t rows,
                                                  int64_t cols, int64_t ld,
                                                  const double* __restrict__ scratch) {
  const double mean = scratch[kZsBlocks], sd = scratch[kZsBlocks + 1];
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRT) {
    float* p = M + (e / cols) * ld + e % cols;
    *p = (float)(((double)*p - mean) / sd);
  }
}

// Z-score per row, or row + column (scopes of the z-score of Sec. II-A).
// flags[0] = 1 if an entry is NaN/Inf, flags[1] = 1 if a row or column has
// zero spread (every writer stores the same 1.0).  Moments in FP64, two
// passes; sd = 0 when fewer than ddof + 1 entries.
__global__ __launch_bounds__(kRT) void k_zs_rows(const float* __restrict__ M, int64_t cols,
                                                 int64_t ld, int ddof, double2* __restrict__ rs,
                                                 double* flags) {
  __shared__ double red[4];
  const float* row = M + (int64_t)blockIdx.x * ld;
  double s = 0.0, bad = 0.0;
  for (int64_t j = threadIdx.x; j < cols; j += kRT) {
    const double x = (double)row[j];
    if (!isfinite(x)) bad += 1.0;
    s += x;
  }
  const double mean = block_sum(s, red) / (double)cols;
  const double nb = block_sum(bad, red);
  double q = 0.0;
  for (int64_t j = threadIdx.x; j < cols; j += kRT) {
    const double d = (double)row[j] - mean;
    q += d * d;
  }
  const double qs = block_sum(q, red);
  if (threadIdx.x == 0) {
    const double sd = cols - ddof >= 1 ? sqrt(qs / (double)(cols - ddof)) : 0.0;
    rs[blockIdx.x] = make_double2(mean, sd);
    if (nb > 0.0) flags[0] = 1.0;
    if (!(sd > 0.0)) flags[1] = 1.0;
  }
}

// Column moments, one thread per column walking down the rows (coalesced
// across the wave).
__global__ __launch_bounds__(kRT) void k_zs_cols(const float* __restrict__ M, int64_t rows,
                                                 int64_t cols, int64_t ld, int ddof,
                                                 double2* __restrict__ cs, double* flags) {
  const int64_t j = (int64_t)blockIdx.x * kRT + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < rows; ++i) s += (double)M[i * ld + j];
  const double mean = s / (double)rows;
  double q = 0.0;
  for (int64_t i = 0; i < rows; ++i) {
    const double d = (double)M[i * ld + j] - mean;
    q += d * d;
  }
  const double sd = rows - ddof >= 1 ? sqrt(q / (double)(rows - ddof)) : 0.0;
  cs[j] = make_double2(mean, sd);
  if (!(sd > 0.0)) flags[1] = 1.0;
}

__global__ __launch_bounds__(kRT) void k_zs_apply_rc(float* __restrict__ M, int64_t rows,
                                                     int64_t cols, int64_t ld,
                                                     const double2* __restrict__ rs,
                                                     const double2* __restrict__ cs) {
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRT) {
    const int64_t i = e / cols, j = e % cols;
    float* p = M + i * ld + j;
    const double x = (double)*p;
    const double2 r = rs[i];
    const double zr = (x - r.x) / r.y;
    if (cs) {
      const double2 c = cs[j];
      *p = (float)((zr + (x - c.x) / c.y) / sqrt(2.0));
    } else {
      *p = (float)zr;
    }
  }
}

__global__ __launch_bounds__(kRT) void k_zs_flags_clear(double* flags) {
  if (threadIdx.x < 8) flags[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(kRT) void k_fill_identity(float* __restrict__ M, int64_t n,
                                                       int64_t ld) {
  const int64_t tot = n * n;
  for (int64_t e = (int64_t)blockIdx.x * kRT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * kRT) {
    const int64_t i = e / n, j = e % n;
    M[i * ld + j] = (i == j) ? 1.0f : 0.0f;
  }
}

__global__ void k_state_set(DevState* st, int32_t t, int32_t active, int32_t run_pc) {
  if (threadIdx.x == 0) {
    st->t = t;
    st->wsel = 0;
    st->active = active;
    st->run_pc = run_pc;
  }
}

__global__ void k_state_init(DevState* st, int32_t t0) {
  if (threadIdx.x == 0) {
    st->h = 0.0;
    st->t = t0;
    st->active = 1;
    st->run_pc = 0;
    st->conv = 0;
    st->wsel = 0;
    st->pad = 0;
  }
}

unsigned grid_for(int64_t n, int64_t cap) {
  int64_t b = (n + kRT - 1) / kRT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_finish_h(const double* hpart, int64_t n, int64_t count, DevState* st, Rule rule,
                           hipStream_t s) {
  k_finish_h<<<1, kRT, 0, s>>>(hpart, n, count, st, rule.tol, rule.update_last);
  return hipGetLastError();
}

hipError_t launch_coop_finalize(const float* part, int splits, int64_t Nep, const double* nWrow,
                                float* P, int64_t ldp, int64_t Ne, Rule rule, float* Tside,
                                bf16_t* Ph, bf16_t* Pl, const int32_t* gate, hipStream_t s) {
  const int64_t n = Ne * Ne;
  k_coop_finalize<<<dim3((unsigned)((n + kRT - 1) / kRT)), kRT, 0, s>>>(
      part, splits, Nep, nWrow, P, ldp, Ne, rule.alpha, Tside, Ph, Pl, gate);
  return hipGetLastError();
}

hipError_t launch_split_offdiag(const float* M, int64_t n, int64_t ld, bf16_t* Mh, bf16_t* Ml,
                                hipStream_t s) {
  k_split_offdiag<<<grid_for(n * n, 8192), kRT, 0, s>>>(M, n, ld, Mh, Ml);
  return hipGetLastError();
}

hipError_t launch_diagonals(const float* P, int64_t ldp, double* dP, int64_t Ne,
                            const float* Tside, double* nP, double* dC, int64_t ldc, int64_t Na,
                            const double2* cstat, const double* csq, int64_t nslots, double* nC,
                            Rule rule, const DevState* st, hipStream_t s, int part) {
  const int64_t b0 = part == kDiagC ? Ne : 0;
  const int64_t nb = (part == kDiagC ? 0 : Ne) + (part == kDiagP ? 0 : (Na + 63) / 64);
  if (nb == 0) return hipSuccess;
  k_diagonals<<<dim3((unsigned)nb), kRT, 0, s>>>(P, ldp, dP, Ne, Tside, nP, dC, ldc, Na, cstat,
                                                 csq, nslots, nC, rule.alpha, rule.diag_alpha,
                                                 rule.n_own, rule.sigma_ddof, st, 0, 0.0, 0.0, b0);
  return hipGetLastError();
}

hipError_t launch_diagonals_schedule(const float* P, int64_t ldp, double* dP, int64_t Ne,
                                     const float* Tside, double* nP, double* dC, int64_t ldc,
                                     int64_t Na, const double2* cstat, const double* csq,
                                     int64_t nslots, double* nC, Rule rule, double keep, double g,
                                     const DevState* st, hipStream_t s) {
  const int64_t nb = Ne + (Na + 63) / 64;
  k_diagonals<<<dim3((unsigned)nb), kRT, 0, s>>>(P, ldp, dP, Ne, Tside, nP, dC, ldc, Na, cstat,
                                                 csq, nslots, nC, rule.alpha, rule.diag_alpha,
                                                 rule.n_own, rule.sigma_ddof, st, 1, keep, g, 0);
  return hipGetLastError();
}

hipError_t launch_pearson_z(const float* E, int64_t G, int64_t S, int64_t lde, double2* stat,
                            float* Zt, int64_t Gp, int64_t Sp, hipStream_t s) {
  if (Gp % 128 || Sp % 16 || G > Gp || S > Sp) return hipErrorInvalidValue;
  k_pearson_stats<<<dim3((unsigned)((G + kRT / 64 - 1) / (kRT / 64))), kRT, 0, s>>>(E, G, S, lde,
                                                                                  stat);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_pearson_z<<<dim3((unsigned)((Sp + 63) / 64), (unsigned)(Gp / 64)), kRT, 0, s>>>(
      E, G, S, lde, stat, Zt, Gp, Sp);
  return hipGetLastError();
}

hipError_t launch_take_diag(float* M, int64_t n, int64_t ld, double* d, hipStream_t s) {
  k_take_diag<<<dim3((unsigned)((n + kRT - 1) / kRT)), kRT, 0, s>>>(M, n, ld, d);
  return hipGetLastError();
}

hipError_t launch_put_diag(float* M, int64_t n, int64_t ld, const double* d, hipStream_t s) {
  k_put_diag<<<dim3((unsigned)((n + kRT - 1) / kRT)), kRT, 0, s>>>(M, n, ld, d);
  return hipGetLastError();
}

hipError_t launch_state_set(DevState* st, int32_t t, int32_t active, int32_t run_pc,
                            hipStream_t s) {
  k_state_set<<<1, 64, 0, s>>>(st, t, active, run_pc);
  return hipGetLastError();
}

size_t w_norm_scratch_doubles(int64_t Nep, int64_t Nap) {
  const size_t fused = (size_t)(Nap / 64) * (size_t)Nep + (size_t)(Nep / 64) * (size_t)Nap;
  const size_t chunks = (size_t)kColChunks * (size_t)Nap;
  return fused > chunks ? fused : chunks;
}

hipError_t launch_w_norms(const float* W, int64_t Ne, int64_t Na, int64_t ldw, int64_t Nep,
                          double* nr, double* nc, double* scr, bf16_t* Wh, bf16_t* Wl, bf16_t* Wth,
                          bf16_t* Wtl, int64_t ldt, const int32_t* gate, hipStream_t s) {
  const int64_t Nap = ldw;
  if (Nep % 64 || Nap % 64 || Ne > Nep || Na > Nap) return hipErrorInvalidValue;
  if (Wh && (ldt < Nep || ldt % 8)) return hipErrorInvalidValue;  // 16-byte plane stores
  double* rowpart = scr;
  double* colpart = scr + (Nap / 64) * Nep;
  const dim3 grid((unsigned)(Nap / 64), (unsigned)(Nep / 64));
  if (Wh)
    k_w_norms<true><<<grid, kRT, 0, s>>>(W, Ne, Na, ldw, Nep, rowpart, colpart, Wh, Wl, Wth, Wtl,
                                         ldt, gate);
  else
    k_w_norms<false><<<grid, kRT, 0, s>>>(W, Ne, Na, ldw, Nep, rowpart, colpart, nullptr, nullptr,
                                          nullptr, nullptr, ldt, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nb = Nep + (Nap + kRT - 1) / kRT;
  k_w_norms_sum<<<dim3((unsigned)nb), kRT, 0, s>>>(rowpart, colpart, Nep, Nap, nr, nc, gate);
  return hipGetLastError();
}

hipError_t launch_row_sqnorms(const float* M, int64_t rows, int64_t cols, int64_t ld, double* out,
                              const int32_t* gate, hipStream_t s) {
  k_row_sqnorms<<<dim3((unsigned)rows), kRT, 0, s>>>(M, cols, ld, out, gate);
  return hipGetLastError();
}

hipError_t launch_col_sqnorms(const float* M, int64_t rows, int64_t cols, int64_t ld, double* out,
                              double* scratch, const int32_t* gate, hipStream_t s) {
  const int nch = upd::col_chunks(rows);
  const int64_t chunk = (rows + nch - 1) / nch;
  const unsigned gx = (unsigned)((cols + kRT - 1) / kRT);
  k_col_sqnorms_part<<<dim3(gx, (unsigned)nch), kRT, 0, s>>>(M, rows, cols, ld, chunk, scratch,
                                                             gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_col_sqnorms_sum<<<dim3(gx), kRT, 0, s>>>(scratch, cols, nch, out, gate);
  return hipGetLastError();
}

hipError_t launch_zscore_stats(const float* M, int64_t rows, int64_t cols, int64_t ld,
                               double* scratch, hipStream_t s, int ddof) {
  const int64_t n = rows * cols;
  k_zs_clear<<<1, kRT, 0, s>>>(scratch);
  k_zs_sum<<<kZsBlocks, kRT, 0, s>>>(M, rows, cols, ld, scratch, 0);
  k_zs_finish<<<1, kRT, 0, s>>>(scratch, n, 0, ddof);
  k_zs_sum<<<kZsBlocks, kRT, 0, s>>>(M, rows, cols, ld, scratch, 1);
  k_zs_finish<<<1, kRT, 0, s>>>(scratch, n, 1, ddof);
  return hipGetLastError();
}

hipError_t launch_zscore_rc_stats(const float* M, int64_t rows, int64_t cols, int64_t ld, int ddof,
                                  double* flags, double2* rs, double2* cs, hipStream_t s) {
  k_zs_flags_clear<<<1, kRT, 0, s>>>(flags);
  k_zs_rows<<<dim3((unsigned)rows), kRT, 0, s>>>(M, cols, ld, ddof, rs, flags);
  if (cs)
    k_zs_cols<<<dim3((unsigned)((cols + kRT - 1) / kRT)), kRT, 0, s>>>(M, rows, cols, ld, ddof, cs,
                                                                         flags);
  return hipGetLastError();
}

hipError_t launch_zscore_rc_apply(float* M, int64_t rows, int64_t cols, int64_t ld,
                                  const double2* rs, const double2* cs, hipStream_t s) {
  k_zs_apply_rc<<<grid_for(rows * cols, 4096), kRT, 0, s>>>(M, rows, cols, ld, rs, cs);
  return hipGetLastError();
}

hipError_t launch_zscore_apply(float* M, int64_t rows, int64_t cols, int64_t ld,
                               const double* scratch, hipStream_t s) {
  k_zs_apply<<<grid_for(rows * cols, 4096), kRT, 0, s>>>(M, rows, cols, ld, scratch);
  return hipGetLastError();
}

hipError_t launch_fill_identity(float* M, int64_t n, int64_t ld, hipStream_t s) {
  k_fill_identity<<<grid_for(n * n, 4096), kRT, 0, s>>>(M, n, ld);
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, int32_t t0, hipStream_t s) {
  k_state_init<<<1, 64, 0, s>>>(st, t0);
  return hipGetLastError();
}

}  // namespace panda
