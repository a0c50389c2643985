// Packed-symmetric storage of the co-regulatory network C (Sec. II-B: C is
// symmetric, and the C update of Eq. 5 keeps it so): the upper kPT x kPT
// tiles only, about half the bytes of the full matrix (the memory note of
// Sec. II-C, and larger gene sets on one GPU).  These kernels move C in and
// out of that layout and take what the iteration needs from it at load time
// (its diagonal and its column norms); the products and the C update read
// and write the layout directly.
#include "panda_internal.h"

namespace panda {
namespace {

constexpr int kNT = 256;                          // threads per block
constexpr int kTileF = (int)(kPT * kPT);          // floats per tile
constexpr int kPerThread = kTileF / kNT;          // entries per thread and tile
constexpr int kLdsLd = (int)kPT + 1;              // staged tile row length

// (a, b), a <= b, of packed tile u.
__device__ __forceinline__ void tile_of(int64_t u, int64_t& a, int64_t& b) {
  int64_t j = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > u) --j;
  while ((j + 1) * (j + 2) / 2 <= u) ++j;
  b = j;
  a = u - j * (j + 1) / 2;
}

// One block per upper tile; consecutive threads take consecutive entries of
// a tile row, so the source rows are read along their length.
__global__ __launch_bounds__(kNT) void k_pack_sym(const float* __restrict__ src, int64_t n,
                                                  int64_t lds, float* __restrict__ dst) {
  int64_t a, b;
  tile_of(blockIdx.x, a, b);
  float* t = dst + (int64_t)blockIdx.x * kTileF;
  for (int q = 0; q < kPerThread; ++q) {
    const int e = threadIdx.x + q * kNT, r = e / (int)kPT, c = e % (int)kPT;
    const int64_t gi = a * kPT + r, gj = b * kPT + c;
    float v = 0.0f;
    if (gi < n && gj < n) v = gi <= gj ? src[gi * lds + gj] : src[gj * lds + gi];
    t[e] = v;
  }
}

// The tile is staged in LDS so that both its own rows and its mirror image
// (the rows of block b, for an off-diagonal tile) are written along rows, 16
// bytes per lane where the row allows (dst 16-byte aligned there and the four
// columns inside n), entry by entry at the edges.
typedef float fv4 __attribute__((ext_vector_type(4)));
constexpr int kC4 = (int)kPT / 4;                 // 16-byte chunks per tile row
constexpr int kPerThread4 = kTileF / 4 / kNT;     // chunks per thread and tile

__device__ __forceinline__ void store4(float* __restrict__ dst, int64_t gi, int64_t gj, int64_t n,
                                       int64_t ldd, const float (&v)[4]) {
  if (gi >= n) return;
  float* p = dst + gi * ldd + gj;
  if (gj + 3 < n && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
    __builtin_nontemporal_store((fv4){v[0], v[1], v[2], v[3]}, reinterpret_cast<fv4*>(p));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (gj + e < n) p[e] = v[e];
  }
}

__global__ __launch_bounds__(kNT) void k_unpack_sym(const float* __restrict__ src, int64_t n,
                                                    float* __restrict__ dst, int64_t ldd) {
  __shared__ float ts[kPT * kLdsLd];
  int64_t a, b;
  tile_of(blockIdx.x, a, b);
  const fv4* t = reinterpret_cast<const fv4*>(src + (int64_t)blockIdx.x * kTileF);
  fv4 v4[kPerThread4];
#pragma unroll
  for (int q = 0; q < kPerThread4; ++q) v4[q] = __builtin_nontemporal_load(t + threadIdx.x + q * kNT);
#pragma unroll
  for (int q = 0; q < kPerThread4; ++q) {
    const int e = threadIdx.x + q * kNT, r = e / kC4, c = (e % kC4) * 4;
    const float v[4] = {v4[q].x, v4[q].y, v4[q].z, v4[q].w};
#pragma unroll
    for (int k = 0; k < 4; ++k) ts[r * kLdsLd + c + k] = v[k];
    store4(dst, a * kPT + r, b * kPT + c, n, ldd, v);
  }
  if (a == b) return;  // a diagonal tile holds both of its triangles
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPerThread4; ++q) {
    const int e = threadIdx.x + q * kNT, r = e / kC4, c = (e % kC4) * 4;
    // C[b kPT + r][a kPT + c + k] = tile entry (c + k, r)
    const float v[4] = {ts[c * kLdsLd + r], ts[(c + 1) * kLdsLd + r], ts[(c + 2) * kLdsLd + r],
                        ts[(c + 3) * kLdsLd + r]};
    store4(dst, b * kPT + r, a * kPT + c, n, ldd, v);
  }
}

__global__ __launch_bounds__(kNT) void k_identity_packed(float* __restrict__ dst, int64_t n,
                                                         float dval, float oval) {
  int64_t a, b;
  tile_of(blockIdx.x, a, b);
  float* t = dst + (int64_t)blockIdx.x * kTileF;
  for (int q = 0; q < kPerThread; ++q) {
    const int e = threadIdx.x + q * kNT, r = e / (int)kPT, c = e % (int)kPT;
    const int64_t gi = a * kPT + r, gj = b * kPT + c;
    t[e] = (gi < n && gj < n) ? (gi == gj ? dval : oval) : 0.0f;
  }
}

__global__ __launch_bounds__(kNT) void k_take_diag_packed(float* __restrict__ C, int64_t n,
                                                          double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const int64_t blk = i / kPT, r = i % kPT;
  float* p = C + packed_tile(blk, blk) * kTileF + r * (kPT + 1);
  d[i] = (double)*p;
  *p = 0.0f;
}

// Column sums of squares of every upper tile (a, b): column c of the tile
// is part of column b kPT + c of C (slot a); for a < b, row r of the tile is
// the mirror image's column a kPT + r (slot b).  Every column of C gets one
// slot value from each block of rows.
__global__ __launch_bounds__(kNT) void k_packed_sq_part(const float* __restrict__ C,
                                                        int64_t Nap, double* __restrict__ slots) {
  __shared__ float ts[kPT * kLdsLd];
  int64_t a, b;
  tile_of(blockIdx.x, a, b);
  const fv4* t = reinterpret_cast<const fv4*>(C + (int64_t)blockIdx.x * kTileF);
  fv4 v4[kPerThread4];
#pragma unroll
  for (int q = 0; q < kPerThread4; ++q) v4[q] = t[threadIdx.x + q * kNT];
#pragma unroll
  for (int q = 0; q < kPerThread4; ++q) {
    const int e = threadIdx.x + q * kNT, r = e / kC4, c = (e % kC4) * 4;
    ts[r * kLdsLd + c] = v4[q].x;
    ts[r * kLdsLd + c + 1] = v4[q].y;
    ts[r * kLdsLd + c + 2] = v4[q].z;
    ts[r * kLdsLd + c + 3] = v4[q].w;
  }
  __syncthreads();
  // threads 0-127: column th of the tile (rows in order); 128-255: row th -
  // 128 (columns in order), the mirror's column, for off-diagonal tiles
  const int th = threadIdx.x;
  double s = 0.0;
  if (th < (int)kPT) {
    for (int r = 0; r < (int)kPT; ++r) {
      const double x = ts[r * kLdsLd + th];
      s += x * x;
    }
    slots[a * Nap + b * kPT + th] = s;
  } else if (a < b) {
    const int r = th - (int)kPT;
    for (int c = 0; c < (int)kPT; ++c) {
      const double x = ts[r * kLdsLd + c];
      s += x * x;
    }
    slots[b * Nap + a * kPT + r] = s;
  }
}

__global__ __launch_bounds__(kNT) void k_packed_sq_sum(const double* __restrict__ slots,
                                                       int64_t Nap, int64_t nT,
                                                       double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (j >= Nap) return;
  double s = 0.0;
  for (int64_t k = 0; k < nT; ++k) s += slots[k * Nap + j];
  out[j] = s;
}

unsigned tiles_of(int64_t Nap) {
  const int64_t nT = Nap / kPT;
  return (unsigned)(nT * (nT + 1) / 2);
}

}  // namespace

hipError_t launch_pack_sym(const float* src, int64_t n, int64_t lds, float* dst, int64_t Nap,
                           hipStream_t s) {
  if (Nap % kPT || n > Nap) return hipErrorInvalidValue;
  k_pack_sym<<<dim3(tiles_of(Nap)), kNT, 0, s>>>(src, n, lds, dst);
  return hipGetLastError();
}

hipError_t launch_unpack_sym(const float* src, int64_t n, int64_t Nap, float* dst, int64_t ldd,
                             hipStream_t s) {
  if (Nap % kPT || n > Nap) return hipErrorInvalidValue;
  k_unpack_sym<<<dim3(tiles_of(Nap)), kNT, 0, s>>>(src, n, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_identity_packed(float* dst, int64_t n, int64_t Nap, double dval, double oval,
                                  hipStream_t s) {
  if (Nap % kPT || n > Nap) return hipErrorInvalidValue;
  k_identity_packed<<<dim3(tiles_of(Nap)), kNT, 0, s>>>(dst, n, (float)dval, (float)oval);
  return hipGetLastError();
}

hipError_t launch_take_diag_packed(float* C, int64_t n, double* d, hipStream_t s) {
  k_take_diag_packed<<<dim3((unsigned)((n + kNT - 1) / kNT)), kNT, 0, s>>>(C, n, d);
  return hipGetLastError();
}

hipError_t launch_col_sqnorms_packed(const float* C, int64_t Nap, double* slots, double* out,
                                     hipStream_t s) {
  if (Nap % kPT) return hipErrorInvalidValue;
  k_packed_sq_part<<<dim3(tiles_of(Nap)), kNT, 0, s>>>(C, Nap, slots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_packed_sq_sum<<<dim3((unsigned)((Nap + kNT - 1) / kNT)), kNT, 0, s>>>(slots, Nap, Nap / kPT,
                                                                          out);
  return hipGetLastError();
}

}  // namespace panda
