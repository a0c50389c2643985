// Node-label randomisation as a permutation null (the option of the paper's
// C implementation that relabels nodes on input, Sec. III): each null
// instance relabels the genes of the co-expression prior C and/or the TFs of
// the interaction prior P with its own permutation, keeps the motif prior W,
// and runs the message passing to convergence; the converged W of all
// instances are folded into a per-edge mean and standard deviation (FP64,
// Welford's update), against which the real network's edges are z-scored.
#include <math.h>

#include <algorithm>
#include <vector>

#include "host_internal.h"

using namespace panda;

namespace {

constexpr int kNT = 256;

// out[i][j] = M[perm[i]][perm[j]]: one output row per block (grid-stride),
// written along the row; the reads gather from one input row, which stays in
// cache while the block walks it.  perm holds a permutation of 0 .. n-1.
__global__ __launch_bounds__(kNT) void k_permute_sym(const float* __restrict__ M, int64_t n,
                                                     int64_t ldm, const int32_t* __restrict__ perm,
                                                     float* __restrict__ out, int64_t ldo) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const float* src = M + (int64_t)perm[i] * ldm;
    float* dst = out + i * ldo;
    for (int64_t j = threadIdx.x; j < n; j += kNT) dst[j] = src[perm[j]];
  }
}

// The same with the source row staged in LDS first (read once, along the
// row), so the gather runs on LDS: for rows of up to kRowLds entries.
constexpr int kPermNT = 512;
constexpr int64_t kRowLds = 160 * 1024 / 4;
__global__ __launch_bounds__(kPermNT) void k_permute_sym_lds(const float* __restrict__ M,
                                                             int64_t n, int64_t ldm,
                                                             const int32_t* __restrict__ perm,
                                                             float* __restrict__ out,
                                                             int64_t ldo) {
  extern __shared__ float row[];
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const float* src = M + (int64_t)perm[i] * ldm;
    __syncthreads();  // the previous row's gathers are done
    for (int64_t j = threadIdx.x; j < n; j += kPermNT) row[j] = src[j];
    __syncthreads();
    float* dst = out + i * ldo;
    for (int64_t j = threadIdx.x; j < n; j += kPermNT)
      __builtin_nontemporal_store(row[perm[j]], dst + j);  // not read again here
  }
}

// Welford's update of the running mean and sum of squared deviations with
// sample number k1 = k + 1 (mean and m2 start at zero).
__global__ __launch_bounds__(kNT) void k_null_accum(const float* __restrict__ W, int64_t total,
                                                    double* __restrict__ mean,
                                                    double* __restrict__ m2, double k1) {
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kNT) {
    const double x = W[e], mu = mean[e], d = x - mu;
    const double nmu = mu + d / k1;
    m2[e] += d * (x - nmu);
    mean[e] = nmu;
  }
}

__global__ __launch_bounds__(kNT) void k_null_finish(const double* __restrict__ mean,
                                                     const double* __restrict__ m2, int64_t total,
                                                     double K, float* __restrict__ mean_out,
                                                     float* __restrict__ sd_out) {
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kNT) {
    mean_out[e] = (float)mean[e];
    sd_out[e] = (float)sqrt(m2[e] / K);
  }
}

// z = (W - mean) / sd per edge; 0 where the null has no spread.
__global__ __launch_bounds__(kNT) void k_null_zscore(const float* __restrict__ W,
                                                     const float* __restrict__ mean,
                                                     const float* __restrict__ sd, int64_t total,
                                                     float* __restrict__ z) {
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kNT) {
    const double s = sd[e];
    z[e] = s > 0.0 ? (float)(((double)W[e] - (double)mean[e]) / s) : 0.0f;
  }
}

unsigned grid_for(int64_t total) {
  const int64_t b = (total + kNT - 1) / kNT;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_permute_sym(const float* M, int64_t n, int64_t ldm, const int32_t* perm,
                              float* out, int64_t ldo, hipStream_t s) {
  const unsigned g = (unsigned)(n < 16384 ? n : 16384);
  if (n <= kRowLds) {
    // set on every call: the attribute belongs to the current device
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_permute_sym_lds),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(kRowLds * 4));
    if (e != hipSuccess) return e;
    k_permute_sym_lds<<<dim3(g), dim3(kPermNT), (size_t)n * 4, s>>>(M, n, ldm, perm, out, ldo);
  } else {
    k_permute_sym<<<dim3(g), dim3(kNT), 0, s>>>(M, n, ldm, perm, out, ldo);
  }
  return hipGetLastError();
}

// Every row of perm (count rows of n entries, device memory) a permutation of
// 0 .. n-1.  Synchronises the stream.
panda_status check_perms(const int32_t* perm, int64_t count, int64_t n, hipStream_t s,
                         const char* what) {
  std::vector<int32_t> h((size_t)(count * n));
  HIP_TRY(hipMemcpyAsync(h.data(), perm, h.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<char> seen((size_t)n);
  for (int64_t k = 0; k < count; ++k) {
    std::fill(seen.begin(), seen.end(), 0);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t v = h[(size_t)(k * n + i)];
      if (v < 0 || v >= n || seen[(size_t)v]) return fail(PANDA_ERR_ARG, "null: %s is not a permutation", what);
      seen[(size_t)v] = 1;
    }
  }
  return PANDA_OK;
}

struct NullLayout {
  char* ctx;
  float *P, *C, *W;
  double *mean, *m2;
};

size_t null_layout(int64_t Ne, int64_t Na, const panda_options* opt, char* base, NullLayout* L) {
  Carver cv{base};
  NullLayout l;
  l.ctx = cv.take<char>(panda_workspace_bytes(Ne, Na, opt));
  l.P = cv.take<float>((size_t)(Ne * Ne));
  l.C = cv.take<float>((size_t)(Na * Na));
  l.W = cv.take<float>((size_t)(Ne * Na));
  l.mean = cv.take<double>((size_t)(Ne * Na));
  l.m2 = cv.take<double>((size_t)(Ne * Na));
  if (L) *L = l;
  return cv.off;
}

}  // namespace

extern "C" {

panda_status panda_permute_sym(const float* M, int64_t n, int64_t ldm, const int32_t* perm,
                               float* out, int64_t ldo, hipStream_t s) {
  if (!M || !perm || !out || n < 1 || n > (1 << 20) || ldm < n || ldo < n)
    return fail(PANDA_ERR_ARG, "permute_sym: bad arguments%s");
  PANDA_TRY(check_perms(perm, 1, n, s, "perm"));
  HIP_TRY(launch_permute_sym(M, n, ldm, perm, out, ldo, s));
  return PANDA_OK;
}

size_t panda_null_workspace_bytes(int64_t Ne, int64_t Na, const panda_options* opt) {
  if (!dims_ok(Ne, Na)) return 0;
  return null_layout(Ne, Na, opt, nullptr, nullptr);
}

panda_status panda_null(const float* W0, const float* P0, const float* C0, int64_t Ne,
                        int64_t Na, int32_t K, const int32_t* gene_perm, const int32_t* tf_perm,
                        const panda_options* opt, void* workspace, size_t ws_bytes, float* mean,
                        float* sd, int32_t* iters, hipStream_t s) {
  if (!W0 || !mean || !sd || K < 1 || !dims_ok(Ne, Na))
    return fail(PANDA_ERR_ARG, "null: bad arguments%s");
  panda_options o;
  if (opt)
    o = *opt;
  else
    panda_default_options(&o);
  PANDA_TRY(check_options(o));
  if (!workspace || ws_bytes < panda_null_workspace_bytes(Ne, Na, &o) ||
      reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(PANDA_ERR_WORKSPACE, "null: workspace too small or misaligned%s");
  if (gene_perm) PANDA_TRY(check_perms(gene_perm, K, Na, s, "gene_perm"));
  if (tf_perm) PANDA_TRY(check_perms(tf_perm, K, Ne, s, "tf_perm"));
  NullLayout L;
  null_layout(Ne, Na, &o, static_cast<char*>(workspace), &L);
  const int64_t total = Ne * Na;
  HIP_TRY(hipMemsetAsync(L.mean, 0, (size_t)total * 8, s));
  HIP_TRY(hipMemsetAsync(L.m2, 0, (size_t)total * 8, s));
  const size_t ctx_bytes = panda_workspace_bytes(Ne, Na, &o);
  panda_status result = PANDA_OK;
  for (int32_t k = 0; k < K; ++k) {
    // relabelled priors of instance k (an identity prior stays the identity)
    const float* Pk = P0;
    const float* Ck = C0;
    if (tf_perm && P0) {
      HIP_TRY(launch_permute_sym(P0, Ne, Ne, tf_perm + (int64_t)k * Ne, L.P, Ne, s));
      Pk = L.P;
    }
    if (gene_perm && C0) {
      HIP_TRY(launch_permute_sym(C0, Na, Na, gene_perm + (int64_t)k * Na, L.C, Na, s));
      Ck = L.C;
    }
    panda_ctx* c = nullptr;
    PANDA_TRY(panda_ctx_create(Ne, Na, &o, L.ctx, ctx_bytes, s, &c));
    panda_status st = panda_ctx_load(c, W0, Pk, Ck, 0);
    if (st == PANDA_OK) st = run_loaded(c);
    int32_t t = 0;
    if (st == PANDA_OK) st = panda_ctx_store(c, L.W, nullptr, nullptr, nullptr, &t);
    const bool active = st == PANDA_OK && c->host->active;
    panda_ctx_destroy(c);
    if (st != PANDA_OK) return st;
    if (active) result = PANDA_NOT_CONVERGED;
    if (iters) iters[k] = t;
    k_null_accum<<<dim3(grid_for(total)), dim3(kNT), 0, s>>>(L.W, total, L.mean, L.m2,
                                                              (double)(k + 1));
    HIP_TRY(hipGetLastError());
  }
  k_null_finish<<<dim3(grid_for(total)), dim3(kNT), 0, s>>>(L.mean, L.m2, total, (double)K, mean,
                                                             sd);
  HIP_TRY(hipGetLastError());
  return result;
}

panda_status panda_null_zscore(const float* W, const float* mean, const float* sd, int64_t Ne,
                               int64_t Na, float* z, hipStream_t s) {
  if (!W || !mean || !sd || !z || !dims_ok(Ne, Na))
    return fail(PANDA_ERR_ARG, "null_zscore: bad arguments%s");
  const int64_t total = Ne * Na;
  k_null_zscore<<<dim3(grid_for(total)), dim3(kNT), 0, s>>>(W, mean, sd, total, z);
  HIP_TRY(hipGetLastError());
  return PANDA_OK;
}

}  // extern "C"
