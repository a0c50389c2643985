// Kernels of the learned warm start (not in the paper): per-edge features
// of the priors, the 16-64-64-1 MLP (inference, gradient, Adam) and the
// target / prediction maps.  The MLP runs on bf16 matrix cores with FP32
// accumulation; feature statistics and the sketch bases are FP64.
//
// MLP layout.  A wave handles 32 edges at a time with both layers computed
// transposed (Z^T = W X^T), so each lane owns one edge (lane % 32) and the
// 32 x 32 result layout of v_mfma_f32_32x32x16_bf16 puts hidden units in the
// lane's registers: unit(b, r, h) = 32 b + 8 (r / 4) + 4 h + r % 4 for output
// block b, register r and lane half h = lane / 32.  The next contraction over
// those 64 units is issued in k-steps s whose element e (of lane half h) is
// the lane's own register (b = s / 2, r = 8 (s % 2) + e); the weight operand
// is gathered in the matching unit order, so activations never leave the
// registers in the forward pass.  The weight gradients contract over edges:
// they go through a per-wave LDS transpose ([unit][edge]) into accumulators
// that live across all of the wave's edges; bias gradients come from a
// constant-one column of the same products.
#include "warm_internal.h"

namespace panda {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;           // threads per block
constexpr int kWaves = kT / 64;
constexpr int NF = kMlpFeatures;  // 16
constexpr int NH = kMlpHidden;    // 64

__device__ __forceinline__ int unit_of(int b, int r, int h) {
  return 32 * b + 8 * (r >> 2) + 4 * h + (r & 3);
}
__device__ __forceinline__ int kunit(int s, int h, int e) {
  return unit_of(s >> 1, 8 * (s & 1) + e, h);
}
__device__ __forceinline__ __bf16 bq(float x) { return (__bf16)x; }
__device__ __forceinline__ float fq(__bf16 x) { return (float)x; }

// Weights of one block in LDS: bf16 matrices, FP32 biases, bf16-rounded w3.
struct MlpShared {
  alignas(16) __bf16 W1[NH][NF];
  alignas(16) __bf16 W2[NH][NH];
  float b1[NH], b2[NH], w3[NH];
  float b3;
};

__device__ __forceinline__ void load_params(const float* __restrict__ p, MlpShared& sm) {
  for (int i = threadIdx.x; i < NH * NF; i += kT) sm.W1[i / NF][i % NF] = bq(p[kOffW1 + i]);
  for (int i = threadIdx.x; i < NH * NH; i += kT) sm.W2[i / NH][i % NH] = bq(p[kOffW2 + i]);
  for (int i = threadIdx.x; i < NH; i += kT) {
    sm.b1[i] = p[kOffB1 + i];
    sm.b2[i] = p[kOffB2 + i];
    sm.w3[i] = fq(bq(p[kOffW3 + i]));
  }
  if (threadIdx.x == 0) sm.b3 = p[kOffB3];
  __syncthreads();
}

// Weight operands of one wave (constant over its edges).
struct MlpOps {
  bf16x8 A1[2];     // W1 rows 32 mb + lane%32, features 8h..8h+7
  bf16x8 A2[2][4];  // W2 rows 32 mb + lane%32, k-step s in the unit order above
  __device__ __forceinline__ void build(const MlpShared& sm, int lane) {
    const int h = lane >> 5, m = lane & 31;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int e = 0; e < 8; ++e) A1[mb][e] = sm.W1[32 * mb + m][8 * h + e];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) A2[mb][s][e] = sm.W2[32 * mb + m][kunit(s, h, e)];
    }
  }
};

// Forward pass of the 32 edges of one wave; lane = (edge lane%32, half h).
struct MlpFwd {
  bf16x8 x;           // features 8h..8h+7 of the lane's edge (bf16)
  floatx16 z1[2];     // layer-1 pre-activations (without bias)
  bf16x8 h1[4];       // bf16 activations in k-step order
  floatx16 z2[2];     // layer-2 pre-activations (with bias after run)
  float y;
  __device__ __forceinline__ void run(const MlpShared& sm, const MlpOps& op, const float* __restrict__ F,
                                      int64_t row, bool valid, int lane) {
    const int h = lane >> 5;
    if (valid) {
      const f4 a = *reinterpret_cast<const f4*>(F + row * NF + 8 * h);
      const f4 b = *reinterpret_cast<const f4*>(F + row * NF + 8 * h + 4);
      x[0] = bq(a.x); x[1] = bq(a.y); x[2] = bq(a.z); x[3] = bq(a.w);
      x[4] = bq(b.x); x[5] = bq(b.y); x[6] = bq(b.z); x[7] = bq(b.w);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = bq(0.0f);
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      floatx16 zero;
#pragma unroll
      for (int r = 0; r < 16; ++r) zero[r] = 0.0f;
      z1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(op.A1[mb], x, zero, 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        z1[b][r] += sm.b1[unit_of(b, r, h)];
        const float v = z1[b][r] > 0.0f ? z1[b][r] : 0.0f;
        h1[2 * b + (r >> 3)][r & 7] = bq(v);
      }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) z2[mb][r] = 0.0f;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        z2[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(op.A2[mb][s], h1[s], z2[mb], 0, 0, 0);
    }
    float part = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int u = unit_of(b, r, h);
        z2[b][r] += sm.b2[u];
        part += sm.w3[u] * (z2[b][r] > 0.0f ? z2[b][r] : 0.0f);
      }
    y = part + __shfl_xor(part, 32) + sm.b3;
  }
};

// y for n feature rows.  Grid-stride over 32-edge chunks, one per wave.
__global__ __launch_bounds__(kT) void k_mlp_forward(const float* __restrict__ p,
                                                    const float* __restrict__ F, int64_t n,
                                                    float* __restrict__ y) {
  __shared__ MlpShared sm;
  load_params(p, sm);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  MlpOps op;
  op.build(sm, lane);
  const int64_t chunks = (n + 31) / 32;
  for (int64_t c = (int64_t)blockIdx.x * kWaves + wave; c < chunks;
       c += (int64_t)gridDim.x * kWaves) {
    const int64_t row = c * 32 + (lane & 31);
    MlpFwd f;
    f.run(sm, op, F, row, row < n, lane);
    if (lane < 32 && row < n) y[row] = f.y;
  }
}

// Gradient of the mean squared error over a batch of n edges (rows idx[e] of
// F and target, or e itself when idx is null).  Every wave writes its partial
// gradient (and loss sum) to its own slot; k_mlp_reduce sums the slots in a
// fixed order.  All waves of a block run the same number of chunk rounds
// (masked past the end) because the LDS transposes need block barriers.
struct GradShared {
  MlpShared w;
  alignas(16) __bf16 dz2[kWaves][NH][32];  // [unit][edge] per wave
  alignas(16) __bf16 h1[kWaves][NH][32];
  alignas(16) __bf16 dz1[kWaves][NH][32];
  alignas(16) __bf16 x[kWaves][NF][32];
};

__global__ __launch_bounds__(kT) void k_mlp_grad(const float* __restrict__ p,
                                                 const float* __restrict__ F, int64_t nrows,
                                                 const float* __restrict__ target,
                                                 const int64_t* __restrict__ idx, int64_t n,
                                                 float* __restrict__ part,
                                                 double* __restrict__ lpart) {
  __shared__ GradShared sm;
  load_params(p, sm.w);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, m = lane & 31;
  MlpOps op;
  op.build(sm.w, lane);
  // A operands of dH1^T = W2^T dZ2^T: rows = layer-1 units 32 mb + m, k-step
  // s over layer-2 units in the register order of dz2
  bf16x8 A3[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) A3[mb][s][e] = sm.w.W2[kunit(s, h, e)][32 * mb + m];
  floatx16 g2[2][3], g1[2];  // dW2 | db2 (third block: column 0), dW1 | db1 (column 16)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) g1[a][r] = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) g2[a][b][r] = 0.0f;
  }
  float gw3[2][16];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) gw3[b][r] = 0.0f;
  float gb3 = 0.0f;
  double loss = 0.0;
  bf16x8 ones, zeros;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    ones[e] = bq(1.0f);
    zeros[e] = bq(0.0f);
  }
  const float inv = 2.0f / (float)n;
  const int64_t chunks = (n + 31) / 32;
  const int64_t rounds = (chunks + (int64_t)gridDim.x * kWaves - 1) / ((int64_t)gridDim.x * kWaves);
  for (int64_t rd = 0; rd < rounds; ++rd) {
    const int64_t c = (rd * gridDim.x + blockIdx.x) * kWaves + wave;
    const int64_t e = c * 32 + m;
    int64_t row = e < n ? (idx ? idx[e] : e) : -1;
    const bool valid = row >= 0 && row < nrows;
    if (!valid) row = 0;
    MlpFwd f;
    f.run(sm.w, op, F, row, valid, lane);
    const float err = valid ? f.y - target[row] : 0.0f;
    const float dy = inv * err;
    if (h == 0) {
      loss += (double)err * (double)err;
      gb3 += dy;
    }
    // layer 2 backward (registers: lane's units of half h)
    bf16x8 dzq[4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int u = unit_of(b, r, h);
        const float h2 = f.z2[b][r] > 0.0f ? f.z2[b][r] : 0.0f;
        gw3[b][r] += dy * h2;
        const float dz = f.z2[b][r] > 0.0f ? dy * sm.w.w3[u] : 0.0f;
        dzq[2 * b + (r >> 3)][r & 7] = bq(dz);
        sm.dz2[wave][u][m] = bq(dz);
      }
    // dH1^T (64 x 32 edges) = W2^T dZ2^T, then dZ1 = dH1 * (z1 > 0)
    floatx16 dh1[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) dh1[mb][r] = 0.0f;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        dh1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3[mb][s], dzq[s], dh1[mb], 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int u = unit_of(b, r, h);
        sm.dz1[wave][u][m] = bq(f.z1[b][r] > 0.0f ? dh1[b][r] : 0.0f);
        sm.h1[wave][u][m] = f.h1[2 * b + (r >> 3)][r & 7];
      }
#pragma unroll
    for (int ee = 0; ee < 8; ++ee) sm.x[wave][8 * h + ee][m] = f.x[ee];
    __syncthreads();
    // weight gradients: contractions over the wave's 32 edges in two k-steps
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int e0 = 16 * s + 8 * h;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(&sm.dz2[wave][32 * mb + m][e0]);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(&sm.h1[wave][32 * nb + m][e0]);
          g2[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b2, g2[mb][nb], 0, 0, 0);
        }
        g2[mb][2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, m == 0 ? ones : zeros, g2[mb][2],
                                                            0, 0, 0);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&sm.dz1[wave][32 * mb + m][e0]);
        const bf16x8 b1 = m < NF ? *reinterpret_cast<const bf16x8*>(&sm.x[wave][m][e0])
                                 : (m == NF ? ones : zeros);
        g1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, g1[mb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // dw3: sum over the 32 lanes of each half (same units, different edges)
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float v = gw3[b][r];
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      gw3[b][r] = v;
    }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    gb3 += __shfl_xor(gb3, off);
    loss += __shfl_xor(loss, off);
  }
  const int64_t slot = (int64_t)blockIdx.x * kWaves + wave;
  float* out = part + slot * kMlpParams;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = unit_of(mb, r, h);  // layer-2 unit (dW2, db2) / layer-1 unit (dW1, db1)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) out[kOffW2 + row * NH + 32 * nb + m] = g2[mb][nb][r];
      if (m == 0) out[kOffB2 + row] = g2[mb][2][r];
      if (m < NF) out[kOffW1 + row * NF + m] = g1[mb][r];
      if (m == NF) out[kOffB1 + row] = g1[mb][r];
      if (m == 0) out[kOffW3 + row] = gw3[mb][r];
    }
  if (lane == 0) {
    out[kOffB3] = gb3;
    lpart[slot] = loss;
  }
}

// grad[k] = sum over slots (fixed order, FP64); loss = sum of squares / n.
__global__ __launch_bounds__(kT) void k_mlp_reduce(const float* __restrict__ part, int64_t slots,
                                                   const double* __restrict__ lpart, int64_t n,
                                                   float* __restrict__ grad,
                                                   double* __restrict__ loss) {
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k < kMlpParams) {
    double s = 0.0;
    for (int64_t i = 0; i < slots; ++i) s += (double)part[i * kMlpParams + k];
    grad[k] = (float)s;
  }
  if (k == 0 && loss) {
    double s = 0.0;
    for (int64_t i = 0; i < slots; ++i) s += lpart[i];
    *loss = s / (double)n;
  }
}

// One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1.
__global__ __launch_bounds__(kT) void k_mlp_adam(float* __restrict__ p, float* __restrict__ mo,
                                                 float* __restrict__ vo,
                                                 const float* __restrict__ g, int32_t t, float lr,
                                                 float beta1, float beta2, float eps) {
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k >= kMlpParams) return;
  const float gk = g[k];
  const float m = beta1 * mo[k] + (1.0f - beta1) * gk;
  const float v = beta2 * vo[k] + (1.0f - beta2) * gk * gk;
  mo[k] = m;
  vo[k] = v;
  const float mh = m / (1.0f - powf(beta1, (float)t));
  const float vh = v / (1.0f - powf(beta2, (float)t));
  p[k] = p[k] - lr * mh / (sqrtf(vh) + eps);
}

// out = (a - b) * scale over n entries of two strided matrices (rows x cols).
__global__ __launch_bounds__(kT) void k_ws_affine(const float* __restrict__ A, int64_t lda,
                                                  const float* __restrict__ B, int64_t ldb,
                                                  int64_t rows, int64_t cols, double scale,
                                                  double shift_scale, float* __restrict__ out,
                                                  int64_t ldo) {
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const int64_t i = e / cols, j = e % cols;
    const double a = A[i * lda + j], b = B[i * ldb + j];
    out[i * ldo + j] = (float)(shift_scale * b + scale * a);
  }
}

// ------------------------------------------------------------- features ---
constexpr int kSk = kSketch;  // 6

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Y = M X (rows x 6, FP64) for M rows x cols (FP32, leading dimension ld) and
// X cols x 6 (FP64).  A block covers 16 rows (4 per wave) and walks the
// columns in chunks of 256 staged in LDS.
constexpr int kSkRows = 16;
__global__ __launch_bounds__(kT) void k_skinny(const float* __restrict__ M, int64_t rows,
                                               int64_t cols, int64_t ld,
                                               const double* __restrict__ X,
                                               double* __restrict__ Y) {
  __shared__ double xs[kT][kSk];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kSkRows + wave * (kSkRows / kWaves);
  double acc[kSkRows / kWaves][kSk];
#pragma unroll
  for (int q = 0; q < kSkRows / kWaves; ++q)
#pragma unroll
    for (int k = 0; k < kSk; ++k) acc[q][k] = 0.0;
  for (int64_t c0 = 0; c0 < cols; c0 += kT) {
    __syncthreads();
    {
      const int64_t c = c0 + threadIdx.x;
#pragma unroll
      for (int k = 0; k < kSk; ++k) xs[threadIdx.x][k] = c < cols ? X[c * kSk + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSkRows / kWaves; ++q) {
      const int64_t r = r0 + q;
      if (r >= rows) continue;
      for (int j = lane; j < kT; j += 64) {
        const int64_t c = c0 + j;
        if (c >= cols) break;
        const double v = (double)M[r * ld + c];
#pragma unroll
        for (int k = 0; k < kSk; ++k) acc[q][k] += v * xs[j][k];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kSkRows / kWaves; ++q) {
    const int64_t r = r0 + q;
#pragma unroll
    for (int k = 0; k < kSk; ++k) {
      const double s = wave_sum(acc[q][k]);
      if (lane == 0 && r < rows) Y[r * kSk + k] = s;
    }
  }
}

// out[j][k] = sum_i M[i][j] z[i][k] (M rows x cols), one thread per column.
__global__ __launch_bounds__(kT) void k_colskinny(const float* __restrict__ M, int64_t rows,
                                                  int64_t cols, int64_t ld,
                                                  const double* __restrict__ z,
                                                  double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (j >= cols) return;
  double acc[kSk];
#pragma unroll
  for (int k = 0; k < kSk; ++k) acc[k] = 0.0;
  for (int64_t i = 0; i < rows; ++i) {
    const double v = (double)M[i * ld + j];
#pragma unroll
    for (int k = 0; k < kSk; ++k) acc[k] += v * z[i * kSk + k];
  }
#pragma unroll
  for (int k = 0; k < kSk; ++k) out[j * kSk + k] = acc[k];
}

__device__ __forceinline__ double bsum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// Cholesky QR of Y (n x 6): G = Y^T Y (one block), L L^T = G with the pivot
// rule (stop at L_kk^2 <= rel * max diag G), Q = Y L^-T on the first k
// columns, zero after.
__global__ __launch_bounds__(kT) void k_cholqr_factor(const double* __restrict__ Y, int64_t n,
                                                      double rel, double* __restrict__ Linv) {
  __shared__ double red[4];
  __shared__ double G[kSk][kSk];
  for (int a = 0; a < kSk; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += kT) s += Y[i * kSk + a] * Y[i * kSk + b];
      const double t = bsum(s, red);
      if (threadIdx.x == 0) G[a][b] = G[b][a] = t;
    }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double L[kSk][kSk] = {};
  double mx = 0.0;
  for (int a = 0; a < kSk; ++a) mx = G[a][a] > mx ? G[a][a] : mx;
  const double thr = rel * mx;
  int k = kSk;
  for (int j = 0; j < kSk; ++j) {
    double piv = G[j][j];
    for (int q = 0; q < j; ++q) piv -= L[j][q] * L[j][q];
    if (!(piv > thr)) {
      k = j;
      break;
    }
    L[j][j] = sqrt(piv);
    for (int i = j + 1; i < kSk; ++i) {
      double v = G[i][j];
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      L[i][j] = v / L[j][j];
    }
  }
  // inverse of the leading k x k block (lower triangular), forward substitution
  double Li[kSk][kSk] = {};
  for (int c = 0; c < k; ++c) {
    Li[c][c] = 1.0 / L[c][c];
    for (int i = c + 1; i < k; ++i) {
      double v = 0.0;
      for (int q = c; q < i; ++q) v -= L[i][q] * Li[q][c];
      Li[i][c] = v / L[i][i];
    }
  }
  for (int a = 0; a < kSk; ++a)
    for (int b = 0; b < kSk; ++b) Linv[a * kSk + b] = (a < k && b < k) ? Li[a][b] : 0.0;
}

// Q[i][c] = sum_m Y[i][m] Linv[c][m]  (Q = Y L^-T).
__global__ __launch_bounds__(kT) void k_cholqr_apply(const double* __restrict__ Y, int64_t n,
                                                     const double* __restrict__ Linv,
                                                     double* __restrict__ Q) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < kSk; ++c) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kSk; ++q) s += Y[i * kSk + q] * Linv[c * kSk + q];
    Q[i * kSk + c] = s;
  }
}

// X (rows x 6 FP64) from an FP32 input with leading dimension 6.
__global__ __launch_bounds__(kT) void k_widen6(const float* __restrict__ in, int64_t rows,
                                               double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < rows * kSk) out[i] = (double)in[i];
}

// Row sums (blocks [0, rows)) and column sums (threads of the remaining
// blocks) of M (FP64 results).
__global__ __launch_bounds__(kT) void k_degrees(const float* __restrict__ M, int64_t rows,
                                                int64_t cols, int64_t ld, double* __restrict__ dr,
                                                double* __restrict__ dc) {
  __shared__ double red[4];
  if ((int64_t)blockIdx.x < rows) {
    const int64_t i = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < cols; j += kT) s += (double)M[i * ld + j];
    const double t = bsum(s, red);
    if (threadIdx.x == 0) dr[i] = t;
    return;
  }
  const int64_t j = ((int64_t)blockIdx.x - rows) * kT + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < rows; ++i) s += (double)M[i * ld + j];
  dc[j] = s;
}

// Population mean and variance (two passes, FP64) of column `col` of an
// n x stride FP64 array; one block per vector.
struct VecRef {
  const double* v;
  int64_t n, stride;
};
__global__ __launch_bounds__(kT) void k_vec_moments(const VecRef* __restrict__ vecs,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  const VecRef r = vecs[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < r.n; i += kT) s += r.v[i * r.stride];
  const double mean = bsum(s, red) / (double)r.n;
  double q = 0.0, q2 = 0.0;
  for (int64_t i = threadIdx.x; i < r.n; i += kT) {
    const double d = r.v[i * r.stride] - mean;
    q += d * d;
    q2 += r.v[i * r.stride] * r.v[i * r.stride];
  }
  const double var = bsum(q, red) / (double)r.n;
  const double msq = bsum(q2, red) / (double)r.n;
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x + 0] = mean;
    out[3 * blockIdx.x + 1] = var;
    out[3 * blockIdx.x + 2] = msq;
  }
}

// S = (R0 + A0) / 2 in place of A0.
__global__ __launch_bounds__(kT) void k_half_sum(const float* __restrict__ R, float* __restrict__ A,
                                                 int64_t rows, int64_t cols, int64_t ld) {
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const int64_t o = (e / cols) * ld + e % cols;
    A[o] = (float)(0.5 * ((double)R[o] + (double)A[o]));
  }
}

// The 16 features of every edge, z-scored with the statistics st[f] =
// (mean, 1 / std or 0 for a constant feature).
__global__ __launch_bounds__(kT) void k_ws_assemble(
    int64_t Ne, int64_t Na, const float* __restrict__ W0, const float* __restrict__ S, int64_t ld,
    const double* __restrict__ dr, const double* __restrict__ dc, const double* __restrict__ a,
    const double* __restrict__ b, const double* __restrict__ c, const double* __restrict__ d,
    const double2* __restrict__ st, float* __restrict__ F) {
  const int64_t n = Ne * Na;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const int64_t i = e / Na, j = e % Na;
    double g[NF];
    g[0] = W0[i * ld + j];
    g[1] = dr[i];
    g[2] = dc[j];
#pragma unroll
    for (int k = 0; k < kSk; ++k) {
      g[3 + k] = a[i * kSk + k] * b[j * kSk + k];
      g[9 + k] = c[i * kSk + k] * d[j * kSk + k];
    }
    g[15] = S[i * ld + j];
    float o[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) o[f] = (float)((g[f] - st[f].x) * st[f].y);
    f4* dst = reinterpret_cast<f4*>(F + e * NF);
#pragma unroll
    for (int q = 0; q < NF / 4; ++q) dst[q] = f4{o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]};
  }
}

// Feature statistics from the vector moments (m = {mean, var, mean square}
// for dr, dc, a_0..5, b_0..5, c_0..5, d_0..5) and the two full reductions
// zW = (mean, std) of W0 and zS of S.  A product feature u_i v_j over all
// edges has mean m_u m_v and second moment E[u^2] E[v^2].
__global__ void k_ws_stats(const double* __restrict__ m, const double* __restrict__ zW,
                           const double* __restrict__ zS, double2* __restrict__ st) {
  if (threadIdx.x != 0) return;
  auto put = [&](int f, double mean, double var, double scale2) {
    // var below rounding of the mean: a constant feature
    const double sd = var > 1e-24 * scale2 ? sqrt(var) : 0.0;
    st[f] = make_double2(mean, sd > 0.0 ? 1.0 / sd : 0.0);
  };
  put(0, zW[0], zW[1] * zW[1], zW[0] * zW[0] + 1e-300);
  put(1, m[0], m[1], m[2] + 1e-300);
  put(2, m[3], m[4], m[5] + 1e-300);
  for (int k = 0; k < kSk; ++k) {
    const double* A = m + 3 * (2 + k);
    const double* B = m + 3 * (8 + k);
    const double* C = m + 3 * (14 + k);
    const double* D = m + 3 * (20 + k);
    const double mp = A[0] * B[0], mq = C[0] * D[0];
    const double sp = A[2] * B[2], sq = C[2] * D[2];
    put(3 + k, mp, sp - mp * mp, sp + 1e-300);
    put(9 + k, mq, sq - mq * mq, sq + 1e-300);
  }
  put(15, zS[0], zS[1] * zS[1], zS[0] * zS[0] + 1e-300);
}

unsigned grid_cap(int64_t n, int64_t cap) {
  int64_t b = (n + kT - 1) / kT;
  if (b > cap) b = cap;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ------------------------------------------------------------ launchers --

int64_t mlp_grad_slots(int64_t n) {
  const int64_t chunks = (n + 31) / 32;
  int64_t blocks = (chunks + kWaves - 1) / kWaves;
  if (blocks > kMlpGradBlocks) blocks = kMlpGradBlocks;
  if (blocks < 1) blocks = 1;
  return blocks * kWaves;
}

hipError_t launch_mlp_forward(const float* p, const float* F, int64_t n, float* y, hipStream_t s) {
  const int64_t chunks = (n + 31) / 32;
  int64_t blocks = (chunks + kWaves - 1) / kWaves;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_mlp_forward<<<dim3((unsigned)blocks), dim3(kT), 0, s>>>(p, F, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* p, const float* F, int64_t nrows, const float* target,
                           const int64_t* idx, int64_t n, float* part, double* lpart, float* grad,
                           double* loss, hipStream_t s) {
  const int64_t slots = mlp_grad_slots(n);
  k_mlp_grad<<<dim3((unsigned)(slots / kWaves)), dim3(kT), 0, s>>>(p, F, nrows, target, idx, n,
                                                                  part, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_mlp_reduce<<<dim3((unsigned)((kMlpParams + kT - 1) / kT)), dim3(kT), 0, s>>>(
      part, slots, lpart, n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* g, int32_t t, float lr,
                           float beta1, float beta2, float eps, hipStream_t s) {
  k_mlp_adam<<<dim3((unsigned)((kMlpParams + kT - 1) / kT)), dim3(kT), 0, s>>>(
      p, m, v, g, t, lr, beta1, beta2, eps);
  return hipGetLastError();
}

hipError_t launch_ws_affine(const float* A, int64_t lda, const float* B, int64_t ldb,
                            int64_t rows, int64_t cols, double scale, double shift_scale,
                            float* out, int64_t ldo, hipStream_t s) {
  k_ws_affine<<<grid_cap(rows * cols, 8192), dim3(kT), 0, s>>>(A, lda, B, ldb, rows, cols, scale,
                                                               shift_scale, out, ldo);
  return hipGetLastError();
}

hipError_t launch_ws_sketch(const float* M, int64_t n, int64_t ld, const double* X, double* tmp,
                            double* Y, hipStream_t s) {
  const unsigned nb = (unsigned)((n + kSkRows - 1) / kSkRows);
  k_skinny<<<dim3(nb), dim3(kT), 0, s>>>(M, n, n, ld, X, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_skinny<<<dim3(nb), dim3(kT), 0, s>>>(M, n, n, ld, tmp, Y);
  return hipGetLastError();
}

hipError_t launch_skinny(const float* M, int64_t rows, int64_t cols, int64_t ld, const double* X,
                         double* Y, hipStream_t s) {
  k_skinny<<<dim3((unsigned)((rows + kSkRows - 1) / kSkRows)), dim3(kT), 0, s>>>(M, rows, cols,
                                                                                 ld, X, Y);
  return hipGetLastError();
}

hipError_t launch_colskinny(const float* M, int64_t rows, int64_t cols, int64_t ld,
                            const double* z, double* out, hipStream_t s) {
  k_colskinny<<<dim3((unsigned)((cols + kT - 1) / kT)), dim3(kT), 0, s>>>(M, rows, cols, ld, z,
                                                                          out);
  return hipGetLastError();
}

hipError_t launch_cholqr(const double* Y, int64_t n, double rel, double* Linv, double* Q,
                         hipStream_t s) {
  k_cholqr_factor<<<1, kT, 0, s>>>(Y, n, rel, Linv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_cholqr_apply<<<dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s>>>(Y, n, Linv, Q);
  return hipGetLastError();
}

hipError_t launch_widen6(const float* in, int64_t rows, double* out, hipStream_t s) {
  k_widen6<<<dim3((unsigned)((rows * kSk + kT - 1) / kT)), dim3(kT), 0, s>>>(in, rows, out);
  return hipGetLastError();
}

hipError_t launch_degrees(const float* M, int64_t rows, int64_t cols, int64_t ld, double* dr,
                          double* dc, hipStream_t s) {
  const unsigned nb = (unsigned)(rows + (cols + kT - 1) / kT);
  k_degrees<<<dim3(nb), dim3(kT), 0, s>>>(M, rows, cols, ld, dr, dc);
  return hipGetLastError();
}

hipError_t launch_vec_moments(const VecRefHost* vecs, int count, double* out, hipStream_t s) {
  static_assert(sizeof(VecRefHost) == sizeof(VecRef), "same layout");
  k_vec_moments<<<dim3((unsigned)count), dim3(kT), 0, s>>>(reinterpret_cast<const VecRef*>(vecs),
                                                           out);
  return hipGetLastError();
}

hipError_t launch_half_sum(const float* R, float* A, int64_t rows, int64_t cols, int64_t ld,
                           hipStream_t s) {
  k_half_sum<<<grid_cap(rows * cols, 8192), dim3(kT), 0, s>>>(R, A, rows, cols, ld);
  return hipGetLastError();
}

hipError_t launch_ws_stats(const double* m, const double* zW, const double* zS, double2* st,
                           hipStream_t s) {
  k_ws_stats<<<1, 64, 0, s>>>(m, zW, zS, st);
  return hipGetLastError();
}

hipError_t launch_ws_assemble(int64_t Ne, int64_t Na, const float* W0, const float* S, int64_t ld,
                              const double* dr, const double* dc, const double* a,
                              const double* b, const double* c, const double* d,
                              const double2* st, float* F, hipStream_t s) {
  k_ws_assemble<<<grid_cap(Ne * Na, 16384), dim3(kT), 0, s>>>(Ne, Na, W0, S, ld, dr, dc, a, b, c,
                                                              d, st, F);
  return hipGetLastError();
}

}  // namespace panda
