// Internal declarations of the learned warm start (features, MLP kernels).
#pragma once

#include "panda_internal.h"

namespace panda {

constexpr int kMlpFeatures = 16;
constexpr int kMlpHidden = 64;
constexpr int kSketch = 6;  // sketch columns per side
// packed parameters: W1[64][16], b1[64], W2[64][64] (out, in), b2[64], w3[64], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpFeatures;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden;
constexpr int kMlpParams = kOffB3 + 1;  // 5313
constexpr int64_t kMlpGradBlocks = 512;  // blocks of the gradient kernel (4 slots each)
constexpr double kSketchPivotRel = 1e-10;

// Per-wave partial gradients of a batch of n edges.
int64_t mlp_grad_slots(int64_t n);

hipError_t launch_mlp_forward(const float* p, const float* F, int64_t n, float* y, hipStream_t s);
// part: mlp_grad_slots(n) * kMlpParams floats, lpart: mlp_grad_slots(n) doubles.
// Rows idx[e] outside [0, nrows) count as padding (no contribution).
hipError_t launch_mlp_grad(const float* p, const float* F, int64_t nrows, const float* target,
                           const int64_t* idx, int64_t n, float* part, double* lpart, float* grad,
                           double* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* g, int32_t t, float lr,
                           float beta1, float beta2, float eps, hipStream_t s);
// out = shift_scale * B + scale * A, element-wise over rows x cols.
hipError_t launch_ws_affine(const float* A, int64_t lda, const float* B, int64_t ldb,
                            int64_t rows, int64_t cols, double scale, double shift_scale,
                            float* out, int64_t ldo, hipStream_t s);

// Feature building blocks (all FP64 outputs; 6-column arrays row-major).
hipError_t launch_ws_sketch(const float* M, int64_t n, int64_t ld, const double* X, double* tmp,
                            double* Y, hipStream_t s);  // Y = M (M X), M n x n
hipError_t launch_skinny(const float* M, int64_t rows, int64_t cols, int64_t ld, const double* X,
                         double* Y, hipStream_t s);     // Y = M X
hipError_t launch_colskinny(const float* M, int64_t rows, int64_t cols, int64_t ld,
                            const double* z, double* out, hipStream_t s);  // out = M^T z
hipError_t launch_cholqr(const double* Y, int64_t n, double rel, double* Linv, double* Q,
                         hipStream_t s);
hipError_t launch_widen6(const float* in, int64_t rows, double* out, hipStream_t s);
hipError_t launch_degrees(const float* M, int64_t rows, int64_t cols, int64_t ld, double* dr,
                          double* dc, hipStream_t s);
struct VecRefHost {
  const double* v;
  int64_t n, stride;
};
// out[3 k + {0, 1, 2}] = mean, variance, mean square of vector k (device table).
hipError_t launch_vec_moments(const VecRefHost* vecs, int count, double* out, hipStream_t s);
hipError_t launch_half_sum(const float* R, float* A, int64_t rows, int64_t cols, int64_t ld,
                           hipStream_t s);
hipError_t launch_ws_stats(const double* m, const double* zW, const double* zS, double2* st,
                           hipStream_t s);
hipError_t launch_ws_assemble(int64_t Ne, int64_t Na, const float* W0, const float* S, int64_t ld,
                              const double* dr, const double* dc, const double* a,
                              const double* b, const double* c, const double* d,
                              const double2* st, float* F, hipStream_t s);

}  // namespace panda
