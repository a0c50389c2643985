// Host side of the learned warm start: feature construction from a loaded
// context, the MLP entry points and the warm state of a context.  See
// include/panda.h for the definitions.
#include <math.h>

#include <vector>

#include "host_internal.h"
#include "warm_internal.h"

using namespace panda;

namespace {

struct FeatLayout {
  float* S;  // Nep x Nap: A0, then S = (R0 + A0) / 2
  double *dr, *dc, *omP, *omC, *tmpP, *yP, *a, *zP, *b, *tmpC, *yC, *d, *zC, *c;
  double *LinvP, *LinvC, *mom, *zsW, *zsS, *zsD;
  VecRefHost* vref;
  double2* st;
};

constexpr int kNumVec = 2 + 4 * kSketch;  // dr, dc, a_k, b_k, c_k, d_k

size_t feat_layout(int64_t Ne, int64_t Na, char* base, FeatLayout* L) {
  const int64_t Nep = round_up(Ne, kPadE), Nap = round_up(Na, kPadA);
  Carver cv{base};
  FeatLayout l;
  l.S = cv.take<float>((size_t)Nep * Nap);
  l.dr = cv.take<double>((size_t)Ne);
  l.dc = cv.take<double>((size_t)Na);
  double** sixNe[] = {&l.omP, &l.tmpP, &l.yP, &l.a, &l.zP, &l.c};
  for (double** q : sixNe) *q = cv.take<double>((size_t)Ne * kSketch);
  double** sixNa[] = {&l.omC, &l.tmpC, &l.yC, &l.d, &l.zC, &l.b};
  for (double** q : sixNa) *q = cv.take<double>((size_t)Na * kSketch);
  l.LinvP = cv.take<double>(kSketch * kSketch);
  l.LinvC = cv.take<double>(kSketch * kSketch);
  l.mom = cv.take<double>(3 * kNumVec);
  l.zsW = cv.take<double>(kZsScratch);
  l.zsS = cv.take<double>(kZsScratch);
  l.zsD = cv.take<double>(kZsScratch);
  l.vref = cv.take<VecRefHost>(kNumVec);
  l.st = cv.take<double2>(kMlpFeatures);
  if (L) *L = l;
  return cv.off;
}

bool aligned(const void* p) { return p && reinterpret_cast<uintptr_t>(p) % kAlign == 0; }

}  // namespace

extern "C" {

size_t panda_ws_features_workspace_bytes(int64_t Ne, int64_t Na) {
  if (!dims_ok(Ne, Na)) return 0;
  return feat_layout(Ne, Na, nullptr, nullptr);
}

panda_status panda_ws_features(panda_ctx* c, const float* omegaP, const float* omegaC, float* F,
                               double* tau, void* workspace, size_t ws_bytes) {
  if (!c || !c->loaded || !omegaP || !omegaC || !F)
    return fail(PANDA_ERR_ARG, "ws_features: bad arguments%s");
  const int64_t Ne = c->Ne, Na = c->Na, Nep = c->Nep, Nap = c->Nap;
  if (!aligned(workspace) || ws_bytes < feat_layout(Ne, Na, nullptr, nullptr))
    return fail(PANDA_ERR_WORKSPACE, "ws_features: workspace too small or misaligned%s");
  if (!c->skpart) return fail(PANDA_ERR_ARG, "ws_features: context of a batch%s");
  if (c->packed) return fail(PANDA_ERR_ARG, "ws_features: needs a context with C stored whole (packed_c = 0)%s");
  FeatLayout L;
  feat_layout(Ne, Na, static_cast<char*>(workspace), &L);
  hipStream_t s = c->stream;
  c->r_next = false;  // R serves as scratch below
  const float* W0 = c->W[c->executed & 1];
  // one-step similarities R0 = T(P0, W0) (into R) and A0 = T(W0, C0) (into S)
  HIP_TRY(launch_resp(c->P, Nep, c->dP, W0, Nap, Nep, Nap, Ne, Na, c->nP, c->nWc, c->R,
                      c->skpart, nullptr, s));
  HIP_TRY(launch_tanimoto_store(W0, Nap, c->C, Nap, Nep, Nap, Nap, Ne, Na, c->nWr, c->nC, L.S,
                                Nap, c->skpart, nullptr, s, c->dC));
  HIP_TRY(launch_half_sum(c->R, L.S, Ne, Na, Nap, s));
  // statistics of W0, S and S - W0 (tau)
  HIP_TRY(launch_zscore_stats(W0, Ne, Na, Nap, L.zsW, s));
  HIP_TRY(launch_zscore_stats(L.S, Ne, Na, Nap, L.zsS, s));
  HIP_TRY(launch_ws_affine(L.S, Nap, W0, Nap, Ne, Na, 1.0, -1.0, c->R, Nap, s));
  HIP_TRY(launch_zscore_stats(c->R, Ne, Na, Nap, L.zsD, s));
  // degrees and the two sketch bases
  HIP_TRY(launch_degrees(W0, Ne, Na, Nap, L.dr, L.dc, s));
  // the sketches use the whole P0 and C0: their diagonals go back in for now
  // (the vectors hold the FP32 values taken out at load, so this is exact)
  HIP_TRY(launch_put_diag(c->P, Ne, Nep, c->dP, s));
  HIP_TRY(launch_put_diag(c->C, Na, Nap, c->dC, s));
  HIP_TRY(launch_widen6(omegaP, Ne, L.omP, s));
  HIP_TRY(launch_widen6(omegaC, Na, L.omC, s));
  HIP_TRY(launch_ws_sketch(c->P, Ne, Nep, L.omP, L.tmpP, L.yP, s));
  HIP_TRY(launch_cholqr(L.yP, Ne, kSketchPivotRel, L.LinvP, L.a, s));
  HIP_TRY(launch_skinny(c->P, Ne, Ne, Nep, L.a, L.zP, s));          // P0 a
  HIP_TRY(launch_colskinny(W0, Ne, Na, Nap, L.zP, L.b, s));         // b = W0^T P0 a
  HIP_TRY(launch_ws_sketch(c->C, Na, Nap, L.omC, L.tmpC, L.yC, s));
  HIP_TRY(launch_cholqr(L.yC, Na, kSketchPivotRel, L.LinvC, L.d, s));
  HIP_TRY(launch_skinny(c->C, Na, Na, Nap, L.d, L.zC, s));          // C0 d
  HIP_TRY(launch_skinny(W0, Ne, Na, Nap, L.zC, L.c, s));            // c = W0 C0 d
  HIP_TRY(launch_take_diag(c->P, Ne, Nep, c->dP, s));
  HIP_TRY(launch_take_diag(c->C, Na, Nap, c->dC, s));
  // moments of the 26 vectors, then the statistics of the 16 features
  VecRefHost refs[kNumVec];
  refs[0] = VecRefHost{L.dr, Ne, 1};
  refs[1] = VecRefHost{L.dc, Na, 1};
  for (int k = 0; k < kSketch; ++k) {
    refs[2 + k] = VecRefHost{L.a + k, Ne, kSketch};
    refs[8 + k] = VecRefHost{L.b + k, Na, kSketch};
    refs[14 + k] = VecRefHost{L.c + k, Ne, kSketch};
    refs[20 + k] = VecRefHost{L.d + k, Na, kSketch};
  }
  HIP_TRY(hipMemcpyAsync(L.vref, refs, sizeof refs, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_vec_moments(L.vref, kNumVec, L.mom, s));
  HIP_TRY(launch_ws_stats(L.mom, L.zsW + kZsBlocks, L.zsS + kZsBlocks, L.st, s));
  HIP_TRY(launch_ws_assemble(Ne, Na, W0, L.S, Nap, L.dr, L.dc, L.a, L.b, L.c, L.d, L.st, F, s));
  double sd[2];
  HIP_TRY(hipMemcpyAsync(sd, L.zsD + kZsBlocks, sizeof sd, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));  // also keeps refs alive until copied
  if (tau) *tau = sd[1];
  return PANDA_OK;
}

panda_status panda_mlp_forward(const float* params, const float* F, int64_t n, float* y,
                               hipStream_t s) {
  if (!params || !F || !y || n < 1) return fail(PANDA_ERR_ARG, "mlp_forward: bad arguments%s");
  HIP_TRY(launch_mlp_forward(params, F, n, y, s));
  return PANDA_OK;
}

size_t panda_mlp_grad_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  const int64_t slots = mlp_grad_slots(n);
  return align_up((size_t)slots * kMlpParams * sizeof(float)) +
         align_up((size_t)slots * sizeof(double)) + align_up(sizeof(double));
}

panda_status panda_mlp_grad(const float* params, const float* F, int64_t nrows,
                            const float* target, const int64_t* idx, int64_t n, float* grad,
                            double* loss, void* workspace, size_t ws_bytes, hipStream_t s) {
  if (!params || !F || !target || !grad || n < 1 || nrows < 1 || (!idx && n > nrows))
    return fail(PANDA_ERR_ARG, "mlp_grad: bad arguments%s");
  if (!aligned(workspace) || ws_bytes < panda_mlp_grad_workspace_bytes(n))
    return fail(PANDA_ERR_WORKSPACE, "mlp_grad: workspace too small or misaligned%s");
  const int64_t slots = mlp_grad_slots(n);
  Carver cv{static_cast<char*>(workspace)};
  float* part = cv.take<float>((size_t)slots * kMlpParams);
  double* lpart = cv.take<double>((size_t)slots);
  HIP_TRY(launch_mlp_grad(params, F, nrows, target, idx, n, part, lpart, grad, loss, s));
  return PANDA_OK;
}

panda_status panda_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                            float lr, float beta1, float beta2, float eps, hipStream_t s) {
  if (!params || !m || !v || !grad || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f) ||
      !(beta1 < 1.0f) || !(beta2 >= 0.0f) || !(beta2 < 1.0f) || !(eps >= 0.0f))
    return fail(PANDA_ERR_ARG, "mlp_adam: bad arguments%s");
  HIP_TRY(launch_mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps, s));
  return PANDA_OK;
}

panda_status panda_mlp_train_step(float* params, float* m, float* v, int32_t step, float lr,
                                  const float* F, int64_t nrows, const float* target,
                                  const int64_t* idx, int64_t n, float* grad, double* loss,
                                  void* workspace, size_t ws_bytes, hipStream_t s) {
  PANDA_TRY(panda_mlp_grad(params, F, nrows, target, idx, n, grad, loss, workspace, ws_bytes, s));
  return panda_mlp_adam(params, m, v, grad, step, lr, 0.9f, 0.999f, 1e-8f, s);
}

panda_status panda_ws_target(const float* W0, const float* Wstar, int64_t rows, int64_t cols,
                             double tau, float* out, hipStream_t s) {
  if (!W0 || !Wstar || !out || rows < 1 || cols < 1 || !(tau > 0.0) || !isfinite(tau))
    return fail(PANDA_ERR_ARG, "ws_target: bad arguments%s");
  HIP_TRY(launch_ws_affine(Wstar, cols, W0, cols, rows, cols, 1.0 / tau, -1.0 / tau, out, cols, s));
  return PANDA_OK;
}

panda_status panda_ws_predict(const float* W0, const float* y, int64_t rows, int64_t cols,
                              double tau, float* Wpred, hipStream_t s) {
  if (!W0 || !y || !Wpred || rows < 1 || cols < 1 || !isfinite(tau))
    return fail(PANDA_ERR_ARG, "ws_predict: bad arguments%s");
  HIP_TRY(launch_ws_affine(y, cols, W0, cols, rows, cols, tau, 1.0, Wpred, cols, s));
  return PANDA_OK;
}

panda_status panda_ws_init(panda_ctx* c, const float* Wpred, int32_t t0) {
  if (!c || !c->loaded || !Wpred || t0 < 0) return fail(PANDA_ERR_ARG, "ws_init: bad arguments%s");
  if (!c->skpart) return fail(PANDA_ERR_ARG, "ws_init: context of a batch%s");
  hipStream_t s = c->stream;
  const int64_t Ne = c->Ne, Na = c->Na, Nep = c->Nep, Nap = c->Nap;
  // the predicted W becomes the current W (buffer 0, padding zero)
  HIP_TRY(hipMemsetAsync(c->W[0], 0, (size_t)Nep * Nap * 4, s));
  HIP_TRY(hipMemcpy2DAsync(c->W[0], (size_t)Nap * 4, Wpred, (size_t)Na * 4, (size_t)Na * 4,
                           (size_t)Ne, hipMemcpyDeviceToDevice, s));
  float* W = c->W[0];
  HIP_TRY(launch_w_norms(W, Ne, Na, Nap, Nep, c->nWr, c->nWc, c->colscr, c->Wh, c->Wl, c->Wth,
                         c->Wtl, Nep, nullptr, s));
  HIP_TRY(launch_state_set(c->st, t0, 1, 1, s));
  const int32_t* run_pc = &c->st->run_pc;
  // off-diagonals: the update rule of Eq. 5 with alpha = 1 gives T itself
  Rule r1 = c->rule;
  r1.alpha = 1.0;
  if (c->b3)
    HIP_TRY(launch_coop_partial_b3(c->Wh, c->Wl, Nap, Nep, Nap, c->splits, c->ppart, run_pc, s));
  else
    HIP_TRY(launch_coop_partial(W, Nap, Nep, Nap, c->splits, c->ppart, run_pc, s));
  HIP_TRY(launch_coop_finalize(c->ppart, c->splits, Nep, c->nWr, c->P, Nep, Ne, r1,
                               c->rule.sigma_from_T ? c->Tside : nullptr, c->Ph, c->Pl, run_pc, s));
  if (c->b3)
    HIP_TRY(launch_coreg_update_b3(c->Wth, c->Wtl, Nep, Nep, c->C, Nap, Nap, Na,
                                   c->nWc, r1, c->cstat, c->csq, c->corder, run_pc, s,
                                   c->packed));
  else
    HIP_TRY(launch_coreg_update(W, Nap, Nep, c->C, Nap, Nap, Na, c->nWc, r1, c->cstat, c->csq,
                                c->corder, run_pc, s, c->packed));
  // diagonals: t0 steps of Eq. 6 in closed form with sigma of the rebuilt rows
  const double a = c->rule.alpha;
  double g = 0.0;
  for (int32_t tau = 1; tau <= t0; ++tau) g += pow(1.0 - a, (double)(t0 - tau)) * exp(2.0 * a * tau);
  const double keep = pow(1.0 - a, (double)t0);
  HIP_TRY(launch_diagonals_schedule(c->P, Nep, c->dP, Ne,
                                    c->rule.sigma_from_T ? c->Tside : nullptr, c->nP, c->dC, Nap,
                                    Na, c->cstat, c->rule.sigma_from_T ? c->csq : nullptr,
                                    coreg_slots(Nap), c->nC, c->rule, keep, g, c->st, s));
  HIP_TRY(launch_state_set(c->st, t0, 1, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->t0 = t0;
  c->executed = 0;
  c->enqueued = 0;
  c->r_next = false;
  c->host->t = t0;
  c->host->active = 1;
  c->host->conv = 0;
  return PANDA_OK;
}

}  // extern "C"
