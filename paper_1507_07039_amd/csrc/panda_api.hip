// Host side of libpanda.so: argument checks, workspace layout, the
// iteration sequence of Sec. II-B and the C ABI declared in include/panda.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "host_internal.h"

using namespace panda;

namespace panda {

thread_local char g_err[512] = "";

panda_status fail(panda_status st, const char* fmt, const char* what) {
  snprintf(g_err, sizeof g_err, fmt, what);
  return st;
}

panda_status hip_fail(hipError_t e, const char* where) {
  snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
  return PANDA_ERR_HIP;
}

}  // namespace panda

namespace panda {

Rule rule_of(const panda_options& o) {
  Rule r;
  r.alpha = o.alpha;
  r.tol = o.tol;
  r.diag_alpha = o.diag_alpha;
  r.sigma_from_T = o.sigma_from_T;
  r.n_own = o.n_own;
  r.h_undamped = o.h_undamped;
  r.update_last = o.update_last;
  r.sigma_ddof = o.sigma_ddof;
  return r;
}

panda_status check_options(const panda_options& o) {
  if (!(o.alpha > 0.0) || !(o.alpha <= 1.0)) return fail(PANDA_ERR_ARG, "alpha must be in (0, 1]%s");
  if (!(o.tol >= 0.0) || !isfinite(o.tol)) return fail(PANDA_ERR_ARG, "tol must be finite and >= 0%s");
  if (o.max_iter < 1) return fail(PANDA_ERR_ARG, "max_iter must be >= 1%s");
  if (o.poll_every < 1) return fail(PANDA_ERR_ARG, "poll_every must be >= 1%s");
  if (o.precision != PANDA_PREC_FP32 && o.precision != PANDA_PREC_BF16X3)
    return fail(PANDA_ERR_ARG, "unknown precision%s");
  if (o.sigma_ddof != 0 && o.sigma_ddof != 1) return fail(PANDA_ERR_ARG, "sigma_ddof must be 0 or 1%s");
  if (o.packed_c != 0 && o.packed_c != 1) return fail(PANDA_ERR_ARG, "packed_c must be 0 or 1%s");
  if (o.zscore_mode < PANDA_ZSCORE_GLOBAL || o.zscore_mode > PANDA_ZSCORE_ROWCOL)
    return fail(PANDA_ERR_ARG, "unknown zscore_mode%s");
  return PANDA_OK;
}

// Dimensions that keep every index and the tiled grids within range.
bool dims_ok(int64_t Ne, int64_t Na) {
  return Ne >= 1 && Na >= 1 && Ne <= (1 << 16) && Na <= (1 << 18);
}

}  // namespace panda

namespace panda {

LayoutSpec single_spec(int64_t Ne, int64_t Na, bool packed_c, int32_t precision) {
  const int64_t Nep = round_up(Ne, kPadE), Nap = round_up(Na, kPadA);
  const int64_t blocks = precision == PANDA_PREC_BF16X3 ? 512 : 1024;
  const int64_t nh = std::max(rect_tiles(Nep, Nap), rect_hpart_slots_b3(Nep, Nap));
  return LayoutSpec{false, nh, coop_splits(Nep, Nap, blocks), packed_c};
}

// Workspace layout shared by the size queries and the contexts.
size_t ctx_layout(int64_t Ne, int64_t Na, int32_t precision, const LayoutSpec& spec, panda_ctx* c,
                  char* base) {
  const int64_t Nep = round_up(Ne, kPadE), Nap = round_up(Na, kPadA);
  Carver cv{base};
  const size_t nw = (size_t)Nep * (size_t)Nap;
  float* w0 = cv.take<float>(nw);
  float* w1 = cv.take<float>(nw);
  float* r = cv.take<float>(nw);
  // slack after P: the next-R tiles of the FP32 form read its last row past N_e
  float* p = cv.take<float>((size_t)Nep * Nep + (size_t)next_r_p_slack(Nep));
  float* cc = cv.take<float>(spec.packed_c ? (size_t)packed_floats(Nap) : (size_t)Nap * Nap);
  float* ts = cv.take<float>((size_t)Nep * Nep);
  const int splits = (int)spec.ppart_splits;
  float* pp = cv.take<float>((size_t)splits * Nep * Nep);
  float* sk = spec.batched ? nullptr : cv.take<float>(rect_partial_floats());
  double* dp = cv.take<double>((size_t)Nep);
  double* dc = cv.take<double>((size_t)Nap);
  double* np_ = cv.take<double>((size_t)Nep);
  double* nc = cv.take<double>((size_t)Nap);
  double* nwr = cv.take<double>((size_t)Nep);
  double* nwc = cv.take<double>((size_t)Nap);
  double* scr = cv.take<double>(w_norm_scratch_doubles(Nep, Nap));
  const int64_t nh = spec.hpart_tiles;
  double* hp = cv.take<double>((size_t)nh);
  double2* cs = cv.take<double2>((size_t)coreg_slots(Nap) * Nap);
  double* cq = cv.take<double>((size_t)coreg_slots(Nap) * Nap);
  // z-score scratch, large enough for an identity prior of either side in any scope
  const int64_t nid = Nep > Nap ? Nep : Nap;
  double* zs = cv.take<double>(zscore_scratch_doubles(nid, nid, PANDA_ZSCORE_ROWCOL));
  uint32_t* co = cv.take<uint32_t>((size_t)coreg_tiles(Nap));
  DevState* st = cv.take<DevState>(1);
  // split-BF16 operand planes
  const bool b3 = precision == PANDA_PREC_BF16X3;
  uint32_t* cor = !spec.batched
                      ? cv.take<uint32_t>((size_t)(coreg_tiles(Nap) + next_r_tiles(Nep, Nap)))
                      : nullptr;
  bf16_t* sh[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (b3) {
    sh[0] = cv.take<bf16_t>(nw);                   // W hi, row-major
    sh[1] = cv.take<bf16_t>(nw);                   // W lo
    sh[2] = cv.take<bf16_t>(nw);                   // W^T hi, gene-major
    sh[3] = cv.take<bf16_t>(nw);                   // W^T lo
    sh[4] = cv.take<bf16_t>((size_t)Nep * Nep);    // P hi, zero diagonal
    sh[5] = cv.take<bf16_t>((size_t)Nep * Nep);    // P lo
  }
  if (c) {
    c->Nep = Nep;
    c->Nap = Nap;
    c->W[0] = w0;
    c->W[1] = w1;
    c->R = r;
    c->P = p;
    c->C = cc;
    c->Tside = ts;
    c->ppart = pp;
    c->skpart = sk;
    c->dP = dp;
    c->dC = dc;
    c->nP = np_;
    c->nC = nc;
    c->nWr = nwr;
    c->nWc = nwc;
    c->colscr = scr;
    c->splits = splits;
    c->hpart = hp;
    c->nh = b3 ? rect_hpart_slots_b3(c->Nep, c->Nap) : rect_tiles(c->Nep, c->Nap);  // h partials the A + W tiling writes
    c->cstat = cs;
    c->csq = cq;
    c->zs = zs;
    c->corder = co;
    c->corder_r = cor;
    c->r_next = false;
    c->st = st;
    c->b3 = b3;
    c->packed = spec.packed_c;
    c->Wh = sh[0];
    c->Wl = sh[1];
    c->Wth = sh[2];
    c->Wtl = sh[3];
    c->Ph = sh[4];
    c->Pl = sh[5];
  }
  return cv.off;
}

panda_status ctx_setup(panda_ctx* c, int64_t Ne, int64_t Na, const panda_options& o,
                       const LayoutSpec& spec, char* base, hipStream_t stream) {
  c->Ne = Ne;
  c->Na = Na;
  c->opt = o;
  c->rule = rule_of(o);
  c->stream = stream;
  ctx_layout(Ne, Na, o.precision, spec, c, base);
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->host), sizeof(DevState),
                        hipHostMallocDefault));
  c->loaded = false;
  return PANDA_OK;
}

panda_status ctx_fill_order(panda_ctx* c) {
  // host table, copied before it goes away
  std::vector<uint32_t> order((size_t)coreg_tiles(c->Nap));
  coreg_order_fill(c->Nap, kCoregGroup, order.data());
  HIP_TRY(hipMemcpyAsync(c->corder, order.data(), order.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice, c->stream));
  std::vector<uint32_t> order_r;
  if (c->corder_r) {
    order_r.resize(order.size() + (size_t)next_r_tiles(c->Nep, c->Nap));
    coreg_next_r_order_fill(c->Nep, c->Nap, order.data(), order_r.data());
    HIP_TRY(hipMemcpyAsync(c->corder_r, order_r.data(), order_r.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PANDA_OK;
}

void ctx_free(panda_ctx* c) {
  if (c->host) (void)hipHostFree(c->host);
  c->host = nullptr;
  if (c->snap) {
    (void)hipHostFree(c->snap);
    for (hipEvent_t& e : c->snap_ev) (void)hipEventDestroy(e);
  }
  c->snap = nullptr;
  if (c->ev[0][0])
    for (int i = 0; i < kMaxPending; ++i)
      for (int p = 0; p <= PANDA_NPHASE; ++p) (void)hipEventDestroy(c->ev[i][p]);
  c->ev[0][0] = nullptr;
}

// The z-scored identity of order n (Sec. II-A: an absent prior is the
// identity, z-scored like any network) in closed form: every row, every
// column and the whole matrix hold one 1 among zeros, so the result has one
// value on the diagonal (dv) and one off it (ov).  Mean m = 1/n; sum of
// squared deviations over n^2 entries n (1 - m)^2 + (n^2 - n) m^2 = n - 1,
// over a row (1 - m)^2 + (n - 1) m^2; the row + column scope gives
// (Zr + Zc) / sqrt 2 = sqrt 2 Zr.  False when the std is 0 (n = 1).
bool identity_zscore(int64_t n, int32_t mode, int32_t ddof, double* dv, double* ov) {
  const double m = 1.0 / (double)n, nn = (double)n;
  const double cnt = mode == PANDA_ZSCORE_GLOBAL ? nn * nn : nn;
  const double ss = mode == PANDA_ZSCORE_GLOBAL ? nn * (1.0 - m) * (1.0 - m) + (nn * nn - nn) * m * m
                                                : (1.0 - m) * (1.0 - m) + (nn - 1.0) * m * m;
  if (cnt - ddof < 1.0) return false;
  const double sd = sqrt(ss / (cnt - ddof));
  if (!(sd > 0.0)) return false;
  const double f = mode == PANDA_ZSCORE_ROWCOL ? sqrt(2.0) : 1.0;
  *dv = f * (1.0 - m) / sd;
  *ov = f * (-m) / sd;
  return true;
}

size_t zscore_scratch_doubles(int64_t rows, int64_t cols, int32_t mode) {
  if (mode == PANDA_ZSCORE_GLOBAL) return kZsScratch;
  const size_t rc = 8 + 2 * (size_t)rows + (mode == PANDA_ZSCORE_ROWCOL ? 2 * (size_t)cols : 0);
  return rc > kZsScratch ? rc : kZsScratch;
}

panda_status zscore(float* M, int64_t rows, int64_t cols, int64_t ld, int32_t mode, int32_t ddof,
                    double* scratch, hipStream_t s) {
  if (mode == PANDA_ZSCORE_GLOBAL) {
    HIP_TRY(launch_zscore_stats(M, rows, cols, ld, scratch, s, ddof));
    double tail[3];
    HIP_TRY(hipMemcpyAsync(tail, scratch + kZsBlocks, sizeof tail, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (tail[2] != 0.0) return fail(PANDA_ERR_NONFINITE, "network contains NaN or Inf%s");
    if (!(tail[1] > 0.0)) return fail(PANDA_ERR_DEGENERATE, "network is constant (std = 0)%s");
    HIP_TRY(launch_zscore_apply(M, rows, cols, ld, scratch, s));
    return PANDA_OK;
  }
  double* flags = scratch;
  double2* rs = reinterpret_cast<double2*>(scratch + 8);
  double2* cs = mode == PANDA_ZSCORE_ROWCOL ? rs + rows : nullptr;
  HIP_TRY(launch_zscore_rc_stats(M, rows, cols, ld, ddof, flags, rs, cs, s));
  double f[2];
  HIP_TRY(hipMemcpyAsync(f, flags, sizeof f, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (f[0] != 0.0) return fail(PANDA_ERR_NONFINITE, "network contains NaN or Inf%s");
  if (f[1] != 0.0)
    return fail(PANDA_ERR_DEGENERATE, "a row or column of the network is constant (std = 0)%s");
  HIP_TRY(launch_zscore_rc_apply(M, rows, cols, ld, rs, cs, s));
  return PANDA_OK;
}

}  // namespace panda

namespace {

// z-score of a strided matrix using `scratch`; synchronises the stream.

// Phase boundary marker: records event `p` of the current pending
// iteration when timing is on.
panda_status mark(panda_ctx* c, int p) {
  if (!c->timing) return PANDA_OK;
  HIP_TRY(hipEventRecord(c->ev[c->npend][p], c->stream));
  return PANDA_OK;
}

// Sum the elapsed times of the pending timed iterations (stream synced).
panda_status collect_times(panda_ctx* c) {
  for (int i = 0; i < c->npend; ++i)
    for (int p = 0; p < PANDA_NPHASE; ++p) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev[i][p], c->ev[i][p + 1]));
      c->tot_ms[p] += ms;
      c->cnt[p] += 1;
    }
  c->npend = 0;
  return PANDA_OK;
}

// Read the device state back (synchronises the stream).
panda_status read_state(panda_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->executed = c->host->t - c->t0;
  return collect_times(c);
}

// Enqueue one iteration: R, A + W update, h, P update, C update, diagonals.
// Iteration k (counted from the load) reads W[k % 2] and writes W[(k+1) % 2];
// iterations past convergence are skipped on the device, so the executed
// ones are always a prefix of the enqueued ones.
panda_status enqueue_iteration(panda_ctx* c) {
  if (c->timing && c->npend == kMaxPending) PANDA_TRY(read_state(c));
  const int64_t k = c->enqueued;
  float* Wold = c->W[k & 1];
  float* Wnew = c->W[(k + 1) & 1];
  hipStream_t s = c->stream;
  const int32_t* active = &c->st->active;
  const int32_t* run_pc = &c->st->run_pc;
  PANDA_TRY(mark(c, PANDA_PHASE_R));
  // Eq. 3: R = T(P, W), K = N_e (computed by the last C update unless the
  // state is new)
  const bool next_r = c->corder_r != nullptr;
  if (next_r) {
    if (!c->r_next) {
      if (c->b3)
        HIP_TRY(launch_resp_tiles_b3(c->Ph, c->Pl, c->Nep, c->dP, c->Wth, c->Wtl, c->Nep,
                                     c->Nap, c->Ne, c->Na, Wold, c->Nap, c->nP, c->nWc, c->R,
                                     active, s));
      else
        HIP_TRY(launch_resp_tiles(c->P, c->Nep, c->dP, c->Nap, c->Ne, c->Na, Wold, c->Nap,
                                  c->nP, c->nWc, c->R, active, s));
    }
  } else if (c->b3)
    HIP_TRY(launch_resp_b3(c->Ph, c->Pl, c->Nep, c->dP, c->Wth, c->Wtl, c->Nep, c->Nep, c->Nap,
                           c->Ne, c->Na, Wold, c->Nap, c->nP, c->nWc, c->R, c->skpart, active, s));
  else
    HIP_TRY(launch_resp(c->P, c->Nep, c->dP, Wold, c->Nap, c->Nep, c->Nap, c->Ne, c->Na, c->nP,
                        c->nWc, c->R, c->skpart, active, s));
  PANDA_TRY(mark(c, PANDA_PHASE_AW));
  // Eq. 4 + Eq. 2 + Eq. 7 partials: A = T(W, C), K = N_a
  if (c->b3)
    HIP_TRY(launch_avail_wupdate_b3(c->Wh, c->Wl, Wold, c->C, c->dC, c->R, Wnew, c->Nap, c->Nep,
                                    c->Nap, c->Ne, c->Na, c->nWr, c->nC, c->rule, c->hpart,
                                    c->skpart, active, s, c->packed));
  else
    HIP_TRY(launch_avail_wupdate(Wold, c->C, c->dC, c->R, Wnew, c->Nap, c->Nep, c->Nap, c->Ne,
                                 c->Na, c->nWr, c->nC, c->rule, c->hpart, c->skpart, active, s,
                                 c->packed));
  PANDA_TRY(mark(c, PANDA_PHASE_H));
  HIP_TRY(launch_finish_h(c->hpart, c->nh, c->Ne * c->Na, c->st, c->rule, s));
  // squared norms (and split planes) of the new W
  HIP_TRY(launch_w_norms(Wnew, c->Ne, c->Na, c->Nap, c->Nep, c->nWr, c->nWc, c->colscr, c->Wh,
                         c->Wl, c->Wth, c->Wtl, c->Nep, run_pc, s));
  PANDA_TRY(mark(c, PANDA_PHASE_PPART));
  // Eq. 5, P: T(W_i., W_m.) of the new W
  if (c->b3)
    HIP_TRY(launch_coop_partial_b3(c->Wh, c->Wl, c->Nap, c->Nep, c->Nap, c->splits, c->ppart,
                                   run_pc, s));
  else
    HIP_TRY(launch_coop_partial(Wnew, c->Nap, c->Nep, c->Nap, c->splits, c->ppart, run_pc, s));
  PANDA_TRY(mark(c, PANDA_PHASE_PFIN));
  HIP_TRY(launch_coop_finalize(c->ppart, c->splits, c->Nep, c->nWr, c->P, c->Nep, c->Ne, c->rule,
                               c->rule.sigma_from_T ? c->Tside : nullptr, c->Ph, c->Pl, run_pc,
                               s));
  // Eq. 6 for P, and |P_i.|^2, before the C update when it also computes
  // the next R (which needs them)
  if (next_r)
    HIP_TRY(launch_diagonals(c->P, c->Nep, c->dP, c->Ne,
                             c->rule.sigma_from_T ? c->Tside : nullptr, c->nP, c->dC, c->Nap,
                             c->Na, c->cstat, c->rule.sigma_from_T ? c->csq : nullptr,
                             coreg_slots(c->Nap), c->nC, c->rule, c->st, s, kDiagP));
  PANDA_TRY(mark(c, PANDA_PHASE_C));
  // Eq. 5, C: T(W_.k, W_.j) of the new W, upper tiles, mirrored (and the
  // next iteration's R = T(P, W) of the new P and W)
  if (next_r && c->b3)
    HIP_TRY(launch_coreg_update_next_r_b3(c->Wth, c->Wtl, c->Nep, c->Nep, c->C, c->Nap, c->Nap,
                                          c->Na, c->nWc, c->rule, c->cstat, c->csq, c->corder_r,
                                          run_pc, s, c->packed, c->Ph, c->Pl, c->dP, c->nP,
                                          Wnew, c->Nap, c->Ne, c->R));
  else if (next_r)
    HIP_TRY(launch_coreg_update_next_r(Wnew, c->Nap, c->Nep, c->C, c->Nap, c->Nap, c->Na, c->nWc,
                                       c->rule, c->cstat, c->csq, c->corder_r, run_pc, s,
                                       c->packed, c->P, c->dP, c->nP, c->Ne, c->R));
  else if (c->b3)
    HIP_TRY(launch_coreg_update_b3(c->Wth, c->Wtl, c->Nep, c->Nep, c->C, c->Nap,
                                   c->Nap, c->Na, c->nWc, c->rule, c->cstat, c->csq, c->corder,
                                   run_pc, s, c->packed));
  else
    HIP_TRY(launch_coreg_update(Wnew, c->Nap, c->Nep, c->C, c->Nap, c->Nap, c->Na, c->nWc,
                                c->rule, c->cstat, c->csq, c->corder, run_pc, s, c->packed));
  PANDA_TRY(mark(c, PANDA_PHASE_DIAG));
  // Eq. 6, and |P_i.|^2, |C_.j|^2 for the next iteration
  HIP_TRY(launch_diagonals(c->P, c->Nep, c->dP, c->Ne, c->rule.sigma_from_T ? c->Tside : nullptr,
                           c->nP, c->dC, c->Nap, c->Na, c->cstat,
                           c->rule.sigma_from_T ? c->csq : nullptr, coreg_slots(c->Nap), c->nC,
                           c->rule, c->st, s, next_r ? kDiagC : kDiagBoth));
  c->r_next = next_r;
  PANDA_TRY(mark(c, PANDA_NPHASE));
  if (c->timing) c->npend += 1;
  c->enqueued += 1;
  return PANDA_OK;
}

panda_status copy_in(float* dst, int64_t ldd, const float* src, int64_t rows, int64_t cols,
                     hipStream_t s) {
  HIP_TRY(hipMemcpy2DAsync(dst, (size_t)ldd * 4, src, (size_t)cols * 4, (size_t)cols * 4,
                           (size_t)rows, hipMemcpyDeviceToDevice, s));
  return PANDA_OK;
}

}  // namespace

namespace panda {

// Enqueue ahead and read h back every poll_every iterations; iterations
// enqueued past convergence are no-ops on the device.
// Iterate to convergence or max_iter.  The host never makes the device wait
// for it: the state after a polled iteration is copied to a pinned slot (with
// an event) as soon as that iteration is enqueued, and the host looks at it
// only after enqueueing the next iteration, so the device always has work
// queued while the host waits.  The one iteration enqueued after convergence
// runs gated (its kernels return at once: the executed iterations are always
// a prefix of the enqueued ones), so the result is that of polling at once.
panda_status run_loaded(panda_ctx* c) {
  const int64_t max_iter = c->opt.max_iter, poll = c->opt.poll_every;
  if (!c->snap) {
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->snap), 2 * sizeof(DevState),
                          hipHostMallocDefault));
    for (hipEvent_t& e : c->snap_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  int64_t pending = -1;  // polled iteration whose state copy is awaited
  while (c->enqueued < max_iter) {
    PANDA_TRY(enqueue_iteration(c));
    const int64_t k = c->enqueued;
    if (pending >= 0) {
      HIP_TRY(hipEventSynchronize(c->snap_ev[pending & 1]));
      if (!c->snap[pending & 1].active) break;
      pending = -1;
    }
    if (k % poll == 0 && k < max_iter) {
      HIP_TRY(hipMemcpyAsync(&c->snap[k & 1], c->st, sizeof(DevState), hipMemcpyDeviceToHost,
                             c->stream));
      HIP_TRY(hipEventRecord(c->snap_ev[k & 1], c->stream));
      pending = k;
    }
  }
  PANDA_TRY(read_state(c));
  c->enqueued = c->executed;
  return PANDA_OK;
}

}  // namespace panda

extern "C" {

void panda_default_options(panda_options* o) {
  if (!o) return;
  o->alpha = 0.1;
  o->tol = 1e-3;
  o->max_iter = 200;
  o->diag_alpha = 1;
  o->sigma_from_T = 0;
  o->n_own = 0;
  o->h_undamped = 0;
  o->update_last = 0;
  o->poll_every = 1;
  o->precision = PANDA_PREC_FP32;
  o->sigma_ddof = 0;
  o->zscore_mode = PANDA_ZSCORE_GLOBAL;
  o->packed_c = 0;
}

panda_status panda_ctx_set_timing(panda_ctx* c, int32_t enable) {
  if (!c) return fail(PANDA_ERR_ARG, "set_timing: NULL context%s");
  if (enable && !c->ev[0][0]) {
    for (int i = 0; i < kMaxPending; ++i)
      for (int p = 0; p <= PANDA_NPHASE; ++p) HIP_TRY(hipEventCreate(&c->ev[i][p]));
  }
  if (!enable && c->timing) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    panda_status st = collect_times(c);
    if (st != PANDA_OK) return st;
  }
  c->timing = enable != 0;
  for (int p = 0; p < PANDA_NPHASE; ++p) {
    c->tot_ms[p] = 0.0;
    c->cnt[p] = 0;
  }
  return PANDA_OK;
}

panda_status panda_ctx_phase_times(panda_ctx* c, double* total_ms, int64_t* count) {
  if (!c) return fail(PANDA_ERR_ARG, "phase_times: NULL context%s");
  if (c->timing && c->npend) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    panda_status st = collect_times(c);
    if (st != PANDA_OK) return st;
  }
  for (int p = 0; p < PANDA_NPHASE; ++p) {
    if (total_ms) total_ms[p] = c->tot_ms[p];
    if (count) count[p] = c->cnt[p];
  }
  return PANDA_OK;
}

const char* panda_status_string(panda_status s) {
  switch (s) {
    case PANDA_OK: return "ok";
    case PANDA_NOT_CONVERGED: return "not converged";
    case PANDA_ERR_ARG: return "invalid argument";
    case PANDA_ERR_DEGENERATE: return "degenerate network (std = 0)";
    case PANDA_ERR_NONFINITE: return "non-finite input";
    case PANDA_ERR_HIP: return "HIP runtime error";
    case PANDA_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PANDA_STATUS_MAX_ENUM: break;  // sizes the enum, no status
  }
  return "unknown status";
}

const char* panda_last_error(void) { return g_err; }

size_t panda_normalize_workspace_bytes(void) { return align_up(kZsScratch * sizeof(double)); }

panda_status panda_normalize(float* M, int64_t rows, int64_t cols, void* workspace,
                             size_t ws_bytes, hipStream_t stream) {
  if (!M || rows < 1 || cols < 1) return fail(PANDA_ERR_ARG, "normalize: bad matrix%s");
  if (!workspace || ws_bytes < panda_normalize_workspace_bytes() ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "normalize: workspace too small or misaligned%s");
  return zscore(M, rows, cols, cols, PANDA_ZSCORE_GLOBAL, 0, static_cast<double*>(workspace),
                stream);
}

size_t panda_normalize_ex_workspace_bytes(int64_t rows, int64_t cols, int32_t zscore_mode) {
  if (rows < 1 || cols < 1 || zscore_mode < PANDA_ZSCORE_GLOBAL ||
      zscore_mode > PANDA_ZSCORE_ROWCOL)
    return 0;
  return align_up(zscore_scratch_doubles(rows, cols, zscore_mode) * sizeof(double));
}

panda_status panda_normalize_ex(float* M, int64_t rows, int64_t cols, int32_t zscore_mode,
                                int32_t ddof, void* workspace, size_t ws_bytes,
                                hipStream_t stream) {
  if (!M || rows < 1 || cols < 1) return fail(PANDA_ERR_ARG, "normalize_ex: bad matrix%s");
  if (zscore_mode < PANDA_ZSCORE_GLOBAL || zscore_mode > PANDA_ZSCORE_ROWCOL || ddof < 0 ||
      ddof > 1)
    return fail(PANDA_ERR_ARG, "normalize_ex: unknown zscore_mode or ddof%s");
  if (!workspace || ws_bytes < panda_normalize_ex_workspace_bytes(rows, cols, zscore_mode) ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "normalize_ex: workspace too small or misaligned%s");
  return zscore(M, rows, cols, cols, zscore_mode, ddof, static_cast<double*>(workspace), stream);
}

namespace {
struct TaniLayout {
  float *Xp, *Yp, *Op, *part;
  double *nx, *ny, *scr;
};
static size_t tanimoto_layout(int64_t M, int64_t K, int64_t N, char* base, TaniLayout* L) {
  const int64_t Mp = round_up(M, kPadE), Kp = round_up(K, kPadK), Np = round_up(N, kPadA);
  Carver cv{base};
  float* xp = cv.take<float>((size_t)Mp * Kp);
  float* yp = cv.take<float>((size_t)Kp * Np);
  float* op = cv.take<float>((size_t)Mp * Np);
  float* pt = cv.take<float>(rect_partial_floats());
  double* nx = cv.take<double>((size_t)Mp);
  double* ny = cv.take<double>((size_t)Np);
  double* sc = cv.take<double>((size_t)kColChunks * (size_t)Np);
  if (L) *L = TaniLayout{xp, yp, op, pt, nx, ny, sc};
  return cv.off;
}
}  // namespace

size_t panda_tanimoto_workspace_bytes(int64_t M, int64_t K, int64_t N) {
  if (M < 1 || K < 1 || N < 1) return 0;
  return tanimoto_layout(M, K, N, nullptr, nullptr);
}

panda_status panda_tanimoto(const float* X, const float* Y, int64_t M, int64_t K, int64_t N,
                            float* Out, void* workspace, size_t ws_bytes, hipStream_t s) {
  if (!X || !Y || !Out || M < 1 || K < 1 || N < 1 || M > (1 << 20) || N > (1 << 20) ||
      K > (1 << 20))
    return fail(PANDA_ERR_ARG, "tanimoto: bad arguments%s");
  const size_t need = panda_tanimoto_workspace_bytes(M, K, N);
  if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "tanimoto: workspace too small or misaligned%s");
  const int64_t Mp = round_up(M, kPadE), Kp = round_up(K, kPadK), Np = round_up(N, kPadA);
  TaniLayout L;
  tanimoto_layout(M, K, N, static_cast<char*>(workspace), &L);
  HIP_TRY(hipMemsetAsync(L.Xp, 0, (size_t)Mp * Kp * 4, s));
  HIP_TRY(hipMemsetAsync(L.Yp, 0, (size_t)Kp * Np * 4, s));
  panda_status st = copy_in(L.Xp, Kp, X, M, K, s);
  if (st != PANDA_OK) return st;
  st = copy_in(L.Yp, Np, Y, K, N, s);
  if (st != PANDA_OK) return st;
  HIP_TRY(launch_row_sqnorms(L.Xp, Mp, Kp, Kp, L.nx, nullptr, s));
  HIP_TRY(launch_col_sqnorms(L.Yp, Kp, Np, Np, L.ny, L.scr, nullptr, s));
  HIP_TRY(launch_tanimoto_store(L.Xp, Kp, L.Yp, Np, Mp, Np, Kp, M, N, L.nx, L.ny, L.Op, Np, L.part,
                                nullptr, s));
  HIP_TRY(hipMemcpy2DAsync(Out, (size_t)N * 4, L.Op, (size_t)Np * 4, (size_t)N * 4, (size_t)M,
                           hipMemcpyDeviceToDevice, s));
  return PANDA_OK;
}

namespace {
struct PearsonLayout {
  double2* stat;
  float* Zt;
};
static size_t pearson_layout(int64_t G, int64_t S, char* base, PearsonLayout* L) {
  const int64_t Gp = round_up(G, kPadA), Sp = round_up(S, kPadK);
  Carver cv{base};
  double2* st = cv.take<double2>((size_t)G);
  float* zt = cv.take<float>((size_t)Sp * Gp);
  if (L) *L = PearsonLayout{st, zt};
  return cv.off;
}
}  // namespace

size_t panda_pearson_workspace_bytes(int64_t G, int64_t S) {
  if (G < 1 || S < 2) return 0;
  return pearson_layout(G, S, nullptr, nullptr);
}

namespace {
bool pearson_args_ok(const float* E, int64_t G, int64_t S, int64_t lde, const float* C,
                     int64_t ldc) {
  return E && C && G >= 1 && S >= 2 && G <= (1 << 18) && S <= (1 << 20) && lde >= S && ldc >= G;
}

// The two kernels of the prior on a scratch region laid out by
// pearson_layout; every byte of it that they read they have written first.
panda_status pearson_enqueue(const float* E, int64_t G, int64_t S, int64_t lde, float* C,
                             int64_t ldc, char* base, hipStream_t s) {
  const int64_t Gp = round_up(G, kPadA), Sp = round_up(S, kPadK);
  PearsonLayout L;
  pearson_layout(G, S, base, &L);
  HIP_TRY(launch_pearson_z(E, G, S, lde, L.stat, L.Zt, Gp, Sp, s));
  HIP_TRY(launch_corr(L.Zt, Gp, Sp, G, C, ldc, s));
  return PANDA_OK;
}

// Scratch of panda_pearson_noalloc, one copy on every GPU the library runs
// on, held until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device array: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[PANDA_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];

panda_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PANDA_ERR_ARG, "pearson_noalloc: device id out of range%s");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PANDA_ERR_HIP, "pearson_noalloc: no device address for the scratch array%s");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PANDA_OK;
}
}  // namespace

panda_status panda_pearson(const float* E, int64_t G, int64_t S, int64_t lde, float* C,
                           int64_t ldc, void* workspace, size_t ws_bytes, hipStream_t s) {
  if (!pearson_args_ok(E, G, S, lde, C, ldc)) return fail(PANDA_ERR_ARG, "pearson: bad arguments%s");
  const size_t need = panda_pearson_workspace_bytes(G, S);
  if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "pearson: workspace too small or misaligned%s");
  return pearson_enqueue(E, G, S, lde, C, ldc, static_cast<char*>(workspace), s);
}

panda_status panda_pearson_noalloc(const float* E, int64_t G, int64_t S, int64_t lde, float* C,
                                   int64_t ldc, hipStream_t s) {
  if (!pearson_args_ok(E, G, S, lde, C, ldc))
    return fail(PANDA_ERR_ARG, "pearson_noalloc: bad arguments%s");
  const size_t need = panda_pearson_workspace_bytes(G, S);
  if (need > (size_t)PANDA_NOALLOC_SCRATCH_BYTES) {
    snprintf(g_err, sizeof g_err,
             "pearson_noalloc: G = %lld genes x S = %lld samples need %zu bytes of scratch, more "
             "than the %zu the library holds; use panda_pearson with a workspace",
             (long long)G, (long long)S, need, (size_t)PANDA_NOALLOC_SCRATCH_BYTES);
    return PANDA_ERR_ARG;
  }
  void* base = nullptr;
  PANDA_TRY(scratch_address(&base));
  return pearson_enqueue(E, G, S, lde, C, ldc, static_cast<char*>(base), s);
}

size_t panda_workspace_bytes(int64_t Ne, int64_t Na, const panda_options* opt) {
  (void)opt;
  if (!dims_ok(Ne, Na)) return 0;
  return ctx_layout(Ne, Na, opt ? opt->precision : PANDA_PREC_FP32,
                    single_spec(Ne, Na, opt && opt->packed_c,
                                opt ? opt->precision : PANDA_PREC_FP32),
                    nullptr,
                    nullptr);
}

panda_status panda_ctx_create(int64_t Ne, int64_t Na, const panda_options* opt, void* workspace,
                              size_t ws_bytes, hipStream_t stream, panda_ctx** out) {
  if (!out) return fail(PANDA_ERR_ARG, "ctx_create: out is NULL%s");
  *out = nullptr;
  if (!dims_ok(Ne, Na)) return fail(PANDA_ERR_ARG, "ctx_create: bad dimensions%s");
  panda_options o;
  if (opt)
    o = *opt;
  else
    panda_default_options(&o);
  panda_status st = check_options(o);
  if (st != PANDA_OK) return st;
  if (!workspace || ws_bytes < panda_workspace_bytes(Ne, Na, &o) ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "ctx_create: workspace too small or misaligned%s");
  panda_ctx* c = new (std::nothrow) panda_ctx();
  if (!c) return fail(PANDA_ERR_ARG, "ctx_create: out of host memory%s");
  st = ctx_setup(c, Ne, Na, o, single_spec(Ne, Na, o.packed_c != 0, o.precision),
                 static_cast<char*>(workspace),
                 stream);
  if (st != PANDA_OK) {
    delete c;
    return st;
  }
  *out = c;
  return PANDA_OK;
}

void panda_ctx_destroy(panda_ctx* c) {
  if (!c) return;
  ctx_free(c);
  delete c;
}

panda_status panda_ctx_load(panda_ctx* c, const float* W, const float* P, const float* C,
                            int32_t t) {
  if (!c || !W || t < 0) return fail(PANDA_ERR_ARG, "ctx_load: bad arguments%s");
  hipStream_t s = c->stream;
  const int64_t Ne = c->Ne, Na = c->Na, Nep = c->Nep, Nap = c->Nap;
  HIP_TRY(hipMemsetAsync(c->W[0], 0, (size_t)Nep * Nap * 4, s));
  HIP_TRY(hipMemsetAsync(c->W[1], 0, (size_t)Nep * Nap * 4, s));
  HIP_TRY(hipMemsetAsync(c->P, 0, (size_t)Nep * Nep * 4, s));
  if (!c->packed) HIP_TRY(hipMemsetAsync(c->C, 0, (size_t)Nap * Nap * 4, s));
  HIP_TRY(hipMemsetAsync(c->Tside, 0, (size_t)Nep * Nep * 4, s));
  panda_status st = copy_in(c->W[0], Nap, W, Ne, Na, s);
  if (st != PANDA_OK) return st;
  if (P) {
    st = copy_in(c->P, Nep, P, Ne, Ne, s);
  } else {
    HIP_TRY(launch_fill_identity(c->P, Ne, Nep, s));
    st = zscore(c->P, Ne, Ne, Nep, c->opt.zscore_mode, c->opt.sigma_ddof, c->zs, s);
  }
  if (st != PANDA_OK) return st;
  if (c->packed) {
    // the upper tiles of C (every stored entry is written: no clearing)
    if (C) {
      HIP_TRY(launch_pack_sym(C, Na, Na, c->C, Nap, s));
    } else {
      double dv, ov;
      if (!identity_zscore(Na, c->opt.zscore_mode, c->opt.sigma_ddof, &dv, &ov))
        return fail(PANDA_ERR_DEGENERATE, "identity C of order 1 has std 0%s");
      HIP_TRY(launch_identity_packed(c->C, Na, Nap, dv, ov, s));
    }
  } else if (C) {
    st = copy_in(c->C, Nap, C, Na, Na, s);
  } else {
    HIP_TRY(launch_fill_identity(c->C, Na, Nap, s));
    st = zscore(c->C, Na, Na, Nap, c->opt.zscore_mode, c->opt.sigma_ddof, c->zs, s);
  }
  if (st != PANDA_OK) return st;
  // squared norms of the loaded state (later iterations produce their own)
  HIP_TRY(hipMemsetAsync(c->nP, 0, (size_t)Nep * 8, s));
  HIP_TRY(hipMemsetAsync(c->nWr, 0, (size_t)Nep * 8, s));
  HIP_TRY(hipMemsetAsync(c->nC, 0, (size_t)Nap * 8, s));
  HIP_TRY(hipMemsetAsync(c->nWc, 0, (size_t)Nap * 8, s));
  HIP_TRY(launch_row_sqnorms(c->P, Ne, Ne, Nep, c->nP, nullptr, s));
  if (c->packed)
    HIP_TRY(launch_col_sqnorms_packed(c->C, Nap, c->csq, c->nC, s));
  else
    HIP_TRY(launch_col_sqnorms(c->C, Na, Na, Nap, c->nC, c->colscr, nullptr, s));
  // the diagonals of P and C move to their FP64 vectors (zero in the matrices)
  HIP_TRY(launch_take_diag(c->P, Ne, Nep, c->dP, s));
  if (c->packed)
    HIP_TRY(launch_take_diag_packed(c->C, Na, c->dC, s));
  else
    HIP_TRY(launch_take_diag(c->C, Na, Nap, c->dC, s));
  if (c->b3) {
    // planes of the loaded state; padding and the P/C diagonals stay zero
    const size_t nw = (size_t)Nep * Nap;
    HIP_TRY(hipMemsetAsync(c->Wh, 0, nw * 2, s));
    HIP_TRY(hipMemsetAsync(c->Wl, 0, nw * 2, s));
    HIP_TRY(hipMemsetAsync(c->Wth, 0, nw * 2, s));
    HIP_TRY(hipMemsetAsync(c->Wtl, 0, nw * 2, s));
    HIP_TRY(hipMemsetAsync(c->Ph, 0, (size_t)Nep * Nep * 2, s));
    HIP_TRY(hipMemsetAsync(c->Pl, 0, (size_t)Nep * Nep * 2, s));
    HIP_TRY(launch_split_offdiag(c->P, Ne, Nep, c->Ph, c->Pl, s));
  }
  // norms (and planes) of W exactly as an iteration computes them, so a
  // stored state resumes bit for bit
  HIP_TRY(launch_w_norms(c->W[0], Ne, Na, Nap, Nep, c->nWr, c->nWc, c->colscr, c->Wh, c->Wl,
                         c->Wth, c->Wtl, Nep, nullptr, s));
  PANDA_TRY(ctx_fill_order(c));
  // h partial slots the A + W product never writes add zeros
  HIP_TRY(hipMemsetAsync(c->hpart, 0, (size_t)c->nh * sizeof(double), s));
  HIP_TRY(launch_state_init(c->st, t, s));
  c->r_next = false;
  c->t0 = t;
  c->executed = 0;
  c->enqueued = 0;
  c->host->h = 0.0;
  c->host->t = t;
  c->host->active = 1;
  c->host->conv = 0;
  c->loaded = true;
  return PANDA_OK;
}

panda_status panda_iterate(panda_ctx* c, double* h, int32_t* t) {
  if (!c || !c->loaded) return fail(PANDA_ERR_ARG, "iterate: context not loaded%s");
  if (c->host->active) {
    panda_status st = enqueue_iteration(c);
    if (st != PANDA_OK) return st;
  }
  panda_status st = read_state(c);
  if (st != PANDA_OK) return st;
  c->enqueued = c->executed;
  if (h) *h = c->host->h;
  if (t) *t = c->host->t;
  return PANDA_OK;
}

panda_status panda_ctx_store(panda_ctx* c, float* W, float* P, float* C, double* h, int32_t* t) {
  if (!c || !c->loaded) return fail(PANDA_ERR_ARG, "ctx_store: context not loaded%s");
  panda_status st = read_state(c);
  if (st != PANDA_OK) return st;
  hipStream_t s = c->stream;
  const float* Wc = c->W[c->executed & 1];
  if (W)
    HIP_TRY(hipMemcpy2DAsync(W, (size_t)c->Na * 4, Wc, (size_t)c->Nap * 4, (size_t)c->Na * 4,
                             (size_t)c->Ne, hipMemcpyDeviceToDevice, s));
  if (P) {
    HIP_TRY(hipMemcpy2DAsync(P, (size_t)c->Ne * 4, c->P, (size_t)c->Nep * 4, (size_t)c->Ne * 4,
                             (size_t)c->Ne, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_put_diag(P, c->Ne, c->Ne, c->dP, s));
  }
  if (C) {
    if (c->packed)
      HIP_TRY(launch_unpack_sym(c->C, c->Na, c->Nap, C, c->Na, s));
    else
      HIP_TRY(hipMemcpy2DAsync(C, (size_t)c->Na * 4, c->C, (size_t)c->Nap * 4, (size_t)c->Na * 4,
                               (size_t)c->Na, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_put_diag(C, c->Na, c->Na, c->dC, s));
  }
  if (h) *h = c->host->h;
  if (t) *t = c->host->t;
  return PANDA_OK;
}

panda_status panda_run(const float* W0, const float* P0, const float* C0, int64_t Ne, int64_t Na,
                       double alpha, double tol, int32_t max_iter, float* W, float* P, float* C,
                       void* workspace, size_t ws_bytes, const panda_options* opt,
                       int32_t* iters, double* h, hipStream_t stream) {
  if (!W0 || !W || !P || !C) return fail(PANDA_ERR_ARG, "run: NULL matrix pointer%s");
  panda_options o;
  if (opt)
    o = *opt;
  else
    panda_default_options(&o);
  o.alpha = alpha;
  o.tol = tol;
  o.max_iter = max_iter;
  panda_ctx* c = nullptr;
  panda_status st = panda_ctx_create(Ne, Na, &o, workspace, ws_bytes, stream, &c);
  if (st != PANDA_OK) return st;
  st = panda_ctx_load(c, W0, P0, C0, 0);
  if (st == PANDA_OK) st = run_loaded(c);
  if (st == PANDA_OK) st = panda_ctx_store(c, W, P, C, h, iters);
  if (st == PANDA_OK && c->host->active) st = PANDA_NOT_CONVERGED;
  panda_ctx_destroy(c);
  return st;
}

}  // extern "C"
