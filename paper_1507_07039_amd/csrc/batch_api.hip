// Host side of the batched form: workspace layout of n networks, the work
// lists of the grouped launches, the tile autotuner, graph capture of one
// iteration and the panda_batch_* entry points of include/panda.h.
#include <algorithm>
#include <new>
#include <vector>

#include "batch_internal.h"
#include "host_internal.h"
#include "update_device.h"

using namespace panda;

namespace {

constexpr int kNumLists = kBTNum;  // one work list per grouped product
constexpr int64_t kCtrCount = (int64_t)kNumLists * kNumXcd * kCtrStride;
constexpr int kMaxBatch = 1 << 16;

// Buffers of network i sized for every tile candidate: the smallest A + W
// tile (64 x 64) and the smallest W W^T chunk.
LayoutSpec batch_spec(int64_t Ne, int64_t Na) {
  const int64_t Nep = round_up(Ne, kPadE), Nap = round_up(Na, kPadA);
  const int64_t c0 = coop_chunk_of(0);
  return LayoutSpec{true, (Nep / 64) * (Nap / 64), (Nap + c0 - 1) / c0};
}

}  // namespace

struct panda_batch {
  int32_t n;
  panda_options opt;
  Rule rule;
  hipStream_t stream;
  std::vector<panda_ctx> ctx;
  BInst* d_inst;
  std::vector<BInst> h_inst;
  struct List {
    int32_t* d_seg_inst;
    int64_t* d_seg_first;
    std::vector<int32_t> seg_inst;
    std::vector<int64_t> seg_first;
    WorkList wl;
    int64_t nb;
  } lists[kNumLists];
  // flat grids: norms (part, sum), P finalisation, diagonals, W planes
  int64_t* d_flat[5];
  std::vector<int64_t> h_flat[5];
  FlatList flat[5];
  bool b3;  // split-BF16 products
  int32_t* ctr;
  DevState* d_states;
  DevState* h_states;  // pinned
  int32_t tiles[kNumLists];
  hipStream_t cap;  // capture stream (default priority)
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool have_graph;
};

namespace {

enum { kFlatPart = 0, kFlatSum = 1, kFlatPfin = 2, kFlatDiag = 3, kFlatPlanes = 4, kNumFlat = 5 };

// Layout of the whole batch workspace: header (descriptors, work lists,
// counters, state gather buffer), then each network's region.
size_t batch_layout(int32_t n, const int64_t* Ne, const int64_t* Na, int32_t precision,
                    panda_batch* b, char* base) {
  Carver cv{base};
  BInst* di = cv.take<BInst>((size_t)n);
  int32_t* si[kNumLists];
  int64_t* sf[kNumLists];
  for (int l = 0; l < kNumLists; ++l) {
    si[l] = cv.take<int32_t>((size_t)n);
    sf[l] = cv.take<int64_t>((size_t)n + 1);
  }
  int64_t* fl[kNumFlat];
  for (int f = 0; f < kNumFlat; ++f) fl[f] = cv.take<int64_t>((size_t)n + 1);
  int32_t* ctr = cv.take<int32_t>((size_t)kCtrCount);
  DevState* ds = cv.take<DevState>((size_t)n);
  if (b) {
    b->d_inst = di;
    for (int l = 0; l < kNumLists; ++l) {
      b->lists[l].d_seg_inst = si[l];
      b->lists[l].d_seg_first = sf[l];
    }
    for (int f = 0; f < kNumFlat; ++f) b->d_flat[f] = fl[f];
    b->ctr = ctr;
    b->d_states = ds;
  }
  for (int32_t i = 0; i < n; ++i) {
    char* ib = base ? base + cv.off : nullptr;
    const size_t sz = ctx_layout(Ne[i], Na[i], precision, batch_spec(Ne[i], Na[i]),
                                 b ? &b->ctx[(size_t)i] : nullptr, ib);
    cv.off += align_up(sz);
  }
  return cv.off;
}

// Items and cost per item of network c in grouped product `phase`.
void phase_items(const panda_ctx& c, int phase, int choice, int64_t* count, int64_t* cost) {
  int64_t bm, bn;
  switch (phase) {
    case kBTResp:
      rect_tile_shape(choice, &bm, &bn);
      *count = (c.Nep / bm) * (c.Nap / bn);
      *cost = c.Nep + 64;
      return;
    case kBTAvail:
      rect_tile_shape(choice, &bm, &bn);
      *count = (c.Nep / bm) * (c.Nap / bn);
      *cost = c.Nap + 64;
      return;
    case kBTCoop: {
      const int64_t chunk = coop_chunk_of(choice), T = c.Nep / kCoopTile;
      *count = T * (T + 1) / 2 * ((c.Nap + chunk - 1) / chunk);
      *cost = std::min(chunk, c.Nap);
      return;
    }
    default:
      *count = coreg_tiles(c.Nap);
      *cost = c.Nep + 256;
      return;
  }
}

// Work list of one grouped product: networks in decreasing cost per item
// (largest first), then eight queues of about equal total cost.
panda_status build_list(panda_batch* b, int phase) {
  const int32_t n = b->n;
  std::vector<int64_t> cnt((size_t)n), cost((size_t)n);
  for (int32_t i = 0; i < n; ++i)
    phase_items(b->ctx[(size_t)i], phase, b->tiles[phase], &cnt[(size_t)i], &cost[(size_t)i]);
  auto& L = b->lists[phase];
  L.seg_inst.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) L.seg_inst[(size_t)i] = i;
  std::stable_sort(L.seg_inst.begin(), L.seg_inst.end(),
                   [&](int32_t a, int32_t c) { return cost[(size_t)a] > cost[(size_t)c]; });
  L.seg_first.assign((size_t)n + 1, 0);
  double total_cost = 0.0;
  for (int32_t s = 0; s < n; ++s) {
    const int32_t i = L.seg_inst[(size_t)s];
    L.seg_first[(size_t)s + 1] = L.seg_first[(size_t)s] + cnt[(size_t)i];
    total_cost += (double)cnt[(size_t)i] * (double)cost[(size_t)i];
  }
  const int64_t total = L.seg_first[(size_t)n];
  // queue boundaries: item where the running cost first reaches x/8 of the total
  WorkList wl;
  wl.xb[0] = 0;
  wl.xb[kNumXcd] = total;
  int32_t s = 0;
  double before = 0.0;  // cost of segments before s
  for (int x = 1; x < kNumXcd; ++x) {
    const double target = total_cost * x / kNumXcd;
    while (s < n) {
      const int32_t i = L.seg_inst[(size_t)s];
      const double seg = (double)cnt[(size_t)i] * (double)cost[(size_t)i];
      if (before + seg >= target) break;
      before += seg;
      ++s;
    }
    int64_t item = total;
    if (s < n) {
      const int32_t i = L.seg_inst[(size_t)s];
      const int64_t k = (int64_t)((target - before) / (double)cost[(size_t)i]);
      item = L.seg_first[(size_t)s] + std::min(k, cnt[(size_t)i]);
    }
    wl.xb[x] = std::max(item, wl.xb[x - 1]);
  }
  wl.seg_inst = L.d_seg_inst;
  wl.seg_first = L.d_seg_first;
  wl.nseg = n;
  wl.ctr = b->ctr + (int64_t)phase * kNumXcd * kCtrStride;
  L.wl = wl;
  L.nb = batch_grid(phase, b->tiles[phase], b->rule.sigma_from_T != 0, b->b3);
  HIP_TRY(hipMemcpyAsync(L.d_seg_inst, L.seg_inst.data(), (size_t)n * sizeof(int32_t),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(L.d_seg_first, L.seg_first.data(), ((size_t)n + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return PANDA_OK;
}

// Device descriptors of all networks for the current tile choices.
panda_status upload_insts(panda_batch* b) {
  int64_t bm, bn;
  rect_tile_shape(b->tiles[kBTAvail], &bm, &bn);
  const int64_t chunk = coop_chunk_of(b->tiles[kBTCoop]);
  b->h_inst.resize((size_t)b->n);
  for (int32_t i = 0; i < b->n; ++i) {
    const panda_ctx& c = b->ctx[(size_t)i];
    BInst& d = b->h_inst[(size_t)i];
    d.Ne = c.Ne;
    d.Na = c.Na;
    d.Nep = c.Nep;
    d.Nap = c.Nap;
    d.W[0] = c.W[0];
    d.W[1] = c.W[1];
    d.R = c.R;
    d.P = c.P;
    d.C = c.C;
    d.Tside = c.Tside;
    d.ppart = c.ppart;
    d.dP = c.dP;
    d.dC = c.dC;
    d.nP = c.nP;
    d.nC = c.nC;
    d.nWr = c.nWr;
    d.nWc = c.nWc;
    d.colscr = c.colscr;
    d.hpart = c.hpart;
    d.cstat = c.cstat;
    d.csq = c.csq;
    d.corder = c.corder;
    d.st = c.st;
    d.Wh = c.Wh;
    d.Wl = c.Wl;
    d.Wth = c.Wth;
    d.Wtl = c.Wtl;
    d.Ph = c.Ph;
    d.Pl = c.Pl;
    d.nh = (c.Nep / bm) * (c.Nap / bn);
    d.chunk = chunk;
    d.splits = (c.Nap + chunk - 1) / chunk;
  }
  HIP_TRY(hipMemcpyAsync(b->d_inst, b->h_inst.data(), (size_t)b->n * sizeof(BInst),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return PANDA_OK;
}

// Flat grids (network order): blocks per network of each element phase.
panda_status build_flat(panda_batch* b) {
  const int32_t n = b->n;
  for (int f = 0; f < kNumFlat; ++f) b->h_flat[f].assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    const panda_ctx& c = b->ctx[(size_t)i];
    const int64_t gx = (c.Na + upd::kUT - 1) / upd::kUT;
    const int64_t cnt[kNumFlat] = {c.Ne + gx * upd::col_chunks(c.Ne), gx,
                                   (c.Ne * c.Ne + upd::kUT - 1) / upd::kUT, c.Ne + gx,
                                   b->b3 ? (c.Nep / 64) * (c.Nap / 64) : 0};
    for (int f = 0; f < kNumFlat; ++f)
      b->h_flat[f][(size_t)i + 1] = b->h_flat[f][(size_t)i] + cnt[f];
  }
  for (int f = 0; f < kNumFlat; ++f) {
    if (b->h_flat[f][(size_t)n] >= ((int64_t)1 << 31))
      return fail(PANDA_ERR_ARG, "batch: grid too large%s");
    b->flat[f] = FlatList{b->d_flat[f], n, b->h_flat[f][(size_t)n]};
    HIP_TRY(hipMemcpyAsync(b->d_flat[f], b->h_flat[f].data(), ((size_t)n + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, b->stream));
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  return PANDA_OK;
}

panda_status launch_phase(panda_batch* b, int phase, hipStream_t s) {
  const auto& L = b->lists[phase];
  switch (phase) {
    case kBTResp:
      HIP_TRY(launch_batch_resp(b->tiles[phase], b->b3, b->d_inst, L.wl, L.nb, s));
      break;
    case kBTAvail:
      HIP_TRY(launch_batch_avail(b->tiles[phase], b->b3, b->d_inst, L.wl, b->rule, L.nb, s));
      break;
    case kBTCoop: HIP_TRY(launch_batch_coop_partial(b->b3, b->d_inst, L.wl, L.nb, s)); break;
    default:
      HIP_TRY(launch_batch_coreg(b->tiles[phase], b->b3, b->d_inst, L.wl, b->rule, L.nb, s));
  }
  return PANDA_OK;
}

// One iteration of every network: R, A + W, h, norms, P, C, diagonals.
// Only kernel launches, so the sequence can be captured in a graph.
panda_status enqueue_batch_iteration(panda_batch* b, hipStream_t s) {
  HIP_TRY(launch_batch_reset(b->ctr, kCtrCount, s));
  PANDA_TRY(launch_phase(b, kBTResp, s));
  PANDA_TRY(launch_phase(b, kBTAvail, s));
  HIP_TRY(launch_batch_finish_h(b->d_inst, b->n, b->rule, s));
  HIP_TRY(launch_batch_norms(b->d_inst, b->flat[kFlatPart], b->flat[kFlatSum], s));
  if (b->b3) HIP_TRY(launch_batch_planes(b->d_inst, b->flat[kFlatPlanes], s));
  PANDA_TRY(launch_phase(b, kBTCoop, s));
  HIP_TRY(launch_batch_coop_finalize(b->d_inst, b->flat[kFlatPfin], b->rule, s));
  PANDA_TRY(launch_phase(b, kBTCoreg, s));
  HIP_TRY(launch_batch_diagonals(b->d_inst, b->flat[kFlatDiag], b->rule, s));
  return PANDA_OK;
}

void drop_graph(panda_batch* b) {
  if (b->have_graph) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
  }
  b->have_graph = false;
}

panda_status capture_graph(panda_batch* b) {
  drop_graph(b);
  if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  panda_status st = enqueue_batch_iteration(b, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (st != PANDA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graph = g;
  b->have_graph = true;
  return PANDA_OK;
}

panda_status gather_states(panda_batch* b) {
  HIP_TRY(launch_batch_gather(b->d_inst, b->n, b->d_states, b->stream));
  HIP_TRY(hipMemcpyAsync(b->h_states, b->d_states, (size_t)b->n * sizeof(DevState),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return PANDA_OK;
}

panda_status apply_tiles(panda_batch* b) {
  for (int l = 0; l < kNumLists; ++l) PANDA_TRY(build_list(b, l));
  PANDA_TRY(upload_insts(b));
  drop_graph(b);
  return PANDA_OK;
}

panda_status check_shapes(int32_t n, const int64_t* Ne, const int64_t* Na) {
  if (n < 1 || n > kMaxBatch || !Ne || !Na) return fail(PANDA_ERR_ARG, "batch: bad count%s");
  for (int32_t i = 0; i < n; ++i)
    if (!dims_ok(Ne[i], Na[i])) return fail(PANDA_ERR_ARG, "batch: bad dimensions%s");
  return PANDA_OK;
}

}  // namespace

extern "C" {

size_t panda_batch_workspace_bytes(int32_t n, const int64_t* Ne, const int64_t* Na,
                                   const panda_options* opt) {
  if (check_shapes(n, Ne, Na) != PANDA_OK) return 0;
  return batch_layout(n, Ne, Na, opt ? opt->precision : PANDA_PREC_FP32, nullptr, nullptr);
}

panda_status panda_batch_create(int32_t n, const int64_t* Ne, const int64_t* Na,
                                const panda_options* opt, void* workspace, size_t ws_bytes,
                                hipStream_t stream, panda_batch** out) {
  if (!out) return fail(PANDA_ERR_ARG, "batch_create: out is NULL%s");
  *out = nullptr;
  PANDA_TRY(check_shapes(n, Ne, Na));
  panda_options o;
  if (opt)
    o = *opt;
  else
    panda_default_options(&o);
  PANDA_TRY(check_options(o));
  if (!workspace || ws_bytes < batch_layout(n, Ne, Na, o.precision, nullptr, nullptr) ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(PANDA_ERR_WORKSPACE, "batch_create: workspace too small or misaligned%s");
  panda_batch* b = new (std::nothrow) panda_batch();
  if (!b) return fail(PANDA_ERR_ARG, "batch_create: out of host memory%s");
  b->n = n;
  b->opt = o;
  b->rule = rule_of(o);
  b->stream = stream;
  b->b3 = o.precision == PANDA_PREC_BF16X3;
  b->ctx.resize((size_t)n);
  batch_layout(n, Ne, Na, o.precision, b, static_cast<char*>(workspace));
  panda_status st = PANDA_OK;
  for (int32_t i = 0; i < n && st == PANDA_OK; ++i) {
    char* ib = reinterpret_cast<char*>(b->ctx[(size_t)i].W[0]);  // start of network i's region
    st = ctx_setup(&b->ctx[(size_t)i], Ne[i], Na[i], o, batch_spec(Ne[i], Na[i]), ib, stream);
  }
  if (st == PANDA_OK) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_states),
                                 (size_t)n * sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess) st = hip_fail(e, "hipHostMalloc");
  }
  for (int32_t i = 0; i < n && st == PANDA_OK; ++i) st = ctx_fill_order(&b->ctx[(size_t)i]);
  if (st == PANDA_OK) st = build_flat(b);
  if (st == PANDA_OK) st = apply_tiles(b);
  if (st != PANDA_OK) {
    panda_batch_destroy(b);
    return st;
  }
  *out = b;
  return PANDA_OK;
}

void panda_batch_destroy(panda_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->h_states) (void)hipHostFree(b->h_states);
  for (auto& c : b->ctx) ctx_free(&c);
  delete b;
}

int32_t panda_batch_tile_candidates(int32_t phase) {
  return (phase >= 0 && phase < kBTNum) ? batch_tile_candidates(phase) : 0;
}

panda_status panda_batch_get_tiles(const panda_batch* b, int32_t* choice) {
  if (!b || !choice) return fail(PANDA_ERR_ARG, "batch_get_tiles: NULL argument%s");
  for (int l = 0; l < kNumLists; ++l) choice[l] = b->tiles[l];
  return PANDA_OK;
}

panda_status panda_batch_set_tiles(panda_batch* b, const int32_t* choice) {
  if (!b || !choice) return fail(PANDA_ERR_ARG, "batch_set_tiles: NULL argument%s");
  for (int l = 0; l < kNumLists; ++l)
    if (choice[l] < 0 || choice[l] >= batch_tile_candidates(l, b->b3))
      return fail(PANDA_ERR_ARG, "batch_set_tiles: choice out of range%s");
  for (int l = 0; l < kNumLists; ++l) b->tiles[l] = choice[l];
  return apply_tiles(b);
}

panda_status panda_batch_autotune(panda_batch* b, int32_t reps, float* best_ms) {
  if (!b || reps < 1) return fail(PANDA_ERR_ARG, "batch_autotune: bad arguments%s");
  hipStream_t s = b->stream;
  // zero state: every network's region (the order tables are written again)
  for (auto& c : b->ctx) {
    const size_t bytes = ctx_layout(c.Ne, c.Na, b->opt.precision, batch_spec(c.Ne, c.Na), nullptr,
                                    nullptr);
    HIP_TRY(hipMemsetAsync(c.W[0], 0, bytes, s));
    c.loaded = false;
  }
  for (auto& c : b->ctx) PANDA_TRY(ctx_fill_order(&c));
  PANDA_TRY(upload_insts(b));
  HIP_TRY(launch_batch_gates(b->d_inst, b->n, 1, 1, s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  panda_status st = PANDA_OK;
  for (int phase = 0; phase < kNumLists && st == PANDA_OK; ++phase) {
    float best = 1e30f;
    int bestc = 0;
    for (int c = 0; c < batch_tile_candidates(phase, b->b3) && st == PANDA_OK; ++c) {
      b->tiles[phase] = c;
      st = build_list(b, phase);
      if (st == PANDA_OK) st = upload_insts(b);
      float tmin = 1e30f;
      for (int r = 0; r <= reps && st == PANDA_OK; ++r) {  // r = 0 warms up
        if (hipSuccess != launch_batch_reset(b->ctr, kCtrCount, s) ||
            hipSuccess != hipEventRecord(e0, s)) {
          st = fail(PANDA_ERR_HIP, "batch_autotune: launch failed%s");
          break;
        }
        st = launch_phase(b, phase, s);
        if (st != PANDA_OK) break;
        float ms = 0.0f;
        if (hipSuccess != hipEventRecord(e1, s) || hipSuccess != hipEventSynchronize(e1) ||
            hipSuccess != hipEventElapsedTime(&ms, e0, e1)) {
          st = fail(PANDA_ERR_HIP, "batch_autotune: timing failed%s");
          break;
        }
        if (r > 0) tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        bestc = c;
      }
    }
    b->tiles[phase] = bestc;
    if (best_ms) best_ms[phase] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PANDA_OK) return st;
  return apply_tiles(b);
}

panda_status panda_batch_load(panda_batch* b, int32_t i, const float* W, const float* P,
                              const float* C, int32_t t) {
  if (!b || i < 0 || i >= b->n) return fail(PANDA_ERR_ARG, "batch_load: bad network index%s");
  return panda_ctx_load(&b->ctx[(size_t)i], W, P, C, t);
}

panda_status panda_batch_iterate(panda_batch* b, int32_t steps, int32_t use_graph,
                                 int32_t* active) {
  if (!b || steps < 0) return fail(PANDA_ERR_ARG, "batch_iterate: bad arguments%s");
  for (const auto& c : b->ctx)
    if (!c.loaded) return fail(PANDA_ERR_ARG, "batch_iterate: a network is not loaded%s");
  if (use_graph && steps > 0 && !b->have_graph) PANDA_TRY(capture_graph(b));
  for (int32_t k = 0; k < steps; ++k) {
    if (use_graph)
      HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    else
      PANDA_TRY(enqueue_batch_iteration(b, b->stream));
  }
  PANDA_TRY(gather_states(b));
  if (active) {
    int32_t a = 0;
    for (int32_t i = 0; i < b->n; ++i) a += b->h_states[i].active != 0;
    *active = a;
  }
  return PANDA_OK;
}

panda_status panda_batch_run(panda_batch* b, int32_t use_graph, int32_t* steps) {
  if (!b) return fail(PANDA_ERR_ARG, "batch_run: NULL batch%s");
  int32_t done = 0, active = b->n;
  while (active > 0 && done < b->opt.max_iter) {
    const int32_t k = std::min(b->opt.poll_every, b->opt.max_iter - done);
    PANDA_TRY(panda_batch_iterate(b, k, use_graph, &active));
    done += k;
  }
  if (steps) *steps = done;
  return active == 0 ? PANDA_OK : PANDA_NOT_CONVERGED;
}

panda_status panda_batch_state(const panda_batch* b, int32_t i, double* h, int32_t* t,
                               int32_t* active) {
  if (!b || i < 0 || i >= b->n) return fail(PANDA_ERR_ARG, "batch_state: bad network index%s");
  const DevState& s = b->h_states[i];
  if (h) *h = s.h;
  if (t) *t = s.t;
  if (active) *active = s.active;
  return PANDA_OK;
}

panda_status panda_batch_store(panda_batch* b, int32_t i, float* W, float* P, float* C,
                               double* h, int32_t* t) {
  if (!b || i < 0 || i >= b->n) return fail(PANDA_ERR_ARG, "batch_store: bad network index%s");
  return panda_ctx_store(&b->ctx[(size_t)i], W, P, C, h, t);
}

}  // extern "C"
