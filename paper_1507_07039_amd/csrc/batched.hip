// Grouped kernels of the batched form: every phase of one PANDA iteration
// (Sec. II-B) runs for all networks of a batch in one launch.
//
// The four similarity products (R, A + W, W W^T partials, C update) are
// persistent kernels over a work list of (network, tile) items.  The list is
// cut into eight queues of about equal cost, one per XCD; a block takes items
// from its own XCD's queue (consecutive items share operand strips in that
// XCD's L2) and then from the other queues, so uneven networks balance out.
// Each item is computed whole by one block with the same tile code and
// epilogues as the single-network form, and the split-K partials of W W^T go
// to fixed slots, so results do not depend on which block took which item.
// Networks whose gate is closed (converged: Eq. 7 below tol) skip their items.
// The element-wise phases are flat grids over all networks.
#include "batch_internal.h"
#include "epilogues.h"
#include "update_device.h"

namespace panda {
namespace {

using namespace gemm;

// Candidate tilings (index = autotuner choice).
using RectT0 = BlockGemm<64, 128, 1, 4, true, false, 16>;
using RectT1 = BlockGemm<64, 64, 2, 2, true, false, 16>;
using RectT2 = BlockGemm<64, 128, 2, 2, true, false, 16>;
using SymT0 = BlockGemm<128, 128, 2, 2, false, false, 16>;
using SymT1 = BlockGemm<128, 128, 2, 2, false, false, 32>;
using SymT2 = BlockGemm<128, 128, 1, 4, false, false, 16>;
using CoopT = BlockGemm<64, 64, 2, 2, true, true, 32>;
constexpr int64_t kCoopChunks[4] = {512, 1024, 2048, 4096};
// Split-BF16 batches: the tilings of candidate 0 on the split-BF16 block
// GEMMs of the single-network form (R register-staged; A + W with direct
// loads and C split as it is read, 64 x 128 so that the item lists are those
// of candidate 0; W W^T and the C update as in the single-network form).
using RectB3A = BlockGemmB3P<64, 128, 1, 4, true, 3>;
static_assert(RectB3::BM == RectT0::BM && RectB3::BN == RectT0::BN &&
                  RectB3A::BM == RectT0::BM && RectB3A::BN == RectT0::BN &&
                  SymB3::BM == SymT0::BM && CoopB3::BM == CoopT::BM && CoopB3::BK == CoopT::BK,
              "split-BF16 tiles share the work lists of candidate 0");

// Largest s with seg_first[s] <= it.
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ first, int nseg,
                                            int64_t it) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// --------------------------------------------------------------- phases --
// R = T(P, W) (Eq. 3) for one tile.  B3: split-BF16 products on the planes
// of P and of W^T.
template <bool B3>
struct PhResp {
  template <class G>
  static constexpr int smem_bytes() { return G::MAIN_BYTES; }
  template <class G>
  __device__ __forceinline__ void run(const BInst& d, int64_t local, char* smem, double*) const {
    const DevState* st = d.st;
    if (st->active == 0) return;
    const float* W = d.W[st->wsel];
    const int64_t nMT = d.Nep / G::BM;
    const int64_t m0 = (local % nMT) * G::BM, n0 = (local / nMT) * G::BN;
    G g;
    if constexpr (B3)
      g.run(OpsB3{d.Ph, d.Pl, d.Nep, d.Wth, d.Wtl, d.Nep}, m0, n0, 0, d.Nep, smem);
    else
      g.run(OpsF32{d.P, d.Nep, W, d.Nap}, m0, n0, 0, d.Nep, smem);
    EpiStoreT epi{d.R, d.Nap, d.Ne, d.Na, d.nP, d.nWc, d.dP, W, d.Nap};
    epi_tile(g, epi, m0, n0);
  }
};

// A = T(W, C) (Eq. 4) fused with the W update (Eq. 2) and the tile's h
// partial (Eq. 7).  B3: W's planes against C split as it is read.
template <bool B3>
struct PhAvail {
  double alpha;
  int32_t h_undamped;
  template <class G>
  static constexpr int smem_bytes() { return G::MAIN_BYTES; }
  template <class G>
  __device__ __forceinline__ void run(const BInst& d, int64_t local, char* smem,
                                      double* red) const {
    const DevState* st = d.st;
    if (st->active == 0) return;
    const int ws = st->wsel;
    const float* Wold = d.W[ws];
    const int64_t nMT = d.Nep / G::BM;
    const int64_t m0 = (local % nMT) * G::BM, n0 = (local / nMT) * G::BN;
    G g;
    if constexpr (B3)
      g.run(OpsB3F{d.Wh, d.Wl, d.Nap, d.C, d.Nap, d.Nep}, m0, n0, 0, d.Nap, smem);
    else
      g.run(OpsF32{Wold, d.Nap, d.C, d.Nap}, m0, n0, 0, d.Nap, smem);
    EpiWUpdate epi{Wold, d.R,   d.W[ws ^ 1], d.Nap, d.Ne,       d.Na,    d.nWr,
                   d.nC, d.dC,  alpha,       h_undamped, d.hpart, 0.0};
    epi_tile(g, epi, m0, n0);
    epi.end_tile(local, red);
  }
};

// W W^T partial product of one upper 64 x 64 tile over one K chunk (first
// half of the P update, Eq. 5).  B3: on W's planes.
template <bool B3>
struct PhCoop {
  template <class G>
  static constexpr int smem_bytes() { return G::MAIN_BYTES; }
  template <class G>
  __device__ __forceinline__ void run(const BInst& d, int64_t local, char* smem, double*) const {
    const DevState* st = d.st;
    if (st->run_pc == 0) return;
    const float* W = d.W[st->wsel];
    const int64_t T = d.Nep / kPB, nU = T * (T + 1) / 2;
    const int64_t u = local % nU, sp = local / nU;
    int64_t I, J;
    tri_tile(u, I, J);
    const int64_t m0 = I * kPB, n0 = J * kPB;
    int64_t kb = sp * d.chunk, ke = kb + d.chunk;
    if (ke > d.Nap) ke = d.Nap;
    G g;
    if constexpr (B3)
      g.run(OpsB3{d.Wh, d.Wl, d.Nap, d.Wh, d.Wl, d.Nap}, m0, n0, kb, ke, smem);
    else
      g.run(OpsF32{W, d.Nap, W, d.Nap}, m0, n0, kb, ke, smem);
    float* ps = d.ppart + sp * d.Nep * d.Nep;
    g.for_each([&](int r, int c, float v) { ps[(m0 + r) * d.Nep + n0 + c] = v; });
  }
};

// C update (Eq. 5) of one upper 128 x 128 tile, mirrored, with the row sums
// for the sigma of Eq. 6.  B3: on the planes of W^T.
template <bool SIGT, bool B3>
struct PhCoreg {
  double alpha;
  template <class G>
  static constexpr int smem_bytes() { return coreg_smem_bytes<G, SIGT>(); }
  template <class G>
  __device__ __forceinline__ void run(const BInst& d, int64_t local, char* smem, double*) const {
    const DevState* st = d.st;
    if (st->run_pc == 0) return;
    const float* W = d.W[st->wsel];
    const uint32_t ij = d.corder[local];
    const int64_t I = ij & 0xffff, J = ij >> 16;
    const double nval = coreg_norm_load(d.nWc, I, J, d.Na);
    G g;
    if constexpr (B3)
      g.run(OpsB3{d.Wth, d.Wtl, d.Nep, d.Wth, d.Wtl, d.Nep}, I * kCB, J * kCB, 0, d.Nep, smem);
    else
      g.run(OpsF32{W, d.Nap, W, d.Nap}, I * kCB, J * kCB, 0, d.Nep, smem);
    coreg_epilogue<SIGT, false>(g, smem, I, J, d.C, d.Nap, d.Na, nval, alpha, d.cstat, d.csq, d.Nap);
  }
};

// Persistent grouped product: blocks drain the per-XCD queues, their own
// first.  Every block exits once all eight queues are empty.
template <class G, class Ph>
__global__ __launch_bounds__(G::NT) void k_group_gemm(const BInst* __restrict__ bi, WorkList wl,
                                                      Ph ph) {
  __shared__ __align__(16) char smem[Ph::template smem_bytes<G>()];
  __shared__ double red[8];
  __shared__ int64_t s_item;
  const int x0 = (int)(blockIdx.x % kNumXcd);
  for (int v = 0; v < kNumXcd; ++v) {
    const int x = (x0 + v) % kNumXcd;
    const int64_t beg = wl.xb[x], end = wl.xb[x + 1];
    if (beg >= end) continue;
    for (;;) {
      __syncthreads();  // the previous item is done with smem and s_item
      if (threadIdx.x == 0) s_item = beg + (int64_t)atomicAdd(wl.ctr + x * kCtrStride, 1);
      __syncthreads();
      const int64_t it = s_item;
      if (it >= end) break;
      const int seg = find_segment(wl.seg_first, wl.nseg, it);
      ph.template run<G>(bi[wl.seg_inst[seg]], it - wl.seg_first[seg], smem, red);
    }
  }
}

// ------------------------------------------------------ element phases --
constexpr int kUT = upd::kUT;

__global__ __launch_bounds__(kUT) void k_batch_finish_h(const BInst* __restrict__ bi, double tol,
                                                        int32_t update_last) {
  __shared__ double red[4];
  const BInst& d = bi[blockIdx.x];
  upd::finish_h(d.hpart, d.nh, d.Ne * d.Na, d.st, tol, update_last, red);
}

// Squared norms of the new W, first pass: blocks [0, Ne) are rows of W,
// the rest are (row chunk, group of 256 columns) partial column sums with the
// same chunking as the single-network form.
__global__ __launch_bounds__(kUT) void k_batch_norms_part(const BInst* __restrict__ bi,
                                                          FlatList fl) {
  __shared__ double red[4];
  const int seg = find_segment(fl.seg_first, fl.nseg, blockIdx.x);
  const BInst& d = bi[seg];
  const DevState* st = d.st;
  if (st->run_pc == 0) return;
  const float* W = d.W[st->wsel];
  int64_t q = (int64_t)blockIdx.x - fl.seg_first[seg];
  if (q < d.Ne) {
    const double tot = upd::row_sqnorm(W + q * d.Nap, d.Na, red);
    if (threadIdx.x == 0) d.nWr[q] = tot;
    return;
  }
  q -= d.Ne;
  const int64_t gx = (d.Na + kUT - 1) / kUT;
  const int64_t ch = q / gx, j = (q % gx) * kUT + threadIdx.x;
  if (j >= d.Na) return;
  const int nch = upd::col_chunks(d.Ne);
  const int64_t chunk = (d.Ne + nch - 1) / nch;
  const int64_t r0 = ch * chunk;
  const int64_t r1 = r0 + chunk < d.Ne ? r0 + chunk : d.Ne;
  d.colscr[ch * d.Na + j] = upd::col_sqnorm_part(W, d.Nap, j, r0, r1);
}

__global__ __launch_bounds__(kUT) void k_batch_norms_sum(const BInst* __restrict__ bi,
                                                         FlatList fl) {
  const int seg = find_segment(fl.seg_first, fl.nseg, blockIdx.x);
  const BInst& d = bi[seg];
  if (d.st->run_pc == 0) return;
  const int64_t j = ((int64_t)blockIdx.x - fl.seg_first[seg]) * kUT + threadIdx.x;
  if (j >= d.Na) return;
  const int nch = upd::col_chunks(d.Ne);
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += d.colscr[(int64_t)c * d.Na + j];
  d.nWc[j] = s;
}

// bf16 planes of the new W, one 64 x 64 tile per block: row-major (read
// along rows) and, through LDS, gene-major (written along its rows).  Only
// the real Ne x Na region is written; the padding stays zero from the load.
__global__ __launch_bounds__(kUT) void k_batch_planes(const BInst* __restrict__ bi, FlatList fl) {
  __shared__ float tile[64][65];
  const int seg = find_segment(fl.seg_first, fl.nseg, blockIdx.x);
  const BInst& d = bi[seg];
  if (d.st->run_pc == 0) return;
  const float* W = d.W[d.st->wsel];
  const int64_t q = (int64_t)blockIdx.x - fl.seg_first[seg], nbx = d.Nap / 64;
  const int64_t r0 = (q / nbx) * 64, c0 = (q % nbx) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += kUT / 64) {
    const int64_t r = r0 + rr, c = c0 + tx;
    float v = 0.0f;
    if (r < d.Ne && c < d.Na) {
      v = W[r * d.Nap + c];
      bf16_t h, l;
      upd::split_bf16(v, h, l);
      d.Wh[r * d.Nap + c] = h;
      d.Wl[r * d.Nap + c] = l;
    }
    tile[rr][tx] = v;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += kUT / 64) {
    const int64_t c = c0 + cc, r = r0 + tx;
    if (r < d.Ne && c < d.Na) {
      bf16_t h, l;
      upd::split_bf16(tile[tx][cc], h, l);
      d.Wth[c * d.Nep + r] = h;
      d.Wtl[c * d.Nep + r] = l;
    }
  }
}

__global__ __launch_bounds__(kUT) void k_batch_coop_finalize(const BInst* __restrict__ bi,
                                                             FlatList fl, double alpha,
                                                             int32_t sigma_from_T) {
  const int seg = find_segment(fl.seg_first, fl.nseg, blockIdx.x);
  const BInst& d = bi[seg];
  if (d.st->run_pc == 0) return;
  const int64_t e = ((int64_t)blockIdx.x - fl.seg_first[seg]) * kUT + threadIdx.x;
  upd::coop_finalize_entry(e, d.ppart, (int)d.splits, d.Nep, d.nWr, d.P, d.Nep, d.Ne, alpha,
                           sigma_from_T ? d.Tside : nullptr, d.Ph, d.Pl);
}

// Eq. 6: blocks [0, Ne) are rows of P, the rest cover the rows of C, one
// thread each.
__global__ __launch_bounds__(kUT) void k_batch_diagonals(const BInst* __restrict__ bi,
                                                         FlatList fl, double alpha,
                                                         int32_t diag_alpha, int32_t n_own,
                                                         int32_t sigma_from_T, int32_t ddof) {
  __shared__ double red[4];
  const int seg = find_segment(fl.seg_first, fl.nseg, blockIdx.x);
  const BInst& d = bi[seg];
  const DevState* st = d.st;
  if (st->run_pc == 0) return;
  const upd::DiagRule dr = upd::diag_rule(alpha, diag_alpha, n_own, ddof, st->t);
  const int64_t q = (int64_t)blockIdx.x - fl.seg_first[seg];
  if (q < d.Ne) {
    upd::diag_p_row(q, d.P, d.Nep, d.dP, d.Ne, d.Na, sigma_from_T ? d.Tside : nullptr, d.nP, dr,
                    red);
    return;
  }
  const int64_t r = (q - d.Ne) * kUT + threadIdx.x;
  if (r < d.Na)
    upd::diag_c_row(r, d.dC, d.Nap, d.Ne, d.Na, d.cstat, sigma_from_T ? d.csq : nullptr,
                    d.Nap / kCB, d.nC, dr);
}

__global__ __launch_bounds__(kUT) void k_batch_reset(int32_t* ctr, int64_t count) {
  for (int64_t i = threadIdx.x; i < count; i += kUT) ctr[i] = 0;
}

__global__ __launch_bounds__(kUT) void k_batch_gather(const BInst* __restrict__ bi, int32_t n,
                                                      DevState* out) {
  const int64_t i = (int64_t)blockIdx.x * kUT + threadIdx.x;
  if (i < n) out[i] = *bi[i].st;
}

__global__ __launch_bounds__(kUT) void k_batch_gates(const BInst* __restrict__ bi, int32_t n,
                                                     int32_t active, int32_t run_pc) {
  const int64_t i = (int64_t)blockIdx.x * kUT + threadIdx.x;
  if (i < n) {
    bi[i].st->active = active;
    bi[i].st->run_pc = run_pc;
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kUT - 1) / kUT); }

template <class G, class Ph>
hipError_t group_launch(const BInst* bi, const WorkList& wl, const Ph& ph, int64_t nb,
                        hipStream_t s) {
  if (wl.xb[kNumXcd] == 0) return hipSuccess;
  k_group_gemm<G, Ph><<<dim3((unsigned)nb), dim3(G::NT), 0, s>>>(bi, wl, ph);
  return hipGetLastError();
}

template <class G, class Ph>
int64_t group_grid() {
  // computed once per kernel (a function-local static: thread-safe initialisation)
  static const int64_t nb =
      resident_blocks(reinterpret_cast<const void*>(&k_group_gemm<G, Ph>), G::NT);
  return nb;
}

}  // namespace

// ------------------------------------------------------------ launchers --

int batch_tile_candidates(int phase, bool b3) {
  switch (phase) {
    case kBTResp:
    case kBTAvail:
    case kBTCoreg: return b3 ? 1 : 3;
    case kBTCoop: return 4;
  }
  return 0;
}

void rect_tile_shape(int choice, int64_t* bm, int64_t* bn) {
  switch (choice) {
    case 1: *bm = RectT1::BM; *bn = RectT1::BN; return;
    case 2: *bm = RectT2::BM; *bn = RectT2::BN; return;
    default: *bm = RectT0::BM; *bn = RectT0::BN; return;
  }
}

int64_t coop_chunk_of(int choice) { return kCoopChunks[choice < 0 || choice > 3 ? 0 : choice]; }

int64_t batch_grid(int phase, int choice, bool sigT, bool b3) {
  if (b3) {
    switch (phase) {
      case kBTResp: return group_grid<RectB3, PhResp<true>>();
      case kBTAvail: return group_grid<RectB3A, PhAvail<true>>();
      case kBTCoop: return group_grid<CoopB3, PhCoop<true>>();
      case kBTCoreg:
        return sigT ? group_grid<SymB3, PhCoreg<true, true>>()
                    : group_grid<SymB3, PhCoreg<false, true>>();
    }
    return 0;
  }
  switch (phase) {
    case kBTResp:
      if (choice == 1) return group_grid<RectT1, PhResp<false>>();
      if (choice == 2) return group_grid<RectT2, PhResp<false>>();
      return group_grid<RectT0, PhResp<false>>();
    case kBTAvail:
      if (choice == 1) return group_grid<RectT1, PhAvail<false>>();
      if (choice == 2) return group_grid<RectT2, PhAvail<false>>();
      return group_grid<RectT0, PhAvail<false>>();
    case kBTCoop: return group_grid<CoopT, PhCoop<false>>();
    case kBTCoreg:
      if (sigT) {
        if (choice == 1) return group_grid<SymT1, PhCoreg<true, false>>();
        if (choice == 2) return group_grid<SymT2, PhCoreg<true, false>>();
        return group_grid<SymT0, PhCoreg<true, false>>();
      }
      if (choice == 1) return group_grid<SymT1, PhCoreg<false, false>>();
      if (choice == 2) return group_grid<SymT2, PhCoreg<false, false>>();
      return group_grid<SymT0, PhCoreg<false, false>>();
  }
  return 0;
}

hipError_t launch_batch_resp(int choice, bool b3, const BInst* bi, const WorkList& wl, int64_t nb,
                             hipStream_t s) {
  if (b3) return group_launch<RectB3>(bi, wl, PhResp<true>{}, nb, s);
  if (choice == 1) return group_launch<RectT1>(bi, wl, PhResp<false>{}, nb, s);
  if (choice == 2) return group_launch<RectT2>(bi, wl, PhResp<false>{}, nb, s);
  return group_launch<RectT0>(bi, wl, PhResp<false>{}, nb, s);
}

hipError_t launch_batch_avail(int choice, bool b3, const BInst* bi, const WorkList& wl, Rule rule,
                              int64_t nb, hipStream_t s) {
  if (b3) return group_launch<RectB3A>(bi, wl, PhAvail<true>{rule.alpha, rule.h_undamped}, nb, s);
  const PhAvail<false> ph{rule.alpha, rule.h_undamped};
  if (choice == 1) return group_launch<RectT1>(bi, wl, ph, nb, s);
  if (choice == 2) return group_launch<RectT2>(bi, wl, ph, nb, s);
  return group_launch<RectT0>(bi, wl, ph, nb, s);
}

hipError_t launch_batch_coop_partial(bool b3, const BInst* bi, const WorkList& wl, int64_t nb,
                                     hipStream_t s) {
  if (b3) return group_launch<CoopB3>(bi, wl, PhCoop<true>{}, nb, s);
  return group_launch<CoopT>(bi, wl, PhCoop<false>{}, nb, s);
}

hipError_t launch_batch_coreg(int choice, bool b3, const BInst* bi, const WorkList& wl, Rule rule,
                              int64_t nb, hipStream_t s) {
  if (b3) {
    if (rule.sigma_from_T)
      return group_launch<SymB3>(bi, wl, PhCoreg<true, true>{rule.alpha}, nb, s);
    return group_launch<SymB3>(bi, wl, PhCoreg<false, true>{rule.alpha}, nb, s);
  }
  if (rule.sigma_from_T) {
    const PhCoreg<true, false> ph{rule.alpha};
    if (choice == 1) return group_launch<SymT1>(bi, wl, ph, nb, s);
    if (choice == 2) return group_launch<SymT2>(bi, wl, ph, nb, s);
    return group_launch<SymT0>(bi, wl, ph, nb, s);
  }
  const PhCoreg<false, false> ph{rule.alpha};
  if (choice == 1) return group_launch<SymT1>(bi, wl, ph, nb, s);
  if (choice == 2) return group_launch<SymT2>(bi, wl, ph, nb, s);
  return group_launch<SymT0>(bi, wl, ph, nb, s);
}

hipError_t launch_batch_planes(const BInst* bi, const FlatList& fl, hipStream_t s) {
  if (fl.total == 0) return hipSuccess;
  k_batch_planes<<<dim3((unsigned)fl.total), dim3(kUT), 0, s>>>(bi, fl);
  return hipGetLastError();
}

hipError_t launch_batch_finish_h(const BInst* bi, int32_t n, Rule rule, hipStream_t s) {
  k_batch_finish_h<<<dim3((unsigned)n), dim3(kUT), 0, s>>>(bi, rule.tol, rule.update_last);
  return hipGetLastError();
}

hipError_t launch_batch_norms(const BInst* bi, const FlatList& part, const FlatList& sum,
                              hipStream_t s) {
  k_batch_norms_part<<<dim3((unsigned)part.total), dim3(kUT), 0, s>>>(bi, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_batch_norms_sum<<<dim3((unsigned)sum.total), dim3(kUT), 0, s>>>(bi, sum);
  return hipGetLastError();
}

hipError_t launch_batch_coop_finalize(const BInst* bi, const FlatList& fl, Rule rule,
                                      hipStream_t s) {
  k_batch_coop_finalize<<<dim3((unsigned)fl.total), dim3(kUT), 0, s>>>(bi, fl, rule.alpha,
                                                                        rule.sigma_from_T);
  return hipGetLastError();
}

hipError_t launch_batch_diagonals(const BInst* bi, const FlatList& fl, Rule rule, hipStream_t s) {
  k_batch_diagonals<<<dim3((unsigned)fl.total), dim3(kUT), 0, s>>>(
      bi, fl, rule.alpha, rule.diag_alpha, rule.n_own, rule.sigma_from_T, rule.sigma_ddof);
  return hipGetLastError();
}

hipError_t launch_batch_reset(int32_t* ctr, int64_t count, hipStream_t s) {
  k_batch_reset<<<1, kUT, 0, s>>>(ctr, count);
  return hipGetLastError();
}

hipError_t launch_batch_gather(const BInst* bi, int32_t n, DevState* out, hipStream_t s) {
  k_batch_gather<<<dim3(blocks_for(n)), dim3(kUT), 0, s>>>(bi, n, out);
  return hipGetLastError();
}

hipError_t launch_batch_gates(const BInst* bi, int32_t n, int32_t active, int32_t run_pc,
                              hipStream_t s) {
  k_batch_gates<<<dim3(blocks_for(n)), dim3(kUT), 0, s>>>(bi, n, active, run_pc);
  return hipGetLastError();
}

}  // namespace panda
