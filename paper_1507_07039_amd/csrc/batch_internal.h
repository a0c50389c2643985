// Device-side description of a batch of independent networks and the
// launchers of the grouped kernels that iterate all of them together.
#pragma once

#include "panda_internal.h"

namespace panda {

// One network of a batch, as the grouped kernels see it (device memory).
// Every pointer is into that network's own workspace region; the current W
// is W[st->wsel].
struct BInst {
  int64_t Ne, Na, Nep, Nap;
  float* W[2];
  float* R;
  float* P;
  float* C;
  float* Tside;
  float* ppart;
  double* dP;  // diagonals of P and C (FP64; zero in the matrices)
  double* dC;
  double* nP;
  double* nC;
  double* nWr;
  double* nWc;
  double* colscr;
  double* hpart;
  double2* cstat;
  double* csq;
  const uint32_t* corder;
  DevState* st;
  // split-BF16 batches: operand planes of W (row-major, and gene-major as
  // W^T) and of P's off-diagonal part; null in FP32 batches
  bf16_t *Wh, *Wl, *Wth, *Wtl, *Ph, *Pl;
  int64_t nh;      // h partials written by the chosen A + W tiling
  int64_t splits;  // K splits of the W W^T partials for the chosen chunk
  int64_t chunk;   // K columns per split
};

// Counter slots of one work list: one per XCD, a cache line apart.
constexpr int kCtrStride = 32;
constexpr int kNumXcd = 8;

// Work items of one grouped launch: segments of consecutive items that
// belong to one network, and the item ranges of the eight per-XCD queues.
// Blocks take items from their own XCD's queue first, then from the others.
struct WorkList {
  const int32_t* seg_inst;   // network of segment s
  const int64_t* seg_first;  // first item of segment s; seg_first[nseg] = total
  int32_t nseg;
  int32_t* ctr;              // kNumXcd counters, kCtrStride ints apart
  int64_t xb[kNumXcd + 1];   // queue x holds items [xb[x], xb[x + 1])
};

// Flat grid over all networks: block b belongs to segment s when
// seg_first[s] <= b < seg_first[s + 1] (segments in network order).
struct FlatList {
  const int64_t* seg_first;
  int32_t nseg;
  int64_t total;
};

// Tile candidates of the grouped products (the autotuner picks one each).
// A split-BF16 batch (b3) has one tiling for R, A + W and the C update (the
// shapes of candidate 0) and the same K chunks for W W^T.
enum BatchTile { kBTResp = 0, kBTAvail = 1, kBTCoop = 2, kBTCoreg = 3, kBTNum = 4 };
int batch_tile_candidates(int phase, bool b3 = false);
void rect_tile_shape(int choice, int64_t* bm, int64_t* bn);  // R and A + W tiles
int64_t coop_chunk_of(int choice);                           // K chunk of W W^T
// Persistent grid of a grouped product with candidate `choice` (sigT: the
// C-update variant that keeps the similarity sums).
int64_t batch_grid(int phase, int choice, bool sigT, bool b3);

hipError_t launch_batch_resp(int choice, bool b3, const BInst* bi, const WorkList& wl, int64_t nb,
                             hipStream_t s);
hipError_t launch_batch_avail(int choice, bool b3, const BInst* bi, const WorkList& wl, Rule rule,
                              int64_t nb, hipStream_t s);
hipError_t launch_batch_coop_partial(bool b3, const BInst* bi, const WorkList& wl, int64_t nb,
                                     hipStream_t s);
hipError_t launch_batch_coreg(int choice, bool b3, const BInst* bi, const WorkList& wl, Rule rule,
                              int64_t nb, hipStream_t s);
// bf16 planes of the new W (split-BF16 batches): (Nep / 64) x (Nap / 64)
// blocks per network.
hipError_t launch_batch_planes(const BInst* bi, const FlatList& fl, hipStream_t s);
hipError_t launch_batch_finish_h(const BInst* bi, int32_t n, Rule rule, hipStream_t s);
// norms of the new W: part = Ne row blocks + (col groups x row chunks) per
// network; sum = col groups per network.
hipError_t launch_batch_norms(const BInst* bi, const FlatList& part, const FlatList& sum,
                              hipStream_t s);
hipError_t launch_batch_coop_finalize(const BInst* bi, const FlatList& fl, Rule rule,
                                      hipStream_t s);
hipError_t launch_batch_diagonals(const BInst* bi, const FlatList& fl, Rule rule, hipStream_t s);
hipError_t launch_batch_reset(int32_t* ctr, int64_t count, hipStream_t s);
hipError_t launch_batch_gather(const BInst* bi, int32_t n, DevState* out, hipStream_t s);
hipError_t launch_batch_gates(const BInst* bi, int32_t n, int32_t active, int32_t run_pc,
                              hipStream_t s);

}  // namespace panda
