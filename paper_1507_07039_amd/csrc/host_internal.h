// Host-side internals shared by the single-network API (panda_api.hip) and
// the batched API (batch_api.hip): error reporting, the workspace carver, the
// per-network context and its workspace layout.
#pragma once

#include "panda.h"

#include <stdio.h>

#include "panda_internal.h"

namespace panda {

// Error text of the calling thread (panda_last_error); returns st.
panda_status fail(panda_status st, const char* fmt, const char* what = "");
panda_status hip_fail(hipError_t e, const char* where);

#define HIP_TRY(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return panda::hip_fail(e_, #call);  \
  } while (0)

#define PANDA_TRY(call)                      \
  do {                                       \
    panda_status s_ = (call);                \
    if (s_ != PANDA_OK) return s_;           \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace (sizes only when base is null).
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align_up(count * sizeof(T));
    return p;
  }
};

constexpr size_t kZsScratch = kZsBlocks + 8;  // doubles
// Scratch (doubles) of a z-score of a rows x cols network with the given
// scope: the global form's block partials, or 8 flags plus the per-row and
// per-column moments.
size_t zscore_scratch_doubles(int64_t rows, int64_t cols, int32_t mode);
// Diagonal and off-diagonal value of the z-scored identity of order n; false
// if its standard deviation is 0.
bool identity_zscore(int64_t n, int32_t mode, int32_t ddof, double* dv, double* ov);
// Z-score in place (Sec. II-A) with the scope and normaliser of the
// options; synchronises the stream to read the degeneracy flags.
panda_status zscore(float* M, int64_t rows, int64_t cols, int64_t ld, int32_t mode, int32_t ddof,
                    double* scratch, hipStream_t s);
constexpr int kMaxPending = 16;               // timed iterations between read-backs

Rule rule_of(const panda_options& o);
panda_status check_options(const panda_options& o);
// PANDA() from a loaded context until h < tol or max_iter (panda_run's loop).
panda_status run_loaded(panda_ctx* c);
bool dims_ok(int64_t Ne, int64_t Na);

// Sizes of the buffers whose extent depends on the tile schedule.  The
// single-network schedule fixes them; a batch sizes them for the smallest
// tile and K chunk among its candidates, and needs no stream-K scratch.
struct LayoutSpec {
  bool batched;
  int64_t hpart_tiles;  // per-tile h partials of the A + W product
  int64_t ppart_splits; // K splits of the W W^T partial products
  bool packed_c = false; // C as its upper tiles (packed_tile)
};
LayoutSpec single_spec(int64_t Ne, int64_t Na, bool packed_c, int32_t precision);

}  // namespace panda

struct panda_ctx {
  int64_t Ne, Na, Nep, Nap;
  panda_options opt;
  panda::Rule rule;
  hipStream_t stream;
  float* W[2];
  float* R;
  float* P;
  float* C;
  float* Tside;
  float* ppart;   // split-K partial products of W W^T
  float* skpart;  // stream-K partial tiles (single-network schedule only)
  double* dP;     // diagonal of P (FP64; P holds zero there)
  double* dC;     // diagonal of C
  double* nP;     // |P_i.|^2
  double* nC;     // |C_.j|^2
  double* nWr;    // |W_i.|^2
  double* nWc;    // |W_.j|^2
  double* colscr; // column-norm scratch
  double* hpart;
  double2* cstat;
  double* csq;
  double* zs;
  uint32_t* corder;  // launch order of the upper C tiles
  uint32_t* corder_r;  // the same with the R tiles of the next iteration (split-BF16)
  bool r_next;  // R holds T(P, W) of the current state (computed by the last C update)
  panda::DevState* st;
  bool b3;  // split-BF16 products
  bool packed;  // C stored as its upper tiles (packed_tile)
  panda::bf16_t *Wh, *Wl, *Wth, *Wtl, *Ph, *Pl;  // split planes (C stays FP32)
  panda::DevState* host;  // pinned
  panda::DevState* snap;  // pinned, two slots: states copied ahead (run_loaded)
  hipEvent_t snap_ev[2];
  int splits;
  int64_t nh;
  int32_t t0;
  int64_t executed;  // iterations known to have run since load
  int64_t enqueued;  // iterations enqueued since load
  bool loaded;
  // phase timing
  bool timing;
  int npend;
  hipEvent_t ev[16][PANDA_NPHASE + 1];
  double tot_ms[PANDA_NPHASE];
  int64_t cnt[PANDA_NPHASE];
};

namespace panda {

// Workspace layout of one network: fills c (when not null) with pointers
// into base and returns the bytes used.
size_t ctx_layout(int64_t Ne, int64_t Na, int32_t precision, const LayoutSpec& spec, panda_ctx* c,
                  char* base);
// Context over an already carved workspace (no argument checks), with its
// pinned state mirror; ctx_free releases what ctx_setup acquired.
panda_status ctx_setup(panda_ctx* c, int64_t Ne, int64_t Na, const panda_options& o,
                       const LayoutSpec& spec, char* base, hipStream_t stream);
void ctx_free(panda_ctx* c);
// Launch-order table of the upper C tiles (synchronises the context's stream).
panda_status ctx_fill_order(panda_ctx* c);

}  // namespace panda
