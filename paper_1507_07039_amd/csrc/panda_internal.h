// Internal declarations shared by the HIP sources of libpanda.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace panda {

// Device-resident iteration state.  Kernels read the gates and skip their
// work once the run has converged, so the host can enqueue iterations ahead
// of reading h back.
struct DevState {
  double h;        // h of the last completed iteration (Eq. 7)
  int32_t t;       // number of completed iterations (t of Eq. 6 during the P/C phase)
  int32_t active;  // 1 while h >= tol: gates R, A, W and h
  int32_t run_pc;  // 1 when the current iteration updates P and C: gates Eq. 5-6
  int32_t conv;    // 1 once h < tol
  int32_t pad[2];
};

// Scalars of the update rules.
struct Rule {
  double alpha;
  double tol;
  int32_t diag_alpha;
  int32_t sigma_from_T;
  int32_t n_own;
  int32_t h_undamped;
  int32_t update_last;
};

constexpr int kBK = 16;       // K-step of the GEMM main loop (floats)
constexpr int kThreads = 256; // threads per GEMM block (4 waves of 64)

// Padding of the internal state: rows of W / P to 64, genes to 256.
constexpr int64_t kPadE = 64;
constexpr int64_t kPadA = 256;
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------ launchers --
// Similarity matrix T(X, Y) of padded operands: X is Mp x Kp (row-major,
// k contiguous), Y is Kp x Np (row-major, n contiguous).  Mp % 64 == 0,
// Np % 256 == 0, Kp % 16 == 0.  Out[i][j] written for i < M, j < N.
hipError_t launch_tanimoto_store(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                 int64_t Mp, int64_t Np, int64_t Kp, int64_t M, int64_t N,
                                 float* Out, int64_t ldo, const int32_t* gate, hipStream_t s);

// A = T(W, C) fused with the W update of Eq. 2 and the h partials of Eq. 7.
hipError_t launch_avail_wupdate(const float* Wold, const float* C, const float* R, float* Wnew,
                                int64_t ld, int64_t Nep, int64_t Nap, int64_t Ne, int64_t Na,
                                Rule rule, double* hpart, const int32_t* gate, hipStream_t s);
int64_t avail_wupdate_blocks(int64_t Nep, int64_t Nap);

// C update (Eq. 5) on the upper tiles of T(W^T, W) with mirror writes and
// per-row partial sums for the sigma of Eq. 6.
hipError_t launch_coreg_update(const float* W, int64_t ldw, int64_t Nep, float* C, int64_t ldc,
                               int64_t Nap, int64_t Na, Rule rule, double2* cstat,
                               const int32_t* gate, hipStream_t s);
int64_t coreg_slots(int64_t Nap);

// P update, split over K: partial products of W W^T on upper tiles.
hipError_t launch_coop_partial(const float* W, int64_t ldw, int64_t Nep, int64_t Nap, int splits,
                               float* part, double* pnrm, const int32_t* gate, hipStream_t s);
int coop_splits(int64_t Nep, int64_t Nap);

// Rest of the iteration: h, P finalisation and both diagonals.
hipError_t launch_finish_h(const double* hpart, int64_t n, int64_t count, DevState* st,
                           Rule rule, hipStream_t s);
hipError_t launch_coop_finalize(const float* part, const double* pnrm, int splits, float* P,
                                int64_t ldp, int64_t Ne, Rule rule, float* Tside,
                                const int32_t* gate, hipStream_t s);
hipError_t launch_diagonals(float* P, int64_t ldp, int64_t Ne, const float* Tside, float* C,
                            int64_t ldc, int64_t Na, const double2* cstat, int64_t nslots,
                            Rule rule, const DevState* st, hipStream_t s);

// Z-score (Sec. II-A) on a strided matrix; scratch holds kZsBlocks + 8 doubles.
constexpr int kZsBlocks = 1024;
hipError_t launch_zscore_stats(const float* M, int64_t rows, int64_t cols, int64_t ld,
                               double* scratch, hipStream_t s);
hipError_t launch_zscore_apply(float* M, int64_t rows, int64_t cols, int64_t ld,
                               const double* scratch, hipStream_t s);
hipError_t launch_fill_identity(float* M, int64_t n, int64_t ld, hipStream_t s);
hipError_t launch_state_init(DevState* st, int32_t t0, hipStream_t s);

}  // namespace panda
