// Internal declarations shared by the HIP translation units of libmpid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mpid.h"

namespace mpid {

constexpr int kThreads = 256;   // block size of every kernel
constexpr int kNbMax = 32;      // largest panel width (K of the blocked update)
constexpr int kRtMax = 256;     // largest row tile of the reflector sweep
constexpr int kRtMin = 64;      // smallest row tile of the reflector sweep
constexpr int kRowTileG = 256;  // row tile of the ingest / blocked-update kernels
constexpr int kColTileG = 64;   // column tile of the blocked update
constexpr int kFinCols = 32;    // columns per block of the norm reduction
constexpr int kFC = 16;         // columns per block of the step finalization
constexpr int kFL = kThreads / kFC;  // its tile lanes
constexpr int kBatchMaxN = 2048;  // widest matrix of the batched path
constexpr int kBatchMaxGroups = ID_BATCH_MAX_GROUPS;  // most workgroups sharing one item

// Device-resident control block of one factorization.  Every field is written
// by exactly one kind of kernel and read only by later kernels on the stream.
struct FactorState {
  int32_t done;      // factorization finished (k valid)
  int32_t end_flag;  // current panel ends after the step that set it
  int32_t jb;        // reflectors generated in the current panel
  int32_t last_jb;   // jb of the panel that just ended (for the host)
  int32_t info;      // ID_INFO_NONFINITE when the input holds NaN/Inf
  uint32_t fmax_bits;  // max |F| of the current panel, as float bits
  uint32_t vmax_bits;  // largest column norm after the last recomputation (float bits)
  uint32_t nabove;   // live columns whose norm exceeds rel_tol |R_00| after the last recomputation
  int64_t k;         // rank (valid when done)
  double r00;        // |R_00|
  double alpha;      // leading entry of the current pivot column
  double fro2;       // ||A||_F^2
  int64_t off;       // first step of the current panel
  int64_t ncur;      // columns of the current (compacted) working copy
  uint32_t nred;     // blocks of the panel-end column reduction that finished
  int32_t swap_other;  // the column whose swap-order key the step's swap changed
  int32_t swap_key;    // ... and its new key
  int32_t pad1;
};

// The host's copy of the state after a panel (pinned host memory, written by
// the device); seq tells which panel of which call it holds.
struct FactorHostSlot {
  FactorState s;
  int64_t seq;
};

// Per-block partial of the pivot search.
struct AmaxPart {
  double v;     // largest column norm of the block (-1 if none)
  double s2;    // sum of squared column norms of the block
  int32_t pos;  // position of the largest column in the working layout
  int32_t key;  // its position in the swap order (tie-break: smaller wins)
};

// Layout of the factorization workspace (all offsets in bytes).
struct FactorPlan {
  int64_t m, n, kcap;
  int32_t dtype, prec, nb, wbytes;  // wbytes: 4 (fp32 working copy) or 8
  int64_t ldw, ldv, ldf;
  int64_t ntile_s_max, ntile_g, nfold_max;
  size_t off_w0, off_w1, off_v, off_f, off_zpart, off_auxpart, off_nrm2part, off_zfold,
      off_afold, off_nfold, off_colpart,
      off_nu, off_nuo, off_amax, off_colid0, off_colid1, off_pvflag, off_pivpos, off_pivid,
      off_permw, off_posof, off_tau, off_vscale, off_rorig, off_state, off_slot, off_wrow,
      off_vrow, off_keypos;
  size_t bytes;
};

bool make_factor_plan(int64_t m, int64_t n, int32_t dtype, const id_opts* o, FactorPlan* p);

int factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
               const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
               int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s);

// The same factorization for callers that cannot allocate: "work" is the
// library's static scratch, the host reads each panel's end state with a copy
// into host memory it already owns (no pinned slot, no events), so nothing is
// allocated.  ID_FLAG_GRAM, ID_FLAG_CHOLQR and ID_FLAG_PROFILE are refused
// (ID_ERR_UNSUPPORTED).
int factor_run_noalloc(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                       const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                       int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s);

void last_profile(id_profile* out);

// The factorization through the FP64 Gram matrix (ID_FLAG_GRAM).
size_t gram_workspace(int64_t m, int64_t n, int32_t dtype, const id_opts* o);
int gram_factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                    int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s);
// G = A^T A (FP64, n x n, both triangles, ld n) with the Gram path's kernels;
// part: gram_matrix_workspace(m, n) bytes of partial tiles; *info =
// ID_INFO_NONFINITE when A holds NaN / Inf (left alone otherwise).
size_t gram_matrix_workspace(int64_t m, int64_t n);
int gram_matrix_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda, double* G,
                    void* part, size_t part_bytes, int32_t* info, hipStream_t s);

// The factorization through a shifted CholeskyQR3 R factor (ID_FLAG_CHOLQR).
size_t cholqr_workspace(int64_t m, int64_t n, int32_t dtype, const id_opts* o);
int cholqr_factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                      const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                      int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s);

int solve_T_run(const double* R, int64_t ldr, int64_t k, int64_t n, double* T, int64_t ldt,
                int32_t* info, hipStream_t s);
int round_run(double* X, int64_t rows, int64_t cols, int64_t ld, int32_t mode, hipStream_t s);

// X = op(R)^{-1} B for upper-triangular R (k x k, ldr); trans = 0 solves R X = B,
// trans = 1 solves R^T X = B.  B (k x ncols, ldb) and X (ldx) may alias.
int trsm_upper_run(const double* R, int64_t ldr, int64_t k, const double* B, int64_t ldb,
                   int64_t ncols, double* X, int64_t ldx, int trans, hipStream_t s);
// X = R^{-1} R^{-T} B in one launch (B is overwritten with R^{-T} B; X may
// alias B).
int trsm_normal_run(const double* R, int64_t ldr, int64_t k, double* B, int64_t ldb,
                    int64_t ncols, double* X, int64_t ldx, hipStream_t s);

// C = alpha * op(A) op(B) + beta * C (column-major float64; ta/tb: 0 = N, 1 = T).
// Bytes of split-K partials gemm64 uses for an M x N product with contraction K
// when given them (0: no split).
size_t gemm64_split_workspace(int64_t M, int64_t N, int64_t K);
// C = A B, A (M x K, lda) in its storage dtype, B and C float64 (column-major);
// b_upper != 0: B is upper triangular and the products skip its zero part.
int gemm64_typed_run(const void* A, int32_t dtype, int64_t M, int64_t N, int64_t K, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, int b_upper,
                     hipStream_t s);
int gemm64_run(int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
               int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
               hipStream_t s);

int reconstruct_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const int32_t* perm, int64_t k, const double* T, int64_t ldt, double* Y,
                    int64_t ldy, int32_t residual, hipStream_t s);

size_t batch_item_workspace(int64_t m, int64_t n, const id_opts* o);
int factor_batched_run(id_batch_item* items, int32_t batch, const int32_t* slots, int32_t nslots,
                       int32_t* queue, int64_t max_n, int32_t dtype, const id_opts* o,
                       int32_t block_threads, int32_t num_groups, hipStream_t s);
// T of every item (after the batched factorization, same stream).
int trsm_batched_run(const id_batch_item* items, int32_t batch, int64_t max_n, hipStream_t s);

// Lock-step batches (items: host array; see id_factor_lockstep).
size_t lockstep_workspace(const id_batch_item* items, int32_t batch, int32_t dtype,
                          const id_opts* o);
int lockstep_run(id_batch_item* items, int32_t batch, int32_t dtype, const id_opts* o, void* work,
                 size_t work_bytes, hipStream_t s);

size_t backward_workspace(int64_t m, int64_t n, int64_t k);
int backward_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                 const int32_t* perm, int64_t k, const double* T, int64_t ldt, const double* Rb,
                 int64_t ldrb, const double* gT, int64_t ldgt, const double* gY, int64_t ldgy,
                 double* gA, int64_t ldga, void* work, size_t work_bytes, int32_t* info,
                 hipStream_t s);

size_t sketch_workspace(int64_t l, int64_t m, int64_t n);
// sketch_run with column j of A taken from A(:, acols[j]) (acols may be null)
// and the contraction split for about target_blocks blocks (0: the default);
// accumulate != 0 adds the product to Y instead of overwriting it
size_t sketch_workspace_target(int64_t l, int64_t m, int64_t n, int target_blocks);
int sketch_run_cols(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const int32_t* acols, const double* Om, int64_t l, int64_t ldo, double* Y,
                    int64_t ldy, void* work, size_t work_bytes, int target_blocks, hipStream_t s,
                    int accumulate = 0);
int sketch_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda, const double* Om,
               int64_t l, int64_t ldo, double* Y, int64_t ldy, void* work, size_t work_bytes,
               hipStream_t s);

__host__ __device__ inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
__host__ __device__ inline int64_t ceil_div(int64_t x, int64_t a) { return (x + a - 1) / a; }

// Host-side diagnostics on stderr, switched on by the environment variable
// MPID_LOG (1: a line per factorization call and per settled panel; 2: also
// the geometry of every pivot step's launches).  Read at each use.
int log_level();
void log_printf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
#define MPID_LOG(level, ...)                                         \
  do {                                                               \
    if (::mpid::log_level() >= (level)) ::mpid::log_printf(__VA_ARGS__); \
  } while (0)

// Returns ID_ERR_HIP from the enclosing function when a HIP call fails.
#define MPID_HIP(expr)                              \
  do {                                              \
    if ((expr) != hipSuccess) return ID_ERR_HIP;    \
  } while (0)

#define MPID_LAUNCH_CHECK()                                  \
  do {                                                       \
    if (hipGetLastError() != hipSuccess) return ID_ERR_HIP;  \
  } while (0)

}  // namespace mpid
