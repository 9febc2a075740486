/*
 * mpid.h -- C ABI of the MI355X (gfx950) column interpolative decomposition.
 *
 * The column ID approximates A (m x n) by k of its own columns,
 *     A ~= A(:, J) P,   P = [I_k  T] Z^T,   T = R11^{-1} R12,
 * where A Z = Q R is a column-pivoted QR truncated after k steps
 * (Dunton & Fox, arXiv 2012.00706: Section 1.1, eq. (4)-(8); Algorithm 1 for
 * the double-precision ID, Algorithm 2 for the mixed/low-precision ID).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major.  "ld" arguments are leading dimensions in
 *     elements.  Pointers are DEVICE pointers unless marked [host].
 *   - The caller owns every buffer.  The library allocates no device memory
 *     in these calls; scratch space is the caller's workspace ("work").
 *   - Indices are 0-based.  perm is int32 with A(:, perm) = Q R, J = perm[0:k].
 *   - R, T, Y and gradients are float64: products are evaluated in double
 *     precision (remark after Lemma 1).
 *   - "stream" is a hipStream_t passed as void*; NULL means the default stream.
 *   - Synchronous return codes (< 0) report bad arguments, workspace and HIP
 *     errors; numerical conditions are reported through "info" codes (> 0).
 */
#ifndef MPID_H
#define MPID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return / info codes ------------------------------------------------ */
#define ID_OK 0
#define ID_ERR_ARG (-1)         /* invalid argument (null pointer, size, ld, option) */
#define ID_ERR_DTYPE (-2)       /* unknown dtype or precision */
#define ID_ERR_WORKSPACE (-3)   /* work_bytes smaller than id_workspace_size() */
#define ID_ERR_HIP (-4)         /* a HIP runtime call failed */
#define ID_ERR_UNSUPPORTED (-5) /* combination not supported */
#define ID_ERR_SCRATCH (-6)     /* problem larger than id_factor_noalloc's static scratch */
#define ID_INFO_NONFINITE 1     /* A holds NaN or Inf: nothing was factored (k = 0) */
#define ID_INFO_SINGULAR 2      /* R11 has |R_ii| <= n * 2^-53 * |R_00|; T not formed */
#define ID_INFO_RANK_FULL 3     /* k = n: T has no columns, P is a permutation */
#define ID_INFO_ABORTED 4       /* batched item abandoned (see id_factor_batched) */
#define ID_INFO_GRAM_LIMIT 5    /* ID_FLAG_GRAM stopped at its resolution floor (see id_factor) */
#define ID_INFO_CHOLQR_BREAKDOWN 6 /* ID_FLAG_CHOLQR: A lacks full numerical column rank (k = 0) */

/* Most workgroups that may share one batched item. */
#define ID_BATCH_MAX_GROUPS 16

/* ---- storage dtype of A -------------------------------------------------- */
#define ID_F32 0
#define ID_F64 1

/* ---- precision policy of the factorization -------------------------------
 * ID_PREC_F64:        working copy, sweeps and the blocked trailing update in
 *                     float64 (the double-precision ID of Algorithm 1).
 * ID_PREC_MIXED_F16:  working copy in float32; the blocked trailing update on
 *                     FP16 matrix cores with FP32 accumulation (operands scaled
 *                     by powers of two, which is exact, so they stay in FP16
 *                     range); column norms, R, the recomputation of norms and the
 *                     triangular solve in float64 (Algorithm 2, mixed variant).
 * ID_PREC_MIXED_BF16: as above with BF16 operands (no scaling needed).
 * ID_PREC_MIXED_BF16X3: as ID_PREC_MIXED_BF16, each operand split into a sum of
 *                     two BF16 numbers (x = hi + lo) and the product formed as
 *                     hi*hi + hi*lo + lo*hi on BF16 matrix cores with FP32
 *                     accumulation: the update error drops from about 2^-8 to
 *                     about 2^-16 of its size at three times the (idle) matrix
 *                     work of the bandwidth-bound update.
 * ID_PREC_MIXED_F32:  as above with FP32 operands on FP32 matrix cores (the
 *                     single-precision low arithmetic of Algorithm 2).       */
#define ID_PREC_F64 0
#define ID_PREC_MIXED_F16 1
#define ID_PREC_MIXED_BF16 2
#define ID_PREC_MIXED_BF16X3 3
#define ID_PREC_MIXED_F32 4

/* ---- adaptive rank rules (used when k_fixed == 0) ------------------------
 * ID_RANK_PIVOT_REL: stop before step j >= 1 once the largest remaining column
 *                    norm is <= rel_tol * |R_00|, or is zero.
 * ID_RANK_FROB_REL:  stop once the Frobenius norm of the remaining block is
 *                    <= rel_tol * ||A||_F (then ||A - A(:,J)P||_F <= rel_tol ||A||_F
 *                    up to rounding).                                       */
#define ID_RANK_PIVOT_REL 0
#define ID_RANK_FROB_REL 1

/* ---- flags --------------------------------------------------------------- */
#define ID_FLAG_NO_PIVOT 1 /* unpivoted Householder QR (perm = identity) */
#define ID_FLAG_PROFILE 2  /* time every kernel with HIP events (see id_last_profile) */
#define ID_FLAG_GRAM 4     /* tall-skinny front end: pivots and R from the FP64 Gram
                              matrix A^T A (one pivoted Cholesky); see id_factor */
#define ID_FLAG_CHOLQR 32  /* tall-skinny front end: the pivoted factorization of the
                              n x n R factor of a shifted CholeskyQR3; see id_factor */
/* Simulated low precision (Section 3: variables held in single or half
 * precision while arithmetic accumulates in higher precision): every value the
 * factorization keeps -- the working copy, the reflectors, F, the rows of R,
 * the column norms, beta / tau -- is rounded to the nearest binary32
 * (ID_FLAG_ROUND_F32) or binary16 (ID_FLAG_ROUND_F16) number; sums and
 * products still accumulate in the kernels' precision.  With ID_FLAG_ROUND_F16
 * the FP16 update (ID_PREC_MIXED_F16) drops its power-of-two operand scaling,
 * so tiny values underflow as in the paper's simulation.  id_round then gives
 * the coefficients T the same precision.  ID_FLAG_ROUND_F32 takes
 * ID_PREC_MIXED_F32 and ID_FLAG_ROUND_F16 takes ID_PREC_MIXED_F16 (other
 * combinations are invalid arguments); not with ID_FLAG_GRAM or ID_FLAG_CHOLQR. */
#define ID_FLAG_ROUND_F32 8
#define ID_FLAG_ROUND_F16 16

typedef struct {
  int32_t prec;      /* ID_PREC_* */
  int32_t rank_rule; /* ID_RANK_* */
  int64_t k_fixed;   /* > 0: exactly min(k_fixed, k_max) steps; 0: adaptive */
  double rel_tol;    /* adaptive tolerance, >= 0 */
  int64_t k_max;     /* cap on k; 0 means min(m, n) */
  int32_t nb;        /* panel width of the blocked update, 1..32; 0 = 32 */
  int32_t flags;     /* ID_FLAG_* */
} id_opts;

/* Bytes of device workspace id_factor needs for an m x n input of storage
 * dtype "dtype" under "opts" [host].  Returns 0 for invalid arguments. */
size_t id_workspace_size(int64_t m, int64_t n, int32_t dtype, const id_opts* opts);

/* Column-pivoted Householder QR of A truncated after k steps (Section 1.1,
 * eq. (6)-(7); the MGSQR(A, k) step of Algorithms 1 and 2 -- computed here
 * with Householder reflectors, a blocked trailing update and norm downdating).
 *
 *   A      [in]  m x n, lda >= max(1, m), storage dtype "dtype" (ID_F32/ID_F64).
 *                Not modified.
 *   opts   [host] precision, rank selection and panel width.
 *   work   [in]  device workspace of work_bytes >= id_workspace_size(...).
 *   perm   [out] n int32: the column order; J = perm[0:k].
 *   R      [out] float64, ldr >= kcap where kcap = min(m, n, k_max, k_fixed>0 ?
 *                k_fixed : inf).  Rows 0..k-1 of the k x n upper-trapezoidal
 *                factor in pivot order are written (zeros below the diagonal);
 *                rows k..kcap-1 are left untouched.
 *   k_out  [host,out] the rank k.
 *   info   [host,out] 0, ID_INFO_NONFINITE, or ID_INFO_GRAM_LIMIT
 *          (ID_FLAG_GRAM) / ID_INFO_CHOLQR_BREAKDOWN (ID_FLAG_CHOLQR).
 *
 * ID_FLAG_GRAM (tall inputs): pivots and R come from a pivoted Cholesky
 * factorization of the FP64 Gram matrix A^T A (equal to the Householder
 * pivots and R up to row signs in exact arithmetic).  Its residual norms are
 * resolved only down to about sqrt(8 n 2^-53) |R_00|: an adaptive rel_tol
 * below 1e-6 returns ID_ERR_UNSUPPORTED, and the factorization stops before
 * any step whose pivot's residual norm is at or below that floor, fixed rank
 * included, with info = ID_INFO_GRAM_LIMIT and k the steps completed (R and T
 * of those steps are valid).  The flag supports k <= 2048 and no
 * ID_FLAG_NO_PIVOT / ID_FLAG_PROFILE.
 *
 * ID_FLAG_CHOLQR (tall inputs, m >= n): A = Q R0 from CholeskyQR passes on
 * the FP64 matrix cores (each a Gram product and a right multiplication by
 * the inverse triangular factor): two (CholeskyQR2, R0 = R2 R1) when the
 * first Cholesky factorization succeeds and ||R2 - I||_F <= 1/2, else three
 * (R0 = R3 R2 R1), the first shifted by 11 (m n + n (n + 1)) 2^-53 ||A||_F^2
 * when its plain factorization fails (shifted CholeskyQR3).  Then the FP64
 * pivoted factorization of the n x n R0, whose pivots and R are those of A:
 * residual norms resolved down to about 2^-53 ||A|| (the Gram front end:
 * about 2^-26.5 ||A||).  Needs full numerical column rank: the shifted pass
 * leaves A R1^{-1} with a condition number of about
 * kappa(A) sqrt(11 (m n + n^2) 2^-53), which the plain passes take only below
 * about 2^26.5, so kappa(A) must stay below about 2^53 / sqrt(11 (m n + n^2))
 * (2e12 at 3000 x 200).  Beyond that a Cholesky pivot fails or R3 is not near
 * the identity (||R3 - I||_F > 1/2): info = ID_INFO_CHOLQR_BREAKDOWN and
 * k = 0 (nothing factored; perm = identity).  A = 0 gives k = 0, info 0.
 * The workspace holds two m x n FP64 copies.  opts->prec is ignored (the
 * factorization of R0 is FP64); ID_FLAG_GRAM, ID_FLAG_NO_PIVOT,
 * ID_FLAG_PROFILE and the ROUND flags are refused (ID_ERR_UNSUPPORTED), as is
 * m < n.
 *
 * Pivoting follows the largest remaining column norm with ties going to the
 * first column in the current (LAPACK swap) order.  The call enqueues work on
 * "stream" and waits for it while it runs (the number of pivot steps is data
 * dependent); it returns with k and info known and the final gather of perm
 * and R still enqueued: they are complete when the stream's work is, and the
 * workspace must not be reused on another stream before then.  Concurrent
 * calls must use distinct workspaces.  A single
 * ID that can be captured in a graph (k and info left in device memory, no
 * host synchronization) is id_factor_batched with a batch of one item, whose
 * workgroups share it (up to ID_BATCH_MAX_GROUPS). */
int id_factor(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
              const id_opts* opts, void* work, size_t work_bytes, int32_t* perm, double* R,
              int64_t ldr, int64_t* k_out, int32_t* info, void* stream);

/* ---- allocation-free factorization -------------------------------------
 * For callers that cannot allocate: code under HIP graph capture setup, tight
 * serving loops, harnesses that forbid hipMalloc.  id_factor_noalloc computes
 * exactly what id_factor computes (same kernels, same results bit for bit),
 * but its workspace is a static device array of ID_NOALLOC_SCRATCH_MB MiB
 * inside the library (one per GPU, held from the library's load until the
 * process ends) and it calls no hipMalloc, hipHostMalloc, hipFree or event
 * creation: the host reads each panel's end state with a copy into host
 * memory of its own, which waits for the stream (so panels are not enqueued
 * ahead of the host; a little slower than id_factor).
 *
 *   Arguments as in id_factor, without work / work_bytes.
 *   Returns ID_ERR_SCRATCH when id_workspace_size(m, n, dtype, opts) exceeds
 *   id_noalloc_scratch_bytes() (nothing is enqueued), ID_ERR_UNSUPPORTED for
 *   ID_FLAG_GRAM, ID_FLAG_CHOLQR or ID_FLAG_PROFILE, ID_ERR_ARG when "stream" does not belong
 *   to the current device (whose scratch is used).
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents (each call initializes what it reads before reading it):
 * calls that overlap on one GPU -- from several host threads or on several
 * streams -- race and must not be made. */
#define ID_NOALLOC_SCRATCH_MB 128

/* Bytes of the static scratch of id_factor_noalloc [host]. */
size_t id_noalloc_scratch_bytes(void);

int id_factor_noalloc(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                      const id_opts* opts, int32_t* perm, double* R, int64_t ldr, int64_t* k_out,
                      int32_t* info, void* stream);

/* Interpolation coefficients T = R11^{-1} R12 in float64 (eq. (8); the
 * coefficient step of Algorithms 1 and 2; Remark 1.1's pseudo-inverse equals
 * the inverse whenever R11 is nonsingular, which this call checks).
 *
 *   R     [in]  k x n upper trapezoidal (as written by id_factor), ldr >= k.
 *   k, n  [host] rank and column count, 0 <= k <= n.
 *   T     [out] k x (n-k), ldt >= max(1, k).
 *   info  [out] device int32: 0, ID_INFO_SINGULAR (T not written) or
 *               ID_INFO_RANK_FULL (k == n, nothing to write).
 * Asynchronous on "stream". */
int id_solve_T(const double* R, int64_t ldr, int64_t k, int64_t n, double* T, int64_t ldt,
               int32_t* info, void* stream);

/* X (rows x cols, column-major, ld >= max(1, rows), float64, device) rounded in
 * place to the nearest binary32 (mode 1) or binary16 (mode 2) values -- the
 * low-precision coefficient matrix of the simulated single / half precision ID
 * (Section 3).  cols <= 65535.  ID_ERR_ARG for other modes or sizes.
 * Asynchronous on "stream". */
int id_round(double* X, int64_t rows, int64_t cols, int64_t ld, int32_t mode, void* stream);

/* Reconstruction Y = A(:, J) P in float64 (eq. (4)-(5) with P from eq. (8),
 * products in double precision as in the remark after Lemma 1):
 * Y(:, perm[j]) = A(:, perm[j]) for j < k, Y(:, perm[k+c]) = A(:, J) T(:, c).
 * If "residual" is nonzero, Y receives A - A(:, J) P instead.
 *
 *   A    [in]  m x n, lda, storage dtype "dtype".
 *   perm [in]  n int32 permutation; k [host] rank.
 *   T    [in]  k x (n-k) float64, ldt >= max(1, k).
 *   Y    [out] m x n float64, ldy >= max(1, m).
 * Asynchronous on "stream". */
int id_reconstruct(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                   const int32_t* perm, int64_t k, const double* T, int64_t ldt, double* Y,
                   int64_t ldy, int32_t residual, void* stream);

/* Bytes of device workspace id_backward needs [host]. */
size_t id_backward_workspace_size(int64_t m, int64_t n, int64_t k);

/* Adjoint of the ID with the skeleton J = perm[0:k] held fixed (not in the
 * paper).  With B = A(:, J), C = A(:, Jc) the coefficients are the least-squares
 * solution T = B^+ C, which equals R11^{-1} R12 (eq. (6)-(8)).  Given
 * cotangents gT of T (k x (n-k)) and/or gY of Y = A(:, J) P (m x n), writes
 * gA = d<gT, T> / dA + d<gY, Y> / dA:
 *     Tbar = gT + B^T gY(:, Jc),   X = (B^T B)^{-1} Tbar,
 *     gA(:, Jc) = B X,
 *     gA(:, J)  = (C - B T) X^T - B X T^T + gY(:, J) + gY(:, Jc) T^T.
 * (B^T B)^{-1} is applied through an R factor of B: the caller's Rb when given
 * (any upper-triangular R with R^T R = B^T B, e.g. R11 = the first k columns of
 * the R that an FP64 id_factor wrote when it chose J), else that of an
 * unpivoted FP64 Householder QR of B computed here.
 *
 *   A       [in]  m x n, lda, storage dtype "dtype"; perm [in] n int32; k [host].
 *   T       [in]  k x (n-k) float64, ldt.
 *   Rb      [in]  k x k float64 upper triangular, ldrb >= k, or NULL.
 *   gT      [in]  k x (n-k) float64, ldgt, or NULL.
 *   gY      [in]  m x n float64, ldgy, or NULL.
 *   gA      [out] m x n float64, ldga.
 *   work    [in]  workspace of >= id_backward_workspace_size(m, n, k) bytes.
 *   info    [host,out] 0 or ID_INFO_SINGULAR (B numerically rank deficient;
 *           gA is then left undefined and nothing more is enqueued).
 * Waits once, for the check of R's diagonal (while the first products run;
 * with Rb NULL also inside the QR of B), then enqueues the rest on "stream"
 * and returns: gA is complete when the stream's work is (stream-ordered, like
 * id_reconstruct); work must not be reused on another stream before then. */
int id_backward(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                const int32_t* perm, int64_t k, const double* T, int64_t ldt, const double* Rb,
                int64_t ldrb, const double* gT, int64_t ldgt, const double* gY, int64_t ldgy,
                double* gA, int64_t ldga, void* work, size_t work_bytes, int32_t* info,
                void* stream);

/* ---- sketching front end ----------------------------------------------
 * Randomized column ID (Section 5 names sketching as future work; the paper
 * gives no algorithm).  A random test matrix Omega (l x m, l << m, drawn by
 * the caller, e.g. standard Gaussian entries) compresses the columns of A:
 * Y = Omega A (l x n).  id_factor on Y (FP64, any rank rule) then chooses the
 * skeleton J = perm[0:k] and id_solve_T on Y's R gives T = R_Y11^{-1} R_Y12,
 * so that A ~ A(:, J) T.  For A of exact rank r <= l the result is exact at
 * k = r (Omega injective on the range of A). */

/* Bytes of device workspace id_sketch needs [host]; 0 for invalid sizes. */
size_t id_sketch_workspace_size(int64_t l, int64_t m, int64_t n);

/* Y = Omega A in float64 on the FP64 matrix cores (contraction split over
 * row chunks, chunks summed in a fixed order: the result does not depend on
 * scheduling).
 *   A       [in]  m x n column-major, lda >= max(1, m), dtype ID_F32/ID_F64.
 *   Omega   [in]  l x m float64, ROW-major, ldo >= max(1, m):
 *                 Omega(r, i) = Omega[r * ldo + i].
 *   Y       [out] l x n float64 column-major, ldy >= max(1, l).
 *   work    [in]  workspace of >= id_sketch_workspace_size(l, m, n) bytes,
 *                 8-byte aligned.
 * A non-finite entry of A or Omega propagates into Y (id_factor on Y then
 * reports ID_INFO_NONFINITE).  m = 0 gives Y = 0.  Asynchronous on "stream". */
int id_sketch(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
              const double* Omega, int64_t l, int64_t ldo, double* Y, int64_t ldy, void* work,
              size_t work_bytes, void* stream);

/* ---- batched IDs -------------------------------------------------------
 * One descriptor per matrix, in DEVICE memory (so a call can be captured in a
 * HIP graph and replayed).  Inputs: A, m, n, lda, work.  Outputs: perm, R, T,
 * k, info.  Each item needs its own workspace of
 * id_batch_item_workspace_size(m, n, opts) bytes, 256-byte aligned; the
 * caller owns every buffer.  Every item uses the same opts (same rank rule and
 * tolerance or fixed k).  kcap = min(m, n, k_max if > 0, k_fixed if > 0). */
typedef struct {
  const void* A;  /* m x n column-major, storage dtype of the call */
  int64_t m, n, lda;
  void* work;     /* this item's workspace */
  int32_t* perm;  /* [out] n int32 */
  double* R;      /* [out] k x n float64 in pivot order (R11 upper triangular), ldr >= kcap */
  int64_t ldr;
  double* T;      /* [out] k x (n - k) float64, ldt >= kcap; untouched when info != 0 */
  int64_t ldt;
  int64_t k;      /* [out] rank */
  int32_t info;   /* [out] 0, ID_INFO_NONFINITE, ID_INFO_SINGULAR, ID_INFO_RANK_FULL or
                     ID_INFO_ABORTED */
  int32_t groups; /* [in] workgroups that share this item (1..ID_BATCH_MAX_GROUPS;
                     0 = 1); used only when a slot list is given */
} id_batch_item;

/* Bytes of workspace one batched item of size m x n needs [host]; 0 for
 * invalid arguments (the batched path supports n <= 2048). */
size_t id_batch_item_workspace_size(int64_t m, int64_t n, const id_opts* opts);

/* Many column IDs of uneven sizes (the factorization of Algorithms 1 and 2
 * plus T = R11^{-1} R12) in one persistent launch, then one launch of the
 * batched triangular solve.  Workgroups take slots from a device work queue in
 * the order of "slots"; an item whose index fills items[i].groups consecutive
 * slots is factored by that many workgroups together (each owns a range of
 * the working columns; they agree on pivots and reflectors through exchanges
 * in the item's workspace).  No host synchronization, so the call may be
 * captured in a HIP graph.
 *
 *   items         [in/out] device array of "batch" descriptors.
 *   slots         device array of "nslots" item indices (each item's entries
 *                 consecutive, exactly max(groups, 1) of them), or NULL: one
 *                 workgroup per item, in index order (groups ignored).
 *   queue         device int32 scratch for the work counter (reset here).
 *   max_n         [host] largest n of the batch (sizes the solve grid).
 *   dtype, opts   [host] as in id_factor (opts->flags must be 0).
 *   block_threads [host] 256 or 512 threads per workgroup; 0 = 512.
 *   num_groups    [host] persistent workgroups; 0 or more than the compute
 *                 units = one per compute unit (all must be resident at once).
 * Returns ID_ERR_ARG / ID_ERR_DTYPE for invalid host arguments and
 * ID_ERR_UNSUPPORTED when max_n > 2048; per-item conditions go to items[i].info.
 * An item whose groups exceed the launch's workgroups (num_groups after the
 * caps above) is marked ID_INFO_ABORTED (k = 0) at once, without waiting.
 * A workgroup that waits more than 20 s for the others sharing its item marks
 * the item ID_INFO_ABORTED (k = 0) and every workgroup of the item leaves; a
 * slot list that breaks the rules above ends that way or factors items twice.
 * Calls that share "queue" or an item's workspace must not overlap. */
int id_factor_batched(id_batch_item* items, int32_t batch, const int32_t* slots, int32_t nslots,
                      int32_t* queue, int64_t max_n, int32_t dtype, const id_opts* opts,
                      int32_t block_threads, int32_t num_groups, void* stream);

/* ---- lock-step batches ----------------------------------------------------
 * Many column IDs (the factorization of Algorithms 1 and 2 plus
 * T = R11^{-1} R12, per item) advanced together: every launch runs one kernel
 * of a pivot step (the sweep over the trailing block, the step's finalization)
 * or of a panel end (the blocked update, the column norms) for all unfinished
 * items at once, so each launch streams the trailing blocks of the whole batch
 * and the per-step latencies are shared.  Every item is computed exactly as
 * by id_factor with the same options (the same kernels on its own workspace;
 * only the sweep's tile shapes may differ, which changes rounding order).
 * The host reads every item's state after each panel, so the call
 * synchronizes the stream and cannot be captured in a graph (id_factor_batched
 * can).
 *
 *   items       [in/out] HOST array of "batch" descriptors.  In: A, m, n, lda,
 *               work (device, id_workspace_size(m, n, dtype, opts) bytes, the
 *               same workspace id_factor uses), perm, R, ldr, T, ldt (device
 *               outputs as in id_factor_batched; T untouched when info != 0).
 *               Out: k and info (ID_INFO_NONFINITE, ID_INFO_SINGULAR,
 *               ID_INFO_RANK_FULL or 0, as id_factor then id_solve_T report).
 *               "groups" is ignored.
 *   dtype, opts as in id_factor (ID_FLAG_GRAM, ID_FLAG_CHOLQR and
 *               ID_FLAG_PROFILE refused: ID_ERR_UNSUPPORTED).
 *   work        shared device workspace of id_lockstep_workspace_size bytes
 *               (item tables and block maps).
 * Returns ID_ERR_ARG / ID_ERR_WORKSPACE / ID_ERR_DTYPE for invalid arguments,
 * ID_ERR_UNSUPPORTED for an item with more than 49152 rows (one finalization
 * round trip covers 192 row tiles of at most 256 rows), ID_ERR_HIP on a HIP
 * failure.  Calls that share "work" or an item's workspace must not overlap. */
size_t id_lockstep_workspace_size(const id_batch_item* items, int32_t batch, int32_t dtype,
                                  const id_opts* opts);
int id_factor_lockstep(id_batch_item* items, int32_t batch, int32_t dtype, const id_opts* opts,
                       void* work, size_t work_bytes, void* stream);

/* Per-kernel timing of the calling thread's last id_factor call made with
 * ID_FLAG_PROFILE (instrumentation, not part of the method).  Times come from
 * HIP events recorded around each launch on the call's stream; "bytes" are the
 * algorithmic bytes of the work the kernels did:
 *   sweep: one read of the trailing block per pivot step j,
 *          (m - j) * (n - j - 1) * s bytes, s = 4 (fp32 working copy) or 8;
 *   gemm:  one read and one write of the refreshed block per panel,
 *          2 * (m - j_end) * (n - j_end) * s bytes.
 * Launches that found nothing to do (after the rank was reached or a panel
 * ended early) are not counted. */
typedef struct {
  int64_t sweep_launches;
  double sweep_ms, sweep_bytes;
  int64_t finalize_launches;
  double finalize_ms;
  int64_t gemm_launches;
  double gemm_ms, gemm_bytes;
  double other_ms; /* ingest, norm reductions, bookkeeping */
  double total_ms; /* first to last event of the call */
} id_profile;

int id_last_profile(id_profile* out);

/* Human-readable text for a return or info code [host]. */
const char* id_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* MPID_H */
