// Triangular solves in FP64: T = R11^{-1} R12 (eq. (8); the coefficient step of
// Algorithms 1 and 2) and the general X = op(R)^{-1} B used by the adjoint.
//
// Each block owns 16 right-hand-side columns and walks the 64-row blocks of R
// in dependency order: the contribution of the already-solved row blocks is
// accumulated tile by tile on the FP64 matrix cores, then the 64 x 64 diagonal
// block is solved in registers.  Columns are independent, so blocks never
// synchronize with each other.
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#include "device_util.h"
#include "mpid_internal.h"

namespace mpid {

constexpr int kTB = 64;

typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kTC = 16;  // right-hand-side columns per block

// The value of v in lane SRC of each row of 16 lanes (DPP row broadcast).
template <int SRC>
__device__ __forceinline__ double row_bcast(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x150 + SRC, 0xF,
                                                            0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32),
                                                            0x150 + SRC, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Step II of the diagonal-block solve for one column held by a row of 16
// lanes (lane rg holds rows rg, rg + 16, rg + 32, rg + 48 in x): x_II is
// broadcast from its lane, scaled by 1 / op(R)(II, II), and eliminated from
// the rows below (trans) or above (no trans) it.
template <int II, int TRANS>
__device__ __forceinline__ void diag_step(double (&x)[4], const double (*Rs)[kTB + 1],
                                          const double* rinv, int rg) {
  constexpr int Q = II >> 4, SRC = II & 15;
  const double xi = row_bcast<SRC>(x[Q]) * rinv[II];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rg + 16 * q;
    const double rr = Rs[r][II];
    const bool upd = TRANS ? (r > II) : (r < II);
    x[q] = upd ? x[q] - rr * xi : x[q];
  }
  if (rg == SRC) x[Q] = xi;
}

template <int TRANS, int... Is>
__device__ __forceinline__ void diag_solve(double (&x)[4], const double (*Rs)[kTB + 1],
                                           const double* rinv, int rg,
                                           std::integer_sequence<int, Is...>) {
  (diag_step<TRANS ? Is : kTB - 1 - Is, TRANS>(x, Rs, rinv, rg), ...);
}

// trans = 0: R X = B (back substitution over row blocks, last first).
// trans = 1: R^T X = B (forward substitution, first row block first).
// Per row block I: As = B(I, cols) - sum_L op(R)(I, L) X(L, cols) on the FP64
// matrix cores (wave w owns rows 16w..16w+15), then op(R)(I, I) As = rhs is
// solved with each wave owning four columns, one per row of 16 lanes, in
// registers: the 64 dependent steps pass the solved entry by a DPP row
// broadcast, without LDS round trips or block barriers (rows past the block's
// end hold 0 and have 1 / op(R)(i, i) = 0, so their steps change nothing).
// Columns c0 .. c0 + kTC - 1 of the solve, by one 256-thread block.
__device__ __forceinline__ void trsm_block(const double* __restrict__ R, int64_t ldr, int64_t k,
                                           const double* B, int64_t ldb, int64_t ncols, double* X,
                                           int64_t ldx, int trans, int64_t c0) {
  __shared__ double Rs[kTB][kTB + 1];
  __shared__ double Xs[kTB][kTC + 1];
  __shared__ double As[kTB][kTC + 1];
  __shared__ double rinv[kTB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int la = tid % kTB, lb = tid / kTB;  // load mapping, rows fastest
  const int64_t nblk = ceil_div(k, kTB);
  // Loads are unconditional and issued as one group (a conditional load
  // makes the compiler wait for every earlier load first); entries outside
  // the matrix read R(0, 0) (finite: a nonzero diagonal entry) and are
  // weighted 0.
  auto load_R_tile = [&](int64_t i0, int64_t l0) {
    // Rs[ii][ll] = op(R)(i0 + ii, l0 + ll)
    double v[16], w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = lb + 4 * q;
      const int64_t i = i0 + (trans ? b : la), l = l0 + (trans ? la : b);
      const bool in = i < k && l < k;
      w[q] = in ? 1.0 : 0.0;
      v[q] = R[in ? (trans ? i * ldr + l : l * ldr + i) : 0];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = lb + 4 * q;
      if (!trans)
        Rs[la][b] = v[q] * w[q];
      else
        Rs[b][la] = v[q] * w[q];
    }
  };
  for (int64_t bi = 0; bi < nblk; ++bi) {
    const int64_t I = trans ? bi : nblk - 1 - bi;
    const int64_t i0 = I * kTB;
    const int ib = (int)((k - i0) < kTB ? (k - i0) : kTB);
    {
      // right-hand side (entries outside read B(0, 0), weighted 0) and the
      // reciprocal diagonal, as one group of loads
      double bv[kTC / 4], bw[kTC / 4];
#pragma unroll
      for (int q = 0; q < kTC / 4; ++q) {
        const int64_t c = c0 + lb + 4 * q;
        const bool in = la < ib && c < ncols;
        bw[q] = in ? 1.0 : 0.0;
        bv[q] = B[in ? c * ldb + i0 + la : 0];
      }
      const int td = tid < ib ? tid : 0;
      const double dg = R[(i0 + td) * ldr + i0 + td];
#pragma unroll
      for (int q = 0; q < kTC / 4; ++q) As[la][lb + 4 * q] = bv[q] * bw[q];
      if (tid < kTB) rinv[tid] = tid < ib ? 1.0 / dg : 0.0;
    }
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t bl = 0; bl < bi; ++bl) {
      const int64_t L = trans ? bl : nblk - 1 - bl;
      const int64_t l0 = L * kTB;
      __syncthreads();
      // solved rows of block L (rows past k read row k - 1 and columns past
      // ncols read column ncols - 1: both solved by this block, finite;
      // weighted 0), issued with the R tile
      double xv[kTC / 4], xw[kTC / 4];
#pragma unroll
      for (int q = 0; q < kTC / 4; ++q) {
        const int64_t c = c0 + lb + 4 * q, xr = l0 + la;
        xw[q] = (xr < k && c < ncols) ? 1.0 : 0.0;
        xv[q] = X[(c < ncols ? c : ncols - 1) * ldx + (xr < k ? xr : k - 1)];
      }
      load_R_tile(i0, l0);
#pragma unroll
      for (int q = 0; q < kTC / 4; ++q) Xs[la][lb + 4 * q] = xv[q] * xw[q];
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < kTB / 4; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Rs[16 * wv + li][4 * ks + g], Xs[4 * ks + g][li],
                                                   acc, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) As[16 * wv + g + 4 * r][li] -= acc[r];
    load_R_tile(i0, i0);
    __syncthreads();
    {
      const int col = 4 * wv + (lane >> 4), rg = lane & 15;  // 4 columns x 16 row groups
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = As[rg + 16 * q][col];
      if (!trans)
        diag_solve<0>(x, Rs, rinv, rg, std::make_integer_sequence<int, kTB>());
      else
        diag_solve<1>(x, Rs, rinv, rg, std::make_integer_sequence<int, kTB>());
#pragma unroll
      for (int q = 0; q < 4; ++q) As[rg + 16 * q][col] = x[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTC / 4; ++q) {
      const int b = lb + 4 * q;
      const int64_t c = c0 + b;
      if (la < ib && c < ncols) X[c * ldx + i0 + la] = As[la][b];
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_trsm_upper(const double* __restrict__ R, int64_t ldr,
                                                        int64_t k, const double* B, int64_t ldb,
                                                        int64_t ncols, double* X, int64_t ldx,
                                                        int trans, const int32_t* info) {
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = !(info && *info == ID_INFO_SINGULAR);
  __syncthreads();
  if (!s_go) return;
  trsm_block(R, ldr, k, B, ldb, ncols, X, ldx, trans, (int64_t)blockIdx.x * kTC);
}

// T = R11^{-1} R12 of every item of a batch: blockIdx.x = item, blockIdx.y =
// column block.  Items with a nonzero info (failed, singular R11, aborted, or
// k == n) and column blocks beyond an item's n - k leave at once.
__global__ __launch_bounds__(kThreads) void k_trsm_batched(const id_batch_item* __restrict__ items) {
  const id_batch_item& it = items[blockIdx.x];
  const int64_t k = it.k, n = it.n;
  const int64_t c0 = (int64_t)blockIdx.y * kTC;
  if (it.info != 0 || k <= 0 || c0 >= n - k) return;
  trsm_block(it.R, it.ldr, k, it.R + k * it.ldr, it.ldr, n - k, it.T, it.ldt, 0, c0);
}

// info = ID_INFO_SINGULAR when some |R_ii| <= n * 2^-53 * |R_00| (or R_00 = 0),
// ID_INFO_RANK_FULL when k == n, else 0.
__global__ __launch_bounds__(kThreads) void k_check_diag(const double* __restrict__ R, int64_t ldr,
                                                         int64_t k, int64_t n, int32_t* info) {
  __shared__ double dscr[4];
  const int tid = threadIdx.x;
  const double r00 = k > 0 ? fabs(R[0]) : 0.0;
  const double thr = (double)n * ldexp(1.0, -53) * r00;
  double bad = 0.0;
  for (int64_t i = tid; i < k; i += kThreads)
    if (!(fabs(R[i * ldr + i]) > thr)) bad += 1.0;
  bad = block_sum(bad, dscr);
  if (tid == 0) {
    if (k > 0 && (bad > 0.0 || r00 == 0.0))
      *info = ID_INFO_SINGULAR;
    else
      *info = (k == n) ? ID_INFO_RANK_FULL : 0;
  }
}

int trsm_upper_run(const double* R, int64_t ldr, int64_t k, const double* B, int64_t ldb,
                   int64_t ncols, double* X, int64_t ldx, int trans, hipStream_t s) {
  if (k <= 0 || ncols <= 0) return ID_OK;
  k_trsm_upper<<<dim3((unsigned)ceil_div(ncols, kTC)), kThreads, 0, s>>>(R, ldr, k, B, ldb, ncols,
                                                                         X, ldx, trans, nullptr);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

// X = R^{-1} R^{-T} B (the normal-equations solve (R^T R)^{-1} B): both
// solves of a column block back to back in one launch, R^{-T} B written over
// B first.
__global__ __launch_bounds__(kThreads) void k_trsm_upper_normal(const double* __restrict__ R,
                                                               int64_t ldr, int64_t k, double* B,
                                                               int64_t ldb, int64_t ncols,
                                                               double* X, int64_t ldx) {
  const int64_t c0 = (int64_t)blockIdx.x * kTC;
  trsm_block(R, ldr, k, B, ldb, ncols, B, ldb, 1, c0);
  __syncthreads();  // the first solve's last reads of LDS are done
  trsm_block(R, ldr, k, B, ldb, ncols, X, ldx, 0, c0);
}

int trsm_normal_run(const double* R, int64_t ldr, int64_t k, double* B, int64_t ldb,
                    int64_t ncols, double* X, int64_t ldx, hipStream_t s) {
  if (k <= 0 || ncols <= 0) return ID_OK;
  k_trsm_upper_normal<<<dim3((unsigned)ceil_div(ncols, kTC)), kThreads, 0, s>>>(R, ldr, k, B, ldb,
                                                                                ncols, X, ldx);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

int trsm_batched_run(const id_batch_item* items, int32_t batch, int64_t max_n, hipStream_t s) {
  if (batch <= 0 || max_n <= 0) return ID_OK;
  k_trsm_batched<<<dim3((unsigned)batch, (unsigned)ceil_div(max_n, kTC)), kThreads, 0, s>>>(items);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

int solve_T_run(const double* R, int64_t ldr, int64_t k, int64_t n, double* T, int64_t ldt,
                int32_t* info, hipStream_t s) {
  if (!info || k < 0 || n < k) return ID_ERR_ARG;
  if (k > 0 && (!R || ldr < k)) return ID_ERR_ARG;
  if (n - k > 0 && k > 0 && (!T || ldt < k)) return ID_ERR_ARG;
  k_check_diag<<<1, kThreads, 0, s>>>(R, ldr, k, n, info);
  MPID_LAUNCH_CHECK();
  if (k == 0 || n == k) return ID_OK;
  k_trsm_upper<<<dim3((unsigned)ceil_div(n - k, kTC)), kThreads, 0, s>>>(
      R, ldr, k, R + k * ldr, ldr, n - k, T, ldt, 0, info);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

// X (rows x cols, column-major, ld) rounded in place to the nearest binary32
// (mode 1) or binary16 (mode 2) values: the low-precision coefficients of
// the simulated single / half precision ID.
__global__ __launch_bounds__(kThreads) void k_round(double* X, int64_t rows, int64_t cols,
                                                    int64_t ld, int mode) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= rows || c >= cols) return;
  double* p = X + c * ld + i;
  *p = mode == 1 ? (double)(float)*p : (double)(_Float16)*p;
}

int round_run(double* X, int64_t rows, int64_t cols, int64_t ld, int32_t mode, hipStream_t s) {
  if (rows < 0 || cols < 0 || (mode != 1 && mode != 2)) return ID_ERR_ARG;
  if (rows == 0 || cols == 0) return ID_OK;
  if (!X || ld < rows || cols > 65535) return ID_ERR_ARG;
  k_round<<<dim3((unsigned)ceil_div(rows, kThreads), (unsigned)cols), kThreads, 0, s>>>(X, rows, cols,
                                                                                       ld, mode);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

}  // namespace mpid
