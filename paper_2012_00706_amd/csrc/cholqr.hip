// Tall-skinny front end through a CholeskyQR R factor (ID_FLAG_CHOLQR).
//
// The column-pivoted QR of A and of any R0 with A = Q R0 (Q with orthonormal
// columns) are the same factorization: the column norms and every Householder
// step agree (Section 1.1, eq. (6)-(7)), so the pivots and R of A are those of
// the n x n matrix R0.  R0 comes from CholeskyQR passes: a pass on a matrix
// X computes R = chol(X^T X) and the next matrix X R^{-1}.
//   * CholeskyQR2 (Yamamoto, Nakatsukasa, Yanagisawa and Fukaya 2015):
//     R1 = chol(A^T A), A1 = A R1^{-1}, R2 = chol(A1^T A1), R0 = R2 R1.  It
//     is taken when the first Cholesky factorization succeeds and
//     ||R2 - I||_F <= 1/2: then kappa(A1) <= 3, so the second pass leaves an
//     orthonormal Q = A1 R2^{-1} to working precision.
//   * Otherwise a third pass, R3 = chol(A2^T A2) with A2 = A1 R2^{-1},
//     R0 = R3 R2 R1, accepted when ||R3 - I||_F <= 1/2.  When the first
//     factorization fails, it is redone on A^T A + s I with
//     s = 11 (m n + n (n + 1)) u_64 ||A||_F^2 (the same Gram matrix, kept
//     aside) and all three passes run: shifted CholeskyQR3 (Fukaya, Kannan,
//     Nakatsukasa, Yamamoto and Yanagisawa 2020).
// Each pass reads its matrix twice on the FP64 matrix cores (the Gram product
// and the right multiplication by the triangular R^{-1}, whose zero half is
// skipped); the pivoted factorization (FP64 Householder, the single-matrix
// path) then runs on R0.  Unlike the Gram front end, residual norms are
// resolved down to about u_64 ||A|| instead of sqrt(u_64) ||A||.
// The route needs A to have full numerical column rank: the shift leaves A1
// with a condition number of about kappa(A) sqrt(11 (m n + n^2) u_64), and
// the plain passes need it below about u_64^{-1/2}.  When a plain pass breaks
// down, or the last R is not close to the identity, the call reports
// ID_INFO_CHOLQR_BREAKDOWN and factors nothing (k = 0).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "device_util.h"
#include "mpid_internal.h"

namespace mpid {

namespace {

constexpr int kCB = 64;  // Cholesky panel width

// Flags written by the device (int32 each): [0] A non-finite, [1] a Cholesky
// pivot not positive / not finite, [2] the pass's R far from the identity,
// [3] A = 0.
enum { CF_NONFINITE = 0, CF_BREAKDOWN = 1, CF_NOT_ORTHO = 2, CF_ZERO = 3, CF_COUNT = 4 };

__global__ void k_cq_zero_flags(int32_t* f) {
  if (threadIdx.x < CF_COUNT) f[threadIdx.x] = 0;
}

// X = I (n x n, ld n).
__global__ __launch_bounds__(kThreads) void k_cq_eye(double* __restrict__ X, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n * n) return;
  X[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// G_ii += c trace(G), one block; flags a zero A (trace 0).
__global__ __launch_bounds__(kThreads) void k_cq_shift(double* __restrict__ G, int64_t n,
                                                       double c, int32_t* __restrict__ flags) {
  __shared__ double dscr[4];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) t += G[i * n + i];
  t = block_sum(t, dscr);
  if (threadIdx.x == 0 && t == 0.0) flags[CF_ZERO] = 1;
  const double s = c * t;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) G[i * n + i] += s;
}

// X[0 .. count) = 0.
__global__ __launch_bounds__(kThreads) void k_cq_zero(double* __restrict__ X, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e < count) X[e] = 0.0;
}

// The wave-uniform value of lane "lane"'s v.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Cholesky factorization of the diagonal block G(p0 : p0 + nb, same) after
// the earlier panels' updates (upper factor R_pp with R_pp^T R_pp = G_pp), by
// one wavefront: the block's upper triangle is staged through LDS
// (coalesced), then lane j holds column j in registers.  Step c reads G(c, c)
// from lane c, every lane scales its entry of row c by 1 / sqrt(G(c, c)) and
// publishes it in LDS (double-buffered: one barrier per step), and every lane
// updates its column, G(i, j) -= R(c, i) R(c, j).  Rows and columns past nb are the
// identity (finite, and they leave the block's entries alone).  Writes
// R(p0 + i, p0 + j) for i, j < nb (zero below the diagonal) and flags a
// pivot that is not positive and finite (replaced by 1 so that nothing
// becomes NaN).
__global__ __launch_bounds__(kCB) void k_cq_chol_diag(const double* __restrict__ G, int64_t n,
                                                      int64_t p0, int nb,
                                                      double* __restrict__ R,
                                                      int32_t* __restrict__ flags) {
  __shared__ double Gs[kCB][kCB + 1];  // Gs[i][j] = G(p0 + i, p0 + j), j >= i
  __shared__ double row[2][kCB];
  const int j = threadIdx.x;
  {
    // lane i loads row i of the block, column by column (coalesced across
    // lanes): all 64 loads unconditional from clamped in-bounds addresses and
    // in flight together, masked when they go to LDS
    const int i = j;
    const int64_t ic = i < nb ? i : 0;
    double t[kCB];
#pragma unroll
    for (int jj = 0; jj < kCB; ++jj) {
      const int64_t jc = jj < nb ? jj : 0;
      t[jj] = G[(p0 + jc) * n + p0 + ic];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int jj = 0; jj < kCB; ++jj)
      Gs[i][jj] = (i < nb && jj < nb) ? (jj >= i ? t[jj] : 0.0) : (i == jj ? 1.0 : 0.0);
  }
  __syncthreads();
  double g[kCB];  // g[i] = G(i, j), then R(i, j)
#pragma unroll
  for (int i = 0; i < kCB; ++i) g[i] = Gs[i][j];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    double* rw = row[c & 1];
    double d = readlane_f64(g[c], c);  // G(c, c), from lane c
    if (!(d > 0.0) || !isfinite(d)) {
      bad = true;
      d = 1.0;
    }
    // 1 / sqrt(G(c, c)): the hardware estimate refined by two Newton steps
    double y = __builtin_amdgcn_rsq(d);
    y = y * (1.5 - 0.5 * d * y * y);
    y = y * (1.5 - 0.5 * d * y * y);
    const double rcj = j == c ? d * y : g[c] * y;  // R(c, j)
    g[c] = rcj;
    rw[j] = rcj;  // row c of R, published
    __syncthreads();
#pragma unroll
    for (int i = c + 1; i < kCB; ++i) g[i] -= rw[i] * rcj;
  }
  if (bad && j == 0) flags[CF_BREAKDOWN] = 1;
#pragma unroll
  for (int i = 0; i < kCB; ++i) Gs[i][j] = i <= j ? g[i] : 0.0;
  __syncthreads();
  for (int e = j; e < kCB * kCB; e += kCB) {
    const int i = e % kCB, jj = e / kCB;
    if (i < nb && jj < nb) R[(p0 + jj) * n + p0 + i] = Gs[i][jj];
  }
}

// ||R - I||_F^2 in two steps: part[j] = sum_i (R(i, j) - delta_ij)^2 (one
// block per column), then flags[CF_NOT_ORTHO] when the sum exceeds 1/4 (or is
// not finite).  Below it ||R - I||_2 <= 1/2, so the pass's matrix X
// (R = chol(X^T X)) has kappa(X) = kappa(R) <= 3.
__global__ __launch_bounds__(kThreads) void k_cq_dev_cols(const double* __restrict__ R, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double dscr[4];
  const int64_t j = blockIdx.x;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const double v = R[j * n + i] - (i == j ? 1.0 : 0.0);
    ss += v * v;
  }
  ss = block_sum(ss, dscr);
  if (threadIdx.x == 0) part[j] = ss;
}

__global__ __launch_bounds__(kThreads) void k_cq_dev_check(const double* __restrict__ part,
                                                           int64_t n, int32_t* __restrict__ flags) {
  __shared__ double dscr[4];
  double ss = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += kThreads) ss += part[j];
  ss = block_sum(ss, dscr);
  if (threadIdx.x == 0 && !(ss <= 0.25)) flags[CF_NOT_ORTHO] = 1;
}

__global__ void k_cq_iota(int32_t* perm, int64_t n) {
  const int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (l < n) perm[l] = (int32_t)l;
}

struct CqPlan {
  int64_t m, n;
  size_t off_g, off_g0, off_r[3], off_rinv, off_r0, off_tmp, off_part, off_a[2], off_flags,
      off_inner;
  size_t part_bytes, inner_bytes, bytes;
  id_opts inner;  // the pivoted factorization of R0 (FP64)
};

bool make_cq_plan(int64_t m, int64_t n, int32_t dtype, const id_opts* o, CqPlan* p) {
  if (!o || !p || m < 0 || n < 0) return false;
  if (dtype != ID_F32 && dtype != ID_F64) return false;
  std::memset(p, 0, sizeof(*p));
  p->m = m;
  p->n = n;
  p->inner = *o;
  p->inner.prec = ID_PREC_F64;
  p->inner.flags = 0;
  FactorPlan fp;
  const int64_t nn = n > 0 ? n : 1, mm = m > 0 ? m : 1;
  if (!make_factor_plan(nn, nn, ID_F64, &p->inner, &fp)) return false;
  p->inner_bytes = fp.bytes;
  p->part_bytes = gram_matrix_workspace(mm, nn);
  if (p->part_bytes == 0) return false;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off += (b + 255) / 256 * 256;
    return at;
  };
  const size_t n2 = (size_t)nn * nn * 8;
  p->off_g = take(n2);
  p->off_g0 = take(n2);
  for (int q = 0; q < 3; ++q) p->off_r[q] = take(n2);
  p->off_rinv = take(n2);
  p->off_r0 = take(n2);
  p->off_tmp = take(n2);
  p->off_part = take(p->part_bytes);
  p->off_a[0] = take((size_t)mm * nn * 8);
  p->off_a[1] = take((size_t)mm * nn * 8);
  p->off_flags = take(CF_COUNT * 4);
  p->off_inner = take(p->inner_bytes);
  p->bytes = off;
  return true;
}

// R = chol(G) by 64-column panels: the diagonal block by one wavefront, the
// block row right of it by a triangular solve with its transpose, the
// trailing matrix updated on the matrix cores.  G is overwritten; R's strictly
// lower triangle is zeroed first.
int cholesky_run(double* G, int64_t n, double* R, int32_t* flags, hipStream_t s) {
  k_cq_zero<<<dim3((unsigned)ceil_div(n * n, kThreads)), kThreads, 0, s>>>(R, n * n);
  MPID_LAUNCH_CHECK();
  for (int64_t p0 = 0; p0 < n; p0 += kCB) {
    const int nb = (int)(n - p0 < kCB ? n - p0 : kCB);
    k_cq_chol_diag<<<1, kCB, 0, s>>>(G, n, p0, nb, R, flags);
    MPID_LAUNCH_CHECK();
    const int64_t r0 = p0 + nb, nr = n - r0;
    if (nr <= 0) continue;
    // R(p0 : r0, r0 : n) = R_pp^{-T} G(p0 : r0, r0 : n)
    int rc = trsm_upper_run(R + p0 * n + p0, n, nb, G + r0 * n + p0, n, nr, R + r0 * n + p0, n, 1,
                            s);
    if (rc) return rc;
    // G(r0 : n, r0 : n) -= R(p0 : r0, r0 : n)^T R(p0 : r0, r0 : n)
    rc = gemm64_run(1, 0, nr, nr, nb, -1.0, R + r0 * n + p0, n, R + r0 * n + p0, n, 1.0,
                    G + r0 * n + r0, n, s);
    if (rc) return rc;
  }
  return ID_OK;
}

}  // namespace

size_t cholqr_workspace(int64_t m, int64_t n, int32_t dtype, const id_opts* o) {
  CqPlan p;
  if (!make_cq_plan(m, n, dtype, o, &p)) return 0;
  return p.bytes;
}

int cholqr_factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                      const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                      int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s) {
  if (!o) return ID_ERR_ARG;
  if (o->flags & (ID_FLAG_GRAM | ID_FLAG_NO_PIVOT | ID_FLAG_PROFILE | ID_FLAG_ROUND_F32 |
                  ID_FLAG_ROUND_F16))
    return ID_ERR_UNSUPPORTED;
  CqPlan pl;
  if (!make_cq_plan(m, n, dtype, o, &pl)) return ID_ERR_ARG;
  if (!k_out || !info) return ID_ERR_ARG;
  if (n > 0 && !perm) return ID_ERR_ARG;
  if (m > 0 && n > 0 && !A) return ID_ERR_ARG;
  if (lda < (m > 1 ? m : 1)) return ID_ERR_ARG;
  FactorPlan fp;
  if (!make_factor_plan(m, n, dtype, o, &fp)) return ID_ERR_ARG;
  if (fp.kcap > 0 && (!R || ldr < fp.kcap)) return ID_ERR_ARG;
  if (m < n) return ID_ERR_UNSUPPORTED;  // R0 needs full column rank: a tall A
  if (!work || work_bytes < pl.bytes) return ID_ERR_WORKSPACE;
  *info = 0;
  *k_out = 0;
  if (m == 0 || n == 0 || fp.kcap == 0) {
    if (n > 0) {
      k_cq_iota<<<dim3((unsigned)ceil_div(n, kThreads)), kThreads, 0, s>>>(perm, n);
      MPID_LAUNCH_CHECK();
    }
    return ID_OK;
  }
  char* wb = (char*)work;
  double* G = (double*)(wb + pl.off_g);
  double* Rk[3] = {(double*)(wb + pl.off_r[0]), (double*)(wb + pl.off_r[1]),
                   (double*)(wb + pl.off_r[2])};
  double* Rinv = (double*)(wb + pl.off_rinv);
  double* R0 = (double*)(wb + pl.off_r0);
  double* Tmp = (double*)(wb + pl.off_tmp);
  double* Ab[2] = {(double*)(wb + pl.off_a[0]), (double*)(wb + pl.off_a[1])};
  int32_t* flags = (int32_t*)(wb + pl.off_flags);
  double* G0 = (double*)(wb + pl.off_g0);
  const size_t n2 = (size_t)n * n * sizeof(double);
  int rc;
  int32_t hf[CF_COUNT];
  auto read_flags = [&]() -> int {
    MPID_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    MPID_HIP(hipStreamSynchronize(s));
    return ID_OK;
  };
  // k = 0 with the identity permutation and the given info
  auto stop = [&](int32_t why) -> int {
    *info = why;
    k_cq_iota<<<dim3((unsigned)ceil_div(n, kThreads)), kThreads, 0, s>>>(perm, n);
    MPID_LAUNCH_CHECK();
    return ID_OK;
  };
  const unsigned eye_blocks = (unsigned)ceil_div(n * n, kThreads);
  // X_{q+1} = X_q R_q^{-1} (R_q^{-1} formed by a triangular solve on I)
  auto next_matrix = [&](const void* Xq, int32_t dq, int64_t ldq, const double* Rq,
                         double* Xn) -> int {
    k_cq_eye<<<eye_blocks, kThreads, 0, s>>>(Rinv, n);
    MPID_LAUNCH_CHECK();
    int r = trsm_upper_run(Rq, n, n, Rinv, n, n, Rinv, n, 0, s);
    if (r) return r;
    return gemm64_typed_run(Xq, dq, m, n, n, ldq, Rinv, n, Xn, m, 1, s);
  };
  // flags[CF_NOT_ORTHO] when ||R - I||_F > 1/2 (column sums staged in Tmp)
  auto check_identity = [&](const double* Rq) -> int {
    k_cq_dev_cols<<<dim3((unsigned)n), kThreads, 0, s>>>(Rq, n, Tmp);
    MPID_LAUNCH_CHECK();
    k_cq_dev_check<<<1, kThreads, 0, s>>>(Tmp, n, flags);
    MPID_LAUNCH_CHECK();
    return ID_OK;
  };
  k_cq_zero_flags<<<1, 64, 0, s>>>(flags);
  MPID_LAUNCH_CHECK();
  // pass 1: R1 = chol(A^T A), the Gram matrix kept aside for a shifted retry
  if ((rc = gram_matrix_run(A, dtype, m, n, lda, G, wb + pl.off_part, pl.part_bytes,
                            &flags[CF_NONFINITE], s)))
    return rc;
  k_cq_shift<<<1, kThreads, 0, s>>>(G, n, 0.0, flags);  // flags A = 0
  MPID_LAUNCH_CHECK();
  MPID_HIP(hipMemcpyAsync(G0, G, n2, hipMemcpyDeviceToDevice, s));
  if ((rc = cholesky_run(G, n, Rk[0], flags, s))) return rc;
  if ((rc = read_flags())) return rc;
  if (hf[CF_NONFINITE]) return stop(ID_INFO_NONFINITE);
  if (hf[CF_ZERO]) return stop(0);  // rank 0, as on the other routes
  const bool shifted = hf[CF_BREAKDOWN] != 0;
  if (shifted) {
    k_cq_zero_flags<<<1, 64, 0, s>>>(flags);
    MPID_LAUNCH_CHECK();
    const double c = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) *
                     std::ldexp(1.0, -53);
    k_cq_shift<<<1, kThreads, 0, s>>>(G0, n, c, flags);
    MPID_LAUNCH_CHECK();
    if ((rc = cholesky_run(G0, n, Rk[0], flags, s))) return rc;
  }
  // pass 2 on A1 = A R1^{-1}
  if ((rc = next_matrix(A, dtype, lda, Rk[0], Ab[0]))) return rc;
  if ((rc = gram_matrix_run(Ab[0], ID_F64, m, n, m, G, wb + pl.off_part, pl.part_bytes,
                            &flags[CF_NONFINITE], s)))
    return rc;
  if ((rc = cholesky_run(G, n, Rk[1], flags, s))) return rc;
  if ((rc = check_identity(Rk[1]))) return rc;
  if ((rc = read_flags())) return rc;
  if (hf[CF_NONFINITE]) return stop(ID_INFO_NONFINITE);
  if (hf[CF_BREAKDOWN]) return stop(ID_INFO_CHOLQR_BREAKDOWN);
  if (!shifted && !hf[CF_NOT_ORTHO]) {
    // CholeskyQR2: R0 = R2 R1
    if ((rc = gemm64_run(0, 0, n, n, n, 1.0, Rk[1], n, Rk[0], n, 0.0, R0, n, s))) return rc;
  } else {
    // pass 3 on A2 = A1 R2^{-1}: R0 = R3 R2 R1
    k_cq_zero_flags<<<1, 64, 0, s>>>(flags);
    MPID_LAUNCH_CHECK();
    if ((rc = next_matrix(Ab[0], ID_F64, m, Rk[1], Ab[1]))) return rc;
    if ((rc = gram_matrix_run(Ab[1], ID_F64, m, n, m, G, wb + pl.off_part, pl.part_bytes,
                              &flags[CF_NONFINITE], s)))
      return rc;
    if ((rc = cholesky_run(G, n, Rk[2], flags, s))) return rc;
    if ((rc = check_identity(Rk[2]))) return rc;
    if ((rc = gemm64_run(0, 0, n, n, n, 1.0, Rk[2], n, Rk[1], n, 0.0, Tmp, n, s))) return rc;
    if ((rc = gemm64_run(0, 0, n, n, n, 1.0, Tmp, n, Rk[0], n, 0.0, R0, n, s))) return rc;
    if ((rc = read_flags())) return rc;
    if (hf[CF_NONFINITE]) return stop(ID_INFO_NONFINITE);
    if (hf[CF_BREAKDOWN] || hf[CF_NOT_ORTHO]) return stop(ID_INFO_CHOLQR_BREAKDOWN);
  }
  // the pivoted factorization of the n x n R0 (same rank rule and options)
  return factor_run(R0, ID_F64, n, n, n, &pl.inner, wb + pl.off_inner, pl.inner_bytes, perm, R,
                    ldr, k_out, info, s);
}

}  // namespace mpid
