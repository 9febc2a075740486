// FP64 matrix-core GEMM and the two consumers of the factorization that are
// pure products: the reconstruction A(:, J) P (eq. (4)-(5), (8); evaluated in
// double precision as in the remark after Lemma 1) and the adjoint of T and of
// the reconstruction with the skeleton held fixed.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "mpid_internal.h"

namespace mpid {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename TA, typename TC>
struct G64Args {
  int ta, tb;
  int64_t M, N, K;
  double alpha;
  const TA* A;  // op(A): M x K; amap maps op(A)'s column index (ta == 0)
  int64_t lda;
  const int32_t* amap;
  const double* B;  // op(B): K x N
  int64_t ldb;
  double beta;
  const TC* Cin;  // Cin(i, cinmap[j])
  int64_t ldcin;
  const int32_t* cinmap;
  double* C;  // C(i, cmap[j])
  int64_t ldc;
  const int32_t* cmap;
  // optional second output of the large-tile kernel (no split K):
  // E(i, j) = (Ein ? Ein(i, einmap[j]) : 0) - C(i, cmap[j])
  double* E;
  int64_t lde;
  const double* Ein;
  int64_t ldein;
  const int32_t* einmap;
  // op(B) upper triangular (zero below the diagonal): the large-tile kernel
  // contracts a column tile only over the rows of B at or above its last column
  int b_upper;
};

// C = alpha op(A) op(B) + beta Cin, 64 x 64 tile per block, K chunks of 16
// staged through LDS (the next chunk loaded into registers during the
// products), four waves of 2 x 2 FP64 16x16x4 MFMA blocks.
template <typename TA, typename TC>
__global__ __launch_bounds__(kThreads) void k_gemm64(G64Args<TA, TC> a) {
  __shared__ double As[16][64 + 1];  // As[kk][i] = op(A)(m0 + i, k0 + kk)
  __shared__ double Bs[16][64 + 1];  // Bs[kk][j] = op(B)(k0 + kk, n0 + j)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (f64x4){0.0, 0.0, 0.0, 0.0};

  // the next K chunk's operands are loaded into registers while the current
  // one is multiplied out of LDS
  // Loads are unconditional, from indices clamped into the operands, and
  // issued as one group (a conditional load makes the compiler wait for every
  // earlier load first); entries outside the operands are weighted 0.  A
  // clamped entry is a real entry of the same operand row or column, so a
  // non-finite value there already reaches every output it could reach here.
  double ra[4], rb[4], wa[4], wb[4];
  auto load = [&](int64_t k0) {
    // op(A) columns through the column map: the four map entries first
    int64_t col[4];
    if (a.ta == 0 && a.amap) {  // uniform
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gk = k0 + tid / 64 + 4 * q;
        col[q] = (int64_t)a.amap[gk < a.K ? gk : a.K - 1];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gk = k0 + tid / 64 + 4 * q;
        col[q] = gk < a.K ? gk : a.K - 1;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (a.ta == 0) {
        const int i = tid % 64, kk = tid / 64 + 4 * q;
        const int64_t gi = m0 + i, gk = k0 + kk;
        const int64_t gic = gi < a.M ? gi : a.M - 1;
        wa[q] = (gi < a.M && gk < a.K) ? 1.0 : 0.0;
        ra[q] = (double)a.A[col[q] * a.lda + gic];
      } else {
        const int kk = tid % 16, i = tid / 16 + 16 * q;
        const int64_t gi = m0 + i, gk = k0 + kk;
        const int64_t gic = gi < a.M ? gi : a.M - 1, gkc = gk < a.K ? gk : a.K - 1;
        wa[q] = (gi < a.M && gk < a.K) ? 1.0 : 0.0;
        ra[q] = (double)a.A[gic * a.lda + gkc];
      }
      if (a.tb == 0) {
        const int kk = tid % 16, j = tid / 16 + 16 * q;
        const int64_t gj = n0 + j, gk = k0 + kk;
        const int64_t gjc = gj < a.N ? gj : a.N - 1, gkc = gk < a.K ? gk : a.K - 1;
        wb[q] = (gj < a.N && gk < a.K) ? 1.0 : 0.0;
        rb[q] = a.B[gjc * a.ldb + gkc];
      } else {
        const int j = tid % 64, kk = tid / 64 + 4 * q;
        const int64_t gj = n0 + j, gk = k0 + kk;
        const int64_t gjc = gj < a.N ? gj : a.N - 1, gkc = gk < a.K ? gk : a.K - 1;
        wb[q] = (gj < a.N && gk < a.K) ? 1.0 : 0.0;
        rb[q] = a.B[gkc * a.ldb + gjc];
      }
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < a.K; k0 += 16) {
    __syncthreads();  // the previous chunk's products are done with LDS
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (a.ta == 0)
        As[tid / 64 + 4 * q][tid % 64] = ra[q] * wa[q];
      else
        As[tid % 16][tid / 16 + 16 * q] = ra[q] * wa[q];
      if (a.tb == 0)
        Bs[tid % 16][tid / 16 + 16 * q] = rb[q] * wb[q];
      else
        Bs[tid / 64 + 4 * q][tid % 64] = rb[q] * wb[q];
    }
    __syncthreads();
    if (k0 + 16 < a.K) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = As[4 * ks + g][wr + 16 * x + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = Bs[4 * ks + g][wc + 16 * y + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
  }
  // acc[x][y][r] = C(m0 + wr + 16x + g + 4r, n0 + wc + 16y + li); the
  // column maps, then every Cin entry (clamped indices, used only in range),
  // are loaded as groups before the stores
  int64_t cj[2], ij[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int64_t j = n0 + wc + 16 * y + li;
    const int64_t jc = j < a.N ? j : a.N - 1;
    cj[y] = a.cmap ? (int64_t)a.cmap[jc] : jc;
    ij[y] = a.cinmap ? (int64_t)a.cinmap[jc] : jc;
  }
  double cin[2][2][4];
  if (a.beta != 0.0) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = m0 + wr + 16 * x + g + 4 * r;
          cin[x][y][r] = (double)a.Cin[ij[y] * a.ldcin + (i < a.M ? i : a.M - 1)];
        }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int64_t j = n0 + wc + 16 * y + li;
      if (j >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + wr + 16 * x + g + 4 * r;
        if (i >= a.M) continue;
        double v = a.alpha * acc[x][y][r];
        if (a.beta != 0.0) v += a.beta * cin[x][y][r];
        a.C[cj[y] * a.ldc + i] = v;
      }
    }
}

// Larger products: a 128 x 128 tile per block, the four waves as 2 x 2 each
// computing a 64 x 64 part from 4 x 4 FP64 16x16x4 MFMA blocks (four times the
// matrix-core work of k_gemm64 between two barriers), K in chunks of 16
// through LDS with the next chunk loaded into registers during the products.
// Operand and output lane layouts are those of k_gemm64.  With gridDim.z > 1
// (split K) block z sums the K range [z kc, (z + 1) kc) into its own partial
// P + z M N (column-major, ld M) and k_gemm64_reduce applies the epilogue.
// Two waves per SIMD: the register budget (236 of 256) keeps the 64 accumulators
// in VGPRs without spilling.  One launch may run two products that share M
// and K: the blocks with blockIdx.y >= ny0 compute the second (a1).
template <typename TA, typename TC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm64t(
    G64Args<TA, TC> a0, G64Args<TA, TC> a1, unsigned ny0, int64_t kc, double* __restrict__ P) {
  const bool second = blockIdx.y >= ny0;
  const G64Args<TA, TC>& a = second ? a1 : a0;
  const unsigned by = second ? blockIdx.y - ny0 : blockIdx.y;
  __shared__ double As[16][128 + 2];  // As[kk][i] = op(A)(m0 + i, k0 + kk)
  __shared__ double Bs[16][128 + 2];  // Bs[kk][j] = op(B)(k0 + kk, n0 + j)
  __shared__ int32_t smap[3][128];    // the tile's output, Cin and Ein columns
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.x * 128, n0 = (int64_t)by * 128;
  const int wr = (wv & 1) * 64, wc = (wv >> 1) * 64;
  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke0 = kb + kc < a.K ? kb + kc : a.K;
  const int64_t ke = (a.b_upper && ke0 > n0 + 128) ? n0 + 128 : ke0;
  f64x4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = (f64x4){0.0, 0.0, 0.0, 0.0};

  // Loads are unconditional from indices clamped into the operands and issued
  // as one group; entries outside the product are zeroed when they go to LDS
  // (a clamped entry is a real entry of the same operand row or column).
  double ra[8], rb[8];
  auto load = [&](int64_t k0) {
    int64_t col[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t gk = k0 + tid / 128 + 2 * q;
      const int64_t gkc = gk < ke ? gk : ke - 1;
      col[q] = (a.ta == 0 && a.amap) ? (int64_t)a.amap[gkc] : gkc;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (a.ta == 0) {  // op(A)(i, kk): 128 consecutive rows of one column per half-block
        const int64_t gi = m0 + tid % 128;
        ra[q] = (double)a.A[col[q] * a.lda + (gi < a.M ? gi : a.M - 1)];
      } else {          // A(kk, i) row-major in the contraction
        const int64_t gi = m0 + tid / 16 + 16 * q, gk = k0 + tid % 16;
        ra[q] = (double)a.A[(gi < a.M ? gi : a.M - 1) * a.lda + (gk < ke ? gk : ke - 1)];
      }
      if (a.tb == 0) {  // B(kk, j) = B[j ldb + kk]
        const int64_t gj = n0 + tid / 16 + 16 * q, gk = k0 + tid % 16;
        rb[q] = a.B[(gj < a.N ? gj : a.N - 1) * a.ldb + (gk < ke ? gk : ke - 1)];
      } else {          // B(kk, j) = B[kk ldb + j]
        const int64_t gj = n0 + tid % 128, gk = k0 + tid / 128 + 2 * q;
        rb[q] = a.B[(gk < ke ? gk : ke - 1) * a.ldb + (gj < a.N ? gj : a.N - 1)];
      }
    }
  };
  if (kb < ke) load(kb);
  // the epilogue's column maps, ready by its time (the main loop's barriers
  // publish them)
  if (tid < 128) {
    const int64_t j = n0 + tid;
    const int64_t jc = j < a.N ? j : a.N - 1;
    smap[0][tid] = a.cmap ? a.cmap[jc] : (int32_t)jc;
    smap[1][tid] = a.cinmap ? a.cinmap[jc] : (int32_t)jc;
    smap[2][tid] = a.einmap ? a.einmap[jc] : (int32_t)jc;
  }
  if (kb >= ke) __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    __syncthreads();  // the previous chunk's products are done with LDS
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (a.ta == 0) {
        const int i = tid % 128, kk = tid / 128 + 2 * q;
        As[kk][i] = (m0 + i < a.M && k0 + kk < ke) ? ra[q] : 0.0;
      } else {
        const int kk = tid % 16, i = tid / 16 + 16 * q;
        As[kk][i] = (m0 + i < a.M && k0 + kk < ke) ? ra[q] : 0.0;
      }
      if (a.tb == 0) {
        const int kk = tid % 16, j = tid / 16 + 16 * q;
        Bs[kk][j] = (n0 + j < a.N && k0 + kk < ke) ? rb[q] : 0.0;
      } else {
        const int j = tid % 128, kk = tid / 128 + 2 * q;
        Bs[kk][j] = (n0 + j < a.N && k0 + kk < ke) ? rb[q] : 0.0;
      }
    }
    __syncthreads();
    if (k0 + 16 < ke) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double af[4], bf[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = As[4 * ks + g][wr + 16 * x + li];
#pragma unroll
      for (int y = 0; y < 4; ++y) bf[y] = Bs[4 * ks + g][wc + 16 * y + li];
      // operands fed swapped (the product comes out transposed): a lane's
      // four results are then four columns of C at one row, and the 16 lanes
      // of a lane group hold 16 consecutive rows -- 128-byte segments of the
      // column-major output instead of 32-byte ones
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[y], af[x], acc[x][y], 0, 0, 0);
    }
  }
  // acc[x][y][r] = product(m0 + wr + 16x + li, n0 + wc + 16y + g + 4r)
  const int64_t ib = m0 + wr + li;
  if (gridDim.z > 1) {
    double* Pz = P + (int64_t)blockIdx.z * a.M * a.N;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = ib + 16 * x, j = n0 + wc + 16 * y + g + 4 * r;
          if (i < a.M && j < a.N) Pz[j * a.M + i] = acc[x][y][r];
        }
    return;
  }
  // per group y: every Cin / Ein load of its 16 outputs issued before any of
  // them is used (one memory round trip per group, not one per output row)
  const bool hasc = a.beta != 0.0, hase = a.E && a.Ein;
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    double cin[4][4], ein[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jl = wc + 16 * y + g + 4 * r;
      const int64_t ij = smap[1][jl], ej = smap[2][jl];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t i = ib + 16 * x;
        const int64_t icl = i < a.M ? i : a.M - 1;
        cin[r][x] = hasc ? (double)a.Cin[ij * a.ldcin + icl] : 0.0;
        ein[r][x] = hase ? a.Ein[ej * a.ldein + icl] : 0.0;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jl = wc + 16 * y + g + 4 * r;
      const int64_t j = n0 + jl;
      if (j >= a.N) continue;
      const int64_t cj = smap[0][jl];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t i = ib + 16 * x;
        if (i >= a.M) continue;
        double v = a.alpha * acc[x][y][r];
        if (hasc) v += a.beta * cin[r][x];
        a.C[cj * a.ldc + i] = v;
        if (a.E) a.E[j * a.lde + i] = ein[r][x] - v;
      }
    }
  }
}

// Split-K epilogue: C(i, cmap[j]) = alpha sum_z P_z(i, j) + beta Cin(i, cinmap[j]),
// the partials summed in z order.
template <typename TA, typename TC>
__global__ __launch_bounds__(kThreads) void k_gemm64_reduce(G64Args<TA, TC> a, int nz,
                                                            const double* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= a.M) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += P[((int64_t)z * a.N + j) * a.M + i];
  double v = a.alpha * s;
  if (a.beta != 0.0) v += a.beta * (double)a.Cin[(a.cinmap ? (int64_t)a.cinmap[j] : j) * a.ldcin + i];
  a.C[(a.cmap ? (int64_t)a.cmap[j] : j) * a.ldc + i] = v;
}

// Split-K plan of the large-tile product: with few output tiles and a long
// contraction the K range is split so that the grid has about two blocks per
// compute unit; P must then hold nz M N doubles.
static int gemm_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(M, 128) * ceil_div(N, 128);
  int nz = 1;
  while (nz < 16 && tiles * nz * 2 <= 512 && K / (nz * 2) >= 128) nz *= 2;
  return nz;
}

size_t gemm64_split_workspace(int64_t M, int64_t N, int64_t K) {
  const int nz = gemm_splits(M, N, K);
  return nz > 1 ? (size_t)nz * M * N * 8 : 0;
}

template <typename TA, typename TC>
static int gemm_launch(const G64Args<TA, TC>& a, hipStream_t s, double* P = nullptr,
                       size_t p_bytes = 0) {
  if (a.M <= 0 || a.N <= 0) return ID_OK;
  // small products take the 64 x 64 tile (which has no second output)
  if (!a.E && (a.M < 128 || a.N < 64 || a.K < 16)) {
    k_gemm64<TA, TC><<<dim3((unsigned)ceil_div(a.M, 64), (unsigned)ceil_div(a.N, 64)), kThreads,
                       0, s>>>(a);
    MPID_LAUNCH_CHECK();
    return ID_OK;
  }
  int nz = gemm_splits(a.M, a.N, a.K);
  if (nz > 1 && (a.E || !P || p_bytes < (size_t)nz * a.M * a.N * 8)) nz = 1;
  const int64_t kc = round_up(ceil_div(a.K, nz), 16);
  const unsigned ny = (unsigned)ceil_div(a.N, 128);
  k_gemm64t<TA, TC><<<dim3((unsigned)ceil_div(a.M, 128), ny, (unsigned)nz), kThreads, 0, s>>>(
      a, a, ny, kc, P);
  MPID_LAUNCH_CHECK();
  if (nz > 1) {
    k_gemm64_reduce<TA, TC><<<dim3((unsigned)ceil_div(a.M, kThreads), (unsigned)a.N), kThreads, 0,
                              s>>>(a, nz, P);
    MPID_LAUNCH_CHECK();
  }
  return ID_OK;
}

// Two large-tile products with the same M and K (and A operand layout) in one
// launch: one grid, so the blocks of both fill the chip together.
template <typename TA, typename TC>
static int gemm_launch2(const G64Args<TA, TC>& a0, const G64Args<TA, TC>& a1, hipStream_t s) {
  if (a0.M != a1.M || a0.K != a1.K) return ID_ERR_ARG;
  if (a0.M <= 0 || (a0.N <= 0 && a1.N <= 0)) return ID_OK;
  const unsigned ny0 = (unsigned)ceil_div(a0.N, 128), ny1 = (unsigned)ceil_div(a1.N, 128);
  k_gemm64t<TA, TC><<<dim3((unsigned)ceil_div(a0.M, 128), ny0 + ny1, 1), kThreads, 0, s>>>(
      a0, a1, ny0, round_up(a0.K, 16), nullptr);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

// C = A B with A (M x K) in its storage dtype (fp32 or fp64, column-major, lda)
// and B, C float64; b_upper: B is upper triangular (its zeros are skipped).
int gemm64_typed_run(const void* A, int32_t dtype, int64_t M, int64_t N, int64_t K, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, int b_upper,
                     hipStream_t s) {
  if (dtype == ID_F64) {
    G64Args<double, double> a;
    std::memset(&a, 0, sizeof(a));
    a.M = M, a.N = N, a.K = K, a.alpha = 1.0;
    a.A = (const double*)A, a.lda = lda, a.B = B, a.ldb = ldb;
    a.C = C, a.ldc = ldc, a.b_upper = b_upper;
    return gemm_launch(a, s);
  }
  G64Args<float, double> a;
  std::memset(&a, 0, sizeof(a));
  a.M = M, a.N = N, a.K = K, a.alpha = 1.0;
  a.A = (const float*)A, a.lda = lda, a.B = B, a.ldb = ldb;
  a.C = C, a.ldc = ldc, a.b_upper = b_upper;
  return gemm_launch(a, s);
}

int gemm64_run(int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
               int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
               hipStream_t s) {
  G64Args<double, double> a;
  std::memset(&a, 0, sizeof(a));
  a.ta = ta;
  a.tb = tb;
  a.M = M;
  a.N = N;
  a.K = K;
  a.alpha = alpha;
  a.A = A;
  a.lda = lda;
  a.B = B;
  a.ldb = ldb;
  a.beta = beta;
  a.Cin = C;
  a.ldcin = ldc;
  a.C = C;
  a.ldc = ldc;
  return gemm_launch(a, s);
}

// Y(:, cols[j]) = zero ? 0 : (double) A(:, cols[j]), j < ncols (cols may be null = identity);
// the destination column is dcols[j] (null = j).
template <typename TA>
__global__ __launch_bounds__(kThreads) void k_gather_cols(const TA* __restrict__ A, int64_t lda,
                                                          int64_t m, const int32_t* cols,
                                                          double* __restrict__ Y, int64_t ldy,
                                                          const int32_t* dcols, int zero) {
  const int64_t j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  const int64_t sc = cols ? (int64_t)cols[j] : j;
  const int64_t dc = dcols ? (int64_t)dcols[j] : j;
  Y[dc * ldy + i] = zero ? 0.0 : (double)A[sc * lda + i];
}

template <typename TA>
static int gather(const TA* A, int64_t lda, int64_t m, const int32_t* cols, int64_t ncols,
                  double* Y, int64_t ldy, const int32_t* dcols, int zero, hipStream_t s) {
  if (m <= 0 || ncols <= 0) return ID_OK;
  k_gather_cols<TA><<<dim3((unsigned)ceil_div(m, kThreads), (unsigned)ncols), kThreads, 0, s>>>(
      A, lda, m, cols, Y, ldy, dcols, zero);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

template <typename TA>
static int reconstruct_impl(const TA* A, int64_t m, int64_t n, int64_t lda, const int32_t* perm,
                            int64_t k, const double* T, int64_t ldt, double* Y, int64_t ldy,
                            int32_t residual, hipStream_t s) {
  int rc = gather<TA>(A, lda, m, perm, k, Y, ldy, perm, residual ? 1 : 0, s);
  if (rc) return rc;
  if (n - k <= 0) return ID_OK;
  G64Args<TA, TA> a;
  std::memset(&a, 0, sizeof(a));
  a.ta = 0;
  a.tb = 0;
  a.M = m;
  a.N = n - k;
  a.K = k;
  a.alpha = residual ? -1.0 : 1.0;
  a.A = A;
  a.lda = lda;
  a.amap = perm;
  a.B = T;
  a.ldb = ldt;
  a.beta = residual ? 1.0 : 0.0;
  a.Cin = A;
  a.ldcin = lda;
  a.cinmap = perm + k;
  a.C = Y;
  a.ldc = ldy;
  a.cmap = perm + k;
  return gemm_launch(a, s);
}

int reconstruct_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const int32_t* perm, int64_t k, const double* T, int64_t ldt, double* Y,
                    int64_t ldy, int32_t residual, hipStream_t s) {
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (m < 0 || n < 0 || k < 0 || k > n) return ID_ERR_ARG;
  if (m == 0 || n == 0) return ID_OK;
  if (!A || !perm || !Y || lda < m || ldy < m) return ID_ERR_ARG;
  if (k > 0 && n - k > 0 && (!T || ldt < k)) return ID_ERR_ARG;
  if (dtype == ID_F64)
    return reconstruct_impl<double>((const double*)A, m, n, lda, perm, k, T, ldt, Y, ldy,
                                    residual, s);
  return reconstruct_impl<float>((const float*)A, m, n, lda, perm, k, T, ldt, Y, ldy, residual,
                                 s);
}

// ---------------------------------------------------------------- fused adjoint products

typedef double f64x4v __attribute__((ext_vector_type(4)));

// Padded copies of the coefficient blocks for the fused kernel: Xp / Tp are X
// and T (k x nc) with the leading dimension kq = k rounded up to 16 and rows
// k..kq-1 zero; Xq / Tq are their transposes (nc x k) with the leading
// dimension nq = nc rounded up to 16 and rows nc..nq-1 zero.  Every 32-byte
// group of four contraction entries a lane reads is then aligned and in range.
__global__ __launch_bounds__(kThreads) void k_adj_prep(const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ T, int64_t ldt,
                                                       int64_t k, int64_t nc, int64_t kq,
                                                       int64_t nq, double* __restrict__ Xp,
                                                       double* __restrict__ Tp,
                                                       double* __restrict__ Xq,
                                                       double* __restrict__ Tq) {
  __shared__ double tx[32][33], tt[32][33];
  const int lx = threadIdx.x % 32, ly = threadIdx.x / 32;  // 32 x 8
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;  // r: k, c: nc
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t r = r0 + lx, c = c0 + ly + 8 * q;
    const bool in = r < k && c < nc;
    const double x = in ? X[c * ldx + r] : 0.0, t = in ? T[c * ldt + r] : 0.0;
    if (r < kq && c < nc) {
      Xp[c * kq + r] = x;
      Tp[c * kq + r] = t;
    }
    tx[ly + 8 * q][lx] = x;
    tt[ly + 8 * q][lx] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t c = c0 + lx, r = r0 + ly + 8 * q;  // Xq(c, r) = X(r, c)
    if (r < k && c < nq) {
      Xq[r * nq + c] = tx[lx][ly + 8 * q];
      Tq[r * nq + c] = tt[lx][ly + 8 * q];
    }
  }
}

template <typename TA>
struct AdjArgs {
  int64_t m, k, nc, kq, nq;
  const double* Bm;  // B = A(:, J), m x k, ld m
  const double* Xp;  // X, kq x nc (rows past k zero)
  const double* Tp;  // T, kq x nc
  const double* Xq;  // X^T, nq x k (rows past nc zero)
  const double* Tq;  // T^T, nq x k
  const TA* A;
  int64_t lda;
  const double* gY;  // may be null
  int64_t ldgy;
  const int32_t* perm;  // J = perm[0:k], Jc = perm[k:n]
  double* gA;
  int64_t ldga;
};

constexpr int kAdjChunk = 128;  // coefficient columns per pass
constexpr int kAdjKMax = 256;   // largest k the fused kernel takes

// The adjoint's products for a strip of 16 RB rows i, without D and E in
// memory.  For each chunk of 128 columns j of the n - k coefficient columns:
//   phase 1: P_X = B(i, :) X(:, j), P_T = B(i, :) T(:, j)        (K = k)
//            gA(i, Jc[j]) = P_X,  E = gY(i, Jc[j]) - P_X,  D = A(i, Jc[j]) - P_T
//            (E and D go to LDS)
//   phase 2: acc(i, c) += sum_j D(i, j) X(c, j) + E(i, j) T(c, j)   (K = 2 x 128)
// and finally gA(i, J[c]) = gY(i, J[c]) + acc(i, c).  Wave w of the NW owns
// columns [CPW w, CPW (w + 1)) of each chunk in phase 1 (CPW = 128 / NW) and
// 4 NB2 / NW blocks of 16 columns c of k in phase 2 (4 NB2 16 >= k), for all
// RB row blocks of the strip.
// Operand lanes: a lane supplies A(row li, kk) and B(kk, col li) and receives
// C(row li, col g + 4 r) (operands fed swapped, as in k_gemm64t).  The
// contraction runs in groups of 16 in which lane group g takes the four
// consecutive entries 4 g .. 4 g + 3, so a lane reads each B operand as one
// aligned 32-byte load per group (from the padded copies, L2-resident), two
// or four groups ahead of their products, and feeds it to the RB row blocks' products
// (the strip height sets how much matrix-core work each operand byte carries:
// the products are bound by these operand reads); the A operands come from
// LDS in the same order.  Columns past nc or k read clamped in-range columns
// and are never stored; rows past m are zero in LDS and not stored.
template <typename TA, int NB2, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_adj_fused(AdjArgs<TA> a) {
  constexpr int NT = 64 * NW;                   // threads (NW waves)
  constexpr int KB = 64 * NB2;                  // largest k of this instantiation
  constexpr int RS = 16 * RB;                   // rows of the strip
  constexpr int CPW = kAdjChunk / NW;           // chunk columns per wave in phase 1
  constexpr int NB1 = CPW / 16;                 // ... as 16-column blocks
  constexpr int NBK = 4 * NB2 / NW;             // 16-column blocks of k per wave in phase 2
  static_assert(NB1 >= 1 && NBK >= 1 && NBK * NW == 4 * NB2, "wave split");
  // operand groups in flight: four for a block that is the only one on its
  // compute unit with one wave per SIMD (32-row strips, four waves), two
  // when each SIMD has other waves to switch to
  constexpr int PD = (RB == 2 && NW == 4) ? 4 : 2;
  __shared__ double Bs[KB][RS];                 // Bs[kk][i] = B(i0 + i, kk)
  __shared__ double Es[kAdjChunk][RS];          // Es[j][i] = E(i0 + i, c0 + j)
  __shared__ double Ds[kAdjChunk][RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int64_t m = a.m, k = a.k, nc = a.nc;
  const int64_t i0 = (int64_t)blockIdx.x * RS;
  int64_t iw[RB], ic[RB];  // this lane's output rows (one per row block)
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    iw[rb] = i0 + 16 * rb + li;
    ic[rb] = iw[rb] < m ? iw[rb] : m - 1;
  }
  const int ng1 = (int)(a.kq / 16);  // contraction groups of phase 1
  // the strip of B (rows past m and columns past k zero)
  for (int e = tid; e < KB * RS; e += NT) {
    const int r = e % RS, kk = e / RS;
    const int64_t gi = i0 + r;
    Bs[kk][r] = (gi < m && kk < k) ? a.Bm[(int64_t)kk * m + gi] : 0.0;
  }
  f64x4 acc2[RB][NBK], acc3[RB][NBK];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int nb = 0; nb < NBK; ++nb) {
      acc2[rb][nb] = (f64x4){0.0, 0.0, 0.0, 0.0};
      acc3[rb][nb] = acc2[rb][nb];
    }
  for (int64_t c0 = 0; c0 < nc; c0 += kAdjChunk) {
    // the epilogue's inputs: rows i, columns Jc[j] for the lane's outputs
    // j = c0 + CPW w + 16 nb + g + 4 r (loaded ahead of the products)
    double ein[RB][NB1][4], cin[RB][NB1][4];
#pragma unroll
    for (int nb = 0; nb < NB1; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = c0 + CPW * wv + 16 * nb + g + 4 * r;
        const int64_t col = a.perm[k + (j < nc ? j : nc - 1)];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          ein[rb][nb][r] = a.gY ? a.gY[col * a.ldgy + ic[rb]] : 0.0;
          cin[rb][nb][r] = (double)a.A[col * a.lda + ic[rb]];
        }
      }
    __syncthreads();  // Bs ready (first pass); Es / Ds free (later passes)
    // ---- phase 1, one 16-column block nb at a time: the B operands are
    // columns j = c0 + CPW w + 16 nb + li of X and T
    f64x4 px[RB][NB1], pt[RB][NB1];
#pragma unroll
    for (int nb = 0; nb < NB1; ++nb) {
      const int64_t j = c0 + CPW * wv + 16 * nb + li;
      const int64_t jc = j < nc ? j : nc - 1;
      const double* xcol = a.Xp + jc * a.kq + 4 * g;
      const double* tcol = a.Tp + jc * a.kq + 4 * g;
      f64x4 ax[RB], at[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        ax[rb] = (f64x4){0.0, 0.0, 0.0, 0.0};
        at[rb] = ax[rb];
      }
      // PD groups of operand loads in flight, rotated through registers
      f64x4v xb[PD], tb[PD];
#pragma unroll
      for (int p = 0; p < PD; ++p) {
        const int qq = p < ng1 ? p : 0;
        xb[p] = *(const f64x4v*)(xcol + 16 * qq);
        tb[p] = *(const f64x4v*)(tcol + 16 * qq);
      }
      for (int q = 0; q < ng1; q += PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
          if (q + p < ng1) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int rb = 0; rb < RB; ++rb) {
                const double af = Bs[16 * (q + p) + 4 * g + s][16 * rb + li];
                ax[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[p][s], af, ax[rb], 0, 0, 0);
                at[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[p][s], af, at[rb], 0, 0, 0);
              }
            if (q + p + PD < ng1) {
              xb[p] = *(const f64x4v*)(xcol + 16 * (q + p + PD));
              tb[p] = *(const f64x4v*)(tcol + 16 * (q + p + PD));
            }
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        px[rb][nb] = ax[rb];
        pt[rb][nb] = at[rb];
      }
    }
    // ---- epilogue: gA(i, Jc[j]) = P_X; E and D to LDS (zero past nc / m)
#pragma unroll
    for (int nb = 0; nb < NB1; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jl = CPW * wv + 16 * nb + g + 4 * r;
        const int64_t j = c0 + jl;
        const int64_t col = j < nc ? (int64_t)a.perm[k + j] : 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const bool ok = j < nc && iw[rb] < m;
          const double w = px[rb][nb][r];
          if (ok) a.gA[col * a.ldga + iw[rb]] = w;
          Es[jl][16 * rb + li] = ok ? ein[rb][nb][r] - w : 0.0;
          Ds[jl][16 * rb + li] = ok ? cin[rb][nb][r] - pt[rb][nb][r] : 0.0;
        }
      }
    __syncthreads();
    // ---- phase 2, one 16-column block nb of k at a time: acc2 += D X(c, j)^T
    // and acc3 += E T(c, j)^T over the chunk's j (two independent chains per
    // row block), the B operands read from the transposed copies (j
    // consecutive)
    {
      const int64_t jn = nc - c0 < kAdjChunk ? nc - c0 : kAdjChunk;
      const int ng2 = (int)ceil_div(jn, (int64_t)16);
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb) {
        const int64_t c = (int64_t)16 * (NBK * wv + nb) + li;
        const int64_t cc = c < k ? c : k - 1;
        const double* xrow = a.Xq + cc * a.nq + c0 + 4 * g;
        const double* trow = a.Tq + cc * a.nq + c0 + 4 * g;
        f64x4 ax[RB], at[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          ax[rb] = acc2[rb][nb];
          at[rb] = acc3[rb][nb];
        }
        f64x4v xb[PD], tb[PD];
#pragma unroll
        for (int p = 0; p < PD; ++p) {
          const int qq = p < ng2 ? p : 0;
          xb[p] = *(const f64x4v*)(xrow + 16 * qq);
          tb[p] = *(const f64x4v*)(trow + 16 * qq);
        }
        for (int q = 0; q < ng2; q += PD) {
#pragma unroll
          for (int p = 0; p < PD; ++p) {
            if (q + p < ng2) {
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const int jl = 16 * (q + p) + 4 * g + s;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                  ax[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[p][s], Ds[jl][16 * rb + li],
                                                                ax[rb], 0, 0, 0);
                  at[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[p][s], Es[jl][16 * rb + li],
                                                                at[rb], 0, 0, 0);
                }
              }
              if (q + p + PD < ng2) {
                xb[p] = *(const f64x4v*)(xrow + 16 * (q + p + PD));
                tb[p] = *(const f64x4v*)(trow + 16 * (q + p + PD));
              }
            }
          }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          acc2[rb][nb] = ax[rb];
          acc3[rb][nb] = at[rb];
        }
      }
    }
  }
  // ---- gA(i, J[c]) = gY(i, J[c]) + acc2 + acc3
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (iw[rb] < m) {
#pragma unroll
      for (int nb = 0; nb < NBK; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t c = (int64_t)16 * (NBK * wv + nb) + g + 4 * r;
          if (c < k) {
            const int64_t col = a.perm[c];
            const double y = a.gY ? a.gY[col * a.ldgy + iw[rb]] : 0.0;
            a.gA[col * a.ldga + iw[rb]] = y + (acc2[rb][nb][r] + acc3[rb][nb][r]);
          }
        }
    }
  }
}

// ---------------------------------------------------------------- adjoint

// B^T gY(:, Jc) has few output tiles: its contraction is split for about this
// many blocks (fewer, longer chunks than a sketch of the whole input: less
// partial-sum traffic)
constexpr int kBwdSketchBlocks = 1024;

struct BwdPlan {
  size_t off_b, off_de, off_xt, off_tbar, off_rq, off_permq, off_info, off_fws, off_sk,
      off_p, off_pad;
  size_t fws_bytes, sk_bytes, p_bytes, bytes;
};

// A thread's pinned word and event for reading the singular-R check of
// id_backward without waiting for the whole stream (released when the thread
// ends).
struct BwdHostInfo {
  int32_t* p = nullptr;
  hipEvent_t ev = nullptr;
  BwdHostInfo() = default;
  BwdHostInfo(const BwdHostInfo&) = delete;
  BwdHostInfo& operator=(const BwdHostInfo&) = delete;
  ~BwdHostInfo() {
    if (p) (void)hipHostFree(p);
    if (ev) (void)hipEventDestroy(ev);
  }
};
static BwdHostInfo& bwd_host_info() {
  static thread_local BwdHostInfo h;
  return h;
}

static bool make_bwd_plan(int64_t m, int64_t n, int64_t k, BwdPlan* p) {
  if (m < 0 || n < 0 || k < 0 || k > n) return false;
  const int64_t mm = m > 0 ? m : 1, kk = k > 0 ? k : 1, cc = (n - k) > 0 ? (n - k) : 1;
  std::memset(p, 0, sizeof(*p));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  p->off_b = take((size_t)mm * kk * 8);       // B = A(:, J) in FP64
  p->off_de = take((size_t)mm * 2 * cc * 8);  // [D | E], m x 2(n-k)
  p->off_xt = take((size_t)kk * 2 * cc * 8);  // [X | T], k x 2(n-k)
  p->off_tbar = take((size_t)kk * cc * 8);
  p->off_rq = take((size_t)kk * kk * 8);
  p->off_permq = take((size_t)kk * 4);
  p->off_info = take(64);
  id_opts o;
  std::memset(&o, 0, sizeof(o));
  o.prec = ID_PREC_F64;
  o.k_fixed = kk;
  o.flags = ID_FLAG_NO_PIVOT;
  FactorPlan fp;
  if (!make_factor_plan(mm, kk, ID_F64, &o, &fp)) return false;
  p->fws_bytes = fp.bytes;
  p->off_fws = take(fp.bytes);
  // partials of B^T gY(:, Jc): k x (n-k) with a contraction over all m
  // rows, split over row chunks (few output tiles, long contraction)
  p->sk_bytes = sketch_workspace_target(kk, mm, cc, kBwdSketchBlocks);
  p->off_sk = take(p->sk_bytes);
  // split-K partials of the m x k product with the 2(n-k) contraction
  p->p_bytes = gemm64_split_workspace(mm, kk, 2 * cc);
  p->off_p = take(p->p_bytes > 0 ? p->p_bytes : 8);
  // the fused products' padded coefficient copies: X, T (k rounded up to 16
  // rows) and their transposes (n - k rounded up to 16 rows)
  p->off_pad = take((size_t)4 * round_up(kk, 16) * round_up(cc, 16) * 8);
  p->bytes = off;
  return true;
}

size_t backward_workspace(int64_t m, int64_t n, int64_t k) {
  BwdPlan p;
  return make_bwd_plan(m, n, k, &p) ? p.bytes : 0;
}

static int env_flag(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return (v && *v) ? std::atoi(v) : dflt;
}

// The products of the adjoint as separate launches (any k): W with E beside
// it and D in one launch of the large-tile kernel, then gA(:, J) over the
// 2 (n - k) contraction with split K.
template <typename TA>
static int products_unfused(const TA* A, int64_t m, int64_t k, int64_t nc, int64_t lda,
                            const int32_t* perm, const double* T, int64_t ldt, const double* gY,
                            int64_t ldgy, double* gA, int64_t ldga, const double* Bm, double* DE,
                            double* XT, double* P, size_t p_bytes, hipStream_t s) {
  int rc;
  const double* X = XT;
  if ((rc = gather<double>(T, ldt, k, nullptr, nc, XT + k * nc, k, nullptr, 0, s))) return rc;
  // gA(:, Jc) = W = B X with E = gY(:, Jc) - W beside it, and D = A(:, Jc) - B T:
  // two products with the operand B, one launch
  {
    G64Args<double, TA> w, d;
    std::memset(&w, 0, sizeof(w));
    w.M = m, w.N = nc, w.K = k, w.alpha = 1.0;
    w.A = Bm, w.lda = m, w.B = X, w.ldb = k;
    w.C = gA, w.ldc = ldga, w.cmap = perm + k;
    w.E = DE + m * nc, w.lde = m, w.Ein = gY, w.ldein = ldgy, w.einmap = perm + k;
    std::memset(&d, 0, sizeof(d));
    d.M = m, d.N = nc, d.K = k, d.alpha = -1.0, d.beta = 1.0;
    d.A = Bm, d.lda = m, d.B = XT + k * nc, d.ldb = k;
    d.Cin = A, d.ldcin = lda, d.cinmap = perm + k;
    d.C = DE, d.ldc = m;
    if ((rc = gemm_launch2(w, d, s))) return rc;
  }
  // gA(:, J) = gY(:, J) + [D | E] [X | T]^T
  {
    G64Args<double, double> a;
    std::memset(&a, 0, sizeof(a));
    a.tb = 1;
    a.M = m, a.N = k, a.K = 2 * nc, a.alpha = 1.0, a.beta = gY ? 1.0 : 0.0;
    a.A = DE, a.lda = m, a.B = XT, a.ldb = k;
    a.Cin = gY, a.ldcin = ldgy, a.cinmap = perm;
    a.C = gA, a.ldc = ldga, a.cmap = perm;
    if ((rc = gemm_launch(a, s, P, p_bytes))) return rc;
  }
  return ID_OK;
}

// With B = A(:, J), C = A(:, Jc), T = B^+ C and X = (B^T B)^{-1} Tbar,
// Tbar = gT + B^T gY(:, Jc):
//   gA(:, Jc) = W = B X
//   gA(:, J)  = gY(:, J) + (C - B T) X^T + (gY(:, Jc) - W) T^T
//             = gY(:, J) + [D | E] [X | T]^T,  D = C - B T, E = gY(:, Jc) - W.
// A and gY are read through column maps (no gathered copies but B); the two
// products with B share nothing but their operand, the last one is a single
// product over the 2 (n - k) contraction, split over K when its output has few
// tiles.  The singularity check of B's R factor is read at the end (one host
// synchronization per call).
template <typename TA>
static int backward_impl(const TA* A, int64_t m, int64_t n, int64_t lda, const int32_t* perm,
                         int64_t k, const double* T, int64_t ldt, const double* Rb, int64_t ldrb,
                         const double* gT, int64_t ldgt, const double* gY, int64_t ldgy,
                         double* gA, int64_t ldga, char* wb, const BwdPlan& p, int32_t* info,
                         hipStream_t s) {
  const int64_t nc = n - k;
  double* Bm = (double*)(wb + p.off_b);
  double* DE = (double*)(wb + p.off_de);
  double* XT = (double*)(wb + p.off_xt);
  double* Tb = (double*)(wb + p.off_tbar);
  double* Rq = (double*)(wb + p.off_rq);
  int32_t* permq = (int32_t*)(wb + p.off_permq);
  int32_t* dinfo = (int32_t*)(wb + p.off_info);
  int rc;
  *info = 0;
  // gA = 0 when there is no skeleton
  if (k == 0) return gather<double>(nullptr, 1, m, nullptr, n, gA, ldga, nullptr, 1, s);
  if (nc == 0) {  // the skeleton is every column: Y = A, gA = gY
    rc = gY ? gather<double>(gY, ldgy, m, perm, k, gA, ldga, perm, 0, s)
            : gather<double>(nullptr, 1, m, nullptr, k, gA, ldga, perm, 1, s);
    return rc;
  }
  if ((rc = gather<TA>(A, lda, m, perm, k, Bm, m, nullptr, 0, s))) return rc;
  // R factor of B: the caller's (any R with R^T R = B^T B, e.g. R11 of the
  // FP64 factorization that chose J), else an unpivoted FP64 Householder QR
  const double* Rf = Rb;
  int64_t ldrf = ldrb;
  if (!Rf) {
    id_opts o;
    std::memset(&o, 0, sizeof(o));
    o.prec = ID_PREC_F64;
    o.k_fixed = k;
    o.flags = ID_FLAG_NO_PIVOT;
    int64_t kq = 0;
    int32_t iq = 0;
    rc = factor_run(Bm, ID_F64, m, k, m, &o, wb + p.off_fws, p.fws_bytes, permq, Rq, k, &kq, &iq,
                    s);
    if (rc) return rc;
    if (iq != 0 || kq != k) {
      *info = ID_INFO_SINGULAR;
      return ID_OK;
    }
    Rf = Rq;
    ldrf = k;
  }
  // the diagonal check of Rf, copied to pinned host memory; the products
  // that do not need it (Tbar = gT + B^T gY(:, Jc)) are enqueued before the
  // host waits for that copy, so the GPU is busy with them meanwhile; the
  // rest is enqueued only for a nonsingular R, and the call then returns with
  // it in flight (no wait at its end)
  if ((rc = solve_T_run(Rf, ldrf, k, k, nullptr, 1, dinfo, s))) return rc;
  BwdHostInfo& hi = bwd_host_info();
  if (!hi.p) MPID_HIP(hipHostMalloc((void**)&hi.p, sizeof(int32_t), hipHostMallocDefault));
  if (!hi.ev) MPID_HIP(hipEventCreateWithFlags(&hi.ev, hipEventDisableTiming));
  MPID_HIP(hipMemcpyAsync(hi.p, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPID_HIP(hipEventRecord(hi.ev, s));
  if (gT) {
    if ((rc = gather<double>(gT, ldgt, k, nullptr, nc, Tb, k, nullptr, 0, s))) return rc;
  } else {
    if ((rc = gather<double>(nullptr, 1, k, nullptr, nc, Tb, k, nullptr, 1, s))) return rc;
  }
  if (gY) {
    // Tbar += B^T gY(:, Jc), added by the product's reduction (B^T as a
    // row-major k x m matrix is B's column-major storage)
    if ((rc = sketch_run_cols(gY, ID_F64, m, nc, ldgy, perm + k, Bm, k, m, Tb, k, wb + p.off_sk,
                              p.sk_bytes, kBwdSketchBlocks, s, 1)))
      return rc;
  }
  MPID_HIP(hipEventSynchronize(hi.ev));
  if (*hi.p == ID_INFO_SINGULAR) {
    *info = ID_INFO_SINGULAR;  // gA is left undefined
    return ID_OK;
  }
  // X = (B^T B)^{-1} Tbar = R^{-1} R^{-T} Tbar into the left half of [X | T]
  double* X = XT;
  if ((rc = trsm_normal_run(Rf, ldrf, k, Tb, k, nc, X, k, s))) return rc;
  double* pad = (double*)(wb + p.off_pad);
  // (the fused kernel reads the padded copies in aligned 32-byte groups)
  if (k <= kAdjKMax && (uintptr_t)pad % 32 == 0 && env_flag("MPID_ADJ_FUSED", 1)) {
    // all three products in one pass over 16-row strips (D and E stay in LDS)
    const int64_t kq = round_up(k, 16), nq = round_up(nc, 16);
    double *Xp = pad, *Tp = pad + kq * nq, *Xq = pad + 2 * kq * nq, *Tq = pad + 3 * kq * nq;
    k_adj_prep<<<dim3((unsigned)ceil_div(kq, 32), (unsigned)ceil_div(nq, 32)), kThreads, 0, s>>>(
        X, k, T, ldt, k, nc, kq, nq, Xp, Tp, Xq, Tq);
    MPID_LAUNCH_CHECK();
    AdjArgs<TA> fa;
    fa.m = m, fa.k = k, fa.nc = nc, fa.kq = kq, fa.nq = nq;
    fa.Bm = Bm, fa.Xp = Xp, fa.Tp = Tp, fa.Xq = Xq, fa.Tq = Tq;
    fa.A = A, fa.lda = lda, fa.gY = gY, fa.ldgy = ldgy, fa.perm = perm;
    fa.gA = gA, fa.ldga = ldga;
    // strips of 32 rows while they still give every compute unit a block
    // (twice the matrix-core work per operand read), else of 16
    int dev = 0, cus = 0;
    MPID_HIP(hipGetDevice(&dev));
    MPID_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int rb = env_flag("MPID_ADJ_RB2", 1) && ceil_div(m, (int64_t)32) >= (cus > 0 ? cus : 256)
                       ? 2 : 1;
    // the 32-row strips' LDS leaves one block per compute unit: eight waves
    // per block then give each SIMD two to switch between
    const int nw = env_flag("MPID_ADJ_WAVES", 8) == 4 ? 4 : 8;
    const dim3 fg((unsigned)ceil_div(m, (int64_t)16 * rb));
    if (k <= 128) {
      if (rb == 2 && nw == 8)
        k_adj_fused<TA, 2, 2, 8><<<fg, 512, 0, s>>>(fa);
      else if (rb == 2)
        k_adj_fused<TA, 2, 2, 4><<<fg, 256, 0, s>>>(fa);
      else
        k_adj_fused<TA, 2, 1, 4><<<fg, 256, 0, s>>>(fa);
    } else {
      if (rb == 2 && nw == 8)
        k_adj_fused<TA, 4, 2, 8><<<fg, 512, 0, s>>>(fa);
      else if (rb == 2)
        k_adj_fused<TA, 4, 2, 4><<<fg, 256, 0, s>>>(fa);
      else
        k_adj_fused<TA, 4, 1, 4><<<fg, 256, 0, s>>>(fa);
    }
    MPID_LAUNCH_CHECK();
  } else {
    if ((rc = products_unfused<TA>(A, m, k, nc, lda, perm, T, ldt, gY, ldgy, gA, ldga, Bm, DE, XT,
                                   (double*)(wb + p.off_p), p.p_bytes, s)))
      return rc;
  }
  return ID_OK;
}


int backward_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                 const int32_t* perm, int64_t k, const double* T, int64_t ldt, const double* Rb,
                 int64_t ldrb, const double* gT, int64_t ldgt, const double* gY, int64_t ldgy,
                 double* gA, int64_t ldga, void* work, size_t work_bytes, int32_t* info,
                 hipStream_t s) {
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (!info || m < 0 || n < 0 || k < 0 || k > n) return ID_ERR_ARG;
  *info = 0;
  if (m == 0 || n == 0) return ID_OK;
  if (!A || !perm || !gA || lda < m || ldga < m) return ID_ERR_ARG;
  if (k > 0 && n - k > 0 && (!T || ldt < k)) return ID_ERR_ARG;
  if (gT && ldgt < (k > 0 ? k : 1)) return ID_ERR_ARG;
  if (gY && ldgy < m) return ID_ERR_ARG;
  if (Rb && ldrb < (k > 0 ? k : 1)) return ID_ERR_ARG;
  BwdPlan p;
  if (!make_bwd_plan(m, n, k, &p)) return ID_ERR_ARG;
  if (!work || work_bytes < p.bytes) return ID_ERR_WORKSPACE;
  if (dtype == ID_F64)
    return backward_impl<double>((const double*)A, m, n, lda, perm, k, T, ldt, Rb, ldrb, gT, ldgt,
                                 gY, ldgy, gA, ldga, (char*)work, p, info, s);
  return backward_impl<float>((const float*)A, m, n, lda, perm, k, T, ldt, Rb, ldrb, gT, ldgt, gY,
                              ldgy, gA, ldga, (char*)work, p, info, s);
}

}  // namespace mpid
