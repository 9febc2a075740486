// Sketching front end: Y = Omega A on the FP64 matrix cores.
//
// Section 5 names sketching as a way to make the ID cheaper; the randomized
// column ID compresses every column of A (m x n) to l << m entries with a
// random test matrix Omega (l x m, drawn by the caller), Y = Omega A, and runs
// the column-pivoted factorization on Y instead of A (the skeleton and T of
// Y are those of the randomized ID of A).  This file forms Y; the
// factorization of Y is the ordinary id_factor on an l x n FP64 matrix.
//
// Y is a product with a long contraction (m) and a small output (l x n), so
// the contraction is split over row chunks: every block forms one 64 x 64
// output tile over one chunk of rows into a partial buffer, and a second
// kernel sums the chunks in a fixed order (deterministic results).  Omega is
// row-major (each of its rows runs along the rows of A), so both operands are
// read along the contraction with the same coalesced pattern.  Blocks are
// remapped so that the tiles of one row chunk run on the same XCD: they share
// that chunk's rows of A and of Omega through the XCD's L2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "mpid_internal.h"

namespace mpid {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kSK = 16;  // rows of the contraction staged per round
constexpr int kOR = kSK * 64 / kThreads;  // contraction rows per thread per operand and round
constexpr int kTH = kSK / kOR;            // threads per tile row / column

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return (v && *v) ? std::atoi(v) : dflt;
}

struct SketchPlan {
  int64_t ntl, ntn, ntiles, S, chunk;
  size_t bytes;
};

bool make_sketch_plan(int64_t l, int64_t m, int64_t n, SketchPlan* p, int target = 0) {
  if (l < 0 || m < 0 || n < 0 || l > ((int64_t)1 << 20) || n > ((int64_t)1 << 30)) return false;
  std::memset(p, 0, sizeof(*p));
  const int64_t mm = m > 0 ? m : 1;
  p->ntl = ceil_div(l > 0 ? l : 1, 64);
  p->ntn = ceil_div(n > 0 ? n : 1, 64);
  p->ntiles = p->ntl * p->ntn;
  // many short chunks: ~16 resident blocks per CU and a short tail
  int64_t S = ceil_div(target > 0 ? target : env_int("MPID_SKETCH_BLOCKS", 4096), p->ntiles);
  const int64_t smax = ceil_div(mm, 8 * kSK);
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  p->chunk = round_up(ceil_div(mm, S), kSK);
  p->S = ceil_div(mm, p->chunk);
  p->bytes = (size_t)p->S * p->ntiles * 64 * 64 * 8;
  return true;
}

template <typename T>
struct Vec2x;  // 16-byte vector of T
template <>
struct Vec2x<float> {
  typedef float4 type;
  static constexpr int n = 4;
};
template <>
struct Vec2x<double> {
  typedef double2 type;
  static constexpr int n = 2;
};

// Partial tile (I, J) over rows [s chunk, (s+1) chunk):
// P[s][I ntn + J](x, y) = sum_i Omega(64 I + x, i) A(i, 64 J + y).
// Four waves, each a 32 x 32 quarter as 2 x 2 FP64 16x16x4 blocks; kSK rows
// of both operands staged in LDS per round, the next two rounds' loads in
// flight in registers.  VEC: every row of Omega and column of A starts on a
// 16-byte boundary, so full rounds use 16-byte loads (the scalar, bounds-
// checked form serves the last round of a chunk and unaligned operands).
// Four waves per SIMD: the register budget keeps 16 blocks resident per CU.
template <typename TA, bool VEC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void
k_sketch_partial(const double* __restrict__ Om, int64_t ldo, const TA* __restrict__ A, int64_t lda,
                 const int32_t* __restrict__ acols, int64_t l, int64_t m, int64_t n, int64_t ntn,
                 int64_t ntiles, int64_t S, int64_t chunk, double* __restrict__ P) {
  __shared__ double Os[kSK][64 + 1];  // Os[kk][x] = Omega(i0 + x, r0 + kk)
  __shared__ double As[kSK][64 + 1];  // As[kk][y] = A(r0 + kk, j0 + y)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  // XCD-aware order: hardware block b runs on XCD b % 8; logical blocks
  // x per .. (x + 1) per - 1 go to XCD x, chunk-major
  const int64_t total = S * ntiles;
  const int64_t per = gridDim.x / 8;
  const int64_t v = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (v >= total) return;
  const int64_t s = v / ntiles, tile = v % ntiles;
  const int64_t I = tile / ntn, J = tile % ntn;
  const int64_t i0 = I * 64, j0 = J * 64;
  const int64_t r0 = s * chunk;
  const int64_t r1 = r0 + chunk < m ? r0 + chunk : m;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;
  // load mapping: tile row / column c = tid / kTH, contraction rows
  // kOR (tid % kTH) .. + kOR - 1 of both operands
  const int lc = tid / kTH, lr = (tid % kTH) * kOR;
  const bool okO = i0 + lc < l, okA = j0 + lc < n;
  const double* orow = Om + (okO ? (i0 + lc) * ldo : 0) + lr;
  // column j of A is A(:, acols[j]) when a column map is given
  const int64_t ac = okA ? (acols ? (int64_t)acols[j0 + lc] : j0 + lc) : 0;
  const TA* acol = A + ac * lda + lr;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (f64x4){0.0, 0.0, 0.0, 0.0};
  double ro[2][kOR];
  TA ra[2][kOR];
  auto load = [&](int q, int64_t k0) {
    if (VEC && k0 + kSK <= r1) {
      typedef typename Vec2x<TA>::type VT;
      constexpr int NA = Vec2x<TA>::n;
#pragma unroll
      for (int e = 0; e < kOR; e += 2) {
        const double2 t = okO ? *(const double2*)(orow + k0 + e) : make_double2(0.0, 0.0);
        ro[q][e] = t.x;
        ro[q][e + 1] = t.y;
      }
#pragma unroll
      for (int e = 0; e < kOR; e += NA) {
        VT t;
        if (okA) {
          t = *(const VT*)(acol + k0 + e);
        } else {
#pragma unroll
          for (int c = 0; c < NA; ++c) t[c] = (TA)0;
        }
#pragma unroll
        for (int c = 0; c < NA; ++c) ra[q][e + c] = t[c];
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < kOR; ++e) {
      const bool in = k0 + lr + e < r1;
      ro[q][e] = (okO && in) ? orow[k0 + e] : 0.0;
      ra[q][e] = (okA && in) ? acol[k0 + e] : (TA)0;
    }
  };
  auto stage = [&](int q) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kOR; ++e) {
      Os[lr + e][lc] = ro[q][e];
      As[lr + e][lc] = (double)ra[q][e];
    }
    __syncthreads();
  };
  auto products = [&]() {
#pragma unroll
    for (int kk = 0; kk < kSK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = Os[kk + g][wr + 16 * x + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = As[kk + g][wc + 16 * y + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  };
  load(0, r0);
  load(1, r0 + kSK);
  for (int64_t k0 = r0; k0 < r1; k0 += 2 * kSK) {
    stage(0);
    if (k0 + 2 * kSK < r1) load(0, k0 + 2 * kSK);
    products();
    if (k0 + kSK >= r1) break;
    stage(1);
    if (k0 + 3 * kSK < r1) load(1, k0 + 3 * kSK);
    products();
  }
  // acc[x][y][r] = tile(wr + 16 x + g + 4 r, wc + 16 y + li); row-major tile
  double* out = P + (s * ntiles + tile) * (64 * 64);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(wr + 16 * x + g + 4 * r) * 64 + wc + 16 * y + li] = acc[x][y][r];
}

// Y(x, y) = sum over the row chunks of the partial tiles, in chunk order.
__global__ __launch_bounds__(kThreads) void k_sketch_reduce(const double* __restrict__ P,
                                                          int64_t S, int64_t ntiles, int64_t ntn,
                                                          int64_t l, int64_t n,
                                                          double* __restrict__ Y, int64_t ldy,
                                                          int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= ntiles * 4096) return;
  const int64_t tile = e / 4096, w = e % 4096;
  const int64_t x = (tile / ntn) * 64 + w / 64, y = (tile % ntn) * 64 + w % 64;
  if (x >= l || y >= n) return;
  double v = 0.0;
  for (int64_t s = 0; s < S; ++s) v += P[(s * ntiles + tile) * 4096 + w];
  double* out = Y + y * ldy + x;
  *out = accumulate ? *out + v : v;
}

template <typename TA>
int sketch_impl(const TA* A, int64_t m, int64_t n, int64_t lda, const int32_t* acols,
                const double* Om, int64_t l, int64_t ldo, double* Y, int64_t ldy,
                const SketchPlan& p, double* P, hipStream_t s, int accumulate) {
  const dim3 grid((unsigned)round_up(p.S * p.ntiles, 8));
  // 16-byte loads need 16-byte aligned rows of Omega and columns of A
  const bool vec = ((uintptr_t)Om % 16 == 0) && (ldo % 2 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((lda * (int64_t)sizeof(TA)) % 16 == 0);
  if (vec)
    k_sketch_partial<TA, true><<<grid, kThreads, 0, s>>>(Om, ldo, A, lda, acols, l, m, n, p.ntn,
                                                         p.ntiles, p.S, p.chunk, P);
  else
    k_sketch_partial<TA, false><<<grid, kThreads, 0, s>>>(Om, ldo, A, lda, acols, l, m, n,
                                                          p.ntn, p.ntiles, p.S, p.chunk, P);
  MPID_LAUNCH_CHECK();
  k_sketch_reduce<<<dim3((unsigned)ceil_div(p.ntiles * 4096, kThreads)), kThreads, 0, s>>>(
      P, p.S, p.ntiles, p.ntn, l, n, Y, ldy, accumulate);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

}  // namespace

size_t sketch_workspace(int64_t l, int64_t m, int64_t n) {
  SketchPlan p;
  if (!make_sketch_plan(l, m, n, &p)) return 0;
  return p.bytes;
}

int sketch_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda, const double* Om,
               int64_t l, int64_t ldo, double* Y, int64_t ldy, void* work, size_t work_bytes,
               hipStream_t s) {
  return sketch_run_cols(A, dtype, m, n, lda, nullptr, Om, l, ldo, Y, ldy, work, work_bytes, 0,
                         s);
}

size_t sketch_workspace_target(int64_t l, int64_t m, int64_t n, int target_blocks) {
  SketchPlan p;
  if (!make_sketch_plan(l, m, n, &p, target_blocks)) return 0;
  return p.bytes;
}

int sketch_run_cols(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const int32_t* acols, const double* Om, int64_t l, int64_t ldo, double* Y,
                    int64_t ldy, void* work, size_t work_bytes, int target_blocks, hipStream_t s,
                    int accumulate) {
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  SketchPlan p;
  if (!make_sketch_plan(l, m, n, &p, target_blocks)) return ID_ERR_ARG;
  if (l == 0 || n == 0) return ID_OK;
  if (!Y || ldy < l) return ID_ERR_ARG;
  if (m > 0 && (!A || !Om || lda < m || ldo < m)) return ID_ERR_ARG;
  if (!work || work_bytes < p.bytes) return ID_ERR_WORKSPACE;
  double* P = (double*)work;
  if (dtype == ID_F64)
    return sketch_impl<double>((const double*)A, m, n, lda, acols, Om, l, ldo, Y, ldy, p, P, s,
                               accumulate);
  return sketch_impl<float>((const float*)A, m, n, lda, acols, Om, l, ldo, Y, ldy, p, P, s,
                            accumulate);
}

}  // namespace mpid
