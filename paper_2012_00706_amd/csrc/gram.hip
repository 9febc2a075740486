// Tall-skinny front end: the same column-pivoted factorization reached through
// the FP64 Gram matrix G = A^T A instead of sweeps over A.
//
// For A Z = Q R (Section 1.1, eq. (6)-(7)) one has Z^T G Z = R^T R, and the
// residual norm of column l after j pivot steps is the l-th diagonal entry of
// the Schur complement of G, d_l = G_ll - sum_{i<j} R_il^2.  Greedy pivoting on
// d (largest first, ties to the first in swap order) is therefore column
// pivoting on A, and row j of R is R_jl = (G_pl - sum_{i<j} R_ip R_il) / R_jj
// with R_jj = sqrt(d_p): a pivoted Cholesky factorization of G.  Only the Gram
// product (FP64 matrix cores, split over row chunks) touches A; the k pivot
// steps then work on n x n data.  Rounding: d is formed to about u_64 ||A||^2, so residual
// norms below ~sqrt(u_64) ||A|| are not resolved and T = R11^{-1} R12 carries
// about kappa(R11)^2 u_64 relative error (kappa(R11) u_64 for the Householder
// path).  Two guards keep the route inside its resolution: adaptive
// tolerances below kGramMinTol are refused (ID_ERR_UNSUPPORTED), and the
// factorization stops, with ID_INFO_GRAM_LIMIT, before any step whose pivot
// has d_p <= kGramFloor n u_64 |R_00|^2 (|R_00|^2 = max_l G_ll): below that the
// Schur diagonal is rounding noise, so neither the pivot nor row j of R would
// mean anything.  This holds for a fixed rank too.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "device_util.h"
#include "mpid_internal.h"

namespace mpid {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kGK64 = 16;     // rows of A staged per round
constexpr int kPC = 16;       // columns per block of a pivot step (16 threads each)
constexpr int kPcR = 16;      // entries of a column of R per thread held in registers
constexpr int kGramBlocks = 4096;  // target blocks of the Gram product (16 resident per CU)
constexpr int kGR = kGK64 * 64 / kThreads;  // rows per thread per round, 64 x 64 tiles
constexpr int kGTH = kGK64 / kGR;           // threads per tile column
constexpr double kGramMinTol = 1e-6;        // smallest adaptive tolerance accepted
constexpr double kGramFloor = 8.0;          // resolution floor of d, in units of n u_64 |R_00|^2

struct GramState {
  int32_t done, info;
  int32_t limit;  // stopped at the resolution floor (ID_INFO_GRAM_LIMIT)
  int32_t pad1;
  int64_t k;
  double r00, fro2;
};

}  // namespace

struct GramPlan {
  int64_t m, n, kcap, gt, nt, ntiles, S, chunk, nblk;
  size_t off_g, off_part, off_rc, off_d, off_pv, off_pos0, off_pos1, off_am0, off_am1, off_state,
      bytes;
};

static bool make_gram_plan(int64_t m, int64_t n, int32_t dtype, const id_opts* o, GramPlan* p) {
  if (!o || !p || m < 0 || n < 0) return false;
  if (dtype != ID_F32 && dtype != ID_F64) return false;
  if (o->rank_rule != ID_RANK_PIVOT_REL && o->rank_rule != ID_RANK_FROB_REL) return false;
  if (o->k_fixed < 0 || o->k_max < 0 || !(o->rel_tol >= 0.0)) return false;
  if (n > 65536 || m > ((int64_t)1 << 34)) return false;
  std::memset(p, 0, sizeof(*p));
  int64_t kcap = m < n ? m : n;
  if (o->k_max > 0 && o->k_max < kcap) kcap = o->k_max;
  if (o->k_fixed > 0 && o->k_fixed < kcap) kcap = o->k_fixed;
  p->m = m;
  p->n = n;
  p->kcap = kcap;
  const int64_t nn = n > 0 ? n : 1, kk = kcap > 0 ? kcap : 1;
  p->gt = 64;
  const int64_t gk = kGK64;
  p->nt = ceil_div(nn, p->gt);
  p->ntiles = p->nt * (p->nt + 1) / 2;
  // split the rows so that the product has enough blocks
  int64_t S = ceil_div(kGramBlocks, p->ntiles);
  const int64_t smax = ceil_div(m > 0 ? m : 1, 8 * gk);
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  p->chunk = round_up(ceil_div(m > 0 ? m : 1, S), gk);
  p->S = ceil_div(m > 0 ? m : 1, p->chunk);
  p->nblk = ceil_div(nn, kPC);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t at = off;
    off += (b + 255) / 256 * 256;
    return at;
  };
  p->off_g = take((size_t)nn * nn * 8);
  p->off_part = take((size_t)p->S * p->ntiles * p->gt * p->gt * 8);
  p->off_rc = take((size_t)nn * kk * 8);
  p->off_d = take((size_t)nn * 8);
  p->off_pv = take((size_t)nn * 4);
  p->off_pos0 = take((size_t)nn * 4);
  p->off_pos1 = take((size_t)nn * 4);
  p->off_am0 = take((size_t)p->nblk * sizeof(AmaxPart));
  p->off_am1 = take((size_t)p->nblk * sizeof(AmaxPart));
  p->off_state = take(sizeof(GramState));
  p->bytes = off;
  return true;
}

size_t gram_workspace(int64_t m, int64_t n, int32_t dtype, const id_opts* o) {
  GramPlan p;
  if (!make_gram_plan(m, n, dtype, o, &p)) return 0;
  return p.bytes;
}

template <typename T>
struct Vec16B;  // 16-byte vector of T
template <>
struct Vec16B<float> {
  typedef float4 type;
  static constexpr int n = 4;
};
template <>
struct Vec16B<double> {
  typedef double2 type;
  static constexpr int n = 2;
};

// Upper tile (I, J), I <= J, of the Gram matrix over rows [s chunk, (s+1) chunk):
// P[s][t] = A(rows, I cols)^T A(rows, J cols) on the FP64 matrix cores, 64 x 64
// tiles.  Four waves, each a 32 x 32 quarter as 2 x 2 16x16x4 blocks; kGK64
// rows of A staged in LDS per round, the next two rounds' loads in flight in
// registers.  VEC: every column of A starts on a 16-byte boundary, so full
// rounds use 16-byte loads (the scalar, bounds-checked form serves the last
// round of a chunk and unaligned inputs).  The 1-D grid is remapped so that
// the tiles of one row chunk run on the same XCD (they share its rows of A
// through that XCD's L2); four waves per SIMD keep 16 blocks resident per CU.
template <typename TA, bool VEC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void
k_gram_partial64(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t nt,
                 int64_t ntiles, int64_t S, int64_t chunk, double* __restrict__ P) {
  __shared__ double As[kGK64][64 + 1];
  __shared__ double Bs[kGK64][64 + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int64_t per = gridDim.x / 8;
  const int64_t v = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (v >= S * ntiles) return;
  const int64_t s = v / ntiles;
  // tile index -> (I, J) with I <= J, row-major over the upper triangle
  int64_t t = v % ntiles, I = 0;
  while (t >= nt - I) {
    t -= nt - I;
    ++I;
  }
  const int64_t J = I + t;
  const int64_t tile = v % ntiles;
  const int64_t i0 = I * 64, j0 = J * 64;
  const int64_t r0 = s * chunk;
  const int64_t r1 = r0 + chunk < m ? r0 + chunk : m;
  const bool diag = I == J;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;
  // load mapping: tile column c = tid / kGTH, rows kGR (tid % kGTH) .. + kGR - 1
  const int lc = tid / kGTH, lr = (tid % kGTH) * kGR;
  const bool okI = i0 + lc < n, okJ = !diag && j0 + lc < n;
  const TA* ci = A + (okI ? (i0 + lc) * lda : 0) + lr;
  const TA* cj = A + (okJ ? (j0 + lc) * lda : 0) + lr;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (f64x4){0.0, 0.0, 0.0, 0.0};
  TA ra[2][kGR], rb[2][kGR];
  auto load = [&](int q, int64_t k0) {
    if (VEC && k0 + kGK64 <= r1) {
      typedef typename Vec16B<TA>::type VT;
      constexpr int NV = Vec16B<TA>::n;
#pragma unroll
      for (int e = 0; e < kGR; e += NV) {
        VT x, y;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          x[c] = (TA)0;
          y[c] = (TA)0;
        }
        if (okI) x = *(const VT*)(ci + k0 + e);
        if (okJ) y = *(const VT*)(cj + k0 + e);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          ra[q][e + c] = x[c];
          rb[q][e + c] = y[c];
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < kGR; ++e) {
      const bool in = k0 + lr + e < r1;
      ra[q][e] = (okI && in) ? ci[k0 + e] : (TA)0;
      rb[q][e] = (okJ && in) ? cj[k0 + e] : (TA)0;
    }
  };
  auto stage = [&](int q) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kGR; ++e) {
      As[lr + e][lc] = (double)ra[q][e];
      Bs[lr + e][lc] = diag ? (double)ra[q][e] : (double)rb[q][e];
    }
    __syncthreads();
  };
  auto products = [&]() {
#pragma unroll
    for (int kk = 0; kk < kGK64; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = As[kk + g][wr + 16 * x + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = Bs[kk + g][wc + 16 * y + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  };
  load(0, r0);
  load(1, r0 + kGK64);
  for (int64_t k0 = r0; k0 < r1; k0 += 2 * kGK64) {
    stage(0);
    if (k0 + 2 * kGK64 < r1) load(0, k0 + 2 * kGK64);
    products();
    if (k0 + kGK64 >= r1) break;
    stage(1);
    if (k0 + 3 * kGK64 < r1) load(1, k0 + 3 * kGK64);
    products();
  }
  double* out = P + (s * ntiles + tile) * (64 * 64);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(wr + 16 * x + g + 4 * r) * 64 + wc + 16 * y + li] = acc[x][y][r];
}

// G = sum over the row chunks of the partial tiles (fixed order), both
// triangles; a non-finite entry marks the input.
__global__ __launch_bounds__(kThreads) void k_gram_reduce(const double* __restrict__ P, int64_t S,
                                                         int64_t ntiles, int64_t nt, int64_t gt,
                                                         int64_t n, double* __restrict__ G,
                                                         int32_t* info) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t tt = gt * gt;
  if (e >= ntiles * tt) return;
  const int64_t tile = e / tt, w = e % tt;
  int64_t t = tile, I = 0;
  while (t >= nt - I) {
    t -= nt - I;
    ++I;
  }
  const int64_t J = I + t;
  const int64_t ii = I * gt + w / gt, jj = J * gt + w % gt;
  if (ii >= n || jj >= n) return;
  if (I == J && w / gt > w % gt) return;  // diagonal tiles: upper half only (symmetric G)
  double v = 0.0;
  for (int64_t s = 0; s < S; ++s) v += P[(s * ntiles + tile) * tt + w];
  if (!isfinite(v)) *info = ID_INFO_NONFINITE;
  G[jj * n + ii] = v;
  G[ii * n + jj] = v;
}

// State, swap-order keys, Schur diagonal, pivot partials of step 0.
__global__ __launch_bounds__(kThreads) void k_pchol_init(const double* __restrict__ G, int64_t n,
                                                        double* __restrict__ d, int* __restrict__ pv,
                                                        int* __restrict__ pos0,
                                                        AmaxPart* __restrict__ am,
                                                        GramState* st) {
  __shared__ AmaxVal ascr[4];
  const int64_t l = (int64_t)blockIdx.x * kPC + (threadIdx.x % kPC);
  AmaxVal c = amax_none();
  if (threadIdx.x < kPC && l < n) {
    const double v = G[l * n + l];
    d[l] = v;
    pv[l] = 0;
    pos0[l] = (int)l;
    if (st->info == 0) {
      c.v = sqrt(v > 0.0 ? v : 0.0);
      c.s2 = v > 0.0 ? v : 0.0;
      c.pos = (int)l;
      c.key = (int)l;
    }
  }
  c = block_amax(c, ascr);
  if (threadIdx.x == 0) {
    AmaxPart o;
    o.v = c.v;
    o.s2 = c.s2;
    o.pos = c.pos;
    o.key = c.key;
    am[blockIdx.x] = o;
  }
}

struct PcholArgs {
  const double* G;
  int64_t n, kcap, nblk;
  double* Rc;  // Rc[l * kcap + i] = R(i, original column l)
  double* d;
  int* pv;
  const int* pos_in;
  int* pos_out;
  const AmaxPart* am_in;
  AmaxPart* am_out;
  GramState* st;
  int64_t j;
  int64_t k_fixed;
  double rel_tol;
  double floor_rel;  // kGramFloor n u_64: the resolution floor of d_p / |R_00|^2
  int rule;
};

// Pivot step j.  Every block reduces the previous step's pivot partials (same
// result everywhere), applies the rank rule, then for its kPC columns forms
// R(j, l), the new Schur diagonal d_l = G_ll - sum_{i<=j} R_il^2 (recomputed, not
// downdated), the swap-order keys after this step's swap, and a pivot partial.
__global__ __launch_bounds__(kThreads) void k_pchol_step(PcholArgs a) {
  __shared__ double rp[2048];
  __shared__ AmaxVal ascr[4];
  __shared__ int s_go;
  const int tid = threadIdx.x;
  const int64_t j = a.j;
  const int jn = (int)j;
  // 16 threads per column: partial sums over i = t, t + 16, ... (coalesced)
  const int cl = tid >> 4, tq = tid & 15;
  const int64_t l = (int64_t)blockIdx.x * kPC + cl;
  const int64_t lc = l < a.n ? l : 0;
  // Round trip 1, everything that does not depend on the pivot, issued as one
  // group: unconditional loads from clamped in-bounds addresses (a
  // conditional load makes the compiler wait for every earlier load first);
  // values out of range are masked after the barrier.  The first kPcR
  // entries per thread of column l of R are kept in registers.
  const AmaxPart pp0 = a.am_in[tid < a.nblk ? tid : 0];
  const int pin = a.pos_in[lc];
  const int pvl = a.pv[lc];
  const double gll = a.G[lc * a.n + lc];
  const double* rl = a.Rc + lc * a.kcap;
  double xr[kPcR];
#pragma unroll
  for (int u = 0; u < kPcR; ++u) {
    const int i = tq + 16 * u;
    xr[u] = rl[i < jn ? i : 0];  // entries i >= j are not used
  }
  if (tid == 0) s_go = a.st->done == 0 && a.st->info == 0;
  AmaxVal best = amax_none();
  if (tid < a.nblk) {
    best.v = pp0.v;
    best.s2 = pp0.s2;
    best.pos = pp0.pos;
    best.key = pp0.key;
  }
  if (a.nblk > kThreads) {  // uniform; more than one partial per thread
    for (int64_t q = tid + kThreads; q < a.nblk; q += kThreads) {
      const AmaxPart pp = a.am_in[q];
      AmaxVal c;
      c.v = pp.v;
      c.s2 = pp.s2;
      c.pos = pp.pos;
      c.key = pp.key;
      best = amax_combine(best, c);
    }
  }
  best = block_amax(best, ascr);  // its barriers also publish s_go
  if (!s_go) return;
  const int p = best.pos;
  const double vp = best.v;
  const double r00 = j == 0 ? vp : a.st->r00;
  const double fro2 = j == 0 ? best.s2 : a.st->fro2;
  bool stop = (j >= a.kcap) || (p < 0);
  if (!stop && a.k_fixed == 0) {
    if (!(vp > 0.0))
      stop = true;
    else if (a.rule == ID_RANK_PIVOT_REL)
      stop = j > 0 && vp <= a.rel_tol * r00;
    else
      stop = sqrt(best.s2) <= a.rel_tol * sqrt(fro2);
  }
  // the resolution guard (every block takes the same decision: same best)
  const bool at_floor = !stop && j > 0 && vp * vp <= a.floor_rel * r00 * r00;
  if (stop || at_floor) {
    if (blockIdx.x == 0 && tid == 0) {
      a.st->done = 1;
      a.st->k = j;
      if (at_floor) a.st->limit = 1;
    }
    return;
  }
  // (reaching kcap is detected by step kcap itself: "done" must not change
  // while other blocks of this step may still read it)
  if (blockIdx.x == 0 && tid == 0 && j == 0) {
    a.st->r00 = r00;
    a.st->fro2 = fro2;
  }
  const double rjj = vp;  // sqrt(d_p)
  // round trip 2: the pivot's column of R (to LDS), G(p, l), its key
  const double gpl = a.G[(int64_t)p * a.n + lc];
  const int pos_p = a.pos_in[p];
  for (int i = tid; i < jn; i += kThreads) rp[i] = a.Rc[(int64_t)p * a.kcap + i];
  __syncthreads();
  AmaxVal cand = amax_none();
  if (l < a.n) {
    const int key = l == p ? jn : (pin == jn ? pos_p : pin);
    const bool live = !pvl && l != p;
    double dot = 0.0, ss = 0.0;
    if (live) {
#pragma unroll
      for (int u = 0; u < kPcR; ++u) {
        const int i = tq + 16 * u;
        if (i < jn) {
          dot += rp[i] * xr[u];
          ss += xr[u] * xr[u];
        }
      }
      for (int i = tq + 16 * kPcR; i < jn; i += 16) {
        const double x = rl[i];
        dot += rp[i] * x;
        ss += x * x;
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      dot += __shfl_xor(dot, off, 64);
      ss += __shfl_xor(ss, off, 64);
    }
    if (tq == 0) {
      a.pos_out[l] = key;
      if (l == p) {
        a.Rc[l * a.kcap + j] = rjj;
        a.pv[l] = 1;
        a.d[l] = 0.0;
      } else if (live) {
        const double r = (gpl - dot) / rjj;
        a.Rc[l * a.kcap + j] = r;
        double dl = gll - (ss + r * r);
        if (!(dl > 0.0)) dl = 0.0;
        a.d[l] = dl;
        cand.v = sqrt(dl);
        cand.s2 = dl;
        cand.pos = (int)l;
        cand.key = key;
      }
    }
  }
  cand = block_amax(cand, ascr);
  if (tid == 0) {
    AmaxPart o;
    o.v = cand.v;
    o.s2 = cand.s2;
    o.pos = cand.pos;
    o.key = cand.key;
    a.am_out[blockIdx.x] = o;
  }
}

// perm (swap order: perm[pos[l]] = l) and R in pivot order from Rc.
__global__ __launch_bounds__(kThreads) void k_pchol_perm(const int* __restrict__ pos, int64_t n,
                                                        int32_t* __restrict__ perm) {
  const int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (l < n) perm[pos[l]] = (int32_t)l;
}

__global__ __launch_bounds__(kThreads) void k_pchol_gather(const int32_t* __restrict__ perm,
                                                          const double* __restrict__ Rc,
                                                          int64_t kcap, int64_t n, int64_t k,
                                                          double* __restrict__ R, int64_t ldr) {
  const int64_t c = blockIdx.x;
  const int64_t i = (int64_t)blockIdx.y * kThreads + threadIdx.x;
  if (c >= n || i >= k) return;
  const int l = perm[c];
  R[c * ldr + i] = (c >= k || i <= c) ? Rc[(int64_t)l * kcap + i] : 0.0;
}

__global__ void k_gram_iota(int32_t* perm, int64_t n) {
  const int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (l < n) perm[l] = (int32_t)l;
}

static int identity_perm(int32_t* perm, int64_t n, hipStream_t s) {
  if (n <= 0) return ID_OK;
  k_gram_iota<<<dim3((unsigned)ceil_div(n, kThreads)), kThreads, 0, s>>>(perm, n);
  MPID_LAUNCH_CHECK();
  MPID_HIP(hipStreamSynchronize(s));
  return ID_OK;
}

__global__ void k_gram_state_init(GramState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->done = 0;
    st->info = 0;
    st->limit = 0;
    st->k = 0;
    st->r00 = 0.0;
    st->fro2 = 0.0;
  }
}

// G = A^T A in FP64 (both triangles): the partial tiles over row chunks, then
// their sum in a fixed order; a non-finite entry sets *info.
static int gram_product(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                        const GramPlan& pl, double* P, double* G, int32_t* info, hipStream_t s) {
  {
    const dim3 g1((unsigned)round_up(pl.S * pl.ntiles, 8));
    // 16-byte loads need 16-byte aligned columns of A
    const int64_t esz = dtype == ID_F64 ? 8 : 4;
    const bool vec = ((uintptr_t)A % 16 == 0) && ((lda * esz) % 16 == 0);
    if (dtype == ID_F64) {
      if (vec)
        k_gram_partial64<double, true><<<g1, kThreads, 0, s>>>(
            (const double*)A, lda, m, n, pl.nt, pl.ntiles, pl.S, pl.chunk, P);
      else
        k_gram_partial64<double, false><<<g1, kThreads, 0, s>>>(
            (const double*)A, lda, m, n, pl.nt, pl.ntiles, pl.S, pl.chunk, P);
    } else {
      if (vec)
        k_gram_partial64<float, true><<<g1, kThreads, 0, s>>>(
            (const float*)A, lda, m, n, pl.nt, pl.ntiles, pl.S, pl.chunk, P);
      else
        k_gram_partial64<float, false><<<g1, kThreads, 0, s>>>(
            (const float*)A, lda, m, n, pl.nt, pl.ntiles, pl.S, pl.chunk, P);
    }
  }
  MPID_LAUNCH_CHECK();
  k_gram_reduce<<<dim3((unsigned)ceil_div(pl.ntiles * pl.gt * pl.gt, kThreads)), kThreads, 0, s>>>(
      P, pl.S, pl.ntiles, pl.nt, pl.gt, n, G, info);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

// For other front ends: the bytes of partial tiles gram_matrix_run needs, and
// G = A^T A (FP64, n x n, both triangles) with *info = ID_INFO_NONFINITE if A
// holds NaN/Inf (info is left alone otherwise).
size_t gram_matrix_workspace(int64_t m, int64_t n) {
  id_opts o;
  std::memset(&o, 0, sizeof(o));
  o.k_fixed = 1;
  GramPlan pl;
  if (!make_gram_plan(m, n, ID_F64, &o, &pl)) return 0;
  return (size_t)pl.S * pl.ntiles * pl.gt * pl.gt * 8;
}

int gram_matrix_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda, double* G,
                    void* part, size_t part_bytes, int32_t* info, hipStream_t s) {
  id_opts o;
  std::memset(&o, 0, sizeof(o));
  o.k_fixed = 1;
  GramPlan pl;
  if (!make_gram_plan(m, n, dtype, &o, &pl)) return ID_ERR_ARG;
  if (part_bytes < (size_t)pl.S * pl.ntiles * pl.gt * pl.gt * 8) return ID_ERR_WORKSPACE;
  if (m <= 0 || n <= 0) return ID_OK;
  return gram_product(A, dtype, m, n, lda, pl, (double*)part, G, info, s);
}

int gram_factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                    const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                    int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s) {
  GramPlan pl;
  if (!make_gram_plan(m, n, dtype, o, &pl)) return ID_ERR_ARG;
  if (o->flags & (ID_FLAG_NO_PIVOT | ID_FLAG_PROFILE | ID_FLAG_ROUND_F32 | ID_FLAG_ROUND_F16))
    return ID_ERR_UNSUPPORTED;
  if (!k_out || !info) return ID_ERR_ARG;
  if (n > 0 && !perm) return ID_ERR_ARG;
  if (m > 0 && n > 0 && !A) return ID_ERR_ARG;
  if (lda < (m > 1 ? m : 1)) return ID_ERR_ARG;
  if (pl.kcap > 0 && (!R || ldr < pl.kcap)) return ID_ERR_ARG;
  if (!work || work_bytes < pl.bytes) return ID_ERR_WORKSPACE;
  if (pl.kcap > 2048) return ID_ERR_UNSUPPORTED;  // column of R staged in LDS
  // adaptive tolerances below the route's resolution cannot be honoured
  if (o->k_fixed == 0 && o->rel_tol < kGramMinTol) return ID_ERR_UNSUPPORTED;
  *info = 0;
  *k_out = 0;
  if (m == 0 || n == 0 || pl.kcap == 0) return identity_perm(perm, n, s);
  char* wb = (char*)work;
  double* G = (double*)(wb + pl.off_g);
  double* P = (double*)(wb + pl.off_part);
  double* Rc = (double*)(wb + pl.off_rc);
  double* d = (double*)(wb + pl.off_d);
  int* pv = (int*)(wb + pl.off_pv);
  int* pos[2] = {(int*)(wb + pl.off_pos0), (int*)(wb + pl.off_pos1)};
  AmaxPart* am[2] = {(AmaxPart*)(wb + pl.off_am0), (AmaxPart*)(wb + pl.off_am1)};
  GramState* st = (GramState*)(wb + pl.off_state);

  k_gram_state_init<<<1, 64, 0, s>>>(st);
  MPID_LAUNCH_CHECK();
  {
    const int rg = gram_product(A, dtype, m, n, lda, pl, P, G, &st->info, s);
    if (rg) return rg;
  }
  k_pchol_init<<<dim3((unsigned)pl.nblk), kThreads, 0, s>>>(G, n, d, pv, pos[0], am[0], st);
  MPID_LAUNCH_CHECK();

  // pivot steps, enqueued in groups; the host looks at the device state one
  // group behind, so the GPU does not wait for it (steps after the stop return)
  GramState* hs = nullptr;
  MPID_HIP(hipHostMalloc((void**)&hs, 2 * sizeof(GramState), hipHostMallocDefault));
  hipEvent_t ev[2];
  if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(hs);
    return ID_ERR_HIP;
  }
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    (void)hipHostFree(hs);
    return ID_ERR_HIP;
  }
  int rc = ID_OK;
  const int64_t group = 32;
  int64_t j = 0, gidx = 0;
  bool finished = false;
  PcholArgs pa;
  pa.G = G;
  pa.n = n;
  pa.kcap = pl.kcap;
  pa.nblk = pl.nblk;
  pa.Rc = Rc;
  pa.d = d;
  pa.pv = pv;
  pa.st = st;
  pa.k_fixed = o->k_fixed;
  pa.rel_tol = o->rel_tol;
  pa.floor_rel = kGramFloor * (double)n * std::ldexp(1.0, -53);
  pa.rule = o->rank_rule;
  while (!finished && j < pl.kcap + 1) {
    const int64_t jend = j + group < pl.kcap + 1 ? j + group : pl.kcap + 1;
    for (; j < jend; ++j) {
      pa.j = j;
      pa.pos_in = pos[j & 1];
      pa.pos_out = pos[(j + 1) & 1];
      pa.am_in = am[j & 1];
      pa.am_out = am[(j + 1) & 1];
      k_pchol_step<<<dim3((unsigned)pl.nblk), kThreads, 0, s>>>(pa);
      if (hipGetLastError() != hipSuccess) {
        rc = ID_ERR_HIP;
        break;
      }
    }
    if (rc) break;
    const int slot = (int)(gidx & 1);
    if (hipMemcpyAsync(&hs[slot], st, sizeof(GramState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ev[slot], s) != hipSuccess) {
      rc = ID_ERR_HIP;
      break;
    }
    // look at the previous group (the one just enqueued keeps the GPU busy)
    if (gidx >= 1) {
      const int prev = (int)((gidx - 1) & 1);
      if (hipEventSynchronize(ev[prev]) != hipSuccess) {
        rc = ID_ERR_HIP;
        break;
      }
      if (hs[prev].done || hs[prev].info) finished = true;
    }
    ++gidx;
  }
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = ID_ERR_HIP;
  GramState fin;
  if (!rc && hipMemcpy(&fin, st, sizeof(GramState), hipMemcpyDeviceToHost) != hipSuccess)
    rc = ID_ERR_HIP;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  (void)hipHostFree(hs);
  if (rc) return rc;
  if (fin.info) {
    *info = fin.info;
    *k_out = 0;
    return identity_perm(perm, n, s);
  }
  const int64_t k = fin.done ? fin.k : pl.kcap;
  *k_out = k;
  if (fin.limit) *info = ID_INFO_GRAM_LIMIT;
  // the keys after the last executed step are in pos[k & 1]
  k_pchol_perm<<<dim3((unsigned)ceil_div(n, kThreads)), kThreads, 0, s>>>(pos[k & 1], n, perm);
  MPID_LAUNCH_CHECK();
  if (k > 0) {
    k_pchol_gather<<<dim3((unsigned)n, (unsigned)ceil_div(k, kThreads)), kThreads, 0, s>>>(
        perm, Rc, pl.kcap, n, k, R, ldr);
    MPID_LAUNCH_CHECK();
  }
  MPID_HIP(hipStreamSynchronize(s));
  return ID_OK;
}

}  // namespace mpid
