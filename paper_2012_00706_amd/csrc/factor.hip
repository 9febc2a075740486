// Rank-k column-pivoted Householder QR on gfx950 (MI355X).
//
// The method is the truncated column-pivoted QR  A Z = Q R  of the column ID
// (Section 1.1, eq. (6)-(7); the MGSQR(A, k) step of Algorithms 1 and 2), with
// Householder reflectors and a lazily blocked ("left-looking within a panel")
// trailing update: inside a panel of up to nb pivots the trailing columns are
// not touched; each step only
//   1. picks the remaining column of largest (downdated) norm,
//   2. brings that column up to date (w = W(:,p) - V F(p,:)^T),
//   3. builds its reflector and sweeps the stale trailing block once to get
//      the new column of F and the new row of R,
//   4. downdates the remaining column norms,
// and at the end of the panel one matrix-core update W -= V F^T refreshes the
// trailing block, recomputes every column norm in FP64 from the refreshed
// data, and compacts away the columns that were pivoted.
//
// Data layout: the working copy W is ROW-major (ld = ldw >= n, multiple of 64)
// so that the dominant operation -- W^T v over a tall block -- streams rows
// with fully coalesced 16-byte loads, lanes owning columns and the reflector
// entry of a row being a broadcast value.  Reflectors are stored unscaled
// (V(:,c) = Vraw(:,c) * vscale[c]) column-major; F is column-major over the
// positions of the current layout.  R is accumulated by ORIGINAL column id and
// gathered into pivot order at the end.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "device_util.h"
#include "mpid_internal.h"

namespace mpid {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename S>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

enum { OP_F64 = 0, OP_F16 = 1, OP_BF16 = 2, OP_BF16X3 = 3, OP_F32 = 4 };

// Storage rounding of the simulated low precision (ID_FLAG_ROUND_F32 /
// ID_FLAG_ROUND_F16): a value the factorization keeps (working copy,
// reflectors, F, R, column norms) is rounded to the nearest binary32 or
// binary16 number; arithmetic on it stays in the kernel's precision.
enum { RM_NONE = 0, RM_F32 = 1, RM_F16 = 2 };
__device__ __forceinline__ double rnd(double x, int mode) {
  if (mode == RM_F32) return (double)(float)x;
  if (mode == RM_F16) return (double)(_Float16)x;
  return x;
}
template <typename S>
__device__ __forceinline__ S rnd_store(double x, int mode) {
  return (S)rnd(x, mode);
}
// the same with the mode fixed at compile time (kernels whose registers are
// tight: the run-time branch raised their register count)
template <int RM>
__device__ __forceinline__ double rndc(double x) {
  if (RM == RM_F32) return (double)(float)x;
  if (RM == RM_F16) return (double)(_Float16)x;
  return x;
}

constexpr int kPrefetch = 4;  // sweep rows per thread loaded ahead of the pivot search
constexpr int kFinZ = (192 + kFL - 1) / kFL;  // column partials per lane and round trip in the finalization
constexpr int kFinA = 24;     // reflector-product partials per thread and round trip
constexpr int kFold = 32;     // row tiles summed per folded partial (tall inputs)
constexpr int kSweepU = 4;    // sweep rows per thread in flight in the main loop
// the same where the step's trailing block is far larger than the caches (the
// loop is bound by bytes in flight over memory latency, which is longer there)
constexpr int kSweepUDeep = 8;
constexpr double kDeepBytes = 256.0 * 1024 * 1024;  // the Infinity Cache
// main-loop rows per thread loaded with the second round trip: 8 where the
// registers allow it without lowering occupancy (fp32, row tiles <= 128)
template <typename S, int G>
constexpr int overlap_rows() {
  return (sizeof(S) == 4 && G >= 2) ? 8 : 4;
}

// ----------------------------------------------------------------- plan

bool make_factor_plan(int64_t m, int64_t n, int32_t dtype, const id_opts* o, FactorPlan* p) {
  if (!o || !p || m < 0 || n < 0) return false;
  if (dtype != ID_F32 && dtype != ID_F64) return false;
  if (o->prec != ID_PREC_F64 && o->prec != ID_PREC_MIXED_F16 && o->prec != ID_PREC_MIXED_BF16 &&
      o->prec != ID_PREC_MIXED_BF16X3 && o->prec != ID_PREC_MIXED_F32)
    return false;
  if (o->rank_rule != ID_RANK_PIVOT_REL && o->rank_rule != ID_RANK_FROB_REL) return false;
  if (o->k_fixed < 0 || o->k_max < 0 || !(o->rel_tol >= 0.0)) return false;
  // the simulated single / half precision pairs with its own update
  if ((o->flags & ID_FLAG_ROUND_F32) && (o->flags & ID_FLAG_ROUND_F16)) return false;
  if ((o->flags & ID_FLAG_ROUND_F32) && o->prec != ID_PREC_MIXED_F32) return false;
  if ((o->flags & ID_FLAG_ROUND_F16) && o->prec != ID_PREC_MIXED_F16) return false;
  const int nb = o->nb == 0 ? kNbMax : o->nb;
  if (nb < 1 || nb > kNbMax) return false;
  if (m > (int64_t)1 << 31 || n > (int64_t)1 << 30) return false;
  int64_t kcap = m < n ? m : n;
  if (o->k_max > 0 && o->k_max < kcap) kcap = o->k_max;
  if (o->k_fixed > 0 && o->k_fixed < kcap) kcap = o->k_fixed;
  std::memset(p, 0, sizeof(*p));
  p->m = m;
  p->n = n;
  p->kcap = kcap;
  p->dtype = dtype;
  p->prec = o->prec;
  p->nb = nb;
  p->wbytes = o->prec == ID_PREC_F64 ? 8 : 4;
  const int64_t mm = m > 0 ? m : 1, nn = n > 0 ? n : 1, kk = kcap > 0 ? kcap : 1;
  // rows of the working copy an odd multiple of 256 bytes apart, so that
  // consecutive rows start in different memory channels
  const int64_t q256 = 256 / p->wbytes;
  p->ldw = round_up(nn, 64);
  if ((p->ldw / q256) % 2 == 0) p->ldw += q256;
  p->ldv = round_up(mm, 64);
  p->ldf = round_up(nn, 64);
  p->ntile_s_max = ceil_div(mm, kRtMin);
  p->ntile_g = ceil_div(mm, kRowTileG);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  p->off_w0 = take((size_t)mm * p->ldw * p->wbytes);
  p->off_w1 = take((size_t)mm * p->ldw * p->wbytes);
  p->off_v = take((size_t)kNbMax * p->ldv * p->wbytes);
  p->off_f = take((size_t)kNbMax * p->ldf * 8);
  // per-tile partials, plus a row of zeros after the last tile (zeroed by
  // k_init, never written by a sweep or fold)
  p->off_zpart = take((size_t)(p->ntile_s_max + 1) * p->ldf * 8);
  p->off_auxpart = take((size_t)(p->ntile_s_max + 1) * kNbMax * 8);
  p->off_nrm2part = take((size_t)(p->ntile_s_max + 1) * 8);
  const int64_t nfold = ceil_div(p->ntile_s_max, kFold);
  p->nfold_max = nfold;
  p->off_zfold = take((size_t)(nfold + 1) * p->ldf * 8);
  p->off_afold = take((size_t)(nfold + 1) * kNbMax * 8);
  p->off_nfold = take((size_t)(nfold + 1) * 8);
  p->off_colpart = take((size_t)p->ntile_g * p->ldf * 8);
  p->off_nu = take((size_t)p->ldf * 8);
  p->off_nuo = take((size_t)p->ldf * 8);
  p->off_amax = take((size_t)(p->ldf / kFC + 8) * sizeof(AmaxPart));
  p->off_colid0 = take((size_t)p->ldf * 4);
  p->off_colid1 = take((size_t)p->ldf * 4);
  p->off_pvflag = take((size_t)p->ldf * 4);
  p->off_pivpos = take((size_t)kNbMax * 4);
  p->off_pivid = take((size_t)kk * 4);
  p->off_permw = take((size_t)nn * 4);
  p->off_posof = take((size_t)nn * 4);
  p->off_tau = take((size_t)kk * 8);
  p->off_vscale = take((size_t)kNbMax * 8);
  p->off_rorig = take((size_t)kk * nn * 8);
  p->off_state = take(sizeof(FactorState));
  p->off_slot = take(2 * sizeof(FactorHostSlot));  // panel end states (allocation-free calls)
  p->off_wrow = take((size_t)p->ldf * 8);
  p->off_vrow = take((size_t)kNbMax * 8);
  p->off_keypos = take((size_t)p->ldf * 4);
  p->bytes = off;
  return true;
}

// ----------------------------------------------------------------- kernels

// zrow[0..2] / frow[0..2]: the zero rows of the per-tile and the folded
// partials (ldf, kNbMax and 1 entries).
struct InitArgs {
  FactorState* st;
  int *colid0, *pvflag, *permw, *posof;
  int64_t n, ldf;
  double *zrow_z, *zrow_a, *zrow_n, *frow_z, *frow_a, *frow_n;
};

__device__ __forceinline__ void init_block(const InitArgs& a, const int64_t bx) {
  FactorState* st = a.st;
  int *colid0 = a.colid0, *pvflag = a.pvflag, *permw = a.permw, *posof = a.posof;
  const int64_t n = a.n, ldf = a.ldf;
  double *zrow_z = a.zrow_z, *zrow_a = a.zrow_a, *zrow_n = a.zrow_n;
  double *frow_z = a.frow_z, *frow_a = a.frow_a, *frow_n = a.frow_n;
  const int64_t l = bx * kThreads + threadIdx.x;
  if (l < ldf) {
    colid0[l] = (int)l;
    pvflag[l] = 0;
    zrow_z[l] = 0.0;
    frow_z[l] = 0.0;
  }
  if (l < kNbMax) {
    zrow_a[l] = 0.0;
    frow_a[l] = 0.0;
  }
  if (l == 0) {
    zrow_n[0] = 0.0;
    frow_n[0] = 0.0;
  }
  if (l < n) {
    permw[l] = (int)l;
    posof[l] = (int)l;
  }
  if (l == 0) {
    st->done = 0;
    st->end_flag = 0;
    st->jb = 0;
    st->last_jb = 0;
    st->info = 0;
    st->fmax_bits = 0u;
    st->vmax_bits = 0u;
    st->nabove = 0u;
    st->nred = 0u;
    st->k = 0;
    st->r00 = 0.0;
    st->alpha = 0.0;
    st->fro2 = 0.0;
    st->off = 0;
    st->ncur = n;
  }
}

__global__ __launch_bounds__(kThreads) void k_init(InitArgs a) { init_block(a, blockIdx.x); }

// A (column-major, lda) -> W (row-major, ldw) in the working precision, with
// the per-row-tile partial sums of squares of every column (FP64) and a
// NaN/Inf check.  Block: 64 columns x kRowTileG rows, LDS transpose.
template <typename TA, typename S>
struct IngestArgs {
  const TA* A;
  int64_t lda, m, n;
  S* W;
  int64_t ldw;
  double* colpart;
  int64_t ldf;
  FactorState* st;
  int rmode;
};

template <typename TA, typename S>
__device__ __forceinline__ void ingest_block(const IngestArgs<TA, S>& ia, const int64_t bx,
                                             const int64_t tg) {
  const TA* __restrict__ A = ia.A;
  S* __restrict__ W = ia.W;
  double* __restrict__ colpart = ia.colpart;
  const int64_t lda = ia.lda, m = ia.m, n = ia.n, ldw = ia.ldw, ldf = ia.ldf;
  const int rmode = ia.rmode;
  __shared__ S tile[64][65];
  __shared__ double ssq[4][64];
  const int tid = threadIdx.x;
  const int64_t c0 = bx * 64;
  const int64_t rb = tg * kRowTileG;
  const int64_t re = rb + kRowTileG < m ? rb + kRowTileG : m;
  double ss = 0.0;
  bool bad = false;
  for (int64_t rs = rb; rs < re; rs += 64) {
    // the 16 loads of a thread issued as one group: unconditional, from
    // clamped in-range addresses (tile entries outside the matrix are never
    // stored or summed)
    TA xv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = q * 4 + tid / 64, rr = tid % 64;
      const int64_t r = rs + rr, c = c0 + cc;
      xv[q] = A[(c < n ? c : n - 1) * lda + (r < re ? r : re - 1)];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = q * 4 + tid / 64, rr = tid % 64;
      const int64_t r = rs + rr, c = c0 + cc;
      if (r < re && c < n && !isfinite((double)xv[q])) bad = true;
      tile[cc][rr] = rmode ? rnd_store<S>((double)xv[q], rmode) : (S)xv[q];
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int rr = tid / 64 + 4 * q, cc = tid % 64;
      const int64_t r = rs + rr, c = c0 + cc;
      if (r < re && c < n) {
        const S v = tile[cc][rr];
        W[r * ldw + c] = v;
        ss += (double)v * (double)v;
      }
    }
    __syncthreads();
  }
  ssq[tid / 64][tid % 64] = ss;
  __syncthreads();
  if (tid < 64) {
    const int64_t c = c0 + tid;
    if (c < n) colpart[tg * ldf + c] = ssq[0][tid] + ssq[1][tid] + ssq[2][tid] + ssq[3][tid];
  }
  if (bad) ia.st->info = ID_INFO_NONFINITE;
}

template <typename TA, typename S>
__global__ __launch_bounds__(kThreads) void k_ingest(IngestArgs<TA, S> a) {
  ingest_block<TA, S>(a, blockIdx.x, blockIdx.y);
}

// One block of the column-norm reduction (see k_colreduce).
__device__ __forceinline__ void colreduce_block(
    const double* __restrict__ colpart, int64_t ldf, int64_t tg0, int64_t tg1, int64_t ncols_base,
    int subtract_jb, double* __restrict__ nu, double* __restrict__ nuo, AmaxPart* __restrict__ amax,
    const int* __restrict__ colid, const int* __restrict__ posof, int* __restrict__ pvflag,
    int* __restrict__ keypos, FactorState* st, double rel_tol, int rmode,
    double (*red)[kFinCols + 1], AmaxVal* ascr, const int bid) {
  const int tid = threadIdx.x, cl = tid % kFinCols, tl = tid / kFinCols;
  const int64_t ncols = subtract_jb ? st->ncur - st->jb : ncols_base;
  const int64_t l = (int64_t)bid * kFinCols + cl;
  red[tl][cl] = l < ncols ? strided_sum(colpart + l, ldf, tg0 + tl, tg1, 8) : 0.0;
  __syncthreads();
  AmaxVal cand = amax_none();
  int above = 0;
  if (tl == 0 && l < ncols) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) tot += red[q][cl];
    const double v = rnd(sqrt(tot), rmode);
    nu[l] = v;
    nuo[l] = v;
    pvflag[l] = 0;
    cand.v = v;
    cand.s2 = tot;
    cand.pos = (int)l;
    cand.key = posof[colid[l]];
    keypos[l] = cand.key;
    above = v > rel_tol * st->r00 ? 1 : 0;
  }
  cand = block_amax(cand, ascr);
  const int nabove = __syncthreads_count(above);
  if (tid == 0) {
    if (rel_tol >= 0.0 && nabove > 0) atomicAdd(&st->nabove, (uint32_t)nabove);
    AmaxPart o;
    o.v = cand.v;
    o.s2 = cand.s2;
    o.pos = cand.pos;
    o.key = cand.key;
    amax[bid] = o;
    // the host's view of how close the rank rule is (norms are >= 0)
    if (cand.v > 0.0) atomicMax(&st->vmax_bits, __float_as_uint((float)cand.v));
  }
}

// Column norms from per-row-tile partial sums of squares (FP64): nu = nu_orig
// = sqrt(sum); clears the per-panel pivot flags; per-block pivot partials.
// With rel_tol >= 0, also counts the columns whose norm exceeds
// rel_tol |R_00| (the pivot-relative threshold, in the step's own arithmetic).
// Norms only shrink under the later reflectors, so the next stop comes within
// that many steps plus one.
// At a panel's end (hs != nullptr) the last block to finish also advances the
// state to the next panel and publishes it to the host slot hs with tag seq.
// Block: 32 columns x 8 tile lanes.
struct ColArgs {
  const double* colpart;
  int64_t ldf, tg0, tg1, ncols_base;
  int subtract_jb;
  double *nu, *nuo;
  AmaxPart* amax;
  const int *colid, *posof;
  int *pvflag, *keypos;
  FactorState* st;
  double rel_tol;
  int rmode;
  FactorHostSlot* hs;
  int64_t seq;
};

__device__ __forceinline__ void colreduce_body(const ColArgs& c, const int bid, const int nblk) {
  __shared__ double red[8][kFinCols + 1];
  __shared__ AmaxVal ascr[4];
  __shared__ int s_go, s_last;
  FactorState* st = c.st;
  FactorHostSlot* hs = c.hs;
  const int tid = threadIdx.x;
  if (tid == 0) s_go = (st->done == 0);
  __syncthreads();
  if (s_go)
    colreduce_block(c.colpart, c.ldf, c.tg0, c.tg1, c.ncols_base, c.subtract_jb, c.nu, c.nuo,
                    c.amax, c.colid, c.posof, c.pvflag, c.keypos, st, c.rel_tol, c.rmode, red,
                    ascr, bid);
  if (hs == nullptr) return;
  if (tid == 0) {
    __threadfence();  // this block's counts before its arrival
    s_last = atomicAdd(&st->nred, 1u) == (uint32_t)nblk - 1u;
  }
  __syncthreads();
  if (s_last && tid == 0) {
    __threadfence();  // every block's counts (vmax_bits, nabove) before reading them
    st->nred = 0u;
    if (st->done) {
      // panels enqueued after the stop must not match any step's jb
      st->jb = 0;
    } else {
      st->last_jb = st->jb;
      st->off += st->jb;
      st->ncur -= st->jb;
      st->jb = 0;
      st->end_flag = 0;
      st->fmax_bits = 0u;
    }
    hs->s = *st;
    __threadfence_system();  // the state before its tag
    __hip_atomic_store(&hs->seq, c.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(kThreads) void k_colreduce(ColArgs c) {
  colreduce_body(c, blockIdx.x, gridDim.x);
}

template <typename S>
struct StepArgs {
  const S* W;
  int64_t ldw, m, n, ncur;
  S* V;
  int64_t ldv;
  double* F;
  int64_t ldf;
  double* vscale;
  double* tau;
  FactorState* st;
  AmaxPart* amax;
  int namax;
  int* pvflag;
  const int* colid;
  int* pivpos;
  int* pivid;
  int* permw;
  int* posof;
  double* zpart;
  double* auxpart;
  double* nrm2part;
  double* nu;
  double* nuo;
  double* rorig;
  double* wrow;  // the step's row of W, for the finalization (written by the sweep)
  double* vrow;  // the step's row of the panel's reflectors (unscaled)
  int* keypos;   // swap-order key of each working position
  int64_t kcap, k_fixed;
  double rel_tol, tol3z;
  int rule, nopivot, nb;
  int want_fmax;  // the panel update scales FP16 operands by the panel's max |F|
  int rmode;      // storage rounding (RM_*)
  // per step; j and ncur above are the host's bounds (j <= the step's row,
  // ncur >= the live column count), the exact values live in the state
  int64_t j;
  int jj;
  int64_t t0;
  int ntile, nchunk, Rt, CW;
  int64_t tguard;  // row of zeros in zpart / auxpart / nrm2part (past every tile)
};

// One pivot step, part 1.  Grid: (row tiles of Rt <= 256 rows) x (column
// chunks of CW positions), padded to a multiple of 8 and remapped so that the
// chunks of one row tile run on the same XCD (they share the pivot column and
// the reflector rows through that XCD's L2).  G = 256 / Rt threads share a row.
//  - reduces the pivot partials, applies the rank rule, records the pivot
//    (and which column's swap-order key the swap changed);
//  - w = W(i,p) - sum_c V(i,c) F(p,c) for the tile's rows i >= j;
//  - z(l) = sum_{i>j} W(i,l) w(i) for the chunk's columns (the sweep);
//  - partial sums over the tile of V(i,c) w(i) (c split across the chunks)
//    and, in chunk 0, of w(i)^2; chunk 0 also stores w as reflector jj;
//  - the tile holding row j copies that row of W and of the panel's earlier
//    reflectors for the finalization.
// Everything that does not depend on the pivot -- flags, pivot partials, the
// reflector entries of the tile and the first rows of the sweep -- is loaded
// in one round trip before the pivot is known.
template <typename S, int G, int U = kSweepU>
__device__ __forceinline__ void sweep_block(const StepArgs<S>& a, const int bid, const int nblk) {
  typedef typename Vec16<S>::type VT;
  constexpr int VEC = Vec16<S>::n;
  constexpr int SLOTS = kNbMax / G;
  __shared__ double wsh[kThreads];
  __shared__ double gsh[kNbMax];
  __shared__ double red[kThreads * VEC];
  __shared__ double zred[4][kNbMax];
  __shared__ AmaxVal ascr[4];
  __shared__ double dscr[4];
  __shared__ int s_go, s_info;
  __shared__ double s_r00, s_fro2;
  __shared__ int64_t s_off, s_ncur;
  FactorState* st = a.st;
  const int tid = threadIdx.x;
  const int total = a.ntile * a.nchunk;
  const int per = nblk / 8;
  const int v = (bid % 8) * per + bid / 8;
  if (v >= total) return;
  const int64_t tile = a.t0 + v / a.nchunk;
  const int chunk = v % a.nchunk;
  const int jj = a.jj;
  const int64_t jlb = a.j;  // lower bound of this step's row
  const int64_t r0 = tile * a.Rt;
  const int64_t r1 = r0 + a.Rt < a.m ? r0 + a.Rt : a.m;

  // ---- round trip 1: nothing here depends on the pivot (or on the exact
  // panel offset: the rows loaded from the bound jlb on are a superset).
  // Loads of this round trip are unconditional, from clamped in-bounds
  // addresses (values out of range are never used, or masked after the
  // pivot search): conditional loads make the compiler wait for earlier
  // ones in between, which would split the round trip.
  // the first pivot partial of every thread (there is at least one)
  const AmaxPart pp0 = a.amax[tid < a.namax ? tid : 0];
  // sweep geometry and the first rows of the sweep
  const int TPR = a.CW / VEC;
  const int RG = kThreads / TPR;
  const int rg = tid / TPR, cv = tid % TPR;
  const int64_t l0 = (int64_t)chunk * a.CW + (int64_t)cv * VEC;
  const int64_t ib = (r0 > jlb + 1 ? r0 : jlb + 1) + rg;
  const S* base = a.W + l0;
  VT pf[kPrefetch];
  {
    const S* pbase = a.W + (l0 < a.ncur ? l0 : 0);
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int64_t i = ib + (int64_t)u * RG;
      pf[u] = *(const VT*)(pbase + (i < r1 ? i : r0) * a.ldw);
    }
  }
  // reflector entries of this thread's row: c = gi, gi + G, ...
  const int rsub = tid / G, gi = tid % G;
  const int64_t iw = r0 + rsub;
  // (masked after the pivot search: a select next to its load is turned
  // back into a conditional load; reflectors the panel has not generated yet
  // are read from reflector 0's cached line instead of from memory)
  S vr[SLOTS];
  {
    const int64_t iwc = iw < a.m ? iw : a.m - 1;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
      const int c = gi + G * q;
      vr[q] = a.V[(int64_t)(c < jj ? c : 0) * a.ldv + iwc];
    }
  }
  // the step state, after the vector loads are on their way
  if (tid == 0) {
    s_go = (st->done == 0 && st->end_flag == 0);
    s_info = st->info;
    s_r00 = st->r00;
    s_fro2 = st->fro2;
    s_off = st->off;
    s_ncur = st->ncur;
  }
  // pivot partials
  AmaxVal best = amax_none();
  if (tid < a.namax) {
    best.v = pp0.v;
    best.s2 = pp0.s2;
    best.pos = pp0.pos;
    best.key = pp0.key;
  }
  if (a.namax > kThreads) {  // uniform; more than one partial per thread
    for (int q = tid + kThreads; q < a.namax; q += kThreads) {
      const AmaxPart pp = a.amax[q];
      AmaxVal c;
      c.v = pp.v;
      c.s2 = pp.s2;
      c.pos = pp.pos;
      c.key = pp.key;
      best = amax_combine(best, c);
    }
  }
  best = block_amax(best, ascr);  // its barriers also publish the flags
  if (!s_go) return;
  const int64_t j = s_off + jj;
  const int64_t ncur = s_ncur;
  const int nchunk = (int)ceil_div(ncur, a.CW);
  const bool colok = l0 < ncur;
  const bool rowok = iw >= j && iw < r1;
  int p = best.pos;
  double vp = best.v;
  if (a.nopivot) {
    p = jj;
    vp = jj < ncur ? a.nu[jj] : 0.0;
  }
  bool stop = (j >= a.kcap) || (jj >= ncur) || (p < 0) || (s_info != 0);
  if (!stop && a.k_fixed == 0) {
    if (!(vp > 0.0)) {
      stop = true;
    } else if (a.rule == ID_RANK_PIVOT_REL) {
      if (j > 0 && vp <= a.rel_tol * s_r00) stop = true;
    } else {
      const double fro2 = j == 0 ? best.s2 : s_fro2;
      if (sqrt(best.s2) <= a.rel_tol * sqrt(fro2)) stop = true;
    }
  }
  if (stop) {
    if (bid == 0 && tid == 0) {
      st->done = 1;
      st->k = j;
      st->end_flag = 1;
    }
    return;
  }
  if (bid == 0 && tid == 0) {
    a.pivpos[jj] = p;
    a.pvflag[p] = 1;
    const int q = a.colid[p];
    a.pivid[j] = q;
    const int pa = a.posof[q];
    const int other = a.permw[j];
    a.permw[pa] = other;
    a.posof[other] = pa;
    a.permw[j] = q;
    a.posof[q] = (int)j;
    // the only live column whose key changed (q is pivoted)
    st->swap_other = other;
    st->swap_key = pa;
    st->jb = jj + 1;
    if (j == 0) st->fro2 = best.s2;
  }
  if (r1 <= j || chunk >= nchunk) {
    // below the step's row or past the live columns: the bound-sized grid
    // leaves zero partials wherever the finalization sums
    if (r1 <= j) {
      if (rg == 0 && l0 < a.ncur)
#pragma unroll
        for (int e = 0; e < VEC; ++e) a.zpart[tile * a.ldf + l0 + e] = 0.0;
      if (tid < jj && chunk < nchunk && tid % nchunk == chunk)
        a.auxpart[tile * kNbMax + tid] = 0.0;
      if (chunk == 0 && tid == 0) a.nrm2part[tile] = 0.0;
    }
    return;
  }

  // keep the reflector entries of the step's rows only: other rows of the
  // tile and columns c >= jj hold stale workspace data (possibly not even
  // finite): drop them, never scale by 0
#pragma unroll
  for (int q = 0; q < SLOTS; ++q)
    if (!(rowok && gi + G * q < jj)) vr[q] = (S)0;

  // ---- round trip 2: F(c, p) and the pivot column itself, both loads issued
  // before either is used (unconditional, clamped; w below is masked by rowok)
  const double wp = (double)a.W[(iw < a.m ? iw : a.m - 1) * a.ldw + p];  // same on the G lanes
  const double fp = a.F[(int64_t)(tid % kNbMax) * a.ldf + p];
  const double vsp = a.vscale[tid % kNbMax];
  // the first kOverlap rows of the main loop, in flight with round trip 2
  // (issued after its loads, so waiting for those leaves these outstanding;
  // rows past the tile are loaded from r1 - 1 and not used)
  int64_t i1 = ib + (int64_t)kPrefetch * RG;
  if (i1 <= j) i1 += (j + 1 - i1 + RG - 1) / RG * RG;
  constexpr int kOverlap = overlap_rows<S, G>();
  VT x0[kOverlap];
  {
    const S* pb = a.W + (colok ? l0 : 0);
#pragma unroll
    for (int u = 0; u < kOverlap; ++u) {
      const int64_t r = i1 + (int64_t)u * RG;
      x0[u] = *(const VT*)(pb + (r < r1 ? r : r1 - 1) * a.ldw);
    }
  }
  if (tid < kNbMax) gsh[tid] = tid < jj ? vsp * fp : 0.0;
  __syncthreads();
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) part += (double)vr[q] * gsh[gi + G * q];
#pragma unroll
  for (int off = 1; off < G; off <<= 1) part += __shfl_xor(part, off, 64);
  // valid on all G lanes of the row; rows below the step (loaded from the
  // lower bound jlb on) and past the matrix contribute nothing
  const double w = rowok ? (a.rmode ? rnd(wp - part, a.rmode) : wp - part) : 0.0;
  const bool lead = chunk == 0;
  if (gi == 0 && rsub < a.Rt) {
    wsh[rsub] = iw == j ? 0.0 : w;  // row j holds alpha, kept apart
    if (rowok && lead) {
      a.V[(int64_t)jj * a.ldv + iw] = (S)w;
      if (iw == j) st->alpha = w;
    }
  }
  // row j of the panel's earlier reflectors, for the finalization (the
  // entries are masked to c < jj above)
  if (lead && iw == j) {
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) a.vrow[gi + G * q] = (double)vr[q];
  }
  // tile partials of sum_{i>j} V(i,c) w(i) for c = chunk, chunk + nchunk, ...
  {
    const double wz = (rowok && iw > j) ? w : 0.0;
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
      const int c0 = G * q;  // the slot's columns are c0 .. c0 + G - 1
      if (c0 < jj) {
        double z = (double)vr[q] * wz;
#pragma unroll
        for (int off = G; off < 64; off <<= 1) z += __shfl_xor(z, off, 64);
        const int c = c0 + gi;
        if (lane < G && c < jj && c % nchunk == chunk) zred[wv][c] = z;
      }
    }
  }
  double nn = (lead && rowok && iw > j && gi == 0) ? w * w : 0.0;
  if (lead) nn = block_sum(nn, dscr);
  __syncthreads();
  if (tid < jj && tid % nchunk == chunk)
    a.auxpart[tile * kNbMax + tid] = zred[0][tid] + zred[1][tid] + zred[2][tid] + zred[3][tid];
  if (lead && tid == 0) a.nrm2part[tile] = nn;

  // ---- the sweep: z(l) = sum_{i in tile, i > j} W(i, l) w(i)
  double acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc[e] = 0.0;
  if (colok) {
    // only rows i > j: rows from the bound jlb up to j may hold stale data
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int64_t i = ib + (int64_t)u * RG;
      if (i > j && i < r1) {
        const double w0 = wsh[i - r0];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += (double)pf[u][e] * w0;
      }
    }
    // the rows loaded with round trip 2
#pragma unroll
    for (int u = 0; u < kOverlap; ++u) {
      const int64_t r = i1 + (int64_t)u * RG;
      if (r < r1) {
        const double w0 = wsh[r - r0];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += (double)x0[u][e] * w0;
      }
    }
    int64_t i = i1 + (int64_t)kOverlap * RG;
    // U independent row loads in flight per thread: the loop is bound by
    // memory latency times the number of its iterations
    for (; i + (U - 1) * RG < r1; i += U * RG) {
      VT x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = *(const VT*)(base + (i + u * RG) * a.ldw);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double wu = wsh[i + u * RG - r0];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += (double)x[u][e] * wu;
      }
    }
    for (; i < r1; i += RG) {
      const VT x0 = *(const VT*)(base + i * a.ldw);
      const double w0 = wsh[i - r0];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += (double)x0[e] * w0;
    }
  }
  if (RG > 1) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[tid * VEC + e] = acc[e];
    __syncthreads();
    if (rg == 0) {
      for (int gq = 1; gq < RG; ++gq)
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += red[(gq * TPR + cv) * VEC + e];
    }
  }
  if (rg == 0 && colok) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) a.zpart[tile * a.ldf + l0 + e] = acc[e];
  }
  // the tile holding row j passes that row on to the finalization (these
  // blocks stream the fewest rows; the load is left to their end)
  if (r0 <= j && rg == 0 && colok) {
    const VT xr = *(const VT*)(base + j * a.ldw);
#pragma unroll
    for (int e = 0; e < VEC; ++e) a.wrow[l0 + e] = (double)xr[e];
  }
}

template <typename S, int G, int U>
__global__ __launch_bounds__(kThreads) void k_sweep(StepArgs<S> a) {
  sweep_block<S, G, U>(a, blockIdx.x, gridDim.x);
}

// Tall inputs (more row tiles than one round trip of the finalization
// covers): sums the per-tile partials of the step in groups of kFold tiles,
// in tile order, so that the finalization reads ceil(ntile / kFold) of them.
// Thread = (column or reflector-product slot, group); its kFold loads are
// issued as one group (unconditional, clamped; tiles past the end weighted 0).
// Grid: ceil((ncur + kNbMax + 1) nfold / kThreads).
template <typename S>
__global__ __launch_bounds__(kThreads) void k_fold(StepArgs<S> a, double* __restrict__ zf,
                                                   double* __restrict__ af,
                                                   double* __restrict__ nf, int64_t nfold) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t ncol = a.ncur, slots = ncol + kNbMax + 1;
  if (e >= slots * nfold) return;
  const int64_t gidx = e / slots, sl = e % slots;
  const int64_t tend = a.t0 + a.ntile;
  const int64_t tb = a.t0 + gidx * kFold;
  double x[kFold], w[kFold];
#pragma unroll
  for (int u = 0; u < kFold; ++u) {
    const int64_t t = tb + u;
    const int64_t tc = t < tend ? t : tend - 1;
    w[u] = t < tend ? 1.0 : 0.0;
    if (sl < ncol)
      x[u] = a.zpart[tc * a.ldf + sl];
    else if (sl < ncol + kNbMax)
      x[u] = a.auxpart[tc * kNbMax + (sl - ncol)];
    else
      x[u] = a.nrm2part[tc];
  }
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kFold; ++u) t += x[u] * w[u];
  if (sl < ncol)
    zf[gidx * a.ldf + sl] = t;
  else if (sl < ncol + kNbMax)
    af[gidx * kNbMax + (sl - ncol)] = t;
  else
    nf[gidx] = t;
}

// One pivot step, part 2.  Grid: ceil(ncur / FC) blocks of FC columns x
// 256 / FC tile lanes (FC = 16 for one matrix, 32 in lock-step launches).
// Finishes the reflector (dlarfg conventions), forms the new
// column of F and the new row of R, downdates the column norms (with the
// cancellation test that ends the panel), and emits pivot partials.
// Every load is issued before the first barrier (the step's row of W and of
// the reflectors and the swap-order keys come from the sweep and the norm
// reduction, not from rows that depend on the step), so the kernel costs one
// memory round trip.
// Returns, in thread 0, the largest |F| entry the block formed (for the FP16
// operand scaling of the panel update; the caller folds it into the state),
// or -1 when the step did not run.
template <typename S, int RM, int FC = kFC>
__device__ __forceinline__ float finalize_block(const StepArgs<S>& a, const int bid) {
  constexpr int FL = kThreads / FC;             // tile lanes per column
  constexpr int FZ = (192 + FL - 1) / FL;      // column partials per lane and round trip
  __shared__ double red[FL][FC + 1];
  __shared__ double ared[8][kNbMax + 1];
  __shared__ double Fsh[kNbMax][FC + 1];
  __shared__ double aux[kNbMax];
  __shared__ double vj[kNbMax];
  __shared__ double dscr[4];
  __shared__ int s_go;
  __shared__ double s_alpha;
  __shared__ int64_t s_off, s_ncur;
  __shared__ int s_swo, s_swk;
  FactorState* st = a.st;
  const int tid = threadIdx.x, cl = tid % FC, tl = tid / FC;
  const int jj = a.jj;
  const int64_t tend = a.t0 + a.ntile;
  const int64_t l = (int64_t)bid * FC + cl;
  const bool lb = l < a.ncur;  // within the host's column bound

  // Round trip 1: loads that depend neither on each other nor on the exact
  // step (partials below the step's row were zeroed by the sweep).  They are
  // unconditional, from clamped in-bounds addresses, and masked after the
  // barrier: a conditional load (or a select next to its load, which the
  // compiler turns into one) makes it wait for every earlier load first.
  const int64_t lc = lb ? l : 0;
  double nl = a.nu[lc], nlo = a.nuo[lc];
  int pv = a.pvflag[lc], id = a.colid[lc];
  // the step's row and swap-order key, left by the sweep
  double wj = a.wrow[lc];
  int key = a.keypos[lc];
  double vjr = a.vrow[tid % kNbMax];
  double fv[kNbMax / FL];
#pragma unroll
  for (int q = 0; q < kNbMax / FL; ++q) fv[q] = a.F[(int64_t)(tl + FL * q) * a.ldf + lc];
  double vsc = a.vscale[tid % kNbMax];
  // partial sums over the row tiles [t0, tend), one batch of loads per round
  // trip (one batch covers up to FZ FL = kFinA 8 = 192 tiles); tiles past
  // tend read the zero row "tguard" of the partial arrays (no weights: they
  // would take a register per load)
  const int ca = tid % kNbMax, sla = tid / kNbMax;
  const int64_t caa = ca < jj ? ca : 0;
  double sz = 0.0, sa = 0.0, sn = 0.0;
  {
    const int64_t nbz = ceil_div(a.ntile, (int64_t)FZ * FL);
    const int64_t nba = ceil_div(a.ntile, (int64_t)kFinA * 8);
    const int64_t nbn = ceil_div(a.ntile, (int64_t)kThreads);
    const int64_t nbat = nbz > nba ? (nbz > nbn ? nbz : nbn) : (nba > nbn ? nba : nbn);
    for (int64_t b = 0; b < nbat; ++b) {
      double xz[FZ], xa[kFinA];
#pragma unroll
      for (int u = 0; u < FZ; ++u) {
        const int64_t t = a.t0 + tl + FL * (b * FZ + u);
        xz[u] = a.zpart[(t < tend ? t : a.tguard) * a.ldf + lc];
      }
#pragma unroll
      for (int u = 0; u < kFinA; ++u) {
        const int64_t t = a.t0 + sla + 8 * (b * kFinA + u);
        xa[u] = a.auxpart[(t < tend ? t : a.tguard) * kNbMax + caa];
      }
      const int64_t tn = a.t0 + tid + (int64_t)kThreads * b;
      const double xn = a.nrm2part[tn < tend ? tn : a.tguard];
      // keep the scheduler from interleaving the sums with the loads (it
      // would wait for all loads issued so far, several times per batch)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < FZ; ++u) sz += xz[u];
#pragma unroll
      for (int u = 0; u < kFinA; ++u) sa += xa[u];
      sn += xn;
    }
  }
  if (tid == 0) {
    s_go = (st->jb == jj + 1);
    s_alpha = st->alpha;
    s_off = st->off;
    s_ncur = st->ncur;
    s_swo = st->swap_other;
    s_swk = st->swap_key;
  }
#pragma unroll
  for (int q = 0; q < kNbMax / FL; ++q)  // rows >= jj hold stale workspace data: zeroed
    Fsh[tl + FL * q][cl] = tl + FL * q < jj ? fv[q] : 0.0;
  ared[sla][ca] = sa;  // columns >= jj unused
  red[tl][cl] = sz;    // positions >= ncur unused

  const double xnorm2 = block_sum(sn, dscr);  // also publishes the LDS writes above
  if (!s_go) return -1.0f;
  if (!(tl == 0 && lb)) {
    nl = 0.0;
    nlo = 1.0;
    pv = 1;
    id = 0;
  }
  if (tid >= jj) vsc = 0.0;
  const int64_t j = s_off + jj;
  const bool lv = l < s_ncur;
  // this step's swap moved one live column in the swap order
  if (tl == 0 && lv && id == s_swo) {
    key = s_swk;
    a.keypos[l] = key;
  }
  if (!(tl == 0 && lv)) {
    wj = 0.0;
    key = 0;
  }
  if (tid >= jj) vjr = 0.0;
  const double alpha = s_alpha;
  double beta, tau, scale;
  if (xnorm2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scale = 0.0;
  } else {
    const double h = hypot(alpha, sqrt(xnorm2));
    beta = rndc<RM>(alpha >= 0.0 ? -h : h);
    tau = rndc<RM>((beta - alpha) / beta);
    scale = rndc<RM>(1.0 / (alpha - beta));
  }
  if (tid < kNbMax) {  // zero past jj (the partials there may be stale, even NaN)
    double z = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) z += ared[q][tid];
    const double vjc = vsc * vjr;
    vj[tid] = tid < jj ? vjc : 0.0;
    aux[tid] = tid < jj ? vjc + vsc * scale * z : 0.0;
  }
  __syncthreads();

  AmaxVal cand = amax_none();
  float fabsmax = 0.0f;
  bool flag = false;
  if (tl == 0 && lv) {
    double zt = 0.0;
#pragma unroll
    for (int q = 0; q < FL; ++q) zt += red[q][cl];
    const double y = wj + scale * zt;
    double s1 = 0.0, s2 = 0.0;
    // all kNbMax slots (zero past jj): the unrolled loop issues its LDS
    // reads together instead of one dependent read per reflector
#pragma unroll
    for (int c = 0; c < kNbMax; ++c) {
      const double fc = Fsh[c][cl];
      s1 += fc * aux[c];
      s2 += vj[c] * fc;
    }
    const double f = rndc<RM>(tau * (y - s1));
    a.F[(int64_t)jj * a.ldf + l] = f;
    if (!pv) {
      const double r = rndc<RM>(wj - s2 - f);
      a.rorig[(int64_t)id * a.kcap + j] = r;
      if (nl != 0.0) {
        double t = fabs(r) / nl;
        t = (1.0 + t) * (1.0 - t);
        if (t < 0.0) t = 0.0;
        const double ratio = nl / nlo;
        if (t * ratio * ratio <= a.tol3z) {
          flag = true;
        } else {
          nl = rndc<RM>(nl * sqrt(t));
          a.nu[l] = nl;
        }
      }
      cand.v = nl;
      cand.s2 = nl * nl;
      cand.pos = (int)l;
      cand.key = key;
      fabsmax = (float)fabs(f);
    }
  }
  if (flag) st->end_flag = 1;
  // the pivot candidates and the largest |F| entry (for the FP16 operand
  // scaling) live in lanes 0 .. FC - 1 of the first wave (tl == 0): a
  // reduction over those lanes, no barrier (the other lanes hold no
  // candidate, so this is the block-wide result, bit for bit)
  float fm = fabsmax;
  if (tid < 64) {
#pragma unroll
    for (int off = FC / 2; off > 0; off >>= 1) {
      fm = fmaxf(fm, __shfl_xor(fm, off, 64));
      AmaxVal b;
      b.v = __shfl_xor(cand.v, off, 64);
      b.s2 = __shfl_xor(cand.s2, off, 64);
      b.pos = __shfl_xor(cand.pos, off, 64);
      b.key = __shfl_xor(cand.key, off, 64);
      cand = amax_combine(cand, b);
    }
  }
  if (tid == 0) {
    AmaxPart o;
    o.v = cand.v;
    o.s2 = cand.s2;
    o.pos = cand.pos;
    o.key = cand.key;
    a.amax[bid] = o;
  }
  if (bid == 0 && tid == 0) {
    a.tau[j] = tau;
    a.vscale[jj] = scale;
    const int p = a.pivpos[jj];
    a.rorig[(int64_t)a.colid[p] * a.kcap + j] = beta;
    if (j == 0) st->r00 = fabs(beta);
    if (jj + 1 >= a.nb) st->end_flag = 1;
    if (j + 1 >= a.kcap) {
      st->done = 1;
      st->k = j + 1;
      st->end_flag = 1;
    }
  }
  return fm;
}

template <typename S, int RM, int FC>
__global__ __launch_bounds__(kThreads) void k_finalize(StepArgs<S> a) {
  const float fm = finalize_block<S, RM, FC>(a, blockIdx.x);
  // (one word for every block: its read-modify-writes queue up and the
  // launch ends only when they are done, so it is updated only when used)
  if (a.want_fmax && threadIdx.x == 0 && fm >= 0.0f)
    atomicMax(&a.st->fmax_bits, __float_as_uint(fm));
}

template <typename S>
struct GemmArgs {
  const S* W;
  S* Wn;
  int64_t ldw, m, ncur;
  const S* V;
  int64_t ldv;
  const double* F;
  int64_t ldf;
  const double* vscale;
  FactorState* st;
  const int* pivpos;
  const int* colid;
  int* colid_n;
  double* colpart;
  int64_t off, tg0;
  int64_t gx, gy;  // column blocks and row tiles of the grid
};

// End of a panel: Wn(i, newpos(l)) = W(i, l) - sum_c V(i, c) F(c, l) for rows
// i >= off + jb, on the matrix cores (FP64 MFMA, or FP16/BF16 MFMA with FP32
// accumulation), skipping the pivoted positions (compaction), and the FP64
// sums of squares of every refreshed column per row tile.
// Block: 64 positions x kRowTileG rows, processed in 64-row slices.  Per
// slice each thread first issues its 16 loads of the W tile (coalesced rows),
// the waves form the 64 x 64 product as 16x16 MFMA blocks (positions along
// the MFMA rows) and park it in LDS, then each thread writes its column of the
// refreshed tile to the compacted position.
template <typename S, int OP, int RM>
__device__ __forceinline__ void panel_gemm_block(const GemmArgs<S>& a, const uint32_t bid,
                                                 const uint32_t nblk) {
  typedef typename std::conditional<OP == OP_F64, double, float>::type AccT;
  __shared__ int spiv[kNbMax];
  __shared__ double svs[kNbMax];
  __shared__ int cidx[64];
  __shared__ AccT accs[64][64 + 1];
  __shared__ double ssq[4][64];
  // A operands: FP64 as 4 position blocks x 8 k-steps x 64 lanes; FP16/BF16 as
  // 8-element vectors (BF16x3: leading parts, then the remainders)
  constexpr int kOpA = OP == OP_F64 ? 4 * 8 * 64 : 1;
  constexpr int kOpH = OP == OP_F16 ? 256 : 1;
  constexpr int kOpB = (OP == OP_BF16 || OP == OP_BF16X3) ? 512 : 1;
  constexpr int kOpF = OP == OP_F32 ? 4 * 8 * 64 : 1;
  __shared__ float opaf[kOpF];
  __shared__ double opa64[kOpA];
  __shared__ f16x8 opah[kOpH];
  __shared__ bf16x8 opab[kOpB];
  __shared__ int s_go, s_jb;
  __shared__ uint32_t s_fmax;
  __shared__ int64_t s_off, s_ncur;
  FactorState* st = a.st;
  const int tid = threadIdx.x;
  // XCD-aware block order (hardware block b runs on XCD b % 8): each XCD
  // takes a contiguous range of row tiles with all their column blocks, so a
  // row tile's reflector rows are read from HBM once, not once per XCD.  The
  // indices are uniform and kept in scalar registers (the division is
  // expanded into vector instructions, which would move everything derived
  // from them into vector registers).
  const uint32_t per = nblk / 8u;
  const uint32_t vb = (bid % 8u) * per + bid / 8u;
  if (vb >= (uint32_t)(a.gx * a.gy)) return;
  const int64_t bx = __builtin_amdgcn_readfirstlane((int)(vb % (uint32_t)a.gx));
  const int64_t by = __builtin_amdgcn_readfirstlane((int)(vb / (uint32_t)a.gx));
  if (tid == 0) {
    s_go = (st->done == 0);
    s_jb = st->jb;
    s_fmax = st->fmax_bits;
    s_off = st->off;
    s_ncur = st->ncur;
  }
  if (tid < kNbMax) spiv[tid] = a.pivpos[tid];
  if (tid >= 64 && tid < 64 + kNbMax) svs[tid - 64] = a.vscale[tid - 64];
  __syncthreads();
  if (!s_go) return;
  if (tid == 0 && bx == 0 && by == 0) {  // refilled after
    st->vmax_bits = 0u;
    st->nabove = 0u;
  }
  const int jb = s_jb;
  const int64_t ncur = s_ncur;  // a.ncur is the host's bound that sized the grid
  const int64_t jend = s_off + jb;
  const int64_t l0 = bx * 64;
  const int64_t tg = a.tg0 + by;
  const int64_t rbase = tg * kRowTileG;
  const int64_t rbeg = rbase > jend ? rbase : jend;
  const int64_t rend = rbase + kRowTileG < a.m ? rbase + kRowTileG : a.m;

  if (tid < 64) {
    const int64_t l = l0 + tid;
    int before = 0;
    bool pv = false;
    for (int c = 0; c < jb; ++c) {
      before += spiv[c] < l;
      pv |= spiv[c] == l;
    }
    cidx[tid] = (l < ncur && !pv) ? (int)(l - before) : -1;
  }
  __syncthreads();

  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, li = lane & 15;
  const int cc = tid % 64, rq = tid / 64;  // write-out mapping: column cc, rows rq + 4q
  const int myout = cidx[cc];
  int sF = 0, sV = 0;
  if (OP == OP_F16 && RM != RM_F16) {
    const float fmax = __uint_as_float(s_fmax);
    int e = 0;
    if (fmax > 0.0f) frexpf(fmax, &e);
    sF = 15 - e;
    sV = 14;
  }
  const double fscl = ldexp(1.0, sF);
  const float vscl = ldexpf(1.0f, sV);
  const double descale = ldexp(1.0, -(sF + sV));

  // A operands (F^T rows = positions) staged once in LDS, in the lane order of
  // the matrix-core instruction: 256 threads = 4 position blocks x 64 lanes
  {
    const int lb = tid >> 6;
    // (all eight loads issued before any is used: unconditional, from a
    // clamped position; stale rows c >= jb and positions past ncur are
    // dropped by selects on the computed values)
    if (OP == OP_F64) {
      const int64_t pos = l0 + 16 * lb + (4 * (li % 4) + li / 4);
      const int64_t posc = pos < ncur ? pos : 0;
      double fv[8];
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) fv[s8] = a.F[(int64_t)(4 * s8 + g) * a.ldf + posc];
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        const int c = 4 * s8 + g;
        opa64[(lb * 8 + s8) * 64 + lane] = (c < jb && pos < ncur) ? fv[s8] * 1.0 : 0.0;
      }
    } else if (OP == OP_F32) {
      // FP32 16x16x4: step e uses k index c = 8 g + e of lane group g
      const int64_t pos = l0 + 16 * lb + li;
      const int64_t posc = pos < ncur ? pos : 0;
      double fv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) fv[e] = a.F[(int64_t)(8 * g + e) * a.ldf + posc];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 8 * g + e;
        opaf[(lb * 8 + e) * 64 + lane] = (c < jb && pos < ncur) ? (float)fv[e] : 0.0f;
      }
    } else {
      const int64_t pos = l0 + 16 * lb + li;
      const int64_t posc = pos < ncur ? pos : 0;
      double fv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) fv[e] = a.F[(int64_t)(8 * g + e) * a.ldf + posc];
      f16x8 xh;
      bf16x8 xb, xl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 8 * g + e;
        const float x = (c < jb && pos < ncur) ? (float)(fv[e] * fscl) : 0.0f;
        xh[e] = (_Float16)x;
        const __bf16 h = (__bf16)x;
        xb[e] = h;
        xl[e] = (__bf16)(x - (float)h);
      }
      if (OP == OP_F16) {
        opah[tid] = xh;
      } else {
        opab[tid] = xb;
        opab[256 + tid] = xl;
      }
    }
  }
  __syncthreads();

  // The W loads of SL 64-row slices are issued together (64 fp32 or 32 fp64
  // values per thread in flight), then each slice's product is formed on the
  // matrix cores, parked in LDS and written out compacted.
  constexpr int SL = sizeof(S) == 4 ? 4 : 1;
  double ss = 0.0;
  for (int sb0 = 0; sb0 < kRowTileG / 64; sb0 += SL) {
    S wt[SL][16];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int64_t rs = rbase + 64 * (sb0 + sl);
      const S* rowb = a.W + rs * a.ldw + l0;  // uniform base of the slice
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t r = rs + rq + 4 * q;
        const uint32_t o = (uint32_t)((rq + 4 * q) * a.ldw + cc);
        wt[sl][q] = (myout >= 0 && r >= rbeg && r < rend) ? rowb[o] : (S)0;
      }
    }
    // the reflector entries of the slices' rows, with the W loads (each an
    // unconditional load from a clamped row; selects on the computed values
    // drop rows outside [rbeg, rend) and stale columns c >= jb)
    S vv[SL][8];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int64_t row = rbase + 64 * (sb0 + sl) + 16 * wv + li;
      const int64_t rowc = row < rend ? row : rend - 1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = OP == OP_F64 ? 4 * e + g : 8 * g + e;
        vv[sl][e] = a.V[(int64_t)c * a.ldv + rowc];
      }
    }
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int64_t rs = rbase + 64 * (sb0 + sl);
      if (rs + 64 <= rbeg || rs >= rend) continue;  // uniform across the block
      const int64_t row = rs + 16 * wv + li;
      const bool rowok = row >= rbeg && row < rend;
      if (OP == OP_F64) {
        double b64[8];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
          const int c = 4 * s8 + g;
          b64[s8] = (c < jb && rowok) ? (double)vv[sl][s8] * svs[c] : 0.0;
        }
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s8 = 0; s8 < 8; ++s8)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opa64[(lb * 8 + s8) * 64 + lane], b64[s8],
                                                       acc, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) accs[16 * wv + li][16 * lb + 4 * g + r] = (AccT)acc[r];
        }
      } else if (OP == OP_F32) {
        float bf[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = 8 * g + e;
          bf[e] = (c < jb && rowok) ? (float)((double)vv[sl][e] * svs[c]) : 0.0f;
        }
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int e = 0; e < 8; ++e)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(opaf[(lb * 8 + e) * 64 + lane], bf[e], acc,
                                                       0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) accs[16 * wv + li][16 * lb + 4 * g + r] = (AccT)acc[r];
        }
      } else {
        f16x8 bh;
        bf16x8 bb, bbl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = 8 * g + e;
          const float x =
              (c < jb && rowok) ? (float)((double)vv[sl][e] * svs[c]) * vscl : 0.0f;
          if (OP == OP_F16) {
            bh[e] = (_Float16)x;
          } else {
            const __bf16 h = (__bf16)x;
            bb[e] = h;
            if (OP == OP_BF16X3) bbl[e] = (__bf16)(x - (float)h);
          }
        }
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
          if (OP == OP_F16) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(opah[lb * 64 + lane], bh, acc, 0, 0, 0);
          } else if (OP == OP_BF16) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opab[lb * 64 + lane], bb, acc, 0, 0, 0);
          } else {
            const bf16x8 ahi = opab[lb * 64 + lane], alo = opab[256 + lb * 64 + lane];
            // small terms first, then the leading product
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bb, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bbl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bb, acc, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) accs[16 * wv + li][16 * lb + 4 * g + r] = (AccT)acc[r];
        }
      }
      __syncthreads();
      // refreshed column cc of the slice, written to its compacted position
      if (myout >= 0) {
        S* outb = a.Wn + rs * a.ldw;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int rr = rq + 4 * q;
          const int64_t r = rs + rr;
          if (r >= rbeg && r < rend) {
            const double vd = (double)wt[sl][q] - (double)accs[rr][cc] * descale;
            const S v = (S)rndc<RM>(vd);
            outb[(uint32_t)(rr * a.ldw + myout)] = v;
            ss += (double)v * (double)v;
          }
        }
      }
      __syncthreads();
    }
  }
  ssq[rq][cc] = ss;
  __syncthreads();
  if (tid < 64 && cidx[tid] >= 0) {
    a.colpart[tg * a.ldf + cidx[tid]] = ssq[0][tid] + ssq[1][tid] + ssq[2][tid] + ssq[3][tid];
    if (by == 0) a.colid_n[cidx[tid]] = a.colid[l0 + tid];
  }
}

template <typename S, int OP, int RM>
__global__ __launch_bounds__(kThreads) void k_panel_gemm(GemmArgs<S> a) {
  panel_gemm_block<S, OP, RM>(a, blockIdx.x, gridDim.x);
}

// perm (swap order) and R gathered into pivot order: R(i, c) = Rorig(i, perm[c])
// for i < k, zero below the diagonal of the first k columns.
struct FinishArgs {
  const int* permw;
  int32_t* perm_out;
  const double* rorig;
  int64_t kcap, n, k;
  double* R;
  int64_t ldr;
};

__device__ __forceinline__ void finish_block(const FinishArgs& a, const int64_t c,
                                             const int64_t by) {
  const int64_t i = by * kThreads + threadIdx.x;
  if (c >= a.n) return;
  const int id = a.permw[c];
  if (by == 0 && threadIdx.x == 0) a.perm_out[c] = id;
  if (i < a.k) a.R[c * a.ldr + i] = (c >= a.k || i <= c) ? a.rorig[(int64_t)id * a.kcap + i] : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_finish(FinishArgs a) {
  finish_block(a, blockIdx.x, blockIdx.y);
}

__global__ void k_iota(int32_t* perm, int64_t n) {
  const int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (l < n) perm[l] = (int32_t)l;
}

// ----------------------------------------------------------------- host driver

static int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  if (!s || !*s) return dflt;
  return std::atoi(s);
}

// ---- argument blocks of one factorization's kernels, from its plan and
// workspace (shared by the single-matrix driver and the lock-step batches)

static InitArgs make_init_args(const FactorPlan& pl, char* wb) {
  InitArgs a;
  a.st = (FactorState*)(wb + pl.off_state);
  a.colid0 = (int*)(wb + pl.off_colid0);
  a.pvflag = (int*)(wb + pl.off_pvflag);
  a.permw = (int*)(wb + pl.off_permw);
  a.posof = (int*)(wb + pl.off_posof);
  a.n = pl.n;
  a.ldf = pl.ldf;
  a.zrow_z = (double*)(wb + pl.off_zpart) + pl.ntile_s_max * pl.ldf;
  a.zrow_a = (double*)(wb + pl.off_auxpart) + pl.ntile_s_max * kNbMax;
  a.zrow_n = (double*)(wb + pl.off_nrm2part) + pl.ntile_s_max;
  a.frow_z = (double*)(wb + pl.off_zfold) + pl.nfold_max * pl.ldf;
  a.frow_a = (double*)(wb + pl.off_afold) + pl.nfold_max * kNbMax;
  a.frow_n = (double*)(wb + pl.off_nfold) + pl.nfold_max;
  return a;
}
static int64_t init_blocks(const FactorPlan& pl) {
  return ceil_div(pl.ldf > pl.n ? pl.ldf : pl.n, kThreads);
}

template <typename TA, typename S>
static IngestArgs<TA, S> make_ingest_args(const FactorPlan& pl, char* wb, const TA* A, int64_t lda,
                                          int rmode) {
  IngestArgs<TA, S> a;
  a.A = A;
  a.lda = lda;
  a.m = pl.m;
  a.n = pl.n;
  a.W = (S*)(wb + pl.off_w0);
  a.ldw = pl.ldw;
  a.colpart = (double*)(wb + pl.off_colpart);
  a.ldf = pl.ldf;
  a.st = (FactorState*)(wb + pl.off_state);
  a.rmode = rmode;
  return a;
}

// The norm reduction after the ingest (buf 0, all n columns) or at the end of
// a panel that wrote buffer buf (row tile groups from tg0, at most ncols_ub
// live columns, the count of columns above rel_tol |R_00| when rel_tol >= 0,
// the state published to hs with tag seq).
static ColArgs make_col_args(const FactorPlan& pl, char* wb, int buf, int64_t tg0,
                             int64_t ncols_ub, int subtract_jb, double rel_tol, int rmode,
                             FactorHostSlot* hs, int64_t seq) {
  ColArgs c;
  c.colpart = (double*)(wb + pl.off_colpart);
  c.ldf = pl.ldf;
  c.tg0 = tg0;
  c.tg1 = ceil_div(pl.m, kRowTileG);
  c.ncols_base = ncols_ub;
  c.subtract_jb = subtract_jb;
  c.nu = (double*)(wb + pl.off_nu);
  c.nuo = (double*)(wb + pl.off_nuo);
  c.amax = (AmaxPart*)(wb + pl.off_amax);
  c.colid = (int*)(wb + (buf ? pl.off_colid1 : pl.off_colid0));
  c.posof = (int*)(wb + pl.off_posof);
  c.pvflag = (int*)(wb + pl.off_pvflag);
  c.keypos = (int*)(wb + pl.off_keypos);
  c.st = (FactorState*)(wb + pl.off_state);
  c.rel_tol = rel_tol;
  c.rmode = rmode;
  c.hs = hs;
  c.seq = seq;
  return c;
}

// The fields of a pivot step's arguments that stay fixed over the call.
template <typename S>
static StepArgs<S> make_step_args(const FactorPlan& pl, char* wb, const id_opts* o, int rmode,
                                  int want_fmax) {
  StepArgs<S> a;
  std::memset(&a, 0, sizeof(a));
  a.ldw = pl.ldw;
  a.m = pl.m;
  a.n = pl.n;
  a.V = (S*)(wb + pl.off_v);
  a.ldv = pl.ldv;
  a.F = (double*)(wb + pl.off_f);
  a.ldf = pl.ldf;
  a.vscale = (double*)(wb + pl.off_vscale);
  a.tau = (double*)(wb + pl.off_tau);
  a.st = (FactorState*)(wb + pl.off_state);
  a.amax = (AmaxPart*)(wb + pl.off_amax);
  a.pvflag = (int*)(wb + pl.off_pvflag);
  a.pivpos = (int*)(wb + pl.off_pivpos);
  a.pivid = (int*)(wb + pl.off_pivid);
  a.permw = (int*)(wb + pl.off_permw);
  a.posof = (int*)(wb + pl.off_posof);
  a.zpart = (double*)(wb + pl.off_zpart);
  a.auxpart = (double*)(wb + pl.off_auxpart);
  a.nrm2part = (double*)(wb + pl.off_nrm2part);
  a.nu = (double*)(wb + pl.off_nu);
  a.nuo = (double*)(wb + pl.off_nuo);
  a.rorig = (double*)(wb + pl.off_rorig);
  a.wrow = (double*)(wb + pl.off_wrow);
  a.vrow = (double*)(wb + pl.off_vrow);
  a.keypos = (int*)(wb + pl.off_keypos);
  a.tguard = pl.ntile_s_max;
  a.kcap = pl.kcap;
  a.k_fixed = o->k_fixed;
  a.rel_tol = o->rel_tol;
  a.tol3z = std::sqrt(pl.wbytes == 8 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
  a.rule = o->rank_rule;
  a.nopivot = (o->flags & ID_FLAG_NO_PIVOT) ? 1 : 0;
  a.nb = pl.nb;
  a.want_fmax = want_fmax;
  a.rmode = rmode;
  return a;
}

// The panel update of buffer cur into cur ^ 1, grid sized from the offset
// lower bound off_lb.
template <typename S>
static GemmArgs<S> make_gemm_args(const FactorPlan& pl, char* wb, int cur, int64_t off_lb) {
  GemmArgs<S> g;
  S* W[2] = {(S*)(wb + pl.off_w0), (S*)(wb + pl.off_w1)};
  int* colid[2] = {(int*)(wb + pl.off_colid0), (int*)(wb + pl.off_colid1)};
  const int64_t ncur_ub = pl.n - off_lb;
  g.W = W[cur];
  g.Wn = W[cur ^ 1];
  g.ldw = pl.ldw;
  g.m = pl.m;
  g.ncur = ncur_ub;
  g.V = (S*)(wb + pl.off_v);
  g.ldv = pl.ldv;
  g.F = (double*)(wb + pl.off_f);
  g.ldf = pl.ldf;
  g.vscale = (double*)(wb + pl.off_vscale);
  g.st = (FactorState*)(wb + pl.off_state);
  g.pivpos = (int*)(wb + pl.off_pivpos);
  g.colid = colid[cur];
  g.colid_n = colid[cur ^ 1];
  g.colpart = (double*)(wb + pl.off_colpart);
  g.off = off_lb;
  g.tg0 = off_lb / kRowTileG;
  g.gx = ceil_div(ncur_ub, 64);
  g.gy = ceil_div(pl.m, kRowTileG) - g.tg0;
  return g;
}

static FinishArgs make_finish_args(const FactorPlan& pl, char* wb, int32_t* perm, double* R,
                                   int64_t ldr, int64_t k) {
  FinishArgs f;
  f.permw = (int*)(wb + pl.off_permw);
  f.perm_out = perm;
  f.rorig = (double*)(wb + pl.off_rorig);
  f.kcap = pl.kcap;
  f.n = pl.n;
  f.k = k;
  f.R = R;
  f.ldr = ldr;
  return f;
}


struct SweepShape {
  int Rt, CW;
};

static SweepShape choose_sweep_shape(int64_t rows, int64_t ncur, int wbytes) {
  SweepShape sh;
  const int vec = 16 / wbytes;
  const int cw_max = kThreads * vec;  // one row group
  int cw = env_int("MPID_SWEEP_CW", wbytes == 4 ? 512 : 256);
  if (cw < 64 * vec) cw = 64 * vec;
  if (cw > cw_max) cw = cw_max;
  // round to a power of two number of lanes per row
  int tpr = cw / vec, t = 1;
  while (t * 2 <= tpr) t *= 2;
  sh.CW = t * vec;
  const int64_t nchunk = ceil_div(ncur, sh.CW);
  const int target = env_int("MPID_SWEEP_BLOCKS", 1024);
  int rt = env_int("MPID_SWEEP_RT", 0);
  if (rt <= 0) {
    rt = kRtMin;
    while (rt < kRtMax && ceil_div(rows, rt) * nchunk > target) rt *= 2;
  }
  // the sweep kernel supports row tiles of 64, 128 or 256 rows
  sh.Rt = rt <= 64 ? 64 : (rt <= 128 ? 128 : 256);
  return sh;
}

// ---- host resources of the calling thread

// Pinned host memory, grown on demand.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
static int pinned_reserve(PinnedBuf& b, size_t bytes, unsigned flags) {
  if (b.bytes >= bytes) return ID_OK;
  if (b.p) MPID_HIP(hipHostFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  MPID_HIP(hipHostMalloc(&b.p, bytes, flags));
  b.bytes = bytes;
  return ID_OK;
}

// What a thread's calls keep between calls -- pinned slots and staging
// buffers, events -- released when the thread ends (every call has
// synchronized its stream before returning, so nothing is in flight).
struct ThreadRes {
  PinnedBuf slot;                 // the single-matrix driver's two panel-end slots
  hipEvent_t pev[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> prof_events;  // ID_FLAG_PROFILE
  PinnedBuf stage[2], lslots[2];  // lock-step tables and panel-end states
  PinnedBuf probe;                // lock-step mid-panel end flags
  hipEvent_t ev_stage[2] = {nullptr, nullptr}, ev_slot[2] = {nullptr, nullptr};
  hipEvent_t ev_probe = nullptr;
  int64_t ncalls = 0;             // tags the panel-end states of this thread's calls
  ThreadRes() = default;
  ThreadRes(const ThreadRes&) = delete;
  ThreadRes& operator=(const ThreadRes&) = delete;
  ~ThreadRes() {
    for (PinnedBuf* b : {&slot, &stage[0], &stage[1], &lslots[0], &lslots[1], &probe})
      if (b->p) (void)hipHostFree(b->p);
    for (hipEvent_t e :
         {pev[0], pev[1], ev_stage[0], ev_stage[1], ev_slot[0], ev_slot[1], ev_probe})
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : prof_events)
      if (e) (void)hipEventDestroy(e);
  }
};
static ThreadRes& thread_res() {
  static thread_local ThreadRes r;
  return r;
}

// ---- opt-in per-kernel event timing (ID_FLAG_PROFILE)

static thread_local id_profile g_last_profile;

void last_profile(id_profile* out) { *out = g_last_profile; }

namespace {
enum { PK_SWEEP = 0, PK_FINALIZE, PK_GEMM, PK_OTHER };
struct ProfRec {
  int kind;
  int64_t j;  // pivot step (sweep/finalize) or panel end row (gemm)
  size_t e0;  // index of the start event; the end event is e0 + 1
};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t>* pool = nullptr;
  std::vector<ProfRec> recs;
  size_t used = 0;
  hipEvent_t ev(size_t i) {
    while (pool->size() <= i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool->push_back(e);
    }
    return (*pool)[i];
  }
  void begin(int kind, int64_t j, hipStream_t s) {
    if (!on) return;
    recs.push_back({kind, j, used});
    (void)hipEventRecord(ev(used), s);
    ++used;
  }
  void end(hipStream_t s) {
    if (!on) return;
    (void)hipEventRecord(ev(used), s);
    ++used;
  }
  // Launches a kernel; when profiling, its start and stop events are taken at
  // the kernel's own execution boundaries (hipExtLaunchKernelGGL).
  template <typename K, typename... Args>
  void launch(int kind, int64_t j, K kernel, dim3 grid, hipStream_t s, Args... args) {
    if (!on) {
      kernel<<<grid, kThreads, 0, s>>>(args...);
      return;
    }
    recs.push_back({kind, j, used});
    hipEvent_t e0 = ev(used), e1 = ev(used + 1);
    used += 2;
    hipExtLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, s, e0, e1, 0, args...);
  }
  float ms(const ProfRec& r) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, (*pool)[r.e0], (*pool)[r.e0 + 1]) != hipSuccess) return 0.0f;
    return t;
  }
};
}  // namespace

// Waits (after the panel's event completed) until the host slot holds the
// state tagged seq: the device's system-scope release makes it visible by
// then; a bounded wait turns anything else into an error.
static int await_slot(const FactorHostSlot* hs, int64_t seq) {
  for (long spin = 0; spin < (1L << 26); ++spin) {
    if (__atomic_load_n(&hs->seq, __ATOMIC_ACQUIRE) == seq) return ID_OK;
  }
  return ID_ERR_HIP;
}

template <typename TA, typename S, int OP, int RM>
static int factor_impl(const TA* A, int64_t lda, const FactorPlan& pl, const id_opts* o,
                       char* wb, int32_t* perm, double* R, int64_t ldr, int64_t* k_out,
                       int32_t* info, bool noalloc, hipStream_t s) {
  const int64_t m = pl.m, n = pl.n, kcap = pl.kcap;
  S* W[2] = {(S*)(wb + pl.off_w0), (S*)(wb + pl.off_w1)};
  double* zfold = (double*)(wb + pl.off_zfold);
  double* afold = (double*)(wb + pl.off_afold);
  double* nfoldb = (double*)(wb + pl.off_nfold);
  int* colid[2] = {(int*)(wb + pl.off_colid0), (int*)(wb + pl.off_colid1)};
  const int64_t ntg = ceil_div(m, kRowTileG);
  ThreadRes& tr = thread_res();
  Profiler prof;
  prof.on = (o->flags & ID_FLAG_PROFILE) != 0;
  prof.pool = &tr.prof_events;
  id_profile acc;
  std::memset(&acc, 0, sizeof(acc));
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
  if (prof.on) {
    ev_t0 = prof.ev(0);
    ev_t1 = prof.ev(1);
    prof.used = 2;
    MPID_HIP(hipEventRecord(ev_t0, s));
  }
  const double sbytes = (double)pl.wbytes;
  const int rmode = RM;
  MPID_LOG(1, "id_factor: m=%lld n=%lld dtype=%s prec=%d flags=%d kcap=%lld nb=%d k_fixed=%lld "
              "rel_tol=%g rule=%d workspace=%zu bytes%s",
           (long long)m, (long long)n, sizeof(TA) == 8 ? "f64" : "f32", o->prec, o->flags,
           (long long)kcap, pl.nb, (long long)o->k_fixed, o->rel_tol, o->rank_rule, pl.bytes,
           noalloc ? " (static scratch)" : "");
  prof.begin(PK_OTHER, 0, s);
  k_init<<<dim3((unsigned)init_blocks(pl)), kThreads, 0, s>>>(make_init_args(pl, wb));
  MPID_LAUNCH_CHECK();
  k_ingest<TA, S><<<dim3((unsigned)ceil_div(n, 64), (unsigned)ntg), kThreads, 0, s>>>(
      make_ingest_args<TA, S>(pl, wb, A, lda, rmode));
  MPID_LAUNCH_CHECK();
  int namax = (int)ceil_div(n, kFinCols);
  k_colreduce<<<dim3((unsigned)namax), kThreads, 0, s>>>(
      make_col_args(pl, wb, 0, 0, n, 0, -1.0, rmode, nullptr, 0));
  MPID_LAUNCH_CHECK();
  prof.end(s);

  StepArgs<S> a =
      make_step_args<S>(pl, wb, o, rmode, (OP == OP_F16 && rmode != RM_F16) ? 1 : 0);

  // Panels are enqueued one ahead of what the host knows: before panel P is
  // enqueued the host has read the state after panel P - 2, whose offset is a
  // lower bound for the panel's real offset (each panel advances it by its
  // data-dependent jb <= nb).  Grids are sized from these bounds and the
  // kernels take the exact offset and column count from the device state.
  // Every live panel compacts into the other buffer, so panel P works on
  // buffer P & 1.
  // The panel-end reduction writes the state after panel P into slot P & 1,
  // tagged with this call's number and P.  The slots are pinned host memory
  // (allocated on a thread's first call, read after the panel's event), or,
  // in an allocation-free call, two slots in the workspace that the host
  // copies into host memory of its own (the copy waits for the stream).
  FactorHostSlot mirror[2];
  FactorHostSlot* hslot = nullptr;
  hipEvent_t* pev = tr.pev;
  FactorHostSlot* dslot = (FactorHostSlot*)(wb + pl.off_slot);
  FactorHostSlot* kslot = dslot;  // the slots the kernels write
  if (!noalloc) {
    if (!tr.slot.p) {
      const int rs = pinned_reserve(tr.slot, 2 * sizeof(FactorHostSlot), hipHostMallocCoherent);
      if (rs) return rs;
      FactorHostSlot* h = (FactorHostSlot*)tr.slot.p;
      h[0].seq = h[1].seq = 0;
    }
    hslot = (FactorHostSlot*)tr.slot.p;
    for (int q = 0; q < 2; ++q)
      if (!pev[q]) MPID_HIP(hipEventCreateWithFlags(&pev[q], hipEventDisableTiming));
    kslot = hslot;
  }
  const int64_t seq0 = (++tr.ncalls) << 24;
  const int sweep_u = env_int("MPID_SWEEP_U", 0);
  int64_t off_lb = 0;     // lower bound of the offset of the panel being enqueued
  int64_t known_off = 0;  // exact offset at the start of the first unsettled panel
  const FactorState* fin = nullptr;
  // resolves profiler records of one panel once its end state is known
  auto settle = [&](int panel_id, int64_t start_off, const FactorState& h) {
    if (!prof.on) return;
    const int64_t live_end = h.done ? h.k : start_off + h.last_jb;
    for (const ProfRec& r : prof.recs) {
      if (r.j / 1024 != panel_id) continue;  // j packs (panel, step)
      const int64_t jj = r.j % 1024;
      const double t = prof.ms(r);
      const int64_t jd = start_off + jj;
      if (r.kind == PK_SWEEP) {
        if (jd < live_end) {
          acc.sweep_launches += 1;
          acc.sweep_ms += t;
          acc.sweep_bytes += (double)(m - jd) * (double)(n - jd - 1) * sbytes;
        }
      } else if (r.kind == PK_FINALIZE) {
        if (jd < live_end) {
          acc.finalize_launches += 1;
          acc.finalize_ms += t;
        }
      } else if (r.kind == PK_GEMM) {
        if (!h.done) {
          const int64_t je = start_off + h.last_jb;
          acc.gemm_launches += 1;
          acc.gemm_ms += t;
          acc.gemm_bytes += 2.0 * (double)(m - je) * (double)(n - je) * sbytes;
        }
      } else {
        acc.other_ms += t;
      }
    }
  };
  // Pivot-relative rule: the end state counts the columns above the stop
  // threshold; a panel enqueued right after its predecessor settled launches
  // at most that many steps plus one (the rest would only find the done flag).
  const bool count_rule = o->k_fixed == 0 && o->rank_rule == ID_RANK_PIVOT_REL;
  const double count_tol = count_rule ? o->rel_tol : -1.0;
  int64_t step_lim = pl.nb;  // from the last settled end state
  int64_t enq_last = 0;      // steps enqueued for the last panel
  int settled = 0;           // panels whose end state has been processed
  bool drain = false;        // near the end: settle every panel before the next
  const FactorState* fin_drain = nullptr;
  auto settle_upto = [&](int target, const FactorState** done_state) -> int {
    while (settled <= target) {
      const FactorHostSlot* hs;
      if (noalloc) {
        FactorHostSlot* dst = &mirror[settled & 1];
        MPID_HIP(hipMemcpyAsync(dst, &dslot[settled & 1], sizeof(FactorHostSlot),
                                hipMemcpyDeviceToHost, s));
        MPID_HIP(hipStreamSynchronize(s));
        if (dst->seq != seq0 + settled + 1) return ID_ERR_HIP;
        hs = dst;
      } else {
        MPID_HIP(hipEventSynchronize(pev[settled & 1]));
        const int rs = await_slot(&hslot[settled & 1], seq0 + settled + 1);
        if (rs) return rs;
        hs = &hslot[settled & 1];
      }
      const FactorState& h = hs->s;
      settle(settled, known_off, h);
      {
        float vm;
        std::memcpy(&vm, &h.vmax_bits, sizeof(float));
        MPID_LOG(1, "panel %d settled: start %lld, steps %d, done %d (k %lld), live norms above "
                    "the rank threshold %u, largest norm %.4g, drain %d",
                 settled, (long long)known_off, h.done ? (int)(h.k - known_off) : h.last_jb,
                 h.done, (long long)h.k, h.nabove, (double)vm, (int)drain);
      }
      ++settled;
      if (h.done) {
        *done_state = &h;
        return ID_OK;
      }
      if (h.last_jb <= 0) return ID_ERR_HIP;  // a live panel always makes progress
      known_off += h.last_jb;
      step_lim = count_rule ? (int64_t)h.nabove + 1 : pl.nb;
      // the rank rule is near: largest norm within a few panels' decay of the
      // threshold, or kcap within two panels
      float vmaxf;
      std::memcpy(&vmaxf, &h.vmax_bits, sizeof(float));
      const double vmax = (double)vmaxf;
      if (known_off + 2 * pl.nb >= kcap ||
          (o->k_fixed == 0 &&
           (o->rank_rule != ID_RANK_PIVOT_REL || vmax <= 16.0 * o->rel_tol * h.r00)))
        drain = true;
    }
    return ID_OK;
  };
  // One pivot step (sweep, fold for tall inputs, finalization) of panel
  // `panel`, grids sized from the offset lower bound off_b.  Returns 1 when
  // the bounds leave nothing to launch.
  auto launch_step = [&](int panel, int jj, int64_t off_b) -> int {
    const int64_t ncur_b = n - off_b;
    const int64_t jlb = off_b + jj;
    if (jlb >= kcap || jj >= ncur_b) return 1;
    const SweepShape sh = choose_sweep_shape(m - jlb, ncur_b, pl.wbytes);
    a.ncur = ncur_b;
    a.j = jlb;
    a.jj = jj;
    a.Rt = sh.Rt;
    a.CW = sh.CW;
    a.t0 = jlb / sh.Rt;
    a.ntile = (int)(ceil_div(m, sh.Rt) - a.t0);
    a.nchunk = (int)ceil_div(ncur_b, sh.CW);
    a.namax = namax;
    const int64_t total = (int64_t)a.ntile * a.nchunk;
    const dim3 sgrid((unsigned)round_up(total, 8));
    MPID_LOG(2, "step: panel %d, jj %d, rows from %lld, columns <= %lld: %lld-row tiles x "
                "%d-column chunks = %lld blocks%s",
             panel, jj, (long long)jlb, (long long)ncur_b, (long long)sh.Rt, sh.CW,
             (long long)total, a.ntile > kFinZ * kFL ? " (partials folded)" : "");
    const int64_t tag = (int64_t)panel * 1024 + jj;
    // a trailing block beyond the Infinity Cache streams from HBM at its
    // longer latency: more row loads in flight per thread
    const bool deep = sweep_u > 0 ? sweep_u == kSweepUDeep
                                  : (double)(m - jlb) * (double)ncur_b * pl.wbytes > kDeepBytes;
    if (sh.Rt >= 256)
      prof.launch(PK_SWEEP, tag, deep ? k_sweep<S, 1, kSweepUDeep> : k_sweep<S, 1, kSweepU>,
                  sgrid, s, a);
    else if (sh.Rt >= 128)
      prof.launch(PK_SWEEP, tag, deep ? k_sweep<S, 2, kSweepUDeep> : k_sweep<S, 2, kSweepU>,
                  sgrid, s, a);
    else
      prof.launch(PK_SWEEP, tag, deep ? k_sweep<S, 4, kSweepUDeep> : k_sweep<S, 4, kSweepU>,
                  sgrid, s, a);
    MPID_LAUNCH_CHECK();
    // the finalization's grid sets how many pivot partials the next sweep reads
    // (16 columns per block: with 32 the benchmark took 12.02-12.08 instead of
    // 11.87-11.91 ms per ID -- one matrix's step wants more, smaller blocks)
    const auto kfin = k_finalize<S, RM, kFC>;
    namax = (int)ceil_div(ncur_b, kFC);
    if (a.ntile > kFinZ * kFL) {
      // tall input: fold the partials so that one round trip reads them
      const int64_t nfold = ceil_div(a.ntile, kFold);
      const int64_t nthr = (ncur_b + kNbMax + 1) * nfold;
      prof.launch(PK_FINALIZE, tag, k_fold<S>, dim3((unsigned)ceil_div(nthr, kThreads)), s, a,
                  zfold, afold, nfoldb, nfold);
      MPID_LAUNCH_CHECK();
      StepArgs<S> af = a;
      af.zpart = zfold;
      af.auxpart = afold;
      af.nrm2part = nfoldb;
      af.t0 = 0;
      af.ntile = (int)nfold;
      af.tguard = pl.nfold_max;
      prof.launch(PK_FINALIZE, tag, kfin, dim3((unsigned)namax), s, af);
    } else {
      prof.launch(PK_FINALIZE, tag, kfin, dim3((unsigned)namax), s, a);
    }
    MPID_LAUNCH_CHECK();
    return ID_OK;
  };
  for (int panel = 0;; ++panel) {
    const int cur = panel & 1;
    a.W = W[cur];
    a.colid = colid[cur];
    int jj0 = 0;  // first step not yet enqueued
    if (drain && settled < panel) {
      // the panel's first step goes ahead of the wait for the previous panel
      // (sized from the lagged bound), so the GPU is not idle meanwhile; if
      // the stop came first it only finds the done flag
      const int rl = launch_step(panel, 0, off_lb);
      if (rl < 0) return rl;
      jj0 = rl == ID_OK ? 1 : 0;
      const int rc = settle_upto(panel - 1, &fin_drain);
      if (rc) return rc;
      if (fin_drain) {
        fin = fin_drain;
        break;
      }
      off_lb = known_off;
    }
    const int64_t ncur_ub = n - off_lb;
    // the limit holds only when the previous panel's end state is known
    int64_t nsteps = settled == panel ? std::min<int64_t>(pl.nb, step_lim) : pl.nb;
    if (settled == panel - 1 && panel > 0) {
      // the previous panel is still in flight from off_lb: when it runs all
      // enqueued steps (a panel rarely ends early), this one starts at
      // off_lb + enq_last and needs at most kcap - that many steps, and with
      // the pivot-relative count from the state before that panel at most
      // step_lim - enq_last; if it does end early, a later panel takes the
      // remaining steps
      nsteps = std::min<int64_t>(nsteps, std::max<int64_t>(1, kcap - (off_lb + enq_last)));
      if (count_rule && settled > 0)
        nsteps = std::min<int64_t>(nsteps, std::max<int64_t>(1, step_lim - enq_last));
    }
    int64_t launched = jj0;
    for (int jj = jj0; jj < nsteps; ++jj) {
      const int rl = launch_step(panel, jj, off_lb);
      if (rl < 0) return rl;
      if (rl != ID_OK) break;
      ++launched;
    }
    enq_last = launched;
    const GemmArgs<S> g = make_gemm_args<S>(pl, wb, cur, off_lb);
    prof.launch(PK_GEMM, (int64_t)panel * 1024, k_panel_gemm<S, OP, RM>,
                dim3((unsigned)round_up(g.gx * g.gy, 8)), s, g);
    MPID_LAUNCH_CHECK();
    namax = (int)ceil_div(ncur_ub, kFinCols);
    prof.begin(PK_OTHER, (int64_t)panel * 1024, s);
    k_colreduce<<<dim3((unsigned)namax), kThreads, 0, s>>>(
        make_col_args(pl, wb, cur ^ 1, g.tg0, ncur_ub, 1, count_tol, rmode, &kslot[cur],
                      seq0 + panel + 1));
    MPID_LAUNCH_CHECK();
    prof.end(s);
    if (!noalloc) MPID_HIP(hipEventRecord(pev[cur], s));
    // Settle panels up to the previous one (the panel just enqueued keeps the
    // GPU busy meanwhile).  Near the end (drain) the next iteration settles
    // this panel before enqueueing another, so no idle panel follows the stop.
    // A panel's slot and event are reused two panels later, after settling.
    if (!drain) {
      const FactorState* d = nullptr;
      const int rc = settle_upto(panel - 1, &d);
      if (rc) return rc;
      if (d) {
        fin = d;
        break;
      }
      off_lb = known_off;
    }
  }
  if (!fin->done) return ID_ERR_HIP;
  // (the panel enqueued after the stop, if any, only finds the done flag; its
  // norm reduction writes the other host slot, so fin stays valid, and the
  // gather below is ordered after it on the stream: no wait here)
  const int64_t k = fin->k;
  *k_out = k;
  *info = fin->info;
  MPID_LOG(1, "id_factor: k=%lld info=%d after %d panels", (long long)k, fin->info, settled);
  k_finish<<<dim3((unsigned)n, (unsigned)(k > 0 ? ceil_div(k, kThreads) : 1)), kThreads, 0, s>>>(
      make_finish_args(pl, wb, perm, R, ldr, k));
  MPID_LAUNCH_CHECK();
  // the static scratch is shared by every call on the device: it is free again
  // only when this call's work is done
  if (noalloc) MPID_HIP(hipStreamSynchronize(s));
  if (prof.on) {
    MPID_HIP(hipEventRecord(ev_t1, s));
    MPID_HIP(hipEventSynchronize(ev_t1));
    // records of a panel enqueued after the stop are never settled
    float t = 0.0f;
    MPID_HIP(hipEventElapsedTime(&t, ev_t0, ev_t1));
    acc.total_ms = t;
    g_last_profile = acc;
  }
  return ID_OK;
}

static int factor_dispatch(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                           const id_opts* o, void* work, size_t work_bytes, int32_t* perm,
                           double* R, int64_t ldr, int64_t* k_out, int32_t* info, bool noalloc,
                           hipStream_t s) {
  FactorPlan pl;
  if (!make_factor_plan(m, n, dtype, o, &pl)) return ID_ERR_ARG;
  if (!k_out || !info) return ID_ERR_ARG;
  if (n > 0 && !perm) return ID_ERR_ARG;
  if (m > 0 && n > 0 && !A) return ID_ERR_ARG;
  if (lda < (m > 1 ? m : 1)) return ID_ERR_ARG;
  if (pl.kcap > 0 && (!R || ldr < pl.kcap)) return ID_ERR_ARG;
  if (!work || work_bytes < pl.bytes) return ID_ERR_WORKSPACE;
  *info = 0;
  if (m == 0 || n == 0 || pl.kcap == 0) {
    *k_out = 0;
    if (n > 0) {
      k_iota<<<dim3((unsigned)ceil_div(n, kThreads)), kThreads, 0, s>>>(perm, n);
      MPID_LAUNCH_CHECK();
    }
    return ID_OK;
  }
  char* wb = (char*)work;
  const bool f64in = dtype == ID_F64;
  const int32_t rflags = o->flags & (ID_FLAG_ROUND_F32 | ID_FLAG_ROUND_F16);
#define MPID_IMPL(S, OP, RM)                                                                      \
  (f64in ? factor_impl<double, S, OP, RM>((const double*)A, lda, pl, o, wb, perm, R, ldr, k_out,  \
                                          info, noalloc, s)                                       \
         : factor_impl<float, S, OP, RM>((const float*)A, lda, pl, o, wb, perm, R, ldr, k_out,    \
                                         info, noalloc, s))
  // the simulated precisions pair with their own update (checked by the plan)
  if (rflags == ID_FLAG_ROUND_F32) return MPID_IMPL(float, OP_F32, RM_F32);
  if (rflags == ID_FLAG_ROUND_F16) return MPID_IMPL(float, OP_F16, RM_F16);
  switch (pl.prec) {
    case ID_PREC_F64:
      return MPID_IMPL(double, OP_F64, RM_NONE);
    case ID_PREC_MIXED_F16:
      return MPID_IMPL(float, OP_F16, RM_NONE);
    case ID_PREC_MIXED_F32:
      return MPID_IMPL(float, OP_F32, RM_NONE);
    case ID_PREC_MIXED_BF16X3:
      return MPID_IMPL(float, OP_BF16X3, RM_NONE);
    default:
      return MPID_IMPL(float, OP_BF16, RM_NONE);
  }
#undef MPID_IMPL
}

int factor_run(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
               const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
               int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s) {
  return factor_dispatch(A, dtype, m, n, lda, o, work, work_bytes, perm, R, ldr, k_out, info,
                         false, s);
}

int factor_run_noalloc(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                       const id_opts* o, void* work, size_t work_bytes, int32_t* perm, double* R,
                       int64_t ldr, int64_t* k_out, int32_t* info, hipStream_t s) {
  if (o && (o->flags & (ID_FLAG_GRAM | ID_FLAG_CHOLQR | ID_FLAG_PROFILE))) return ID_ERR_UNSUPPORTED;
  return factor_dispatch(A, dtype, m, n, lda, o, work, work_bytes, perm, R, ldr, k_out, info,
                         true, s);
}

// ----------------------------------------------------------------- lock-step batches
//
// Many factorizations advanced together, each the single-matrix algorithm on
// its own workspace: every launch runs one kernel of a pivot step or of a
// panel end for all unfinished items at once, so a step's launch streams the
// trailing blocks of every item (the per-step latencies of one matrix are paid
// once per batch, not once per item).  All items start each panel together;
// an item whose panel ended early, or that finished, leaves the rest of the
// panel's launches at once.  The host reads every item's state after each
// panel, one panel behind the GPU as in the single-matrix driver, to size the
// next panel's grids and to drop finished items.
//
// Block b of a launch belongs to table entry map[b]; its index inside the
// item is b minus the entry's first block of that launch kind.

enum { LK_SWEEP = 0, LK_FIN, LK_GEMM, LK_COL, LK_INIT, LK_INGEST, LK_FINISH, LK_KINDS };

// columns per finalization block in lock-step launches: a step's launch has
// blocks for every item's columns, and each block is one memory round trip, so
// wider blocks (fewer rounds of blocks) shorten the launch
constexpr int kFCMany = 32;

template <typename S>
struct ManyItem {
  StepArgs<S> step;  // j: the panel's offset lower bound (a step adds jj)
  GemmArgs<S> gemm;
  ColArgs col;
  InitArgs init;
  FinishArgs finish;
  const void* A;  // ingest: the input, its working copy and norm partials
  int64_t lda;
  S* w0;
  double* colpart;
  int64_t ingest_gx;
  int namax0, namax1;  // pivot partials of the panel's first / later sweeps
  int first[LK_KINDS];
  int nblk[LK_KINDS];
  int user;  // index of the item in the caller's array
};

// Argument blocks read from an item table in device memory, field by field
// through the constant address space: a pointer loaded that way is known to
// address global memory, so every access derived from it is a global (not a
// flat) memory instruction -- flat accesses also count as LDS accesses, and
// the waits they force would serialize the kernels' round trips.  The field
// lists name every member of the structs above.
template <typename T>
using ConstPtr = const T __attribute__((address_space(4)))*;

#define MPID_STEP_FIELDS(X)                                                                      \
  X(W) X(ldw) X(m) X(n) X(ncur) X(V) X(ldv) X(F) X(ldf) X(vscale) X(tau) X(st) X(amax) X(namax) \
  X(pvflag) X(colid) X(pivpos) X(pivid) X(permw) X(posof) X(zpart) X(auxpart) X(nrm2part) X(nu) \
  X(nuo) X(rorig) X(wrow) X(vrow) X(keypos) X(kcap) X(k_fixed) X(rel_tol) X(tol3z) X(rule)       \
  X(nopivot) X(nb) X(want_fmax) X(rmode) X(j) X(jj) X(t0) X(ntile) X(nchunk) X(Rt) X(CW)        \
  X(tguard)
#define MPID_GEMM_FIELDS(X)                                                                      \
  X(W) X(Wn) X(ldw) X(m) X(ncur) X(V) X(ldv) X(F) X(ldf) X(vscale) X(st) X(pivpos) X(colid)     \
  X(colid_n) X(colpart) X(off) X(tg0) X(gx) X(gy)
#define MPID_COL_FIELDS(X)                                                                       \
  X(colpart) X(ldf) X(tg0) X(tg1) X(ncols_base) X(subtract_jb) X(nu) X(nuo) X(amax) X(colid)   \
  X(posof) X(pvflag) X(keypos) X(st) X(rel_tol) X(rmode) X(hs) X(seq)
#define MPID_INIT_FIELDS(X)                                                                      \
  X(st) X(colid0) X(pvflag) X(permw) X(posof) X(n) X(ldf) X(zrow_z) X(zrow_a) X(zrow_n)         \
  X(frow_z) X(frow_a) X(frow_n)
#define MPID_FINISH_FIELDS(X) X(permw) X(perm_out) X(rorig) X(kcap) X(n) X(k) X(R) X(ldr)
#define MPID_COPY_FIELD(f) d.f = s->f;

template <typename S>
__device__ __forceinline__ StepArgs<S> load_args(ConstPtr<StepArgs<S>> s) {
  StepArgs<S> d;
  MPID_STEP_FIELDS(MPID_COPY_FIELD)
  return d;
}
template <typename S>
__device__ __forceinline__ GemmArgs<S> load_args(ConstPtr<GemmArgs<S>> s) {
  GemmArgs<S> d;
  MPID_GEMM_FIELDS(MPID_COPY_FIELD)
  return d;
}
__device__ __forceinline__ ColArgs load_args(ConstPtr<ColArgs> s) {
  ColArgs d;
  MPID_COL_FIELDS(MPID_COPY_FIELD)
  return d;
}
__device__ __forceinline__ InitArgs load_args(ConstPtr<InitArgs> s) {
  InitArgs d;
  MPID_INIT_FIELDS(MPID_COPY_FIELD)
  return d;
}
__device__ __forceinline__ FinishArgs load_args(ConstPtr<FinishArgs> s) {
  FinishArgs d;
  MPID_FINISH_FIELDS(MPID_COPY_FIELD)
  return d;
}

// The table entry of this block of a lock-step launch.
template <typename S>
__device__ __forceinline__ ConstPtr<ManyItem<S>> many_entry(const ManyItem<S>* it, const int* map) {
  return (ConstPtr<ManyItem<S>>)it + ((ConstPtr<int>)map)[blockIdx.x];
}

template <typename S, int G>
__global__ __launch_bounds__(kThreads) void k_sweep_many(const ManyItem<S>* __restrict__ it,
                                                         const int* __restrict__ map, int jj) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  StepArgs<S> a = load_args<S>(&q->step);
  a.j += jj;
  a.jj = jj;
  a.namax = jj == 0 ? q->namax0 : q->namax1;
  sweep_block<S, G, kSweepUDeep>(a, (int)blockIdx.x - q->first[LK_SWEEP], q->nblk[LK_SWEEP]);
}

template <typename S, int RM>
__global__ __launch_bounds__(kThreads) void k_finalize_many(const ManyItem<S>* __restrict__ it,
                                                            const int* __restrict__ map, int jj) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  StepArgs<S> a = load_args<S>(&q->step);
  a.j += jj;
  a.jj = jj;
  const float fm = finalize_block<S, RM, kFCMany>(a, (int)blockIdx.x - q->first[LK_FIN]);
  if (a.want_fmax && threadIdx.x == 0 && fm >= 0.0f)
    atomicMax(&a.st->fmax_bits, __float_as_uint(fm));
}

template <typename S, int OP, int RM>
__global__ __launch_bounds__(kThreads) void k_panel_gemm_many(const ManyItem<S>* __restrict__ it,
                                                              const int* __restrict__ map) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  const GemmArgs<S> g = load_args<S>(&q->gemm);
  panel_gemm_block<S, OP, RM>(g, blockIdx.x - (uint32_t)q->first[LK_GEMM],
                              (uint32_t)q->nblk[LK_GEMM]);
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_colreduce_many(const ManyItem<S>* __restrict__ it,
                                                             const int* __restrict__ map) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  const ColArgs c = load_args(&q->col);
  colreduce_body(c, (int)blockIdx.x - q->first[LK_COL], q->nblk[LK_COL]);
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_init_many(const ManyItem<S>* __restrict__ it,
                                                        const int* __restrict__ map) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  const InitArgs a = load_args(&q->init);
  init_block(a, (int64_t)blockIdx.x - q->first[LK_INIT]);
}

template <typename TA, typename S>
__global__ __launch_bounds__(kThreads) void k_ingest_many(const ManyItem<S>* __restrict__ it,
                                                          const int* __restrict__ map) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  IngestArgs<TA, S> a;
  a.A = (const TA*)q->A;
  a.lda = q->lda;
  a.m = q->step.m;
  a.n = q->step.n;
  a.W = q->w0;
  a.ldw = q->step.ldw;
  a.colpart = q->colpart;
  a.ldf = q->step.ldf;
  a.st = q->step.st;
  a.rmode = q->step.rmode;
  const int64_t gx = q->ingest_gx;
  const int64_t lb = (int64_t)blockIdx.x - q->first[LK_INGEST];
  ingest_block<TA, S>(a, lb % gx, lb / gx);
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_finish_many(const ManyItem<S>* __restrict__ it,
                                                          const int* __restrict__ map) {
  const ConstPtr<ManyItem<S>> q = many_entry(it, map);
  const FinishArgs f = load_args(&q->finish);
  const int64_t lb = (int64_t)blockIdx.x - q->first[LK_FINISH];
  finish_block(f, lb % f.n, lb / f.n);
}

// k and info of every item (one block per table entry, in the caller's
// order): the factorization's own info (non-finite input) if set, else
// ID_INFO_SINGULAR when some |R_ii| <= n 2^-53 |R_00| (or R_00 = 0),
// ID_INFO_RANK_FULL when k == n, else 0 -- the conditions of id_solve_T.
template <typename S>
__global__ __launch_bounds__(kThreads) void k_check_many(const ManyItem<S>* __restrict__ it,
                                                         id_batch_item* __restrict__ items) {
  __shared__ double dscr[4];
  const ManyItem<S>& q = it[blockIdx.x];
  id_batch_item& bi = items[q.user];
  const FactorState* st = q.step.st;
  const int64_t k = q.finish.k, n = q.finish.n;
  const int32_t finfo = st->info;
  const double* R = bi.R;
  const int64_t ldr = bi.ldr;
  const int tid = threadIdx.x;
  const double r00 = (finfo == 0 && k > 0) ? fabs(R[0]) : 0.0;
  const double thr = (double)n * ldexp(1.0, -53) * r00;
  double bad = 0.0;
  if (finfo == 0)
    for (int64_t i = tid; i < k; i += kThreads)
      if (!(fabs(R[i * ldr + i]) > thr)) bad += 1.0;
  bad = block_sum(bad, dscr);
  if (tid == 0) {
    bi.k = k;
    if (finfo != 0)
      bi.info = finfo;
    else if (k > 0 && (bad > 0.0 || r00 == 0.0))
      bi.info = ID_INFO_SINGULAR;
    else
      bi.info = (k == n) ? ID_INFO_RANK_FULL : 0;
  }
}

namespace {

// flags[t] = 1 when item t's current panel has ended (or the item is done),
// for the first n items of the table: the host's mid-panel look at whether the
// rest of a panel's steps would find anything to do.
template <typename S>
__global__ __launch_bounds__(kThreads) void k_probe_many(const ManyItem<S>* __restrict__ it, int n,
                                                         int32_t* __restrict__ flags) {
  const int t = (int)(blockIdx.x * kThreads + threadIdx.x);
  if (t >= n) return;
  const FactorState* st = it[t].step.st;
  flags[t] = (st->end_flag || st->done) ? 1 : 0;
}

struct LockPlan {
  int Rt = 128;
  std::vector<FactorPlan> pl;   // per item
  std::vector<int> cw;          // sweep column chunk per item
  int64_t cap[LK_KINDS] = {0};  // map capacity per launch kind (blocks)
  int64_t max_n = 0;
  size_t off_items = 0, off_ditems = 0, off_slots = 0, off_probe = 0, off_map[LK_KINDS] = {0};
  size_t bytes = 0;
};

constexpr int kManyTileMax = kFinZ * kFL;  // row tiles one finalization round trip covers
constexpr int kManyBlocks = 4096;          // sweep blocks that fill the chip several times over
constexpr int kProbe = 4;                  // steps before a panel's mid-panel look

int lockstep_sweep_blocks(const FactorPlan& pl, int Rt, int cw, int64_t off) {
  const int64_t ntile = ceil_div(pl.m, Rt) - off / Rt;
  return (int)round_up(ntile * ceil_div(pl.n - off, cw), 8);
}

}  // namespace

// Validates the batch and lays out the shared workspace.
static int make_lock_plan(const id_batch_item* items, int32_t batch, int32_t dtype,
                          const id_opts* o, LockPlan* lp) {
  if (!items || batch < 0 || !o) return ID_ERR_ARG;
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (o->flags & (ID_FLAG_GRAM | ID_FLAG_CHOLQR | ID_FLAG_PROFILE)) return ID_ERR_UNSUPPORTED;
  lp->pl.resize(batch);
  lp->cw.resize(batch);
  int64_t max_m = 0;
  for (int32_t i = 0; i < batch; ++i) {
    const id_batch_item& it = items[i];
    FactorPlan& pl = lp->pl[i];
    if (!make_factor_plan(it.m, it.n, dtype, o, &pl)) return ID_ERR_ARG;
    if (it.m > 0 && it.n > 0 && !it.A) return ID_ERR_ARG;
    if (it.lda < (it.m > 1 ? it.m : 1)) return ID_ERR_ARG;
    if (it.n > 0 && !it.perm) return ID_ERR_ARG;
    if (pl.kcap > 0 && (!it.R || it.ldr < pl.kcap)) return ID_ERR_ARG;
    if (pl.kcap > 0 && it.n > pl.kcap && (!it.T || it.ldt < pl.kcap)) return ID_ERR_ARG;
    if (!it.work) return ID_ERR_WORKSPACE;
    max_m = std::max<int64_t>(max_m, it.m);
    lp->max_n = std::max<int64_t>(lp->max_n, it.n);
  }
  // one row-tile height for the batch, every item's tiles within one round
  // trip of the finalization (no folding): the tallest tiles (the fixed
  // latencies of a block are shared by the most rows) unless the batch then
  // has too few blocks to fill the chip
  if (ceil_div(max_m, kRtMax) > kManyTileMax) return ID_ERR_UNSUPPORTED;
  const int cw_env = env_int("MPID_LOCKSTEP_CW", 0);
  for (int32_t i = 0; i < batch; ++i) {
    const FactorPlan& pl = lp->pl[i];
    const int v = pl.wbytes == 8 ? 2 : 4;  // values per 16-byte load
    // the chunk (64, 128 or 256 lanes per row) that leaves the fewest idle
    // lanes over the item's columns, the wider one on ties
    int cw = 64 * v;
    for (int c = 128 * v; c <= 256 * v; c *= 2)
      if (ceil_div(pl.n, c) * c <= ceil_div(pl.n, cw) * cw) cw = c;
    if (cw_env == 64 * v || cw_env == 128 * v || cw_env == 256 * v) cw = cw_env;
    lp->cw[i] = cw;
  }
  int rt = env_int("MPID_LOCKSTEP_RT", 0);
  if (rt <= 0) {
    const int64_t target = env_int("MPID_LOCKSTEP_BLOCKS", kManyBlocks);
    rt = kRtMax;
    while (rt > kRtMin && ceil_div(max_m, rt / 2) <= kManyTileMax) {
      int64_t blocks = 0;
      for (int32_t i = 0; i < batch; ++i)
        blocks += lockstep_sweep_blocks(lp->pl[i], rt, lp->cw[i], 0);
      if (blocks >= target) break;
      rt /= 2;
    }
  }
  if (rt != 64 && rt != 128 && rt != 256) return ID_ERR_ARG;
  if (ceil_div(max_m, rt) > kManyTileMax) return ID_ERR_UNSUPPORTED;
  lp->Rt = rt;
  for (int32_t i = 0; i < batch; ++i) {
    const FactorPlan& pl = lp->pl[i];
    // the grids of the first panel (offset 0) are the largest
    lp->cap[LK_SWEEP] += lockstep_sweep_blocks(pl, rt, lp->cw[i], 0);
    lp->cap[LK_FIN] += ceil_div(pl.n, kFCMany);
    lp->cap[LK_GEMM] += round_up(ceil_div(pl.n, 64) * ceil_div(pl.m, kRowTileG), 8);
    lp->cap[LK_COL] += ceil_div(pl.n, kFinCols);
    lp->cap[LK_INIT] += init_blocks(pl);
    lp->cap[LK_INGEST] += ceil_div(pl.n, 64) * ceil_div(pl.m, kRowTileG);
    lp->cap[LK_FINISH] += pl.n * (pl.kcap > 0 ? ceil_div(pl.kcap, kThreads) : 1);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += (bytes + 255) / 256 * 256;
    return o2;
  };
  static_assert(sizeof(ManyItem<float>) == sizeof(ManyItem<double>), "item table layout");
  lp->off_items = take(sizeof(ManyItem<float>) * (size_t)std::max(batch, 1));
  lp->off_ditems = take(sizeof(id_batch_item) * (size_t)std::max(batch, 1));
  lp->off_slots = take(sizeof(FactorHostSlot) * (size_t)std::max(batch, 1));
  lp->off_probe = take(sizeof(int32_t) * (size_t)std::max(batch, 1));
  for (int kd = 0; kd < LK_KINDS; ++kd) lp->off_map[kd] = take(4 * (size_t)std::max<int64_t>(lp->cap[kd], 1));
  lp->bytes = off;
  return ID_OK;
}

size_t lockstep_workspace(const id_batch_item* items, int32_t batch, int32_t dtype,
                          const id_opts* o) {
  LockPlan lp;
  if (make_lock_plan(items, batch, dtype, o, &lp) != ID_OK) return 0;
  return lp.bytes;
}

template <typename TA, typename S, int OP, int RM, int G>
static int lockstep_impl(id_batch_item* items, int32_t batch, const id_opts* o, const LockPlan& lp,
                         char* shared, hipStream_t s) {
  const int rmode = RM;
  const int Rt = lp.Rt;
  const int want_fmax = (OP == OP_F16 && RM != RM_F16) ? 1 : 0;
  // the batch's working set is far beyond the caches: the deeper sweep loop
  ManyItem<S>* d_items = (ManyItem<S>*)(shared + lp.off_items);
  id_batch_item* d_bi = (id_batch_item*)(shared + lp.off_ditems);
  FactorHostSlot* d_slots = (FactorHostSlot*)(shared + lp.off_slots);
  int32_t* d_probe = (int32_t*)(shared + lp.off_probe);
  int* d_map[LK_KINDS];
  for (int kd = 0; kd < LK_KINDS; ++kd) d_map[kd] = (int*)(shared + lp.off_map[kd]);

  ThreadRes& tr = thread_res();
  PinnedBuf* stage = tr.stage;
  PinnedBuf* hslots = tr.lslots;
  hipEvent_t* ev_stage = tr.ev_stage;
  hipEvent_t* ev_slot = tr.ev_slot;
  for (int q = 0; q < 2; ++q) {
    if (!ev_stage[q]) MPID_HIP(hipEventCreateWithFlags(&ev_stage[q], hipEventDisableTiming));
    if (!ev_slot[q]) MPID_HIP(hipEventCreateWithFlags(&ev_slot[q], hipEventDisableTiming));
  }
  const size_t tbl_bytes = sizeof(ManyItem<S>) * (size_t)batch;
  int64_t map_total = 0;
  for (int kd = 0; kd < LK_KINDS; ++kd) map_total += lp.cap[kd];
  const size_t stage_bytes = tbl_bytes + 4 * (size_t)map_total;
  for (int q = 0; q < 2; ++q) {
    int rc = pinned_reserve(stage[q], stage_bytes, hipHostMallocDefault);
    if (rc) return rc;
    rc = pinned_reserve(hslots[q], sizeof(FactorHostSlot) * (size_t)batch, hipHostMallocDefault);
    if (rc) return rc;
  }
  {
    const int rc = pinned_reserve(tr.probe, sizeof(int32_t) * (size_t)std::max(batch, 1),
                                  hipHostMallocDefault);
    if (rc) return rc;
    if (!tr.ev_probe) MPID_HIP(hipEventCreateWithFlags(&tr.ev_probe, hipEventDisableTiming));
  }
  const int32_t* hprobe = (const int32_t*)tr.probe.p;
  int upload = 0;  // uploads so far (staging buffer upload & 1)
  // staging buffer for the next upload: its table and per-kind maps
  struct Stage {
    ManyItem<S>* tbl;
    int* map[LK_KINDS];
  };
  auto begin_stage = [&](Stage* st) -> int {
    const int q = upload & 1;
    MPID_HIP(hipEventSynchronize(ev_stage[q]));  // its last copy has been read
    char* b = (char*)stage[q].p;
    st->tbl = (ManyItem<S>*)b;
    size_t off = tbl_bytes;
    for (int kd = 0; kd < LK_KINDS; ++kd) {
      st->map[kd] = (int*)(b + off);
      off += 4 * (size_t)lp.cap[kd];
    }
    return ID_OK;
  };
  // copies the table (entries) and the maps of the given kinds (blocks used)
  auto end_stage = [&](const Stage& st, int entries, const int64_t* used) -> int {
    const int q = upload & 1;
    MPID_HIP(hipMemcpyAsync(d_items, st.tbl, sizeof(ManyItem<S>) * (size_t)entries,
                            hipMemcpyHostToDevice, s));
    for (int kd = 0; kd < LK_KINDS; ++kd)
      if (used[kd] > 0)
        MPID_HIP(hipMemcpyAsync(d_map[kd], st.map[kd], 4 * (size_t)used[kd],
                                hipMemcpyHostToDevice, s));
    MPID_HIP(hipEventRecord(ev_stage[q], s));
    ++upload;
    return ID_OK;
  };

  // per-item host view
  std::vector<int64_t> known_off(batch, 0), k(batch, 0);
  std::vector<int32_t> finfo(batch, 0);
  std::vector<char> done(batch, 0);
  std::vector<int> namax_cr(batch, 0);
  std::vector<StepArgs<S>> base(batch);
  for (int32_t i = 0; i < batch; ++i) {
    char* wb = (char*)items[i].work;
    base[i] = make_step_args<S>(lp.pl[i], wb, o, rmode, want_fmax);
    namax_cr[i] = (int)ceil_div(lp.pl[i].n, kFinCols);
    // nothing to factor: k = 0 (the initialization still runs for perm)
    if (items[i].m == 0 || items[i].n == 0 || lp.pl[i].kcap == 0) done[i] = 1;
  }
  MPID_LOG(1, "id_factor_lockstep: %d items, %d-row tiles, shared workspace %zu bytes", (int)batch,
           Rt, lp.bytes);

  // ---- prologue: initialization, ingest, column norms of every item
  MPID_HIP(hipMemcpyAsync(d_bi, items, sizeof(id_batch_item) * (size_t)batch,
                          hipMemcpyHostToDevice, s));
  {
    Stage st;
    int rc = begin_stage(&st);
    if (rc) return rc;
    int64_t used[LK_KINDS] = {0};
    for (int32_t i = 0; i < batch; ++i) {
      const FactorPlan& pl = lp.pl[i];
      char* wb = (char*)items[i].work;
      ManyItem<S>& q = st.tbl[i];
      std::memset(&q, 0, sizeof(q));
      q.user = i;
      q.step = base[i];
      q.init = make_init_args(pl, wb);
      q.A = items[i].A;
      q.lda = items[i].lda;
      q.w0 = (S*)(wb + pl.off_w0);
      q.colpart = (double*)(wb + pl.off_colpart);
      q.ingest_gx = ceil_div(pl.n, 64);
      q.col = make_col_args(pl, wb, 0, 0, pl.n, 0, -1.0, rmode, nullptr, 0);
      const int64_t nb_kind[3] = {init_blocks(pl),
                                  done[i] ? 0 : q.ingest_gx * ceil_div(pl.m, kRowTileG),
                                  done[i] ? 0 : ceil_div(pl.n, kFinCols)};
      const int kinds[3] = {LK_INIT, LK_INGEST, LK_COL};
      for (int t = 0; t < 3; ++t) {
        const int kd = kinds[t];
        q.first[kd] = (int)used[kd];
        q.nblk[kd] = (int)nb_kind[t];
        for (int64_t b = 0; b < nb_kind[t]; ++b) st.map[kd][used[kd] + b] = i;
        used[kd] += nb_kind[t];
      }
    }
    rc = end_stage(st, batch, used);
    if (rc) return rc;
    if (used[LK_INIT] > 0)
      k_init_many<S><<<dim3((unsigned)used[LK_INIT]), kThreads, 0, s>>>(d_items, d_map[LK_INIT]);
    MPID_LAUNCH_CHECK();
    if (used[LK_INGEST] > 0)
      k_ingest_many<TA, S><<<dim3((unsigned)used[LK_INGEST]), kThreads, 0, s>>>(
          d_items, d_map[LK_INGEST]);
    MPID_LAUNCH_CHECK();
    if (used[LK_COL] > 0)
      k_colreduce_many<S><<<dim3((unsigned)used[LK_COL]), kThreads, 0, s>>>(d_items,
                                                                            d_map[LK_COL]);
    MPID_LAUNCH_CHECK();
  }

  // ---- panels
  const bool count_rule = o->k_fixed == 0 && o->rank_rule == ID_RANK_PIVOT_REL;
  const double count_tol = count_rule ? o->rel_tol : -1.0;
  const int64_t seq0 = (++tr.ncalls) << 24;
  std::vector<int> in_panel[2];  // items (caller's index) of the last two panels
  std::vector<int> order;
  std::vector<int64_t> lim;
  // the next panel enqueued takes the mid-panel look when every live item
  // ended the last settled panel before its step limit (and the first panel)
  bool probe_next = true;
  std::vector<int64_t> lim_enq[2];  // the step limits the last two panels had
  auto settle = [&](int panel) -> int {
    const int q = panel & 1;
    MPID_HIP(hipEventSynchronize(ev_slot[q]));
    const FactorHostSlot* hs = (const FactorHostSlot*)hslots[q].p;
    bool all_early = true;
    for (const int i : in_panel[q]) {
      if (done[i]) continue;
      const FactorHostSlot& sl = hs[i];
      if (sl.seq != seq0 + panel + 1) return ID_ERR_HIP;
      const FactorState& h = sl.s;
      if (h.done) {
        done[i] = 1;
        k[i] = h.k;
        finfo[i] = h.info;
        continue;
      }
      if (h.last_jb <= 0) return ID_ERR_HIP;  // a live panel always makes progress
      if (h.last_jb >= lim_enq[q][i]) all_early = false;
      known_off[i] += h.last_jb;
    }
    probe_next = all_early;
    return ID_OK;
  };
  int panel = 0;
  for (;; ++panel) {
    const int cur = panel & 1;
    // live items, most steps first (a step's launch covers a prefix of them)
    order.clear();
    for (int32_t i = 0; i < batch; ++i)
      if (!done[i]) order.push_back(i);
    if (order.empty()) break;
    lim.assign(batch, 0);
    for (const int i : order) {
      const FactorPlan& pl = lp.pl[i];
      lim[i] = std::min<int64_t>({(int64_t)pl.nb, pl.kcap - known_off[i], pl.n - known_off[i]});
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return lim[x] > lim[y]; });
    lim_enq[cur] = lim;
    Stage st;
    int rc = begin_stage(&st);
    if (rc) return rc;
    int64_t used[LK_KINDS] = {0};
    std::vector<int64_t> sw_end(order.size()), fin_end(order.size());
    for (size_t t = 0; t < order.size(); ++t) {
      const int i = order[t];
      const FactorPlan& pl = lp.pl[i];
      char* wb = (char*)items[i].work;
      const int64_t off_lb = known_off[i];
      const int64_t ncur_b = pl.n - off_lb;
      ManyItem<S>& q = st.tbl[t];
      std::memset(&q, 0, sizeof(q));
      q.user = i;
      StepArgs<S>& a = q.step;
      a = base[i];
      a.W = (const S*)(wb + (cur ? pl.off_w1 : pl.off_w0));
      a.colid = (const int*)(wb + (cur ? pl.off_colid1 : pl.off_colid0));
      a.ncur = ncur_b;
      a.j = off_lb;
      a.Rt = Rt;
      a.CW = lp.cw[i];
      a.t0 = off_lb / Rt;
      a.ntile = (int)(ceil_div(pl.m, Rt) - a.t0);
      a.nchunk = (int)ceil_div(ncur_b, a.CW);
      q.namax0 = namax_cr[i];
      q.namax1 = (int)ceil_div(ncur_b, kFCMany);
      q.gemm = make_gemm_args<S>(pl, wb, cur, off_lb);
      q.col = make_col_args(pl, wb, cur ^ 1, q.gemm.tg0, ncur_b, 1, count_tol, rmode,
                            &d_slots[i], seq0 + panel + 1);
      const int64_t nb_kind[4] = {round_up((int64_t)a.ntile * a.nchunk, 8), q.namax1,
                                  round_up(q.gemm.gx * q.gemm.gy, 8), ceil_div(ncur_b, kFinCols)};
      for (int kd = 0; kd < 4; ++kd) {
        q.first[kd] = (int)used[kd];
        q.nblk[kd] = (int)nb_kind[kd];
        int* mp = st.map[kd] + used[kd];
        for (int64_t b = 0; b < nb_kind[kd]; ++b) mp[b] = (int)t;
        used[kd] += nb_kind[kd];
      }
      sw_end[t] = used[LK_SWEEP];
      fin_end[t] = used[LK_FIN];
      namax_cr[i] = (int)nb_kind[LK_COL];
    }
    rc = end_stage(st, (int)order.size(), used);
    if (rc) return rc;
    MPID_LOG(2, "lock-step panel %d: %zu items, %lld sweep blocks, %lld update blocks", panel,
             order.size(), (long long)used[LK_SWEEP], (long long)used[LK_GEMM]);
    const int64_t lmax = lim[order[0]];
    size_t live = order.size();
    // Mid-panel looks (the first panel, and any panel after one in which
    // every item ended early): every kProbe steps the items' end flags are
    // copied to the host, which reads them once kProbe more steps are
    // enqueued (the GPU is busy with those meanwhile) and launches no further
    // steps when every live item's panel has already ended.  Stopping a panel
    // early is always correct: its update applies the steps that ran.
    const bool probe = probe_next && lmax >= 2 * kProbe;
    size_t probe_live = 0;  // items the outstanding look covers (0: none)
    for (int jj = 0; jj < lmax; ++jj) {
      while (live > 0 && lim[order[live - 1]] <= jj) --live;
      if (live == 0) break;
      const unsigned gs = (unsigned)sw_end[live - 1], gf = (unsigned)fin_end[live - 1];
      k_sweep_many<S, G><<<dim3(gs), kThreads, 0, s>>>(d_items, d_map[LK_SWEEP], jj);
      MPID_LAUNCH_CHECK();
      k_finalize_many<S, RM><<<dim3(gf), kThreads, 0, s>>>(d_items, d_map[LK_FIN], jj);
      MPID_LAUNCH_CHECK();
      if (!probe || (jj + 1) % kProbe != 0 || jj + 1 >= lmax) continue;
      if (probe_live > 0) {
        // the look issued kProbe steps ago
        MPID_HIP(hipEventSynchronize(tr.ev_probe));
        bool all_ended = true;
        for (size_t t = 0; t < probe_live && all_ended; ++t) all_ended = hprobe[t] != 0;
        if (all_ended) {
          MPID_LOG(2, "lock-step panel %d: every item ended by step %d", panel, jj + 1 - kProbe);
          break;
        }
      }
      probe_live = live;
      k_probe_many<S><<<dim3((unsigned)ceil_div((int64_t)live, kThreads)), kThreads, 0, s>>>(
          d_items, (int)live, d_probe);
      MPID_LAUNCH_CHECK();
      MPID_HIP(hipMemcpyAsync(tr.probe.p, d_probe, sizeof(int32_t) * live, hipMemcpyDeviceToHost,
                              s));
      MPID_HIP(hipEventRecord(tr.ev_probe, s));
    }
    k_panel_gemm_many<S, OP, RM><<<dim3((unsigned)used[LK_GEMM]), kThreads, 0, s>>>(
        d_items, d_map[LK_GEMM]);
    MPID_LAUNCH_CHECK();
    k_colreduce_many<S><<<dim3((unsigned)used[LK_COL]), kThreads, 0, s>>>(d_items,
                                                                          d_map[LK_COL]);
    MPID_LAUNCH_CHECK();
    MPID_HIP(hipMemcpyAsync(hslots[cur].p, d_slots, sizeof(FactorHostSlot) * (size_t)batch,
                            hipMemcpyDeviceToHost, s));
    MPID_HIP(hipEventRecord(ev_slot[cur], s));
    in_panel[cur] = order;
    // the previous panel's end states (this panel keeps the GPU busy)
    if (panel > 0) {
      rc = settle(panel - 1);
      if (rc) return rc;
    }
  }
  // the last enqueued panel (if any) only found finished items
  if (panel > 0) {
    const int rc = settle(panel - 1);
    if (rc) return rc;
  }
  MPID_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i < batch; ++i)
    if (!done[i]) return ID_ERR_HIP;

  // ---- R, perm, k and info of every item, then T = R11^{-1} R12
  {
    Stage st;
    int rc = begin_stage(&st);
    if (rc) return rc;
    int64_t used[LK_KINDS] = {0};
    for (int32_t i = 0; i < batch; ++i) {
      const FactorPlan& pl = lp.pl[i];
      char* wb = (char*)items[i].work;
      ManyItem<S>& q = st.tbl[i];
      std::memset(&q, 0, sizeof(q));
      q.user = i;
      q.step = base[i];
      q.finish = make_finish_args(pl, wb, items[i].perm, items[i].R, items[i].ldr, k[i]);
      const int64_t nbk = pl.n * (k[i] > 0 ? ceil_div(k[i], kThreads) : 1);
      q.first[LK_FINISH] = (int)used[LK_FINISH];
      q.nblk[LK_FINISH] = (int)nbk;
      for (int64_t b = 0; b < nbk; ++b) st.map[LK_FINISH][used[LK_FINISH] + b] = i;
      used[LK_FINISH] += nbk;
    }
    rc = end_stage(st, batch, used);
    if (rc) return rc;
    if (used[LK_FINISH] > 0)
      k_finish_many<S><<<dim3((unsigned)used[LK_FINISH]), kThreads, 0, s>>>(d_items,
                                                                            d_map[LK_FINISH]);
    MPID_LAUNCH_CHECK();
    k_check_many<S><<<dim3((unsigned)batch), kThreads, 0, s>>>(d_items, d_bi);
    MPID_LAUNCH_CHECK();
  }
  {
    const int rc = trsm_batched_run(d_bi, batch, lp.max_n, s);
    if (rc) return rc;
  }
  std::vector<id_batch_item> out(batch);
  MPID_HIP(hipMemcpyAsync(out.data(), d_bi, sizeof(id_batch_item) * (size_t)batch,
                          hipMemcpyDeviceToHost, s));
  MPID_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i < batch; ++i) {
    items[i].k = out[i].k;
    items[i].info = out[i].info;
  }
  MPID_LOG(1, "id_factor_lockstep: done after %d panels", panel);
  return ID_OK;
}

int lockstep_run(id_batch_item* items, int32_t batch, int32_t dtype, const id_opts* o, void* work,
                 size_t work_bytes, hipStream_t s) {
  LockPlan lp;
  const int rc = make_lock_plan(items, batch, dtype, o, &lp);
  if (rc) return rc;
  if (batch == 0) return ID_OK;
  if (!work || work_bytes < lp.bytes) return ID_ERR_WORKSPACE;
  char* sh = (char*)work;
  const bool f64in = dtype == ID_F64;
  const int32_t rflags = o->flags & (ID_FLAG_ROUND_F32 | ID_FLAG_ROUND_F16);
#define MPID_LS(S, OP, RM)                                                                     \
  (lp.Rt == 256   ? (f64in ? lockstep_impl<double, S, OP, RM, 1>(items, batch, o, lp, sh, s)    \
                           : lockstep_impl<float, S, OP, RM, 1>(items, batch, o, lp, sh, s))    \
   : lp.Rt == 128 ? (f64in ? lockstep_impl<double, S, OP, RM, 2>(items, batch, o, lp, sh, s)    \
                           : lockstep_impl<float, S, OP, RM, 2>(items, batch, o, lp, sh, s))    \
                  : (f64in ? lockstep_impl<double, S, OP, RM, 4>(items, batch, o, lp, sh, s)    \
                           : lockstep_impl<float, S, OP, RM, 4>(items, batch, o, lp, sh, s)))
  if (rflags == ID_FLAG_ROUND_F32) return MPID_LS(float, OP_F32, RM_F32);
  if (rflags == ID_FLAG_ROUND_F16) return MPID_LS(float, OP_F16, RM_F16);
  switch (o->prec) {
    case ID_PREC_F64:
      return MPID_LS(double, OP_F64, RM_NONE);
    case ID_PREC_MIXED_F16:
      return MPID_LS(float, OP_F16, RM_NONE);
    case ID_PREC_MIXED_F32:
      return MPID_LS(float, OP_F32, RM_NONE);
    case ID_PREC_MIXED_BF16X3:
      return MPID_LS(float, OP_BF16X3, RM_NONE);
    default:
      return MPID_LS(float, OP_BF16, RM_NONE);
  }
#undef MPID_LS
}


}  // namespace mpid
