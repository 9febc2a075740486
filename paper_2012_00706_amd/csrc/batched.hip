// Many column IDs of uneven sizes in one persistent launch.
//
// Workgroups repeatedly take the next slot from a device work queue (an
// atomic counter over a caller-given slot list, e.g. largest item first).  A
// slot names an item; an item listed G times in a row is factored by G
// workgroups together.  The method is that of the single-matrix path
// (Section 1.1, eq. (6)-(7); the MGSQR(A, k) step of Algorithms 1 and 2):
// row-major working copy, per pivot the pivot-column update, reflector, one
// sweep of the stale trailing block, new F column and R row, norm downdating;
// per panel the matrix-core update W -= V F^T with compaction and FP64 norm
// recomputation.
//
// With G workgroups each owns a contiguous range of the working columns (its
// sweep, F/R/downdate and panel update; the ranges are re-split evenly after
// every panel, whose update compacts all of them into one layout) and a slice
// of the rows for the pivot column; they agree on every decision through two
// exchanges per pivot step (and one more per panel, after the update):
//   A: pivot candidates, "end the panel" flags and the panel's max |F|;
//   B: partial sums of the pivot column (||w||^2, V^T w) and its leading entry.
// Every workgroup publishes its part with a device-scope release and reads the
// others' with acquire loads; partial sums are combined in workgroup order, so
// all of them compute bitwise the same reflector and pivot.  A wait that exceeds
// its time limit marks the item aborted and every workgroup leaves, so the grid
// always drains.  T = R11^{-1} R12 is solved afterwards by a batched launch of
// the triangular-solve kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>

#include "device_util.h"
#include "mpid_internal.h"

namespace mpid {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename S>
struct BVec;
template <>
struct BVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct BVec<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

enum { BOP_F64 = 0, BOP_F16 = 1, BOP_BF16 = 2, BOP_BF16X3 = 3, BOP_F32 = 4 };

// pointer into the global address space
template <typename T>
using GlobalPtr = T __attribute__((address_space(1)))*;

// id_batch_item as device code reads it: the same layout with the pointers
// typed as global memory, so that everything derived from them uses global
// instead of flat (generic) memory instructions (flat accesses also count as
// LDS accesses and force extra waits)
struct BatchItemDev {
  GlobalPtr<const void> A;
  int64_t m, n, lda;
  GlobalPtr<void> work;
  GlobalPtr<int32_t> perm;
  GlobalPtr<double> R;
  int64_t ldr;
  GlobalPtr<double> T;
  int64_t ldt;
  int64_t k;
  int32_t info;
  int32_t groups;
};
static_assert(sizeof(BatchItemDev) == sizeof(id_batch_item), "layout");
static_assert(offsetof(BatchItemDev, groups) == offsetof(id_batch_item, groups), "layout");

}  // namespace

struct BatchOpts {
  int64_t k_fixed, k_max;
  double rel_tol, tol3z;
  int rule, nb;
  uint64_t wait_ticks;  // time limit of one exchange wait, in wall-clock ticks
};

// One workgroup's part of one exchange.  "tag" (the exchange's sequence
// number) is stored last, with release semantics.
struct XSlot {
  int64_t tag;
  double v, s2;      // pivot candidate: largest column norm, sum of squared norms
  int32_t pos, key;  // its position and swap-order key
  int32_t flag;      // a downdate asked to end the panel
  int32_t bad;       // the ingest met NaN/Inf
  float fmax;        // max |F| over the workgroup's columns in this panel
  int32_t pad;
  double nrm2, alpha;    // partial ||w(j+1:m)||^2; leading entry w(j)
  double zsum[kNbMax];   // partial V(j+1:m, c)^T w(j+1:m)
};

struct BatchLayout {
  int64_t kcap, ldw, ldv, ldf;
  size_t off_w0, off_w1, off_v, off_f, off_nu, off_nuo, off_colid0, off_colid1, off_pvflag,
      off_permw, off_posof, off_rorig, off_xs, off_abort, bytes;
};

__host__ __device__ inline int64_t batch_kcap(int64_t m, int64_t n, int64_t k_fixed,
                                              int64_t k_max) {
  int64_t kc = m < n ? m : n;
  if (k_max > 0 && k_max < kc) kc = k_max;
  if (k_fixed > 0 && k_fixed < kc) kc = k_fixed;
  return kc;
}

__host__ __device__ inline BatchLayout batch_layout(int64_t m, int64_t n, int64_t kcap, int wb) {
  BatchLayout L;
  const int64_t mm = m > 0 ? m : 1, nn = n > 0 ? n : 1, kk = kcap > 0 ? kcap : 1;
  L.kcap = kcap;
  // rows an odd multiple of 256 bytes apart (different memory channels)
  const int64_t q256 = 256 / wb;
  L.ldw = round_up(nn, 64);
  if ((L.ldw / q256) % 2 == 0) L.ldw += q256;
  L.ldv = kNbMax;  // reflectors row-major: V(i, c) at i * kNbMax + c
  L.ldf = round_up(nn, 64);
  size_t off = 0;
#define MPID_TAKE(field, bytes_)              \
  L.field = off;                              \
  off += ((size_t)(bytes_) + 255) / 256 * 256;
  MPID_TAKE(off_w0, (size_t)mm * L.ldw * wb);
  MPID_TAKE(off_w1, (size_t)mm * L.ldw * wb);
  MPID_TAKE(off_v, (size_t)mm * kNbMax * wb);
  MPID_TAKE(off_f, (size_t)kNbMax * L.ldf * 8);
  MPID_TAKE(off_nu, (size_t)L.ldf * 8);
  MPID_TAKE(off_nuo, (size_t)L.ldf * 8);
  MPID_TAKE(off_colid0, (size_t)L.ldf * 4);
  MPID_TAKE(off_colid1, (size_t)L.ldf * 4);
  MPID_TAKE(off_pvflag, (size_t)L.ldf * 4);
  MPID_TAKE(off_permw, (size_t)nn * 4);
  MPID_TAKE(off_posof, (size_t)nn * 4);
  MPID_TAKE(off_rorig, (size_t)kk * nn * 8);
  MPID_TAKE(off_xs, (size_t)kBatchMaxGroups * sizeof(XSlot));
  MPID_TAKE(off_abort, 4);
#undef MPID_TAKE
  L.bytes = off;
  return L;
}

template <int BT>
struct BatchSmem {
  union {
    double red[BT * 4 + 128];  // sweep row-group partials, z-aux partials, wave maxima
    double tile[64 * 65];      // ingest transpose tile (viewed as S); panel-update operands
  };
  double zc[kBatchMaxN];  // z(l) of the current step, by offset in the column range
  double colss[BT / 64][64];
  double g[kNbMax], aux[kNbMax], vj[kNbMax], vscale[kNbMax], zsum[kNbMax];
  double dscr[BT / 64];
  AmaxVal ascr[BT / 64];
  int cidx[64];
  int piv[kNbMax];
  int item, grp, ngrp;
  int xfail;
  // reduced results of the last exchange
  AmaxVal best;
  int anyflag, anybad;
  float fmax;
  double xnorm2, alpha;
};

template <int BT>
__device__ __forceinline__ double bsum(double v, double* scr) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) scr[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < BT / 64; ++q) t += scr[q];
  __syncthreads();
  return t;
}

template <int BT>
__device__ __forceinline__ AmaxVal bamax(AmaxVal a, AmaxVal* scr) {
  a = wave_amax(a);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) scr[wv] = a;
  __syncthreads();
  AmaxVal r = scr[0];
#pragma unroll
  for (int q = 1; q < BT / 64; ++q) r = amax_combine(r, scr[q]);
  __syncthreads();
  return r;
}

// Publish this workgroup's slot (payload already written) and wait for the
// other G - 1.  Returns false when the item was aborted (uniform).
template <int BT>
__device__ bool exchange(XSlot* xs, int* abortp, int g, int G, int64_t seq, uint64_t wait_ticks,
                         BatchSmem<BT>& sm) {
  // The barrier completes every wave's stores; one device-scope release by
  // thread 0 then publishes them all, and the tag store follows it.
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&xs[g].tag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Lanes 0 .. G-1 of wave 0 poll one tag each with relaxed loads (no cache
  // maintenance while spinning) and acquire once the tags are there.
  if (threadIdx.x < G) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&xs[threadIdx.x].tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           seq) {
      if (__hip_atomic_load(abortp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        sm.xfail = 1;
        break;
      }
      if (wall_clock64() - t0 > wait_ticks) {
        __hip_atomic_store(abortp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sm.xfail = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  const bool ok = sm.xfail == 0;
  __syncthreads();
  return ok;
}

// Exchange A: candidates, flags, panel max |F|; reduced into sm.best etc.
template <int BT>
__device__ bool exchange_a(XSlot* xs, int* abortp, int g, int G, int64_t seq, uint64_t wt,
                           AmaxVal mine, int flag, int bad, float fmax, BatchSmem<BT>& sm) {
  if (G == 1) {
    if (threadIdx.x == 0) {
      sm.best = mine;
      sm.anyflag = flag;
      sm.anybad = bad;
      sm.fmax = fmax;
    }
    __syncthreads();
    return true;
  }
  if (threadIdx.x == 0) {
    XSlot& s = xs[g];
    s.v = mine.v;
    s.s2 = mine.s2;
    s.pos = mine.pos;
    s.key = mine.key;
    s.flag = flag;
    s.bad = bad;
    s.fmax = fmax;
  }
  if (!exchange<BT>(xs, abortp, g, G, seq, wt, sm)) return false;
  if (threadIdx.x == 0) {
    AmaxVal b = amax_none();
    int fl = 0, bd = 0;
    float fm = 0.0f;
    double s2 = 0.0;
    for (int q = 0; q < G; ++q) {  // fixed order: identical in every workgroup
      const XSlot& s = xs[q];
      AmaxVal c;
      c.v = s.v;
      c.s2 = 0.0;
      c.pos = s.pos;
      c.key = s.key;
      b = amax_combine(b, c);
      s2 += s.s2;
      fl |= s.flag;
      bd |= s.bad;
      fm = fmaxf(fm, s.fmax);
    }
    b.s2 = s2;
    sm.best = b;
    sm.anyflag = fl;
    sm.anybad = bd;
    sm.fmax = fm;
  }
  __syncthreads();
  return true;
}

// Largest not-yet-pivoted column norm of the range [cs, cs + cn).
template <int BT>
__device__ AmaxVal range_best(const double* nu, const int* pvflag, const int* cid,
                              const int* posof, int64_t cs, int64_t cn, BatchSmem<BT>& sm) {
  AmaxVal best = amax_none();
  for (int64_t l = cs + threadIdx.x; l < cs + cn; l += BT) {
    if (!pvflag[l]) {
      AmaxVal c;
      c.v = nu[l];
      c.s2 = c.v * c.v;
      c.pos = (int)l;
      c.key = posof[cid[l]];
      best = amax_combine(best, c);
    }
  }
  return bamax<BT>(best, sm.ascr);
}

// Workgroup g of G on one item.  All branches on shared decisions are uniform
// within the workgroup and, through the exchanges, across the G workgroups.
template <typename S, typename TA, int OP, int BT>
__device__ void factor_item(id_batch_item& it, int g, int G, const BatchOpts& o,
                            BatchSmem<BT>& sm) {
  typedef typename BVec<S>::type VT;
  constexpr int VEC = BVec<S>::n;
  constexpr int NW = BT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m = it.m, n = it.n, lda = it.lda;
  const int64_t kcap = batch_kcap(m, n, o.k_fixed, o.k_max);
  const BatchLayout L = batch_layout(m, n, kcap, (int)sizeof(S));
  const BatchItemDev& di = reinterpret_cast<const BatchItemDev&>(it);
  char* wb = (char*)di.work;
  S* const W0 = (S*)(wb + L.off_w0);
  S* const W1 = (S*)(wb + L.off_w1);
  S* V = (S*)(wb + L.off_v);
  double* F = (double*)(wb + L.off_f);
  double* nu = (double*)(wb + L.off_nu);
  double* nuo = (double*)(wb + L.off_nuo);
  int* const colid0 = (int*)(wb + L.off_colid0);
  int* const colid1 = (int*)(wb + L.off_colid1);
  int* pvflag = (int*)(wb + L.off_pvflag);
  int* permw = (int*)(wb + L.off_permw);
  int* posof = (int*)(wb + L.off_posof);
  double* rorig = (double*)(wb + L.off_rorig);
  XSlot* xs = (XSlot*)(wb + L.off_xs);
  int* abortp = (int*)(wb + L.off_abort);
  const int64_t ldw = L.ldw, ldf = L.ldf;
  const TA* A = (const TA*)di.A;
  int32_t* perm_out = (int32_t*)di.perm;
  double* R_out = (double*)di.R;
  const uint64_t wt = o.wait_ticks;
  int64_t seq = 0;

  // This workgroup's column range: the live positions 0 .. ncur-1 split evenly
  // (multiples of 4 positions); re-split after every panel, when the update
  // compacts all ranges into one contiguous layout.
  int64_t ncur = n, cs = 0, cn = 0;
  auto split = [&]() {
    const int64_t span = round_up(ceil_div(ncur > 0 ? ncur : 1, G), 4);
    cs = (int64_t)g * span < ncur ? (int64_t)g * span : ncur;
    cn = ncur - cs < span ? ncur - cs : span;
  };
  split();

  if (tid == 0) sm.xfail = 0;
  for (int64_t l = cs + tid; l < cs + cn; l += BT) {
    colid0[l] = (int)l;
    pvflag[l] = 0;
    permw[l] = (int)l;
    posof[l] = (int)l;
    perm_out[l] = (int)l;
  }
  if (g == 0 && tid == 0) {
    it.k = 0;
    it.info = 0;
  }
  __syncthreads();
  if (m == 0 || n == 0 || kcap == 0) return;

  // ---- ingest of the own columns: W0 (row-major) and FP64 column norms
  double bad = 0.0;
  {
    S* tile = (S*)sm.tile;  // 64 x 65
    for (int64_t c0 = cs; c0 < cs + cn; c0 += 64) {
      const int64_t cend = cs + cn;
      double ss = 0.0;
      for (int64_t r0 = 0; r0 < m; r0 += 64) {
        for (int e = tid; e < 4096; e += BT) {
          const int rr = e & 63, cc = e >> 6;
          const int64_t r = r0 + rr, c = c0 + cc;
          S v = (S)0;
          if (r < m && c < cend) {
            const TA x = A[c * lda + r];
            if (!isfinite((double)x)) bad = 1.0;
            v = (S)x;
          }
          tile[cc * 65 + rr] = v;
        }
        __syncthreads();
        for (int e = tid; e < 4096; e += BT) {
          const int cc = e & 63, rr = e >> 6;  // cc == lane
          const int64_t r = r0 + rr, c = c0 + cc;
          if (r < m && c < cend) {
            const S v = tile[cc * 65 + rr];
            W0[r * ldw + c] = v;
            ss += (double)v * (double)v;
          }
        }
        __syncthreads();
      }
      sm.colss[wv][lane] = ss;
      __syncthreads();
      if (tid < 64 && c0 + tid < cend) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) t += sm.colss[q][tid];
        nu[c0 + tid] = sqrt(t);
        nuo[c0 + tid] = sqrt(t);
      }
      __syncthreads();
    }
  }
  const int bad_any = bsum<BT>(bad, sm.dscr) > 0.0;

  int64_t off = 0, kout = 0;
  int cur = 0, jb = 0;
  double r00 = 0.0, fro2 = 0.0;
  AmaxVal mine = range_best<BT>(nu, pvflag, colid0, posof, cs, cn, sm);
  int myflag = 0;
  float myfmax = 0.0f;
  bool aborted = false;
  for (;;) {
    // ---- exchange A: pivot candidates, panel-end flags, panel max |F|
    if (!exchange_a<BT>(xs, abortp, g, G, ++seq, wt, mine, myflag, bad_any, myfmax, sm)) {
      aborted = true;
      break;
    }
    if (sm.anybad) {
      if (g == 0 && tid == 0) it.info = ID_INFO_NONFINITE;
      return;
    }
    if (jb > 0 && (sm.anyflag || jb >= o.nb)) {
      // ---- end of panel: W_next = W - V F^T on rows >= off + jb for the own
      //      columns, compacted, with the FP64 recomputation of their norms
      const int64_t jend = off + jb;
      S* Wc = cur ? W1 : W0;
      int* cid = cur ? colid1 : colid0;
      S* Wn = cur ? W0 : W1;
      int* cidn = cur ? colid0 : colid1;
      const int g4 = lane >> 4, li = lane & 15;
      int sF = 0, sV = 0;
      if (OP == BOP_F16) {
        int e = 0;
        if (sm.fmax > 0.0f) frexpf(sm.fmax, &e);
        sF = 15 - e;
        sV = 14;
      }
      const double fscl = ldexp(1.0, sF);
      const float vscl = ldexpf(1.0f, sV);
      const double descale = ldexp(1.0, -(sF + sV));
      // new positions: all of the panel's pivots leave, whatever range they
      // were in, so the next panel's layout is contiguous
      for (int64_t l0 = cs; l0 < cs + cn; l0 += 64) {
        if (tid < 64) {
          const int64_t l = l0 + tid;
          int before = 0;
          bool pv = false;
          for (int c = 0; c < jb; ++c) {
            before += sm.piv[c] < l;
            pv |= sm.piv[c] == l;
          }
          sm.cidx[tid] = (l < cs + cn && !pv) ? (int)(l - before) : -1;
        }
        // B operands (F at the positions l0 .. l0 + 63) staged in LDS in the lane
        // order of the matrix-core instruction: lane (lg, ll) of position block
        // lb holds F(l0 + 16 lb + ll, c) for its k indices c = 8 lg + e
        for (int idx = tid; idx < 256; idx += BT) {
          const int lb = idx >> 6, ln = idx & 63, lg = ln >> 4, ll = ln & 15;
          const int64_t pos = l0 + 16 * lb + ll;
          const bool pok = pos < cs + cn;
          if (OP == BOP_F64) {
            double* fb = sm.tile + lb * 512 + ln;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * lg + e;
              fb[e * 64] = (c < jb && pok) ? F[(int64_t)c * ldf + pos] : 0.0;
            }
          } else if (OP == BOP_F32) {
            float* fb = (float*)sm.tile + lb * 512 + ln;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * lg + e;
              fb[e * 64] = (c < jb && pok) ? (float)F[(int64_t)c * ldf + pos] : 0.0f;
            }
          } else {
            f16x8 xh;
            bf16x8 xb, xl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * lg + e;
              const float x = (c < jb && pok) ? (float)(F[(int64_t)c * ldf + pos] * fscl) : 0.0f;
              xh[e] = (_Float16)x;
              const __bf16 h = (__bf16)x;
              xb[e] = h;
              xl[e] = (__bf16)(x - (float)h);
            }
            if (OP == BOP_F16) {
              ((f16x8*)sm.tile)[idx] = xh;
            } else {
              ((bf16x8*)sm.tile)[idx] = xb;
              ((bf16x8*)sm.tile)[256 + idx] = xl;
            }
          }
        }
        __syncthreads();
        // Each wave takes 16 rows at a time: the product tile (16 rows x 64
        // positions) has the matrix rows along the instruction's M side, so a
        // lane's results are one position of four rows and the 16 lanes of a
        // group cover 16 consecutive positions (coalesced loads and stores).
        double ssl[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t rs = jend + 16 * wv; rs < m; rs += 16 * NW) {
          // A operand: V(rs + li, 8 g4 .. 8 g4 + 7), one row-major 8-vector
          const int64_t arow = rs + li;
          S va[8];
          if (arow < m && 8 * g4 < jb) {
            const S* vp = V + arow * kNbMax + 8 * g4;
#pragma unroll
            for (int q = 0; q < 8 / VEC; ++q) {
              const VT t = *(const VT*)(vp + q * VEC);
#pragma unroll
              for (int e = 0; e < VEC; ++e) va[q * VEC + e] = t[e];
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) va[e] = (S)0;
          }
          // output rows of this lane: rs + g4 + 4 r (FP64 instruction) or
          // rs + 4 g4 + r (FP16/BF16 instruction)
          S wv4[4][4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t orow = OP == BOP_F64 ? rs + g4 + 4 * r : rs + 4 * g4 + r;
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
              const int64_t pos = l0 + 16 * lb + li;
              wv4[lb][r] = (orow < m && pos < cs + cn) ? Wc[orow * ldw + pos] : (S)0;
            }
          }
          if (OP == BOP_F64) {
            double a64[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * g4 + e;
              a64[e] = c < jb ? (double)va[e] * sm.vscale[c] : 0.0;
            }
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
              const double* fb = sm.tile + lb * 512 + lane;
              f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int e = 0; e < 8; ++e)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a64[e], fb[e * 64], acc, 0, 0, 0);
              const int ci = sm.cidx[16 * lb + li];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int64_t orow = rs + g4 + 4 * r;
                if (orow < m && ci >= 0) {
                  const S v = (S)((double)wv4[lb][r] - acc[r]);
                  Wn[orow * ldw + ci] = v;
                  ssl[lb] += (double)v * (double)v;
                }
              }
            }
          } else if (OP == BOP_F32) {
            float a32[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * g4 + e;
              a32[e] = c < jb ? (float)((double)va[e] * sm.vscale[c]) : 0.0f;
            }
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
              const float* fb = (const float*)sm.tile + lb * 512 + lane;
              f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int e = 0; e < 8; ++e)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[e], fb[e * 64], acc, 0, 0, 0);
              const int ci = sm.cidx[16 * lb + li];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int64_t orow = rs + 4 * g4 + r;
                if (orow < m && ci >= 0) {
                  const S v = (S)((double)wv4[lb][r] - (double)acc[r]);
                  Wn[orow * ldw + ci] = v;
                  ssl[lb] += (double)v * (double)v;
                }
              }
            }
          } else {
            f16x8 ah;
            bf16x8 ab, abl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 8 * g4 + e;
              const float x = c < jb ? (float)((double)va[e] * sm.vscale[c]) * vscl : 0.0f;
              if (OP == BOP_F16) {
                ah[e] = (_Float16)x;
              } else {
                const __bf16 h = (__bf16)x;
                ab[e] = h;
                if (OP == BOP_BF16X3) abl[e] = (__bf16)(x - (float)h);
              }
            }
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
              f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
              if (OP == BOP_F16) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    ah, ((const f16x8*)sm.tile)[lb * 64 + lane], acc, 0, 0, 0);
              } else if (OP == BOP_BF16) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    ab, ((const bf16x8*)sm.tile)[lb * 64 + lane], acc, 0, 0, 0);
              } else {
                const bf16x8 bhi = ((const bf16x8*)sm.tile)[lb * 64 + lane];
                const bf16x8 blo = ((const bf16x8*)sm.tile)[256 + lb * 64 + lane];
                // small terms first, then the leading product
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(abl, bhi, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, blo, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bhi, acc, 0, 0, 0);
              }
              const int ci = sm.cidx[16 * lb + li];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int64_t orow = rs + 4 * g4 + r;
                if (orow < m && ci >= 0) {
                  const S v = (S)((double)wv4[lb][r] - (double)acc[r] * descale);
                  Wn[orow * ldw + ci] = v;
                  ssl[lb] += (double)v * (double)v;
                }
              }
            }
          }
        }
        // column sums of squares: over the four lane groups, then the waves
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
          double x = ssl[lb];
          x += __shfl_xor(x, 16, 64);
          x += __shfl_xor(x, 32, 64);
          if (g4 == 0) sm.colss[wv][16 * lb + li] = x;
        }
        __syncthreads();
        if (tid < 64 && sm.cidx[tid] >= 0) {
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) t += sm.colss[q][tid];
          const int np = sm.cidx[tid];
          nu[np] = sqrt(t);
          nuo[np] = sqrt(t);
          pvflag[np] = 0;
          cidn[np] = cid[l0 + tid];
        }
        __syncthreads();
      }
      off += jb;
      ncur -= jb;
      split();
      cur ^= 1;
      jb = 0;
      // the new ranges hold columns other workgroups just wrote: wait for them
      if (G > 1 && !exchange<BT>(xs, abortp, g, G, ++seq, wt, sm)) {
        aborted = true;
        break;
      }
      mine = range_best<BT>(nu, pvflag, cur ? colid1 : colid0, posof, cs, cn, sm);
      myflag = 0;
      myfmax = 0.0f;
      if (!exchange_a<BT>(xs, abortp, g, G, ++seq, wt, mine, 0, 0, 0.0f, sm)) {
        aborted = true;
        break;
      }
    }

    const int64_t j = off + jb;
    S* Wc = cur ? W1 : W0;
    int* cid = cur ? colid1 : colid0;
    // ---- 1. pivot and rank rule (identical decisions in every workgroup)
    const AmaxVal best = sm.best;
    const int p = best.pos;
    const double vp = best.v;
    if (j == 0) fro2 = best.s2;
    bool stop = (j >= kcap) || (p < 0);
    if (!stop && o.k_fixed == 0) {
      if (!(vp > 0.0))
        stop = true;
      else if (o.rule == ID_RANK_PIVOT_REL)
        stop = j > 0 && vp <= o.rel_tol * r00;
      else
        stop = sqrt(best.s2) <= o.rel_tol * sqrt(fro2);
    }
    if (stop) {
      kout = j;
      break;
    }
    const bool owner = p >= cs && p < cs + cn;
    if (tid == 0) {
      sm.piv[jb] = p;
      if (owner) pvflag[p] = 1;
      if (g == 0) {
        const int q = cid[p];
        const int pa = posof[q];
        const int other = permw[j];
        permw[pa] = other;
        posof[other] = pa;
        permw[j] = q;
        posof[q] = (int)j;
      }
    }
    if (tid < kNbMax) sm.g[tid] = tid < jb ? sm.vscale[tid] * F[(int64_t)tid * ldf + p] : 0.0;
    __syncthreads();

    // ---- 2. pivot column w = W(:,p) - V F(p,:)^T on this workgroup's slice of
    //         the rows j .. m-1, stored as reflector jb; its partial sums
    const int64_t slice = ceil_div(m - j, G);
    const int64_t rlo = j + (int64_t)g * slice;
    const int64_t rhi = rlo + slice < m ? rlo + slice : m;
    // One pass over the slice: each row's reflector entries are loaded once and
    // serve both w(i) and the partial sums V(i, c) w(i) (i > j).
    double nn = 0.0;
    double zacc[kNbMax];
#pragma unroll
    for (int c = 0; c < kNbMax; ++c) zacc[c] = 0.0;
    for (int64_t i = rlo + tid; i < rhi; i += BT) {
      S vr[kNbMax];
      const S* vrow = V + i * kNbMax;
#pragma unroll
      for (int cb = 0; cb < kNbMax; cb += VEC) {
        if (cb < jb) {  // uniform
          const VT t = *(const VT*)(vrow + cb);
#pragma unroll
          for (int e = 0; e < VEC; ++e) vr[cb + e] = cb + e < jb ? t[e] : (S)0;
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) vr[cb + e] = (S)0;
        }
      }
      double w = (double)Wc[i * ldw + p];
#pragma unroll
      for (int c = 0; c < kNbMax; ++c) w -= (double)vr[c] * sm.g[c];
      V[i * kNbMax + jb] = (S)w;
      if (i == j) {
        sm.alpha = w;
      } else {
        nn += w * w;
#pragma unroll
        for (int c = 0; c < kNbMax; ++c) zacc[c] += (double)vr[c] * w;
      }
    }
    const double nn_part = bsum<BT>(nn, sm.dscr);  // barrier: the slice of column jb is visible
#pragma unroll
    for (int c = 0; c < kNbMax; ++c) {
      if (c < jb) {  // uniform
        const double z = wave_sum(zacc[c]);
        if (lane == 0) sm.red[wv * kNbMax + c] = z;
      }
    }
    __syncthreads();
    if (tid < jb) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) t += sm.red[q * kNbMax + tid];
      sm.zsum[tid] = t;
    }
    __syncthreads();
    // ---- exchange B: the partial sums, combined in workgroup order
    if (G == 1) {
      if (tid == 0) {
        sm.xnorm2 = nn_part;
        // sm.alpha already holds w(j)
      }
      __syncthreads();
    } else {
      XSlot& s = xs[g];
      if (tid == 0) {
        s.nrm2 = nn_part;
        s.alpha = g == 0 ? sm.alpha : 0.0;
      }
      if (tid < jb) s.zsum[tid] = sm.zsum[tid];
      if (!exchange<BT>(xs, abortp, g, G, ++seq, wt, sm)) {
        aborted = true;
        break;
      }
      if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += xs[q].nrm2;
        sm.xnorm2 = t;
        sm.alpha = xs[0].alpha;
      }
      if (tid < jb) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += xs[q].zsum[tid];
        sm.zsum[tid] = t;
      }
      __syncthreads();
    }
    // ---- 3. reflector (dlarfg conventions), the same in every workgroup
    const double alpha = sm.alpha, xnorm2 = sm.xnorm2;
    double beta, tau, scale;
    if (xnorm2 == 0.0) {
      beta = alpha;
      tau = 0.0;
      scale = 0.0;
    } else {
      const double h = hypot(alpha, sqrt(xnorm2));
      beta = alpha >= 0.0 ? -h : h;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (j == 0) r00 = fabs(beta);
    if (tid < jb) {
      const double vjc = sm.vscale[tid] * (double)V[j * kNbMax + tid];
      sm.vj[tid] = vjc;
      sm.aux[tid] = vjc + sm.vscale[tid] * scale * sm.zsum[tid];
    }
    // ---- 4. sweep of the own columns: z(l) = sum_{i>j} W(i,l) w(i)
    {
      int tpr = 16;
      while (tpr < BT && (int64_t)tpr * VEC < cn) tpr *= 2;
      const int RG = BT / tpr;
      const int rg = tid / tpr, cv = tid % tpr;
      const S* wcol = V + jb;  // w(i) at wcol[i * kNbMax]
      for (int64_t cb = 0; cb < cn; cb += (int64_t)tpr * VEC) {
        const int64_t l0 = cb + (int64_t)cv * VEC;  // offset in the range
        double acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0.0;
        if (l0 < cn) {
          const S* base = Wc + cs + l0;
          int64_t i = j + 1 + rg;
          // U independent row loads in flight per thread (U * BT * VEC * s bytes
          // per workgroup) to cover the memory latency of one compute unit
          constexpr int U = BT >= 512 ? 8 : 16;
          for (; i + (U - 1) * RG < m; i += U * RG) {
            VT x[U];
            double w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = *(const VT*)(base + (i + u * RG) * ldw);
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = (double)wcol[(i + u * RG) * kNbMax];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc[e] += (double)x[u][e] * w[u];
          }
          for (; i < m; i += RG) {
            const VT x0 = *(const VT*)(base + i * ldw);
            const double w0 = (double)wcol[i * kNbMax];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += (double)x0[e] * w0;
          }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < VEC; ++e) sm.red[tid * VEC + e] = acc[e];
        __syncthreads();
        if (rg == 0 && l0 < cn) {
          for (int q = 1; q < RG; ++q)
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += sm.red[(q * tpr + cv) * VEC + e];
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (l0 + e < cn) sm.zc[l0 + e] = acc[e];
        }
      }
      __syncthreads();
    }
    // ---- 5. own columns: new F column, R row, downdated norms, next candidate
    double flag = 0.0;
    float fm = 0.0f;
    AmaxVal cand = amax_none();
    for (int64_t l = cs + tid; l < cs + cn; l += BT) {
      // the column's own data first (one group with the F loads below), its
      // swap-order key (which depends on the id) right after the F loads
      const double wj = (double)Wc[j * ldw + l];
      const int pvl = pvflag[l];
      const int id = cid[l];
      double nl = nu[l];
      const double nlo = nuo[l];
      const double y = wj + scale * sm.zc[l - cs];
      double s1 = 0.0, s2 = 0.0;
      int key = 0;
      // F(c, l) for c < jb, loaded 16 rows at a time as one group (rows
      // >= jb hold stale data: excluded by the select on the products)
      for (int c0 = 0; c0 < jb; c0 += 16) {
        double fc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) fc[u] = F[(int64_t)((c0 + u) & (kNbMax - 1)) * ldf + l];
        if (c0 == 0) key = posof[id];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int c = c0 + u;
          s1 += c < jb ? fc[u] * sm.aux[c & (kNbMax - 1)] : 0.0;
          s2 += c < jb ? sm.vj[c & (kNbMax - 1)] * fc[u] : 0.0;
        }
      }
      if (jb == 0) key = posof[id];
      const double f = tau * (y - s1);
      F[(int64_t)jb * ldf + l] = f;
      if (!pvl) {
        const double r = wj - s2 - f;
        rorig[(int64_t)id * kcap + j] = r;
        if (nl != 0.0) {
          double t = fabs(r) / nl;
          t = (1.0 + t) * (1.0 - t);
          if (t < 0.0) t = 0.0;
          const double ratio = nl / nlo;
          if (t * ratio * ratio <= o.tol3z) {
            flag = 1.0;
          } else {
            nl = nl * sqrt(t);
            nu[l] = nl;
          }
        }
        fm = fmaxf(fm, (float)fabs(f));
        AmaxVal c;
        c.v = nl;
        c.s2 = nl * nl;
        c.pos = (int)l;
        c.key = key;
        cand = amax_combine(cand, c);
      }
    }
    if (tid == 0) {
      if (owner) rorig[(int64_t)cid[p] * kcap + j] = beta;
      sm.vscale[jb] = scale;
    }
    {
      float x = fm;
#pragma unroll
      for (int offs = 32; offs > 0; offs >>= 1) x = fmaxf(x, __shfl_xor(x, offs, 64));
      if (lane == 0) sm.red[wv] = (double)x;
    }
    __syncthreads();
    float fm_blk = 0.0f;
#pragma unroll
    for (int q = 0; q < NW; ++q) fm_blk = fmaxf(fm_blk, (float)sm.red[q]);
    myfmax = fmaxf(jb == 0 ? 0.0f : myfmax, fm_blk);
    myflag = bsum<BT>(flag, sm.dscr) > 0.0 ? 1 : 0;
    mine = bamax<BT>(cand, sm.ascr);  // its barriers also publish F, vscale
    ++jb;
    if (j + 1 >= kcap) {
      kout = j + 1;
      // one more exchange so that every workgroup's R entries are visible
      if (!exchange_a<BT>(xs, abortp, g, G, ++seq, wt, mine, 0, 0, 0.0f, sm)) aborted = true;
      break;
    }
  }
  if (aborted) {
    if (tid == 0) {
      it.k = 0;
      it.info = ID_INFO_ABORTED;
    }
    return;
  }
  if (g != 0) return;

  // ---- outputs (workgroup 0): k, perm (swap order), R in pivot order; R11
  //      checked for numerical singularity (T is then left unwritten)
  const int64_t k = kout;
  for (int64_t l = tid; l < n; l += BT) perm_out[l] = permw[l];
  for (int64_t e = tid; e < k * n; e += BT) {
    const int64_t c = e / k, i = e % k;
    const int id = permw[c];
    R_out[c * it.ldr + i] = (c >= k || i <= c) ? rorig[(int64_t)id * kcap + i] : 0.0;
  }
  __syncthreads();
  double sing = 0.0;
  if (k > 0) {
    const double d0 = fabs(R_out[0]);
    const double thr = (double)n * ldexp(1.0, -53) * d0;
    for (int64_t i = tid; i < k; i += BT)
      if (!(fabs(R_out[i * it.ldr + i]) > thr)) sing = 1.0;
  }
  sing = bsum<BT>(sing, sm.dscr);
  if (tid == 0) {
    it.k = k;
    it.info = sing > 0.0 ? ID_INFO_SINGULAR : (k == n ? ID_INFO_RANK_FULL : 0);
  }
}

// Resets the work counter and every item's exchange area (tags, abort flag);
// runs on the stream before the factorization.
template <typename S>
__global__ void k_batch_prepare(id_batch_item* items, int32_t batch, int32_t* queue, int64_t k_fixed,
                                int64_t k_max) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *queue = 0;
  if (t >= (int64_t)batch * (kBatchMaxGroups + 1)) return;
  const int i = (int)(t / (kBatchMaxGroups + 1)), q = (int)(t % (kBatchMaxGroups + 1));
  const id_batch_item& it = items[i];
  const BatchLayout L = batch_layout(it.m, it.n, batch_kcap(it.m, it.n, k_fixed, k_max),
                                     (int)sizeof(S));
  char* wb = (char*)it.work;
  if (q < kBatchMaxGroups)
    ((XSlot*)(wb + L.off_xs))[q].tag = 0;
  else
    *(int*)(wb + L.off_abort) = 0;
}

template <typename S, typename TA, int OP, int BT>
__global__ __launch_bounds__(BT) void k_batched_factor(id_batch_item* items, int32_t batch,
                                                       const int32_t* slots, int32_t nslots,
                                                       int32_t* queue, BatchOpts o) {
  __shared__ BatchSmem<BT> sm;
  for (;;) {
    if (threadIdx.x == 0) {
      const int q = atomicAdd(queue, 1);
      int item = -1, g = 0, G = 1;
      if (q < nslots) {
        item = slots ? slots[q] : q;
        if (item < 0 || item >= batch) {
          item = -2;  // malformed slot: skipped
        } else {
          G = slots ? items[item].groups : 1;
          G = G < 1 ? 1 : (G > kBatchMaxGroups ? kBatchMaxGroups : G);
          // position within the run of equal entries ending at q
          while (g < G && q - g - 1 >= 0 && slots && slots[q - g - 1] == item) ++g;
          if (g >= G) {
            item = -2;
          } else if (G > (int)gridDim.x) {
            // its G workgroups can never all be running: the first marks the
            // item abandoned at once instead of waiting for the others
            if (g == 0) {
              items[item].k = 0;
              items[item].info = ID_INFO_ABORTED;
            }
            item = -2;
          }
        }
      }
      sm.item = item;
      sm.grp = g;
      sm.ngrp = G;
    }
    __syncthreads();
    const int item = sm.item, g = sm.grp, G = sm.ngrp;
    __syncthreads();
    if (item == -1) return;  // the queue is drained: every workgroup leaves
    if (item >= 0) factor_item<S, TA, OP, BT>(items[item], g, G, o, sm);
    __syncthreads();
  }
}

size_t batch_item_workspace(int64_t m, int64_t n, const id_opts* o) {
  if (!o || m < 0 || n < 0 || n > kBatchMaxN) return 0;
  if (o->prec < ID_PREC_F64 || o->prec > ID_PREC_MIXED_F32) return 0;
  const int wb = o->prec == ID_PREC_F64 ? 8 : 4;
  return batch_layout(m, n, batch_kcap(m, n, o->k_fixed, o->k_max), wb).bytes;
}

template <typename S, typename TA, int OP>
static int launch_batched(id_batch_item* items, int32_t batch, const int32_t* slots,
                          int32_t nslots, int32_t* queue, const BatchOpts& bo, int bt, int groups,
                          hipStream_t s) {
  const int64_t nprep = (int64_t)batch * (kBatchMaxGroups + 1);
  k_batch_prepare<S><<<dim3((unsigned)ceil_div(nprep > 0 ? nprep : 1, 256)), 256, 0, s>>>(
      items, batch, queue, bo.k_fixed, bo.k_max);
  MPID_LAUNCH_CHECK();
  const dim3 grid((unsigned)groups);
  if (bt == 256)
    k_batched_factor<S, TA, OP, 256><<<grid, 256, 0, s>>>(items, batch, slots, nslots, queue, bo);
  else
    k_batched_factor<S, TA, OP, 512><<<grid, 512, 0, s>>>(items, batch, slots, nslots, queue, bo);
  MPID_LAUNCH_CHECK();
  return ID_OK;
}

int factor_batched_run(id_batch_item* items, int32_t batch, const int32_t* slots, int32_t nslots,
                       int32_t* queue, int64_t max_n, int32_t dtype, const id_opts* o,
                       int32_t block_threads, int32_t num_groups, hipStream_t s) {
  if (!o || !items || !queue || batch < 0) return ID_ERR_ARG;
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (o->prec < ID_PREC_F64 || o->prec > ID_PREC_MIXED_F32) return ID_ERR_DTYPE;
  if (o->flags != 0 || o->k_fixed < 0 || o->k_max < 0 || !(o->rel_tol >= 0.0)) return ID_ERR_ARG;
  if (o->rank_rule != ID_RANK_PIVOT_REL && o->rank_rule != ID_RANK_FROB_REL) return ID_ERR_ARG;
  const int nb = o->nb == 0 ? kNbMax : o->nb;
  if (nb < 1 || nb > kNbMax) return ID_ERR_ARG;
  if (max_n < 0 || max_n > kBatchMaxN) return ID_ERR_UNSUPPORTED;
  const int bt = block_threads == 0 ? 512 : block_threads;
  if (bt != 256 && bt != 512) return ID_ERR_ARG;
  if (!slots) nslots = batch;
  if (nslots < 0) return ID_ERR_ARG;
  if (batch == 0) return ID_OK;
  int dev = 0, cus = 0, rate_khz = 0;
  MPID_HIP(hipGetDevice(&dev));
  MPID_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  MPID_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  int groups = num_groups;
  if (groups <= 0) groups = cus > 0 ? cus : 256;
  // every workgroup of the grid must be resident at once for the shared items
  // to progress: at most one per compute unit
  if (cus > 0 && groups > cus) groups = cus;
  if (groups > nslots) groups = nslots > 0 ? nslots : 1;
  BatchOpts bo;
  bo.k_fixed = o->k_fixed;
  bo.k_max = o->k_max;
  bo.rel_tol = o->rel_tol;
  bo.rule = o->rank_rule;
  bo.nb = nb;
  const bool f64w = o->prec == ID_PREC_F64;
  bo.tol3z = std::sqrt(f64w ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
  // one exchange wait gives up after 20 s
  bo.wait_ticks = (uint64_t)(rate_khz > 0 ? rate_khz : 100000) * 1000ull * 20ull;
  int rc;
  if (f64w) {
    rc = dtype == ID_F64
             ? launch_batched<double, double, BOP_F64>(items, batch, slots, nslots, queue, bo, bt, groups, s)
             : launch_batched<double, float, BOP_F64>(items, batch, slots, nslots, queue, bo, bt, groups, s);
  } else if (o->prec == ID_PREC_MIXED_F16) {
    rc = dtype == ID_F64
             ? launch_batched<float, double, BOP_F16>(items, batch, slots, nslots, queue, bo, bt, groups, s)
             : launch_batched<float, float, BOP_F16>(items, batch, slots, nslots, queue, bo, bt, groups, s);
  } else if (o->prec == ID_PREC_MIXED_F32) {
    rc = dtype == ID_F64
             ? launch_batched<float, double, BOP_F32>(items, batch, slots, nslots, queue, bo, bt, groups, s)
             : launch_batched<float, float, BOP_F32>(items, batch, slots, nslots, queue, bo, bt, groups, s);
  } else if (o->prec == ID_PREC_MIXED_BF16) {
    rc = dtype == ID_F64
             ? launch_batched<float, double, BOP_BF16>(items, batch, slots, nslots, queue, bo, bt, groups, s)
             : launch_batched<float, float, BOP_BF16>(items, batch, slots, nslots, queue, bo, bt, groups, s);
  } else {
    rc = dtype == ID_F64
             ? launch_batched<float, double, BOP_BF16X3>(items, batch, slots, nslots, queue, bo, bt, groups, s)
             : launch_batched<float, float, BOP_BF16X3>(items, batch, slots, nslots, queue, bo, bt, groups, s);
  }
  if (rc) return rc;
  return trsm_batched_run(items, batch, max_n, s);
}

}  // namespace mpid
