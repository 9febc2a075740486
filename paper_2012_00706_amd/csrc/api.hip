// extern "C" entry points of libmpid (declared in include/mpid.h).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>

#include "mpid.h"
#include "mpid_internal.h"

namespace mpid {

int log_level() {
  const char* v = std::getenv("MPID_LOG");
  return (v && *v) ? std::atoi(v) : 0;
}

void log_printf(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fputs("[mpid] ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
}

}  // namespace mpid

extern "C" {

size_t id_workspace_size(int64_t m, int64_t n, int32_t dtype, const id_opts* opts) {
  if (opts && (opts->flags & ID_FLAG_GRAM) && (opts->flags & ID_FLAG_CHOLQR)) return 0;
  if (opts && (opts->flags & ID_FLAG_GRAM)) return mpid::gram_workspace(m, n, dtype, opts);
  if (opts && (opts->flags & ID_FLAG_CHOLQR)) return mpid::cholqr_workspace(m, n, dtype, opts);
  mpid::FactorPlan p;
  if (!mpid::make_factor_plan(m, n, dtype, opts, &p)) return 0;
  return p.bytes;
}

int id_factor(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
              const id_opts* opts, void* work, size_t work_bytes, int32_t* perm, double* R,
              int64_t ldr, int64_t* k_out, int32_t* info, void* stream) {
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (!opts) return ID_ERR_ARG;
  if (opts->prec != ID_PREC_F64 && opts->prec != ID_PREC_MIXED_F16 &&
      opts->prec != ID_PREC_MIXED_BF16 && opts->prec != ID_PREC_MIXED_BF16X3 &&
      opts->prec != ID_PREC_MIXED_F32)
    return ID_ERR_DTYPE;
  if ((opts->flags & ID_FLAG_GRAM) && (opts->flags & ID_FLAG_CHOLQR)) return ID_ERR_ARG;
  if (opts->flags & ID_FLAG_GRAM)
    return mpid::gram_factor_run(A, dtype, m, n, lda, opts, work, work_bytes, perm, R, ldr, k_out,
                                 info, (hipStream_t)stream);
  if (opts->flags & ID_FLAG_CHOLQR)
    return mpid::cholqr_factor_run(A, dtype, m, n, lda, opts, work, work_bytes, perm, R, ldr,
                                   k_out, info, (hipStream_t)stream);
  return mpid::factor_run(A, dtype, m, n, lda, opts, work, work_bytes, perm, R, ldr, k_out, info,
                          (hipStream_t)stream);
}

int id_solve_T(const double* R, int64_t ldr, int64_t k, int64_t n, double* T, int64_t ldt,
               int32_t* info, void* stream) {
  return mpid::solve_T_run(R, ldr, k, n, T, ldt, info, (hipStream_t)stream);
}

int id_round(double* X, int64_t rows, int64_t cols, int64_t ld, int32_t mode, void* stream) {
  return mpid::round_run(X, rows, cols, ld, mode, (hipStream_t)stream);
}

int id_reconstruct(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                   const int32_t* perm, int64_t k, const double* T, int64_t ldt, double* Y,
                   int64_t ldy, int32_t residual, void* stream) {
  return mpid::reconstruct_run(A, dtype, m, n, lda, perm, k, T, ldt, Y, ldy, residual,
                               (hipStream_t)stream);
}

size_t id_backward_workspace_size(int64_t m, int64_t n, int64_t k) {
  return mpid::backward_workspace(m, n, k);
}

int id_backward(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                const int32_t* perm, int64_t k, const double* T, int64_t ldt, const double* Rb,
                int64_t ldrb, const double* gT, int64_t ldgt, const double* gY, int64_t ldgy,
                double* gA, int64_t ldga, void* work, size_t work_bytes, int32_t* info,
                void* stream) {
  return mpid::backward_run(A, dtype, m, n, lda, perm, k, T, ldt, Rb, ldrb, gT, ldgt, gY, ldgy,
                            gA, ldga, work, work_bytes, info, (hipStream_t)stream);
}

size_t id_sketch_workspace_size(int64_t l, int64_t m, int64_t n) {
  return mpid::sketch_workspace(l, m, n);
}

int id_sketch(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
              const double* Omega, int64_t l, int64_t ldo, double* Y, int64_t ldy, void* work,
              size_t work_bytes, void* stream) {
  return mpid::sketch_run(A, dtype, m, n, lda, Omega, l, ldo, Y, ldy, work, work_bytes,
                          (hipStream_t)stream);
}

size_t id_batch_item_workspace_size(int64_t m, int64_t n, const id_opts* opts) {
  return mpid::batch_item_workspace(m, n, opts);
}

int id_factor_batched(id_batch_item* items, int32_t batch, const int32_t* slots, int32_t nslots,
                      int32_t* queue, int64_t max_n, int32_t dtype, const id_opts* opts,
                      int32_t block_threads, int32_t num_groups, void* stream) {
  return mpid::factor_batched_run(items, batch, slots, nslots, queue, max_n, dtype, opts,
                                  block_threads, num_groups, (hipStream_t)stream);
}

size_t id_lockstep_workspace_size(const id_batch_item* items, int32_t batch, int32_t dtype,
                                  const id_opts* opts) {
  return mpid::lockstep_workspace(items, batch, dtype, opts);
}

int id_factor_lockstep(id_batch_item* items, int32_t batch, int32_t dtype, const id_opts* opts,
                       void* work, size_t work_bytes, void* stream) {
  return mpid::lockstep_run(items, batch, dtype, opts, work, work_bytes, (hipStream_t)stream);
}

int id_last_profile(id_profile* out) {
  if (!out) return ID_ERR_ARG;
  mpid::last_profile(out);
  return ID_OK;
}

const char* id_status_string(int code) {
  switch (code) {
    case ID_OK:
      return "ok";
    case ID_ERR_ARG:
      return "invalid argument";
    case ID_ERR_DTYPE:
      return "unknown dtype or precision";
    case ID_ERR_WORKSPACE:
      return "workspace too small";
    case ID_ERR_HIP:
      return "HIP runtime error";
    case ID_ERR_UNSUPPORTED:
      return "unsupported combination";
    case ID_ERR_SCRATCH:
      return "problem larger than the static scratch of id_factor_noalloc";
    case ID_INFO_NONFINITE:
      return "input holds NaN or Inf";
    case ID_INFO_SINGULAR:
      return "R11 is numerically singular";
    case ID_INFO_RANK_FULL:
      return "full rank: k == n";
    case ID_INFO_ABORTED:
      return "batched item abandoned: a workgroup sharing it did not arrive in time";
    case ID_INFO_GRAM_LIMIT:
      return "Gram front end stopped at its resolution floor (k is the steps completed)";
    case ID_INFO_CHOLQR_BREAKDOWN:
      return "CholeskyQR front end: A lacks full numerical column rank (nothing factored)";
    default:
      return "unknown code";
  }
}

}  // extern "C"
