// id_factor_noalloc: the column-pivoted QR of id_factor for callers that
// cannot allocate device or pinned memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  Its workspace is a static
// device array of this file; everything else is id_factor's own code path.
//
// In host code the array's name is only a host-side stand-in: its device
// address on each GPU comes from hipGetSymbolAddress, looked up once per
// device with that device current, and only that address is ever passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mpid.h"
#include "mpid_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)ID_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

// The workspace of every allocation-free call on a GPU (each GPU holds its
// own copy until the process ends).  Never used by name outside the lookup.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of scratch, per device (null: not looked up)

// The device address of scratch on the current device; 0 on success.
int scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ID_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ID_ERR_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return ID_OK;
}

}  // namespace

extern "C" {

size_t id_noalloc_scratch_bytes(void) { return kScratchBytes; }

int id_factor_noalloc(const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                      const id_opts* opts, int32_t* perm, double* R, int64_t ldr, int64_t* k_out,
                      int32_t* info, void* stream) {
  if (dtype != ID_F32 && dtype != ID_F64) return ID_ERR_DTYPE;
  if (!opts) return ID_ERR_ARG;
  if (opts->prec != ID_PREC_F64 && opts->prec != ID_PREC_MIXED_F16 &&
      opts->prec != ID_PREC_MIXED_BF16 && opts->prec != ID_PREC_MIXED_BF16X3 &&
      opts->prec != ID_PREC_MIXED_F32)
    return ID_ERR_DTYPE;
  if (opts->flags & (ID_FLAG_GRAM | ID_FLAG_CHOLQR | ID_FLAG_PROFILE)) return ID_ERR_UNSUPPORTED;
  mpid::FactorPlan pl;
  if (!mpid::make_factor_plan(m, n, dtype, opts, &pl)) return ID_ERR_ARG;
  if (pl.bytes > kScratchBytes) return ID_ERR_SCRATCH;
  // the stream must belong to the current device (whose scratch is used)
  if (stream) {
    int sdev = -1, cur = -1;
    if (hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess) return ID_ERR_HIP;
    if (hipGetDevice(&cur) != hipSuccess) return ID_ERR_HIP;
    if (sdev != cur) return ID_ERR_ARG;
  }
  void* work = nullptr;
  const int rc = scratch_ptr(&work);
  if (rc) return rc;
  return mpid::factor_run_noalloc(A, dtype, m, n, lda, opts, work, kScratchBytes, perm, R, ldr,
                                  k_out, info, (hipStream_t)stream);
}

}  // extern "C"
