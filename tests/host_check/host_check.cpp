// Host-side checks of libmpid's C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer: workspace sizing over a grid of shapes and
// options (including sizes whose products overflow a naive 64-bit count),
// and the argument validation of every entry point, all of which return
// before any device call -- so this runs without a GPU.  Prints one line per
// failed expectation and exits with the number of failures.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "mpid.h"

static int g_fail = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
      ++g_fail;                                                        \
    }                                                                  \
  } while (0)

static id_opts opts(int32_t prec, int64_t k_fixed, double tol, int32_t flags = 0, int32_t nb = 0,
                    int64_t k_max = 0) {
  id_opts o;
  std::memset(&o, 0, sizeof(o));
  o.prec = prec;
  o.rank_rule = ID_RANK_PIVOT_REL;
  o.k_fixed = k_fixed;
  o.rel_tol = tol;
  o.k_max = k_max;
  o.nb = nb;
  o.flags = flags;
  return o;
}

int main() {
  const int64_t ms[] = {0, 1, 7, 64, 65, 1000, 20000, 1048576};
  const int64_t ns[] = {0, 1, 31, 32, 33, 500, 2000, 2048};
  const int32_t precs[] = {ID_PREC_F64, ID_PREC_MIXED_F16, ID_PREC_MIXED_BF16,
                           ID_PREC_MIXED_BF16X3, ID_PREC_MIXED_F32};
  // workspace sizes: positive for valid shapes, growing with m and n
  for (int32_t prec : precs)
    for (int32_t dt : {ID_F32, ID_F64})
      for (int64_t n : ns) {
        size_t prev = 0;
        for (int64_t m : ms) {
          id_opts o = opts(prec, 0, 1e-3);
          const size_t w = id_workspace_size(m, n, dt, &o);
          EXPECT(w > 0);
          EXPECT(w >= prev);
          prev = w;
          id_opts g = opts(ID_PREC_F64, 0, 1e-3, ID_FLAG_GRAM);
          (void)id_workspace_size(m, n, dt, &g);
          id_opts c = opts(prec, 0, 1e-3, ID_FLAG_CHOLQR);
          (void)id_workspace_size(m, n, dt, &c);
        }
      }
  // invalid options and sizes give 0
  {
    id_opts o = opts(ID_PREC_F64, 3, 0.0, 0, 33);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
    o = opts(ID_PREC_F64, -1, 0.0);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
    o = opts(ID_PREC_F64, 0, -1.0);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
    o = opts(9, 0, 1e-3);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
    o = opts(ID_PREC_F64, 0, 1e-3);
    EXPECT(id_workspace_size(-1, 10, ID_F32, &o) == 0);
    EXPECT(id_workspace_size(10, -1, ID_F32, &o) == 0);
    EXPECT(id_workspace_size(10, 10, 7, &o) == 0);
    EXPECT(id_workspace_size(INT64_MAX / 2, INT64_MAX / 2, ID_F32, &o) == 0);
    EXPECT(id_workspace_size(10, 10, ID_F32, nullptr) == 0);
    o = opts(ID_PREC_MIXED_F32, 0, 1e-3, ID_FLAG_ROUND_F32 | ID_FLAG_ROUND_F16);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
    o = opts(ID_PREC_MIXED_BF16, 0, 1e-3, ID_FLAG_ROUND_F16);
    EXPECT(id_workspace_size(10, 10, ID_F32, &o) == 0);
  }
  EXPECT(id_backward_workspace_size(100, 10, 11) == 0);
  EXPECT(id_backward_workspace_size(100, 10, 5) > 0);
  EXPECT(id_sketch_workspace_size(-1, 10, 10) == 0);
  EXPECT(id_sketch_workspace_size(8, 100, 10) > 0);
  {
    id_opts o = opts(ID_PREC_MIXED_BF16X3, 0, 1e-4);
    EXPECT(id_batch_item_workspace_size(1000, 4096, &o) == 0);  // n above the batched limit
    EXPECT(id_batch_item_workspace_size(1000, 300, &o) > 0);
  }
  EXPECT(id_noalloc_scratch_bytes() == ((size_t)ID_NOALLOC_SCRATCH_MB << 20));

  // argument validation: every call below returns before touching a device
  void* fake = reinterpret_cast<void*>(0x1000);
  int32_t* fi = static_cast<int32_t*>(fake);
  double* fd = static_cast<double*>(fake);
  int64_t k = -1;
  int32_t info = -1;
  id_opts o = opts(ID_PREC_F64, 2, 0.0);
  EXPECT(id_factor(nullptr, ID_F64, 10, 5, 10, &o, nullptr, 0, nullptr, nullptr, 2, &k, &info,
                   nullptr) == ID_ERR_ARG);
  EXPECT(id_factor(fake, 9, 10, 5, 10, &o, fake, 1 << 20, fi, fd, 2, &k, &info, nullptr) ==
         ID_ERR_DTYPE);
  EXPECT(id_factor(fake, ID_F64, 10, 5, 3, &o, fake, 1 << 20, fi, fd, 2, &k, &info, nullptr) ==
         ID_ERR_ARG);
  EXPECT(id_factor(fake, ID_F64, 10, 5, 10, &o, fake, 16, fi, fd, 2, &k, &info, nullptr) ==
         ID_ERR_WORKSPACE);
  EXPECT(id_factor(fake, ID_F64, 10, 5, 10, &o, fake, 1 << 20, fi, fd, 1, &k, &info,
                   nullptr) == ID_ERR_ARG);  // ldr < kcap
  EXPECT(id_factor(fake, ID_F64, 10, 5, 10, nullptr, fake, 1 << 20, fi, fd, 2, &k, &info,
                   nullptr) == ID_ERR_ARG);
  {
    id_opts big = opts(ID_PREC_MIXED_BF16X3, 0, 1e-3);
    EXPECT(id_factor_noalloc(fake, ID_F32, 20000, 2000, 20000, &big, fi, fd, 2000, &k, &info,
                             nullptr) == ID_ERR_SCRATCH);
    id_opts prof = opts(ID_PREC_F64, 2, 0.0, ID_FLAG_PROFILE);
    EXPECT(id_factor_noalloc(fake, ID_F64, 10, 5, 10, &prof, fi, fd, 2, &k, &info, nullptr) ==
           ID_ERR_UNSUPPORTED);
  }
  {
    // the CholeskyQR front end: refusals before any device call
    id_opts c = opts(ID_PREC_F64, 0, 1e-3, ID_FLAG_CHOLQR);
    const size_t ws = id_workspace_size(100, 10, ID_F64, &c);
    EXPECT(ws >= 2 * 100 * 10 * 8);
    EXPECT(id_factor(fake, ID_F64, 100, 10, 100, &c, fake, ws - 1, fi, fd, 10, &k, &info,
                     nullptr) == ID_ERR_WORKSPACE);
    EXPECT(id_factor(fake, ID_F64, 5, 10, 5, &c, fake, ws, fi, fd, 10, &k, &info, nullptr) ==
           ID_ERR_UNSUPPORTED);  // m < n
    id_opts both = opts(ID_PREC_F64, 0, 1e-3, ID_FLAG_CHOLQR | ID_FLAG_GRAM);
    EXPECT(id_workspace_size(100, 10, ID_F64, &both) == 0);
    EXPECT(id_factor(fake, ID_F64, 100, 10, 100, &both, fake, ws, fi, fd, 10, &k, &info,
                     nullptr) == ID_ERR_ARG);
    id_opts np = opts(ID_PREC_F64, 0, 1e-3, ID_FLAG_CHOLQR | ID_FLAG_NO_PIVOT);
    EXPECT(id_factor(fake, ID_F64, 100, 10, 100, &np, fake, ws, fi, fd, 10, &k, &info,
                     nullptr) == ID_ERR_UNSUPPORTED);
    EXPECT(id_factor_noalloc(fake, ID_F64, 100, 10, 100, &c, fi, fd, 10, &k, &info, nullptr) ==
           ID_ERR_UNSUPPORTED);
  }
  EXPECT(id_solve_T(static_cast<const double*>(fake), 5, 6, 5, static_cast<double*>(fake), 6,
                    static_cast<int32_t*>(fake), nullptr) == ID_ERR_ARG);
  EXPECT(id_reconstruct(fake, ID_F32, 4, 3, 4, static_cast<const int32_t*>(fake), 5,
                        static_cast<const double*>(fake), 5, static_cast<double*>(fake), 4, 0,
                        nullptr) == ID_ERR_ARG);
  EXPECT(id_round(static_cast<double*>(fake), 4, 4, 4, 3, nullptr) == ID_ERR_ARG);
  EXPECT(id_round(static_cast<double*>(fake), 4, 4, 3, 1, nullptr) == ID_ERR_ARG);
  EXPECT(id_round(nullptr, 0, 5, 1, 2, nullptr) == ID_OK);
  EXPECT(id_backward(fake, ID_F32, 4, 3, 4, static_cast<const int32_t*>(fake), 5,
                     static_cast<const double*>(fake), 5, nullptr, 1, nullptr, 1, nullptr, 4,
                     static_cast<double*>(fake), 4, fake, 1 << 20, &info, nullptr) == ID_ERR_ARG);
  {
    const size_t ws = id_sketch_workspace_size(8, 100, 10);
    EXPECT(id_sketch(fake, ID_F32, 100, 10, 100, static_cast<const double*>(fake), 8, 99,
                     static_cast<double*>(fake), 8, fake, ws, nullptr) == ID_ERR_ARG);
    EXPECT(id_sketch(fake, ID_F32, 100, 10, 100, static_cast<const double*>(fake), 8, 100,
                     static_cast<double*>(fake), 8, fake, ws - 8, nullptr) == ID_ERR_WORKSPACE);
  }
  {
    id_opts bo = opts(ID_PREC_MIXED_BF16X3, 0, 1e-4, ID_FLAG_PROFILE);
    EXPECT(id_factor_batched(static_cast<id_batch_item*>(fake), 4, nullptr, 0,
                             static_cast<int32_t*>(fake), 300, ID_F32, &bo, 0, 0,
                             nullptr) != ID_OK);
    id_opts wide = opts(ID_PREC_MIXED_BF16X3, 0, 1e-4);
    EXPECT(id_factor_batched(static_cast<id_batch_item*>(fake), 4, nullptr, 0,
                             static_cast<int32_t*>(fake), 4096, ID_F32, &wide, 0, 0,
                             nullptr) == ID_ERR_UNSUPPORTED);
  }
  EXPECT(id_last_profile(nullptr) == ID_ERR_ARG);
  for (int c = -10; c <= 10; ++c) EXPECT(id_status_string(c) != nullptr);
  EXPECT(std::strcmp(id_status_string(12345), "unknown code") == 0);

  std::printf("host checks: %d failed\n", g_fail);
  return g_fail;
}
