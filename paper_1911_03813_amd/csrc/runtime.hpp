// The context object behind the opaque symtd_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "symtd.h"

struct symtd_ctx {
  int device = 0;
  int cu_count = 256;
  std::string err;
  void* ws = nullptr;   // device workspace, grown on demand
  size_t ws_bytes = 0;
  // side stream for the model terms, and the events of the fork/join
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_model = nullptr, ev_g1 = nullptr, ev_side = nullptr;
  // hand-off flags of the split products (zero between launches) and a
  // device error word set if a hand-off wait ever gives up
  int* flags = nullptr;
  int nflags = 0;
  int* dev_err = nullptr;
  // work-split overrides (0 = automatic)
  int64_t tune_g1_blocks = 0, tune_g2_splits = 0, tune_serial = 0;

  // per-kernel timing (symtd_profile_*)
  struct Pending { int which; hipEvent_t start, stop; hipStream_t st; };
  bool prof = false;
  std::vector<Pending> pending;

  symtd_status fail(symtd_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
  symtd_status hip_fail(hipError_t e, const char* what);
  symtd_status reserve(size_t bytes);
  symtd_status set_device();
  symtd_status check_common(symtd_dtype dt, const void* V, int64_t ldv, const double* nu,
                            int64_t n, int64_t p, int d);
  void prof_begin(int which, hipStream_t st);
  void prof_end(hipStream_t st);
};
