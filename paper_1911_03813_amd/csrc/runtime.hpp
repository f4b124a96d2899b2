// The context object behind the opaque symtd_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "corrected.hpp"
#include "kernels.hpp"
#include "symtd.h"

struct symtd_ctx {
  int device = 0;
  int cu_count = 256;
  std::string err;
  void* ws = nullptr;   // device workspace of the evaluation, grown on demand
  size_t ws_bytes = 0;
  void* sws = nullptr;  // device workspace of the solver state, grown on demand
  size_t sws_bytes = 0;
  void* wide = nullptr; // device scratch of the final fp64 evaluation, grown on demand
  size_t wide_bytes = 0;
  void* noalloc_ws = nullptr;   // this device's fixed scratch array (symtd_fg_noalloc)
  int* host_flag = nullptr;   // pinned host word for polling the solver's stop count
  double fwide_host = 0.0;    // host landing of the final fp64 evaluation
  double* wide_f = nullptr;   // its device word in the scratch `wide`
  // hand-off flags of the split products (tagged with a launch epoch), and
  // the arrival counters of the closing step, one per model (zero between
  // launches)
  int* flags = nullptr;
  int nflags = 0;
  int* final_count = nullptr;
  static constexpr int kFinalCounters = 1024;
  int* epoch_word = nullptr;  // the split products' launch epoch and arrival counter (2 words)
  // error word in pinned host memory: a kernel whose hand-off wait gave up
  // sets it (err_dev is its device address); every call checks it first
  int* err_host = nullptr;
  int* err_dev = nullptr;
  // work-split overrides (0 = automatic)
  int64_t tune_g1_blocks = 0, tune_g2_splits = 0;
  int64_t tune_graph = 1;   // grouped engine: replay captured steps (1) or launch eagerly (0)
  int64_t tune_spin = 0;    // polls before a hand-off wait gives up (0 = automatic)
  int64_t tune_fault = 0;   // testing: hand-off waits watch for a value no block writes

  // per-kernel timing (symtd_profile_*): kernels whose bit is set in
  // prof_mask are bracketed by events taken from a reusable pool
  struct Pending { int which; hipEvent_t start, stop; };
  uint32_t prof_mask = 0;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;

  symtd_status fail(symtd_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
  symtd_status hip_fail(hipError_t e, const char* what);
  symtd_status reserve(size_t bytes);
  symtd_status reserve_solver(size_t bytes);
  symtd_status set_device();
  symtd_status check_common(symtd_dtype dt, const void* V, int64_t ldv, const double* nu,
                            int64_t n, int64_t p, int d);
  // hand-off arguments of a split-product launch
  symtd::Handoff handoff();
  // SYMTD_EDEVICE (and the word cleared) if a kernel set the error word
  symtd_status take_device_error();
  void prof_begin(int which, hipStream_t st);
  void prof_end(int which, hipStream_t st);
  hipEvent_t pool_event();
};

namespace symtd {

// A roctx range over a host-side scope (a solve, a batch of steps, an
// admission): rocprofv3 --marker-trace records it beside the kernels the
// scope enqueued; without a profiler attached the calls do nothing.
struct Marker {
  explicit Marker(const char* what) { roctxRangePushA(what); }
  ~Marker() { roctxRangePop(); }
  Marker(const Marker&) = delete;
  Marker& operator=(const Marker&) = delete;
};

// Launch shape and workspace of one evaluation (the products' splits and the
// element counts of the workspace buffers), from the sizes alone.
struct FgPlan {
  int nt_tot, rp, nblk, nt1, nt2, g1w, nslab, nblocks, nsplit, blk_per_split, rowblocks;
  int64_t npad;
  int64_t ldap;
  size_t apad, wp, wpart, part, ypart, rr, fp;  // element counts
  size_t bytes(size_t esz) const {
    size_t s = 0;
    auto add = [&](size_t b) { s = ((s + 255) & ~(size_t)255) + b; };
    add(apad * esz);
    add(wp * esz);
    add(wpart * sizeof(double));
    add(part * esz);
    add(ypart * esz);
    add(rr * sizeof(double));
    add(rr * sizeof(double));
    add(fp * sizeof(double));
    return s + 256;
  }
};

FgPlan plan_fg(int64_t n, int64_t p, int64_t r, bool f64, int cus, int64_t g1_blocks, int64_t g2_splits);

// The tuning table (symtd_tune_*, process-wide): the first-product blocks
// and second-product splits of an evaluation, and the split length of the
// grouped second product, by (precision, log2 buckets of n, p and the
// evaluated columns).  Lookups return false / the default when no entry
// matches; a result depends only on the shape and the table.
bool tuned_fg(bool f64, int64_t n, int64_t p, int64_t cols, int64_t* g1_blocks, int64_t* g2_splits);
int grouped_split_blocks(bool f64, int64_t n, int64_t p, int64_t cols);

// Algorithm 2 for `ng` models of r columns side by side (model m = columns
// m r .. m r + r - 1 of A, lambda, g_lambda, G_A; f holds ng values).
// Arguments are checked by the caller.
// With `fixed_ws` the workspace is carved from those fixed_bytes instead of
// the context's arena (SYMTD_EINVAL if it does not fit): nothing is
// allocated, and no kernel is timed (timing would create events).
template <typename T>
symtd_status run_fg(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu,
                    int64_t n, int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int ng,
                    int d, double alpha, double* f, double* g_lambda, T* G, int64_t ldg,
                    void* fixed_ws = nullptr, size_t fixed_bytes = 0);

// Randomized range finder starts of `restarts` lanes (restart k = columns
// k r .. k r + r - 1 of V Omega), normalised, written into each lane's x and
// trial point.  Uses the evaluation workspace.
template <typename T> struct LbLane;
template <typename T>
symtd_status run_rrf(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, int64_t n, int64_t p, int64_t r,
                     int restarts, uint64_t seed, const LbLane<T>* lanes_dev);

// f at (lambda, A) evaluated with fp64 products (the stored values of V and A
// widened exactly when T is float), for the relative error of a finished
// solve.  Synchronises `st`; returns f in *f_out.
template <typename T>
symtd_status final_fp64(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n,
                        int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int d, double alpha,
                        double* f_out, const Correction* corr = nullptr);
// The same evaluation enqueued on `st` without waiting: f goes to the device
// word f_dev.  Evaluations enqueued one after another on one stream share the
// context's scratch in stream order.
template <typename T>
symtd_status final_fp64_enqueue(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n,
                                int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int d,
                                double alpha, double* f_dev, const Correction* corr = nullptr);

// noise correction (corrected.hpp): the data's statistics m (and M2, when
// not null) in fp64, and alpha_c = ||X - Delta||^2 from alpha = ||X||^2
// (synchronous; scratch holds ceil(p / 256) + 1 values)
template <typename T>
void launch_stats(hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n, int64_t p, double* m,
                  double* M2);
template <typename T>
symtd_status corrected_alpha(symtd_ctx* ctx, hipStream_t st, const Correction& c, const T* V, int64_t ldv,
                             const double* nu, int64_t n, int64_t p, double alpha, double* out, double* scratch);

// argument checks of a solve request (problem, options, result buffers)
symtd_status check_solve(symtd_ctx* ctx, const symtd_problem* pb, const symtd_solve_opts* o,
                         const symtd_solve_result* out);

// alpha = ||X||^2 into one device fp64 value.  Arguments checked by the caller.
template <typename S>
symtd_status run_normx(symtd_ctx* ctx, hipStream_t st, const S* V, int64_t ldv, const double* nu,
                       int64_t n, int64_t p, int d, double* alpha);

// alpha of several data sets, each into its own device fp64 value, in two
// launches; every value equals what run_normx computes for that set alone.
// Returns after the stream has finished them.
template <typename S>
struct NormXJob { const S* V; int64_t ldv; const double* nu; int64_t n, p; int d; double* alpha; };
template <typename S>
symtd_status run_normx_grouped(symtd_ctx* ctx, hipStream_t st, const std::vector<NormXJob<S>>& jobs);

}  // namespace symtd
