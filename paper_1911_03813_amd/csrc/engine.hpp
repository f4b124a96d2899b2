// The grouped solve engine: many decomposition problems (each with its own
// restarts) advanced together, one evaluation step at a time.
//
// Every problem ("instance") owns one block of device memory carved from an
// arena: its padded copy of V and nu, the evaluation buffers of the grouped
// kernels (grouped.hpp) and the L-BFGS lanes of its restarts (lbfgs.hpp).
// The engine keeps device tables of the live instances (descriptors, work
// items, lanes) and runs steps
//     ggemm1 -> gmodel -> ggemm2 -> gfinal -> lb_dots -> lb_step -> lb_apply
// on its own stream, eagerly or as a captured hipGraph replayed K times
// between polls of the per-lane stop flags.  Instances can be added and
// removed between polls (the served form does so continuously).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "grouped.hpp"
#include "lbfgs.hpp"
#include "runtime.hpp"
#include "symtd.h"

namespace symtd {

// First-fit allocator over one device region (256-byte granules), with
// coalescing of neighbouring free ranges.
class Arena {
 public:
  void reset(char* base, size_t size) {
    base_ = base;
    size_ = size;
    used_ = 0;
    free_.clear();
    if (size) free_[0] = size;
  }
  char* alloc(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rem = it->second - bytes;
        free_.erase(it);
        if (rem) free_[off + bytes] = rem;
        used_ += bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p, size_t bytes) {
    bytes = round(bytes);
    size_t off = (size_t)(p - base_);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* p = base ? (X*)(base + off) : nullptr;
    off += count * sizeof(X);
    return p;
  }
};

template <typename T>
struct EngineInst {
  uint64_t id = 0;
  symtd_problem pb{};
  symtd_solve_opts o{};
  int64_t n = 0, p = 0, r = 0, ld = 0, N = 0, trace_len = 0;
  int R = 0, nb = 0;
  char* block = nullptr;
  size_t bytes = 0;
  GInst<T> g{};
  std::vector<LbLane<T>> lanes;
  LbState* states = nullptr;
  double* alpha_dev = nullptr;
  double* trace = nullptr;
  double alpha = 0.0, scale = 1.0;
  bool done = false;
  double t_admit = 0.0;    // host clock at admission (served form)

  // layout of the instance block; with base == nullptr only sizes
  void carve(void* base) {
    const int64_t cols = r * R;
    const int nt = (int)((cols + 15) / 16);
    const int64_t nblk = (p + 15) / 16;
    const int ntile = (int)((p + GG1_TILE - 1) / GG1_TILE);
    const int split_blk = grouped_split_blocks(sizeof(T) == 8, n, p, cols);
    const int nsplit = (int)((nblk + split_blk - 1) / split_blk);
    const int64_t ldy = 64 * ((n + 63) / 64);
    const int m = o.m;
    Carver c(base);
    g.V = c.take<T>((size_t)ld * p);
    g.nu = c.take<double>((size_t)p);
    T* A_t = c.take<T>((size_t)ld * cols);
    g.A = A_t;
    g.G = c.take<T>((size_t)ld * cols);
    double* lam_t = c.take<double>((size_t)cols);
    g.lam = lam_t;
    g.f = c.take<double>((size_t)R);
    g.glam = c.take<double>((size_t)cols);
    g.Wp = c.take<T>((size_t)nblk * nt * 256);
    g.wpart = c.take<double>((size_t)ntile * cols);
    g.Ypart = c.take<T>((size_t)nsplit * nt * 16 * ldy);
    g.B = c.take<double>((size_t)R * r * r);
    g.C = c.take<double>((size_t)R * r * r);
    g.YM = c.take<double>((size_t)n * cols);
    double* x = c.take<double>((size_t)R * N);
    double* gg = c.take<double>((size_t)R * N);
    double* dd = c.take<double>((size_t)R * N);
    double* S = c.take<double>((size_t)R * m * N);
    double* Y = c.take<double>((size_t)R * m * N);
    double* part = c.take<double>((size_t)R * nb * LB_ND);
    states = c.take<LbState>((size_t)R);
    alpha_dev = c.take<double>(1);
    trace = c.take<double>((size_t)R * std::max<int64_t>(trace_len, 1));
    bytes = c.off + 256;
    g.ldv = ld; g.lda = ld; g.ldg = ld;
    g.n = (int)n; g.p = (int)p; g.d = pb.d; g.r = (int)r; g.R = R; g.cols = (int)cols; g.nt = nt;
    g.ntile = ntile; g.nsplit = nsplit; g.ldy = ldy; g.split_blk = split_blk;
    if (!base) return;
    lanes.resize(R);
    for (int k = 0; k < R; ++k) {
      LbLane<T>& L = lanes[k];
      L.N = N; L.n = (int)n; L.r = (int)r; L.ld = (int)ld; L.nb = nb; L.inst = 0;
      L.seed = o.seed; L.restart = k;
      L.A0 = o.A0 ? (const T*)o.A0 + (size_t)k * r * n : nullptr;
      L.x = x + (size_t)k * N; L.g = gg + (size_t)k * N; L.d = dd + (size_t)k * N;
      L.S = S + (size_t)k * m * N; L.Y = Y + (size_t)k * m * N;
      L.lam_t = lam_t + (size_t)k * r; L.A_t = A_t + (size_t)k * r * ld;
      L.f_t = g.f + k; L.glam_t = g.glam + (size_t)k * r; L.G_t = g.G + (size_t)k * r * ld;
      L.part = part + (size_t)k * nb * LB_ND;
      L.trace = trace_len > 0 ? trace + (size_t)k * trace_len : nullptr;
      L.trace_len = trace_len;
      L.state = states + k;
      L.done_flag = nullptr;
      L.m = m; L.pgtol = o.pgtol; L.ftol = o.ftol; L.max_iters = o.max_iters; L.max_evals = o.max_evals;
      L.scale = 1.0;
    }
  }
};

template <typename T>
class GroupEngine {
 public:
  explicit GroupEngine(symtd_ctx* ctx) : ctx_(ctx) {}
  ~GroupEngine() { release_all(); }

  symtd_status init(hipStream_t caller, char* region, size_t bytes, bool use_graph) {
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&st_, hipStreamNonBlocking)) != hipSuccess) return ctx_->hip_fail(e, "engine stream");
    if ((e = hipEventCreateWithFlags(&ev_, hipEventDisableTiming)) != hipSuccess) return ctx_->hip_fail(e, "engine event");
    if ((e = hipHostMalloc((void**)&host_, sizeof(int) * 16, hipHostMallocDefault)) != hipSuccess)
      return ctx_->hip_fail(e, "engine host buffer");
    arena_.reset(region, bytes);
    use_graph_ = use_graph;
    // work queued by the caller before this point (inputs) comes first
    if ((e = hipEventRecord(ev_, caller)) != hipSuccess || (e = hipStreamWaitEvent(st_, ev_, 0)) != hipSuccess)
      return ctx_->hip_fail(e, "engine fork");
    return SYMTD_OK;
  }

  hipStream_t stream() const { return st_; }
  Arena& arena() { return arena_; }
  size_t live() const { return live_.size(); }

  // bytes an instance needs in the arena
  static size_t footprint(const symtd_problem& pb, const symtd_solve_opts& o, int64_t trace_len) {
    EngineInst<T> I;
    shape(I, pb, o, trace_len);
    I.carve(nullptr);
    return I.bytes;
  }

  // Admit instances: copy V and nu, compute alpha, draw the starts.  Returns
  // EREJECTED (nothing admitted) if the arena cannot hold them all.
  symtd_status admit(std::vector<EngineInst<T>*>& batch) {
    hipError_t e;
    std::vector<char*> got;
    for (auto* I : batch) {
      I->block = arena_.alloc(I->bytes);
      if (!I->block) {
        for (size_t i = 0; i < got.size(); ++i) arena_.release(batch[i]->block, batch[i]->bytes);
        return ctx_->fail(SYMTD_EREJECTED, "instance of %zu bytes does not fit the engine memory", I->bytes);
      }
      got.push_back(I->block);
      I->carve(I->block);
    }
    const size_t esz = sizeof(T);
    for (auto* I : batch) {
      // zero everything from the V copy's padding to the lane vectors and states
      if ((e = hipMemsetAsync(I->block, 0, I->bytes - 256, st_)) != hipSuccess) return ctx_->hip_fail(e, "engine zero");
      if ((e = hipMemcpy2DAsync((void*)I->g.V, (size_t)I->ld * esz, I->pb.V, (size_t)I->pb.ldv * esz, (size_t)I->n * esz,
                                (size_t)I->p, hipMemcpyDeviceToDevice, st_)) != hipSuccess ||
          (e = hipMemcpyAsync((void*)I->g.nu, I->pb.nu, sizeof(double) * I->p, hipMemcpyDeviceToDevice, st_)) != hipSuccess)
        return ctx_->hip_fail(e, "engine copy-in");
      if (I->trace_len > 0 &&
          (e = hipMemsetAsync(I->trace, 0xFF, sizeof(double) * I->R * I->trace_len, st_)) != hipSuccess)
        return ctx_->hip_fail(e, "engine trace");
    }
    // alpha of every new instance
    std::vector<double> alphas(batch.size(), 0.0);
    std::vector<NormXJob<T>> jobs;
    for (auto* I : batch)
      if (I->o.alpha_mode == SYMTD_ALPHA_COMPUTE)
        jobs.push_back(NormXJob<T>{I->g.V, I->ld, I->g.nu, I->n, I->p, I->pb.d, I->alpha_dev});
    const bool any = !jobs.empty();
    if (any) {
      // every new instance's alpha in one grouped launch (synchronised on return)
      symtd_status s = run_normx_grouped<T>(ctx_, st_, jobs);
      if (s != SYMTD_OK) return s;
      for (size_t i = 0; i < batch.size(); ++i)
        if (batch[i]->o.alpha_mode == SYMTD_ALPHA_COMPUTE &&
            (e = hipMemcpy(&alphas[i], batch[i]->alpha_dev, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
          return ctx_->hip_fail(e, "engine alpha read");
    }
    for (size_t i = 0; i < batch.size(); ++i) {
      auto* I = batch[i];
      I->alpha = I->o.alpha_mode == SYMTD_ALPHA_COMPUTE ? alphas[i] : I->o.alpha_mode == SYMTD_ALPHA_GIVEN ? I->o.alpha : 0.0;
      I->scale = I->alpha > 0.0 ? I->alpha : 1.0;
      I->g.alpha = I->alpha;
      for (auto& L : I->lanes) L.scale = I->scale;
    }
    // starts: tables of just the new instances of each kind
    symtd_status s;
    int rmax = 1;
    for (auto* I : batch) rmax = std::max<int>(rmax, (int)I->r);
    bool rrf = false, gauss = false, given = false;
    for (auto* I : batch) {
      if (I->o.A0) given = true;
      else if (I->o.init == SYMTD_INIT_GAUSS) gauss = true;
      else rrf = true;
    }
    // the start kernels pick their instances through per-kind lane/item lists
    if (given || gauss) {
      std::vector<EngineInst<T>*> gsub, asub;
      for (auto* I : batch)
        if (I->o.A0) asub.push_back(I);
        else if (I->o.init == SYMTD_INIT_GAUSS) gsub.push_back(I);
      if (!asub.empty()) {
        if ((s = upload(asub, true)) != SYMTD_OK) return s;
        launch_init_given<T>(nbmax_, nlanes_, st_, d_lanes_);
      }
      if (!gsub.empty()) {
        if ((s = upload(gsub, true)) != SYMTD_OK) return s;
        launch_init_gauss<T>(nbmax_, nlanes_, st_, d_lanes_);
        launch_norm_cols<T>(nlanes_, rmax, st_, d_lanes_);
      }
    }
    if (rrf) {
      std::vector<EngineInst<T>*> sub;
      for (auto* I : batch) if (!I->o.A0 && I->o.init != SYMTD_INIT_GAUSS) sub.push_back(I);
      if ((s = upload(sub, true)) != SYMTD_OK) return s;
      int maxchunks = 1;
      for (auto* I : sub)
        maxchunks = std::max<int>(maxchunks, (int)std::min<int64_t>(1024, ((I->p + 15) / 16 * I->g.nt * 256 + 255) / 256));
      launch_gomega<T>(maxchunks, (int)sub.size(), st_, d_ginst_, d_seeds_);
      launch_ggemm2<T>(true, n_g2_, st_, d_ginst_, d_items_ + off_g2_);
      launch_grrf_finish<T>(nlanes_, rmax, st_, d_lanes_, d_ginst_);
    }
    if ((e = hipGetLastError()) != hipSuccess) return ctx_->hip_fail(e, "engine starts");
    for (auto* I : batch) live_.push_back(I);
    dirty_ = true;
    return SYMTD_OK;
  }

  // K evaluation steps of every live instance
  symtd_status run(int K) {
    if (live_.empty()) return SYMTD_OK;
    Marker mk("grouped steps");
    symtd_status s;
    if (dirty_) {
      if ((s = upload(live_, false)) != SYMTD_OK) return s;
      drop_graph();
      dirty_ = false;
    }
    hipError_t e;
    if (use_graph_) {
      // the K steps between two polls are one captured graph, so that only
      // one launch boundary separates the polls (consecutive launches of a
      // one-step graph leave a gap of several microseconds between steps)
      if (exec_ && graph_steps_ != K) drop_graph();
      if (!exec_) {
        if ((e = hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return ctx_->hip_fail(e, "graph capture");
        for (int k = 0; k < K; ++k) enqueue_step();
        if ((e = hipStreamEndCapture(st_, &graph_)) != hipSuccess) return ctx_->hip_fail(e, "graph capture end");
        if ((e = hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0)) != hipSuccess)
          return ctx_->hip_fail(e, "graph instantiate");
        graph_steps_ = K;
      }
      if ((e = hipGraphLaunch(exec_, st_)) != hipSuccess) return ctx_->hip_fail(e, "graph launch");
    } else {
      for (int k = 0; k < K; ++k) enqueue_step();
      if ((e = hipGetLastError()) != hipSuccess) return ctx_->hip_fail(e, "engine step");
    }
    steps_ += K;
    return SYMTD_OK;
  }

  // Mark instances whose lanes have all stopped; returns them in `done`.
  symtd_status poll(std::vector<EngineInst<T>*>& done) {
    done.clear();
    if (live_.empty() || dirty_) return SYMTD_OK;   // no step has run on the current tables
    hipError_t e;
    lane_done_host_.resize(nlanes_);
    if ((e = hipMemcpyAsync(lane_done_host_.data(), d_lane_done_, sizeof(int) * nlanes_, hipMemcpyDeviceToHost, st_)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st_)) != hipSuccess)
      return ctx_->hip_fail(e, "engine poll");
    if (symtd_status s = ctx_->take_device_error(); s != SYMTD_OK) return s;
    int L = 0;
    for (auto* I : live_) {
      bool all = true;
      for (int k = 0; k < I->R; ++k) all = all && lane_done_host_[L + k] != 0;
      L += I->R;
      if (all && !I->done) {
        I->done = true;
        done.push_back(I);
      }
    }
    return SYMTD_OK;
  }

  // Results of finished instances (host figures; A and lambda to device or
  // host buffers).  The lane states of all of them come back in one round of
  // copies with one wait; then every instance's result copies and its fp64
  // evaluation at the best restart's point are enqueued, and one more wait
  // brings all the f values back.
  symtd_status collect_many(const std::vector<EngineInst<T>*>& set, const std::vector<symtd_solve_result*>& outs,
                            bool host_outputs) {
    if (set.empty()) return SYMTD_OK;
    hipError_t e;
    size_t nst = 0;
    for (auto* I : set) nst += (size_t)I->R;
    const size_t need = nst * sizeof(LbState) + set.size() * sizeof(double);
    if (need > pin_bytes_) {
      if (pin_) (void)hipHostFree(pin_);
      pin_ = nullptr;
      pin_bytes_ = 0;
      if ((e = hipHostMalloc(&pin_, need, hipHostMallocDefault)) != hipSuccess) return ctx_->hip_fail(e, "engine staging");
      pin_bytes_ = need;
    }
    if (set.size() > fdev_cap_) {
      if (fdev_) (void)hipFree(fdev_);   // the previous collection waited for its use
      fdev_ = nullptr;
      fdev_cap_ = 0;
      if ((e = hipMalloc(&fdev_, sizeof(double) * set.size())) != hipSuccess) {
        (void)hipGetLastError();
        return ctx_->fail(SYMTD_ENOMEM, "engine result buffer");
      }
      fdev_cap_ = set.size();
    }
    LbState* hs = (LbState*)pin_;
    double* fh = (double*)((char*)pin_ + nst * sizeof(LbState));
    size_t off = 0;
    for (auto* I : set) {
      if ((e = hipMemcpyAsync(hs + off, I->states, sizeof(LbState) * I->R, hipMemcpyDeviceToHost, st_)) != hipSuccess)
        return ctx_->hip_fail(e, "engine collect");
      off += (size_t)I->R;
    }
    if ((e = hipStreamSynchronize(st_)) != hipSuccess) return ctx_->hip_fail(e, "engine collect");
    const hipMemcpyKind kind = host_outputs ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    off = 0;
    for (size_t q = 0; q < set.size(); ++q) {
      EngineInst<T>* I = set[q];
      symtd_solve_result* out = outs[q];
      const LbState* H = hs + off;
      off += (size_t)I->R;
      int best = 0;
      for (int k = 1; k < I->R; ++k)
        if (H[k].f < H[best].f || (std::isnan(H[best].f) && !std::isnan(H[k].f))) best = k;
      const LbLane<T>& B = I->lanes[best];
      if ((e = hipMemcpy2DAsync(out->A, (size_t)out->lda * sizeof(T), B.A_t, (size_t)I->ld * sizeof(T),
                                (size_t)I->n * sizeof(T), (size_t)I->r, kind, st_)) != hipSuccess ||
          (e = hipMemcpyAsync(out->lambda, B.lam_t, sizeof(double) * I->r, kind, st_)) != hipSuccess)
        return ctx_->hip_fail(e, "engine result copy");
      if (out->f_trace && I->trace_len > 0 &&
          (e = hipMemcpyAsync(out->f_trace, I->trace, sizeof(double) * I->R * I->trace_len, hipMemcpyDeviceToHost,
                              st_)) != hipSuccess)
        return ctx_->hip_fail(e, "engine trace copy");
      for (int k = 0; k < I->R; ++k) {
        if (out->f_restarts) out->f_restarts[k] = H[k].f * I->scale;
        if (out->iters_restarts) out->iters_restarts[k] = H[k].iters;
        if (out->evals_restarts) out->evals_restarts[k] = H[k].evals;
        if (out->exit_restarts) out->exit_restarts[k] = H[k].reason;
      }
      // reported f and relative error: fp64 evaluation at the best final point
      symtd_status s = final_fp64_enqueue<T>(ctx_, st_, I->g.V, I->ld, I->g.nu, I->n, I->p, B.A_t, I->ld, B.lam_t,
                                             I->r, I->pb.d, I->alpha, fdev_ + q);
      if (s != SYMTD_OK) return s;
      out->alpha = I->alpha;
      out->iters = H[best].iters;
      out->evals = H[best].evals;
      out->exit_reason = H[best].reason;
      out->best_restart = best;
      out->steps = steps_;
    }
    if ((e = hipMemcpyAsync(fh, fdev_, sizeof(double) * set.size(), hipMemcpyDeviceToHost, st_)) != hipSuccess ||
        (e = hipStreamSynchronize(st_)) != hipSuccess)
      return ctx_->hip_fail(e, "engine collect sync");
    for (size_t q = 0; q < set.size(); ++q) {
      symtd_solve_result* out = outs[q];
      const double a = set[q]->alpha;
      out->f = fh[q];
      out->rel_err = a > 0.0 ? std::sqrt(std::max(out->f, 0.0) / a) : NAN;
    }
    return SYMTD_OK;
  }

  symtd_status collect(EngineInst<T>* I, symtd_solve_result* out, bool host_outputs) {
    return collect_many(std::vector<EngineInst<T>*>{I}, std::vector<symtd_solve_result*>{out}, host_outputs);
  }

  // Remove a finished (or cancelled) instance and free its memory.
  void remove(EngineInst<T>* I) {
    auto it = std::find(live_.begin(), live_.end(), I);
    if (it != live_.end()) live_.erase(it);
    if (I->block) arena_.release(I->block, I->bytes);
    I->block = nullptr;
    dirty_ = true;
  }

  int64_t steps() const { return steps_; }

  symtd_status join(hipStream_t caller) {
    hipError_t e;
    if ((e = hipEventRecord(ev_, st_)) != hipSuccess || (e = hipStreamWaitEvent(caller, ev_, 0)) != hipSuccess)
      return ctx_->hip_fail(e, "engine join");
    return SYMTD_OK;
  }

  static void shape(EngineInst<T>& I, const symtd_problem& pb, const symtd_solve_opts& o, int64_t trace_len) {
    I.pb = pb;
    I.o = o;
    I.n = pb.n; I.p = pb.p; I.r = pb.r; I.R = o.restarts;
    I.ld = 4 * ((pb.n + 3) / 4);
    I.N = I.r + I.ld * I.r;
    I.nb = (int)((I.N + LB_CHUNK - 1) / LB_CHUNK);
    I.trace_len = trace_len;
  }

 private:
  void enqueue_step() {
    launch_ggemm1<T>(true, n_g1_, st_, d_ginst_, d_items_ + off_g1_);
    launch_gmodel<T>(n_gm_, st_, d_ginst_, d_items_ + off_gm_);
    launch_ggemm2<T>(true, n_g2_, st_, d_ginst_, d_items_ + off_g2_);
    launch_gfinal<T>(n_gf_, st_, d_ginst_, d_items_ + off_gf_);
    launch_lb_dots<T>(nbmax_, nlanes_, st_, d_lanes_, d_lbitems_, n_lbi_);
    launch_lb_step<T>(nlanes_, st_, d_lanes_, LbParams{nullptr});
    launch_lb_apply<T>(nbmax_, nlanes_, st_, d_lanes_, d_lbitems_, n_lbi_);
  }

  // descriptor, item and lane tables of `set` into the table buffer
  symtd_status upload(const std::vector<EngineInst<T>*>& set, bool init) {
    std::vector<GInst<T>> gi;
    std::vector<GItem> items;
    std::vector<LbLane<T>> lanes;
    std::vector<uint64_t> seeds;
    std::vector<int> done0;
    const int NTM = sizeof(T) == 8 ? GG_NT_F64 : GG_NT_F32;
    std::vector<GItem> g1, gm, g2, gf;
    std::vector<LbItem> lbi;   // (lane, chunk) blocks of the dot and apply kernels
    nbmax_ = 1;
    for (size_t i = 0; i < set.size(); ++i) {
      EngineInst<T>* I = set[i];
      gi.push_back(I->g);
      seeds.push_back(I->o.seed);
      const int ncg = (I->g.nt + NTM - 1) / NTM;
      for (int t = 0; t < I->g.ntile; ++t)
        for (int cg = 0; cg < ncg; ++cg) g1.push_back({(int)i, t, cg, 0});
      for (int k = 0; k < I->R; ++k) gm.push_back({(int)i, k, 0, 0});
      for (int rb = 0; rb < (int)((I->n + 63) / 64); ++rb)
        for (int sp = 0; sp < I->g.nsplit; ++sp)
          for (int cg = 0; cg < ncg; ++cg) g2.push_back({(int)i, rb, sp, cg});
      for (int c = 0; c < I->g.cols; ++c) gf.push_back({(int)i, c, 0, 0});
      for (int k = 0; k < I->R; ++k) {
        LbLane<T> L = I->lanes[k];
        L.inst = (int)i;
        for (int b = 0; b < L.nb; ++b) lbi.push_back({(int)lanes.size(), b});
        lanes.push_back(L);
        done0.push_back(0);
        nbmax_ = std::max(nbmax_, L.nb);
      }
    }
    off_g1_ = 0; n_g1_ = (int)g1.size();
    off_gm_ = off_g1_ + n_g1_; n_gm_ = (int)gm.size();
    off_g2_ = off_gm_ + n_gm_; n_g2_ = (int)g2.size();
    off_gf_ = off_g2_ + n_g2_; n_gf_ = (int)gf.size();
    items.insert(items.end(), g1.begin(), g1.end());
    items.insert(items.end(), gm.begin(), gm.end());
    items.insert(items.end(), g2.begin(), g2.end());
    items.insert(items.end(), gf.begin(), gf.end());
    nlanes_ = (int)lanes.size();
    n_lbi_ = (int)lbi.size();
    // table buffer: [ginst][seeds][items][lanes][lane_done][lane chunks]
    Carver c(nullptr);
    c.take<GInst<T>>(gi.size() + 1);
    c.take<uint64_t>(seeds.size() + 1);
    c.take<GItem>(items.size() + 1);
    c.take<LbLane<T>>(lanes.size() + 1);
    c.take<int>(lanes.size() + 1);
    c.take<LbItem>(lbi.size() + 1);
    const size_t need = c.off + 256;
    hipError_t e;
    if (need > tab_bytes_) {
      if ((e = hipStreamSynchronize(st_)) != hipSuccess) return ctx_->hip_fail(e, "engine table sync");
      drop_graph();
      if (tab_) (void)hipFree(tab_);
      tab_ = nullptr;
      tab_bytes_ = 0;
      const size_t want = std::max(need * 2, (size_t)1 << 16);
      if ((e = hipMalloc(&tab_, want)) != hipSuccess) {
        (void)hipGetLastError();
        return ctx_->fail(SYMTD_ENOMEM, "engine tables (%zu bytes)", want);
      }
      tab_bytes_ = want;
    }
    Carver t(tab_);
    d_ginst_ = t.take<GInst<T>>(gi.size() + 1);
    d_seeds_ = t.take<uint64_t>(seeds.size() + 1);
    d_items_ = t.take<GItem>(items.size() + 1);
    d_lanes_ = t.take<LbLane<T>>(lanes.size() + 1);
    d_lane_done_ = t.take<int>(lanes.size() + 1);
    d_lbitems_ = t.take<LbItem>(lbi.size() + 1);
    for (size_t L = 0; L < lanes.size(); ++L) lanes[L].done_flag = d_lane_done_ + L;
    // every flag starts low in a new table: a lane that has stopped raises
    // its flag again at each step (its state is final), so nothing is lost
    for (size_t L = 0; L < done0.size(); ++L) done0[L] = 0;
    // the copies below read host vectors; the stream is synchronised before
    // they go out of scope, since table uploads are rare
    if ((e = hipMemcpyAsync(d_ginst_, gi.data(), sizeof(GInst<T>) * gi.size(), hipMemcpyHostToDevice, st_)) != hipSuccess ||
        (e = hipMemcpyAsync(d_seeds_, seeds.data(), sizeof(uint64_t) * seeds.size(), hipMemcpyHostToDevice, st_)) != hipSuccess ||
        (items.size() && (e = hipMemcpyAsync(d_items_, items.data(), sizeof(GItem) * items.size(), hipMemcpyHostToDevice,
                                              st_)) != hipSuccess) ||
        (e = hipMemcpyAsync(d_lanes_, lanes.data(), sizeof(LbLane<T>) * lanes.size(), hipMemcpyHostToDevice, st_)) != hipSuccess ||
        (e = hipMemcpyAsync(d_lane_done_, done0.data(), sizeof(int) * done0.size(), hipMemcpyHostToDevice, st_)) != hipSuccess ||
        (lbi.size() && (e = hipMemcpyAsync(d_lbitems_, lbi.data(), sizeof(LbItem) * lbi.size(), hipMemcpyHostToDevice,
                                            st_)) != hipSuccess) ||
        (e = hipStreamSynchronize(st_)) != hipSuccess)
      return ctx_->hip_fail(e, "engine table upload");
    return SYMTD_OK;
  }

  void drop_graph() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
  }

  void release_all() {
    if (st_) (void)hipStreamSynchronize(st_);
    drop_graph();
    if (tab_) (void)hipFree(tab_);
    if (host_) (void)hipHostFree(host_);
    if (pin_) (void)hipHostFree(pin_);
    if (fdev_) (void)hipFree(fdev_);
    pin_ = nullptr; fdev_ = nullptr; pin_bytes_ = 0; fdev_cap_ = 0;
    if (ev_) (void)hipEventDestroy(ev_);
    if (st_) (void)hipStreamDestroy(st_);
    tab_ = nullptr; host_ = nullptr; ev_ = nullptr; st_ = nullptr;
  }

  symtd_ctx* ctx_;
  hipStream_t st_ = nullptr;
  hipEvent_t ev_ = nullptr;
  int* host_ = nullptr;
  void* pin_ = nullptr;            // pinned staging of collected lane states and f values
  size_t pin_bytes_ = 0;
  double* fdev_ = nullptr;         // device f values of the instances being collected
  size_t fdev_cap_ = 0;
  Arena arena_;
  bool use_graph_ = true, dirty_ = true;
  std::vector<EngineInst<T>*> live_;
  void* tab_ = nullptr;
  size_t tab_bytes_ = 0;
  GInst<T>* d_ginst_ = nullptr;
  uint64_t* d_seeds_ = nullptr;
  GItem* d_items_ = nullptr;
  LbLane<T>* d_lanes_ = nullptr;
  int* d_lane_done_ = nullptr;
  LbItem* d_lbitems_ = nullptr;
  int off_g1_ = 0, n_g1_ = 0, off_gm_ = 0, n_gm_ = 0, off_g2_ = 0, n_g2_ = 0, off_gf_ = 0, n_gf_ = 0;
  int nlanes_ = 0, nbmax_ = 1, n_lbi_ = 0;
  std::vector<int> lane_done_host_;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  int graph_steps_ = 0;           // evaluation steps in the captured graph
  int64_t steps_ = 0;
};

}  // namespace symtd
