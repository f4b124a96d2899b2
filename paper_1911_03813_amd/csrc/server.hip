// The served form: a request loop with continuous batching over the grouped
// engine (engine.hpp).  See include/symtd.h for the contract.
//
// Threads: callers submit / poll / cancel under one mutex; the server thread
// owns the engine, its stream and the server's context.  A submitted request
// is copied (V, nu) into a staging arena on a copy stream before submit
// returns; the server thread admits queued requests in arrival order while
// they fit into the engine arena (their footprint is known at submit),
// copies them in (padded), frees their staging, and from then on steps them
// with everything else that is running.  Finished requests are collected
// into host results and leave the engine, which frees their memory for the
// next admissions.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "runtime.hpp"

using namespace symtd;

struct symtd_server {
  virtual ~symtd_server() = default;
  std::string err;
  virtual symtd_status submit(const symtd_problem* pb, const symtd_solve_opts* o, uint64_t* id) = 0;
  virtual symtd_status poll(symtd_server_result* out, int32_t max, int32_t* n_out, int32_t timeout_ms) = 0;
  virtual symtd_status cancel(uint64_t id) = 0;
  virtual symtd_status stats(symtd_server_stats* out) = 0;
};

namespace {

using Clock = std::chrono::steady_clock;

template <typename T>
struct Request {
  uint64_t id = 0;
  symtd_problem pb{};
  symtd_solve_opts o{};
  char* stage = nullptr;
  size_t stage_bytes = 0;
  size_t footprint = 0;
  double t_submit = 0.0, t_admit = 0.0;
  std::unique_ptr<EngineInst<T>> inst;
};

template <typename T>
class Server final : public symtd_server {
 public:
  ~Server() override { shutdown(); }

  symtd_status start(const symtd_server_opts& o) {
    opts_ = o;
    t0_ = Clock::now();
    symtd_status s = symtd_create(o.device, &ctx_);
    if (s != SYMTD_OK) return fail(s, "symtd_create failed on device %d", o.device);
    // a second context checks submitted requests (the first belongs to the server thread)
    if ((s = symtd_create(o.device, &vctx_)) != SYMTD_OK) return fail(s, "symtd_create failed on device %d", o.device);
    ctx_->tune_graph = o.use_graph ? 1 : 0;
    hipError_t e;
    if ((e = hipSetDevice(o.device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    staging_bytes_ = std::max<size_t>(o.memory_bytes / 2, (size_t)64 << 20);
    if ((e = hipMalloc(&region_, o.memory_bytes)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SYMTD_ENOMEM, "hipMalloc(%zu) for the server memory failed", o.memory_bytes);
    }
    if ((e = hipMalloc(&stage_region_, staging_bytes_)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SYMTD_ENOMEM, "hipMalloc(%zu) for the staging memory failed", staging_bytes_);
    }
    staging_.reset((char*)stage_region_, staging_bytes_);
    if ((e = hipStreamCreateWithFlags(&copy_st_, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "copy stream");
    eng_ = std::make_unique<GroupEngine<T>>(ctx_);
    if ((s = eng_->init(copy_st_, (char*)region_, o.memory_bytes, o.use_graph != 0)) != SYMTD_OK)
      return fail(s, "engine: %s", ctx_->err.c_str());
    thread_ = std::thread([this] { loop(); });
    return SYMTD_OK;
  }

  symtd_status submit(const symtd_problem* pb, const symtd_solve_opts* o, uint64_t* id) override {
    if (!pb || !o || !id) return fail(SYMTD_EINVAL, "null problem, options or id");
    if (pb->dt != opts_.dt || o->prec != opts_.prec) return fail(SYMTD_EINVAL, "request dtype/precision differ from the server's");
    if (o->A0) return fail(SYMTD_EINVAL, "served requests draw their own starts (A0 must be NULL)");
    if (o->sigma != 0.0) return fail(SYMTD_EINVAL, "the noise correction is symtd_solve's only (sigma must be 0)");
    if (o->pause_after != 0 || o->state_out || o->state_in)
      return fail(SYMTD_EINVAL, "pausing and resuming are symtd_solve's only");
    symtd_solve_result dummy{};
    dummy.A = (void*)16; dummy.lambda = (double*)16; dummy.lda = pb->n;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (broken_) return fail(SYMTD_EDEVICE, "server stopped: %s", err.c_str());
      symtd_status s = check_solve(vctx_, pb, o, &dummy);
      if (s != SYMTD_OK) return fail(s, "%s", vctx_->err.c_str());
    }
    auto rq = std::make_unique<Request<T>>();
    rq->pb = *pb;
    rq->o = *o;
    rq->footprint = GroupEngine<T>::footprint(*pb, *o, 0);
    if (Arena::round(rq->footprint) > opts_.memory_bytes)
      return fail(SYMTD_EREJECTED, "request needs %zu bytes, the server has %zu", rq->footprint, opts_.memory_bytes);
    const size_t esz = sizeof(T);
    const size_t vbytes = (size_t)pb->n * pb->p * esz;
    rq->stage_bytes = Arena::round(vbytes) + Arena::round(sizeof(double) * pb->p);
    {
      std::lock_guard<std::mutex> lk(stage_mu_);
      rq->stage = staging_.alloc(rq->stage_bytes);
      if (!rq->stage) return fail(SYMTD_EREJECTED, "staging memory full (%zu bytes in use)", staging_.used());
      hipError_t e;
      char* nu_stage = rq->stage + Arena::round(vbytes);
      if ((e = hipMemcpy2DAsync(rq->stage, (size_t)pb->n * esz, pb->V, (size_t)pb->ldv * esz, (size_t)pb->n * esz,
                                (size_t)pb->p, hipMemcpyDeviceToDevice, copy_st_)) != hipSuccess ||
          (e = hipMemcpyAsync(nu_stage, pb->nu, sizeof(double) * pb->p, hipMemcpyDeviceToDevice, copy_st_)) != hipSuccess ||
          (e = hipStreamSynchronize(copy_st_)) != hipSuccess) {
        staging_.release(rq->stage, rq->stage_bytes);
        return hip_fail(e, "request copy");
      }
      rq->pb.V = rq->stage;
      rq->pb.ldv = pb->n;
      rq->pb.nu = (const double*)nu_stage;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      rq->id = next_id_++;
      rq->t_submit = now();
      *id = rq->id;
      queue_.push_back(std::move(rq));
      ++st_.submitted;
    }
    cv_work_.notify_one();
    return SYMTD_OK;
  }

  symtd_status poll(symtd_server_result* out, int32_t max, int32_t* n_out, int32_t timeout_ms) override {
    if (!n_out || (max > 0 && !out)) return fail(SYMTD_EINVAL, "null output");
    *n_out = 0;
    std::unique_lock<std::mutex> lk(mu_);
    auto ready = [&] { return !done_.empty() || (queue_.empty() && running_ == 0) || broken_; };
    if (timeout_ms < 0) cv_done_.wait(lk, ready);
    else if (timeout_ms > 0) cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    int32_t k = 0;
    while (k < max && !done_.empty()) {
      out[k++] = done_.front();
      done_.pop_front();
    }
    *n_out = k;
    return SYMTD_OK;
  }

  symtd_status cancel(uint64_t id) override {
    std::unique_ptr<Request<T>> rq;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto it = queue_.begin(); it != queue_.end(); ++it)
        if ((*it)->id == id) {
          rq = std::move(*it);
          queue_.erase(it);
          ++st_.cancelled;
          break;
        }
    }
    if (!rq) return fail(SYMTD_EINVAL, "request %llu is not queued", (unsigned long long)id);
    std::lock_guard<std::mutex> lk(stage_mu_);
    staging_.release(rq->stage, rq->stage_bytes);
    cv_done_.notify_all();
    return SYMTD_OK;
  }

  symtd_status stats(symtd_server_stats* out) override {
    if (!out) return fail(SYMTD_EINVAL, "null stats");
    std::lock_guard<std::mutex> lk(mu_);
    *out = st_;
    out->queued = (int64_t)queue_.size();
    out->running = running_;
    out->memory_bytes = opts_.memory_bytes;
    return SYMTD_OK;
  }

 private:
  double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

  symtd_status fail(symtd_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4))) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(err_mu_);
    err = buf;
    return s;
  }
  symtd_status hip_fail(hipError_t e, const char* what) { return fail(SYMTD_EDEVICE, "%s: %s", what, hipGetErrorString(e)); }

  // the server thread
  void loop() {
    (void)hipSetDevice(opts_.device);
    const int K = opts_.check_every > 0 ? opts_.check_every : 4;
    std::vector<EngineInst<T>*> done;
    while (true) {
      std::vector<std::unique_ptr<Request<T>>> take;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (stop_) break;
        // admission in arrival order while the footprints fit the free memory
        size_t free_total = eng_->arena().size() - eng_->arena().used();
        size_t largest = eng_->arena().largest_free();
        while (!queue_.empty()) {
          const size_t need = Arena::round(queue_.front()->footprint);
          if (need > free_total || need > largest) break;
          free_total -= need;
          largest = need <= largest ? largest - need : 0;
          take.push_back(std::move(queue_.front()));
          queue_.pop_front();
        }
        if (take.empty() && running_ == 0) {
          cv_work_.wait_for(lk, std::chrono::milliseconds(20), [&] { return stop_ || !queue_.empty(); });
          continue;
        }
        running_ += (int64_t)take.size();
      }
      symtd_status s = SYMTD_OK;
      if (!take.empty()) {
        std::vector<EngineInst<T>*> batch;
        for (auto& rq : take) {
          rq->inst = std::make_unique<EngineInst<T>>();
          GroupEngine<T>::shape(*rq->inst, rq->pb, rq->o, 0);
          rq->inst->id = rq->id;
          rq->inst->carve(nullptr);
          rq->t_admit = now();
          batch.push_back(rq->inst.get());
        }
        Marker mk("server admission");
        s = eng_->admit(batch);
        if (s == SYMTD_EREJECTED) {
          // the free memory was too fragmented: back to the head of the queue
          std::lock_guard<std::mutex> lk(mu_);
          running_ -= (int64_t)take.size();
          for (auto it = take.rbegin(); it != take.rend(); ++it) {
            (*it)->inst.reset();
            queue_.push_front(std::move(*it));
          }
          take.clear();
          s = SYMTD_OK;
        } else if (s == SYMTD_OK) {
          // the engine holds its own copies now (admit synchronises its stream)
          hipError_t e = hipStreamSynchronize(eng_->stream());
          if (e != hipSuccess) s = hip_fail(e, "admission");
          std::lock_guard<std::mutex> lk(stage_mu_);
          for (auto& rq : take) {
            staging_.release(rq->stage, rq->stage_bytes);
            rq->stage = nullptr;
            live_[rq->inst.get()] = std::move(rq);
          }
          std::lock_guard<std::mutex> lk2(mu_);
          st_.admitted += (int64_t)take.size();
        }
      }
      if (s == SYMTD_OK && eng_->live() > 0) {
        s = eng_->run(K);
        if (s == SYMTD_OK) s = eng_->poll(done);
        if (s == SYMTD_OK) {
          for (auto* I : done) {
            symtd_server_result res{};
            s = finish(I, &res);
            if (s != SYMTD_OK) break;
            eng_->remove(I);
            live_.erase(I);
            std::lock_guard<std::mutex> lk(mu_);
            done_.push_back(res);
            ++st_.completed;
            --running_;
            st_.steps = eng_->steps();
            st_.memory_used = eng_->arena().used();
          }
          if (!done.empty()) cv_done_.notify_all();
          std::lock_guard<std::mutex> lk(mu_);
          st_.steps = eng_->steps();
          st_.memory_used = eng_->arena().used();
        }
      }
      if (s != SYMTD_OK) {
        fail(s, "%s", ctx_->err.c_str());
        abort_all(s);
        return;
      }
    }
  }

  symtd_status finish(EngineInst<T>* I, symtd_server_result* res) {
    Request<T>* rq = live_[I].get();
    const int64_t n = I->n, r = I->r;
    std::vector<T> Ah((size_t)n * r);
    symtd_solve_result out{};
    out.A = Ah.data();
    out.lda = n;
    res->lambda = (double*)std::malloc(sizeof(double) * r);
    res->A = (double*)std::malloc(sizeof(double) * n * r);
    if (!res->lambda || !res->A) return ctx_->fail(SYMTD_ENOMEM, "host result buffers");
    out.lambda = res->lambda;
    symtd_status s = eng_->collect(I, &out, true);
    if (s != SYMTD_OK) return s;
    for (size_t i = 0; i < Ah.size(); ++i) res->A[i] = (double)Ah[i];
    res->id = rq->id;
    res->status = SYMTD_OK;
    res->f = out.f; res->alpha = out.alpha; res->rel_err = out.rel_err;
    res->iters = out.iters; res->evals = out.evals;
    res->exit_reason = out.exit_reason; res->best_restart = out.best_restart;
    res->n = n; res->r = r;
    res->t_submit = rq->t_submit; res->t_admit = rq->t_admit; res->t_done = now();
    return SYMTD_OK;
  }

  // after a device error: every pending request completes with that status
  void abort_all(symtd_status s) {
    std::lock_guard<std::mutex> lk(mu_);
    broken_ = true;
    auto emit = [&](uint64_t id, double ts) {
      symtd_server_result res{};
      res.id = id;
      res.status = s;
      res.t_submit = ts;
      res.t_done = now();
      done_.push_back(res);
    };
    for (auto& kv : live_) emit(kv.second->id, kv.second->t_submit);
    for (auto& rq : queue_) emit(rq->id, rq->t_submit);
    live_.clear();
    queue_.clear();
    running_ = 0;
    cv_done_.notify_all();
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    if (thread_.joinable()) thread_.join();
    eng_.reset();
    live_.clear();
    queue_.clear();
    for (auto& r : done_) symtd_server_result_release(&r);
    done_.clear();
    if (copy_st_) (void)hipStreamDestroy(copy_st_);
    if (region_) (void)hipFree(region_);
    if (stage_region_) (void)hipFree(stage_region_);
    copy_st_ = nullptr; region_ = nullptr; stage_region_ = nullptr;
    if (ctx_) symtd_destroy(ctx_);
    if (vctx_) symtd_destroy(vctx_);
    ctx_ = nullptr;
    vctx_ = nullptr;
  }

  symtd_server_opts opts_{};
  Clock::time_point t0_;
  symtd_ctx* ctx_ = nullptr;
  symtd_ctx* vctx_ = nullptr;
  void* region_ = nullptr;
  void* stage_region_ = nullptr;
  size_t staging_bytes_ = 0;
  Arena staging_;
  hipStream_t copy_st_ = nullptr;
  std::unique_ptr<GroupEngine<T>> eng_;
  std::thread thread_;
  std::mutex mu_, stage_mu_, err_mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::unique_ptr<Request<T>>> queue_;
  std::deque<symtd_server_result> done_;
  std::map<EngineInst<T>*, std::unique_ptr<Request<T>>> live_;
  symtd_server_stats st_{};
  int64_t running_ = 0;
  uint64_t next_id_ = 1;
  bool stop_ = false, broken_ = false;
};

}  // namespace

extern "C" {

symtd_status symtd_server_create(const symtd_server_opts* o, symtd_server** out) {
  if (!o || !out) return SYMTD_EINVAL;
  *out = nullptr;
  if (!((o->dt == SYMTD_F64 && o->prec == SYMTD_PREC_FP64) || (o->dt == SYMTD_F32 && o->prec == SYMTD_PREC_FP32)))
    return SYMTD_EINVAL;
  if (o->memory_bytes < ((size_t)1 << 20) || o->check_every < 0) return SYMTD_EINVAL;
  symtd_server* s = nullptr;
  symtd_status st;
  if (o->dt == SYMTD_F64) {
    auto* srv = new (std::nothrow) Server<double>();
    if (!srv) return SYMTD_ENOMEM;
    st = srv->start(*o);
    s = srv;
  } else {
    auto* srv = new (std::nothrow) Server<float>();
    if (!srv) return SYMTD_ENOMEM;
    st = srv->start(*o);
    s = srv;
  }
  if (st != SYMTD_OK) {
    delete s;
    return st;
  }
  *out = s;
  return SYMTD_OK;
}

symtd_status symtd_server_submit(symtd_server* srv, const symtd_problem* pb, const symtd_solve_opts* o, uint64_t* id) {
  if (!srv) return SYMTD_EINVAL;
  return srv->submit(pb, o, id);
}

symtd_status symtd_server_poll(symtd_server* srv, symtd_server_result* out, int32_t max, int32_t* n_out,
                               int32_t timeout_ms) {
  if (!srv) return SYMTD_EINVAL;
  return srv->poll(out, max, n_out, timeout_ms);
}

symtd_status symtd_server_cancel(symtd_server* srv, uint64_t id) {
  if (!srv) return SYMTD_EINVAL;
  return srv->cancel(id);
}

symtd_status symtd_server_stats_get(symtd_server* srv, symtd_server_stats* out) {
  if (!srv) return SYMTD_EINVAL;
  return srv->stats(out);
}

const char* symtd_server_last_error(const symtd_server* srv) {
  if (!srv) return "null server";
  return srv->err.c_str();
}

void symtd_server_result_release(symtd_server_result* res) {
  if (!res) return;
  std::free(res->A);
  std::free(res->lambda);
  res->A = nullptr;
  res->lambda = nullptr;
}

void symtd_server_destroy(symtd_server* srv) { delete srv; }

}  // extern "C"
