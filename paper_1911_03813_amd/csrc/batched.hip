// Batched entry points: the grouped evaluation of many instances and the
// batched solve on the grouped engine (engine.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "engine.hpp"
#include "grouped.hpp"
#include "runtime.hpp"

using namespace symtd;

namespace {

template <typename T>
symtd_status run_fg_batched(symtd_ctx* ctx, hipStream_t st, int64_t count, const symtd_fg_item* items) {
  // workspace of every instance, then the tables
  const int NTM = sizeof(T) == 8 ? GG_NT_F64 : GG_NT_F32;
  std::vector<GInst<T>> gi(count);
  std::vector<GItem> g1, gm, g2, gf;
  bool vec = true;
  Carver c(nullptr);
  auto plan = [&](Carver& cv) {
    for (int64_t i = 0; i < count; ++i) {
      const symtd_fg_item& it = items[i];
      GInst<T>& G = gi[i];
      const int64_t n = it.n, p = it.p, r = it.r, R = it.models, cols = r * R;
      G.V = (const T*)it.V; G.ldv = it.ldv; G.nu = it.nu;
      G.n = (int)n; G.p = (int)p; G.d = it.d; G.r = (int)r; G.R = (int)R; G.cols = (int)cols;
      G.nt = (int)((cols + 15) / 16);
      G.A = (const T*)it.A; G.lda = it.lda; G.lam = it.lambda;
      G.f = it.f; G.glam = it.g_lambda; G.G = (T*)it.G_A; G.ldg = it.ldg;
      G.alpha = it.alpha;
      const int64_t nblk = (p + 15) / 16;
      G.ntile = (int)((p + GG1_TILE - 1) / GG1_TILE);
      G.split_blk = grouped_split_blocks(sizeof(T) == 8, n, p, cols);
      G.nsplit = (int)((nblk + G.split_blk - 1) / G.split_blk);
      G.ldy = 64 * ((n + 63) / 64);
      G.Wp = cv.take<T>((size_t)nblk * G.nt * 256);
      G.wpart = cv.take<double>((size_t)G.ntile * cols);
      G.Ypart = cv.take<T>((size_t)G.nsplit * G.nt * 16 * G.ldy);
      G.B = cv.take<double>((size_t)R * r * r);
      G.C = cv.take<double>((size_t)R * r * r);
      G.YM = cv.take<double>((size_t)n * cols);
    }
  };
  plan(c);
  for (int64_t i = 0; i < count; ++i) {
    const GInst<T>& G = gi[i];
    const int ncg = (G.nt + NTM - 1) / NTM;
    for (int t = 0; t < G.ntile; ++t)
      for (int cg = 0; cg < ncg; ++cg) g1.push_back({(int)i, t, cg, 0});
    for (int k = 0; k < G.R; ++k) gm.push_back({(int)i, k, 0, 0});
    for (int rb = 0; rb < (G.n + 63) / 64; ++rb)
      for (int sp = 0; sp < G.nsplit; ++sp)
        for (int cg = 0; cg < ncg; ++cg) g2.push_back({(int)i, rb, sp, cg});
    for (int col = 0; col < G.cols; ++col) gf.push_back({(int)i, col, 0, 0});
    vec = vec && (G.ldv % 4 == 0) && (G.lda % 4 == 0) && ((uintptr_t)G.V % 16 == 0) && ((uintptr_t)G.A % 16 == 0);
  }
  std::vector<GItem> all;
  all.insert(all.end(), g1.begin(), g1.end());
  all.insert(all.end(), gm.begin(), gm.end());
  all.insert(all.end(), g2.begin(), g2.end());
  all.insert(all.end(), gf.begin(), gf.end());
  const size_t ws_work = c.off;
  Carver ct(nullptr);
  ct.off = ws_work;
  ct.take<GInst<T>>(count);
  ct.take<GItem>(all.size());
  symtd_status s = ctx->reserve(ct.off + 256);
  if (s != SYMTD_OK) return s;
  Carver cw(ctx->ws);
  plan(cw);
  GInst<T>* d_gi = cw.take<GInst<T>>(count);
  GItem* d_items = cw.take<GItem>(all.size());
  hipError_t e;
  if ((e = hipMemcpyAsync(d_gi, gi.data(), sizeof(GInst<T>) * count, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(d_items, all.data(), sizeof(GItem) * all.size(), hipMemcpyHostToDevice, st)) != hipSuccess)
    return ctx->hip_fail(e, "batched tables");
  const int n1 = (int)g1.size(), nm = (int)gm.size(), n2 = (int)g2.size(), nf = (int)gf.size();
  launch_ggemm1<T>(vec, n1, st, d_gi, d_items);
  launch_gmodel<T>(nm, st, d_gi, d_items + n1);
  launch_ggemm2<T>(vec, n2, st, d_gi, d_items + n1 + nm);
  launch_gfinal<T>(nf, st, d_gi, d_items + n1 + nm + n2);
  if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "batched kernels");
  // the host tables are read by the copies above before they go out of scope
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return ctx->hip_fail(e, "batched sync");
  return SYMTD_OK;
}

template <typename T>
symtd_status run_solve_batched(symtd_ctx* ctx, hipStream_t st, int64_t count, const symtd_problem* pbs,
                               const symtd_solve_opts* opts, symtd_solve_result* outs) {
  std::vector<std::unique_ptr<EngineInst<T>>> insts;
  size_t total = 0;
  int64_t max_evals = 1;
  for (int64_t i = 0; i < count; ++i) {
    auto I = std::make_unique<EngineInst<T>>();
    GroupEngine<T>::shape(*I, pbs[i], opts[i], outs[i].f_trace ? outs[i].trace_len : 0);
    I->id = (uint64_t)i;
    I->carve(nullptr);
    total += Arena::round(I->bytes);
    max_evals = std::max(max_evals, opts[i].max_evals);
    insts.push_back(std::move(I));
  }
  symtd_status s = ctx->reserve_solver(total + 4096);
  if (s != SYMTD_OK) return s;
  GroupEngine<T> eng(ctx);
  if ((s = eng.init(st, (char*)ctx->sws, total + 4096, ctx->tune_graph != 0)) != SYMTD_OK) return s;
  std::vector<EngineInst<T>*> batch;
  for (auto& I : insts) batch.push_back(I.get());
  if ((s = eng.admit(batch)) != SYMTD_OK) return s;
  const int K = opts[0].check_every > 0 ? opts[0].check_every : 8;
  std::vector<EngineInst<T>*> done;
  while (eng.live() > 0) {
    if ((s = eng.run(K)) != SYMTD_OK) return s;
    if ((s = eng.poll(done)) != SYMTD_OK) return s;
    std::vector<symtd_solve_result*> res;
    for (auto* I : done) res.push_back(&outs[I->id]);
    if ((s = eng.collect_many(done, res, false)) != SYMTD_OK) return s;
    for (auto* I : done) eng.remove(I);
    if (eng.steps() > max_evals + 2 * K)
      return ctx->fail(SYMTD_EDEVICE, "batched solve did not stop within %lld steps", (long long)eng.steps());
  }
  for (int64_t i = 0; i < count; ++i) outs[i].steps = eng.steps();
  return eng.join(st);
}

}  // namespace

extern "C" {

symtd_status symtd_fg_batched(symtd_ctx* ctx, void* stream, symtd_dtype dt, symtd_prec prec, int64_t count,
                              const symtd_fg_item* items) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  if (symtd_status s0 = ctx->take_device_error(); s0 != SYMTD_OK) return s0;
  if (count < 0 || (count > 0 && !items)) return ctx->fail(SYMTD_EINVAL, "bad item list");
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)dt, (int)prec);
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  for (int64_t i = 0; i < count; ++i) {
    const symtd_fg_item& it = items[i];
    symtd_status s = ctx->check_common(dt, it.V, it.ldv, it.nu, it.n, it.p, it.d);
    if (s != SYMTD_OK) return ctx->fail(s, "item %lld: %s", (long long)i, ctx->err.c_str());
    if (it.r < 1 || it.models < 1 || it.r * it.models > 0x7fffffffLL)
      return ctx->fail(SYMTD_EINVAL, "item %lld: bad r or models", (long long)i);
    if (it.lda < it.n || it.ldg < it.n) return ctx->fail(SYMTD_EINVAL, "item %lld: lda/ldg < n", (long long)i);
    if (!it.A || !it.lambda || !it.f || !it.g_lambda || !it.G_A)
      return ctx->fail(SYMTD_EINVAL, "item %lld: null pointer", (long long)i);
    if (((uintptr_t)it.A % esz) || ((uintptr_t)it.G_A % esz) || ((uintptr_t)it.lambda % 8) || ((uintptr_t)it.f % 8) ||
        ((uintptr_t)it.g_lambda % 8))
      return ctx->fail(SYMTD_EALIGN, "item %lld: misaligned pointer", (long long)i);
  }
  if (count == 0) return SYMTD_OK;
  symtd_status s = ctx->set_device();
  if (s != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64) return run_fg_batched<double>(ctx, st, count, items);
  return run_fg_batched<float>(ctx, st, count, items);
}

symtd_status symtd_solve_batched(symtd_ctx* ctx, void* stream, int64_t count, const symtd_problem* pbs,
                                 const symtd_solve_opts* opts, symtd_solve_result* outs) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  if (symtd_status s0 = ctx->take_device_error(); s0 != SYMTD_OK) return s0;
  if (count < 0 || (count > 0 && (!pbs || !opts || !outs))) return ctx->fail(SYMTD_EINVAL, "bad problem list");
  for (int64_t i = 0; i < count; ++i) {
    symtd_status s = check_solve(ctx, &pbs[i], &opts[i], &outs[i]);
    if (s != SYMTD_OK) return ctx->fail(s, "problem %lld: %s", (long long)i, ctx->err.c_str());
    if (opts[i].sigma != 0.0)
      return ctx->fail(SYMTD_EINVAL, "problem %lld: the noise correction is symtd_solve's only", (long long)i);
    if (opts[i].pause_after != 0 || opts[i].state_out || opts[i].state_in)
      return ctx->fail(SYMTD_EINVAL, "problem %lld: pausing and resuming are symtd_solve's only", (long long)i);
    if (pbs[i].dt != pbs[0].dt) return ctx->fail(SYMTD_EINVAL, "problem %lld: all problems must share a dtype", (long long)i);
  }
  if (count == 0) return SYMTD_OK;
  symtd_status s = ctx->set_device();
  if (s != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  Marker mk("symtd_solve_batched");
  if (pbs[0].dt == SYMTD_F64) s = run_solve_batched<double>(ctx, st, count, pbs, opts, outs);
  else s = run_solve_batched<float>(ctx, st, count, pbs, opts, outs);
  if (s != SYMTD_OK) return s;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return ctx->hip_fail(e, "batched solve sync");
  return SYMTD_OK;
}

}  // extern "C"
