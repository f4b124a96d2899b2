// Kernels of the stochastic objective and the device Adam solver (stoch.hpp).
#include <math.h>

#include "kcommon.hpp"
#include "philox.hpp"
#include "stoch.hpp"

namespace symtd {

// block (k, y): sample k, rows [256 y, 256 y + 256) of its column
template <typename T>
__global__ __launch_bounds__(256) void k_gather(GatherArgs<T> a) {
  const int64_t k = blockIdx.x;
  const int64_t t = a.draw ? gload(a.draw) : a.draw0;
  uint32_t c[4] = {(uint32_t)(k >> 2), (uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), a.stream};
  philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  const uint32_t x = c[k & 3];
  const int64_t l = (int64_t)(((uint64_t)x * (uint64_t)a.p) >> 32);
  const int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (i < a.lds) a.Vs[k * a.lds + i] = i < a.n ? a.V[l * a.ldv + i] : T(0);
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    a.nus[k] = (double)a.p * a.nu[l] / (double)a.s;
    if (a.idx) a.idx[k] = l;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adam_step(const AdamLane<T>* lanes, AdamParams prm) {
  const AdamLane<T> L = lanes[blockIdx.y];
  const AdamState s = *L.state;
  if (s.done) return;
  const double t = (double)(s.t + 1);
  const double c1 = 1.0 - pow(prm.beta1, t), c2 = 1.0 - pow(prm.beta2, t);
  for (int q = 0; q < AD_CHUNK / 256; ++q) {
    const int64_t e = (int64_t)blockIdx.x * AD_CHUNK + q * 256 + threadIdx.x;
    if (e >= L.N) break;
    const double g = e < L.r ? L.glam[e] : (double)L.G[e - L.r];
    const double m = prm.beta1 * L.m[e] + (1.0 - prm.beta1) * g;
    const double v = prm.beta2 * L.v[e] + (1.0 - prm.beta2) * (g * g);
    const double mhat = m / c1, vhat = v / c2;
    const double x = L.x[e] - s.lr * mhat / (sqrt(vhat) + prm.eps);
    L.m[e] = m;
    L.v[e] = v;
    L.x[e] = x;
    if (e < L.r) L.lam_t[e] = x;
    else L.A_t[e - L.r] = (T)x;
  }
}

template <typename T>
__global__ void k_adam_tick(const AdamLane<T>* lanes, int nl, AdamParams prm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *prm.draw += 1;
  if (i >= nl) return;
  AdamState* s = lanes[i].state;
  if (!s->done) {
    s->t += 1;
    s->steps += 1;
  }
}

template <typename T>
__global__ void k_adam_init(const AdamLane<T>* lanes, int nl, AdamParams prm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const AdamLane<T>& L = lanes[i];
  AdamState* s = L.state;
  const double fe = *L.f_est;
  s->t = s->t_saved = s->steps = s->epochs = 0;
  s->lr = prm.lr0;
  s->f_prev = fe;
  s->fails = s->done = 0;
  s->reason = AD_RUNNING;
  s->action = AD_ACCEPT;
  if (L.trace && L.trace_len > 0) L.trace[0] = fe;
}

template <typename T>
__global__ void k_adam_decide(const AdamLane<T>* lanes, int nl, AdamParams prm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const AdamLane<T>& L = lanes[i];
  AdamState* s = L.state;
  if (s->done) {
    s->action = AD_NONE;
    return;
  }
  s->epochs += 1;
  const double fe = *L.f_est;
  if (L.trace && s->epochs < L.trace_len) L.trace[s->epochs] = fe;
  if (fe < s->f_prev) {
    s->f_prev = fe;
    s->t_saved = s->t;
    s->action = AD_ACCEPT;
  } else {
    s->t = s->t_saved;
    s->fails += 1;
    s->action = AD_RESTORE;
    if (s->fails == 1) {
      s->lr = prm.lr1;
    } else {
      s->done = 1;
      s->reason = AD_CONVERGED;
    }
  }
  if (!s->done && s->epochs >= prm.max_epochs) {
    s->done = 1;
    s->reason = AD_MAX_EPOCHS;
  }
  if (s->done) atomicAdd(prm.done_count, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void k_adam_apply(const AdamLane<T>* lanes) {
  const AdamLane<T> L = lanes[blockIdx.y];
  const int act = L.state->action;
  if (act == AD_NONE) return;
  for (int q = 0; q < AD_CHUNK / 256; ++q) {
    const int64_t e = (int64_t)blockIdx.x * AD_CHUNK + q * 256 + threadIdx.x;
    if (e >= L.N) break;
    if (act == AD_ACCEPT) {
      L.xs[e] = L.x[e];
      L.ms[e] = L.m[e];
      L.vs[e] = L.v[e];
    } else {
      const double x = L.xs[e];
      L.x[e] = x;
      L.m[e] = L.ms[e];
      L.v[e] = L.vs[e];
      if (e < L.r) L.lam_t[e] = x;
      else L.A_t[e - L.r] = (T)x;
    }
  }
}

template <typename T>
void launch_gather(hipStream_t st, const GatherArgs<T>& a) {
  const unsigned gy = (unsigned)((a.lds + 255) / 256);
  hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)a.s, gy), dim3(256), 0, st, a);
}
template <typename T>
void launch_adam_step(int nb, int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm) {
  hipLaunchKernelGGL(k_adam_step<T>, dim3(nb, lanes), dim3(256), 0, st, L, prm);
}
template <typename T>
void launch_adam_tick(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm) {
  hipLaunchKernelGGL(k_adam_tick<T>, dim3((lanes + 255) / 256), dim3(256), 0, st, L, lanes, prm);
}
template <typename T>
void launch_adam_init(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm) {
  hipLaunchKernelGGL(k_adam_init<T>, dim3((lanes + 255) / 256), dim3(256), 0, st, L, lanes, prm);
}
template <typename T>
void launch_adam_decide(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm) {
  hipLaunchKernelGGL(k_adam_decide<T>, dim3((lanes + 255) / 256), dim3(256), 0, st, L, lanes, prm);
}
template <typename T>
void launch_adam_apply(int nb, int lanes, hipStream_t st, const AdamLane<T>* L) {
  hipLaunchKernelGGL(k_adam_apply<T>, dim3(nb, lanes), dim3(256), 0, st, L);
}

#define SYMTD_INST(T)                                                                                  \
  template void launch_gather<T>(hipStream_t, const GatherArgs<T>&);                                  \
  template void launch_adam_step<T>(int, int, hipStream_t, const AdamLane<T>*, AdamParams);           \
  template void launch_adam_tick<T>(int, hipStream_t, const AdamLane<T>*, AdamParams);                \
  template void launch_adam_init<T>(int, hipStream_t, const AdamLane<T>*, AdamParams);                \
  template void launch_adam_decide<T>(int, hipStream_t, const AdamLane<T>*, AdamParams);              \
  template void launch_adam_apply<T>(int, int, hipStream_t, const AdamLane<T>*);
SYMTD_INST(float)
SYMTD_INST(double)
#undef SYMTD_INST

}  // namespace symtd
