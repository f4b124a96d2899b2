// Stochastic objective (Section 5, Lemma 5.1) and the device Adam solver.
//
// A draw is s columns of V taken uniformly with replacement; sample k of draw
// t under `seed` is word k mod 4 of the Philox-4x32-10 block with counter
// (k / 4, t low word, t high word, stream) and key (seed low, seed high)
// (philox.hpp), mapped to the column floor(x p / 2^32).  The sampled data
// set is those columns with weights p nu_i / s, so that its moment tensor is
// an unbiased estimate of X (Lemma 5.1 for nu = 1/p, where the weights are
// 1/s).  Training draws use stream STREAM_SAMPLE with t = the number of
// gradient steps taken before; the fixed set on which the objective is
// estimated after every epoch uses stream STREAM_ESTIMATE, t = 0.
//
// Adam (Kingma & Ba, ICLR 2015) runs one lane per restart over
// x = [lambda; vec A]; all lanes step together on the same draw (their
// columns side by side in one evaluation).  After every epoch the shifted
// objective is estimated on the fixed set: a decrease keeps the state as the
// lane's snapshot; otherwise the snapshot (x, m, v, t) is restored and the
// learning rate drops from lr0 to lr1, and the second time the lane stops
// on its snapshot (Section 5).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

constexpr uint32_t STREAM_SAMPLE = 3, STREAM_ESTIMATE = 4;

// the gathered columns: Vs has leading dimension lds (rows n .. lds-1 zero)
template <typename T>
struct GatherArgs {
  const T* V; int64_t ldv; const double* nu; int64_t n, p;
  int64_t s; uint64_t seed; uint32_t stream;
  const int64_t* draw;          // device word holding t (null: use draw0)
  int64_t draw0;
  T* Vs; int64_t lds; double* nus;
  int64_t* idx;                 // the indices (optional, null)
};
template <typename T>
void launch_gather(hipStream_t st, const GatherArgs<T>& a);

enum AdamAction : int { AD_NONE = 0, AD_ACCEPT = 1, AD_RESTORE = 2 };
enum AdamReason : int { AD_RUNNING = 0, AD_CONVERGED = 1, AD_MAX_EPOCHS = 2 };

struct AdamState {
  int64_t t, t_saved;           // Adam's step count (bias correction), and at the snapshot
  int64_t steps, epochs;        // gradient steps taken, epochs completed
  double lr, f_prev;            // learning rate, last accepted estimate
  int fails, done, action, reason;
};

// One lane: x = [lambda; vec A] (N = r + n r, A column-major with leading
// dimension n); m, v the moments; xs, ms, vs the snapshot.  The trial point
// (the evaluation's inputs) is kept equal to x.
template <typename T>
struct AdamLane {
  int64_t N; int r; int n;
  double *x, *m, *v, *xs, *ms, *vs;
  double* lam_t; T* A_t;                         // evaluation inputs
  const double* glam; const T* G;                // evaluation outputs (gradient)
  const double* f_est;                           // estimate of this lane's objective
  AdamState* state;
  double* trace; int64_t trace_len;              // estimates: start, then after every epoch
};

struct AdamParams {
  double lr0, lr1, beta1, beta2, eps;
  int64_t max_epochs;
  int64_t* draw;                                 // global draw counter
  int* done_count;                               // lanes stopped (incremented once per lane)
};

constexpr int AD_CHUNK = 1024;
// Adam step of every running lane (grid: chunks x lanes)
template <typename T>
void launch_adam_step(int nb, int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm);
// t += 1 for running lanes, the draw counter += 1
template <typename T>
void launch_adam_tick(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm);
// first estimate: f_prev, trace[0], lr = lr0, action = ACCEPT (snapshot = x)
template <typename T>
void launch_adam_init(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm);
// end of an epoch: accept or restore, learning rate, stop
template <typename T>
void launch_adam_decide(int lanes, hipStream_t st, const AdamLane<T>* L, AdamParams prm);
// the copies the decision asks for (grid: chunks x lanes)
template <typename T>
void launch_adam_apply(int nb, int lanes, hipStream_t st, const AdamLane<T>* L);

}  // namespace symtd
