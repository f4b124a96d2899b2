// Device-resident L-BFGS: lane descriptors, per-lane state and launchers.
//
// A lane is one optimisation (one restart of one problem) over
// x = [lambda; vec(A)] (N = r + n r values, A column-major).  Its vectors live
// on the device: x, the accepted gradient g, the direction d and the m
// curvature pairs S, Y (slot-major).  The trial point is written straight
// into the evaluation's inputs (lambda_t fp64, A_t in the storage type with
// leading dimension n) and the evaluation's outputs (f_t, g_lambda_t, G_t with
// leading dimension n) are read back as the trial gradient.
//
// One evaluation step is: evaluate (f_t, gradient) at every lane's trial
// point; k_lb_dots (all inner products the step needs, one pass over the
// lane's vectors); k_lb_step (one thread per lane: the line search and, on
// acceptance, the new direction in the compact representation of Byrd,
// Nocedal and Schnabel, Math. Prog. 63 (1994), eq. (3.13)); k_lb_apply
// (elementwise: accept, store the pair, form the direction, write the next
// trial point).  The launch sequence is the same for every step whatever the
// lanes decide, so the host never waits on a decision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

constexpr int LB_MMAX = 8;            // largest L-BFGS memory
constexpr int LB_CHUNK = 1024;        // vector elements per block of the dot/apply kernels
// inner products computed per lane and evaluation (see k_lb_dots)
constexpr int LB_GTGT = 0, LB_GTD = 1, LB_YTYT = 2, LB_YTD = 3, LB_YTGT = 4, LB_MAXG = 5;
constexpr int LB_GTS = 6, LB_GTY = LB_GTS + LB_MMAX, LB_SYT = LB_GTY + LB_MMAX, LB_YYT = LB_SYT + LB_MMAX;
constexpr int LB_ND = LB_YYT + LB_MMAX;

enum LbPhase : int { LB_START = 0, LB_BRACKET = 1, LB_ZOOM = 2, LB_DONE = 3 };
enum LbAction : int { LB_NONE = 0, LB_START_DIR = 1, LB_TRIAL = 2, LB_ACCEPT_DIR = 3, LB_ACCEPT_FINAL = 4,
                      LB_RESTORE = 5 };

// x holds A with leading dimension ld >= n (N = r + ld r); rows n .. ld-1 of
// A stay zero (their gradient is zero), so the vector kernels need no masking.
template <typename T>
struct LbLane {
  int64_t N; int n; int r; int ld;
  int nb;                       // blocks of LB_CHUNK elements: ceil(N / LB_CHUNK)
  int inst;                     // instance of a grouped solve (0 for a single problem)
  uint64_t seed; int restart;   // key and counter word of the lane's start draws
  const T* A0;                  // caller's start (leading dimension n), or null
  double* x; double* g; double* d; double* S; double* Y;   // S, Y: [m][N]
  double* lam_t; T* A_t;        // trial point (evaluation inputs), A_t leading dimension ld
  const double* f_t; const double* glam_t; const T* G_t;   // evaluation outputs, G_t leading dimension ld
  double scale;                 // phi = f / scale
  double* part;                 // [nb][LB_ND] dot partials
  double* trace; int64_t trace_len;   // f after every accepted step (device), or null
  struct LbState* state;        // this lane's state
  int* done_flag;               // set to 1 when the lane stops, or null
  // options
  int m;
  double pgtol, ftol;
  int64_t max_iters, max_evals;
};

struct LbParams {
  int* done_count;              // lanes that reached LB_DONE (incremented once per lane), or null
};

// Per-lane state (device memory, zero-initialised = phase LB_START).
struct LbState {
  int phase, reason, action, store;
  int count, head, slot, ls_i;
  int64_t iters, evals, ls_evals, ls_limit;
  double f;                     // accepted phi
  double dphi0;                 // slope along d at the accepted point
  double a, a_acc;              // next trial step, accepted step
  double a_prev, f_prev, d_prev;
  double lo_a, lo_f, lo_d, hi_a, hi_f, hi_d;
  int hi_fin, pad;
  double gamma, coef_g;
  double cs[LB_MMAX], cy[LB_MMAX];
  double SY[LB_MMAX][LB_MMAX];  // SY[i][j] = s_i' y_j by ring slot (upper part in time order)
  double YY[LB_MMAX][LB_MMAX];
};

// A block of the dot and apply kernels: chunk `blk` of lane `lane`.  With a
// list of them (the grouped engine), only the chunks the lanes have are
// launched; without one the grid is (largest chunk count) x lanes and blocks
// past a lane's own count return at once.
struct LbItem { int lane, blk; };

template <typename T>
void launch_lb_dots(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev,
                    const LbItem* items = nullptr, int nitems = 0);
template <typename T>
void launch_lb_step(int lanes, hipStream_t st, const LbLane<T>* lanes_dev, const LbParams& prm);
template <typename T>
void launch_lb_apply(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev,
                     const LbItem* items = nullptr, int nitems = 0);

// Starts.  Gaussian: A_0 columns of normals (stream 1) into x; RRF: Omega
// (stream 2) into the packed layout of the second product.  Then column
// normalisation and lambda_0 = 1, and the start becomes the first trial point.
template <typename T>
void launch_init_gauss(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev);
template <typename T>
void launch_omega_packed(dim3 grid, hipStream_t st, T* Wp, int64_t p, int r, int restarts, int nt_tot,
                         int64_t nblk, uint64_t seed);
// x[r + j n + i] of lane k = the fp64 sum over `nsplit` partials of column
// (k r + j) (layout [split][rp][npad]), then columns normalised (one block per
// column of each lane), lambda = 1, trial point = x.
template <typename T>
void launch_rrf_finish(int lanes, int r, hipStream_t st, const LbLane<T>* lanes_dev, const T* Ypart, int64_t npad,
                       int64_t rp, int nsplit);
// columns of A_0 given by the caller (type T, leading dimension n): into x,
// lambda = 1, trial point = x (no normalisation)
template <typename T>
void launch_init_given(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev);
template <typename T>
void launch_norm_cols(int lanes, int r, hipStream_t st, const LbLane<T>* lanes_dev);
// grouped randomized range finder: lane (instance i, restart k) takes columns
// k r .. of instance i's second-product partials
template <typename T> struct GInst;
template <typename T>
void launch_grrf_finish(int lanes, int rmax, hipStream_t st, const LbLane<T>* lanes_dev, const GInst<T>* insts);

}  // namespace symtd
