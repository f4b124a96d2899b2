// ||X||^2 = nu' [V'V]^d nu (Lemma 3.4 applied to X; Section 3.3).
//
// The p x p Gram matrix V'V is visited in 128 x 128 tiles on fp64 matrix
// cores and never stored.  By symmetry only tiles on or above the diagonal
// are formed; an off-diagonal tile stands for itself and its mirror and is
// counted twice.  Each block writes one fp64 partial; a single-block kernel
// sums the partials in a fixed order, so the result is bitwise repeatable.
#include "kcommon.hpp"
#include "kernels.hpp"

namespace symtd {

// (row tile, column tile) of upper-triangular tile pair number b, enumerated
// row by row: row t holds the pairs (t, t), (t, t+1), ..., (t, T-1).
__device__ __forceinline__ void tri_pair(int64_t b, int64_t T, int64_t& tr, int64_t& tc) {
  const double bb = (double)(2 * T + 1);
  int64_t t = (int64_t)((bb - sqrt(bb * bb - 8.0 * (double)b)) * 0.5);
  if (t < 0) t = 0;
  if (t > T - 1) t = T - 1;
  auto start = [T](int64_t s) { return s * T - (s * (s - 1)) / 2; };
  while (t > 0 && start(t) > b) --t;
  while (t + 1 < T && start(t + 1) <= b) ++t;
  tr = t;
  tc = t + (b - start(t));
}

// Elements i .. i+3 of a column of n, loaded from addresses clamped into the
// column, without branches.  VEC (16-byte aligned columns, leading dimension
// a multiple of 4 elements, so a column holds 4 ceil(n/4) elements): one
// vector load of the quad; otherwise four loads.  Element e is valid only
// when i + e < n (and the column exists): nx_elem zeroes the rest where the
// quad is used, so that the load itself is not waited for when it is issued.
template <typename S, bool VEC>
__device__ __forceinline__ void nx_load(Quad<S>& q, const S* col, int64_t i, int64_t n) {
  if constexpr (VEC) {
    const int64_t n4 = (n + 3) & ~(int64_t)3;
    vload4(q, col + (i < n4 ? i : n4 - 4));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) q.e[e] = gload(col + min(i + e, n - 1));
  }
}
template <typename S>
__device__ __forceinline__ double nx_elem(const Quad<S>& q, int e, int64_t i, int64_t n, bool ok) {
  return (ok && i + e < n) ? (double)q.e[e] : 0.0;
}

// tile pair b of data set a, weighted, into *out (a whole block of 256 threads)
template <typename S, bool VEC>
__device__ __forceinline__ void normx_pair(const NormXArgs<S>& a, int64_t b, double* out) {
  using acc_t = v4d;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int g = lane >> 4, c = lane & 15;
  int64_t tr, tc;
  tri_pair(b, a.ntile, tr, tc);
  const int64_t rbase = tr * 128 + (wave >> 1) * 64;
  const int64_t cbase = tc * 128 + (wave & 1) * 64;

  const S* rp[4]; bool rok[4];
  const S* cp[4]; bool cok[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int64_t lr = rbase + 16 * m + c, lc = cbase + 16 * m + c;
    rok[m] = lr < a.p; cok[m] = lc < a.p;
    rp[m] = a.V + (rok[m] ? lr : 0) * a.ldv;
    cp[m] = a.V + (cok[m] ? lc : 0) * a.ldv;
  }
  acc_t acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = acc_t{0, 0, 0, 0};
  // the accumulators stay in AGPRs (left to the compiler, all of them are
  // copied to VGPRs and back at every 16-k step)
  auto pin = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) asm("" : "+a"(acc[m][q]));
  };
  pin();

  // the 16-k steps' row and column quads come through a register ring three
  // deep: the loads of step s + 2 are issued before step s is multiplied.
  // Steps past n load clamped addresses and are zero-filled (never used).
  const int64_t n = a.n;
  auto load = [&](Quad<S> (&rq)[4], Quad<S> (&cq)[4], int64_t i0) {
    const int64_t i = i0 + 4 * g;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      nx_load<S, VEC>(rq[m], rp[m], i, n);
      nx_load<S, VEC>(cq[m], cp[m], i, n);
    }
  };
  auto step = [&](const Quad<S> (&rq)[4], const Quad<S> (&cq)[4], int64_t i0) {
    const int64_t i = i0 + 4 * g;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double x[4], y[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        x[m] = nx_elem(rq[m], s, i, n, rok[m]);
        y[m] = nx_elem(cq[m], s, i, n, cok[m]);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = Mfma<double>::mac(x[m], y[q], acc[m][q]);
    }
    pin();
  };
  Quad<S> ra[4], ca[4], rb[4], cb[4], rc[4], cc[4];
  load(ra, ca, 0);
  load(rb, cb, 16);
  int64_t i0 = 0;
  // (the scheduling barriers keep each step's loads where they are written:
  // left to itself the scheduler sinks them to the end of the loop body and
  // the next step then waits for nearly every load in flight)
  for (; i0 + 32 < n; i0 += 48) {          // three steps, each reaching below n
    load(rc, cc, i0 + 32);
    __builtin_amdgcn_sched_barrier(0);
    step(ra, ca, i0);
    __builtin_amdgcn_sched_barrier(0);
    load(ra, ca, i0 + 48);
    __builtin_amdgcn_sched_barrier(0);
    step(rb, cb, i0 + 16);
    __builtin_amdgcn_sched_barrier(0);
    load(rb, cb, i0 + 64);
    __builtin_amdgcn_sched_barrier(0);
    step(rc, cc, i0 + 32);
    __builtin_amdgcn_sched_barrier(0);
  }
  // now i0 + 32 >= n: at most two steps remain, held in ra/ca and rb/cb
  if (i0 < n) step(ra, ca, i0);
  if (i0 + 16 < n) step(rb, cb, i0 + 16);

  // acc[m][q][v] = (V'V)[rbase + 16m + row(g, v)][cbase + 16q + c]
  double nc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t l = cbase + 16 * q + c;
    nc[q] = l < a.p ? a.nu[l] : 0.0;
  }
  double sum = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t l = rbase + 16 * m + Mfma<double>::row(g, v);
      const double nr = l < a.p ? a.nu[l] : 0.0;
      double rs = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) rs += nc[q] * ipow(acc[m][q][v], a.d);
      sum += nr * rs;
    }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) sum += __shfl_xor(sum, o);
  __shared__ double red[4];
  if (lane == 0) red[wave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double w = (tr == tc) ? 1.0 : 2.0;
    *out = w * (((red[0] + red[1]) + red[2]) + red[3]);
  }
}

template <typename S, bool VEC>
__global__ __launch_bounds__(256) void k_normx(NormXArgs<S> a) {
  normx_pair<S, VEC>(a, blockIdx.x, a.part + blockIdx.x);
}

template <typename S>
__global__ __launch_bounds__(256) void k_gnormx(const GNormX<S>* sets, const NormXItem* items) {
  const NormXItem it = items[blockIdx.x];
  const NormXArgs<S> a = sets[it.set].a;
  normx_pair<S, true>(a, it.pair, a.part + it.pair);
}

// the partials of one set summed in a fixed order: each thread takes a
// strided share, eight loads in flight per round (added pairwise), then a
// tree over the block
constexpr int REDUCE_THREADS = 1024;
__device__ __forceinline__ void reduce_body(const double* part, int64_t count, double* out) {
  __shared__ double s[REDUCE_THREADS];
  constexpr int R = REDUCE_THREADS;
  double acc = 0.0;
  int64_t e = threadIdx.x;
  for (; e + 7 * R < count; e += 8 * R) {
    double v[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) v[h] = part[e + h * R];
    acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  for (; e < count; e += R) acc += part[e];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = R / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

__global__ __launch_bounds__(REDUCE_THREADS) void k_reduce(ReduceArgs a) { reduce_body(a.part, a.count, a.out); }

template <typename S>
__global__ __launch_bounds__(REDUCE_THREADS) void k_greduce(const GNormX<S>* sets) {
  const GNormX<S> g = sets[blockIdx.x];
  reduce_body(g.a.part, g.pairs, g.alpha);
}

void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<float>& a) {
  if (vec) hipLaunchKernelGGL((k_normx<float, true>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_normx<float, false>), grid, dim3(256), 0, st, a);
}
void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<double>& a) {
  if (vec) hipLaunchKernelGGL((k_normx<double, true>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_normx<double, false>), grid, dim3(256), 0, st, a);
}
void launch_reduce(hipStream_t st, const ReduceArgs& a) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(REDUCE_THREADS), 0, st, a);
}
template <typename S>
static void launch_normx_grouped_t(int nitems, int nsets, hipStream_t st, const GNormX<S>* sets,
                                   const NormXItem* items) {
  if (nitems <= 0 || nsets <= 0) return;
  hipLaunchKernelGGL(k_gnormx<S>, dim3(nitems), dim3(256), 0, st, sets, items);
  hipLaunchKernelGGL(k_greduce<S>, dim3(nsets), dim3(REDUCE_THREADS), 0, st, sets);
}
void launch_normx_grouped(int nitems, int nsets, hipStream_t st, const GNormX<float>* sets, const NormXItem* items) {
  launch_normx_grouped_t(nitems, nsets, st, sets, items);
}
void launch_normx_grouped(int nitems, int nsets, hipStream_t st, const GNormX<double>* sets, const NormXItem* items) {
  launch_normx_grouped_t(nitems, nsets, st, sets, items);
}

}  // namespace symtd
