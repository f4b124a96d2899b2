// Device-side building blocks shared by the symtd kernels (gfx950 / CDNA4).
//
// Matrix-core products use the 16x16x4 fp32 and fp64 MFMA instructions.  For
// both, with lane = 16*g + c (g = lane / 16, c = lane % 16):
//   A operand (16 x 4): lane supplies A[c][g]
//   B operand (4 x 16): lane supplies B[g][c]
//   D (16 x 16):        lane holds D[row(g, v)][c] in element v = 0..3, where
//                       row(g, v) = 4*g + v for fp32 and g + 4*v for fp64
// (checked on gfx950 hardware).  The kernels permute the k index freely (a
// product's k index is only a summation index), which lets each lane read 4
// consecutive elements of a column with one vector load and feed them to 4
// successive MFMAs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;

template <> struct Mfma<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <> struct Mfma<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// The narrow forms, for a column subtile of at most 4 columns (lane =
// 16 g + c; layouts checked on gfx950 hardware).  In both, lane (g, c)
// supplies row c of a 16-row subtile as the first operand and column c mod 4
// of a 4-column operand as the second, at the k value of its lane group g.
//
// fp64, v_mfma_f64_4x4x4f64 (four 4x4x4 products): with c = 4 i + x, block i
// takes lane (g, c)'s first operand as row x at k slot g and its second as k
// slot g of column x, and lane 16 x + 4 i + j receives block i's D[x][j]:
// lane (g, c) receives the full product at row 4 (c / 4) + g, column c mod 4.
//
// fp32, v_mfma_f32_4x4x1f32 (sixteen 4x4x1 products, K = 1): block 4 g + c / 4
// is the four lanes 4 (c / 4) + x of group g; it takes lane x's first operand
// as row x and lane j's second as column j, and lane j of the block receives
// D[x][j] in element x.  So lane (g, c) receives rows 4 (c / 4) + x (element
// x), column c mod 4, summed over the k values of its own lane group only:
// the four groups' accumulators add up to the product.
template <typename T> struct Narrow;
template <> struct Narrow<double> {
  using acc_t = double;
  static __device__ __forceinline__ double mac(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Narrow<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ v4f mac(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
  }
};

// Four consecutive elements of a column held by one lane.
template <typename T> struct Quad { T e[4]; };

// Global-memory accesses.  Every buffer the helpers below read or write is
// in global memory, but a pointer that a kernel reads out of a descriptor
// (rather than receiving as an argument) is otherwise accessed with flat
// instructions, whose waits also cover LDS and scalar loads.  T must be a
// scalar or a clang vector type.
typedef double v2d __attribute__((ext_vector_type(2)));
template <typename T> using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ T gload(const T* p) { return *(const global_t<T>*)p; }
template <typename T>
__device__ __forceinline__ void gstore(T* p, const T v) { *(global_t<T>*)p = v; }

// 16-byte-aligned vector load of 4 consecutive elements.
__device__ __forceinline__ void vload4(Quad<float>& q, const float* p) {
  const v4f t = gload(reinterpret_cast<const v4f*>(p));
  q.e[0] = t[0]; q.e[1] = t[1]; q.e[2] = t[2]; q.e[3] = t[3];
}
__device__ __forceinline__ void vload4(Quad<double>& q, const double* p) {
  const v2d t0 = gload(reinterpret_cast<const v2d*>(p));
  const v2d t1 = gload(reinterpret_cast<const v2d*>(p + 2));
  q.e[0] = t0[0]; q.e[1] = t0[1]; q.e[2] = t1[0]; q.e[3] = t1[1];
}
__device__ __forceinline__ void vstore4(float* p, const Quad<float>& q) {
  gstore(reinterpret_cast<v4f*>(p), v4f{q.e[0], q.e[1], q.e[2], q.e[3]});
}
__device__ __forceinline__ void vstore4(double* p, const Quad<double>& q) {
  gstore(reinterpret_cast<v2d*>(p), v2d{q.e[0], q.e[1]});
  gstore(reinterpret_cast<v2d*>(p + 2), v2d{q.e[2], q.e[3]});
}

template <typename T>
__device__ __forceinline__ void zero4(Quad<T>& q) {
  q.e[0] = T(0); q.e[1] = T(0); q.e[2] = T(0); q.e[3] = T(0);
}

// Elements base[i .. i+3] of a column whose valid length is n; elements at
// or past n, and every element when !ok, read as zero.  VEC selects the
// vector load when the whole quad is in range (the caller guarantees the
// alignment that requires).
template <typename T, bool VEC>
__device__ __forceinline__ void load4(Quad<T>& q, const T* base, int64_t i, int64_t n, bool ok) {
  if (VEC && i + 3 < n) {
    if (ok) vload4(q, base + i); else zero4(q);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) q.e[e] = (ok && i + e < n) ? gload(base + i + e) : T(0);
  }
}

// Full chunk: 4 consecutive in-range elements from a valid pointer, with no
// branches (vector load when VEC, the caller guaranteeing 16-byte alignment).
template <typename T, bool VEC>
__device__ __forceinline__ void load_full(Quad<T>& q, const T* p) {
  if constexpr (VEC) {
    vload4(q, p);
  } else {
    q.e[0] = gload(p); q.e[1] = gload(p + 1); q.e[2] = gload(p + 2); q.e[3] = gload(p + 3);
  }
}

// Ragged chunk: col[i .. i+3] with elements at or past n reading as zero.
// Branch-free: every lane loads from a clamped in-range index and the
// out-of-range elements are then replaced by zero.
template <typename T>
__device__ __forceinline__ void load_tail(Quad<T>& q, const T* col, int64_t i, int64_t n) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const T x = gload(col + min(i + e, n - 1));
    q.e[e] = (i + e < n) ? x : T(0);
  }
}

// Hand-off of a stream-K partial result between blocks, which may run on
// different XCDs: each XCD has its own L2, and plain accesses are not
// coherent between them.  The partial moves through relaxed device-scope
// atomic accesses, which the hardware keeps coherent across the XCDs by
// themselves.  The writer stores it with xput4, waits with xput_complete
// until those stores are done, and only then (after a block barrier) raises
// the flag; the reader reads it with xget4 after it has seen the flag.  This
// avoids the L2-wide write-back and invalidation that device-scope release
// and acquire fences perform, which cost far more than the partial itself.
__device__ __forceinline__ void xput64(void* p, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t xget64(const void* p) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t pack2(float x, float y) {
  return (uint64_t)__builtin_bit_cast(uint32_t, x) | ((uint64_t)__builtin_bit_cast(uint32_t, y) << 32);
}
__device__ __forceinline__ void unpack2(uint64_t b, float& x, float& y) {
  x = __builtin_bit_cast(float, (uint32_t)b);
  y = __builtin_bit_cast(float, (uint32_t)(b >> 32));
}
__device__ __forceinline__ void xput4(float* p, const Quad<float>& q) {
  xput64(p, pack2(q.e[0], q.e[1]));
  xput64(p + 2, pack2(q.e[2], q.e[3]));
}
__device__ __forceinline__ void xput4(double* p, const Quad<double>& q) {
#pragma unroll
  for (int e = 0; e < 4; ++e) xput64(p + e, __builtin_bit_cast(uint64_t, q.e[e]));
}
__device__ __forceinline__ void xget4(Quad<float>& q, const float* p) {
  unpack2(xget64(p), q.e[0], q.e[1]);
  unpack2(xget64(p + 2), q.e[2], q.e[3]);
}
__device__ __forceinline__ void xget4(Quad<double>& q, const double* p) {
#pragma unroll
  for (int e = 0; e < 4; ++e) q.e[e] = __builtin_bit_cast(double, xget64(p + e));
}
__device__ __forceinline__ void xput4(float* p, v4f v) {
  xput64(p, pack2(v[0], v[1]));
  xput64(p + 2, pack2(v[2], v[3]));
}
__device__ __forceinline__ v4f xget4v(const float* p) {
  v4f v;
  float x, y;
  unpack2(xget64(p), x, y);
  v[0] = x; v[1] = y;
  unpack2(xget64(p + 2), x, y);
  v[2] = x; v[3] = y;
  return v;
}
// every store this thread issued is complete (s_waitcnt with all counts 0)
__device__ __forceinline__ void xput_complete() { __builtin_amdgcn_s_waitcnt(0); }

// The same wave-uniform value, hidden from loop-invariant code motion.  An
// address used only where a slab ends (a stream-K partial, say) is otherwise
// computed once before the slab loop and kept alive, or spilled, across the
// whole chunk loop; built from this value it is computed where it is used.
__device__ __forceinline__ int64_t opaque_uniform(int64_t x) {
  asm volatile("" : "+s"(x));
  return x;
}

// The epoch of a split-product launch, in [1, 2^30): every block reads the
// stored word (+1) when it starts, and the last block to finish advances it
// (handoff_done), so consecutive launches, graph replays included, never
// share an epoch.  The next launch on the stream starts only after the last
// block has stored the new value.
// One thread reads the word and the block shares it through LDS, so every
// wave holds the same value before any block can have arrived at its end.
__device__ __forceinline__ int handoff_epoch(const int* word) {
  __shared__ int e;
  if (threadIdx.x == 0) e = 1 + __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(e);
}
// Called by every block at its very end.  The block's last arrival (the
// launch's last block) resets the counter and stores the next epoch.
// word[0] is the epoch word, word[1] the arrival counter.
__device__ __forceinline__ void handoff_done(int* word, int64_t nblocks, int epoch) {
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (__hip_atomic_fetch_add(word + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)nblocks - 1) {
      __hip_atomic_store(word + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(word, epoch >= 0x3fffffff ? 0 : epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Spin until a hand-off flag holds `want` (relaxed device-scope loads),
// giving up after `limit` polls that did not see it: then *err (a word of
// pinned host memory that the host checks at its next call) is set and the
// caller goes on with whatever the partial holds, so that every wave still
// exits.  Flags carry the launch's epoch rather than 1/0, so a value left by
// an earlier launch (for instance after a give-up) never satisfies a later
// wait and no flag needs to be lowered.  Returns whether the flag was seen.
__device__ __forceinline__ bool xwait_flag(const int* flag, int want, int* err, int limit) {
  int spins = 0;
  bool ok = true;
  while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != want) {
    if (++spins > limit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  // keeps the compiler from moving the partial's reads above the wait
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return ok;
}

// x^k for a small non-negative integer k (k is uniform across the wave).
__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int t = 0; t < k; ++t) r *= x;
  return r;
}

}  // namespace symtd
