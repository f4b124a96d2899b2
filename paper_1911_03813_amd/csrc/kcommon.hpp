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

// Four consecutive elements of a column held by one lane.
template <typename T> struct Quad { T e[4]; };

// 16-byte-aligned vector load of 4 consecutive elements.
__device__ __forceinline__ void vload4(Quad<float>& q, const float* p) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  q.e[0] = t.x; q.e[1] = t.y; q.e[2] = t.z; q.e[3] = t.w;
}
__device__ __forceinline__ void vload4(Quad<double>& q, const double* p) {
  const double2 t0 = *reinterpret_cast<const double2*>(p);
  const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
  q.e[0] = t0.x; q.e[1] = t0.y; q.e[2] = t1.x; q.e[3] = t1.y;
}
__device__ __forceinline__ void vstore4(float* p, const Quad<float>& q) {
  *reinterpret_cast<float4*>(p) = make_float4(q.e[0], q.e[1], q.e[2], q.e[3]);
}
__device__ __forceinline__ void vstore4(double* p, const Quad<double>& q) {
  *reinterpret_cast<double2*>(p) = make_double2(q.e[0], q.e[1]);
  *reinterpret_cast<double2*>(p + 2) = make_double2(q.e[2], q.e[3]);
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
    for (int e = 0; e < 4; ++e) q.e[e] = (ok && i + e < n) ? base[i + e] : T(0);
  }
}

// Full chunk: 4 consecutive in-range elements from a valid pointer, with no
// branches (vector load when VEC, the caller guaranteeing 16-byte alignment).
template <typename T, bool VEC>
__device__ __forceinline__ void load_full(Quad<T>& q, const T* p) {
  if constexpr (VEC) {
    vload4(q, p);
  } else {
    q.e[0] = p[0]; q.e[1] = p[1]; q.e[2] = p[2]; q.e[3] = p[3];
  }
}

// Ragged chunk: col[i .. i+3] with elements at or past n reading as zero.
// Branch-free: every lane loads from a clamped in-range index and the
// out-of-range elements are then replaced by zero.
template <typename T>
__device__ __forceinline__ void load_tail(Quad<T>& q, const T* col, int64_t i, int64_t n) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const T x = col[min(i + e, n - 1)];
    q.e[e] = (i + e < n) ? x : T(0);
  }
}

// x^k for a small non-negative integer k (k is uniform across the wave).
__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int t = 0; t < k; ++t) r *= x;
  return r;
}

}  // namespace symtd
