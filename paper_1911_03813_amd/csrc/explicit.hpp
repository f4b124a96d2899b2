// The explicit route of Algorithm 1 (fg_explicit): a dense symmetric data
// tensor X (n^d entries; entry (i_1, .., i_d) at i_1 + n i_2 + .. +
// n^{d-1} i_d) and its TTSVs X a_j^{d-1} (eq. (ExpXbdd)).
//
// The first mode is contracted by the first product of the implicit route:
// with X's mode-1 unfolding taken as n x n^{d-1} "observations" of unit
// weight and order 2, that product's epilogue stores Z = X_(1)' A, the
// n^{d-1} x r partial contractions, in its packed layout (kernels.hpp).  The
// remaining d - 2 modes are contracted per column by k_ttsv_tail, which also
// forms the terms a_ij y_ij of w_j = a_j' y_j.  The closing kernel of the
// implicit route then assembles f, g_lambda and G_A from Y and w.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

// X = sum_l nu_l v_l^{(x)d}, summed in fp64 (register tiles of 64 x 64
// entries of the n x n^{d-1} unfolding, 16 observations per LDS step)
template <typename T>
struct MomentArgs {
  const T* V; int64_t ldv; const double* nu; int n; int64_t p; int d;
  int64_t cols;            // n^{d-1}
  T* X;                    // the tensor in the storage type, or
  double* X64;             // (when not null) in fp64
};
template <typename T>
void launch_moment(hipStream_t st, const MomentArgs<T>& a);

// y_ij = sum over m < n^{d-2} of Z(m + n^{d-2} i, j) prod_k a_{digit_k(m), j}
// (digits of m in base n), one block per (i, j); Y in the closing kernel's
// layout (column j at j * npad) and w terms a_ij y_ij in fp64 rows of rp
template <typename T>
struct TtsvTailArgs {
  const T* Wp; int nt_tot;  // packed Z
  const T* A; int64_t lda; int n; int r; int d;
  int64_t m2;               // n^{d-2}
  T* Y; int64_t npad;
  double* wterm; int rp;
};
template <typename T>
void launch_ttsv_tail(hipStream_t st, const TtsvTailArgs<T>& a);

void launch_fill(hipStream_t st, double* x, int64_t count, double v);

}  // namespace symtd
