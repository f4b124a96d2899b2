// Argument blocks and host-side launchers of the symtd kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

// M subtiles (16 observations each) per wave in gemm1.
constexpr int G1_MT_F32 = 4;
constexpr int G1_MT_F64 = 2;
// Column subtiles handled by one launch of gemm1/gemm2 (16 columns each);
// wider ranks are processed in several column groups.
constexpr int NT_MAX_F32 = 7;
constexpr int NT_MAX_F64 = 4;

template <typename T>
struct G1Args {
  const T* V; int64_t ldv; const double* nu; int n; int p;
  const T* A; int64_t lda; int r;
  int col0;      // first column of this launch's column group (multiple of 16)
  int nt_tot;    // column subtiles over all groups: ceil(r / 16)
  int d;
  T* Wp;         // packed W, ceil(p/16) slabs
  double* wpart; // [gridDim.x][16 * nt_tot] fp64 column partials
};

template <typename T>
struct G2Args {
  const T* V; int64_t ldv; int n; int p;
  const T* Wp; int nt_tot; int col0;
  int nblk;           // ceil(p / 16)
  int blk_per_split;  // 16-observation slabs per split
  T* Ypart;           // [nsplit][16 * nt_tot][npad]
  int64_t npad;       // rows of a partial column, multiple of 256
};

template <typename T>
struct GramArgs {
  const T* A; int64_t lda; int n; int r; int d;
  double* B; double* C;  // r x r, column-major
};

template <typename T>
struct FinalGArgs {
  const T* Ypart; int64_t npad; int64_t rp; int nsplit;
  const T* A; int64_t lda; int n; int r; int d;
  const double* lambda; const double* C;
  T* G; int64_t ldg;
};

struct FinalSArgs {
  const double* wpart; int64_t nwpart; int64_t rp;
  const double* B; const double* C; const double* lambda;
  int r; double alpha;
  double* f; double* g_lambda;
};

template <typename S>
struct NormXArgs {
  const S* V; int64_t ldv; const double* nu; int n; int p; int d;
  int64_t ntile;      // ceil(p / 128)
  double* part;       // one fp64 partial per block
};

struct ReduceArgs {
  const double* part; int64_t count; double* out;
};

void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<float>& a);
void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<double>& a);
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<float>& a);
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<double>& a);
void launch_gram(dim3 grid, hipStream_t st, const GramArgs<float>& a);
void launch_gram(dim3 grid, hipStream_t st, const GramArgs<double>& a);
void launch_final_G(dim3 grid, hipStream_t st, const FinalGArgs<float>& a);
void launch_final_G(dim3 grid, hipStream_t st, const FinalGArgs<double>& a);
void launch_final_s(hipStream_t st, const FinalSArgs& a);

void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<float>& a);
void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<double>& a);
void launch_reduce(hipStream_t st, const ReduceArgs& a);

}  // namespace symtd
