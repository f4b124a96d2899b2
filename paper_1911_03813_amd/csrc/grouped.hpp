// Grouped evaluation: Algorithm 2 for many independent instances (each with
// its own V, nu, n, p, d and R side-by-side models of r columns) in four
// launches per evaluation step, driven by work-item tables.
//
//   ggemm1   item (instance, 256-observation tile, column group): Z = V'A on
//            matrix cores straight from L2, epilogue W = D_nu Z^{d-1} (packed
//            as in the single-instance kernels) and per-tile fp64 column sums
//            of nu z^d;
//   gmodel   item (instance, model): B = A'A, C = B^{d-1}, u, w (fixed-order
//            sum of the tile sums), f, g_lambda and Y_M = A D_lambda C, fp64;
//   ggemm2   item (instance, 64-row block, observation split, column group):
//            partial Y = V W on matrix cores, one partial per split;
//   gfinal   item (instance, column): G_A = -2d (sum of partials - Y_M) lambda.
//
// The tiles, splits and summation orders of an instance depend only on its
// own shape, so its results are the same bits whatever else is in the group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

constexpr int GG1_TILE = 256;        // observations per ggemm1 item (4 waves x 4 blocks of 16)
constexpr int GG2_SPLIT_BLK = 16;    // default 16-observation blocks per ggemm2 split (256 observations)
constexpr int GG_NT_F32 = 4;         // column subtiles per item (fp32): few enough registers for three waves per SIMD
constexpr int GG_NT_F64 = 4;         // column subtiles per item (fp64)
constexpr int GG_NT_MAX = GG_NT_F32 > GG_NT_F64 ? GG_NT_F32 : GG_NT_F64;

template <typename T>
struct GInst {
  const T* V; int64_t ldv; const double* nu;
  int n, p, d, r, R, cols, nt;       // cols = R r, nt = ceil(cols / 16)
  const T* A; int64_t lda; const double* lam;
  double* f; double* glam; T* G; int64_t ldg;
  double alpha;
  // workspace
  T* Wp;                             // packed W, ceil(p/16) x nt x 256
  double* wpart; int ntile;          // [ntile][cols], ntile = ceil(p / GG1_TILE)
  T* Ypart; int nsplit; int64_t ldy; // [nsplit][nt*16][ldy], ldy = 64 ceil(n / 64)
  int split_blk;                     // 16-observation blocks per ggemm2 split (GG2_SPLIT_BLK or tuned)
  double* B; double* C;              // R blocks of r x r
  double* YM;                        // n x cols, leading dimension n
};

struct GItem { int inst, a, b, c; };

template <typename T>
void launch_ggemm1(bool vec, int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items);
template <typename T>
void launch_gmodel(int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items);
template <typename T>
void launch_ggemm2(bool vec, int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items);
template <typename T>
void launch_gfinal(int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items);
// Omega of every restart of every instance into its packed W: element
// (l, k r + j) of instance i = normal (l + p j) of (seeds[i], k, stream 2)
template <typename T>
void launch_gomega(int maxchunks, int ninst, hipStream_t st, const GInst<T>* insts, const uint64_t* seeds);

}  // namespace symtd
