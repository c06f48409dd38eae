// Grouped FP64 GEMM of the derivative and filter operators (ghmi_gemm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

// One GEMM problem of a grouped launch: C[M x N] = A[M x K] * B[K x N], row-major,
// with A = Abase + a_off and C = Cbase + c_off (the bases are launch arguments,
// so one tile list serves any state / work-space pair).
struct GemmGroup {
  long long a_off;
  long long c_off;
  const double* B;
  int M, N, K;
  int lda, ldb, ldc;
};

// One output tile of a grouped GEMM launch.
struct GemmTile {
  int g;              // group index
  int m0, n0;         // tile origin
  int pad;
};

namespace ghk {

// Grouped GEMM (ghmi_gemm.hip).  shape: index of a kernel variant (tile
// BM x BN, wave layout, LDS layout of A, k-slice depth; 13 .. 17 load the
// slices directly into LDS and need shape_fits); order: 0 column blocks, 1 row
// blocks or 2 blocks of 8 x 8 tiles per XCD.  role: 0 angular derivative, 1 filter, 2 transposed
// derivative (C += A B), 3 transposed filter, 4 Fourier analysis, 5 Fourier
// synthesis, 6 PhysToSpec and 7 SpecToPhys of the tensor-coupled filter
// (separate kernel symbols).
enum { NUM_TILE_SHAPES = 18, NUM_TILE_ORDERS = 3 };
void tile_dims(int shape, int* bm, int* bn);
// whether a variant can run these groups (the direct-to-LDS ones need even K,
// N, lda, ldb and a_off, and a 16-byte aligned B)
bool shape_fits(int shape, const std::vector<GemmGroup>& groups);
std::vector<GemmTile> build_tiles(const std::vector<GemmGroup>& groups, int shape, int order);
hipError_t gemm(int shape, const GemmTile* tiles, int n_tiles, const GemmGroup* groups,
                const double* Abase, double* Cbase, hipStream_t st, int role);

}  // namespace ghk
