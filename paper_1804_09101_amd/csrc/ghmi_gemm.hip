// Grouped FP64 GEMM of the spectral derivative and filter operators on the
// matrix cores of gfx950 (MI355X): the kernel, the variants the autotuner
// chooses from, and the tile lists of one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "ghmi_gemm.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Grouped FP64 GEMM on the matrix cores: C = A * B for every group of a tile
// list.  One workgroup of WGM x WGN waves computes a BM x BN tile; each wave
// owns a (BM/WGM) x (BN/WGN) sub-tile made of 16x16 blocks of
// v_mfma_f64_16x16x4_f64.  A and B k-slices (BK = 16 or 32: fewer barriers
// per K against twice the LDS) are staged through LDS, double buffered.  B is
// stored k-major ([BK][BN]); A either k-major
// ([BK][BM], AROW = false) or row-major with a one-double pad per row
// ([BM][BK+1], AROW = true: the global-to-LDS store is then a plain row copy
// and the padded rows keep the fragment reads free of bank conflicts).
//
// Fragment layout of v_mfma_f64_16x16x4_f64 (64 lanes):
//   A (16x4): lane l holds A[l % 16][l / 16]
//   B (4x16): lane l holds B[l / 16][l % 16]
//   C (16x16): lane l holds C[l/16 + 4*v][l % 16], v = 0..3 (checked on gfx950)
// ---------------------------------------------------------------------------
// ROLE separates the kernel symbols of the different uses (0: angular
// derivative, 1: filter, 2: transposed derivative of the adjoint, 3: transposed
// filter, 4: Fourier analysis and 5: synthesis of the transform path, 6:
// PhysToSpec and 7: SpecToPhys of the tensor-coupled filter) so that profiles
// attribute time to each.  ROLE 2 adds into C
// (C += A B); the others overwrite C.
template <int BM, int BN, int WGM, int WGN, bool AROW, int BK, int ROLE>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gemm(const GemmTile* __restrict__ tiles,
                                                         const GemmGroup* __restrict__ groups,
                                                         const double* __restrict__ Abase,
                                                         double* __restrict__ Cbase) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(TM * 16 == WM && TN * 16 == WN, "wave sub-tile must be whole 16x16 blocks");
  constexpr int AGRP = BM * BK / 4;     // 4-double groups of one A slice
  constexpr int BGRP = BK * BN / 4;     // 4-double groups of one B slice
  constexpr int APASS = (AGRP + NT - 1) / NT;
  constexpr int BPASS = (BGRP + NT - 1) / NT;
  constexpr int ALD = BK + 1;           // padded row length of row-major A
  __shared__ double As[2][AROW ? BM * ALD : BK * BM];
  __shared__ double Bs[2][BK][BN];

  const GemmTile t = tiles[blockIdx.x];
  const GemmGroup G = groups[t.g];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int M = G.M, N = G.N, K = G.K;
  const double* __restrict__ Ag = Abase + G.a_off;
  double* __restrict__ Cg = Cbase + G.c_off;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[APASS][4], rb[BPASS][4];

  auto load_global = [&](int k0) {
#pragma unroll
    for (int p = 0; p < APASS; ++p) {
      int idx = p * NT + tid;
      if (AGRP % NT != 0 && idx >= AGRP) break;
      int row = t.m0 + idx / (BK / 4), kq = k0 + (idx % (BK / 4)) * 4;
      const double* src = Ag + (long long)row * G.lda + kq;
      if (row < M && kq + 3 < K) {
        double2 v0 = *reinterpret_cast<const double2*>(src);
        double2 v1 = *reinterpret_cast<const double2*>(src + 2);
        ra[p][0] = v0.x; ra[p][1] = v0.y; ra[p][2] = v1.x; ra[p][3] = v1.y;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[p][e] = (row < M && kq + e < K) ? src[e] : 0.0;
      }
    }
#pragma unroll
    for (int p = 0; p < BPASS; ++p) {
      int idx = p * NT + tid;
      if (BGRP % NT != 0 && idx >= BGRP) break;
      int krow = k0 + idx / (BN / 4), col = t.n0 + (idx % (BN / 4)) * 4;
      const double* src = G.B + (long long)krow * G.ldb + col;
      if (krow < K && col + 3 < N) {
        double2 v0 = *reinterpret_cast<const double2*>(src);
        double2 v1 = *reinterpret_cast<const double2*>(src + 2);
        rb[p][0] = v0.x; rb[p][1] = v0.y; rb[p][2] = v1.x; rb[p][3] = v1.y;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[p][e] = (krow < K && col + e < N) ? src[e] : 0.0;
      }
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int p = 0; p < APASS; ++p) {
      int idx = p * NT + tid;
      if (AGRP % NT != 0 && idx >= AGRP) break;
      int row = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (AROW) As[buf][row * ALD + kq + e] = ra[p][e];
        else As[buf][(kq + e) * BM + row] = ra[p][e];
      }
    }
#pragma unroll
    for (int p = 0; p < BPASS; ++p) {
      int idx = p * NT + tid;
      if (BGRP % NT != 0 && idx >= BGRP) break;
      int krow = idx / (BN / 4), col = (idx % (BN / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[buf][krow][col + e] = rb[p][e];
    }
  };

  const int nk = (K + BK - 1) / BK;
  load_global(0);
  store_lds(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_global((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + lane / 16;
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm + i * 16 + (lane & 15);
        af[i] = AROW ? As[buf][m * ALD + kr] : As[buf][kr * BM + m];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = Bs[buf][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_lds(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = t.n0 + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = t.m0 + wm + i * 16 + (lane / 16) + 4 * v;
        if (row < M && col < N) {
          if (ROLE == 2) Cg[(long long)row * G.ldc + col] += acc[i][j][v];
          else Cg[(long long)row * G.ldc + col] = acc[i][j][v];
        }
      }
    }
}

// Direct-to-LDS variant: the k-slices go from global memory straight into
// LDS with the gfx950 global_load_lds_dwordx4 (16 bytes per lane, written to
// LDS in lane order at a wave-uniform base), so no registers stage them and no
// LDS stores are issued.  BK = 16.  The LDS layouts are chosen so that the
// fragment reads of a half-wave (32 lanes) touch every LDS bank once:
//   A slice: 16-byte k-pairs; one load instruction (a, b) brings rows
//     16a .. 16a+15 and k-pairs 4b .. 4b+3, lane l = 16 (kp % 4) + m % 16.
//   B slice: [16][BN] with the k-pairs of odd rows XOR-ed by 8 (128 bytes), so
//     two consecutive k rows fall in opposite halves of the banks.
// Rows past M and columns past N read clamped (finite) data that only reaches
// outputs that are never stored; a ragged last k-slice is clamped the same
// way and its A entries past K are zeroed in LDS before use.  Needs even K,
// lda, ldb, a_off and N, and 16-byte aligned A and B (checked on the host).
typedef __attribute__((address_space(1))) const void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// Launch bounds (the second argument of HIP's __launch_bounds__ is the least
// number of waves per SIMD): four waves per SIMD (at most 128 registers)
// unless the accumulators alone take 128 registers, then two.  The MFMA pipe
// stays fed only at four waves per SIMD: a variant of 130 VGPRs (three waves)
// measured 8% slower.
template <int BM, int BN, int WGM, int WGN>
constexpr int lds_min_waves() {
  return (BM / WGM / 16) * (BN / WGN / 16) * 8 < 128 ? 4 : 2;
}

template <int BM, int BN, int WGM, int WGN, int ROLE>
__global__ __launch_bounds__(64 * WGM * WGN, (lds_min_waves<BM, BN, WGM, WGN>())) void k_gemm_lds(const GemmTile* __restrict__ tiles,
                                                             const GemmGroup* __restrict__ groups,
                                                             const double* __restrict__ Abase,
                                                             double* __restrict__ Cbase) {
  constexpr int NW = WGM * WGN;
  constexpr int BK = 16;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(TM * 16 == WM && TN * 16 == WN, "wave sub-tile must be whole 16x16 blocks");
  static_assert(BM % 16 == 0 && BN % 64 == 0 && BN <= 128, "A in 16-row groups, B rows of 64 or 128 doubles");
  constexpr int AINS = (BM / 16) * 2;   // A load instructions per slice (1 KB each)
  constexpr int BINS = BK * BN / 128;   // B load instructions per slice
  constexpr int ASZ = BM * BK, BSZ = BK * BN;
  __shared__ double lds[2][ASZ + BSZ];

  const GemmTile t = tiles[blockIdx.x];
  const GemmGroup G = groups[t.g];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int M = G.M, N = G.N, K = G.K;
  const double* __restrict__ Ag = Abase + G.a_off;
  double* __restrict__ Cg = Cbase + G.c_off;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // Load instructions of one slice, spread evenly over the waves (wave index
  // made uniform so that the LDS base goes to M0 without a loop over lanes).
  static_assert(AINS % NW == 0 && BINS % NW == 0, "load instructions must split evenly over the waves");
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int a_m = lane & 15, a_kp = lane >> 4;
  auto issue = [&](int k0, int buf) {
#pragma unroll
    for (int p = 0; p < AINS / NW; ++p) {
      const int ins = wv + NW * p, a = ins >> 1, b = ins & 1;
      const int row = min(t.m0 + 16 * a + a_m, M - 1);
      const int k = min(k0 + 2 * (4 * b + a_kp), K - 2);
      __builtin_amdgcn_global_load_lds((gvoid_t*)(Ag + (long long)row * G.lda + k), (lvoid_t*)&lds[buf][ins * 128],
                                       16, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < BINS / NW; ++p) {
      const int r = wv + NW * p;
      const int e = r * 128 + 2 * lane;          // slice element of this lane's LDS pair
      const int krow = e / BN, pos = (e % BN) >> 1;
      const int pair = pos ^ ((krow & 1) << 3);  // the global pair that belongs there
      const int k = min(k0 + krow, K - 1);
      const int col = min(t.n0 + 2 * pair, N - 2);
      __builtin_amdgcn_global_load_lds((gvoid_t*)(G.B + (long long)k * G.ldb + col),
                                       (lvoid_t*)&lds[buf][ASZ + r * 128], 16, 0, 0);
    }
  };

  const int nk = (K + BK - 1) / BK;
  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of slice kt have landed in LDS
    __syncthreads();                 // everyone's have, and slice kt-1 is no longer read
    if (kt + 1 < nk) {
      issue((kt + 1) * BK, buf ^ 1);
    } else if (K - kt * BK < BK) {
      // ragged last slice: zero A's k entries past K (k-pair layout)
      const int kr = K - kt * BK;
      for (int idx = tid; idx < BM * BK; idx += 64 * NW) {
        const int ins = idx >> 7, w = idx & 127;
        const int k = 2 * (4 * (ins & 1) + (w >> 5)) + (w & 1);
        if (k >= kr) lds[buf][idx] = 0.0;
      }
      __syncthreads();
    }
    const double* As = lds[buf];
    const double* Bs = lds[buf] + ASZ;
    // operands of step kk + 2 are read while the MFMAs of step kk run, one
    // LDS read placed between consecutive MFMAs
    auto read = [&](int kk, double (&af)[TM], double (&bf)[TN]) {
      const int kr = kk * 4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int a = (wm >> 4) + i;
        af[i] = As[((a * 2 + (kk >> 1)) * 64 + (2 * (kk & 1) + (lane >> 5)) * 16 + (lane & 15)) * 2 + ((lane >> 4) & 1)];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = wn + j * 16 + (lane & 15);
        bf[j] = Bs[kr * BN + (((c >> 1) ^ ((kr & 1) << 3)) << 1) + (c & 1)];
      }
    };
    constexpr int PD = 2;
    double af[PD + 1][TM], bf[PD + 1][TN];
#pragma unroll
    for (int d = 0; d < PD; ++d) read(d, af[d], bf[d]);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      if (kk + PD < BK / 4) read(kk + PD, af[(kk + PD) % (PD + 1)], bf[(kk + PD) % (PD + 1)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk % (PD + 1)][i], bf[kk % (PD + 1)][j], acc[i][j], 0,
                                                           0, 0);
#pragma unroll
      for (int g = 0; g < TM + TN; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = t.n0 + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = t.m0 + wm + i * 16 + (lane / 16) + 4 * v;
        if (row < M && col < N) {
          if (ROLE == 2) Cg[(long long)row * G.ldc + col] += acc[i][j][v];
          else Cg[(long long)row * G.ldc + col] = acc[i][j][v];
        }
      }
    }
}

}  // namespace

namespace ghk {

// Kernel variants the autotuner chooses from: tile BM x BN, WGM x WGN waves,
// A layout in LDS (row-major padded or k-major).
// Shapes 13 .. 17 load their k-slices directly into LDS (k_gemm_lds); each
// has a register-staged twin of the same tile (7, 6, 9, the 256 x 128
// instantiation below, 3) that a launch falls back to when A's base address is
// not 16-byte aligned.  Both give bitwise the same result.
struct TileShape {
  int bm, bn, wgm, wgn;
  bool arow;
  int bk;
  bool direct;
};
static const TileShape kTiles[] = {
    {64, 64, 2, 2, false, 16, false},  {64, 128, 2, 2, false, 16, false}, {128, 64, 2, 2, false, 16, false},
    {128, 128, 2, 2, false, 16, false}, {96, 64, 2, 2, false, 16, false},  {96, 64, 2, 2, true, 16, false},
    {128, 64, 4, 2, true, 16, false},  {128, 128, 4, 2, true, 16, false}, {64, 128, 2, 4, true, 16, false},
    {192, 64, 4, 2, true, 16, false},  {128, 64, 4, 2, true, 32, false},  {192, 64, 4, 2, true, 32, false},
    {128, 128, 4, 2, true, 32, false}, {128, 128, 4, 2, true, 16, true},  {128, 64, 4, 2, true, 16, true},
    {192, 64, 4, 2, true, 16, true},   {256, 128, 4, 2, true, 16, true},  {128, 128, 2, 2, true, 16, true}};
static_assert(sizeof(kTiles) / sizeof(kTiles[0]) == NUM_TILE_SHAPES, "one table row per tile shape");

void tile_dims(int shape, int* bm, int* bn) {
  *bm = kTiles[shape].bm;
  *bn = kTiles[shape].bn;
}

bool shape_fits(int shape, const std::vector<GemmGroup>& groups) {
  if (shape < 0 || shape >= NUM_TILE_SHAPES) return false;
  if (!kTiles[shape].direct) return true;
  for (const auto& g : groups)
    if ((g.K & 1) || (g.N & 1) || (g.lda & 1) || (g.ldb & 1) || (g.a_off & 1) ||
        (reinterpret_cast<uintptr_t>(g.B) & 15))
      return false;
  return true;
}

// The instantiated variants: (index, BM, BN, WGM, WGN, A row-major, BK) for
// the register-staged kernel (100: the 256 x 128 twin of shape 16, not a
// tuner choice), (index, BM, BN, WGM, WGN) for the direct-to-LDS one.
#define GH_GEMM_STAGED_LIST(X)        \
  X(0, 64, 64, 2, 2, false, 16)       \
  X(1, 64, 128, 2, 2, false, 16)      \
  X(2, 128, 64, 2, 2, false, 16)      \
  X(3, 128, 128, 2, 2, false, 16)     \
  X(4, 96, 64, 2, 2, false, 16)       \
  X(5, 96, 64, 2, 2, true, 16)        \
  X(6, 128, 64, 4, 2, true, 16)       \
  X(7, 128, 128, 4, 2, true, 16)      \
  X(8, 64, 128, 2, 4, true, 16)       \
  X(9, 192, 64, 4, 2, true, 16)       \
  X(10, 128, 64, 4, 2, true, 32)      \
  X(11, 192, 64, 4, 2, true, 32)      \
  X(12, 128, 128, 4, 2, true, 32)     \
  X(100, 256, 128, 4, 2, true, 16)
#define GH_GEMM_DIRECT_LIST(X) \
  X(13, 128, 128, 4, 2)        \
  X(14, 128, 64, 4, 2)         \
  X(15, 192, 64, 4, 2)         \
  X(16, 256, 128, 4, 2)        \
  X(17, 128, 128, 2, 2)

template <int ROLE>
static hipError_t gemm_role(int shape, const GemmTile* tiles, int n_tiles, const GemmGroup* groups,
                            const double* Abase, double* Cbase, hipStream_t st) {
  dim3 grid(n_tiles);
#define GH_GEMM_CASE(i, BM_, BN_, WGM_, WGN_, AROW_, BK_)                                                  \
  case i:                                                                                                  \
    hipLaunchKernelGGL((k_gemm<BM_, BN_, WGM_, WGN_, AROW_, BK_, ROLE>), grid, dim3(64 * WGM_ * WGN_), 0, st, \
                       tiles, groups, Abase, Cbase);                                                       \
    break;
  switch (shape) {
    GH_GEMM_STAGED_LIST(GH_GEMM_CASE)
    default: return hipErrorInvalidValue;
  }
#undef GH_GEMM_CASE
  return hipGetLastError();
}

template <int ROLE>
static hipError_t gemm_direct(int shape, const GemmTile* tiles, int n_tiles, const GemmGroup* groups,
                              const double* Abase, double* Cbase, hipStream_t st) {
  if (reinterpret_cast<uintptr_t>(Abase) & 15) {
    static const int twin[5] = {7, 6, 9, 100, 3};
    return gemm_role<ROLE>(twin[shape - 13], tiles, n_tiles, groups, Abase, Cbase, st);
  }
  dim3 grid(n_tiles);
#define GH_GEMM_DIRECT(i, BM_, BN_, WGM_, WGN_)                                                            \
  case i:                                                                                                  \
    hipLaunchKernelGGL((k_gemm_lds<BM_, BN_, WGM_, WGN_, ROLE>), grid, dim3(64 * WGM_ * WGN_), 0, st, tiles, \
                       groups, Abase, Cbase);                                                              \
    break;
  switch (shape) {
    GH_GEMM_DIRECT_LIST(GH_GEMM_DIRECT)
    default: return hipErrorInvalidValue;
  }
#undef GH_GEMM_DIRECT
  return hipGetLastError();
}

hipError_t gemm(int shape, const GemmTile* tiles, int n_tiles, const GemmGroup* groups,
                const double* Abase, double* Cbase, hipStream_t st, int role) {
  if (n_tiles <= 0) return hipSuccess;
  if (shape >= 13 && shape < NUM_TILE_SHAPES) {
    switch (role) {
      case 0: return gemm_direct<0>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 1: return gemm_direct<1>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 2: return gemm_direct<2>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 3: return gemm_direct<3>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 4: return gemm_direct<4>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 5: return gemm_direct<5>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 6: return gemm_direct<6>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      case 7: return gemm_direct<7>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (role) {
    case 0: return gemm_role<0>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 1: return gemm_role<1>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 2: return gemm_role<2>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 3: return gemm_role<3>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 4: return gemm_role<4>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 5: return gemm_role<5>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 6: return gemm_role<6>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    case 7: return gemm_role<7>(shape, tiles, n_tiles, groups, Abase, Cbase, st);
    default: return hipErrorInvalidValue;
  }
}

// Tile list of one grouped GEMM launch.  Workgroups are dispatched
// round-robin over the 8 XCDs, so list position p runs on XCD p % 8; the list
// interleaves 8 per-XCD sequences.  order 0: each XCD takes whole n-column
// blocks (its slice of the operator stays in its L2 while the field rows
// stream past); order 1: each XCD takes whole row blocks (the field rows are
// fetched once, every XCD reads the operator); order 2: each XCD takes blocks
// of 8 x 8 tiles, about the tiles one XCD runs at a time, so its concurrent
// tiles share 8 row slices of A and 8 column slices of the operator instead of
// 2 and 32 (order 1) or 64 and 1 (order 0): fewer L2 misses per k-slice.
std::vector<GemmTile> build_tiles(const std::vector<GemmGroup>& groups, int shape, int order) {
  int bm, bn;
  tile_dims(shape, &bm, &bn);
  const int NX = 8, SB = 8;
  std::vector<std::vector<GemmTile>> per(NX);
  int block = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    int mt = (groups[g].M + bm - 1) / bm, nt = (groups[g].N + bn - 1) / bn;
    if (order == 0) {
      for (int j = 0; j < nt; ++j, ++block)
        for (int i = 0; i < mt; ++i) per[block % NX].push_back(GemmTile{int(g), i * bm, j * bn, 0});
    } else if (order == 1) {
      for (int i = 0; i < mt; ++i, ++block)
        for (int j = 0; j < nt; ++j) per[block % NX].push_back(GemmTile{int(g), i * bm, j * bn, 0});
    } else {
      for (int i0 = 0; i0 < mt; i0 += SB)
        for (int j0 = 0; j0 < nt; j0 += SB, ++block)
          for (int i = i0; i < std::min(mt, i0 + SB); ++i)
            for (int j = j0; j < std::min(nt, j0 + SB); ++j)
              per[block % NX].push_back(GemmTile{int(g), i * bm, j * bn, 0});
    }
  }
  std::vector<GemmTile> out;
  size_t longest = 0;
  for (auto& v : per) longest = std::max(longest, v.size());
  for (size_t q = 0; q < longest; ++q)
    for (int x = 0; x < NX; ++x)
      if (q < per[x].size()) out.push_back(per[x][q]);
  return out;
}

}  // namespace ghk
