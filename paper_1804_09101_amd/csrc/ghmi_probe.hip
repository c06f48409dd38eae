// Measured ceiling of the FP64 matrix cores: back-to-back
// v_mfma_f64_16x16x4_f64 on eight independent accumulators per wave, no
// memory traffic inside the loop.  The derivative GEMM's utilisation is
// reported against the published FP64 peak; this probe shows how much of that
// peak the chip sustains on the same instruction under full load.
#include <hip/hip_runtime.h>

#include "ghmi.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_mfma_f64_probe(double* __restrict__ out, int iters) {
  d4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * blockIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int gh_probe_mfma_f64(int device, int iters, double* tflops) {
  if (!tflops || iters <= 0) return GH_ERR_ARG;
  *tflops = 0.0;
  if (hipSetDevice(device) != hipSuccess) return GH_ERR_DEVICE;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0)
    return GH_ERR_DEVICE;
  const int blocks = ncu * 8, threads = 256;     // 32 waves per CU, 8 per SIMD
  double* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * blocks * threads) != hipSuccess) return GH_ERR_OOM;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = GH_OK;
  float ms = 0.0f;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = GH_ERR_DEVICE;
  } else {
    hipLaunchKernelGGL(k_mfma_f64_probe, dim3(blocks), dim3(threads), 0, st, out, iters);   // warm-up
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_mfma_f64_probe, dim3(blocks), dim3(threads), 0, st, out, iters);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f)
      rc = GH_ERR_DEVICE;
  }
  if (rc == GH_OK) {
    const double flop = double(blocks) * (threads / 64) * double(iters) * 8.0 * (2.0 * 16 * 16 * 4);
    *tflops = flop / (double(ms) * 1e-3) / 1e12;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(out);
  return rc;
}
