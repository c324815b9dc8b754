// Attainable FP64 matrix-core rate of the current device, the yardstick
// beside the published peak for the MFMA-bound kernels (the Schur
// Cholesky and assembly).  Every wave runs eight independent chains of
// v_mfma_f64_16x16x4 on register operands (no memory traffic inside the
// timed loop), four waves per SIMD so that the matrix cores never wait on
// a dependency; the rate is the best of three timed launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace psdp {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kChains = 8;
constexpr int kIters = 2048;

__global__ void __launch_bounds__(256) k_mfma_rate(double* out) {
  v4d acc[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * threadIdx.x, b = 1.0 + 1e-6 * blockIdx.x;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;   // keeps the chains live
}

}  // namespace
}  // namespace psdp

extern "C" int psdp_fp64_mfma_rate(double* tflops, void* stream) {
  using namespace psdp;
  if (!tflops) return fail(PSDP_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  PSDP_HIP(hipGetDevice(&dev));
  PSDP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 4 * cus;   // 4 workgroups of 4 waves per CU: 4 waves per SIMD
  double* out = nullptr;
  PSDP_HIP(hipMalloc(&out, (size_t)blocks * 256 * sizeof(double)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 0.0;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_mfma_rate, dim3(blocks), dim3(256), 0, st, out);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    // the first launch warms the clocks and is not counted
    const double flops = (double)blocks * 4 * kIters * kChains * 2.0 * 16 * 16 * 4;
    if (e == hipSuccess && rep > 0 && ms > 0.f) best = std::max(best, flops / (ms * 1e-3) / 1e12);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  if (e != hipSuccess) return fail(PSDP_EDEVICE, std::string("FP64 MFMA rate: ") + hipGetErrorString(e));
  *tflops = best;
  return PSDP_OK;
}
