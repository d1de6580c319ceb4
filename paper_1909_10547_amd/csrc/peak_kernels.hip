// Measured ceilings of the device, for the roofline figures: a loop of
// independent MFMAs on register operands (no memory traffic), the same
// instruction the BF16 convolution kernels use.
#include "runtime.h"

namespace fk {

typedef __bf16 bf16x8p __attribute__((ext_vector_type(8)));
typedef float f32x4p __attribute__((ext_vector_type(4)));

// Each wave runs ``iters`` rounds of kChains independent accumulation chains
// of v_mfma_f32_16x16x32_bf16 (16384 flops each), so that the matrix unit
// never waits on a result; one lane's sum is stored so nothing is dead.
constexpr int kChains = 8;

__global__ void __launch_bounds__(256) mfma_peak_kernel(int iters, float *out) {
  const int lane = threadIdx.x & 63;
  bf16x8p a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f / (1 + ((lane + e) & 7)));
    b[e] = (__bf16)(1.0f / (2 + ((lane * 3 + e) & 7)));
  }
  f32x4p c[kChains];
  for (int k = 0; k < kChains; ++k) c[k] = f32x4p{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  if (lane == 0) out[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = s;
}

}  // namespace fk

using namespace fk;

extern "C" fk_status fk_measure_mfma_peak(fk_ctx *ctx, int32_t iters, double *tflops) {
  if (!ctx) return FK_E_ARG;
  if (!tflops || iters < 1) return set_err(ctx, FK_E_ARG, "fk_measure_mfma_peak: need iters >= 1 and tflops");
  *tflops = 0.0;
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, FK_E_HIP, "hipSetDevice failed");
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
    return set_err(ctx, FK_E_HIP, "fk_measure_mfma_peak: device attribute query failed");
  const int grid = 8 * ncu;  // 32 waves per compute unit, 8 per SIMD
  std::vector<std::pair<void *, size_t>> tmp;
  void *d = nullptr;
  fk_status st = dev_alloc(ctx, (size_t)grid * 4 * sizeof(float), &d, &tmp);
  if (st) return st;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float best = 1e30f;
  for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // the first run warms up
    e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(mfma_peak_kernel, dim3(grid), dim3(256), 0, nullptr, iters, (float *)d);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && rep > 0) best = std::min(best, ms);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  dev_free_all(ctx, tmp);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_measure_mfma_peak: %s", hipGetErrorString(e));
  const double flops = (double)grid * 4 * iters * kChains * 16384.0;
  *tflops = flops / (best * 1e-3) / 1e12;
  return FK_OK;
}
