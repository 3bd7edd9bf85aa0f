// Issue-rate probes: what plain FP32 vector FMAs and FP16 matrix-core instructions reach on the device, as the
// measured ceilings beside the published peaks.  Pure arithmetic on registers; each thread writes one value so
// that nothing is optimised away.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace moff {

namespace {
typedef _Float16 probe_half8 __attribute__((ext_vector_type(8)));
typedef float probe_float4 __attribute__((ext_vector_type(4)));
}  // namespace

// 8 independent FMA chains per thread, iters x 8 FMAs (2 flops each), all operands in registers (the 4-byte
// accumulating encoding, as in the transforms).
__global__ __launch_bounds__(256) void k_probe_fma(int iters, float *out) {
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k);
  const float b = 0.5f + 1e-3f * (float)(threadIdx.x & 7), c = 1e-6f * (float)(1 + (threadIdx.x & 3));
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fmaf(b, c, a[k]);   // accumulating form: v_fmac_f32
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 independent accumulators per wavefront, iters x 4 v_mfma_f32_16x16x32_f16 (16 x 16 x 32 x 2 flops each).
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float *out) {
  probe_half8 x, y;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = (_Float16)(0.001f * (float)((threadIdx.x + k) & 7));
    y[k] = (_Float16)(0.002f * (float)((threadIdx.x * 3 + k) & 7));
  }
  probe_float4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = probe_float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc[k], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_probe(int kind, int blocks, int iters, float *out, hipStream_t st) {
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, iters, out);
  else
    hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, st, iters, out);
  return hipGetLastError();
}

}  // namespace moff
