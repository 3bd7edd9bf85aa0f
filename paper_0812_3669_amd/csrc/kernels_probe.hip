// Measurement probes: what plain FP32 vector FMAs and FP16 matrix-core instructions reach on the device (the
// measured ceilings beside the published peaks; pure arithmetic on registers, each thread writes one value so that
// nothing is optimised away), the two exchanges between transform stages, the XCD of each workgroup, and the
// exchange's HBM access patterns alone.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_radix.h"
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
  // two iterations per trip (8 instructions back to back), then the odd one
  for (int i = 0; i + 1 < iters; i += 2) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k & 3] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc[k & 3], 0, 0, 0);
  }
  if (iters & 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc[k], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Exchange probes: batches of 256-point transforms X[k] = (1/256) sum_n x[n] e^(2 pi i n k / 256) (the 1/256 keeps
// the repeated transforms finite), computed two ways that differ in how data moves between stages.  Each
// workgroup keeps its transforms in registers and transforms its own output iters times, then writes it back.
//
// kind 2, LDS exchange (the scheme of the library's FFT passes): 16 threads per transform, thread j holding
// x[j + 16 m]; a radix-16 DFT over m in registers, the twiddle w256^(j k1), the 16 x 16 transpose through padded
// LDS between two barriers, a radix-16 DFT over j; thread j ends with X[j + 16 k2] (natural order).
__global__ __launch_bounds__(256) void k_probe_fft_lds(int iters, float2 *data) {
  __shared__ float2 lds[16][16][17];   // [transform][k1][j], padded
  const int tr = (int)threadIdx.x >> 4, j = (int)threadIdx.x & 15;
  float2 *x = data + ((int64_t)blockIdx.x * 16 + tr) * 256;
  float2 v[16], tw[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = x[j + 16 * m];
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) {
    float sn, cs;
    sincospif((float)(j * k1) / 128.f, &sn, &cs);
    tw[k1] = make_float2(cs, sn);
  }
  for (int it = 0; it < iters; ++it) {
    dft16(v);   // v[k1] = Y[j][k1]
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) lds[tr][k1][j] = cmul(v[k1], tw[k1]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[tr][j][i];   // this thread now holds column k1 = j
    __syncthreads();
    dft16(v);   // v[k2] = X[j + 16 k2]
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cscale(v[k], 1.f / 256.f);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) x[j + 16 * k] = v[k];
}

// Partner value of lane l ^ H within a wavefront: DPP quad permutes for H = 1, 2, the data-share swizzle (xor
// mode, no LDS memory) for H = 4, 8, 16, a backward permute for H = 32.
template <int H>
__device__ __forceinline__ float xlane_xor(float v) {
  const int i = __float_as_int(v);
  int r;
  if constexpr (H == 1)
    r = __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
  else if constexpr (H == 2)
    r = __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
  else if constexpr (H < 32)
    r = __builtin_amdgcn_ds_swizzle(i, (H << 10) | 0x1F);      // and 0x1F, or 0, xor H
  else
    r = __builtin_amdgcn_ds_bpermute((int)((threadIdx.x & 63) ^ 32) << 2, i);
  return __int_as_float(r);
}

// One radix-2 decimation-in-frequency stage of span H across lanes: the lower lane keeps a + b, the upper lane
// (a - b) w_2H^(l mod H).
template <int H>
__device__ __forceinline__ void xlane_stage(float2 (&v)[4], int l, float2 w) {
  const bool upper = (l & H) != 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float2 p = make_float2(xlane_xor<H>(v[q].x), xlane_xor<H>(v[q].y));
    v[q] = upper ? cmul(csub(p, v[q]), w) : cadd(v[q], p);
  }
}

// kind 3, cross-lane exchange: 64 lanes per transform, lane l holding x[l + 64 q], q < 4; eight radix-2
// decimation-in-frequency stages, the first two inside the lane, the last six exchanging partner values across
// lanes (no LDS arrays, no barriers).  Position n ends with X[bitrev8(n)].
__global__ __launch_bounds__(256) void k_probe_fft_xlane(int iters, float2 *data) {
  const int l = (int)threadIdx.x & 63, tr = (int)threadIdx.x >> 6;
  float2 *x = data + ((int64_t)blockIdx.x * 4 + tr) * 256;
  float2 v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = x[l + 64 * q];
  auto w_of = [](int t, int span) {   // e^(2 pi i t / span)
    float sn, cs;
    sincospif(2.f * (float)t / (float)span, &sn, &cs);
    return make_float2(cs, sn);
  };
  const float2 w128a = w_of(l, 256), w128b = w_of(l + 64, 256), w64 = w_of(l, 128);
  const float2 w32 = w_of(l & 31, 64), w16 = w_of(l & 15, 32), w8 = w_of(l & 7, 16), w4 = w_of(l & 3, 8),
               w2 = w_of(l & 1, 4), w1 = make_float2(1.f, 0.f);
  for (int it = 0; it < iters; ++it) {
    {   // span 128: (q, q + 2)
      const float2 a0 = v[0], b0 = v[2], a1 = v[1], b1 = v[3];
      v[0] = cadd(a0, b0);
      v[2] = cmul(csub(a0, b0), w128a);
      v[1] = cadd(a1, b1);
      v[3] = cmul(csub(a1, b1), w128b);
    }
    {   // span 64: (q, q + 1)
      const float2 a0 = v[0], b0 = v[1], a1 = v[2], b1 = v[3];
      v[0] = cadd(a0, b0);
      v[1] = cmul(csub(a0, b0), w64);
      v[2] = cadd(a1, b1);
      v[3] = cmul(csub(a1, b1), w64);
    }
    xlane_stage<32>(v, l, w32);
    xlane_stage<16>(v, l, w16);
    xlane_stage<8>(v, l, w8);
    xlane_stage<4>(v, l, w4);
    xlane_stage<2>(v, l, w2);
    xlane_stage<1>(v, l, w1);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = cscale(v[q], 1.f / 256.f);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) x[l + 64 * q] = v[q];
}

// XCD of each workgroup (kind 4): the hardware register XCC_ID (bits 3:0), as the streaming form reads it to form
// its per-XCD teams; thread 0 of workgroup b writes it to out[b].
__global__ __launch_bounds__(256) void k_probe_xcc(float *out) {
  if (threadIdx.x == 0) out[blockIdx.x] = (float)xcc_id();
}

// Exchange access patterns of the 256-point dual-pol fused path with no arithmetic (kinds 5 and 6), over `ncs`
// channel-samples of column-group tiles [u][p][q / 8][row][q % 8] (complex float, 1 MiB per channel-sample).
// Store pattern (the row pass's): one workgroup per (8-row band, run of 32 channel-samples); per channel-sample
// its 16 transforms (2 pols x 8 rows) of 256 outputs, thread j of transform tr storing output q = j + 16 r, r < 16,
// with non-temporal 8-byte stores.
__global__ __launch_bounds__(256) void k_probe_xstore(float2 *H, int ncs) {
  const int band = (int)(blockIdx.x % 32), run = (int)(blockIdx.x / 32);
  const int b = threadIdx.x, tr = b / 16, p = tr / 8, row = band * 8 + tr % 8, j = b % 16;
  const int u1 = min(ncs, run * 32 + 32);
  for (int u = run * 32; u < u1; ++u) {
    float2 *base = H + ((int64_t)u * 2 + p) * 65536 + row * 8;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int q = j + 16 * r;
      store_stream(base + (q / 8) * 2048 + (q % 8), make_float2((float)u, (float)r));
    }
  }
}

// Load pattern (the column pass's): one workgroup per (8-column group, run of 256 channel-samples); per
// channel-sample 2 pols x 256 rows x 8 columns with non-temporal 8-byte loads, thread (col, p, j) reading rows
// j + 16 m.  Each thread adds what it read and writes the sum over the last element it read (its own).
__global__ __launch_bounds__(256) void k_probe_xload(float2 *H, int ncs) {
  const int cg = (int)(blockIdx.x % 32), run = (int)(blockIdx.x / 32);
  const int b = threadIdx.x, col = b % 8, p = (b / 8) % 2, j = b / 16;
  const int u0 = run * 256, u1 = min(ncs, u0 + 256);
  float acc = 0.f;
  for (int u = u0; u < u1; ++u) {
    const float2 *base = H + ((int64_t)u * 2 + p) * 65536 + cg * 2048 + col;
    float2 x[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = load_stream(base + (j + 16 * m) * 8);
#pragma unroll
    for (int m = 0; m < 16; ++m) acc += x[m].x + x[m].y;
  }
  if (u1 > u0) H[((int64_t)(u1 - 1) * 2 + p) * 65536 + cg * 2048 + (j + 16 * 15) * 8 + col].x = acc;
}

hipError_t launch_probe(int kind, int blocks, int iters, float *out, hipStream_t st) {
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, iters, out);
  else if (kind == 1)
    hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, st, iters, out);
  else if (kind == 2)
    hipLaunchKernelGGL(k_probe_fft_lds, dim3(blocks), dim3(256), 0, st, iters, reinterpret_cast<float2 *>(out));
  else if (kind == 3)
    hipLaunchKernelGGL(k_probe_fft_xlane, dim3(blocks * 4), dim3(256), 0, st, iters, reinterpret_cast<float2 *>(out));
  else if (kind == 4)
    hipLaunchKernelGGL(k_probe_xcc, dim3(blocks), dim3(256), 0, st, out);
  else if (kind == 5)
    hipLaunchKernelGGL(k_probe_xstore, dim3(32 * ((blocks + 31) / 32)), dim3(256), 0, st,
                       reinterpret_cast<float2 *>(out), blocks);
  else
    hipLaunchKernelGGL(k_probe_xload, dim3(32 * ((blocks + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<float2 *>(out), blocks);
  return hipGetLastError();
}

}  // namespace moff
