// Precision form of the spatial transform: the 256-point FFT of 16 transforms at once as two radix-16 DFT-GEMMs
// on the CDNA4 matrix cores (v_mfma_f32_16x16x32_{f16,bf16}), with a split product that recovers FP32-level
// accuracy from 16-bit operands.
//
// A radix-16 stage over 16 transforms is Y = A X with X the 16 complex inputs of one butterfly per transform
// (32 x 16 real, rows [Re x_0..15; Im x_0..15]) and A the real form [[C, -S], [S, C]] of the 16-point DFT (sign
// +), split into a Re-row and an Im-row 16 x 32 operand.  The twiddles of the second stage are folded into its
// matrices (one per butterfly index j2: w16^(r m) w256^(j2 m)), so no VALU twiddle multiply remains.
//
// Split products.  FP16: x = hi + lo with hi = fp16(s x), lo = fp16(s x - hi) and s a power of two per
// (butterfly, transform) column keeping |s x| < 2^14; A = A_hi + A_lo; the product keeps hi.hi + hi.lo + lo.hi,
// accumulated in FP32 (error ~2^-22 of the column maximum).  BF16: three terms hi + mid + lo (24 bits), six
// products (hh, hm, mh, hl, lh, mm); bf16 has FP32's range, so no scaling.  The matrices are generated in FP64
// on the device and split there.
//
// Lane layout of v_mfma_f32_16x16x32 (wave64): A (16 x 32): lane l holds A[l % 16][8 (l / 16) + i], i < 8;
// B (32 x 16): lane l holds B[8 (l / 16) + i][l % 16]; D (16 x 16): lane l holds D[4 (l / 16) + i][l % 16], i < 4.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace moff {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaTerms = 3;           // split terms stored per matrix entry (fp16 uses 2)
// Matrix table: 17 matrices (stage 1, then stage 2 for j2 = 0..15) x 2 parts (Re row, Im row) x kMfmaTerms
// x 64 lanes x 8 values (16-bit).  Stored as uint16 bit patterns.
constexpr int kMfmaMatrices = 17;
constexpr size_t kMfmaTableHalfs = (size_t)kMfmaMatrices * 2 * kMfmaTerms * 64 * 8;
constexpr int kYStride = 16 * 16 + 4;   // floats per (component, transform) of the stage-1 LDS scratch

template <bool BF16>
struct MfmaOps;

template <>
struct MfmaOps<false> {
  typedef half8_t vec;
  static constexpr int terms = 2;
  __device__ static vec load(const uint16_t *p) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    vec v;
    __builtin_memcpy(&v, &u, 16);
    return v;
  }
  __device__ static float4_t mma(vec a, vec b, float4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
  // s x = hi + lo
  __device__ static void split(const float (&x)[8], vec (&t)[3]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const _Float16 h = (_Float16)x[i];
      t[0][i] = h;
      t[1][i] = (_Float16)(x[i] - (float)h);
      t[2][i] = (_Float16)0.0f;
    }
  }
  __device__ static float4_t product(const vec (&a)[3], const vec (&b)[3]) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    c = mma(a[1], b[0], c);
    c = mma(a[0], b[1], c);
    c = mma(a[0], b[0], c);
    return c;
  }
};

template <>
struct MfmaOps<true> {
  typedef bf16x8_t vec;
  static constexpr int terms = 3;
  __device__ static vec load(const uint16_t *p) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    vec v;
    __builtin_memcpy(&v, &u, 16);
    return v;
  }
  __device__ static float4_t mma(vec a, vec b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static void split(const float (&x)[8], vec (&t)[3]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 h = (__bf16)x[i];
      const float r1 = x[i] - (float)h;
      const __bf16 m = (__bf16)r1;
      t[0][i] = h;
      t[1][i] = m;
      t[2][i] = (__bf16)(r1 - (float)m);
    }
  }
  __device__ static float4_t product(const vec (&a)[3], const vec (&b)[3]) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    c = mma(a[1], b[1], c);   // small terms first
    c = mma(a[2], b[0], c);
    c = mma(a[0], b[2], c);
    c = mma(a[1], b[0], c);
    c = mma(a[0], b[1], c);
    c = mma(a[0], b[0], c);
    return c;
  }
};

// The matrix operands a wavefront needs, loaded once and kept in registers: stage 1, and the stage-2 matrices
// of the four butterflies j2 = 4 w + jj the wavefront computes.
template <bool BF16>
struct MfmaMats {
  using V = typename MfmaOps<BF16>::vec;
  V s1[2][3];        // [part][term]
  V s2[4][2][3];     // [jj][part][term]
  __device__ void load(const uint16_t *__restrict__ table, int lane, int wave) {
    constexpr size_t kMat = (size_t)2 * kMfmaTerms * 64 * 8;
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < MfmaOps<BF16>::terms) {
          s1[part][k] = MfmaOps<BF16>::load(table + ((size_t)(part * kMfmaTerms + k) * 64 + lane) * 8);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            s2[jj][part][k] = MfmaOps<BF16>::load(table + (size_t)(1 + 4 * wave + jj) * kMat +
                                                  ((size_t)(part * kMfmaTerms + k) * 64 + lane) * 8);
        } else {
          s1[part][k] = V{};
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) s2[jj][part][k] = V{};
        }
      }
  }
};

// One radix-16 DFT-GEMM over 16 transforms: lane (g = l / 16, t = l % 16) supplies x[8 (g & 1) + i] of component
// (g >> 1) (0 Re, 1 Im) of transform t and receives y[4 g + i] (Re, Im) of transform t.
template <bool BF16>
__device__ __forceinline__ void dft16_mfma(const float (&xin)[8], const typename MfmaOps<BF16>::vec (&are)[3],
                                           const typename MfmaOps<BF16>::vec (&aim)[3], float (&yre)[4],
                                           float (&yim)[4]) {
  using O = MfmaOps<BF16>;
  float x[8];
  float s = 1.f, inv = 1.f;
  if constexpr (!BF16) {
    // per-column power-of-two scale: the 4 lanes of transform t hold its 32 reals
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mx = fmaxf(mx, fabsf(xin[i]));
    mx = fmaxf(mx, __shfl_xor(mx, 16));
    mx = fmaxf(mx, __shfl_xor(mx, 32));
    if (mx > 0.f) {
      int e;
      (void)frexpf(mx, &e);          // mx = f 2^e, f in [0.5, 1)
      s = ldexpf(1.f, 14 - e);
      inv = ldexpf(1.f, e - 14);
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = xin[i] * s;
  typename O::vec b[3];
  O::split(x, b);
  const float4_t dre = O::product(are, b);
  const float4_t dim = O::product(aim, b);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    yre[i] = dre[i] * inv;
    yim[i] = dim[i] * inv;
  }
}

// 256-point FFTs (sign +) of 16 transforms held in LDS, natural order, transform t at x + t * xstride
// (complex64).  ys: LDS scratch of 2 * 16 * kYStride floats.  Wave w computes butterflies j = 4 w .. 4 w + 3 of
// each stage.  out(t, q, value, jj, i) receives output q of transform t in the lane that computed it (each
// (t, q) once).  Contains one barrier; the caller synchronises before x is reused.
template <bool BF16, class Out>
__device__ __forceinline__ void fft256x16_mfma(const float2 *x, int xstride, float *ys, const MfmaMats<BF16> &M,
                                               Out out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & 15, g = lane >> 4, comp = g >> 1, half = g & 1;
  const float *xf = reinterpret_cast<const float *>(x);
  // stage 1: butterfly j takes x[j + 16 m]
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int j = 4 * wave + jj;
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = xf[2 * (t * xstride + j + 16 * (8 * half + i)) + comp];
    float yre[4], yim[4];
    dft16_mfma<BF16>(v, M.s1[0], M.s1[1], yre, yim);
    // stage-1 output (j, r) goes to ys[c][t][r][j]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * g + i;
      ys[(0 * 16 + t) * kYStride + r * 16 + j] = yre[i];
      ys[(1 * 16 + t) * kYStride + r * 16 + j] = yim[i];
    }
  }
  __syncthreads();
  // stage 2: butterfly j2 takes the outputs r = j2 of the stage-1 butterflies j1 = m (twiddles in the matrix)
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int j2 = 4 * wave + jj;
    float v[8];
    const float *src = ys + (comp * 16 + t) * kYStride + j2 * 16 + 8 * half;
    const float4 a0 = *reinterpret_cast<const float4 *>(src);
    const float4 a1 = *reinterpret_cast<const float4 *>(src + 4);
    v[0] = a0.x; v[1] = a0.y; v[2] = a0.z; v[3] = a0.w;
    v[4] = a1.x; v[5] = a1.y; v[6] = a1.z; v[7] = a1.w;
    float yre[4], yim[4];
    dft16_mfma<BF16>(v, M.s2[jj][0], M.s2[jj][1], yre, yim);
#pragma unroll
    for (int i = 0; i < 4; ++i) out(t, j2 + 16 * (4 * g + i), make_float2(yre[i], yim[i]), jj, i);
  }
}

}  // namespace moff
