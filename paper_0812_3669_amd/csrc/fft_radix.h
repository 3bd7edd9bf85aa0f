// Small complex DFTs for the spatial transform F^T (Eq. m6 step 3), sign +: X[k] = sum_m x[m] exp(+2 pi i m k / R).
// The radix-R butterflies are the nodes of the Cooley-Tukey graph of Fig. 1 (rows d-e): each node rotates its
// inputs by a twiddle factor and sums them.  Constants are cos/sin of exact rational multiples of pi.
#pragma once

#include <hip/hip_runtime.h>

namespace moff {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }   // a * (+i)

constexpr float kR2 = 0.70710678118654752440f;     // 1/sqrt(2)
constexpr float kC8 = 0.92387953251128675613f;     // cos(pi/8)
constexpr float kS8 = 0.38268343236508977173f;     // sin(pi/8)
constexpr float kS3 = 0.86602540378443864676f;     // sin(2 pi/3)
constexpr float kC51 = 0.30901699437494742410f;    // cos(2 pi/5)
constexpr float kS51 = 0.95105651629515357212f;    // sin(2 pi/5)
constexpr float kC52 = -0.80901699437494742410f;   // cos(4 pi/5)
constexpr float kS52 = 0.58778525229247312917f;    // sin(4 pi/5)

__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
  const float2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_i(csub(x1, x3));
  x0 = cadd(a, c);
  x1 = cadd(b, d);
  x2 = csub(a, c);
  x3 = csub(b, d);
}

__device__ __forceinline__ void dft3(float2 &x0, float2 &x1, float2 &x2) {
  const float2 t = cadd(x1, x2);
  const float2 m = make_float2(x0.x - 0.5f * t.x, x0.y - 0.5f * t.y);
  const float2 d = cscale(mul_i(csub(x1, x2)), kS3);
  x0 = cadd(x0, t);
  x1 = cadd(m, d);
  x2 = csub(m, d);
}

__device__ __forceinline__ void dft5(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float2 &x4) {
  const float2 s14 = cadd(x1, x4), d14 = csub(x1, x4), s23 = cadd(x2, x3), d23 = csub(x2, x3);
  const float2 r1 = make_float2(x0.x + kC51 * s14.x + kC52 * s23.x, x0.y + kC51 * s14.y + kC52 * s23.y);
  const float2 r2 = make_float2(x0.x + kC52 * s14.x + kC51 * s23.x, x0.y + kC52 * s14.y + kC51 * s23.y);
  const float2 i1 = mul_i(make_float2(kS51 * d14.x + kS52 * d23.x, kS51 * d14.y + kS52 * d23.y));
  const float2 i2 = mul_i(make_float2(kS52 * d14.x - kS51 * d23.x, kS52 * d14.y - kS51 * d23.y));
  x0 = cadd(x0, cadd(s14, s23));
  x1 = cadd(r1, i1);
  x4 = csub(r1, i1);
  x2 = cadd(r2, i2);
  x3 = csub(r2, i2);
}

// w8^1 = (1+i)/sqrt2, w8^3 = (-1+i)/sqrt2
__device__ __forceinline__ float2 mul_w8_1(float2 a) { return make_float2((a.x - a.y) * kR2, (a.x + a.y) * kR2); }
__device__ __forceinline__ float2 mul_w8_3(float2 a) { return make_float2(-(a.x + a.y) * kR2, (a.x - a.y) * kR2); }

__device__ __forceinline__ void dft8(float2 (&x)[8]) {
  dft4(x[0], x[2], x[4], x[6]);
  dft4(x[1], x[3], x[5], x[7]);
  const float2 o1 = mul_w8_1(x[3]), o2 = mul_i(x[5]), o3 = mul_w8_3(x[7]);
  float2 y[8];
  y[0] = cadd(x[0], x[1]);
  y[4] = csub(x[0], x[1]);
  y[1] = cadd(x[2], o1);
  y[5] = csub(x[2], o1);
  y[2] = cadd(x[4], o2);
  y[6] = csub(x[4], o2);
  y[3] = cadd(x[6], o3);
  y[7] = csub(x[6], o3);
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = y[k];
}

// 16 = 4 x 4: inner DFT4 over n2 of x[n1 + 4 n2], twiddle w16^(n1 k1), outer DFT4 over n1; X[k1 + 4 k2].
__device__ __forceinline__ void dft16(float2 (&x)[16]) {
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) dft4(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]);
  // after this, x[n1 + 4 k1] holds y[n1][k1]
  const float2 w1 = make_float2(kC8, kS8), w3 = make_float2(kS8, kC8), w9 = make_float2(-kC8, -kS8);
  x[1 + 4 * 1] = cmul(x[1 + 4 * 1], w1);
  x[1 + 4 * 2] = mul_w8_1(x[1 + 4 * 2]);
  x[1 + 4 * 3] = cmul(x[1 + 4 * 3], w3);
  x[2 + 4 * 1] = mul_w8_1(x[2 + 4 * 1]);
  x[2 + 4 * 2] = mul_i(x[2 + 4 * 2]);
  x[2 + 4 * 3] = mul_w8_3(x[2 + 4 * 3]);
  x[3 + 4 * 1] = cmul(x[3 + 4 * 1], w3);
  x[3 + 4 * 2] = mul_w8_3(x[3 + 4 * 2]);
  x[3 + 4 * 3] = cmul(x[3 + 4 * 3], w9);
  float2 y[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = x[0 + 4 * k1], b = x[1 + 4 * k1], c = x[2 + 4 * k1], d = x[3 + 4 * k1];
    dft4(a, b, c, d);
    y[k1 + 0] = a;
    y[k1 + 4] = b;
    y[k1 + 8] = c;
    y[k1 + 12] = d;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = y[k];
}

template <int R>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
  if constexpr (R == 2) {
    dft2(x[0], x[1]);
  } else if constexpr (R == 3) {
    dft3(x[0], x[1], x[2]);
  } else if constexpr (R == 4) {
    dft4(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 5) {
    dft5(x[0], x[1], x[2], x[3], x[4]);
  } else if constexpr (R == 8) {
    dft8(x);
  } else if constexpr (R == 16) {
    dft16(x);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// Radix factorisation of each supported transform length (first stage first).
template <int N> struct Fac;
template <> struct Fac<32>  { static constexpr int S = 2, R0 = 4, R1 = 8, R2 = 1; };
template <> struct Fac<64>  { static constexpr int S = 2, R0 = 8, R1 = 8, R2 = 1; };
template <> struct Fac<96>  { static constexpr int S = 3, R0 = 3, R1 = 4, R2 = 8; };
template <> struct Fac<128> { static constexpr int S = 2, R0 = 8, R1 = 16, R2 = 1; };
template <> struct Fac<160> { static constexpr int S = 3, R0 = 5, R1 = 4, R2 = 8; };
template <> struct Fac<192> { static constexpr int S = 3, R0 = 3, R1 = 8, R2 = 8; };
template <> struct Fac<256> { static constexpr int S = 2, R0 = 16, R1 = 16, R2 = 1; };
template <> struct Fac<320> { static constexpr int S = 3, R0 = 5, R1 = 8, R2 = 8; };
template <> struct Fac<384> { static constexpr int S = 3, R0 = 3, R1 = 8, R2 = 16; };
template <> struct Fac<512> { static constexpr int S = 3, R0 = 8, R1 = 8, R2 = 8; };

}  // namespace moff
