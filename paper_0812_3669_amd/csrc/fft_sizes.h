// Transform lengths with an FFT pipeline and the LDS row stride of the row pass; shared by the host plan and the
// kernels (pure constexpr, no HIP).
#pragma once

namespace moff {

// Largest radix of the pipeline of length n (0 if n has none): 2^a * {1, 3, 5} lengths use radices 3, 4, 5, 8, 16.
constexpr int fft_radix_max(int n) {
  return n == 32 || n == 64 || n == 96 || n == 160 || n == 192 || n == 320 || n == 512 ? 8
         : n == 128 || n == 256 || n == 384                                             ? 16
                                                                                         : 0;
}

// LDS stride (complex elements) of one row in the row pass: the padded inter-stage layout needs n + R - 1.
constexpr int row_stride(int n) { return n + fft_radix_max(n); }

}  // namespace moff
