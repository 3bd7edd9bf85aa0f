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

// Whether the row pass of length n copies its band's voltages into an LDS table once per sample (tap-group
// metadata then holds the antenna's position in the band list) or gathers them per tap from the voltage row
// (metadata holds the antenna index).  At 320 and 384 the table's registers cost a wave per SIMD, which outweighs
// the coalesced loads.
constexpr bool row_stages_volts(int n) { return n != 320 && n != 384; }

}  // namespace moff
