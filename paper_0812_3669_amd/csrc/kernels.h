// Kernel argument blocks and launchers shared by the C ABI (moff_api.cpp) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "moff_plan.h"

namespace moff {

constexpr int kMaxLds = 160 * 1024;   // LDS per CU on CDNA4

// Rows per band of the row pass (must match band_rows_for in the plan).
constexpr int band_rows_ce(int n, int P) {
  int h = 16;
  while (h > 4 && P * h * n * 8 > 32768) h /= 2;
  return h;
}

struct RowArgs {
  const Band *bands;
  const Chan *chans;
  int band_begin, n_bands;   // bands of this launch
  int c0;                    // first channel of the launch block (fused H indexing)
  int t0, nt;                // samples [t0, t0 + nt)
  int t_group, t_block;
  int n_chan, n_ant;
  const void *volt;
  int volt_fmt;
  const uint32_t *meta;
  const float2 *wk;
  const float2 *tw;
  float2 *io;                // fused: H of the launch block; staged: grid buffer
  int64_t sample_stride;     // staged grid: float2 per sample (P * sum n_c^2)
};

struct ColArgs {
  const Chan *chans;
  int c0;
  int t0, nt, t_block;
  const float2 *tw;
  const float2 *in;          // fused: H of the launch block; staged: grid buffer
  float2 *out;               // staged: grid buffer (in place)
  void *acc;                 // fused: accumulator
  int64_t sample_stride;
};

struct AccArgs {
  const Chan *chans;
  int n_chan;
  int64_t pix_total;
  int64_t nt;
  const float2 *efield;
  int64_t sample_stride;
  void *acc;
};

struct ReadArgs {
  const Chan *chans;
  int n_chan;
  int64_t pix_total;
  const void *acc;
  double scale;
  float2 *img;
};

enum { ROW_MODE_FUSED = 0, ROW_MODE_GRID = 1, ROW_MODE_FFT = 2 };
enum { COL_MODE_FUSED = 0, COL_MODE_FFT = 1 };

size_t rows_lds_bytes(int n, int P, int band_rows, int A, int volt_fmt);
size_t cols_lds_bytes(int n, int P, int W);
hipError_t launch_rows(int n, int P, int mode, const RowArgs &a, int grid, size_t lds, hipStream_t st);
hipError_t launch_cols(int n, int P, int W, int mode, int accm, const ColArgs &a, int grid, int gridy, size_t lds,
                       hipStream_t st);
hipError_t launch_acc_staged(int P, int accm, const AccArgs &a, hipStream_t st);
hipError_t launch_read_image(int P, int accm, const ReadArgs &a, hipStream_t st);
hipError_t launch_twiddle(float2 *tw, int n, hipStream_t st);
hipError_t launch_pack_kernels(const float2 *kern, const int32_t *kidx, const int32_t *grp_chan, float2 *wk,
                               int64_t n_groups, int A, int P, int KK, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_unpack_debug(const void *volt, int fmt, float2 *out, int64_t count, hipStream_t st);

}  // namespace moff
