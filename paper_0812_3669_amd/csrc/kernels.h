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
  const int limit = (n & (n - 1)) == 0 ? 32768 : 16384;
  int h = 16;
  while (h > 4 && P * h * n * 8 > limit) h /= 2;
  return h;
}

// Columns per column-pass workgroup (must match cols_for in the plan): the largest power of two
// <= max(8, 2048 / n) dividing n.
constexpr int cols_ce(int n) {
  int lim = 2048 / n > 8 ? 2048 / n : 8, w = 1;
  while (w * 2 <= lim && n % (w * 2) == 0) w *= 2;
  return w;
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
  const int32_t *band_ant;   // band antenna lists (Band::ant_off, ant_cnt)
  int band_ants_max;         // longest list: entries of the LDS voltage table
  const float2 *wk;
  const float2 *tw;
  float2 *io;                // fused: H of the launch block; staged: grid buffer
  int64_t sample_stride;     // staged grid: float2 per sample (P * sum n_c^2)
  int n_chan_block;          // fused: channels in the launch block (XCD-aware workgroup mapping)
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
  int n_chan_block;          // fused: channels in the launch block (XCD-aware workgroup mapping)
  int full_rows;             // staged FFT: every row of the column holds data (no footprint row range)
};

// XCD-aware workgroup mapping of the fused passes.  Workgroups are dispatched round-robin over the 8 XCDs
// (workgroup b runs on XCD b % 8), so channel c0 + k of a launch block is given to XCD k % 8: its tap tables and
// voltages stay in one XCD's L2 instead of being fetched by all eight.  Padding workgroups get false.
constexpr int kXcds = kStreamXcds;

__device__ inline bool rows_xcd_map(const RowArgs &a, int &band, int &tg) {
  const int x = (int)(blockIdx.x % kXcds), s = (int)(blockIdx.x / kXcds);
  const int tgroups = (a.nt + a.t_group - 1) / a.t_group;
  tg = s % tgroups;
  int slot = s / tgroups;
  for (int k = x; k < a.n_chan_block; k += kXcds) {
    const Chan &ch = a.chans[a.c0 + k];
    if (slot < ch.band_count) {
      band = ch.band_first + slot;
      return true;
    }
    slot -= ch.band_count;
  }
  return false;
}

__device__ inline bool cols_xcd_map(const ColArgs &a, int groups, int &c, int &g) {
  const int x = (int)(blockIdx.x % kXcds), s = (int)(blockIdx.x / kXcds);
  const int k = x + kXcds * (s / groups);
  if (k >= a.n_chan_block) return false;
  c = a.c0 + k;
  g = s % groups;
  return true;
}

// Workgroups of the fused passes for a launch block (host side, same mapping as above).
inline int rows_xcd_grid(const Plan &p, const Block &b, int tgroups) {
  int mx = 0;
  for (int x = 0; x < kXcds; ++x) {
    int n = 0;
    for (int k = x; k < b.c1 - b.c0; k += kXcds) n += p.chans[b.c0 + k].band_count;
    mx = n > mx ? n : mx;
  }
  return kXcds * tgroups * mx;
}

inline int cols_xcd_grid(const Block &b, int groups) {
  return kXcds * groups * ((b.c1 - b.c0 + kXcds - 1) / kXcds);
}

typedef float vfloat2 __attribute__((ext_vector_type(2)));

// The XCD (accelerator complex die) this wave runs on: hardware register XCC_ID (id 20), bits 3:0.  Workgroups
// on one XCD share its L2.
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xFu);   // size 4, offset 0, register 20
}

// Streaming store / load of the row-transform buffer: written once, read once, kept out of the way of the
// tap tables in L2.
__device__ __forceinline__ void store_stream(float2 *p, float2 v) {
  __builtin_nontemporal_store(vfloat2{v.x, v.y}, reinterpret_cast<vfloat2 *>(p));
}
__device__ __forceinline__ float2 load_stream(const float2 *p) {
  const vfloat2 v = __builtin_nontemporal_load(reinterpret_cast<const vfloat2 *>(p));
  return make_float2(v.x, v.y);
}

// Streaming form (one persistent launch per grid size; see k_stream).
struct StreamArgs {
  RowArgs r;                 // c0: first channel of the launch, t0 / nt: the samples
  ColArgs c;                 // t_block: samples per accumulator update
  float2 *ring;              // [kXcds][slots][P n^2] row-transformed samples in column-group tiles
  uint32_t *ctr;             // [kXcds][2][slots] cumulative counters: bands produced, column groups consumed
  int *err;                  // 0, or 1 (a wait timed out)
  int slots;
  int wgs_per_xcd;
  int n_chan_group;          // channels c0 .. c0 + n_chan_group - 1, all of one grid size
  uint32_t spin_limit;
};

// Voltages of G taps at once from a voltage row laid out like the caller's (record = meta >> 16): the row pass
// reads its band's LDS voltage table, or the voltage row itself, this way.  The format branch is uniform and
// outside the unrolled reads, and the reads are unconditional, so all G are issued before the first is used.
template <int P, int G>
__device__ __forceinline__ void load_volts(const void *row, int fmt, const uint32_t (&m)[G], float2 (&e)[G][P]) {
  if (fmt == 0) {
    uint32_t w[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if constexpr (P == 2)
        w[k] = reinterpret_cast<const uint32_t *>(row)[m[k] >> 16];
      else
        w[k] = reinterpret_cast<const uint16_t *>(row)[m[k] >> 16];
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const uint32_t v = w[k];
      e[k][0] = make_float2((float)(int8_t)(v & 0xFF), (float)(int8_t)((v >> 8) & 0xFF));
      if constexpr (P == 2) e[k][1] = make_float2((float)(int8_t)((v >> 16) & 0xFF), (float)(int8_t)(v >> 24));
    }
  } else {
    if constexpr (P == 2) {
      float4 w[G];
#pragma unroll
      for (int k = 0; k < G; ++k) w[k] = reinterpret_cast<const float4 *>(row)[m[k] >> 16];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        e[k][0] = make_float2(w[k].x, w[k].y);
        e[k][1] = make_float2(w[k].z, w[k].w);
      }
    } else {
#pragma unroll
      for (int k = 0; k < G; ++k) e[k][0] = reinterpret_cast<const float2 *>(row)[m[k] >> 16];
    }
  }
}

// One lane's packed kernel values of one tap group (planes contiguous, wk[g][lane][plane]): 16-byte loads.
template <int PL>
__device__ __forceinline__ void load_taps(const float2 *p, float2 (&w)[PL]) {
  if constexpr (PL == 1) {
    w[0] = p[0];
  } else {
#pragma unroll
    for (int q = 0; q < PL / 2; ++q) {
      const float4 v = reinterpret_cast<const float4 *>(p)[q];
      w[2 * q] = make_float2(v.x, v.y);
      w[2 * q + 1] = make_float2(v.z, v.w);
    }
  }
}

// Bytes of one antenna's voltages for one (sample, channel): P pols of (re, im), int8 (format 0) or float.
__host__ __device__ constexpr int volt_rec_bytes(int P, int fmt) { return P * (fmt == 0 ? 2 : 8); }

// Bytes of the row pass's LDS voltage table: one record per antenna of the longest band list, 16-byte aligned.
__host__ __device__ constexpr size_t volt_table_bytes(int band_ants, int P, int fmt) {
  return ((size_t)band_ants * volt_rec_bytes(P, fmt) + 15) / 16 * 16;
}

// One antenna's voltage record (2, 4, 8 or 16 bytes) as a single load, in the low words of a uint4.
template <int P>
__device__ __forceinline__ uint4 fetch_volt_rec(const char *row, int fmt, int ant) {
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (fmt == 0) {
    if constexpr (P == 2)
      v.x = reinterpret_cast<const uint32_t *>(row)[ant];
    else
      v.x = reinterpret_cast<const uint16_t *>(row)[ant];
  } else {
    if constexpr (P == 2) {
      v = reinterpret_cast<const uint4 *>(row)[ant];
    } else {
      const uint2 w = reinterpret_cast<const uint2 *>(row)[ant];
      v.x = w.x;
      v.y = w.y;
    }
  }
  return v;
}

// Writes record i of the LDS voltage table (the layout of one voltage row: load_volts reads it back).
template <int P>
__device__ __forceinline__ void put_volt_rec(char *vtab, int fmt, int i, uint4 v) {
  if (fmt == 0) {
    if constexpr (P == 2)
      reinterpret_cast<uint32_t *>(vtab)[i] = v.x;
    else
      reinterpret_cast<uint16_t *>(vtab)[i] = (uint16_t)v.x;
  } else {
    if constexpr (P == 2)
      reinterpret_cast<uint4 *>(vtab)[i] = v;
    else
      reinterpret_cast<uint2 *>(vtab)[i] = make_uint2(v.x, v.y);
  }
}

// Device-coherent (agent scope) 8-byte store / load: not cached in the non-coherent L1 / L2, so a value
// written by one workgroup is seen by another on any XCD once the writer's stores have completed.
__device__ __forceinline__ void store_coherent(float2 *p, float2 v) {
  uint64_t b;
  __builtin_memcpy(&b, &v, 8);
  __hip_atomic_store(reinterpret_cast<uint64_t *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 load_coherent(const float2 *p) {
  const uint64_t b = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  float2 v;
  __builtin_memcpy(&v, &b, 8);
  return v;
}

enum { LD_PLAIN = 0, LD_STREAM = 1, LD_COHERENT = 2 };

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

// Taps and feedback calibration (kernels_cal.hip).
constexpr int kMaxTaps = 8;

struct TapArgs {
  const Chan *chans;
  const float2 *h;           // row-transformed samples of the launch block (fused path)
  const float2 *tap_tw;      // per (channel, tap): n twiddles exp(+2 pi i j qr / n)
  const int64_t *tap_tw_off; // [C] offset of the channel's tables in tap_tw
  const int2 *tap_idx;       // [C][n_tap] (qr, qc) FFT-order indices
  float2 *out;               // [T][C][n_tap][P]
  int c0, n_chan_block, t0, nt, t_block, n_chan, n_tap, P;
};

struct CalArgs {
  const void *volt;
  int volt_fmt;
  const float2 *tap;         // [nt][C][n_tap][P]
  void *cal;                 // double2 R [C][n_tap][A][P], double Pw [C][n_tap][P], double V [C][A][P]
  int64_t nt;
  int n_chan, n_ant, n_tap, P;
};

struct SolveArgs {
  const Chan *chans;
  const void *cal;
  const float2 *kern;        // [C][A][P][K][K]
  const int2 *origin;        // [C][A] (j0, i0)
  const int2 *tap_cpix;      // [C][n_tap] centred (row, col)
  void *out;                 // double2 [3][C][n_tap][A][P]: S, X, u
  int n_chan, n_ant, n_tap, P, K;
};

hipError_t launch_tap(const TapArgs &a, hipStream_t st);
hipError_t launch_cal_acc(const CalArgs &a, hipStream_t st);
hipError_t launch_cal_solve(const SolveArgs &a, hipStream_t st);

enum { ROW_MODE_FUSED = 0, ROW_MODE_GRID = 1, ROW_MODE_FFT = 2 };
enum { COL_MODE_FUSED = 0, COL_MODE_FFT = 1 };

size_t rows_lds_bytes(int n, int P, int band_rows, int band_ants, int volt_fmt);
size_t cols_lds_bytes(int n, int P, int W);
hipError_t launch_rows(int n, int P, int mode, bool jones, const RowArgs &a, int grid, size_t lds, hipStream_t st);
hipError_t launch_cols(int n, int P, int W, int mode, int accm, const ColArgs &a, int grid, int gridy, size_t lds,
                       hipStream_t st);
hipError_t launch_acc_staged(int P, int accm, const AccArgs &a, hipStream_t st);
hipError_t launch_read_image(int P, int accm, const ReadArgs &a, hipStream_t st);
hipError_t launch_twiddle(float2 *tw, int n, hipStream_t st);
hipError_t launch_pack_kernels(const float2 *kern, const float2 *phase, const int32_t *kidx, const int32_t *grp_chan,
                               float2 *wk, int64_t n_groups, int A, int P, int KK, int planes, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_unpack_debug(const void *volt, int fmt, float2 *out, int64_t count, hipStream_t st);
hipError_t set_lds_limit_ext(const void *fn);
size_t stream_lds_bytes(int n, int P, int band_ants, int volt_fmt);
hipError_t stream_occupancy(int n, int P, int accm, bool jones, int band_ants, int volt_fmt, int *wgs_per_cu);
hipError_t launch_stream(int n, int P, int accm, bool jones, const StreamArgs &a, hipStream_t st);

// precision form (256^2 grids, two pols; kernels_mfma.hip)
constexpr size_t kMfmaTableBytes = (size_t)17 * 2 * 3 * 64 * 8 * 2;
size_t rows_mfma_lds_bytes(int band_ants, int volt_fmt);
size_t cols_mfma_lds_bytes();
hipError_t launch_mfma_table(uint16_t *tab, int bf16, hipStream_t st);
hipError_t launch_rows_mfma(int bf16, const RowArgs &a, const uint16_t *table, int grid, hipStream_t st);
hipError_t launch_cols_mfma(int bf16, int accm, const ColArgs &a, const uint16_t *table, int grid, hipStream_t st);

// Matrix-core row pass (kernels_rowgemm.hip): gridding and row transform as one split-FP16 GEMM over time samples.
struct RgArgs {
  const Chan *chans;
  const int32_t *rows;       // [touched rows][2]: first entry, antenna count (channel c's row jmin at chans[c].rg_first)
  const uint32_t *ents;      // antenna | (row - j0) << 16 | i0 << 20
  const float2 *rk;          // kernels [C][A][P][K][K], phases folded
  const float2 *tw;          // w^m, m < n
  const void *volt;          // int8 [T][C][A][P][2]
  float2 *io;                // H of the launch block (column-group tiles, as the FP32 row pass writes it)
  int c0, n_chan_block, t0, nt, t_block, n_chan, n_ant, K, P;
  int tt;                    // samples per time tile (multiple of 16, <= 128)
  int slots;                 // antenna slots of the LDS tables (the longest row list, rounded up to 16)
};
int rowgemm_grid(const Plan &p, const Block &b, int nt);
hipError_t launch_rowgemm(int n, const RgArgs &a, int grid, hipStream_t st);
hipError_t launch_rg_twiddle(float2 *tw, int n, hipStream_t st);
hipError_t launch_pack_rk(const float2 *kern, const float2 *phase, float2 *rk, int64_t total, int KK, hipStream_t st);

// Exchange buffer of the no-alloc entry point (kernels_noalloc.hip): its device address on the current device
// (looked up once per device) and its size.
constexpr size_t kNoallocExchangeBytes = (size_t)MOFF_NOALLOC_EXCHANGE_BYTES;
hipError_t noalloc_exchange(void **ptr, size_t *bytes);

// Issue-rate probes (kernels_probe.hip): kind 0 FP32 vector FMAs, kind 1 FP16 matrix-core instructions.
hipError_t launch_probe(int kind, int blocks, int iters, float *out, hipStream_t st);

}  // namespace moff
