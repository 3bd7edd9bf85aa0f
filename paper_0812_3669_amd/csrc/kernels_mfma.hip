// Precision form of the fused path (256^2 grids, two pols): the row and column passes of k_rows / k_cols with
// both radix-16 FFT stages on the matrix cores (split FP16 or BF16 products, FP32 accumulation; see
// mfma_fft.h).  Gridding, the row-transform buffer layout and the accumulation are those of the FP32 path.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_sizes.h"
#include "kernels.h"
#include "mfma_fft.h"

namespace moff {

namespace {
constexpr int MN = 256;            // transform length
constexpr int MP = 2;              // pols
constexpr int MHB = 8;             // rows per band (2 pols x 8 rows = 16 transforms)
constexpr int MW = 8;              // columns per column-pass workgroup (2 pols x 8 columns = 16 transforms)
constexpr int MTS = MN + 17;       // odd LDS stride per transform: the 16 lanes of a column hit 16 bank pairs
static_assert(band_rows_ce(MN, MP) == MHB && cols_ce(MN) == MW, "launch geometry of the precision form");
static_assert(row_stages_volts(MN), "the precision form reads voltages from the LDS table");
}  // namespace

// Matrix table (see mfma_fft.h), generated in FP64 from integer-reduced angles and split into 16-bit terms.
__global__ void k_mfma_table(uint16_t *tab, int bf16) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int)kMfmaTableHalfs) return;
  int rest = e;
  const int i = rest % 8;
  rest /= 8;
  const int lane = rest % 64;
  rest /= 64;
  const int term = rest % kMfmaTerms;
  rest /= kMfmaTerms;
  const int part = rest % 2;           // 0: Re row, 1: Im row
  const int mat = rest / 2;            // 0: stage 1, 1 + j2: stage 2
  const int r = lane % 16, k = 8 * (lane / 16) + i, m = k % 16;
  const int j2 = mat == 0 ? 0 : mat - 1;
  const long long num = ((long long)16 * r * m + (long long)j2 * m) % 256;   // angle 2 pi num / 256
  double s, c;
  sincospi(2.0 * (double)num / 256.0, &s, &c);
  const double v = part == 0 ? (k < 16 ? c : -s) : (k < 16 ? s : c);
  uint16_t bits = 0;
  if (!bf16) {
    const _Float16 hi = (_Float16)(float)v;
    const _Float16 lo = (_Float16)(float)(v - (double)(float)hi);
    const _Float16 t = term == 0 ? hi : term == 1 ? lo : (_Float16)0.0f;
    __builtin_memcpy(&bits, &t, 2);
  } else {
    const __bf16 hi = (__bf16)(float)v;
    const double r1 = v - (double)(float)hi;
    const __bf16 md = (__bf16)(float)r1;
    const __bf16 lo = (__bf16)(float)(r1 - (double)(float)md);
    const __bf16 t = term == 0 ? hi : term == 1 ? md : lo;
    __builtin_memcpy(&bits, &t, 2);
  }
  tab[e] = bits;
}

template <bool BF16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_rows_mfma(RowArgs a, const uint16_t *table) {
  extern __shared__ float4 smem4[];
  float2 *grid = reinterpret_cast<float2 *>(smem4);        // [MP][MHB][MTS]
  float *ys = reinterpret_cast<float *>(grid + MP * MHB * MTS);
  char *vtab = reinterpret_cast<char *>(ys + 2 * 16 * kYStride);   // band voltage table (volt_table_bytes)

  int band, tg;
  if (!rows_xcd_map(a, band, tg)) return;
  const Band *bp = a.bands + band;
  const int c = bp->chan, row0 = bp->row0, r_lo = bp->r_lo, r_hi = bp->r_hi;
  const int t_lo = a.t0 + tg * a.t_group;
  const int t_hi = min(a.t0 + a.nt, t_lo + a.t_group);
  const int nrow = r_hi - r_lo + 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g0 = bp->grp_off[wave];
  const int gc = bp->grp_cnt[wave];
  const size_t vbytes = (size_t)a.n_ant * MP * (a.volt_fmt == 0 ? 2 : 8);
  constexpr int GCH = 8;
  MfmaMats<BF16> mats;
  mats.load(table, lane, wave);
  // voltages staged in LDS per sample, as in the FP32 row pass: thread i copies the i-th antenna of the band
  const int bcnt = bp->ant_cnt;
  const int32_t *blist = a.band_ant + bp->ant_off;
  const int my_ant = (int)threadIdx.x < bcnt ? blist[threadIdx.x] : -1;
  auto vrow_of = [&](int t) {
    return reinterpret_cast<const char *>(a.volt) + ((int64_t)t * a.n_chan + c) * vbytes;
  };
  // int8 records (one register) are loaded one sample ahead; float records are copied when they are staged
  const bool pre8 = a.volt_fmt == 0 && my_ant >= 0;
  uint32_t nxt = 0u;
  if (pre8 && t_lo < t_hi) nxt = fetch_volt_rec<MP>(vrow_of(t_lo), 0, my_ant).x;

  for (int t = t_lo; t < t_hi; ++t) {
    // priority 1 while the wave loads and scatters, 0 for the transforms (as in the FP32 row pass)
    __builtin_amdgcn_s_setprio(1);
    if (pre8) {
      if (t == t_lo) put_volt_rec<MP>(vtab, 0, threadIdx.x, make_uint4(nxt, 0u, 0u, 0u));
    } else if (my_ant >= 0) {
      put_volt_rec<MP>(vtab, a.volt_fmt, threadIdx.x, fetch_volt_rec<MP>(vrow_of(t), a.volt_fmt, my_ant));
    }
    for (int i = threadIdx.x + kThreads; i < bcnt; i += kThreads)
      put_volt_rec<MP>(vtab, a.volt_fmt, i, fetch_volt_rec<MP>(vrow_of(t), a.volt_fmt, blist[i]));
    {
      float4 *g4 = reinterpret_cast<float4 *>(grid);
      for (int i = threadIdx.x; i < MP * MHB * MTS / 2; i += kThreads) g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    for (int g = 0; g < gc; g += GCH) {
      uint32_t m[GCH];
      float2 w[GCH][MP];
#pragma unroll
      for (int k = 0; k < GCH; ++k) {
        const bool ok = g + k < gc;
        m[k] = ok ? a.meta[(g0 + g + k) * 64 + lane] : 0u;
#pragma unroll
        for (int p = 0; p < MP; ++p) w[k][p] = make_float2(0.f, 0.f);
        if (ok) load_taps<MP>(a.wk + ((g0 + g + k) * 64 + lane) * MP, w[k]);
      }
      float2 e[GCH][MP];
      load_volts<MP, GCH>(vtab, a.volt_fmt, m, e);
#pragma unroll
      for (int k = 0; k < GCH; ++k) {
        if (g + k < gc) {
          // the cell is an element offset in the FP32 band layout (row stride row_stride(256))
          const int cell = (int)(m[k] & 0xFFFFu);
          const int rr = cell / row_stride(MN), col = cell - rr * row_stride(MN);
#pragma unroll
          for (int p = 0; p < MP; ++p) {
            float2 *cp = grid + (p * MHB + rr) * MTS + col;
            const float2 cur = *cp;
            const float2 wv = w[k][p], ev = e[k][p];
            *cp = make_float2(cur.x + wv.x * ev.x - wv.y * ev.y, cur.y + wv.x * ev.y + wv.y * ev.x);
          }
        }
      }
    }
    __syncthreads();
    if (pre8 && t + 1 < t_hi) nxt = fetch_volt_rec<MP>(vrow_of(t + 1), 0, my_ant).x;
    __builtin_amdgcn_s_setprio(0);
    // 16 row transforms (pol p, band row r) = transform p * 8 + r; outputs back into the grid (its reads
    // finished at the barrier inside the FFT)
    fft256x16_mfma<BF16>(grid, MTS, ys, mats,
                         [&](int tt, int q, float2 v, int, int) { grid[tt * MTS + q] = v; });
    // the next sample's records go to the table (this sample's scatter is over) before the stores are issued, so
    // the wait for their loads does not also wait for the stores
    if (pre8 && t + 1 < t_hi) put_volt_rec<MP>(vtab, 0, threadIdx.x, make_uint4(nxt, 0u, 0u, 0u));
    __syncthreads();
    // touched rows to the column-group tiles of H: [p][q / W][row][q % W], 8 rows x 8 columns contiguous
    float2 *hb = a.io + ((int64_t)(c - a.c0) * a.t_block + (t - a.t0)) * MP * MN * MN;
    for (int i = threadIdx.x; i < MP * nrow * MN; i += kThreads) {
      const int qw = i % MW;
      const int r = (i / MW) % nrow;
      const int rest = i / (MW * nrow);
      const int qg = rest % (MN / MW), p = rest / (MN / MW);
      const int row = r_lo + r;
      store_stream(hb + (int64_t)p * MN * MN + (int64_t)qg * (MN * MW) + row * MW + qw,
                   grid[(p * MHB + (row - row0)) * MTS + qg * MW + qw]);
    }
    __syncthreads();
  }
}

// Two waves per SIMD: unbounded, the BF16 form took 248 VGPRs + 16 AGPRs and ran one wave per SIMD; under the
// bound it fits 246 VGPRs without spilling.
template <bool BF16, int ACC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_cols_mfma(ColArgs a, const uint16_t *table) {
  extern __shared__ float4 smem4[];
  float2 *xs = reinterpret_cast<float2 *>(smem4);          // [16][MTS]: transform p * 8 + col
  float *ys = reinterpret_cast<float *>(xs + 16 * MTS);

  int c, cg;
  if (!cols_xcd_map(a, MN / MW, c, cg)) return;
  const int col0 = cg * MW;
  const int jmin = a.chans[c].jmin, jmax = a.chans[c].jmax;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tt = lane & 15, g = lane >> 4;
  const int p = tt >> 3, col = tt & 7;
  MfmaMats<BF16> mats;
  mats.load(table, lane, wave);

  float acc[4][4][2];
#pragma unroll
  for (int jj = 0; jj < 4; ++jj)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[jj][i][0] = acc[jj][i][1] = 0.f;

  // the sample's tile (2 pols x 256 rows x 8 columns), 16 values per thread, loaded one sample ahead so the
  // loads are in flight during the previous sample's transforms
  constexpr int PER = MP * MN * MW / kThreads;
  float2 nx[PER];
  auto load_tile = [&](int t) {
    const float2 *src = a.in + ((int64_t)(c - a.c0) * a.t_block + (t - a.t0)) * MP * MN * MN + (int64_t)cg * (MN * MW);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + k * kThreads;
      const int pp = i / (MN * MW), rem = i - pp * (MN * MW);
      const int row = rem / MW;
      nx[k] = (row >= jmin && row <= jmax) ? load_stream(src + (int64_t)pp * MN * MN + rem) : make_float2(0.f, 0.f);
    }
  };
  if (a.nt > 0) load_tile(a.t0);
  for (int t = a.t0; t < a.t0 + a.nt; ++t) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + k * kThreads;
      const int pp = i / (MN * MW), rem = i - pp * (MN * MW);
      const int row = rem / MW, cc = rem - row * MW;
      xs[(pp * MW + cc) * MTS + row] = nx[k];
    }
    __syncthreads();
    if (t + 1 < a.t0 + a.nt) load_tile(t + 1);
    fft256x16_mfma<BF16>(xs, MTS, ys, mats, [&](int, int, float2 v, int jj, int i) {
      // lanes t and t ^ 8 hold the two pols of one pixel; the X lane takes Re(X conj Y) = Re(o conj(v)), the Y
      // lane Im(X conj Y) = Re(o conj(i v))
      const float2 o = make_float2(__shfl_xor(v.x, 8), __shfl_xor(v.y, 8));
      const float2 u = p == 0 ? v : make_float2(-v.y, v.x);
      acc[jj][i][0] = fmaf(v.y, v.y, fmaf(v.x, v.x, acc[jj][i][0]));
      acc[jj][i][1] = fmaf(o.y, u.y, fmaf(o.x, u.x, acc[jj][i][1]));
    });
  }

  const int64_t base = (int64_t)4 * a.chans[c].pix_off;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = 4 * wave + jj + 16 * (4 * g + i);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int prod = k == 0 ? p : 2 + p;
        const int64_t idx = base + (int64_t)prod * MN * MN + (int64_t)col0 * MN + q * MW + col;
        if constexpr (ACC == 0) {
          reinterpret_cast<float *>(a.acc)[idx] += acc[jj][i][k];
        } else {
          double2 *o = reinterpret_cast<double2 *>(a.acc);
          double2 sc = o[idx];
          const double xv = (double)acc[jj][i][k];
          const double ts = sc.x + xv;
          if (fabs(sc.x) >= fabs(xv))
            sc.y += (sc.x - ts) + xv;
          else
            sc.y += (xv - ts) + sc.x;
          sc.x = ts;
          o[idx] = sc;
        }
      }
    }
}

size_t rows_mfma_lds_bytes(int band_ants, int volt_fmt) {
  return (size_t)MP * MHB * MTS * 8 + (size_t)2 * 16 * kYStride * 4 + volt_table_bytes(band_ants, MP, volt_fmt);
}
size_t cols_mfma_lds_bytes() { return (size_t)16 * MTS * 8 + (size_t)2 * 16 * kYStride * 4; }

hipError_t launch_mfma_table(uint16_t *tab, int bf16, hipStream_t st) {
  hipLaunchKernelGGL(k_mfma_table, dim3((unsigned)((kMfmaTableHalfs + 255) / 256)), dim3(256), 0, st, tab, bf16);
  return hipGetLastError();
}

hipError_t launch_rows_mfma(int bf16, const RowArgs &a, const uint16_t *table, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  void (*fn)(RowArgs, const uint16_t *) = bf16 ? k_rows_mfma<true> : k_rows_mfma<false>;
  hipError_t e = set_lds_limit_ext((const void *)fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), rows_mfma_lds_bytes(a.band_ants_max, a.volt_fmt), st, a, table);
  return hipGetLastError();
}

hipError_t launch_cols_mfma(int bf16, int accm, const ColArgs &a, const uint16_t *table, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  void (*fn)(ColArgs, const uint16_t *) =
      bf16 ? (accm == 0 ? k_cols_mfma<true, 0> : k_cols_mfma<true, 1>)
           : (accm == 0 ? k_cols_mfma<false, 0> : k_cols_mfma<false, 1>);
  hipError_t e = set_lds_limit_ext((const void *)fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), cols_mfma_lds_bytes(), st, a, table);
  return hipGetLastError();
}

}  // namespace moff
