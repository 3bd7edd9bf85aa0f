// HIP kernels of the MOFF hot path for CDNA4 (gfx950), plain FP32 form.
//
// Eq. m6 per channel c and sample t:  grid (step 2) -> 2-D FFT (step 3) -> |.|^2 products summed over t.
//
// Fused path, per launch block (channels of one grid size x a block of samples):
//   k_rows<FUSED>: one workgroup per (row band, time group).  The band's row range of the channel's grid is
//     built in LDS from the int8 voltages (the channel's voltage row is staged in LDS with coalesced loads)
//     by a deterministic scatter: wavefront w owns the band rows r with (r - row0) % 4 == w and processes the
//     plan's tap groups, 64 taps on 64 distinct cells per instruction, so the sums need no atomics and their
//     order is fixed.  The rows are then transformed (Stockham radix stages, butterflies in registers, LDS
//     exchanges) and written to the block's row-transform buffer H.  Rows no footprint touches are skipped.
//   k_cols<FUSED>: one workgroup per (channel, group of W columns) for all samples of the block: column FFTs
//     (first stage straight from H, reading only rows some footprint touched), then XX, YY, XY products in
//     registers, summed over the block in FP32 and added once to the accumulator (FP32 or FP64 sum + carry).
//   The exchange between the two passes is the row-d inter-module traffic of Fig. 1: a 2-D FFT of a grid larger
//   than one CU's LDS needs one all-to-all, and here it goes through L2/MALL/HBM between two kernels.
// Staged path: k_grid (gridding only), k_rows<ROWFFT> + k_cols<COLFFT> (in-place 2-D FFT), k_acc_staged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <set>
#include <utility>

#include "fft_radix.h"
#include "fft_sizes.h"
#include "kernels.h"

namespace moff {

// ------------------------------------------------------------------------------------------------------------
// Utility kernels
// ------------------------------------------------------------------------------------------------------------

// Twiddle tables of one transform length, generated in FP64 from exact rational angles and rounded once.
// Stage s > 0 (radix R, span L) multiplies input m of butterfly j by w_{L R}^{(j mod L) m}; its table is laid out
// [m][k] (k = j mod L) so that lanes with consecutive k read consecutive LDS words.  Table of the second stage
// (R1 x L1 = R0 R1 entries) first, then that of the third stage (R2 x L2 = n entries) if there is one.
__global__ void k_twiddle_f64(float2 *tw, int n, int r0, int r1, int r2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int s1 = r0 * r1;
  const int total = s1 + (r2 > 1 ? n : 0);
  if (e >= total) return;
  int span, k, m;
  if (e < s1) {
    span = s1;
    m = e / r0;
    k = e - m * r0;
  } else {
    span = n;
    m = (e - s1) / s1;
    k = (e - s1) - m * s1;
  }
  const long long km = (long long)k * m % span;   // exact angle reduction in integers
  double s, c;
  sincospi(2.0 * (double)km / (double)span, &s, &c);
  tw[e] = make_float2((float)c, (float)s);
}

// Packs the caller's kernels into tap-group order wk[g][lane][plane] (a lane's planes are contiguous: one 16-byte
// load for two planes): diagonal kernels [C][A][P][K*K] give P
// planes, Jones kernels [C][A][2][2][K*K] give planes 2 p + q.  Each is multiplied by the phase-centre phase of
// the voltage it multiplies, phase[c][a][q], when one is given (W (phi E) = (W phi) E).
__global__ void k_pack_kernels(const float2 *__restrict__ kern, const float2 *__restrict__ phase,
                               const int32_t *__restrict__ kidx, const int32_t *__restrict__ grp_chan,
                               float2 *__restrict__ wk, int64_t n_groups, int A, int P, int KK, int planes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over groups x 64 lanes
  if (i >= n_groups * 64) return;
  const int64_t g = i >> 6;
  const int lane = (int)(i & 63);
  const int32_t k = kidx[i];
  const int c = grp_chan[g];
  for (int pl = 0; pl < planes; ++pl) {
    float2 v = make_float2(0.f, 0.f);
    if (k >= 0) {
      const int a = k / KK, tap = k - a * KK;
      const int q = planes == 4 ? (pl & 1) : pl;   // pol of the voltage this plane multiplies
      v = kern[(((int64_t)c * A + a) * planes + pl) * KK + tap];
      if (phase) v = cmul(v, phase[((int64_t)c * A + a) * P + q]);
    }
    wk[(g * 64 + lane) * planes + pl] = v;
  }
}

__global__ void k_fill_zero(float4 *p, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// One sample's voltages [C][A][P] -> float (re, im), exactly (int8 values are exact in FP32).
__global__ void k_unpack_debug(const void *volt, int fmt, float2 *out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (fmt == 0) {
    const char2 v = ((const char2 *)volt)[i];
    out[i] = make_float2((float)v.x, (float)v.y);
  } else {
    out[i] = ((const float2 *)volt)[i];
  }
}

// ------------------------------------------------------------------------------------------------------------
// Stockham stage helpers.  A stage of radix R with span L (product of the earlier radices) on an N-point
// transform has NB = N/R butterflies; butterfly j reads x[j + m NB] (natural Stockham index), multiplies input m
// by w_{L R}^{(j mod L) m}, applies the radix-R DFT and produces outputs at natural index
// (j / L) L R + (j mod L) + r L.  Between stages the outputs live in LDS in a padded [r][j] layout (row stride
// NB + 1) so that both the writes (consecutive j) and the next stage's reads avoid bank conflicts.
// ------------------------------------------------------------------------------------------------------------
// tw: the twiddle tables of the transform length (see k_twiddle_f64); stage with span L uses the table at
// offset 0 when L is the first radix and at offset R0 R1 otherwise.
template <int N, int R, int L>
__device__ __forceinline__ void twiddle_dft(float2 (&x)[R], int j, const float2 *__restrict__ tw) {
  if constexpr (L > 1) {
    const int k = j % L;
    constexpr int OFF = L == Fac<N>::R0 ? 0 : Fac<N>::R0 * Fac<N>::R1;
#pragma unroll
    for (int m = 1; m < R; ++m) x[m] = cmul(x[m], tw[OFF + m * L + k]);
  }
  dft<R>(x);
}

// LDS address of natural Stockham index q in the padded layout written by a stage (RP, LP); RP = 0: natural.
template <int N, int RP, int LP>
__device__ __forceinline__ int lds_addr(int q) {
  if constexpr (RP == 0) {
    return q;
  } else {
    constexpr int NBP = N / RP;
    const int k = q % LP;
    const int r = (q / LP) % RP;
    const int j = (q / (LP * RP)) * LP + k;
    return r * (NBP + 1) + j;
  }
}

template <int N, int R>
__device__ __forceinline__ int pad_addr(int j, int r) {
  return r * (N / R + 1) + j;
}

template <int N, int R, int L>
__device__ __forceinline__ int nat_out(int j, int r) {
  return (j / L) * (L * R) + (j % L) + r * L;
}

template <int N> struct Pipe {
  using F = Fac<N>;
  static constexpr int S = F::S;
  static constexpr int R0 = F::R0, R1 = F::R1, R2 = F::R2;
  static constexpr int L1 = R0, L2 = R0 * R1;
  static constexpr int RLAST = S == 2 ? R1 : R2;
  static constexpr int LLAST = S == 2 ? L1 : L2;
  static constexpr int RMAX = (R0 > R1 ? (R0 > R2 ? R0 : R2) : (R1 > R2 ? R1 : R2));
  static constexpr int TS = N + RMAX + 1;   // LDS stride of one transform (odd: spreads banks across transforms)
};

// ------------------------------------------------------------------------------------------------------------
// Row pass
// ------------------------------------------------------------------------------------------------------------
enum RowMode { ROW_FUSED = 0, ROW_GRID = 1, ROW_FFT = 2 };

// In-LDS stage over the band's transforms (rows).  Transform tr (0..ntr) lives at buf + tr_base(tr).
template <int N, int R, int L, int RP, int LP, int MAXB, class Base>
__device__ __forceinline__ void row_stage_lds(float2 *buf, int ntr, const float2 *tw, Base tr_base) {
  constexpr int NB = N / R;
  float2 x[MAXB][R];
  const int total = ntr * NB;
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int b = threadIdx.x + s * kThreads;
    if (b < total) {
      const int tr = b / NB, j = b - tr * NB;
      const float2 *in = buf + tr_base(tr);
#pragma unroll
      for (int m = 0; m < R; ++m) x[s][m] = in[lds_addr<N, RP, LP>(j + m * NB)];
      twiddle_dft<N, R, L>(x[s], j, tw);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int b = threadIdx.x + s * kThreads;
    if (b < total) {
      const int tr = b / NB, j = b - tr * NB;
      float2 *out = buf + tr_base(tr);
#pragma unroll
      for (int r = 0; r < R; ++r) out[pad_addr<N, R>(j, r)] = x[s][r];
    }
  }
  __syncthreads();
}

// Last stage: LDS -> global; dst(tr, q, value) stores output q of transform tr.
template <int N, int R, int L, int RP, int LP, int MAXB, class Base, class Dst>
__device__ __forceinline__ void row_stage_out(const float2 *buf, int ntr, const float2 *tw, Base tr_base, Dst dst) {
  constexpr int NB = N / R;
  const int total = ntr * NB;
#pragma unroll
  for (int s = 0; s < MAXB; ++s) {
    const int b = threadIdx.x + s * kThreads;
    if (b < total) {
      const int tr = b / NB, j = b - tr * NB;
      const float2 *in = buf + tr_base(tr);
      float2 x[R];
#pragma unroll
      for (int m = 0; m < R; ++m) x[m] = in[lds_addr<N, RP, LP>(j + m * NB)];
      twiddle_dft<N, R, L>(x, j, tw);
#pragma unroll
      for (int r = 0; r < R; ++r) dst(tr, nat_out<N, R, L>(j, r), x[r]);
    }
  }
}

template <int N, int P, int MODE, bool KJ, class Out>
__device__ __forceinline__ void row_band(const RowArgs &a, int band, int t_lo, int t_hi, float2 *grid,
                                         const float2 *tws, char *vtab, Out out) {
  static_assert(!KJ || P == 2, "Jones kernels need two pols");
  constexpr int PL = KJ ? 4 : P;                      // packed kernel planes
  using PP = Pipe<N>;
  constexpr int TS = row_stride(N);   // even: rows start on 16-byte boundaries
  static_assert(TS >= N + PP::RMAX - 1, "row stride too small for the padded layout");
  constexpr int HB = band_rows_ce(N, P);             // rows per band
  // tap groups whose loads are issued together; for power-of-two n the first batch's loads are issued before the
  // band-grid clear, so that the clear and its barrier hide their latency (mixed-radix n lack the registers)
  constexpr int GCH = 4;
  constexpr bool EARLY = (N & (N - 1)) == 0;

  const Band *bp = a.bands + band;
  struct {
    int chan, row0, r_lo, r_hi;
  } bd = {bp->chan, bp->row0, bp->r_lo, bp->r_hi};
  const int c = bd.chan;
  const int nrow = bd.r_hi - bd.r_lo + 1;
  const int ntr = P * nrow;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g0 = bp->grp_off[wave];
  const int gc = bp->grp_cnt[wave];
  const size_t vbytes = (size_t)a.n_ant * P * (a.volt_fmt == 0 ? 2 : 8);   // one (t, c) voltage row

  // transform tr = p * nrow + r (pol p, touched row r); P <= 2, so no division
  auto tr_pol = [&](int tr) { return (P == 2 && tr >= nrow) ? 1 : 0; };
  auto tr_base = [&](int tr) {
    const int p = tr_pol(tr), r = tr - p * nrow;
    return (p * HB + (bd.r_lo - bd.row0 + r)) * TS;
  };

  // one tap: grid cell m gets w * e (pol by pol; Jones: both pols into each grid); the cell is the element offset
  // in a pol's band grid (row * TS + column)
  auto scatter_tap = [&](uint32_t m, const float2 (&w)[PL], const float2 (&e)[P]) {
    const int cell = (int)(m & 0xFFFFu);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      float2 *cellp = grid + p * HB * TS + cell;
      float2 cur = *cellp;
      if constexpr (KJ) {
        // grid p receives both pols: K_{p0} E_0 + K_{p1} E_1
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float2 wv = w[2 * p + q], ev = e[q];
          cur = make_float2(cur.x + wv.x * ev.x - wv.y * ev.y, cur.y + wv.x * ev.y + wv.y * ev.x);
        }
      } else {
        const float2 wv = w[p], ev = e[p];
        cur = make_float2(cur.x + wv.x * ev.x - wv.y * ev.y, cur.y + wv.x * ev.y + wv.y * ev.x);
      }
      *cellp = cur;
    }
  };

  // voltages: thread i copies the record of the i-th antenna of the band's list (ascending) into the LDS table
  // vtab before each sample's scatter, so the scatter reads its voltages from LDS (coalesced global loads instead
  // of per-tap gathers).  int8 records (one register) are loaded for the next sample right after this sample's
  // scatter and written to the table after the next sample's clear; float records are copied when they are
  // staged.
  constexpr bool SCAT = MODE == ROW_FUSED || MODE == ROW_GRID;
  constexpr bool STAGE = SCAT && row_stages_volts(N);
  const int bcnt = STAGE ? bp->ant_cnt : 0;
  const int32_t *blist = a.band_ant + bp->ant_off;
  const int my_ant = (STAGE && (int)threadIdx.x < bcnt) ? blist[threadIdx.x] : -1;
  auto vrow_of = [&](int t) {
    return reinterpret_cast<const char *>(a.volt) + ((int64_t)t * a.n_chan + c) * vbytes;
  };
  const bool pre8 = a.volt_fmt == 0 && my_ant >= 0;
  uint32_t nxt = 0u;
  if (pre8 && t_lo < t_hi) nxt = fetch_volt_rec<P>(vrow_of(t_lo), 0, my_ant).x;

  // one batch of tap groups: metadata and packed kernels (global loads)
  auto load_batch = [&](int g, uint32_t (&m)[GCH], float2 (&w)[GCH][PL]) {
#pragma unroll
    for (int k = 0; k < GCH; ++k) {
      const bool ok = g + k < gc;   // uniform: groups past the wave's last are not scattered
      m[k] = ok ? a.meta[(g0 + g + k) * 64 + lane] : 0u;
#pragma unroll
      for (int p = 0; p < PL; ++p) w[k][p] = make_float2(0.f, 0.f);
      if (ok) load_taps<PL>(a.wk + ((g0 + g + k) * 64 + lane) * PL, w[k]);
    }
  };

  for (int t = t_lo; t < t_hi; ++t) {
    if constexpr (SCAT) {
      // wave priority 1 from the tap-group loads to the end of the scatter, 0 for the transforms and stores: a
      // workgroup in its load phase issues ahead of one in its arithmetic phase on the same CU
      __builtin_amdgcn_s_setprio(1);
      // the int8 record loaded after the previous sample's scatter: waiting for it also waits for that sample's
      // stores (vector memory operations complete in order), as the scatter's loads would
      uint32_t m0[GCH];
      float2 w0[GCH][PL];
      if constexpr (EARLY) {
        if (pre8) put_volt_rec<P>(vtab, 0, threadIdx.x, make_uint4(nxt, 0u, 0u, 0u));
        load_batch(0, m0, w0);
      }
      // clear the band grid (16-byte stores over the whole contiguous region, unrolled: no loop between the
      // previous sample's stores and the record write below)
      {
        float4 *g4 = reinterpret_cast<float4 *>(grid);
        constexpr int NCLR = P * HB * TS / 2;
#pragma unroll
        for (int k = 0; k < (NCLR + kThreads - 1) / kThreads; ++k) {
          const int i = threadIdx.x + k * kThreads;
          if (NCLR % kThreads == 0 || i < NCLR) g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      if constexpr (!EARLY)
        if (pre8) put_volt_rec<P>(vtab, 0, threadIdx.x, make_uint4(nxt, 0u, 0u, 0u));
      if (!pre8 && my_ant >= 0)
        put_volt_rec<P>(vtab, a.volt_fmt, threadIdx.x, fetch_volt_rec<P>(vrow_of(t), a.volt_fmt, my_ant));
      for (int i = threadIdx.x + kThreads; i < bcnt; i += kThreads)
        put_volt_rec<P>(vtab, a.volt_fmt, i, fetch_volt_rec<P>(vrow_of(t), a.volt_fmt, blist[i]));
      __syncthreads();
      // deterministic scatter: this wavefront's tap groups, one tap per lane, 64 distinct cells per group;
      // the loads of GCH groups are issued before any of them is used
      {
        auto scatter_batch = [&](int g, const uint32_t (&m)[GCH], const float2 (&w)[GCH][PL]) {
          // voltages of the GCH groups' taps from the LDS table or the voltage row (the loads are branch-free, so
          // all GCH are in flight together; an empty lane reads antenna 0 and adds it with zero weights)
          float2 e[GCH][P];
          if constexpr (STAGE)
            load_volts<P, GCH>(vtab, a.volt_fmt, m, e);
          else
            load_volts<P, GCH>(vrow_of(t), a.volt_fmt, m, e);
#pragma unroll
          for (int k = 0; k < GCH; ++k)
            if (g + k < gc) scatter_tap(m[k], w[k], e[k]);
        };
        int g = 0;
        if constexpr (EARLY) {
          if (gc > 0) scatter_batch(0, m0, w0);
          g = GCH;
        }
        for (; g < gc; g += GCH) {
          uint32_t m[GCH];
          float2 w[GCH][PL];
          load_batch(g, m, w);
          scatter_batch(g, m, w);
        }
      }
      __syncthreads();
      if (pre8 && t + 1 < t_hi) nxt = fetch_volt_rec<P>(vrow_of(t + 1), 0, my_ant).x;
      __builtin_amdgcn_s_setprio(0);
    } else {
      // ROW_FFT: load the band's touched rows from the staged grid
      for (int i = threadIdx.x; i < ntr * N; i += kThreads) {
        const int tr = i / N, col = i - tr * N;
        const int p = tr_pol(tr), r = tr - p * nrow;
        grid[tr_base(tr) + col] =
            a.io[(int64_t)t * a.sample_stride + (int64_t)P * a.chans[c].pix_off + (int64_t)p * N * N +
                 (int64_t)(bd.r_lo + r) * N + col];
      }
      __syncthreads();
    }

    if constexpr (MODE == ROW_GRID) {
      // write the band's touched rows to the staged grid (the rest of the grid was cleared beforehand)
      for (int i = threadIdx.x; i < ntr * N; i += kThreads) {
        const int tr = i / N, col = i - tr * N;
        const int p = tr_pol(tr), r = tr - p * nrow;
        a.io[(int64_t)t * a.sample_stride + (int64_t)P * a.chans[c].pix_off + (int64_t)p * N * N +
             (int64_t)(bd.r_lo + r) * N + col] = grid[tr_base(tr) + col];
      }
      __syncthreads();
    } else {
      // row FFTs of the touched rows
      constexpr int MB0 = (P * HB * (N / PP::R0) + kThreads - 1) / kThreads;
      // staged: natural row-major grid
      auto dst = [&](int tr, int q, float2 v) {
        const int p = tr_pol(tr), row = bd.r_lo + tr - p * nrow;
        if constexpr (MODE == ROW_FUSED) {
          out(c, t, p, row, q, v);
        } else {
          a.io[(int64_t)t * a.sample_stride + (int64_t)P * a.chans[c].pix_off + (int64_t)p * N * N +
               (int64_t)row * N + q] = v;
        }
      };
      if constexpr (PP::S == 2) {
        constexpr int MB1 = (P * HB * (N / PP::R1) + kThreads - 1) / kThreads;
        row_stage_lds<N, PP::R0, 1, 0, 1, MB0>(grid, ntr, tws, tr_base);
        row_stage_out<N, PP::R1, PP::L1, PP::R0, 1, MB1>(grid, ntr, tws, tr_base, dst);
      } else {
        constexpr int MB1 = (P * HB * (N / PP::R1) + kThreads - 1) / kThreads;
        constexpr int MB2 = (P * HB * (N / PP::R2) + kThreads - 1) / kThreads;
        row_stage_lds<N, PP::R0, 1, 0, 1, MB0>(grid, ntr, tws, tr_base);
        row_stage_lds<N, PP::R1, PP::L1, PP::R0, 1, MB1>(grid, ntr, tws, tr_base);
        row_stage_out<N, PP::R2, PP::L2, PP::R1, PP::L1, MB2>(grid, ntr, tws, tr_base, dst);
      }
      __syncthreads();
    }
  }
}

// Fused / staged row pass: one workgroup per (row band, group of t_group samples).  Fused output goes to the
// launch block's H in column-group tiles [p][q / W][row][q % W], so that each column-pass workgroup reads one
// contiguous tile.
template <int N, int P, int MODE, bool KJ>
__global__ __launch_bounds__(kThreads) void k_rows(RowArgs a) {
  constexpr int TS = row_stride(N);
  constexpr int HB = band_rows_ce(N, P);
  extern __shared__ float4 smem4[];
  float2 *grid = reinterpret_cast<float2 *>(smem4);  // [P][HB][TS]
  float2 *tws = grid + P * HB * TS;                  // [2N] twiddle tables
  char *vtab = reinterpret_cast<char *>(tws + 2 * N); // band voltage table (volt_table_bytes)

  int band, tg;
  if constexpr (MODE == ROW_FUSED) {
    if (!rows_xcd_map(a, band, tg)) return;
  } else {
    band = a.band_begin + (int)(blockIdx.x % a.n_bands);
    tg = (int)(blockIdx.x / a.n_bands);
  }
  for (int i = threadIdx.x; i < 2 * N; i += kThreads) tws[i] = a.tw[i];
  const int t_lo = a.t0 + tg * a.t_group;
  const int t_hi = min(a.t0 + a.nt, t_lo + a.t_group);
  row_band<N, P, MODE, KJ>(a, band, t_lo, t_hi, grid, tws, vtab, [&](int c, int t, int p, int row, int q, float2 v) {
    constexpr int W = cols_ce(N);
    store_stream(a.io + (((int64_t)(c - a.c0) * a.t_block + (t - a.t0)) * P + p) * N * N +
                     (int64_t)(q / W) * (N * W) + row * W + (q % W),
                 v);
  });
}

// ------------------------------------------------------------------------------------------------------------
// Column pass
// ------------------------------------------------------------------------------------------------------------
enum ColMode { COL_FUSED = 0, COL_FFT = 1 };

// Swaps the values of adjacent lanes (quad permutation [1,0,3,2]).
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// One column group (W columns of channel c) for samples [t_begin, t_end): column FFTs (first stage straight
// from global memory, only rows some footprint touched), then (FUSED) XX, YY, XY products summed in registers
// and added once to the accumulator, or (FFT) the transformed columns written back to the staged grid.
// src(t): the sample's row-transformed data (FUSED: column-group tiles [p][q / W][row][q % W]; FFT: the staged
// grid).  pre(t) runs (uniformly) before the loads of sample t are issued, post(t) once every thread has
// consumed them.  LD: plain, non-temporal or device-coherent loads.  buf: LDS [P][W][Pipe<N>::TS]; tws: twiddle tables in LDS.
template <int N, int P, int W, int MODE, int ACC, int LD, bool PREFETCH, class Src, class Pre, class Post>
__device__ __forceinline__ void col_group(const ColArgs &a, int c, int cg, int t_begin, int t_end, float2 *buf,
                                          const float2 *tws, Src src, Pre pre, Post post) {
  using PP = Pipe<N>;
  constexpr int TS = PP::TS;
  constexpr int R0 = PP::R0, NB0 = N / R0;
  constexpr int RL = PP::RLAST, LL = PP::LLAST, NBL = N / RL;
  constexpr int NS1 = P * W * NB0;                    // first-stage butterflies per sample
  constexpr int MB0 = (NS1 + kThreads - 1) / kThreads;
  constexpr int NSL = P * W * NBL;                    // last-stage butterflies (one pol each)
  constexpr int MBL = (NSL + kThreads - 1) / kThreads;
  constexpr int PA = P == 2 ? 2 : 1;                  // accumulator reals per pixel and lane

  const int col0 = cg * W;
  const int jmin = a.full_rows ? 0 : a.chans[c].jmin, jmax = a.full_rows ? N - 1 : a.chans[c].jmax;
  const int64_t pstride = (int64_t)N * N;

  float acc[MBL][RL][PA];
#pragma unroll
  for (int s = 0; s < MBL; ++s)
#pragma unroll
    for (int r = 0; r < RL; ++r)
#pragma unroll
      for (int k = 0; k < PA; ++k) acc[s][r][k] = 0.f;

  // first-stage inputs of one sample, straight from global (rows outside [jmin, jmax] are zero)
  float2 xs[MB0][R0];
  auto load_first = [&](int t) {
    const float2 *sp = src(t);
#pragma unroll
    for (int s = 0; s < MB0; ++s) {
      const int b = threadIdx.x + s * kThreads;
      const int col = b % W, p = (b / W) % P, j = b / (W * P);
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int row = j + m * NB0;
        const int64_t off = MODE == COL_FUSED ? (int64_t)col0 * N + row * W + col : (int64_t)row * N + col0 + col;
        const bool ok = b < NS1 && row >= jmin && row <= jmax;
        if constexpr (LD == LD_STREAM)
          xs[s][m] = ok ? load_stream(sp + p * pstride + off) : make_float2(0.f, 0.f);
        else if constexpr (LD == LD_COHERENT)
          xs[s][m] = ok ? load_coherent(sp + p * pstride + off) : make_float2(0.f, 0.f);
        else
          xs[s][m] = ok ? sp[p * pstride + off] : make_float2(0.f, 0.f);
      }
    }
  };
  if (PREFETCH && t_begin < t_end) {
    pre(t_begin);
    load_first(t_begin);
  }

  for (int t = t_begin; t < t_end; ++t) {
    if constexpr (!PREFETCH) {
      pre(t);
      load_first(t);
    }
    __syncthreads();   // the previous sample's last stage has finished reading buf
#pragma unroll
    for (int s = 0; s < MB0; ++s) {
      const int b = threadIdx.x + s * kThreads;
      if (b < NS1) {
        const int col = b % W, p = (b / W) % P, j = b / (W * P);
        dft<R0>(xs[s]);
        float2 *o = buf + (p * W + col) * TS;
#pragma unroll
        for (int r = 0; r < R0; ++r) o[pad_addr<N, R0>(j, r)] = xs[s][r];
      }
    }
    __syncthreads();
    post(t);                // every thread has consumed the inputs of sample t
    if (PREFETCH && t + 1 < t_end) {   // in flight during the remaining stages
      pre(t + 1);
      load_first(t + 1);
    }
    if constexpr (PP::S == 3) {
      constexpr int R1 = PP::R1, NB1 = N / R1;
      constexpr int NS2 = P * W * NB1;
      constexpr int MB1 = (NS2 + kThreads - 1) / kThreads;
      float2 x[MB1][R1];
#pragma unroll
      for (int s = 0; s < MB1; ++s) {
        const int b = threadIdx.x + s * kThreads;
        if (b < NS2) {
          const int col = b % W, p = (b / W) % P, j = b / (W * P);
          const float2 *in = buf + (p * W + col) * TS;
#pragma unroll
          for (int m = 0; m < R1; ++m) x[s][m] = in[lds_addr<N, R0, 1>(j + m * NB1)];
          twiddle_dft<N, R1, PP::L1>(x[s], j, tws);
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < MB1; ++s) {
        const int b = threadIdx.x + s * kThreads;
        if (b < NS2) {
          const int col = b % W, p = (b / W) % P, j = b / (W * P);
          float2 *o = buf + (p * W + col) * TS;
#pragma unroll
          for (int r = 0; r < R1; ++r) o[pad_addr<N, R1>(j, r)] = x[s][r];
        }
      }
      __syncthreads();
    }
    // last stage: one (pol, column, butterfly) per lane; adjacent lanes hold the two pols of one pixel set
    constexpr int RPV = PP::S == 2 ? PP::R0 : PP::R1;
    constexpr int LPV = PP::S == 2 ? 1 : PP::L1;
#pragma unroll
    for (int s = 0; s < MBL; ++s) {
      const int b0 = threadIdx.x + s * kThreads;
      const bool valid = NSL % kThreads == 0 || b0 < NSL;   // the first form: every lane holds a butterfly
      const int b = valid ? b0 : 0;
      const int p = P == 2 ? (b & 1) : 0;
      const int rest = P == 2 ? (b >> 1) : b;
      const int col = rest % W, j = rest / W;
      float2 x[RL];
      const float2 *in = buf + (p * W + col) * TS;
#pragma unroll
      for (int m = 0; m < RL; ++m) x[m] = in[lds_addr<N, RPV, LPV>(j + m * NBL)];
      twiddle_dft<N, RL, LL>(x, j, tws);
      if constexpr (MODE == COL_FUSED) {
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const float2 mine = x[r];
          if constexpr (P == 2) {
            // the X lane takes Re(X conj Y) = Re(Y conj X) and the Y lane Im(X conj Y) = Re(X conj(i Y)): both
            // are Re(other conj(u)) with u = mine on the X lane and i mine on the Y lane
            const float2 other = make_float2(swap_pair(mine.x), swap_pair(mine.y));
            const float2 u = p == 0 ? mine : make_float2(-mine.y, mine.x);
            if (valid) {
              acc[s][r][0] = fmaf(mine.y, mine.y, fmaf(mine.x, mine.x, acc[s][r][0]));   // XX or YY
              acc[s][r][1] = fmaf(other.y, u.y, fmaf(other.x, u.x, acc[s][r][1]));      // Re XY or Im XY
            }
          } else {
            if (valid) acc[s][r][0] = fmaf(mine.y, mine.y, fmaf(mine.x, mine.x, acc[s][r][0]));
          }
        }
      } else {
        if (valid) {
          float2 *dst = a.out + (int64_t)t * a.sample_stride + (int64_t)P * a.chans[c].pix_off;
#pragma unroll
          for (int r = 0; r < RL; ++r) {
            const int q = nat_out<N, RL, LL>(j, r);
            dst[p * pstride + (int64_t)q * N + col0 + col] = x[r];
          }
        }
      }
    }
  }

  if constexpr (MODE == COL_FUSED) {
    // add the block's FP32 partial sums to the accumulator, one writer per (pixel, real)
    constexpr int PR = P == 2 ? 4 : 1;
    const int64_t base = (int64_t)PR * a.chans[c].pix_off;
#pragma unroll
    for (int s = 0; s < MBL; ++s) {
      const int b = threadIdx.x + s * kThreads;
      if (b < NSL) {
        const int p = P == 2 ? (b & 1) : 0;
        const int rest = P == 2 ? (b >> 1) : b;
        const int col = rest % W, j = rest / W;
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int q = nat_out<N, RL, LL>(j, r);
#pragma unroll
          for (int k = 0; k < PA; ++k) {
            const int prod = P == 2 ? (k == 0 ? p : 2 + p) : 0;   // XX, YY, Re XY, Im XY
            const int64_t idx = base + (int64_t)prod * pstride + (int64_t)col0 * N + q * W + col;
            if constexpr (ACC == 0) {
              float *o = reinterpret_cast<float *>(a.acc);
              o[idx] += acc[s][r][k];
            } else {
              // Neumaier compensated summation in FP64: (sum, carry)
              double2 *o = reinterpret_cast<double2 *>(a.acc);
              double2 sc = o[idx];
              const double xv = (double)acc[s][r][k];
              const double tsum = sc.x + xv;
              if (fabs(sc.x) >= fabs(xv))
                sc.y += (sc.x - tsum) + xv;
              else
                sc.y += (xv - tsum) + sc.x;
              sc.x = tsum;
              o[idx] = sc;
            }
          }
        }
      }
    }
  }
}

// Fused / staged column pass: one workgroup per (channel, column group), samples split over gridDim.y.
// Fused dual-pol 256-point form with the FP64 (sum, carry) accumulator: the LDS allows 4 workgroups per CU, and
// the 4-wave bound fits it in 128 VGPRs (4 waves per SIMD instead of 3).
template <int N, int P, int W, int MODE, int ACC>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(N == 256 && P == 2 && MODE == 0 && ACC == 1 ? 4 : 2,
                                   N == 256 && P == 2 && MODE == 0 && ACC == 1 ? 4 : 8)))
void k_cols(ColArgs a) {
  extern __shared__ float4 smem4[];
  float2 *buf = reinterpret_cast<float2 *>(smem4);   // [P][W][TS]
  float2 *tws = buf + P * W * Pipe<N>::TS;            // [2N] twiddle tables

  int c, cg;
  if constexpr (MODE == COL_FUSED) {
    if (!cols_xcd_map(a, N / W, c, cg)) return;
  } else {
    c = a.c0 + (int)(blockIdx.x / (N / W));
    cg = (int)(blockIdx.x % (N / W));
  }
  for (int i = threadIdx.x; i < 2 * N; i += kThreads) tws[i] = a.tw[i];
  const int per = (a.nt + (int)gridDim.y - 1) / (int)gridDim.y;
  const int t_begin = a.t0 + (int)blockIdx.y * per;
  const int t_end = min(a.t0 + a.nt, t_begin + per);
  const int64_t pstride = (int64_t)N * N;
  auto src = [&](int t) -> const float2 * {
    if constexpr (MODE == COL_FUSED)
      return a.in + ((int64_t)(c - a.c0) * a.t_block + (t - a.t0)) * P * pstride;
    else
      return a.in + (int64_t)t * a.sample_stride + (int64_t)P * a.chans[c].pix_off;
  };
  // the next sample's first-stage inputs are prefetched for columns of up to 160 points; longer columns need the
  // registers for occupancy (at 192 the prefetch costs a wave per SIMD, at 256 it gains nothing)
  col_group<N, P, W, MODE, ACC, LD_STREAM, (N <= 160)>(a, c, cg, t_begin, t_end, buf, tws, src, [](int) {}, [](int) {});
}

// ------------------------------------------------------------------------------------------------------------
// Streaming form of the fused path: one persistent launch per grid size.
//
// Teams are the workgroups that share one XCD: at start every workgroup reads the XCD it runs on (hardware
// XCC_ID), takes the next rank on that XCD (a device-scope counter) and waits until every workgroup of the launch
// has registered.  Team x processes channels c0 + x + 8 k, their samples in order.  Ranks below G = N / W own one
// column group each (column FFTs, products, accumulator update every t_block samples, exactly as k_cols); the
// others are row workers taking (sample, band) tasks in sample order (exactly k_rows for one sample).
// Row-transformed samples pass through a ring of S slots per team, written and read with device-coherent
// accesses (they bypass the non-coherent caches and meet at the memory side, where the MALL holds the small
// ring).  A team's L2 alone cannot carry it: plain loads may hit lines of an earlier use of the slot left in the
// CU's L1, and no instruction invalidates only the L1 when a workgroup runs on one CU.  Per slot, two cumulative
// device-scope counters: bands produced and column groups consumed.  A row task for sample u waits until every owner has consumed sample u - S; an owner
// waits until every band of its sample has been produced.  Producers make their stores complete (vmcnt 0) before
// the counter increment.  Every wait is bounded: past the spin limit, or once any workgroup has flagged an
// error, it sets the error flag and returns, so the launch always ends (an XCD with fewer than G + 1
// workgroups flags error 2).  The launch needs all its workgroups resident at once: the host sizes it from the
// occupancy.
// ------------------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ctr_load(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole-workgroup bounded wait until *p >= target (thread 0 polls).
__device__ __forceinline__ void wg_wait(const uint32_t *p, uint32_t target, int *err, uint32_t limit) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (ctr_load(p) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spins > limit) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  __syncthreads();
}

// Samples u' in [0, u] with u' mod S == sl.
__device__ __forceinline__ int64_t slot_count(int64_t u, int sl, int S) { return u < sl ? 0 : (u - sl) / S + 1; }

// Bands produced into slot u % S up to and including sequence index u on XCD x (what the owners of u wait for).
__device__ __forceinline__ uint32_t stream_prod_target(const StreamArgs &s, int x, int64_t u) {
  const int S = s.slots, nt = s.r.nt, sl = (int)(u % S);
  int64_t tot = 0;
  for (int k = 0; k <= (int)(u / nt); ++k) {
    const int64_t lo = (int64_t)k * nt, hi = min((int64_t)(k + 1) * nt - 1, u);
    tot += (int64_t)s.r.chans[s.r.c0 + x + kXcds * k].band_count * (slot_count(hi, sl, S) - slot_count(lo - 1, sl, S));
  }
  return (uint32_t)tot;
}

// Owner of column group w of channel c (k-th channel of XCD x): all samples, accumulator update per t_block.
template <int N, int P, int W, int ACC>
__device__ __forceinline__ void stream_owner(const StreamArgs &s, int x, int w, int k, float2 *work, const float2 *tws) {
  const int S = s.slots, nt = s.r.nt, t0 = s.r.t0;
  const int64_t slot_elems = (int64_t)P * N * N;
  const float2 *ring = s.ring + (int64_t)x * S * slot_elems;
  uint32_t *prod = s.ctr + (int64_t)x * 2 * S, *cons = prod + S;
  const int c = s.r.c0 + x + kXcds * k;
  const int64_t ubase = (int64_t)k * nt - t0;   // sequence index of sample t is ubase + t
  auto src = [&](int t) -> const float2 * { return ring + ((ubase + t) % S) * slot_elems; };
  auto pre = [&](int t) {
    const int64_t u = ubase + t;
    wg_wait(prod + u % S, stream_prod_target(s, x, u), s.err, s.spin_limit);
  };
  auto post = [&](int t) {
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(cons + (ubase + t) % S, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  for (int tb = t0; tb < t0 + nt; tb += s.c.t_block)
    col_group<N, P, W, COL_FUSED, ACC, LD_COHERENT, false>(s.c, c, w, tb, min(t0 + nt, tb + s.c.t_block), work, tws, src, pre,
                                              post);
}

// Row worker r of R on the k-th channel of XCD x: tasks (sample, band) r, r + R, ... in sample order.
template <int N, int P, int W, bool KJ>
__device__ __forceinline__ void stream_rows(const StreamArgs &s, int x, int r, int R, int k, float2 *work,
                                         const float2 *tws) {
  constexpr int G = N / W;
  const int S = s.slots, nt = s.r.nt, t0 = s.r.t0;
  const int64_t slot_elems = (int64_t)P * N * N;
  float2 *ring = s.ring + (int64_t)x * S * slot_elems;
  uint32_t *prod = s.ctr + (int64_t)x * 2 * S, *cons = prod + S;
  const int c = s.r.c0 + x + kXcds * k;
  const int nb = s.r.chans[c].band_count, bf = s.r.chans[c].band_first;
  for (int64_t task = r; task < (int64_t)nt * nb; task += R) {
    const int t = (int)(task / nb), b = (int)(task - (int64_t)t * nb);
    const int64_t u = (int64_t)k * nt + t;
    const int sl = (int)(u % S);
    if (u >= S) wg_wait(cons + sl, (uint32_t)(G * slot_count(u - S, sl, S)), s.err, s.spin_limit);
    float2 *dst = ring + sl * slot_elems;
    char *vtab = reinterpret_cast<char *>(work + P * band_rows_ce(N, P) * row_stride(N));   // after the band grid
    row_band<N, P, ROW_FUSED, KJ>(s.r, bf + b, t0 + t, t0 + t + 1, work, tws, vtab,
                                  [&](int, int, int p, int row, int q, float2 v) {
                                    store_coherent(dst + (int64_t)p * N * N + (q / W) * (N * W) + row * W + (q % W), v);
                                  });
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this thread's slot stores are complete
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(prod + sl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int N, int P, int W, int ACC, bool KJ>
__global__ __launch_bounds__(kThreads) void k_stream(StreamArgs s) {
  constexpr int G = N / W;
  extern __shared__ float4 smem4[];
  int *team = reinterpret_cast<int *>(smem4);            // XCD, rank on it, workgroups on it
  float2 *tws = reinterpret_cast<float2 *>(smem4 + 1);   // [2N] twiddle tables
  float2 *work = tws + 2 * N;                            // row band grid or column buffer
  if (threadIdx.x == 0) {
    uint32_t *reg = s.ctr + kStreamRegWord, *arrived = reg + kXcds;
    const int xcc = xcc_id();
    const uint32_t rank = __hip_atomic_fetch_add(reg + xcc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while (ctr_load(arrived) < gridDim.x) {
      if (__hip_atomic_load(s.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spins > s.spin_limit) {
        __hip_atomic_store(s.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    team[0] = xcc;
    team[1] = (int)rank;
    team[2] = (int)ctr_load(reg + xcc);
    if (team[2] <= G) __hip_atomic_store(s.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int i = threadIdx.x; i < 2 * N; i += kThreads) tws[i] = s.r.tw[i];
  __syncthreads();
  const int x = team[0], w = team[1];
  if (__hip_atomic_load(s.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int nch = x < s.n_chan_group ? (s.n_chan_group - x + kXcds - 1) / kXcds : 0;
  const int R = team[2] - G;
  for (int k = 0; k < nch; ++k) {
    if (w < G)
      stream_owner<N, P, W, ACC>(s, x, w, k, work, tws);
    else if (R > 0)
      stream_rows<N, P, W, KJ>(s, x, w - G, R, k, work, tws);
  }
}

// ------------------------------------------------------------------------------------------------------------
// Staged accumulate: E-field images -> products, summed over the n_t samples, added to the accumulator.
// ------------------------------------------------------------------------------------------------------------
template <int P, int ACC>
__global__ void k_acc_staged(AccArgs a) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= a.pix_total) return;
  // channel of this pixel
  int c = 0;
  while (c + 1 < a.n_chan && a.chans[c + 1].pix_off <= pix) ++c;
  const int64_t local = pix - a.chans[c].pix_off;
  const int64_t nn = (int64_t)a.chans[c].n * a.chans[c].n;
  constexpr int PR = P == 2 ? 4 : 1;
  float s[PR];
#pragma unroll
  for (int k = 0; k < PR; ++k) s[k] = 0.f;
  for (int64_t t = 0; t < a.nt; ++t) {
    const float2 *e = a.efield + t * a.sample_stride + (int64_t)P * a.chans[c].pix_off + local;
    const float2 ex = e[0];
    if constexpr (P == 2) {
      const float2 ey = e[nn];
      s[0] += ex.x * ex.x + ex.y * ex.y;
      s[1] += ey.x * ey.x + ey.y * ey.y;
      s[2] += ex.x * ey.x + ex.y * ey.y;
      s[3] += ex.y * ey.x - ex.x * ey.y;
    } else {
      s[0] += ex.x * ex.x + ex.y * ex.y;
    }
  }
#pragma unroll
  for (int k = 0; k < PR; ++k) {
    const int n = a.chans[c].n, W = a.chans[c].cols;
    const int q = (int)(local / n), pc = (int)(local - (int64_t)q * n);
    const int64_t idx = (int64_t)PR * a.chans[c].pix_off + k * nn + (int64_t)(pc / W) * n * W + q * W + pc % W;
    if constexpr (ACC == 0) {
      reinterpret_cast<float *>(a.acc)[idx] += s[k];
    } else {
      double2 *o = reinterpret_cast<double2 *>(a.acc);
      double2 sc = o[idx];
      const double xv = (double)s[k];
      const double tsum = sc.x + xv;
      if (fabs(sc.x) >= fabs(xv))
        sc.y += (sc.x - tsum) + xv;
      else
        sc.y += (xv - tsum) + sc.x;
      sc.x = tsum;
      o[idx] = sc;
    }
  }
}

// ------------------------------------------------------------------------------------------------------------
// Read-out: accumulator (FFT pixel order) -> centred complex64 image, products XX, YY, XY, YX.
// ------------------------------------------------------------------------------------------------------------
template <int P, int ACC>
__global__ void k_read_image(ReadArgs a) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over output pixels of all channels
  if (pix >= a.pix_total) return;
  int c = 0;
  while (c + 1 < a.n_chan && a.chans[c + 1].pix_off <= pix) ++c;
  const int64_t local = pix - a.chans[c].pix_off;
  const int n = a.chans[c].n;
  const int64_t nn = (int64_t)n * n;
  const int q = (int)(local / n), pcol = (int)(local - (int64_t)q * n);
  // output pixel (q, p) <- FFT index ((q - n/2) mod n, (p - n/2) mod n)
  const int kq = (q + n / 2) % n, kp = (pcol + n / 2) % n;
  const int W = a.chans[c].cols;
  const int64_t src = (int64_t)(kp / W) * n * W + (int64_t)kq * W + kp % W;   // tiled accumulator
  constexpr int PR = P == 2 ? 4 : 1;
  const int64_t abase = (int64_t)PR * a.chans[c].pix_off;
  double v[PR];
#pragma unroll
  for (int k = 0; k < PR; ++k) {
    if constexpr (ACC == 0) {
      v[k] = (double)reinterpret_cast<const float *>(a.acc)[abase + k * nn + src];
    } else {
      const double2 sc = reinterpret_cast<const double2 *>(a.acc)[abase + k * nn + src];
      v[k] = sc.x + sc.y;
    }
    v[k] *= a.scale;
  }
  float2 *o = a.img + (int64_t)PR * a.chans[c].pix_off;
  if constexpr (P == 2) {
    o[0 * nn + local] = make_float2((float)v[0], 0.f);
    o[1 * nn + local] = make_float2((float)v[1], 0.f);
    o[2 * nn + local] = make_float2((float)v[2], (float)v[3]);
    o[3 * nn + local] = make_float2((float)v[2], -(float)v[3]);
  } else {
    o[local] = make_float2((float)v[0], 0.f);
  }
}

// ------------------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------------------
size_t rows_lds_bytes(int n, int P, int band_rows, int band_ants, int volt_fmt) {
  if (!fft_radix_max(n)) return 0;
  return (size_t)P * band_rows * row_stride(n) * 8 + (size_t)2 * n * 8 +
         (row_stages_volts(n) ? volt_table_bytes(band_ants, P, volt_fmt) : 0);
}

size_t cols_lds_bytes(int n, int P, int W) {
  int ts = 0;
  switch (n) {
#define TSCASE(NN) \
  case NN: ts = Pipe<NN>::TS; break;
    TSCASE(32) TSCASE(64) TSCASE(96) TSCASE(128) TSCASE(160) TSCASE(192) TSCASE(256) TSCASE(320) TSCASE(384)
    TSCASE(512)
#undef TSCASE
    default: return 0;
  }
  return (size_t)P * W * ts * 8 + (size_t)2 * n * 8;
}

// Raises a kernel's dynamic LDS limit to the CU's 160 KB once per kernel and device.
hipError_t set_lds_limit_ext(const void *fn) {
  static std::mutex mu;
  static std::set<std::pair<const void *, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count({fn, dev})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
  if (e == hipSuccess) done.insert({fn, dev});
  return e;
}

template <int N, int P>
static hipError_t launch_rows_np(int mode, bool jones, const RowArgs &a, int grid, size_t lds, hipStream_t st) {
  void (*fn)(RowArgs) = nullptr;
  if constexpr (P == 2) {
    if (jones) fn = mode == ROW_FUSED ? k_rows<N, P, ROW_FUSED, true> : k_rows<N, P, ROW_GRID, true>;
  }
  if (!fn)
    fn = mode == ROW_FUSED ? k_rows<N, P, ROW_FUSED, false>
                           : mode == ROW_GRID ? k_rows<N, P, ROW_GRID, false> : k_rows<N, P, ROW_FFT, false>;
  hipError_t e = set_lds_limit_ext((const void *)fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_rows(int n, int P, int mode, bool jones, const RowArgs &a, int grid, size_t lds, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  if (jones && (P != 2 || mode == ROW_FFT)) return hipErrorInvalidValue;
#define RCASE(NN)                                                                                \
  case NN:                                                                                       \
    return P == 2 ? launch_rows_np<NN, 2>(mode, jones, a, grid, lds, st)                         \
                  : launch_rows_np<NN, 1>(mode, jones, a, grid, lds, st);
  switch (n) {
    RCASE(32) RCASE(64) RCASE(96) RCASE(128) RCASE(160) RCASE(192) RCASE(256) RCASE(320) RCASE(384) RCASE(512)
    default: return hipErrorInvalidValue;
  }
#undef RCASE
}

template <int N, int P, int W>
static hipError_t launch_cols_npw(int mode, int accm, const ColArgs &a, int grid, int gridy, size_t lds,
                                  hipStream_t st) {
  void (*fn)(ColArgs) = mode == COL_FFT ? k_cols<N, P, W, COL_FFT, 0>
                                        : (accm == 0 ? k_cols<N, P, W, COL_FUSED, 0> : k_cols<N, P, W, COL_FUSED, 1>);
  hipError_t e = set_lds_limit_ext((const void *)fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(grid, gridy), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <int N, int W>
static hipError_t launch_cols_nw(int P, int mode, int accm, const ColArgs &a, int grid, int gridy, size_t lds,
                                 hipStream_t st) {
  return P == 2 ? launch_cols_npw<N, 2, W>(mode, accm, a, grid, gridy, lds, st)
                : launch_cols_npw<N, 1, W>(mode, accm, a, grid, gridy, lds, st);
}

hipError_t launch_cols(int n, int P, int W, int mode, int accm, const ColArgs &a, int grid, int gridy, size_t lds,
                       hipStream_t st) {
  if (grid <= 0 || gridy <= 0) return hipSuccess;
  // (n, W) pairs follow cols_for(n)
  switch (n) {
    case 32: return W == 32 ? launch_cols_nw<32, 32>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 64: return W == 32 ? launch_cols_nw<64, 32>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 96: return W == 16 ? launch_cols_nw<96, 16>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 128: return W == 16 ? launch_cols_nw<128, 16>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 160: return W == 8 ? launch_cols_nw<160, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 192: return W == 8 ? launch_cols_nw<192, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 256: return W == 8 ? launch_cols_nw<256, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 320: return W == 8 ? launch_cols_nw<320, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 384: return W == 8 ? launch_cols_nw<384, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    case 512: return W == 8 ? launch_cols_nw<512, 8>(P, mode, accm, a, grid, gridy, lds, st) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_acc_staged(int P, int accm, const AccArgs &a, hipStream_t st) {
  const int grid = (int)((a.pix_total + 255) / 256);
  if (grid <= 0) return hipSuccess;
  void (*fn)(AccArgs) = P == 2 ? (accm == 0 ? k_acc_staged<2, 0> : k_acc_staged<2, 1>)
                               : (accm == 0 ? k_acc_staged<1, 0> : k_acc_staged<1, 1>);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_read_image(int P, int accm, const ReadArgs &a, hipStream_t st) {
  const int grid = (int)((a.pix_total + 255) / 256);
  if (grid <= 0) return hipSuccess;
  void (*fn)(ReadArgs) = P == 2 ? (accm == 0 ? k_read_image<2, 0> : k_read_image<2, 1>)
                                : (accm == 0 ? k_read_image<1, 0> : k_read_image<1, 1>);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

int fft_radices(int n, int *r0, int *r1, int *r2) {
  switch (n) {
#define FCASE(NN)        \
  case NN:               \
    *r0 = Fac<NN>::R0;   \
    *r1 = Fac<NN>::R1;   \
    *r2 = Fac<NN>::R2;   \
    return Fac<NN>::S;
    FCASE(32) FCASE(64) FCASE(96) FCASE(128) FCASE(160) FCASE(192) FCASE(256) FCASE(320) FCASE(384) FCASE(512)
#undef FCASE
    default: return 0;
  }
}

hipError_t launch_twiddle(float2 *tw, int n, hipStream_t st) {
  int r0, r1, r2;
  if (!fft_radices(n, &r0, &r1, &r2)) return hipErrorInvalidValue;
  const int total = r0 * r1 + (r2 > 1 ? n : 0);
  hipLaunchKernelGGL(k_twiddle_f64, dim3((total + 255) / 256), dim3(256), 0, st, tw, n, r0, r1, r2);
  return hipGetLastError();
}

hipError_t launch_pack_kernels(const float2 *kern, const float2 *phase, const int32_t *kidx, const int32_t *grp_chan,
                               float2 *wk, int64_t n_groups, int A, int P, int KK, int planes, hipStream_t st) {
  const int64_t total = n_groups * 64;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_kernels, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, kern, phase, kidx,
                     grp_chan, wk, n_groups, A, P, KK, planes);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
  const int64_t n4 = (int64_t)(bytes / 16);
  if (n4 == 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n4 + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, (float4 *)p, n4);
  return hipGetLastError();
}

hipError_t launch_unpack_debug(const void *volt, int fmt, float2 *out, int64_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_debug, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, volt, fmt, out,
                     count);
  return hipGetLastError();
}


template <int N, int P, int W>
static void *stream_fn(int accm, bool jones) {
  if constexpr (P == 2) {
    if (jones) return accm == 0 ? (void *)k_stream<N, P, W, 0, true> : (void *)k_stream<N, P, W, 1, true>;
  }
  return accm == 0 ? (void *)k_stream<N, P, W, 0, false> : (void *)k_stream<N, P, W, 1, false>;
}

static void *stream_kernel(int n, int P, int accm, bool jones) {
#define SCASE(NN)                                                                                        \
  case NN:                                                                                               \
    return P == 2 ? stream_fn<NN, 2, cols_ce(NN)>(accm, jones) : stream_fn<NN, 1, cols_ce(NN)>(accm, jones);
  switch (n) {
    SCASE(32) SCASE(64) SCASE(96) SCASE(128) SCASE(160) SCASE(192) SCASE(256) SCASE(320) SCASE(384) SCASE(512)
    default: return nullptr;
  }
#undef SCASE
}

size_t stream_lds_bytes(int n, int P, int band_ants, int volt_fmt) {
  const size_t rows = (size_t)P * band_rows_ce(n, P) * row_stride(n) * 8 +
                      (row_stages_volts(n) ? volt_table_bytes(band_ants, P, volt_fmt) : 0);
  const size_t cols = cols_lds_bytes(n, P, cols_ce(n)) - (size_t)2 * n * 8;
  return 16 + (size_t)2 * n * 8 + (rows > cols ? rows : cols);   // team record, twiddles, work area
}

hipError_t stream_occupancy(int n, int P, int accm, bool jones, int band_ants, int volt_fmt, int *wgs_per_cu) {
  void *fn = stream_kernel(n, P, accm, jones);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = set_lds_limit_ext(fn);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, (const void *)fn, kThreads,
                                                      stream_lds_bytes(n, P, band_ants, volt_fmt));
}

hipError_t launch_stream(int n, int P, int accm, bool jones, const StreamArgs &a, hipStream_t st) {
  void *fn = stream_kernel(n, P, accm, jones);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = set_lds_limit_ext(fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((void (*)(StreamArgs))fn, dim3(kXcds * a.wgs_per_xcd), dim3(kThreads),
                     stream_lds_bytes(n, P, a.r.band_ants_max, a.r.volt_fmt), st, a);
  return hipGetLastError();
}

}  // namespace moff
