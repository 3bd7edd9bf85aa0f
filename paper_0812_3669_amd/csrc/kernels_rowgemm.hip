// Matrix-core row pass of the fused path (MOFF_FFT_GEMM_FP16): gridding (Eq. m6 step 2) and the row half of the
// spatial transform (step 3) as one GEMM over time samples on the CDNA4 matrix cores.
//
// For grid row j of channel c and pol p the row-transformed grid is
//     H[t][j][k] = sum_i G[t][j][i] w^(i k) = sum_{a in A_j} E[t][a] Phi_a[k],
//     Phi_a[k]   = w^(i0_a k) sum_x W_a[j - j0_a][x] w^(x k),      w = e^(2 pi i / n),
// A_j being the antennas whose footprint covers row j: the footprint of antenna a puts W_a[y][x] E_a on cell
// (j0_a + y, i0_a + x), so the row DFT of the gridded row is a sum over antennas of their voltage times the DFT of
// their kernel row, shifted to their first column.  Over a tile of time samples this is a complex GEMM with the
// samples as M, the antennas as K and the n output columns as N, done as a real GEMM on v_mfma_f32_16x16x32_f16:
//   A (16 samples x 32) = [Re E, Im E] of 16 antennas (interleaved per antenna), exact in FP16 (int8 voltages),
//   two B operands (32 x 16) for 16 output columns k: rows (a, Re), (a, Im) = (Re Phi, -Im Phi) give the real parts
//   of the outputs and (Im Phi, Re Phi) their imaginary parts, so each lane forms Phi once for its own column; Phi
//   is formed in FP32 from the kernel (pre-scaled by a power of two that keeps |Phi| below 2^14) and a w^m table
//   (FP64-generated) and split into hi + lo FP16 terms (two products per operand, FP32 accumulation: FP32-level
//   accuracy, since the voltages need no split).
// There is no scatter: the voltages of a row's antennas are staged in LDS as FP16 pairs once per time tile and
// every output is written once, in the column-group tiles the FP32 column pass reads.
//
// Lane layout of the 16x16x32 instruction (wave64): A: lane l holds A[l % 16][8 (l / 16) + i], i < 8; B: lane l
// holds B[8 (l / 16) + i][l % 16]; D: lane l holds D[4 (l / 16) + i][l % 16], i < 4.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace moff {

namespace {

typedef _Float16 rg_half8 __attribute__((ext_vector_type(8)));
typedef _Float16 rg_half2 __attribute__((ext_vector_type(2)));
typedef uint32_t rg_u4 __attribute__((ext_vector_type(4)));
typedef float rg_float4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 cmul_rg(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ uint32_t f16_pair(int re, int im) {
  const _Float16 hr = (_Float16)(float)re, hi = (_Float16)(float)im;   // |int8| < 2^11: exact
  uint16_t br, bi;
  __builtin_memcpy(&br, &hr, 2);
  __builtin_memcpy(&bi, &hi, 2);
  return (uint32_t)br | ((uint32_t)bi << 16);
}

// Work item of a workgroup: channel c0 + k of the launch block on XCD k % 8 (its kernels, voltages and row table
// stay in one L2), then (row, pol, time tile).
__device__ __forceinline__ bool rg_map(const RgArgs &a, int &c, int &row, int &p, int &tile) {
  const int x = (int)(blockIdx.x % kXcds), s0 = (int)(blockIdx.x / kXcds);
  const int tiles = (a.nt + a.tt - 1) / a.tt;
  tile = s0 % tiles;
  int s = s0 / tiles;
  for (int k = x; k < a.n_chan_block; k += kXcds) {
    const Chan &ch = a.chans[a.c0 + k];
    const int cnt = (ch.jmax - ch.jmin + 1) * a.P;
    if (s < cnt) {
      c = a.c0 + k;
      row = ch.jmin + s / a.P;
      p = s - (s / a.P) * a.P;
      return true;
    }
    s -= cnt;
  }
  return false;
}

}  // namespace

// (x, y) as two FP16 values packed in one word, x in the low half.
__device__ __forceinline__ uint32_t f16x2_bits(float x, float y) {
  const rg_half2 h = {(_Float16)x, (_Float16)y};
  uint32_t u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}
__device__ __forceinline__ float f16_lo_f32(uint32_t u) {
  _Float16 h;
  const uint16_t b = (uint16_t)(u & 0xFFFFu);
  __builtin_memcpy(&h, &b, 2);
  return (float)h;
}

// Split operand words of one antenna slot for output column k: hr = (Re Phi, -Im Phi) and lr the same for the exact
// FP32 residuals Phi - hi, as FP16 pairs (low half first), where Phi = w^(i0 k) sum_x taps[x] w^(x k) from the
// (pre-scaled) kernel row taps, the lane's w^(x k) and the w^m table.
template <int N, int K>
__device__ __forceinline__ void rg_phi_words(const float2 *taps, const float2 *wx, const float2 *tw, int i0, int k,
                                             uint32_t &hr, uint32_t &lr) {
  float2 f = make_float2(0.f, 0.f);
#pragma unroll
  for (int x = 0; x < K; ++x) {
    const float2 w = taps[x];
    f.x = fmaf(w.x, wx[x].x, fmaf(-w.y, wx[x].y, f.x));
    f.y = fmaf(w.x, wx[x].y, fmaf(w.y, wx[x].x, f.y));
  }
  const float2 r = tw[(i0 * k) % N];
  const float px = f.x * r.x - f.y * r.y, py = f.x * r.y + f.y * r.x;
  hr = f16x2_bits(px, -py);
  const float dx = px - f16_lo_f32(hr), dy = py + f16_lo_f32(hr >> 16);   // exact residuals
  lr = f16x2_bits(dx, -dy);
}

// (Im Phi, Re Phi) from (Re Phi, -Im Phi): swap the halves and negate the new low half (exact).
__device__ __forceinline__ uint32_t rg_swapneg(uint32_t u) { return ((u >> 16) | (u << 16)) ^ 0x8000u; }

template <int N, int K>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_rowgemm(RgArgs a) {
  constexpr int W = cols_ce(N);
  constexpr int MT = 8;                       // 16-sample tiles per time tile (at most)
  static_assert(N % 16 == 0, "16 output columns per operand");
  extern __shared__ float4 smem4[];
  int c, row, p, tile;
  if (!rg_map(a, c, row, p, tile)) return;
  const int slots = a.slots;
  float2 *tw = reinterpret_cast<float2 *>(smem4);                       // [N] w^m
  float2 *taps = tw + N;                                                // [slots][K]
  int *i0s = reinterpret_cast<int *>(taps + (size_t)slots * K);          // [slots]
  int *ants = i0s + slots;                                               // [slots]
  uint32_t *E16 = reinterpret_cast<uint32_t *>(ants + slots);            // [tt][stride]
  float *red = reinterpret_cast<float *>(E16 + (size_t)a.tt * (slots + 4)); // [kWaves] bound reduction

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Chan &ch = a.chans[c];
  const int ent_off = a.rows[2 * (ch.rg_first + row - ch.jmin)];
  const int na = a.rows[2 * (ch.rg_first + row - ch.jmin) + 1];
  const int kc = (na + 15) >> 4, ns = kc * 16, stride = ns + 4;

  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = a.tw[i];
  // the row's antennas: kernel row (j - j0) with phases folded, first column, index; zero taps on padding slots.
  // |Phi| <= sum_x |W[x]| <= sum_x (|Re W| + |Im W|) < 2^eb: the taps are scaled by 2^(14 - eb) (exact), so the
  // scaled Phi stays within FP16, and the outputs are scaled back by 2^(eb - 14).
  float bound = 0.f;
  for (int s = threadIdx.x; s < ns; s += kThreads) {
    int i0 = 0, ant = 0;
    float sum = 0.f;
    if (s < na) {
      const uint32_t e = a.ents[ent_off + s];
      ant = (int)(e & 0xFFFFu);
      const int y = (int)((e >> 16) & 7u);
      i0 = (int)(e >> 20);
      const float2 *src = a.rk + (((int64_t)c * a.n_ant + ant) * a.P + p) * (K * K) + y * K;
#pragma unroll
      for (int x = 0; x < K; ++x) {
        const float2 w = src[x];
        taps[s * K + x] = w;
        sum += fabsf(w.x) + fabsf(w.y);
      }
    } else {
#pragma unroll
      for (int x = 0; x < K; ++x) taps[s * K + x] = make_float2(0.f, 0.f);
    }
    i0s[s] = i0;
    ants[s] = ant;
    bound = fmaxf(bound, sum);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bound = fmaxf(bound, __shfl_xor(bound, o));
  if (lane == 0) red[wave] = bound;
  __syncthreads();
  const float bmax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const int eb = bmax > 0.f ? __builtin_amdgcn_frexp_expf(bmax) : 0;   // bmax < 2^eb
  const float sc = ldexpf(1.f, 14 - eb), inv = ldexpf(1.f, eb - 14);
  for (int i = threadIdx.x; i < ns * K; i += kThreads) {
    const float2 w = taps[i];
    taps[i] = make_float2(w.x * sc, w.y * sc);
  }

  // the tile's samples, FP16 (re, im) per antenna slot (zero past the last sample and on padding slots)
  const int t_lo = a.t0 + tile * a.tt;
  const int ntt = min(a.tt, a.t0 + a.nt - t_lo);
  const int mts = (ntt + 15) >> 4;
  if (ns > 0) {
    const int64_t vstride = (int64_t)a.n_chan * a.n_ant * a.P * 2;   // bytes per sample
    const char *vb = reinterpret_cast<const char *>(a.volt) + (int64_t)c * a.n_ant * a.P * 2 + (int64_t)p * 2 +
                     (int64_t)t_lo * vstride;
    // slot s of samples tl, tl + step, ...: the loads of a batch of 8 are issued before any is used (a padding slot
    // reads antenna 0 and a sample past the tile reads the tile's last one; both are stored as zero)
    auto stage_run = [&](int s, int tl_first, int step) {
      const bool live = s < na;
      const char *vp = vb + (int64_t)ants[s] * a.P * 2;
      for (int tl = tl_first; tl < mts * 16; tl += 8 * step) {
        uint32_t pr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          pr[u] = *reinterpret_cast<const uint16_t *>(vp + (int64_t)min(tl + u * step, ntt - 1) * vstride);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t2 = tl + u * step;
          if (t2 < mts * 16)
            E16[t2 * stride + s] = (live && t2 < ntt) ? f16_pair((int)(int8_t)(pr[u] & 0xFFu), (int)(int8_t)(pr[u] >> 8))
                                                      : 0u;
        }
      }
    };
    if (ns <= kThreads) {
      // kThreads / ns samples per pass, thread -> (slot, first sample)
      const int per = kThreads / ns, s = (int)threadIdx.x % ns, tl0 = (int)threadIdx.x / ns;
      if (tl0 < per) stage_run(s, tl0, per);
    } else {
      for (int s = threadIdx.x; s < ns; s += kThreads) stage_run(s, 0, 1);
    }
  }
  __syncthreads();

  const int col16 = lane & 15, g = lane >> 4;
  float2 *H = a.io;
  const int64_t nn = (int64_t)N * N;
  for (int chunk = wave; chunk < N / 16; chunk += kWaves) {
    const int k = chunk * 16 + col16;                          // output column of this lane
    float2 wx[K];
#pragma unroll
    for (int x = 0; x < K; ++x) wx[x] = tw[(x * k) % N];
    rg_float4 Dre[MT], Dim[MT];
    for (int kk = 0; kk < kc; ++kk) {
      // operand rows 8 g + 2 ii (+1) <-> antenna slot 16 kk + 4 g + ii, real (imaginary) voltage part; word ii of
      // the real-part operand is (Re Phi, -Im Phi), of the imaginary-part operand (Im Phi, Re Phi)
      rg_u4 bre_hi, bre_lo, bim_hi, bim_lo;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int s = 16 * kk + 4 * g + ii;
        uint32_t hr, lr;
        rg_phi_words<N, K>(taps + s * K, wx, tw, i0s[s], k, hr, lr);
        bre_hi[ii] = hr;
        bre_lo[ii] = lr;
        bim_hi[ii] = rg_swapneg(hr);
        bim_lo[ii] = rg_swapneg(lr);
      }
      rg_half8 Brh, Brl, Bih, Bil;
      __builtin_memcpy(&Brh, &bre_hi, 16);
      __builtin_memcpy(&Brl, &bre_lo, 16);
      __builtin_memcpy(&Bih, &bim_hi, 16);
      __builtin_memcpy(&Bil, &bim_lo, 16);
      // the first chunk starts the accumulators from the products (no separate clear)
      const rg_float4 z = rg_float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (m < mts) {
          const uint4 av = *reinterpret_cast<const uint4 *>(E16 + (m * 16 + col16) * stride + 16 * kk + 4 * g);
          rg_half8 A;
          __builtin_memcpy(&A, &av, 16);
          Dre[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, Brl, kk == 0 ? z : Dre[m], 0, 0, 0);
          Dim[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, Bil, kk == 0 ? z : Dim[m], 0, 0, 0);
          Dre[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, Brh, Dre[m], 0, 0, 0);
          Dim[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, Bih, Dim[m], 0, 0, 0);
        }
      }
    }
    if (kc == 0) {
#pragma unroll
      for (int m = 0; m < MT; ++m) Dre[m] = Dim[m] = rg_float4{0.f, 0.f, 0.f, 0.f};
    }
    // (Dre, Dim)[m][i] = H[t_lo + 16 m + 4 g + i][row][k]: column-group tiles [p][k / W][row][k % W] of the block
    const int64_t inner = (int64_t)(k / W) * (N * W) + row * W + (k % W);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (m < mts) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int tl = 16 * m + 4 * g + i;
          if (tl < ntt) {
            const int64_t slot = ((int64_t)(c - a.c0) * a.t_block + (t_lo + tl - a.t0)) * a.P + p;
            store_stream(H + slot * nn + inner, make_float2(Dre[m][i] * inv, Dim[m][i] * inv));
          }
        }
      }
    }
  }
}

// w^m = e^(2 pi i m / n), m < n, in FP64 from the exact integer angle, rounded once.
__global__ void k_rg_twiddle(float2 *tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(2.0 * (double)m / (double)n, &s, &c);
  tw[m] = make_float2((float)c, (float)s);
}

// Kernels of the matrix-core row pass: [C][A][P][K][K] with the phase-centre phase of each (c, a, p) folded in.
__global__ void k_pack_rk(const float2 *__restrict__ kern, const float2 *__restrict__ phase, float2 *__restrict__ rk,
                          int64_t total, int KK) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float2 v = kern[i];
  if (phase) v = cmul_rg(v, phase[i / KK]);
  rk[i] = v;
}

template <int N>
static void *rowgemm_fn_n(int K) {
  switch (K) {
    case 2: return (void *)k_rowgemm<N, 2>;
    case 4: return (void *)k_rowgemm<N, 4>;
    case 6: return (void *)k_rowgemm<N, 6>;
    case 8: return (void *)k_rowgemm<N, 8>;
    default: return nullptr;
  }
}

static void *rowgemm_fn(int n, int K) {
  switch (n) {
#define GCASE(NN) \
  case NN: return rowgemm_fn_n<NN>(K);
    GCASE(32) GCASE(64) GCASE(96) GCASE(128) GCASE(160) GCASE(192) GCASE(256) GCASE(320) GCASE(384) GCASE(512)
#undef GCASE
    default: return nullptr;
  }
}

int rowgemm_grid(const Plan &p, const Block &b, int nt) {
  const int tiles = (nt + p.rg_tt - 1) / p.rg_tt;
  int mx = 0;
  for (int x = 0; x < kXcds; ++x) {
    int n = 0;
    for (int k = x; k < b.c1 - b.c0; k += kXcds) {
      const Chan &ch = p.chans[b.c0 + k];
      n += (ch.jmax - ch.jmin + 1) * p.n_pol;
    }
    mx = n > mx ? n : mx;
  }
  return kXcds * tiles * mx;
}

hipError_t launch_rowgemm(int n, const RgArgs &a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  void *fn = rowgemm_fn(n, a.K);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = set_lds_limit_ext(fn);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((void (*)(RgArgs))fn, dim3(grid), dim3(kThreads), rowgemm_lds_bytes(n, a.K, a.slots, a.tt), st,
                     a);
  return hipGetLastError();
}

hipError_t launch_rg_twiddle(float2 *tw, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_rg_twiddle, dim3((n + 255) / 256), dim3(256), 0, st, tw, n);
  return hipGetLastError();
}

hipError_t launch_pack_rk(const float2 *kern, const float2 *phase, float2 *rk, int64_t total, int KK, hipStream_t st) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_rk, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, kern, phase, rk, total, KK);
  return hipGetLastError();
}

}  // namespace moff
