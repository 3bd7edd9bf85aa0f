// Electric-field image taps and the feedback-calibration correlator (Section 6 of the paper; its Discussion
// notes that every pixel of the E-field image is a calibrated tied-array beam).
//
// k_tap: the E-field image of every sample at a few pixels per channel, before squaring.  It reads the
//   row-transformed samples H of the fused path's launch block (column-group tiles [p][q / W][row][q % W]) and
//   finishes the transform for the tapped column with a direct DFT over the rows:
//     E(qr, qc) = sum_j H[j][qc] exp(+2 pi i j qr / n)   (FFT-order indices; twiddles generated on the host in FP64).
// k_cal_acc: per channel, tap m, antenna a and pol p, the sums over samples of E_tap conj(E_a) (Eq. FBeq2's
//   correlation of the correlator's output with one antenna's input), |E_tap|^2 (Eq. FBeq1) and |E_a|^2, in
//   FP64.
// k_cal_solve: each antenna's gain toward the tapped pixel g = B_a(theta) (the image of a unit voltage on that
//   antenna alone: its kernel's DFT at the pixel, FP64), then S = conj(g) R, the exact sum of all visibilities
//   not involving the antenna X = Pw - S - conj(S) + |g|^2 V, and the single-calibrator gain-update factor
//   u = 2 - A conj(S) / Pw.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace moff {

__global__ __launch_bounds__(kThreads) void k_tap(TapArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);   // one wavefront per item
  const int64_t items = (int64_t)a.n_chan_block * a.nt * a.n_tap;
  if (item >= items) return;
  const int m = (int)(item % a.n_tap);
  const int64_t rest = item / a.n_tap;
  const int tl = (int)(rest % a.nt);
  const int ck = (int)(rest / a.nt);
  const int c = a.c0 + ck;
  const int n = a.chans[c].n, W = a.chans[c].cols;
  const int jmin = a.chans[c].jmin, jmax = a.chans[c].jmax;
  const int2 idx = a.tap_idx[(int64_t)c * a.n_tap + m];   // (row index qr, column index qc), FFT order
  const float2 *tw = a.tap_tw + a.tap_tw_off[c] + (int64_t)m * n;
  const float2 *h = a.h + ((int64_t)ck * a.t_block + tl) * a.P * (int64_t)n * n + (int64_t)(idx.y / W) * n * W +
                    (idx.y % W);
  float2 s[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  for (int j = jmin + lane; j <= jmax; j += 64) {
    const float2 w = tw[j];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < a.P) {
        const float2 v = h[(int64_t)p * n * n + (int64_t)j * W];
        s[p].x += v.x * w.x - v.y * w.y;
        s[p].y += v.x * w.y + v.y * w.x;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s[p].x += __shfl_xor(s[p].x, off);
      s[p].y += __shfl_xor(s[p].y, off);
    }
  }
  if (lane == 0) {
    float2 *o = a.out + (((int64_t)(a.t0 + tl) * a.n_chan + c) * a.n_tap + m) * a.P;
    o[0] = s[0];
    if (a.P == 2) o[1] = s[1];
  }
}

// One thread per (c, a, p): all taps of that channel over the samples.
template <int MT>
__global__ __launch_bounds__(kThreads) void k_cal_acc(CalArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n_chan * a.n_ant * a.P;
  if (i >= total) return;
  const int p = (int)(i % a.P);
  const int64_t ca = i / a.P;
  const int ant = (int)(ca % a.n_ant);
  const int c = (int)(ca / a.n_ant);
  double rr[MT], ri[MT], pw[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) rr[m] = ri[m] = pw[m] = 0.0;
  double v = 0.0;
  const int64_t sample_elems = (int64_t)a.n_chan * a.n_ant * a.P;   // voltages of one sample
  for (int64_t t = 0; t < a.nt; ++t) {
    float2 e;
    if (a.volt_fmt == 0) {
      const char2 b = reinterpret_cast<const char2 *>(a.volt)[t * sample_elems + i];
      e = make_float2((float)b.x, (float)b.y);
    } else {
      e = reinterpret_cast<const float2 *>(a.volt)[t * sample_elems + i];
    }
    v += (double)e.x * e.x + (double)e.y * e.y;
    const float2 *tp = a.tap + ((t * a.n_chan + c) * a.n_tap) * a.P + p;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (m < a.n_tap) {
        const float2 z = tp[(int64_t)m * a.P];
        // z conj(e)
        rr[m] += (double)z.x * e.x + (double)z.y * e.y;
        ri[m] += (double)z.y * e.x - (double)z.x * e.y;
        pw[m] += (double)z.x * z.x + (double)z.y * z.y;
      }
    }
  }
  double2 *R = reinterpret_cast<double2 *>(a.cal);
  double *Pw = reinterpret_cast<double *>(R + (int64_t)a.n_chan * a.n_tap * a.n_ant * a.P);
  double *V = Pw + (int64_t)a.n_chan * a.n_tap * a.P;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    if (m < a.n_tap) {
      double2 &r = R[(((int64_t)c * a.n_tap + m) * a.n_ant + ant) * a.P + p];
      r.x += rr[m];
      r.y += ri[m];
      if (ant == 0) Pw[((int64_t)c * a.n_tap + m) * a.P + p] += pw[m];
    }
  }
  V[ca * a.P + p] += v;
}

// One thread per (c, m, a, p).
__global__ __launch_bounds__(kThreads) void k_cal_solve(SolveArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n_chan * a.n_tap * a.n_ant * a.P;
  if (i >= total) return;
  const int p = (int)(i % a.P);
  int64_t rest = i / a.P;
  const int ant = (int)(rest % a.n_ant);
  rest /= a.n_ant;
  const int m = (int)(rest % a.n_tap);
  const int c = (int)(rest / a.n_tap);
  const int n = a.chans[c].n, K = a.K;
  const int2 org = a.origin[(int64_t)c * a.n_ant + ant];    // (j0, i0)
  const int2 pix = a.tap_cpix[(int64_t)c * a.n_tap + m];    // centred (row, col)
  const int qr = pix.x - n / 2, qc = pix.y - n / 2;
  // g = sum_{y, x} K[y][x] exp(+2 pi i ((j0 + y) qr + (i0 + x) qc) / n), angles reduced in integers
  const float2 *kern = a.kern + (((int64_t)c * a.n_ant + ant) * a.P + p) * K * K;
  double gx = 0.0, gy = 0.0;
  for (int y = 0; y < K; ++y)
    for (int x = 0; x < K; ++x) {
      long long r = ((long long)(org.x + y) * qr + (long long)(org.y + x) * qc) % n;
      if (r < 0) r += n;
      double sn, cs;
      sincospi(2.0 * (double)r / (double)n, &sn, &cs);
      const float2 k = kern[y * K + x];
      gx += (double)k.x * cs - (double)k.y * sn;
      gy += (double)k.x * sn + (double)k.y * cs;
    }
  const double2 *R = reinterpret_cast<const double2 *>(a.cal);
  const double *Pw = reinterpret_cast<const double *>(R + (int64_t)a.n_chan * a.n_tap * a.n_ant * a.P);
  const double *V = Pw + (int64_t)a.n_chan * a.n_tap * a.P;
  const double2 r = R[i];
  const double pw = Pw[((int64_t)c * a.n_tap + m) * a.P + p];
  const double v = V[((int64_t)c * a.n_ant + ant) * a.P + p];
  // S = conj(g) r
  const double sx = gx * r.x + gy * r.y, sy = gx * r.y - gy * r.x;
  const double xx = pw - 2.0 * sx + (gx * gx + gy * gy) * v;
  const double inv = pw != 0.0 ? 1.0 / pw : 0.0;
  const double ux = 2.0 - a.n_ant * sx * inv, uy = a.n_ant * sy * inv;   // 2 - A conj(S) / Pw
  double2 *o = reinterpret_cast<double2 *>(a.out);
  o[i] = make_double2(sx, sy);
  o[total + i] = make_double2(xx, 0.0);
  o[2 * total + i] = make_double2(ux, uy);
}

hipError_t launch_tap(const TapArgs &a, hipStream_t st) {
  const int64_t items = (int64_t)a.n_chan_block * a.nt * a.n_tap;
  if (items <= 0) return hipSuccess;
  const int per = kThreads / 64;
  hipLaunchKernelGGL(k_tap, dim3((unsigned)((items + per - 1) / per)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cal_acc(const CalArgs &a, hipStream_t st) {
  const int64_t total = (int64_t)a.n_chan * a.n_ant * a.P;
  if (total <= 0 || a.nt <= 0) return hipSuccess;
  const dim3 grid((unsigned)((total + kThreads - 1) / kThreads));
  if (a.n_tap <= 1)
    hipLaunchKernelGGL(k_cal_acc<1>, grid, dim3(kThreads), 0, st, a);
  else if (a.n_tap <= 4)
    hipLaunchKernelGGL(k_cal_acc<4>, grid, dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_cal_acc<kMaxTaps>, grid, dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cal_solve(const SolveArgs &a, hipStream_t st) {
  const int64_t total = (int64_t)a.n_chan * a.n_tap * a.n_ant * a.P;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cal_solve, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace moff
