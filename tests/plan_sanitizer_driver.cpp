// Host-only driver of the plan builder (plan.cpp) for the sanitizer test: builds plans for several layouts
// (fixed and automatic grid sizes, taps, a single antenna, a footprint leaving the grid) with no HIP code.
#include "fft_sizes.h"
#include "moff_plan.h"
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <random>
#include <vector>
int run(int A, int C, int n, int K, double disk, int P, int ntap, int seed) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0, 1);
  double c = 299792458.0, fref = 130e6, Dm = disk * c / fref;
  std::vector<double> xy(2 * A), f(C);
  for (int a = 0; a < A; ++a) { double r = 0.5 * Dm * sqrt(U(rng)), ph = 2 * M_PI * U(rng); xy[2*a] = r*cos(ph); xy[2*a+1] = r*sin(ph); }
  for (int i = 0; i < C; ++i) f[i] = 100e6 + (i + 0.5) * 30e6 / C;
  std::vector<int> gn(C, n);
  moff_plan_desc d{}; d.n_ant = A; d.n_pol = P; d.n_chan = C; d.ksize = K; d.ant_xy_m = xy.data(); d.freq_hz = f.data();
  d.grid_n = n > 0 ? gn.data() : nullptr; d.cell_lambda = 1.0; d.n_tap = ntap;
  moff::Plan p; std::string err;
  setenv("MOFF_PLAN_THREADS", "1", 1);
  int s = moff::build_plan(d, p, &err);
  if (s) { printf("A=%d C=%d n=%d K=%d: status %d (%s)\n", A, C, n, K, s, err.c_str()); return s; }
  // channels built on several threads give the same plan as one thread
  moff::Plan q; std::string err2;
  setenv("MOFF_PLAN_THREADS", "5", 1);
  if (moff::build_plan(d, q, &err2) != 0) { printf("threaded build failed: %s\n", err2.c_str()); return 1; }
  unsetenv("MOFF_PLAN_THREADS");
  bool same = p.band_ptr == q.band_ptr && p.band_ant == q.band_ant && p.grp_meta == q.grp_meta &&
              p.grp_kidx == q.grp_kidx && p.grp_chan == q.grp_chan && p.n_groups == q.n_groups &&
              p.max_band_ants == q.max_band_ants && p.bands.size() == q.bands.size() && p.ws_total == q.ws_total;
  for (size_t b = 0; same && b < p.bands.size(); ++b) {
    const moff::Band &x = p.bands[b], &y = q.bands[b];
    same = x.chan == y.chan && x.row0 == y.row0 && x.rows == y.rows && x.r_lo == y.r_lo && x.r_hi == y.r_hi &&
           x.ant_off == y.ant_off && x.ant_cnt == y.ant_cnt;
    for (int w = 0; same && w < moff::kWaves; ++w) same = x.grp_off[w] == y.grp_off[w] && x.grp_cnt[w] == y.grp_cnt[w];
  }
  for (size_t c = 0; same && c < p.chans.size(); ++c)
    same = p.chans[c].band_first == q.chans[c].band_first && p.chans[c].band_count == q.chans[c].band_count;
  if (!same) { printf("threaded plan differs from the one-thread plan\n"); return 1; }
  long taps = 0;
  for (auto k : p.grp_kidx) taps += (k >= 0);
  for (auto m : p.grp_meta) if (m == moff::kEmptyTap) { printf("unfilled lane\n"); return 1; }
  // every lane of a wavefront's groups (empty ones included) scatters into that wavefront's rows only, and the
  // cells of one group are distinct
  for (auto &b : p.bands) {
    const int ts = moff::row_stride(p.chans[b.chan].n);
    for (int w = 0; w < moff::kWaves; ++w)
      for (int g = 0; g < b.grp_cnt[w]; ++g) {
        const uint32_t *gm = p.grp_meta.data() + (b.grp_off[w] + g) * moff::kGroupLanes;
        for (int l = 0; l < moff::kGroupLanes; ++l) {
          const int cell = (int)(gm[l] & 0xFFFFu);
          if ((cell / ts) % moff::kWaves != w || cell >= b.rows * ts) { printf("lane outside its rows\n"); return 1; }
          for (int k = 0; k < l; ++k)
            if ((int)(gm[k] & 0xFFFFu) == cell) { printf("two lanes on one cell\n"); return 1; }
        }
      }
  }
  printf("A=%d C=%d n=%d K=%d P=%d: bands %zu groups %lld taps %ld ws %zu\n", A, C, n, K, P, p.bands.size(), (long long)p.n_groups, taps, p.ws_total);
  for (int tb : {1, 8, 64}) for (int cpb : {1, 7, 64}) moff::layout_blocks(p, tb, cpb, 4);
  return 0;
}
int main() {
  int bad = 0;
  bad |= run(64, 1, 64, 4, 30, 1, 0, 1);
  bad |= run(256, 8, 128, 4, 60, 2, 2, 2);
  bad |= run(2048, 4, 256, 4, 200, 2, 8, 3);
  bad |= run(512, 6, 0, 6, 120, 2, 0, 4);      // automatic grid sizes
  bad |= run(1, 1, 32, 8, 1, 2, 1, 5);
  bad |= run(300, 2, 512, 2, 400, 1, 0, 6);
  run(100, 1, 32, 4, 200, 2, 0, 7);            // footprints leave the grid: an error, not a crash
  return bad;
}
