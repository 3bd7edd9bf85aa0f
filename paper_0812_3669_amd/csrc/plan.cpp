// Host plan: geometry, row-band binning and tap groups of the gridding step (Eq. m6 step 2), launch blocks and
// the device workspace layout.  No HIP calls here.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "fft_sizes.h"
#include "moff_plan.h"

namespace moff {

namespace {
constexpr double kCLight = 299792458.0;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr size_t kMfmaTableBytesHost = (size_t)17 * 2 * 3 * 64 * 8 * 2;   // matrices of the split transform

int env_int(const char *name, int dflt, int lo, int hi) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  const long x = std::strtol(v, nullptr, 10);
  return (int)std::min<long>(hi, std::max<long>(lo, x));
}

moff_status fail(std::string *err, moff_status s, const std::string &msg) {
  if (err) *err = msg;
  return s;
}
}  // namespace

// Grid sizes with an FFT pipeline: 2^a * {1, 3, 5}, multiples of 32, up to 512.
bool fft_size_supported(int n) {
  static const int ok[] = {32, 64, 96, 128, 160, 192, 256, 320, 384, 512};
  for (int v : ok)
    if (v == n) return true;
  return false;
}

// Rows per band of the row pass: the band grid (P x rows x n complex64) stays within 32 KB of LDS for
// power-of-two n and within 16 KB for mixed-radix n (their three-stage row transforms hold more registers, and
// shorter bands measured faster there).
int band_rows_for(int n, int P) {
  const size_t limit = (n & (n - 1)) == 0 ? 32768 : 16384;
  int h = 16;
  while (h > 4 && (size_t)P * h * n * 8 > limit) h /= 2;
  return h;
}

// Columns per workgroup of the column pass: the largest power of two <= max(8, 2048 / n) dividing n.
int cols_for(int n) {
  int lim = std::max(8, 2048 / n), w = 1;
  while (w * 2 <= lim && n % (w * 2) == 0) w *= 2;
  return w;
}

size_t rowgemm_lds_bytes(int n, int K, int slots, int tt) {
  return (size_t)n * 8 + (size_t)slots * K * 8 + (size_t)slots * 8 + (size_t)tt * (slots + 4) * 4 + kWaves * 4;
}

int smallest_supported_size(int need) {
  static const int ok[] = {32, 64, 96, 128, 160, 192, 256, 320, 384, 512};
  for (int v : ok)
    if (v >= need) return v;
  return 0;
}

// Row bands, band antenna lists and tap groups of one channel, with offsets local to the channel (the caller
// appends channels in order and shifts the offsets).  Reads the footprint origins and the channel's grid
// geometry only, so channels build independently.
struct ChanBuild {
  std::vector<Band> bands;
  std::vector<int32_t> band_end;   // end of each band's antenna list in `ant`
  std::vector<int32_t> ant;
  std::vector<uint32_t> meta;
  std::vector<int32_t> kidx;
  int64_t n_groups = 0;
  int32_t max_ants = 0;
  moff_status st = MOFF_OK;
  std::string err;
};

void build_channel(const Plan &p, int c, int A, int K, ChanBuild &out) {
  const Chan &ch = p.chans[c];
  const int n = ch.n, h = ch.band_rows;
  const int b_lo = ch.jmin / h, b_hi = ch.jmax / h;
  // antennas whose footprint rows [j0, j0+K-1] meet a band (boundary antennas appear in both bands): bands
  // j0 / h .. (j0 + K - 1) / h, filled in ascending antenna order
  std::vector<std::vector<int32_t>> lists((size_t)(b_hi - b_lo + 1));
  for (int a = 0; a < A; ++a) {
    const int j0 = p.origin[((size_t)c * A + a) * 2];
    for (int b = std::max(b_lo, j0 / h); b <= std::min(b_hi, (j0 + K - 1) / h); ++b)
      lists[(size_t)(b - b_lo)].push_back(a);
  }
  std::vector<int32_t> last_used;
  for (int b = b_lo; b <= b_hi; ++b) {
    Band bd{};
    bd.chan = c;
    bd.row0 = b * h;
    bd.rows = std::min(h, n - bd.row0);
    bd.r_lo = std::max(bd.row0, ch.jmin);
    bd.r_hi = std::min(bd.row0 + bd.rows - 1, ch.jmax);
    const std::vector<int32_t> &bl = lists[(size_t)(b - b_lo)];
    const int32_t lo = (int32_t)out.ant.size();
    out.ant.insert(out.ant.end(), bl.begin(), bl.end());
    const int32_t hi = (int32_t)out.ant.size();
    out.band_end.push_back(hi);
    bd.ant_off = lo;
    bd.ant_cnt = hi - lo;
    if (row_stages_volts(n)) out.max_ants = std::max(out.max_ants, hi - lo);
    // tap groups per wavefront: 64 taps on 64 distinct cells per group, antennas ascending, first fit, so every
    // cell receives its contributions in ascending antenna order (deterministic sums, no atomics).  Lane
    // 16 q + k of a group holds a tap whose LDS word offset is k mod 16, so the 16 lanes a quarter-wave
    // presents to the LDS at once hit 16 different bank pairs.
    const int ts = row_stride(n);
    for (int w = 0; w < kWaves; ++w) {
      const int64_t g0 = out.n_groups;
      last_used.assign((size_t)bd.rows * ts, -1);
      std::vector<uint64_t> used;      // per group: bit 16 q + k set when lane 16 q + k is taken
      std::vector<int32_t> count;
      // per bank key: the first group with a free lane for that key (earlier groups have none, so first fit
      // may start there)
      int64_t first_free[16] = {};
      for (int e = lo; e < hi; ++e) {
        const int a = out.ant[e];
        const int j0 = p.origin[((size_t)c * A + a) * 2], i0 = p.origin[((size_t)c * A + a) * 2 + 1];
        for (int y = 0; y < K; ++y) {
          const int r = j0 + y - bd.row0;
          if (r < 0 || r >= bd.rows || (r % kWaves) != w) continue;
          for (int x = 0; x < K; ++x) {
            const int cell = r * ts + i0 + x;   // element offset in a pol's band grid in LDS
            const int key = cell & 15;
            int64_t g = std::max<int64_t>(first_free[key], (int64_t)last_used[cell] + 1);
            int lane = -1;
            for (;; ++g) {
              if (g == (int64_t)count.size()) {
                count.push_back(0);
                used.push_back(0);
                out.meta.resize(out.meta.size() + kGroupLanes, kEmptyTap);
                out.kidx.resize(out.kidx.size() + kGroupLanes, -1);
              }
              for (int q = 0; q < 4; ++q)
                if (!((used[g] >> (16 * q + key)) & 1)) {
                  lane = 16 * q + key;
                  break;
                }
              if (lane >= 0) break;
            }
            const size_t slot = (size_t)(g0 + g) * kGroupLanes + lane;
            out.meta[slot] = ((uint32_t)(row_stages_volts(n) ? e - lo : a) << 16) | (uint32_t)cell;
            out.kidx[slot] = (a * K + y) * K + x;
            used[g] |= (uint64_t)1 << lane;
            ++count[g];
            last_used[cell] = (int32_t)g;
            const uint64_t key_lanes = 0x0001000100010001ull << key;
            while (first_free[key] < (int64_t)count.size() && (used[first_free[key]] & key_lanes) == key_lanes)
              ++first_free[key];
          }
        }
      }
      // empty lanes get a cell in one of this wavefront's rows (other wavefronts scatter into theirs at the same
      // time) that no other lane of their group uses (same bank key), and zero weights (kidx -1): they add 0
      // there, so the row pass needs no per-lane emptiness test
      for (size_t g = 0; g < count.size(); ++g) {
        uint32_t *gm = out.meta.data() + (size_t)(g0 + (int64_t)g) * kGroupLanes;
        int taken[16][kGroupLanes / 16], n_taken[16] = {};   // cells in use per bank key (4 lanes per key)
        for (int l = 0; l < kGroupLanes; ++l)
          if (gm[l] != kEmptyTap) taken[l & 15][n_taken[l & 15]++] = (int)(gm[l] & 0xFFFFu);
        for (int l = 0; l < kGroupLanes; ++l) {
          if (gm[l] != kEmptyTap) continue;
          const int key = l & 15;
          int cell = -1;
          for (int r = w; r < bd.rows && cell < 0; r += kWaves)   // this wavefront's rows
            for (int cand = r * ts + ((key - r * ts) & 15); cand < (r + 1) * ts && cell < 0; cand += 16) {
              bool busy = false;
              for (int u = 0; u < n_taken[key]; ++u) busy |= taken[key][u] == cand;
              if (!busy) cell = cand;
            }
          if (cell < 0) {
            out.st = MOFF_E_INVALID;
            out.err = "no free cell for an empty tap lane";
            return;
          }
          taken[key][n_taken[key]++] = cell;
          gm[l] = (uint32_t)cell;
        }
      }
      bd.grp_off[w] = g0;
      bd.grp_cnt[w] = (int32_t)count.size();
      out.n_groups += (int64_t)count.size();
    }
    out.bands.push_back(bd);
  }
}

moff_status build_plan(const moff_plan_desc &d, Plan &p, std::string *err) {
  if (d.n_ant < 1 || d.n_ant > 65534) return fail(err, MOFF_E_INVALID, "n_ant must be in [1, 65534]");
  if (d.n_pol != 1 && d.n_pol != 2) return fail(err, MOFF_E_INVALID, "n_pol must be 1 or 2");
  if (d.n_chan < 1) return fail(err, MOFF_E_INVALID, "n_chan must be >= 1");
  if (d.ksize < 2 || d.ksize > 8 || (d.ksize & 1)) return fail(err, MOFF_E_INVALID, "ksize must be even, 2..8");
  if (!d.ant_xy_m || !d.freq_hz) return fail(err, MOFF_E_INVALID, "ant_xy_m and freq_hz must be non-null");
  if (!(d.cell_lambda > 0.0) || !std::isfinite(d.cell_lambda))
    return fail(err, MOFF_E_INVALID, "cell_lambda must be positive");
  if (d.fft_mode != MOFF_FFT_FP32 && d.fft_mode != MOFF_FFT_SPLIT_FP16 && d.fft_mode != MOFF_FFT_SPLIT_BF16 &&
      d.fft_mode != MOFF_FFT_GEMM_FP16)
    return fail(err, MOFF_E_INVALID, "unknown fft_mode");
  if (d.fft_mode == MOFF_FFT_GEMM_FP16 && d.volt_format != MOFF_VOLT_INT8)
    return fail(err, MOFF_E_UNSUPPORTED, "the matrix-core row pass takes int8 voltages (exact in FP16)");
  if (d.acc_mode != MOFF_ACC_FP32 && d.acc_mode != MOFF_ACC_FP64_COMP)
    return fail(err, MOFF_E_INVALID, "unknown acc_mode");
  if (d.volt_format != MOFF_VOLT_INT8 && d.volt_format != MOFF_VOLT_C64)
    return fail(err, MOFF_E_INVALID, "unknown volt_format");
  if (d.time_block < 0) return fail(err, MOFF_E_INVALID, "time_block must be >= 0");
  if (d.n_tap < 0 || d.n_tap > 8) return fail(err, MOFF_E_INVALID, "n_tap must be 0..8");
  if (d.kernel_mode != MOFF_KERNEL_DIAG && d.kernel_mode != MOFF_KERNEL_JONES)
    return fail(err, MOFF_E_INVALID, "unknown kernel_mode");
  if (d.kernel_mode == MOFF_KERNEL_JONES && d.n_pol != 2)
    return fail(err, MOFF_E_INVALID, "Jones kernels need two pols");
  if (d.kernel_mode == MOFF_KERNEL_JONES && d.fft_mode != MOFF_FFT_FP32)
    return fail(err, MOFF_E_UNSUPPORTED, "Jones kernels are built for the FP32 transform");

  p.n_ant = d.n_ant;
  p.n_pol = d.n_pol;
  p.n_chan = d.n_chan;
  p.ksize = d.ksize;
  p.cell_lambda = d.cell_lambda;
  p.fft_mode = d.fft_mode;
  p.acc_mode = d.acc_mode;
  p.volt_format = d.volt_format;
  p.kernel_mode = d.kernel_mode;
  p.n_tap = d.n_tap;
  p.ant_xy.assign(d.ant_xy_m, d.ant_xy_m + 2 * (size_t)d.n_ant);
  p.freq.assign(d.freq_hz, d.freq_hz + d.n_chan);
  for (double v : p.ant_xy)
    if (!std::isfinite(v)) return fail(err, MOFF_E_INVALID, "non-finite antenna position");
  for (double f : p.freq)
    if (!(f > 0.0) || !std::isfinite(f)) return fail(err, MOFF_E_INVALID, "channel frequencies must be positive");

  const int A = p.n_ant, C = p.n_chan, K = p.ksize, P = p.n_pol;
  // launch-block shape of the fused path (defaults; MOFF_T_BLOCK, MOFF_T_GROUP, MOFF_CHANS_PER_BLOCK override)
  if (d.chans_per_block < 0 || d.time_group < 0) return fail(err, MOFF_E_INVALID, "launch shape must be >= 0");
  // defaults: 256 samples x 32 channels per launch block, 32 samples per row-pass workgroup, measured best on
  // MI355X for the 2048-antenna 256^2 workload and neutral-to-better for the 4096-antenna per-channel-size one
  // (8192 channel-samples per launch; each doubling of the block halves the accumulator updates; 512-sample or
  // 64-channel blocks gain nothing more for twice the exchange buffer)
  const int tb = d.time_block > 0 ? d.time_block : env_int("MOFF_T_BLOCK", 256, 1, 4096);
  const int tg = d.time_group > 0 ? d.time_group : env_int("MOFF_T_GROUP", 32, 1, 4096);
  const int cpb = d.chans_per_block > 0 ? d.chans_per_block : env_int("MOFF_CHANS_PER_BLOCK", 32, 1, 1 << 20);

  // ---- per-channel grid size and footprints ------------------------------------------------------------
  p.chans.assign(C, Chan{});
  p.origin.assign((size_t)C * A * 2, 0);
  int64_t pix = 0;
  for (int c = 0; c < C; ++c) {
    const double scale = p.freq[c] / kCLight / p.cell_lambda;   // cells per metre
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int a = 0; a < A; ++a) {
      xmin = std::min(xmin, p.ant_xy[2 * a] * scale);
      xmax = std::max(xmax, p.ant_xy[2 * a] * scale);
      ymin = std::min(ymin, p.ant_xy[2 * a + 1] * scale);
      ymax = std::max(ymax, p.ant_xy[2 * a + 1] * scale);
    }
    int n = d.grid_n ? d.grid_n[c] : 0;
    if (n < 0) return fail(err, MOFF_E_INVALID, "grid_n must be >= 0");
    if (n == 0) {
      // smallest supported size whose centred grid holds every footprint
      const double span = 2.0 * std::max(std::max(std::fabs(xmin), std::fabs(xmax)),
                                          std::max(std::fabs(ymin), std::fabs(ymax)));
      n = smallest_supported_size((int)std::ceil(span) + K + 2);
      if (n == 0) return fail(err, MOFF_E_UNSUPPORTED, "array too large for the supported grid sizes");
    }
    if (!fft_size_supported(n))
      return fail(err, MOFF_E_UNSUPPORTED, "grid size " + std::to_string(n) + " has no FFT pipeline");
    Chan &ch = p.chans[c];
    ch.n = n;
    ch.pix_off = pix;
    pix += (int64_t)n * n;
    ch.jmin = n;
    ch.jmax = -1;
    for (int a = 0; a < A; ++a) {
      const double X = p.ant_xy[2 * a] * scale + n / 2;
      const double Y = p.ant_xy[2 * a + 1] * scale + n / 2;
      const double fx = std::floor(X), fy = std::floor(Y);
      if (!(fx >= -1e9 && fx <= 1e9 && fy >= -1e9 && fy <= 1e9))
        return fail(err, MOFF_E_INVALID, "antenna coordinate out of range");
      const int i0 = (int)fx - K / 2 + 1, j0 = (int)fy - K / 2 + 1;
      if (i0 < 0 || j0 < 0 || i0 + K > n || j0 + K > n)
        return fail(err, MOFF_E_INVALID,
                    "footprint of antenna " + std::to_string(a) + " leaves the " + std::to_string(n) +
                        "^2 grid of channel " + std::to_string(c));
      p.origin[((size_t)c * A + a) * 2 + 0] = j0;
      p.origin[((size_t)c * A + a) * 2 + 1] = i0;
      ch.jmin = std::min(ch.jmin, j0);
      ch.jmax = std::max(ch.jmax, j0 + K - 1);
    }
    ch.band_rows = band_rows_for(n, P);
    ch.cols = cols_for(n);
    ch.col_groups = n / ch.cols;
  }
  p.pix_total = pix;
  if (p.split_mfma()) {
    // the matrix-core transform is built for 256^2 grids with two pols
    if (P != 2) return fail(err, MOFF_E_UNSUPPORTED, "split-precision transform needs two pols");
    for (const Chan &ch : p.chans)
      if (ch.n != 256) return fail(err, MOFF_E_UNSUPPORTED, "split-precision transform is built for 256^2 grids");
  }

  // ---- row bands, band antenna lists and tap groups ------------------------------------------------------
  // channels build on worker threads (MOFF_PLAN_THREADS, default: the host's threads up to 16) and are placed
  // in channel order, so the plan does not depend on the thread count
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int n_thr = std::min(C, env_int("MOFF_PLAN_THREADS", (int)std::min(hw, 16u), 1, 256));
  auto parallel_channels = [&](const std::function<void(int)> &fn) {
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int c; (c = next.fetch_add(1)) < C;) fn(c);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < n_thr; ++t) {
      try {
        pool.emplace_back(work);
      } catch (const std::system_error &) {   // fewer threads: the calling thread takes the remaining channels
        break;
      }
    }
    work();
    for (auto &t : pool) t.join();
  };
  std::vector<ChanBuild> built((size_t)C);
  parallel_channels([&](int c) {
    try {
      build_channel(p, c, A, K, built[(size_t)c]);
    } catch (const std::exception &ex) {
      built[(size_t)c].st = MOFF_E_INVALID;
      built[(size_t)c].err = std::string("plan build failed: ") + ex.what();
    }
  });
  // offsets of each channel's bands, antenna entries and groups; the arrays are sized once and filled in parallel
  std::vector<int64_t> ant_at((size_t)C + 1, 0), grp_at((size_t)C + 1, 0);
  for (int c = 0; c < C; ++c) {
    const ChanBuild &cb = built[(size_t)c];
    if (cb.st != MOFF_OK) return fail(err, cb.st, cb.err);
    ant_at[(size_t)c + 1] = ant_at[(size_t)c] + (int64_t)cb.ant.size();
    grp_at[(size_t)c + 1] = grp_at[(size_t)c] + cb.n_groups;
  }
  if (ant_at[(size_t)C] > INT32_MAX) return fail(err, MOFF_E_UNSUPPORTED, "too many band antenna entries");
  p.bands.clear();
  p.max_band_ants = 0;
  p.band_ptr.assign(1, 0);
  p.n_groups = grp_at[(size_t)C];
  for (int c = 0; c < C; ++c) {
    const ChanBuild &cb = built[(size_t)c];
    Chan &ch = p.chans[c];
    const int32_t ant_base = (int32_t)ant_at[(size_t)c];
    ch.band_first = (int32_t)p.bands.size();
    ch.band_count = (int32_t)cb.bands.size();
    for (size_t b = 0; b < cb.bands.size(); ++b) {
      Band bd = cb.bands[b];
      bd.ant_off += ant_base;
      for (int w = 0; w < kWaves; ++w) bd.grp_off[w] += grp_at[(size_t)c];
      p.bands.push_back(bd);
      p.band_ptr.push_back(ant_base + cb.band_end[b]);
    }
    p.max_band_ants = std::max(p.max_band_ants, cb.max_ants);
  }
  p.band_ant.assign((size_t)ant_at[(size_t)C], 0);
  p.grp_meta.assign((size_t)p.n_groups * kGroupLanes, 0);
  p.grp_kidx.assign((size_t)p.n_groups * kGroupLanes, 0);
  p.grp_chan.assign((size_t)p.n_groups, 0);
  parallel_channels([&](int c) {
    ChanBuild &cb = built[(size_t)c];
    std::copy(cb.ant.begin(), cb.ant.end(), p.band_ant.begin() + ant_at[(size_t)c]);
    std::copy(cb.meta.begin(), cb.meta.end(), p.grp_meta.begin() + grp_at[(size_t)c] * kGroupLanes);
    std::copy(cb.kidx.begin(), cb.kidx.end(), p.grp_kidx.begin() + grp_at[(size_t)c] * kGroupLanes);
    std::fill(p.grp_chan.begin() + grp_at[(size_t)c], p.grp_chan.begin() + grp_at[(size_t)c + 1], c);
    cb = ChanBuild();   // release the channel's copy
  });
  if ((int64_t)p.bands.size() > INT32_MAX / 2) return fail(err, MOFF_E_UNSUPPORTED, "too many bands");
  // matrix-core row pass: the antennas covering each touched row, in ascending order (a counting sort per channel)
  p.rg_rows.clear();
  p.rg_ents.clear();
  p.rg_max_ants = 0;
  if (p.gemm()) {
    for (int c = 0; c < C; ++c) {
      Chan &ch = p.chans[c];
      const int rows = ch.jmax - ch.jmin + 1;
      ch.rg_first = (int32_t)(p.rg_rows.size() / 2);
      std::vector<int32_t> cnt((size_t)rows + 1, 0);
      for (int a = 0; a < A; ++a) {
        const int j0 = p.origin[((size_t)c * A + a) * 2];
        for (int y = 0; y < K; ++y) ++cnt[(size_t)(j0 + y - ch.jmin) + 1];
      }
      for (int r = 0; r < rows; ++r) cnt[(size_t)r + 1] += cnt[(size_t)r];
      const size_t base = p.rg_ents.size();
      p.rg_ents.resize(base + (size_t)A * K);
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (int a = 0; a < A; ++a) {
        const int j0 = p.origin[((size_t)c * A + a) * 2], i0 = p.origin[((size_t)c * A + a) * 2 + 1];
        for (int y = 0; y < K; ++y)
          p.rg_ents[base + (size_t)fill[(size_t)(j0 + y - ch.jmin)]++] =
              (uint32_t)a | ((uint32_t)y << 16) | ((uint32_t)i0 << 20);
      }
      for (int r = 0; r < rows; ++r) {
        p.rg_rows.push_back((int32_t)(base + (size_t)cnt[(size_t)r]));
        p.rg_rows.push_back(cnt[(size_t)r + 1] - cnt[(size_t)r]);
        p.rg_max_ants = std::max(p.rg_max_ants, cnt[(size_t)r + 1] - cnt[(size_t)r]);
      }
    }
    if (p.rg_ents.size() > (size_t)INT32_MAX) return fail(err, MOFF_E_UNSUPPORTED, "row table too large");
    // samples per time tile: 128 if the workgroup's LDS stays within 80 KB (2 per CU, the register-bound occupancy
    // of the kernel), else 64, 32 or 16 (divisors of the default 256-sample block: no short tiles)
    int nmax_rg = 0;
    for (const Chan &ch : p.chans) nmax_rg = std::max(nmax_rg, ch.n);
    const int slots = (p.rg_max_ants + 15) / 16 * 16;
    int tt = 128;
    while (tt > 16 && rowgemm_lds_bytes(nmax_rg, K, slots, tt) > 80 * 1024) tt /= 2;
    if (rowgemm_lds_bytes(nmax_rg, K, slots, tt) > 160 * 1024)
      return fail(err, MOFF_E_UNSUPPORTED, "too many antennas on one grid row for the matrix-core row pass");
    p.rg_tt = tt;
  }

  // full-grid bands of the staged 2-D FFT: every row, whatever the footprints touch
  p.fft_bands.clear();
  p.fft_band_first.assign((size_t)C + 1, 0);
  for (int c = 0; c < C; ++c) {
    const Chan &ch = p.chans[c];
    p.fft_band_first[(size_t)c] = (int32_t)p.fft_bands.size();
    for (int row0 = 0; row0 < ch.n; row0 += ch.band_rows) {
      Band bd{};
      bd.chan = c;
      bd.row0 = row0;
      bd.rows = std::min(ch.band_rows, ch.n - row0);
      bd.r_lo = row0;
      bd.r_hi = row0 + bd.rows - 1;
      p.fft_bands.push_back(bd);
    }
  }
  p.fft_band_first[(size_t)C] = (int32_t)p.fft_bands.size();
  if ((int64_t)p.fft_bands.size() > INT32_MAX / 2) return fail(err, MOFF_E_UNSUPPORTED, "too many bands");

  // ---- workspace layout (launch blocks and the row-transform buffer last) -------------------------------
  size_t off = 0;
  p.tw_sizes.clear();
  p.tw_off.clear();
  for (int c = 0; c < C; ++c)
    if (std::find(p.tw_sizes.begin(), p.tw_sizes.end(), p.chans[c].n) == p.tw_sizes.end())
      p.tw_sizes.push_back(p.chans[c].n);
  p.ws_twiddle = off;
  for (int n : p.tw_sizes) {   // twiddle tables: at most 2n entries per transform length
    p.tw_off.push_back(off);
    off = align256(off + (size_t)2 * n * 8);
  }
  p.ws_bands = off;
  off = align256(off + p.bands.size() * sizeof(Band));
  p.ws_fft_bands = off;
  off = align256(off + p.fft_bands.size() * sizeof(Band));
  p.ws_chans = off;
  off = align256(off + p.chans.size() * sizeof(Chan));
  p.ws_meta = off;
  off = align256(off + p.grp_meta.size() * 4);
  p.ws_kidx = off;
  off = align256(off + p.grp_kidx.size() * 4);
  p.ws_gchan = off;
  off = align256(off + p.grp_chan.size() * 4);
  p.ws_wk = off;
  off = align256(off + (size_t)p.n_groups * p.kplanes() * kGroupLanes * 8);
  p.ws_band_ant = off;
  off = align256(off + p.band_ant.size() * 4);
  p.ws_mfma = off;
  if (p.split_mfma()) off = align256(off + kMfmaTableBytesHost);
  p.rgtw_off.clear();
  if (p.gemm()) {
    p.ws_rg_rows = off;
    off = align256(off + p.rg_rows.size() * 4);
    p.ws_rg_ents = off;
    off = align256(off + p.rg_ents.size() * 4);
    p.ws_rk = off;
    off = align256(off + (size_t)C * A * P * K * K * 8);
    p.ws_rgtw = off;
    for (int n : p.tw_sizes) {
      p.rgtw_off.push_back(off);
      off = align256(off + (size_t)n * 8);
    }
  }
  // streaming form: kStreamXcds rings of stream_slots row-transformed samples of the largest grid, then the
  // counters [kStreamXcds][2][slots] and the error flag
  p.stream_slots = env_int("MOFF_STREAM_SLOTS", 3, 2, kStreamMaxSlots);
  p.spin_limit = (uint32_t)env_int("MOFF_SPIN_LIMIT", 1 << 22, 1 << 10, 1 << 28);
  p.pipeline = env_int("MOFF_PIPELINE", 0, 0, 1);
  p.overlap = env_int("MOFF_OVERLAP", 0, 0, 1);
  int nmax = 0;
  for (int c = 0; c < C; ++c) nmax = std::max(nmax, p.chans[c].n);
  p.ws_ring = off;
  off = align256(off + (size_t)kStreamXcds * p.stream_slots * P * nmax * nmax * 8);
  p.ws_ctr = off;
  off = align256(off + kStreamCtrBytes);
  // taps: twiddle tables (n per tap per channel), their offsets, FFT-order and centred pixel indices, and the
  // footprint origins used by the calibration solve
  if (p.n_tap > 0) {
    size_t tw = 0;
    for (int c = 0; c < C; ++c) tw += (size_t)p.n_tap * p.chans[c].n;
    p.ws_tap_tw = off;
    off = align256(off + tw * 8);
    p.ws_tap_twoff = off;
    off = align256(off + (size_t)C * 8);
    p.ws_tap_idx = off;
    off = align256(off + (size_t)C * p.n_tap * 8);
    p.ws_tap_cpix = off;
    off = align256(off + (size_t)C * p.n_tap * 8);
    p.ws_origin = off;
    off = align256(off + (size_t)C * A * 8);
  }
  p.ws_h = off;
  layout_blocks(p, tb, cpb, tg);
  return MOFF_OK;
}

size_t layout_blocks(Plan &p, int t_block, int chans_per_block, int t_group) {
  p.t_block = std::max(1, t_block);
  p.chans_per_block = std::max(1, chans_per_block);
  p.t_group = std::max(1, std::min(t_group, p.t_block));
  p.blocks.clear();
  for (int c = 0; c < p.n_chan;) {
    Block b{c, c, p.chans[c].n};
    while (b.c1 < p.n_chan && p.chans[b.c1].n == b.n && b.c1 - b.c0 < p.chans_per_block) ++b.c1;
    p.blocks.push_back(b);
    c = b.c1;
  }
  size_t hmax = 0;
  for (const Block &b : p.blocks) {
    size_t s = 0;
    for (int c = b.c0; c < b.c1; ++c) s += (size_t)p.n_pol * p.chans[c].n * p.chans[c].n * 8;
    hmax = std::max(hmax, s * (size_t)p.t_block);
  }
  p.ws_h_bytes = align256(hmax);
  // two buffers when the row pass of the next block overlaps the column pass of this one
  p.ws_total = align256(p.ws_h + p.ws_h_bytes * (p.overlap ? 2 : 1));
  return p.ws_total;
}

}  // namespace moff
