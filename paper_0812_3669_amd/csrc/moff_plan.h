// Host-side plan of the MOFF hot path: geometry, row-band binning, tap groups, launch blocks and workspace
// layout.  Pure host C++ (no HIP calls), so it also runs in processes without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "moff.h"

namespace moff {

constexpr int kStreamXcds = 8;          // XCDs of the device (the dispatcher places workgroup b on XCD b % 8)
constexpr int kStreamMaxSlots = 8;
// counters [kStreamXcds][2][kStreamMaxSlots] uint32, then the error flag (16 bytes), then the team registration:
// workgroups per XCD [kStreamXcds] and the number registered (48 bytes)
constexpr size_t kStreamCtrWords = (size_t)kStreamXcds * 2 * kStreamMaxSlots;
constexpr size_t kStreamErrWord = kStreamCtrWords, kStreamRegWord = kStreamCtrWords + 4;
constexpr size_t kStreamCtrBytes = (kStreamCtrWords + 16) * 4;

constexpr int kThreads = 256;         // threads per workgroup of every hot-path kernel
constexpr int kWaves = kThreads / 64;  // wavefronts per workgroup (64-wide on CDNA)
constexpr int kGroupLanes = 64;       // taps per scatter group (one wavefront instruction)
constexpr uint32_t kEmptyTap = 0xFFFFFFFFu;

// One grid row band of one channel that the footprints touch.  The fused row pass runs one workgroup per
// (band, time group); inside it wavefront w owns the band rows r with (r - row0) % kWaves == w.
struct Band {
  int32_t chan;
  int32_t row0;         // first grid row of the band
  int32_t rows;         // band height (<= band_rows of the channel)
  int32_t r_lo, r_hi;   // rows [r_lo, r_hi] of the band that any footprint touches (absolute)
  int64_t grp_off[kWaves];  // first tap group of each wavefront (index into the group arrays)
  int32_t grp_cnt[kWaves];
  int32_t ant_off, ant_cnt; // the band's antennas: band_ant[ant_off .. ant_off + ant_cnt), ascending
};

struct Chan {
  int32_t n;            // grid size
  int64_t pix_off;      // sum of n^2 over earlier channels
  int32_t band_rows;    // rows per band
  int32_t jmin, jmax;   // rows touched by any footprint
  int32_t band_first;   // first Band index of this channel
  int32_t band_count;
  int32_t cols;         // columns per column-pass workgroup
  int32_t col_groups;   // n / cols
  int32_t rg_first;     // matrix-core row pass: descriptor of row jmin in the row table
};

// A launch block of the fused path: consecutive channels with the same grid size.
struct Block {
  int32_t c0, c1;       // channels [c0, c1)
  int32_t n;
};

struct Plan {
  // description (copied)
  int32_t n_ant = 0, n_pol = 0, n_chan = 0, ksize = 0;
  double cell_lambda = 1.0;
  int32_t fft_mode = 0, acc_mode = 0, time_block = 0, volt_format = 0, kernel_mode = 0, n_tap = 0;
  std::vector<double> ant_xy, freq;

  // geometry
  std::vector<Chan> chans;
  std::vector<int32_t> origin;          // [C][A][2] (j0, i0)
  std::vector<Band> bands;
  // staged 2-D FFT (moff_fft): bands covering every row of each channel's grid (no tap groups), channel c's
  // at fft_band_first[c] .. fft_band_first[c + 1] - 1
  std::vector<Band> fft_bands;
  std::vector<int32_t> fft_band_first;
  std::vector<int32_t> band_ptr;        // [n_bands + 1] into band_ant
  std::vector<int32_t> band_ant;        // antennas of each band, ascending
  int32_t max_band_ants = 0;           // largest band antenna list of the sizes with a voltage table (LDS size)
  // tap groups: meta = (antenna << 16) | cell, the cell being the element offset in a pol's band grid in LDS
  // ((r - row0) * row_stride(n) + i) and the antenna its position in the band's list for sizes whose row pass
  // stages voltages (row_stages_volts), its index otherwise; kidx = a*K*K + y*K + x.  Empty lanes hold antenna 0
  // and a cell no other lane of the group uses, with kidx -1 (zero weights).
  // matrix-core row pass (MOFF_FFT_GEMM_FP16): per touched row of each channel (jmin .. jmax), (first entry, count)
  // of its antenna list; entries antenna | (row - j0) << 16 | i0 << 20, ascending antenna; the longest list, and
  // the samples per time tile the workgroup's LDS holds
  std::vector<int32_t> rg_rows;         // [rows][2]
  std::vector<uint32_t> rg_ents;
  int32_t rg_max_ants = 0, rg_tt = 0;
  std::vector<uint32_t> grp_meta;       // [G][64]
  std::vector<int32_t> grp_kidx;        // [G][64]
  std::vector<int32_t> grp_chan;        // [G] channel of each group
  int64_t n_groups = 0;

  std::vector<Block> blocks;
  int32_t chans_per_block = 16;
  int32_t t_block = 16;                 // samples per fused launch block
  int32_t t_group = 4;                  // samples per row-pass workgroup
  int32_t pipeline = 0;                 // moff_pipeline of the fused path
  int32_t overlap = 0;                  // two-pass form: row pass of block k + 1 overlaps column pass of block k (MOFF_OVERLAP=1)
  void *row_stream = nullptr;           // hipStream_t of the overlapped row passes (created on first use)
  void *ev_rows[2] = {nullptr, nullptr}, *ev_cols[2] = {nullptr, nullptr}, *ev_fork = nullptr;
  int32_t stream_slots = 3;             // ring slots per XCD (streaming form)
  uint32_t spin_limit = 1u << 22;       // bounded waits of the streaming form
  int32_t cu_count = 0;                 // compute units of the bound device
  int64_t pix_total = 0;                // sum of n_c^2

  // workspace layout (byte offsets)
  size_t ws_twiddle = 0;                // float2 tables, one per distinct n, each n entries
  std::vector<int32_t> tw_sizes;        // distinct n values in the order of the tables
  std::vector<size_t> tw_off;           // byte offset of each table
  size_t ws_bands = 0;                  // Band array (device copy)
  size_t ws_fft_bands = 0;              // full-grid bands of the staged FFT (device copy)
  size_t ws_chans = 0;                  // Chan array (device copy)
  size_t ws_meta = 0, ws_kidx = 0, ws_gchan = 0, ws_wk = 0;  // tap groups; packed kernels float2 [G][64][planes]
  size_t ws_band_ant = 0;               // band antenna lists (int32)
  size_t ws_mfma = 0;                   // split-transform matrices (split fft modes only)
  size_t ws_rg_rows = 0, ws_rg_ents = 0, ws_rk = 0, ws_rgtw = 0;   // matrix-core row pass: row table, entries,
                                        // kernels [C][A][P][K][K] with phases folded, w^m tables (one per n)
  std::vector<size_t> rgtw_off;         // byte offset of each w^m table (order of tw_sizes)
  size_t ws_ring = 0, ws_ctr = 0;       // streaming form: per-XCD ring of row-transformed samples; counters
  size_t ws_tap_tw = 0, ws_tap_twoff = 0, ws_tap_idx = 0, ws_tap_cpix = 0, ws_origin = 0;   // taps
  size_t ws_h = 0, ws_h_bytes = 0;      // row-pass output of one launch block
  size_t ws_total = 0;

  // binding state
  void *d_ws = nullptr;
  size_t ws_bound = 0;
  bool bound = false, kernels_set = false, taps_set = false;
  // tap tables staged on the host for the asynchronous upload (kept until the next moff_set_taps)
  std::vector<float> tap_tw_host;       // float2 per entry
  std::vector<int64_t> tap_twoff_host;  // [C]
  std::vector<int32_t> tap_idx_host, tap_cpix_host;   // [C][n_tap][2]

  // kernel timing (moff_profile): events are hipEvent_t stored as void*
  struct ProfRec {
    int kind;
    int64_t cs;
    void *ev0, *ev1;
  };
  bool profiling = false;
  bool capturing = false;
  struct GraphRec {
    const void *volt;
    int64_t nt;
    void *acc;
    void *graph, *exec;   // hipGraph_t, hipGraphExec_t
  };
  std::vector<GraphRec> graphs;
  void *capture_stream = nullptr;   // hipStream_t
  std::vector<ProfRec> prof;
  std::vector<void *> ev_pool;
  size_t ev_used = 0;

  int n_prod() const { return n_pol == 2 ? 4 : 1; }
  int kplanes() const { return kernel_mode == MOFF_KERNEL_JONES ? 4 : n_pol; }   // packed kernel planes
  int acc_reals() const { return n_pol == 2 ? 4 : 1; }
  size_t acc_elem_bytes() const { return acc_mode == MOFF_ACC_FP64_COMP ? 16 : 4; }
  bool gemm() const { return fft_mode == MOFF_FFT_GEMM_FP16; }
  bool split_mfma() const { return fft_mode == MOFF_FFT_SPLIT_FP16 || fft_mode == MOFF_FFT_SPLIT_BF16; }
  size_t volt_sample_bytes() const {  // one time sample, all channels
    return (size_t)n_chan * n_ant * n_pol * (volt_format == MOFF_VOLT_INT8 ? 2 : 8);
  }
};

// Builds the plan; on error returns a status and sets *err.
moff_status build_plan(const moff_plan_desc &d, Plan &p, std::string *err);

// Launch blocks and the row-transform buffer for a launch shape; returns the workspace bytes it needs.
size_t layout_blocks(Plan &p, int t_block, int chans_per_block, int t_group);

// True if the library has an FFT pipeline for grid size n.
bool fft_size_supported(int n);
int band_rows_for(int n, int P);
int cols_for(int n);
int smallest_supported_size(int need);
// LDS bytes of one matrix-core row-pass workgroup: w^m table, taps, first columns and antennas of `slots` antenna
// slots, `tt` samples of FP16 voltages per slot (row stride slots + 4 words) and one float per wavefront.
size_t rowgemm_lds_bytes(int n, int K, int slots, int tt);

}  // namespace moff
