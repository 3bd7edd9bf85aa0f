// C ABI of the MOFF hot path (declared in include/moff.h): validation on the host, then kernel launches on the
// caller's stream.  Device memory is always caller-owned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <exception>
#include <fstream>
#include <map>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "moff.h"
#include "moff_plan.h"

struct moff_plan_s {
  moff::Plan p;
};

namespace {

thread_local std::string g_err;

moff_status set_err(moff_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

moff_status ok() {
  g_err.clear();
  return MOFF_OK;
}

moff_status hip_fail(hipError_t e, const char *what) {
  return set_err(MOFF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

char *ws(const moff::Plan &p, size_t off) { return static_cast<char *>(p.d_ws) + off; }

const moff::Band *d_bands(const moff::Plan &p) { return reinterpret_cast<const moff::Band *>(ws(p, p.ws_bands)); }
const moff::Chan *d_chans(const moff::Plan &p) { return reinterpret_cast<const moff::Chan *>(ws(p, p.ws_chans)); }

const float2 *d_tw(const moff::Plan &p, int n) {
  for (size_t i = 0; i < p.tw_sizes.size(); ++i)
    if (p.tw_sizes[i] == n) return reinterpret_cast<const float2 *>(ws(p, p.tw_off[i]));
  return nullptr;
}

const float2 *d_rgtw(const moff::Plan &p, int n) {
  for (size_t i = 0; i < p.tw_sizes.size() && i < p.rgtw_off.size(); ++i)
    if (p.tw_sizes[i] == n) return reinterpret_cast<const float2 *>(ws(p, p.rgtw_off[i]));
  return nullptr;
}

moff_status need_bound(const moff::Plan &p, bool kernels) {
  if (!p.bound) return set_err(MOFF_E_STATE, "plan is not bound to a workspace (moff_bind)");
  if (kernels && !p.kernels_set) return set_err(MOFF_E_STATE, "kernels are not set (moff_set_kernels)");
  return MOFF_OK;
}

bool is_jones(const moff::Plan &p) { return p.kernel_mode == MOFF_KERNEL_JONES; }

moff::RowArgs row_args(const moff::Plan &p, const void *volt) {
  moff::RowArgs a{};
  a.bands = d_bands(p);
  a.chans = d_chans(p);
  a.n_chan = p.n_chan;
  a.n_ant = p.n_ant;
  a.volt = volt;
  a.volt_fmt = p.volt_format;
  a.meta = reinterpret_cast<const uint32_t *>(ws(p, p.ws_meta));
  a.band_ant = reinterpret_cast<const int32_t *>(ws(p, p.ws_band_ant));
  a.band_ants_max = p.max_band_ants;
  a.wk = reinterpret_cast<const float2 *>(ws(p, p.ws_wk));
  a.t_group = p.t_group;
  a.t_block = p.t_block;
  a.sample_stride = (int64_t)p.n_pol * p.pix_total;
  return a;
}

// Event pair around one launch when profiling is on.
struct ProfScope {
  moff::Plan &p;
  hipStream_t st;
  moff::Plan::ProfRec rec{};
  bool on;
  hipError_t err = hipSuccess;
  ProfScope(moff::Plan &pl, hipStream_t s, int kind, int64_t cs) : p(pl), st(s), on(pl.profiling && !pl.capturing) {
    if (!on) return;
    rec.kind = kind;
    rec.cs = cs;
    rec.ev0 = take();
    rec.ev1 = take();
    if (rec.ev0 && rec.ev1) err = hipEventRecord(static_cast<hipEvent_t>(rec.ev0), st);
  }
  void *take() {
    if (p.ev_used == p.ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      p.ev_pool.push_back(e);
    }
    return p.ev_pool[p.ev_used++];
  }
  hipError_t done() {
    if (!on || !rec.ev0 || !rec.ev1) return err;
    if (err == hipSuccess) err = hipEventRecord(static_cast<hipEvent_t>(rec.ev1), st);
    if (err == hipSuccess) p.prof.push_back(rec);
    return err;
  }
};

int band_begin(const moff::Plan &p, const moff::Block &b) { return p.chans[b.c0].band_first; }
int band_count(const moff::Plan &p, const moff::Block &b) {
  return p.chans[b.c1 - 1].band_first + p.chans[b.c1 - 1].band_count - p.chans[b.c0].band_first;
}

// Internal stream (default priority) and events of the overlapped two-pass form, created on first use.
moff_status ensure_overlap(moff::Plan &p) {
  if (p.row_stream) return MOFF_OK;
  hipStream_t s;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "row stream");
  p.row_stream = s;
  void **evs[5] = {&p.ev_rows[0], &p.ev_rows[1], &p.ev_cols[0], &p.ev_cols[1], &p.ev_fork};
  for (void **e : evs) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "overlap event");
    *e = ev;
  }
  return MOFF_OK;
}

struct Exchange;
moff_status enqueue_two_pass(moff::Plan &p, const void *d_volt, int64_t n_t, void *d_acc, hipStream_t st, int c_lo,
                             int c_hi, void *d_tap = nullptr, const Exchange *ex = nullptr);

// Streaming form: per run of channels with one grid size, clear the counters and launch the persistent kernel
// sized to the device's occupancy (all its workgroups resident at once).
moff_status enqueue_stream(moff::Plan &p, const void *d_volt, int64_t n_t, void *d_acc, hipStream_t st) {
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  const bool jones = is_jones(p);
  moff::StreamArgs s{};
  s.r = row_args(p, d_volt);
  s.r.t0 = 0;
  s.r.nt = (int)n_t;
  s.c.chans = d_chans(p);
  s.c.acc = d_acc;
  s.c.t_block = p.t_block;
  s.c.t0 = 0;
  s.c.nt = (int)n_t;
  uint32_t *ctr = reinterpret_cast<uint32_t *>(ws(p, p.ws_ctr));
  s.ring = reinterpret_cast<float2 *>(ws(p, p.ws_ring));
  s.ctr = ctr;
  s.err = reinterpret_cast<int *>(ctr + moff::kStreamErrWord);
  s.slots = p.stream_slots;
  s.spin_limit = p.spin_limit;
  HIP_TRY(moff::launch_fill_zero(ctr, moff::kStreamCtrBytes, st), "clear stream counters");
  for (int c0 = 0; c0 < p.n_chan;) {
    const int n = p.chans[c0].n;
    int c1 = c0;
    while (c1 < p.n_chan && p.chans[c1].n == n) ++c1;
    int occ = 0;
    HIP_TRY(moff::stream_occupancy(n, p.n_pol, p.acc_mode, jones, p.max_band_ants, p.volt_format, &occ),
            "stream occupancy");
    const int per_xcd = occ * (p.cu_count / moff::kStreamXcds);
    const int owners = n / p.chans[c0].cols;
    if (per_xcd < owners + owners / 2) {
      // too few resident workgroups for column owners plus row workers: this grid size runs two-pass
      moff_status r = enqueue_two_pass(p, d_volt, n_t, d_acc, st, c0, c1);
      if (r) return r;
      c0 = c1;
      continue;
    }
    if (c0 > 0) {   // slot counters and team registration for this launch (the error flag stays)
      HIP_TRY(moff::launch_fill_zero(ctr, moff::kStreamCtrWords * 4, st), "clear stream counters");
      HIP_TRY(moff::launch_fill_zero(ctr + moff::kStreamRegWord, 48, st), "clear stream counters");
    }
    s.r.c0 = s.c.c0 = c0;
    s.r.tw = s.c.tw = d_tw(p, n);
    s.n_chan_group = c1 - c0;
    s.wgs_per_xcd = per_xcd;
    {
      ProfScope ps(p, st, 2, n_t * (c1 - c0));
      HIP_TRY(moff::launch_stream(n, p.n_pol, p.acc_mode, jones, s, st), "streaming pass");
      HIP_TRY(ps.done(), "profile event");
    }
    c0 = c1;
  }
  return MOFF_OK;
}

// Where the two-pass form puts the row-transformed grids of a launch block: by default the workspace's
// exchange region (p.t_block samples of one of the plan's channel blocks); the no-alloc entry point passes a
// fixed buffer of `bytes`, and the launch blocks are cut (channels, then samples) so that one fits it.
struct Exchange {
  float2 *base;
  size_t bytes;
};

// Two-pass form for the channels [c_lo, c_hi) (a union of launch blocks).
moff_status enqueue_two_pass(moff::Plan &p, const void *d_volt, int64_t n_t, void *d_acc, hipStream_t st, int c_lo,
                             int c_hi, void *d_tap, const Exchange *ex) {
  float2 *H0 = ex ? ex->base : reinterpret_cast<float2 *>(ws(p, p.ws_h));
  const bool jones = is_jones(p);
  moff::RowArgs a = row_args(p, d_volt);
  moff::ColArgs ca{};
  ca.chans = d_chans(p);
  ca.acc = d_acc;
  // Overlap: the row passes run on an internal stream, block k into buffer k % 2, while the column pass of
  // block k - 1 runs on the caller's stream; events order rows(k) -> cols(k) and cols(k - 2) -> rows(k).
  const bool dual = p.overlap != 0 && !ex;
  hipStream_t rs = st;
  if (dual) {
    moff_status r = ensure_overlap(p);
    if (r) return r;
    rs = static_cast<hipStream_t>(p.row_stream);
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(p.ev_fork), st), "fork event");
    HIP_TRY(hipStreamWaitEvent(rs, static_cast<hipEvent_t>(p.ev_fork), 0), "fork wait");
  }
  const bool split = p.split_mfma();
  const int bf16 = p.fft_mode == MOFF_FFT_SPLIT_BF16;
  const uint16_t *mtab = reinterpret_cast<const uint16_t *>(ws(p, p.ws_mfma));
  int64_t k = 0;
  // one launch block: channels [b.c0, b.c1) x samples [t0, t0 + nt), the exchange holding `tblk` samples per channel
  auto one_block = [&](const moff::Block &b, int64_t t0, int nt, int tblk) -> moff_status {
    const int slot = dual ? (int)(k % 2) : 0;
    float2 *H = H0 + (size_t)slot * (p.ws_h_bytes / sizeof(float2));
    a.io = H;
    ca.in = H;
    a.t_block = ca.t_block = tblk;
    if (dual && k >= 2)
      HIP_TRY(hipStreamWaitEvent(rs, static_cast<hipEvent_t>(p.ev_cols[slot]), 0), "buffer reuse wait");
    a.band_begin = band_begin(p, b);
    a.n_bands = band_count(p, b);
    a.c0 = b.c0;
    a.n_chan_block = b.c1 - b.c0;
    a.t0 = (int)t0;
    a.nt = nt;
    a.tw = d_tw(p, b.n);
    const int tgroups = (nt + p.t_group - 1) / p.t_group;
    const size_t lds = moff::rows_lds_bytes(b.n, p.n_pol, p.chans[b.c0].band_rows, p.max_band_ants, p.volt_format);
    const int64_t cs = (int64_t)nt * (b.c1 - b.c0);
    {
      ProfScope ps(p, rs, 0, cs);
      const int rgrid = moff::rows_xcd_grid(p, b, tgroups);
      if (p.gemm()) {
        moff::RgArgs g{};
        g.chans = d_chans(p);
        g.rows = reinterpret_cast<const int32_t *>(ws(p, p.ws_rg_rows));
        g.ents = reinterpret_cast<const uint32_t *>(ws(p, p.ws_rg_ents));
        g.rk = reinterpret_cast<const float2 *>(ws(p, p.ws_rk));
        g.tw = d_rgtw(p, b.n);
        g.volt = d_volt;
        g.io = H;
        g.c0 = b.c0;
        g.n_chan_block = b.c1 - b.c0;
        g.t0 = (int)t0;
        g.nt = nt;
        g.t_block = tblk;
        g.n_chan = p.n_chan;
        g.n_ant = p.n_ant;
        g.K = p.ksize;
        g.P = p.n_pol;
        g.tt = p.rg_tt;
        g.slots = (p.rg_max_ants + 15) / 16 * 16;
        HIP_TRY(moff::launch_rowgemm(b.n, g, moff::rowgemm_grid(p, b, nt), rs), "row pass");
      } else if (split)
        HIP_TRY(moff::launch_rows_mfma(bf16, a, mtab, rgrid, rs), "row pass");
      else
        HIP_TRY(moff::launch_rows(b.n, p.n_pol, moff::ROW_MODE_FUSED, jones, a, rgrid, lds, rs), "row pass");
      HIP_TRY(ps.done(), "profile event");
    }
    if (d_tap) {
      // E-field image at the tapped pixels, from this block's row-transformed samples
      moff::TapArgs ta{};
      ta.chans = d_chans(p);
      ta.h = H;
      ta.tap_tw = reinterpret_cast<const float2 *>(ws(p, p.ws_tap_tw));
      ta.tap_tw_off = reinterpret_cast<const int64_t *>(ws(p, p.ws_tap_twoff));
      ta.tap_idx = reinterpret_cast<const int2 *>(ws(p, p.ws_tap_idx));
      ta.out = static_cast<float2 *>(d_tap);
      ta.c0 = b.c0;
      ta.n_chan_block = b.c1 - b.c0;
      ta.t0 = (int)t0;
      ta.nt = nt;
      ta.t_block = tblk;
      ta.n_chan = p.n_chan;
      ta.n_tap = p.n_tap;
      ta.P = p.n_pol;
      HIP_TRY(moff::launch_tap(ta, rs), "tap");
    }
    if (dual) {
      HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(p.ev_rows[slot]), rs), "row event");
      HIP_TRY(hipStreamWaitEvent(st, static_cast<hipEvent_t>(p.ev_rows[slot]), 0), "row wait");
    }
    const int W = p.chans[b.c0].cols;
    ca.c0 = b.c0;
    ca.t0 = (int)t0;
    ca.nt = nt;
    ca.tw = a.tw;
    const int grid = moff::cols_xcd_grid(b, b.n / W);
    ca.n_chan_block = b.c1 - b.c0;
    {
      ProfScope ps(p, st, 1, cs);
      if (split)
        HIP_TRY(moff::launch_cols_mfma(bf16, p.acc_mode, ca, mtab, grid, st), "column pass");
      else
        HIP_TRY(moff::launch_cols(b.n, p.n_pol, W, moff::COL_MODE_FUSED, p.acc_mode, ca, grid, 1,
                                  moff::cols_lds_bytes(b.n, p.n_pol, W), st),
                "column pass");
      HIP_TRY(ps.done(), "profile event");
    }
    if (dual) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(p.ev_cols[slot]), st), "column event");
    ++k;
    return MOFF_OK;
  };
  if (!ex) {
    for (int64_t t0 = 0; t0 < n_t; t0 += p.t_block) {
      const int nt = (int)std::min<int64_t>(p.t_block, n_t - t0);
      for (const moff::Block &b : p.blocks) {
        if (b.c0 < c_lo || b.c1 > c_hi) continue;
        moff_status r = one_block(b, t0, nt, p.t_block);
        if (r) return r;
      }
    }
    return MOFF_OK;
  }
  // fixed exchange buffer: each plan block is cut into channel runs whose one sample fits it, and each run takes
  // as many samples per launch block as fit (at most the plan's time block)
  for (const moff::Block &b : p.blocks) {
    if (b.c0 < c_lo || b.c1 > c_hi) continue;
    const size_t per_cs = (size_t)p.n_pol * b.n * b.n * 8;   // one channel-sample of row-transformed grids
    const int c_run = (int)std::min<size_t>((size_t)(b.c1 - b.c0), ex->bytes / per_cs);
    if (c_run < 1) return set_err(MOFF_E_UNSUPPORTED, "one channel-sample needs more than the exchange buffer");
    for (int c0 = b.c0; c0 < b.c1; c0 += c_run) {
      const moff::Block sb{c0, std::min(b.c1, c0 + c_run), b.n};
      const int tblk = (int)std::min<size_t>((size_t)p.t_block, ex->bytes / (per_cs * (size_t)(sb.c1 - sb.c0)));
      for (int64_t t0 = 0; t0 < n_t; t0 += tblk) {
        moff_status r = one_block(sb, t0, (int)std::min<int64_t>(tblk, n_t - t0), tblk);
        if (r) return r;
      }
    }
  }
  return MOFF_OK;
}

moff_status enqueue_correlate(moff::Plan &p, const void *d_volt, int64_t n_t, void *d_acc, hipStream_t st) {
  if (p.pipeline == MOFF_PIPELINE_STREAM && p.fft_mode == MOFF_FFT_FP32) return enqueue_stream(p, d_volt, n_t, d_acc, st);
  return enqueue_two_pass(p, d_volt, n_t, d_acc, st, 0, p.n_chan);
}

void drop_graphs(moff::Plan &p) {
  for (auto &g : p.graphs) {
    (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(g.exec));
    (void)hipGraphDestroy(static_cast<hipGraph_t>(g.graph));
  }
  p.graphs.clear();
}

}  // namespace

extern "C" {

moff_status moff_probe(int32_t kind, int32_t blocks, int32_t iters, float *d_out, void *stream) {
  if (kind < 0 || kind > 6 || blocks < 1 || iters < 1 || !d_out)
    return set_err(MOFF_E_INVALID, "bad probe arguments");
  HIP_TRY(moff::launch_probe(kind, blocks, iters, d_out, static_cast<hipStream_t>(stream)), "probe");
  return MOFF_OK;
}

const char *moff_status_str(moff_status s) {
  switch (s) {
    case MOFF_OK: return "MOFF_OK";
    case MOFF_E_INVALID: return "MOFF_E_INVALID";
    case MOFF_E_BUDGET: return "MOFF_E_BUDGET";
    case MOFF_E_DEVICE: return "MOFF_E_DEVICE";
    case MOFF_E_UNSUPPORTED: return "MOFF_E_UNSUPPORTED";
    case MOFF_E_STATE: return "MOFF_E_STATE";
  }
  return "MOFF_E_UNKNOWN";
}

const char *moff_last_error(void) { return g_err.c_str(); }

moff_status moff_plan(const moff_plan_desc *desc, moff_plan_t *out) {
  if (!desc || !out) return set_err(MOFF_E_INVALID, "null argument");
  moff_plan_s *h = new (std::nothrow) moff_plan_s();
  if (!h) return set_err(MOFF_E_INVALID, "out of host memory");
  std::string err;
  moff_status s;
  try {
    s = moff::build_plan(*desc, h->p, &err);
  } catch (const std::exception &ex) {   // host allocation or thread creation failed: no exception crosses the C ABI
    s = MOFF_E_INVALID;
    err = std::string("plan build failed on the host: ") + ex.what();
  }
  if (s != MOFF_OK) {
    delete h;
    return set_err(s, err);
  }
  const moff::Plan &p = h->p;
  for (const moff::Chan &c : p.chans) {
    if (moff::rows_lds_bytes(c.n, p.n_pol, c.band_rows, p.max_band_ants, p.volt_format) > (size_t)moff::kMaxLds ||
        moff::cols_lds_bytes(c.n, p.n_pol, c.cols) > (size_t)moff::kMaxLds) {
      delete h;
      return set_err(MOFF_E_UNSUPPORTED, "grid size needs more LDS than a CU has");
    }
  }
  *out = h;
  return ok();
}

void moff_plan_destroy(moff_plan_t plan) {
  if (!plan) return;
  drop_graphs(plan->p);
  if (plan->p.capture_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(plan->p.capture_stream));
  if (plan->p.row_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(plan->p.row_stream));
  for (void *e : {plan->p.ev_rows[0], plan->p.ev_rows[1], plan->p.ev_cols[0], plan->p.ev_cols[1], plan->p.ev_fork})
    if (e) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  for (void *e : plan->p.ev_pool) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  delete plan;
}

moff_status moff_workspace_size(moff_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return set_err(MOFF_E_INVALID, "null argument");
  *bytes = plan->p.ws_total;
  return ok();
}

moff_status moff_acc_size(moff_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return set_err(MOFF_E_INVALID, "null argument");
  const moff::Plan &p = plan->p;
  *bytes = (size_t)p.pix_total * p.acc_reals() * p.acc_elem_bytes();
  return ok();
}

moff_status moff_image_size(moff_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return set_err(MOFF_E_INVALID, "null argument");
  *bytes = (size_t)plan->p.pix_total * plan->p.n_prod() * 8;
  return ok();
}

moff_status moff_grid_n(moff_plan_t plan, int32_t chan, int32_t *n) {
  if (!plan || !n) return set_err(MOFF_E_INVALID, "null argument");
  if (chan < 0 || chan >= plan->p.n_chan) return set_err(MOFF_E_INVALID, "channel out of range");
  *n = plan->p.chans[chan].n;
  return ok();
}

moff_status moff_chan_offset(moff_plan_t plan, int32_t chan, int64_t *pix_off) {
  if (!plan || !pix_off) return set_err(MOFF_E_INVALID, "null argument");
  if (chan < 0 || chan >= plan->p.n_chan) return set_err(MOFF_E_INVALID, "channel out of range");
  *pix_off = plan->p.chans[chan].pix_off;
  return ok();
}

moff_status moff_bind(moff_plan_t plan, void *d_ws, size_t bytes, void *stream) {
  if (!plan || !d_ws) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  if (bytes < p.ws_total) return set_err(MOFF_E_BUDGET, "workspace smaller than moff_workspace_size");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return set_err(MOFF_E_INVALID, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  drop_graphs(p);
  p.d_ws = d_ws;
  p.ws_bound = bytes;
  p.bound = false;
  p.kernels_set = false;
  if (!p.bands.empty())
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_bands), p.bands.data(), p.bands.size() * sizeof(moff::Band),
                           hipMemcpyHostToDevice, st), "upload bands");
  if (!p.fft_bands.empty())
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_fft_bands), p.fft_bands.data(), p.fft_bands.size() * sizeof(moff::Band),
                           hipMemcpyHostToDevice, st), "upload full-grid bands");
  HIP_TRY(hipMemcpyAsync(ws(p, p.ws_chans), p.chans.data(), p.chans.size() * sizeof(moff::Chan),
                         hipMemcpyHostToDevice, st), "upload channels");
  if (p.n_groups) {
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_meta), p.grp_meta.data(), p.grp_meta.size() * 4, hipMemcpyHostToDevice, st),
            "upload tap groups");
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_kidx), p.grp_kidx.data(), p.grp_kidx.size() * 4, hipMemcpyHostToDevice, st),
            "upload tap indices");
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_gchan), p.grp_chan.data(), p.grp_chan.size() * 4, hipMemcpyHostToDevice, st),
            "upload group channels");
  }
  if (!p.band_ant.empty())
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_band_ant), p.band_ant.data(), p.band_ant.size() * 4, hipMemcpyHostToDevice,
                           st),
            "upload band antenna lists");
  for (size_t i = 0; i < p.tw_sizes.size(); ++i)
    HIP_TRY(moff::launch_twiddle(reinterpret_cast<float2 *>(ws(p, p.tw_off[i])), p.tw_sizes[i], st), "twiddles");
  if (p.split_mfma())
    HIP_TRY(moff::launch_mfma_table(reinterpret_cast<uint16_t *>(ws(p, p.ws_mfma)),
                                    p.fft_mode == MOFF_FFT_SPLIT_BF16, st),
            "split-transform matrices");
  if (p.gemm()) {
    if (!p.rg_rows.empty())
      HIP_TRY(hipMemcpyAsync(ws(p, p.ws_rg_rows), p.rg_rows.data(), p.rg_rows.size() * 4, hipMemcpyHostToDevice, st),
              "upload row table");
    if (!p.rg_ents.empty())
      HIP_TRY(hipMemcpyAsync(ws(p, p.ws_rg_ents), p.rg_ents.data(), p.rg_ents.size() * 4, hipMemcpyHostToDevice, st),
              "upload row entries");
    for (size_t i = 0; i < p.tw_sizes.size(); ++i)
      HIP_TRY(moff::launch_rg_twiddle(reinterpret_cast<float2 *>(ws(p, p.rgtw_off[i])), p.tw_sizes[i], st),
              "row-pass twiddles");
  }
  if (p.n_tap > 0)
    HIP_TRY(hipMemcpyAsync(ws(p, p.ws_origin), p.origin.data(), p.origin.size() * 4, hipMemcpyHostToDevice, st),
            "upload footprint origins");
  p.taps_set = false;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "device");
  HIP_TRY(hipDeviceGetAttribute(&p.cu_count, hipDeviceAttributeMultiprocessorCount, dev), "compute units");
  p.bound = true;
  return ok();
}

moff_status moff_set_kernels_phased(moff_plan_t plan, const void *d_kern, const void *d_phase, void *stream) {
  if (!plan || !d_kern) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  HIP_TRY(moff::launch_pack_kernels(static_cast<const float2 *>(d_kern), static_cast<const float2 *>(d_phase),
                                    reinterpret_cast<const int32_t *>(ws(p, p.ws_kidx)),
                                    reinterpret_cast<const int32_t *>(ws(p, p.ws_gchan)),
                                    reinterpret_cast<float2 *>(ws(p, p.ws_wk)), p.n_groups, p.n_ant, p.n_pol,
                                    p.ksize * p.ksize, p.kplanes(), static_cast<hipStream_t>(stream)),
          "pack kernels");
  if (p.gemm())
    HIP_TRY(moff::launch_pack_rk(static_cast<const float2 *>(d_kern), static_cast<const float2 *>(d_phase),
                                 reinterpret_cast<float2 *>(ws(p, p.ws_rk)),
                                 (int64_t)p.n_chan * p.n_ant * p.n_pol * p.ksize * p.ksize, p.ksize * p.ksize,
                                 static_cast<hipStream_t>(stream)),
            "pack row-pass kernels");
  p.kernels_set = true;
  return ok();
}

moff_status moff_set_kernels(moff_plan_t plan, const void *d_kern, void *stream) {
  return moff_set_kernels_phased(plan, d_kern, nullptr, stream);
}

moff_status moff_grid(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_grid, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && (!d_volt || !d_grid)) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  if (n_t == 0) return ok();
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(moff::launch_fill_zero(d_grid, (size_t)n_t * p.n_pol * p.pix_total * 8, st), "clear grid");
  const bool jones = is_jones(p);
  moff::RowArgs a = row_args(p, d_volt);
  a.io = static_cast<float2 *>(d_grid);
  a.t0 = 0;
  a.nt = (int)n_t;
  for (const moff::Block &b : p.blocks) {
    a.band_begin = band_begin(p, b);
    a.n_bands = band_count(p, b);
    a.c0 = b.c0;
    a.tw = d_tw(p, b.n);
    const int tgroups = (int)((n_t + p.t_group - 1) / p.t_group);
    const size_t lds = moff::rows_lds_bytes(b.n, p.n_pol, p.chans[b.c0].band_rows, p.max_band_ants, p.volt_format);
    HIP_TRY(moff::launch_rows(b.n, p.n_pol, moff::ROW_MODE_GRID, jones, a, a.n_bands * tgroups, lds, st), "grid");
  }
  return ok();
}

moff_status moff_fft(moff_plan_t plan, void *d_grid, int64_t n_t, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && !d_grid) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  if (n_t == 0) return ok();
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // every row and column is transformed (the full-grid bands, no footprint row range): the grids may hold data
  // anywhere
  moff::RowArgs a = row_args(p, nullptr);
  a.bands = reinterpret_cast<const moff::Band *>(ws(p, p.ws_fft_bands));
  a.io = static_cast<float2 *>(d_grid);
  a.t0 = 0;
  a.nt = (int)n_t;
  moff::ColArgs ca{};
  ca.chans = d_chans(p);
  ca.in = static_cast<const float2 *>(d_grid);
  ca.out = static_cast<float2 *>(d_grid);
  ca.t0 = 0;
  ca.nt = (int)n_t;
  ca.t_block = 0;
  ca.sample_stride = (int64_t)p.n_pol * p.pix_total;
  ca.full_rows = 1;
  for (const moff::Block &b : p.blocks) {
    a.band_begin = p.fft_band_first[b.c0];
    a.n_bands = p.fft_band_first[b.c1] - p.fft_band_first[b.c0];
    a.c0 = b.c0;
    a.tw = d_tw(p, b.n);
    const int tgroups = (int)((n_t + p.t_group - 1) / p.t_group);
    const size_t lds = moff::rows_lds_bytes(b.n, p.n_pol, p.chans[b.c0].band_rows, p.max_band_ants, p.volt_format);
    HIP_TRY(moff::launch_rows(b.n, p.n_pol, moff::ROW_MODE_FFT, false, a, a.n_bands * tgroups, lds, st), "row fft");
  }
  // samples spread over the second grid dimension (at most 65535 workgroups there; each workgroup then transforms
  // its column group for a run of consecutive samples)
  const int gridy = (int)std::min<int64_t>(n_t, 65535);
  for (const moff::Block &b : p.blocks) {
    const int W = p.chans[b.c0].cols;
    ca.c0 = b.c0;
    ca.tw = d_tw(p, b.n);
    const int grid = (b.c1 - b.c0) * (b.n / W);
    HIP_TRY(moff::launch_cols(b.n, p.n_pol, W, moff::COL_MODE_FFT, 0, ca, grid, gridy,
                              moff::cols_lds_bytes(b.n, p.n_pol, W), st),
            "column fft");
  }
  return ok();
}

moff_status moff_accumulate(moff_plan_t plan, const void *d_efield, int64_t n_t, void *d_acc, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && (!d_efield || !d_acc)) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  if (n_t == 0) return ok();
  moff::AccArgs a{};
  a.chans = d_chans(p);
  a.n_chan = p.n_chan;
  a.pix_total = p.pix_total;
  a.nt = n_t;
  a.efield = static_cast<const float2 *>(d_efield);
  a.sample_stride = (int64_t)p.n_pol * p.pix_total;
  a.acc = d_acc;
  HIP_TRY(moff::launch_acc_staged(p.n_pol, p.acc_mode, a, static_cast<hipStream_t>(stream)), "accumulate");
  return ok();
}

moff_status moff_correlate(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && (!d_volt || !d_acc)) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  if (n_t == 0) return ok();
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  s = enqueue_correlate(p, d_volt, n_t, d_acc, static_cast<hipStream_t>(stream));
  return s ? s : ok();
}

moff_status moff_correlate_noalloc(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && (!d_volt || !d_acc)) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  // the largest channel-sample of row-transformed grids must fit the library's buffer
  for (const moff::Chan &c : p.chans)
    if ((size_t)p.n_pol * c.n * c.n * 8 > moff::kNoallocExchangeBytes)
      return set_err(MOFF_E_UNSUPPORTED, "a channel-sample of this plan needs more than the " +
                                             std::to_string(moff::kNoallocExchangeBytes >> 20) +
                                             " MiB exchange buffer of moff_correlate_noalloc");
  if (n_t == 0) return ok();
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  Exchange ex{};
  void *buf = nullptr;
  HIP_TRY(moff::noalloc_exchange(&buf, &ex.bytes), "exchange buffer address");
  ex.base = static_cast<float2 *>(buf);
  s = enqueue_two_pass(p, d_volt, n_t, d_acc, static_cast<hipStream_t>(stream), 0, p.n_chan, nullptr, &ex);
  return s ? s : ok();
}

moff_status moff_correlate_graph(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > 0 && (!d_volt || !d_acc)) return set_err(MOFF_E_INVALID, "null buffer");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  if (n_t == 0) return ok();
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  if (p.profiling) return set_err(MOFF_E_STATE, "graph replay while kernel timing is on");
  moff::Plan::GraphRec *g = nullptr;
  for (auto &r : p.graphs)
    if (r.volt == d_volt && r.nt == n_t && r.acc == d_acc) g = &r;
  if (!g) {
    if (!p.capture_stream) {
      hipStream_t cs;
      HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
      p.capture_stream = cs;
    }
    hipStream_t cs = static_cast<hipStream_t>(p.capture_stream);
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    p.capturing = true;
    moff_status es = enqueue_correlate(p, d_volt, n_t, d_acc, cs);
    p.capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (es) {
      if (graph) (void)hipGraphDestroy(graph);
      return es;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "instantiate graph");
    }
    p.graphs.push_back({d_volt, n_t, d_acc, graph, exec});
    g = &p.graphs.back();
  }
  HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(g->exec), static_cast<hipStream_t>(stream)), "graph launch");
  return ok();
}

moff_status moff_workspace_size_for(moff_plan_t plan, int32_t time_block, int32_t chans_per_block, size_t *bytes) {
  if (!plan || !bytes) return set_err(MOFF_E_INVALID, "null argument");
  if (time_block < 1 || chans_per_block < 1) return set_err(MOFF_E_INVALID, "launch shape must be >= 1");
  moff::Plan &p = plan->p;
  const int tb = p.t_block, cpb = p.chans_per_block, tg = p.t_group;
  *bytes = moff::layout_blocks(p, time_block, chans_per_block, tg);
  moff::layout_blocks(p, tb, cpb, tg);
  return ok();
}

moff_status moff_set_launch_shape(moff_plan_t plan, int32_t time_block, int32_t chans_per_block, int32_t time_group) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (time_block < 1 || chans_per_block < 1 || time_group < 1)
    return set_err(MOFF_E_INVALID, "launch shape must be >= 1");
  moff::Plan &p = plan->p;
  const int tb = p.t_block, cpb = p.chans_per_block, tg = p.t_group;
  const size_t need = moff::layout_blocks(p, time_block, chans_per_block, time_group);
  if (p.bound && need > p.ws_bound) {
    moff::layout_blocks(p, tb, cpb, tg);
    return set_err(MOFF_E_BUDGET, "bound workspace too small for this launch shape");
  }
  drop_graphs(p);
  return ok();
}

moff_status moff_set_taps(moff_plan_t plan, const int32_t *h_pix, void *stream) {
  if (!plan || !h_pix) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  if (p.n_tap <= 0) return set_err(MOFF_E_STATE, "the plan was made with n_tap = 0");
  const int C = p.n_chan, M = p.n_tap;
  for (int c = 0; c < C; ++c)
    for (int m = 0; m < M; ++m)
      for (int k = 0; k < 2; ++k) {
        const int v = h_pix[((size_t)c * M + m) * 2 + k];
        if (v < 0 || v >= p.chans[c].n) return set_err(MOFF_E_INVALID, "tap pixel outside the channel's image");
      }
  // twiddles exp(+2 pi i j qr / n) of each tap's row index, in FP64 with the angle reduced in integers
  p.tap_tw_host.clear();
  p.tap_twoff_host.assign(C, 0);
  p.tap_idx_host.assign((size_t)C * M * 2, 0);
  p.tap_cpix_host.assign(h_pix, h_pix + (size_t)C * M * 2);
  int64_t off = 0;
  for (int c = 0; c < C; ++c) {
    const int n = p.chans[c].n;
    p.tap_twoff_host[c] = off;
    for (int m = 0; m < M; ++m) {
      const int row = h_pix[((size_t)c * M + m) * 2], col = h_pix[((size_t)c * M + m) * 2 + 1];
      const int qr = (row + n / 2) % n, qc = (col + n / 2) % n;   // FFT order of the centred pixel
      p.tap_idx_host[((size_t)c * M + m) * 2] = qr;
      p.tap_idx_host[((size_t)c * M + m) * 2 + 1] = qc;
      for (int j = 0; j < n; ++j) {
        const long long r = ((long long)j * qr) % n;
        const double ang = 2.0 * M_PI * (double)r / (double)n;
        p.tap_tw_host.push_back((float)std::cos(ang));
        p.tap_tw_host.push_back((float)std::sin(ang));
      }
      off += n;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(ws(p, p.ws_tap_tw), p.tap_tw_host.data(), p.tap_tw_host.size() * 4, hipMemcpyHostToDevice,
                         st), "upload tap twiddles");
  HIP_TRY(hipMemcpyAsync(ws(p, p.ws_tap_twoff), p.tap_twoff_host.data(), (size_t)C * 8, hipMemcpyHostToDevice, st),
          "upload tap offsets");
  HIP_TRY(hipMemcpyAsync(ws(p, p.ws_tap_idx), p.tap_idx_host.data(), p.tap_idx_host.size() * 4,
                         hipMemcpyHostToDevice, st), "upload tap indices");
  HIP_TRY(hipMemcpyAsync(ws(p, p.ws_tap_cpix), p.tap_cpix_host.data(), p.tap_cpix_host.size() * 4,
                         hipMemcpyHostToDevice, st), "upload tap pixels");
  p.taps_set = true;
  return ok();
}

moff_status moff_correlate_tap(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *d_tap,
                               void *stream) {
  if (!plan || !d_volt || !d_acc || !d_tap) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  if (!p.taps_set) return set_err(MOFF_E_STATE, "taps are not set (moff_set_taps)");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  if (n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t too large for one call");
  return enqueue_two_pass(p, d_volt, n_t, d_acc, static_cast<hipStream_t>(stream), 0, p.n_chan, d_tap);
}

moff_status moff_cal_size(moff_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return set_err(MOFF_E_INVALID, "null argument");
  const moff::Plan &p = plan->p;
  const size_t C = p.n_chan, M = p.n_tap, A = p.n_ant, P = p.n_pol;
  *bytes = C * M * A * P * 16 + C * M * P * 8 + C * A * P * 8;
  return ok();
}

moff_status moff_cal_accumulate(moff_plan_t plan, const void *d_volt, const void *d_tap, int64_t n_t, void *d_cal,
                                void *stream) {
  if (!plan || !d_volt || !d_tap || !d_cal) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  if (p.n_tap <= 0) return set_err(MOFF_E_STATE, "the plan was made with n_tap = 0");
  if (n_t < 0) return set_err(MOFF_E_INVALID, "n_t must be >= 0");
  moff::CalArgs a{};
  a.volt = d_volt;
  a.volt_fmt = p.volt_format;
  a.tap = static_cast<const float2 *>(d_tap);
  a.cal = d_cal;
  a.nt = n_t;
  a.n_chan = p.n_chan;
  a.n_ant = p.n_ant;
  a.n_tap = p.n_tap;
  a.P = p.n_pol;
  HIP_TRY(moff::launch_cal_acc(a, static_cast<hipStream_t>(stream)), "calibration sums");
  return ok();
}

moff_status moff_cal_solve(moff_plan_t plan, const void *d_cal, const void *d_kern, void *d_out, void *stream) {
  if (!plan || !d_cal || !d_kern || !d_out) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  if (!p.taps_set) return set_err(MOFF_E_STATE, "taps are not set (moff_set_taps)");
  if (p.kernel_mode != MOFF_KERNEL_DIAG) return set_err(MOFF_E_UNSUPPORTED, "the solve takes diagonal kernels");
  moff::SolveArgs a{};
  a.chans = d_chans(p);
  a.cal = d_cal;
  a.kern = static_cast<const float2 *>(d_kern);
  a.origin = reinterpret_cast<const int2 *>(ws(p, p.ws_origin));
  a.tap_cpix = reinterpret_cast<const int2 *>(ws(p, p.ws_tap_cpix));
  a.out = d_out;
  a.n_chan = p.n_chan;
  a.n_ant = p.n_ant;
  a.n_tap = p.n_tap;
  a.P = p.n_pol;
  a.K = p.ksize;
  HIP_TRY(moff::launch_cal_solve(a, static_cast<hipStream_t>(stream)), "calibration solve");
  return ok();
}

moff_status moff_set_pipeline(moff_plan_t plan, int32_t pipeline) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  moff::Plan &p = plan->p;
  if (pipeline != MOFF_PIPELINE_TWO_PASS && pipeline != MOFF_PIPELINE_STREAM)
    return set_err(MOFF_E_INVALID, "unknown pipeline");
  if (pipeline == MOFF_PIPELINE_STREAM && p.fft_mode != MOFF_FFT_FP32)
    return set_err(MOFF_E_UNSUPPORTED, "the streaming form is built for the FP32 transform");
  drop_graphs(p);
  p.pipeline = pipeline;
  return ok();
}

moff_status moff_stream_status(moff_plan_t plan, int32_t *code) {
  if (!plan || !code) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  HIP_TRY(hipDeviceSynchronize(), "synchronize");
  const uint32_t *ctr = reinterpret_cast<const uint32_t *>(ws(p, p.ws_ctr));
  HIP_TRY(hipMemcpy(code, ctr + moff::kStreamErrWord, 4, hipMemcpyDeviceToHost),
          "read stream status");
  return ok();
}

moff_status moff_get_launch_shape(moff_plan_t plan, int32_t *time_block, int32_t *chans_per_block,
                                  int32_t *time_group) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  if (time_block) *time_block = plan->p.t_block;
  if (chans_per_block) *chans_per_block = plan->p.chans_per_block;
  if (time_group) *time_group = plan->p.t_group;
  return ok();
}

moff_status moff_autotune(moff_plan_t plan, const void *d_volt, int64_t n_t, void *d_acc, void *stream,
                          int32_t *time_block, int32_t *chans_per_block, int32_t *time_group, double *best_ms) {
  if (!plan || !d_volt || !d_acc) return set_err(MOFF_E_INVALID, "null argument");
  if (n_t < 1 || n_t > INT32_MAX / 2) return set_err(MOFF_E_INVALID, "n_t out of range");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  if (p.profiling) return set_err(MOFF_E_STATE, "autotune while kernel timing is on");
  hipStream_t st = static_cast<hipStream_t>(stream);
  static const int tbs[] = {8, 16, 32, 64, 128, 256};
  static const int cpbs[] = {4, 8, 16, 32, 64, 128};
  static const int tgs[] = {2, 4, 8, 16, 32, 64};
  const int tb0 = p.t_block, cpb0 = p.chans_per_block, tg0 = p.t_group;
  // the current shape first, so that the result is never a shape slower than the one the plan had
  std::vector<std::array<int, 3>> cands{{tb0, cpb0, tg0}};
  for (int tb : tbs)
    for (int cpb : cpbs)
      for (int tg : tgs)
        if (tg <= tb && !(tb == tb0 && cpb == cpb0 && tg == tg0)) cands.push_back({tb, cpb, tg});
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event");
  HIP_TRY(hipEventCreate(&e1), "event");
  double best = 1e300;
  int btb = tb0, bcpb = cpb0, btg = tg0;
  moff_status res = MOFF_OK;
  for (const auto &c : cands) {
    const int tb = c[0], cpb = c[1], tg = c[2];
    if (moff::layout_blocks(p, tb, cpb, tg) > p.ws_bound) continue;
    float ms = 0.f;
    if (enqueue_correlate(p, d_volt, n_t, d_acc, st) != MOFF_OK) { res = MOFF_E_DEVICE; break; }
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess && enqueue_correlate(p, d_volt, n_t, d_acc, st) != MOFF_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { res = hip_fail(e, "autotune timing"); break; }
    if (ms < best) {
      best = ms;
      btb = tb;
      bcpb = cpb;
      btg = tg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  moff::layout_blocks(p, btb, bcpb, btg);
  drop_graphs(p);
  if (res) return res;
  if (time_block) *time_block = btb;
  if (chans_per_block) *chans_per_block = bcpb;
  if (time_group) *time_group = btg;
  if (best_ms) *best_ms = best;
  return ok();
}

// Every input of the launch-shape choice, as one line of text (no tabs or newlines).
static std::string tune_key(const moff::Plan &p) {
  std::map<int, int> sizes;
  int64_t rows = 0;
  for (const moff::Chan &ch : p.chans) {
    ++sizes[ch.n];
    rows += ch.jmax - ch.jmin + 1;
  }
  std::ostringstream k;
  k << "cu=" << p.cu_count << " A=" << p.n_ant << " P=" << p.n_pol << " K=" << p.ksize << " C=" << p.n_chan
    << " n=";
  for (const auto &kv : sizes) k << kv.first << "x" << kv.second << ",";
  k << " rows=" << rows << " fft=" << p.fft_mode << " acc=" << p.acc_mode << " volt=" << p.volt_format
    << " kern=" << p.kernel_mode << " pipe=" << p.pipeline << " taps=" << p.n_tap;
  return k.str();
}

moff_status moff_autotune_key(moff_plan_t plan, char *buf, size_t bufsize) {
  if (!plan || !buf) return set_err(MOFF_E_INVALID, "null argument");
  const std::string k = tune_key(plan->p);
  if (k.size() + 1 > bufsize) return set_err(MOFF_E_INVALID, "key buffer too small");
  std::memcpy(buf, k.c_str(), k.size() + 1);
  return ok();
}

moff_status moff_autotune_cached(moff_plan_t plan, const char *cache_path, const void *d_volt, int64_t n_t,
                                 void *d_acc, void *stream, int32_t *time_block, int32_t *chans_per_block,
                                 int32_t *time_group, double *best_ms, int32_t *hit) {
  if (!plan || !cache_path || !d_volt || !d_acc) return set_err(MOFF_E_INVALID, "null argument");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, true);
  if (s) return s;
  const std::string key = tune_key(p);
  int tb = 0, cpb = 0, tg = 0;
  double ms = 0.0;
  bool found = false;
  {
    std::ifstream in(cache_path);
    if (in.is_open()) {
      std::string line;
      while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream v(line.substr(tab + 1));
        int a = 0, b = 0, c = 0;
        double m = 0.0;
        if (v >> a >> b >> c >> m && a > 0 && b > 0 && c > 0 && c <= a) {
          tb = a;
          cpb = b;
          tg = c;
          ms = m;
          found = true;
        }
      }
    }
  }
  const int tb0 = p.t_block, cpb0 = p.chans_per_block, tg0 = p.t_group;
  if (found && moff::layout_blocks(p, tb, cpb, tg) <= p.ws_bound) {
    drop_graphs(p);
    if (time_block) *time_block = tb;
    if (chans_per_block) *chans_per_block = cpb;
    if (time_group) *time_group = tg;
    if (best_ms) *best_ms = ms;
    if (hit) *hit = 1;
    return ok();
  }
  if (found) moff::layout_blocks(p, tb0, cpb0, tg0);   // the cached shape did not fit the bound workspace
  int32_t rtb = 0, rcpb = 0, rtg = 0;
  double rms = 0.0;
  s = moff_autotune(plan, d_volt, n_t, d_acc, stream, &rtb, &rcpb, &rtg, &rms);
  if (s) return s;
  std::ofstream out(cache_path, std::ios::app);
  if (!out.is_open()) return set_err(MOFF_E_INVALID, std::string("cannot write the autotuner cache ") + cache_path);
  out << key << '\t' << rtb << ' ' << rcpb << ' ' << rtg << ' ' << rms << '\n';
  if (!out.good()) return set_err(MOFF_E_INVALID, std::string("cannot write the autotuner cache ") + cache_path);
  if (time_block) *time_block = rtb;
  if (chans_per_block) *chans_per_block = rcpb;
  if (time_group) *time_group = rtg;
  if (best_ms) *best_ms = rms;
  if (hit) *hit = 0;
  return ok();
}

moff_status moff_read_image(moff_plan_t plan, const void *d_acc, int64_t n_samples, int32_t normalize, void *d_img,
                            void *stream) {
  if (!plan || !d_acc || !d_img) return set_err(MOFF_E_INVALID, "null argument");
  if (normalize && n_samples <= 0) return set_err(MOFF_E_INVALID, "normalize needs n_samples > 0");
  moff::Plan &p = plan->p;
  moff_status s = need_bound(p, false);
  if (s) return s;
  moff::ReadArgs a{};
  a.chans = d_chans(p);
  a.n_chan = p.n_chan;
  a.pix_total = p.pix_total;
  a.acc = d_acc;
  a.scale = normalize ? 1.0 / (double)n_samples : 1.0;
  a.img = static_cast<float2 *>(d_img);
  HIP_TRY(moff::launch_read_image(p.n_pol, p.acc_mode, a, static_cast<hipStream_t>(stream)), "read image");
  return ok();
}

moff_status moff_profile(moff_plan_t plan, int32_t enable) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  moff::Plan &p = plan->p;
  p.profiling = enable != 0;
  if (p.profiling) {
    p.prof.clear();
    p.ev_used = 0;
  }
  return ok();
}

moff_status moff_profile_read(moff_plan_t plan, int32_t kind, double *total_ms, int64_t *launches,
                              int64_t *channel_samples) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  moff::Plan &p = plan->p;
  double ms = 0.0;
  int64_t n = 0, cs = 0;
  for (const moff::Plan::ProfRec &r : p.prof) {
    if (r.kind != kind) continue;
    float e = 0.f;
    HIP_TRY(hipEventSynchronize(static_cast<hipEvent_t>(r.ev1)), "profile sync");
    HIP_TRY(hipEventElapsedTime(&e, static_cast<hipEvent_t>(r.ev0), static_cast<hipEvent_t>(r.ev1)),
            "profile elapsed");
    ms += e;
    ++n;
    cs += r.cs;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (channel_samples) *channel_samples = cs;
  return ok();
}

moff_status moff_debug_unpack(moff_plan_t plan, const void *d_volt, float *d_out, void *stream) {
  if (!plan || !d_volt || !d_out) return set_err(MOFF_E_INVALID, "null argument");
  const moff::Plan &p = plan->p;
  HIP_TRY(moff::launch_unpack_debug(d_volt, p.volt_format, reinterpret_cast<float2 *>(d_out),
                                    (int64_t)p.n_chan * p.n_ant * p.n_pol, static_cast<hipStream_t>(stream)),
          "unpack");
  return ok();
}

moff_status moff_debug_tile_counts(moff_plan_t plan, int64_t *n_band_total, int64_t *n_entries, int32_t *band_rows) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  const moff::Plan &p = plan->p;
  if (n_band_total) *n_band_total = (int64_t)p.bands.size();
  if (n_entries) *n_entries = (int64_t)p.band_ant.size();
  if (band_rows)
    for (int c = 0; c < p.n_chan; ++c) band_rows[c] = p.chans[c].band_rows;
  return ok();
}

moff_status moff_debug_tiles(moff_plan_t plan, int32_t *h_origin, int32_t *h_band_ptr, int32_t *h_band_ant) {
  if (!plan) return set_err(MOFF_E_INVALID, "null plan");
  const moff::Plan &p = plan->p;
  if (h_origin) std::memcpy(h_origin, p.origin.data(), p.origin.size() * 4);
  if (h_band_ptr) std::memcpy(h_band_ptr, p.band_ptr.data(), p.band_ptr.size() * 4);
  if (h_band_ant && !p.band_ant.empty()) std::memcpy(h_band_ant, p.band_ant.data(), p.band_ant.size() * 4);
  return ok();
}

}  // extern "C"
