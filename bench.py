"""Benchmark of the MOFF hot path on one MI355X: channel-samples imaged per second.

Workload (the headline configuration): 2048 antennas in a 200-wavelength disk (at 130 MHz), 128 channels over
100-130 MHz, dual polarisation (XX, YY, XY, YX), 4x4 kernels, 256^2 grid, 16384 time samples of int8
voltages, synthetic and seeded (``paper_0812_3669_amd.synth``).  One step = the whole hot path over the whole
integration: zero the accumulator, grid + 2-D FFT + products for all 128 x 16384 channel-samples
(moff_correlate), and the read-out of the 128 images (moff_read_image).  Voltages (17.2 GB) and kernels are
resident in HBM before the timed region starts.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the hot path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12    # MI355X published FP32 vector peak (packed FP32), FLOP/s
PEAK_HBM = 8.0e12              # MI355X HBM3E, B/s
PEAK_MFMA_16 = 2.5e15          # MI355X published dense FP16 / BF16 matrix-core peak, FLOP/s
# Ceilings measured on the box (profiles/peaks_probe.md, profiles/hbm_copy_calibration.md): the FP32
# FMA issue rate of this build (packed FP32 disabled), the FP16 matrix-core instruction rate, and a plain 1 GiB
# device copy (read + write).
MEASURED_FP32_FMA = 119.5e12
MEASURED_MFMA_16 = 1984.6e12
MEASURED_COPY = 5.08e12
# The row-to-column exchange's own HBM access patterns alone (profiles/exchange_pattern_probe.md): the FP32 row
# pass's tile stores and the column pass's tile loads.
MEASURED_EXCHANGE_STORE = 5.70e12
MEASURED_EXCHANGE_LOAD = 7.06e12
# Matrix-core form: a 256-point transform is two radix-16 stages, each 16 complex 16-point DFTs done as real
# GEMMs (4096 complex MACs = 32768 flops per stage), once per split product (FP16 hi/lo: 3, BF16 hi/mid/lo: 6).
# rocprofv3 SQ_INSTS_VALU_MFMA_MOPS_F16 / _BF16 x 512 reads the same count per launch.
MFMA_FLOPS_PER_TRANSFORM = 2 * 16 * 16 * 16 * 8
SPLIT_PRODUCTS = {"split_fp16": 3, "split_bf16": 6}


KERNEL_SOURCES = ("kernels.hip", "kernels_mfma.hip", "kernels_rowgemm.hip", "kernels.h", "fft_radix.h", "fft_sizes.h",
                  "mfma_fft.h")


def _src_hash() -> str:
    """Hash of the kernel sources (the PMC traffic figures are valid only for the kernels they were taken on)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0812_3669_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(form: str, kernel: str, launch_cs: int):
    """HBM bytes per launch of ``kernel`` in arithmetic form ``form`` from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a plain 1 GiB device copy), if it was taken
    on the current kernel sources and the same channel-samples per launch; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    k = d.get("forms", {}).get(form, {}).get(kernel)
    if d.get("src_hash") != _src_hash() or not k or k.get("channel_samples_per_launch") != launch_cs:
        return None
    return k.get("bytes_per_launch")


# the headline workload's fused-path kernels per arithmetic form
TRAFFIC_FORMS = {"fp32": ("k_rows", "k_cols"), "gemm_fp16": ("k_rowgemm", "k_cols"),
                 "split_fp16": ("k_rows_mfma", "k_cols_mfma")}
TRAFFIC_COMMANDS = [   # {dir}: the directory given to --write-traffic
    "rocprofv3 --pmc %s --output-format csv -d {dir}/pmc_%s_%s -o run -- python3 -u bench.py --time 512 --steps 1 "
    "--warmup 1 --no-cpu-baseline --eager --fft %s" % (c, f, c, f)
    for f in TRAFFIC_FORMS for c in ("FETCH_SIZE", "WRITE_SIZE")] + [
    "rocprofv3 --pmc %s --output-format csv -d {dir}/pmccopy_%s -o run -- python3 -u bench.py --calibrate-copy" % (c, c)
    for c in ("FETCH_SIZE", "WRITE_SIZE")]


def write_traffic(pmc_dir: str, launch_cs: int = 8192, out_path: str | None = None) -> dict:
    """Reduces the rocprofv3 --pmc runs of ``TRAFFIC_COMMANDS`` (CSV output under ``pmc_dir``) to
    ``profiles/traffic.json``: per arithmetic form and fused-path kernel, FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch, averaged over dispatches), each scaled by copy bytes / counter reading of the 1 GiB device copy; keyed
    by the kernel sources' hash.  The default launch shape (256 samples x 32 channels) gives ``launch_cs``
    channel-samples."""
    import collections
    import csv

    def per_dispatch(sub):
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        with open(os.path.join(pmc_dir, sub, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: (len(v), sum(v.values()) / len(v)) for k, v in per.items()}

    def pick(table, prefix):
        hits = [(n, v) for k, (n, v) in table.items() if k.startswith(prefix)]
        if not hits:
            raise SystemExit(f"bench: no dispatch of {prefix!r} under {pmc_dir}")
        return max(hits)   # the instantiation with the most dispatches

    copy_kib = (1 << 30) / 1024
    scale = {c: copy_kib / pick(per_dispatch("pmccopy_" + c), "__amd_rocclr_copyBuffer")[1]
             for c in ("FETCH_SIZE", "WRITE_SIZE")}
    forms = {}
    for form, kernels in TRAFFIC_FORMS.items():
        fetch, write = per_dispatch(f"pmc_{form}_FETCH_SIZE"), per_dispatch(f"pmc_{form}_WRITE_SIZE")
        forms[form] = {}
        for k in kernels:
            f = pick(fetch, f"void moff::{k}<")[1]
            w = pick(write, f"void moff::{k}<")[1]
            forms[form][k] = {"channel_samples_per_launch": launch_cs, "fetch_kib": round(f), "write_kib": round(w),
                              "bytes_per_launch": round((f * scale["FETCH_SIZE"] + w * scale["WRITE_SIZE"]) * 1024)}
    d = {"src_hash": _src_hash(),
         "note": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch (KiB), each scaled by what the counter reads "
                 "for a plain 1 GiB device copy (FETCH x%.3f, WRITE x%.3f)" % (scale["FETCH_SIZE"],
                                                                              scale["WRITE_SIZE"]),
         "commands": [c.format(dir=pmc_dir) for c in TRAFFIC_COMMANDS], "forms": forms}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    return d


def rowgemm_mfma_flops(geo, cfg, c: int, n: int) -> float:
    """Matrix-core flops per sample of the GEMM row pass for channel c (grid n): per touched row and pol, 16-column
    chunks x antenna chunks of 16 (the row's list rounded up) x four 16x16x32 products, per 16 samples."""
    import numpy as np
    K = cfg.ksize
    y = geo.ant_xy_m[:, 1] * geo.freqs_hz[c] / 299792458.0 / cfg.cell_lambda + n / 2
    j0 = np.floor(y).astype(np.int64) - K // 2 + 1
    cnt = np.bincount((j0[:, None] + np.arange(K)[None, :]).ravel(), minlength=n)
    kc = (cnt[j0.min():j0.max() + K] + 15) // 16
    return float(cfg.n_pol * (n // 16) * 4 * 16384 * kc.sum() / 16)


def cpu_baseline(cfg, geo, kern_np, volts_dev, budget_s: float = 12.0):
    """The FP64 oracle timed on this host on a bounded sample: channel 0, growing sample counts."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import moff_oracle as ora
    cores = len(os.sched_getaffinity(0))
    ctx = threadpool_limits(limits=cores) if threadpool_limits else None
    try:
        n_done, t_used, t = 0, 0.0, 4
        sel = [0]
        while t_used < budget_s and t <= cfg.n_time:
            v = volts_dev[:t, 0:1].cpu().numpy()
            t0 = time.perf_counter()
            ora.image(v, kern_np[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel], cfg.cell_lambda)
            dt = time.perf_counter() - t0
            n_done, t_used = t, dt
            t *= 2
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": n_done / t_used, "unit": "channel-samples/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle (direct DFT) on channel 0 x {n_done} samples of the same workload, "
                      f"{t_used:.1f} s"}


def serving_bench(args, dev):
    """The serving trace: seeded Poisson arrivals (``--rate``, 200 jobs/s by default), job shapes drawn from the
    serving sets, integration lengths scaled by ``--time-scale``; p50/p99 latency (completion - arrival, queueing
    included) beside aggregate channel-samples/s.  With ``--capacity-trace`` a second trace follows at 0.7 of the measured capacity (jobs/s =
    0.7 x the first trace's channel-samples/s / the mean channel-samples per job), so that the device is not
    saturated and latency reflects service rather than the backlog of a burst."""
    import torch
    from paper_0812_3669_amd import serve

    def one(rate, seed):
        trace = serve.make_trace(seed=seed, n_jobs=args.jobs, rate=rate, time_scale=args.time_scale)
        # memory a previous trace left in torch's caching allocator counts as free for this one
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info(dev)
        budget = int(0.8 * free)
        ex = serve.GpuExecutor(dev)
        sch = serve.Scheduler(ex, hbm_budget=budget, max_slots=args.serve_slots, block=args.serve_block,
                              progress=lambda k, n: print(f"bench: {k}/{n} jobs done", file=sys.stderr, flush=True)
                              if k % 16 == 0 or k == n else None)
        print(f"bench: serving {len(trace)} jobs at {rate:.3g} jobs/s, HBM budget {budget / 2**30:.1f} GiB",
              file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        st = sch.run(trace, realtime=True)
        torch.cuda.synchronize()
        summ = st.summary()
        summ.update({"arrival_rate_jobs_per_s": rate, "hbm_budget_bytes": budget, "trace_seed": seed,
                     "errors": st.errors, "plans_built": ex.plans_built, "plans_reused": ex.plans_reused})
        mean_cs = float(np.mean([j.channel_samples for j in trace]))
        # the slowest jobs: queueing (arrival to admission, host set-up included) and running (admission to image)
        by_id = {j.job_id: j for j in trace}
        slow = sorted(st.times.items(), key=lambda kv: kv[1][2] - kv[1][0], reverse=True)[:5]
        summ["slowest"] = [{"job": k, "antennas": by_id[k].n_ant, "channels": by_id[k].n_chan,
                            "samples": by_id[k].n_time, "grid": by_id[k].grid_n, "form": by_id[k].mode,
                            "queued_s": round(a - r, 3), "running_s": round(f - a, 3)} for k, (r, a, f) in slow]
        return summ, mean_cs

    import numpy as np
    summ, mean_cs = one(args.rate, args.trace_seed)
    runs = [summ]
    if args.capacity_trace:
        rate = 0.7 * summ["channel_samples_per_s"] / mean_cs
        runs.append(one(rate, args.trace_seed + 1)[0])
    head = runs[-1]
    out = {
        "metric": "p99 job latency, serving trace (continuous batching, HBM-budget admission)",
        "value": head["p99_latency_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": head["wall_s"] * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 / split-fp16 matrix-core row pass per job",
        "data": "synthetic (seeded point sources + noise, int8 voltages)",
        "config": {"workload": "serving: Poisson arrivals, %d jobs per trace, antennas {256,1024,4096,8192}, channels "
                               "{16,64,256}, samples {1k,8k,64k} x %.4g, grids {128,256,512}, fp32 or split_fp16, "
                               "%d-sample blocks, %d slots, 2 blocks in flight per job (4 while slots are free)"
                               % (args.jobs, args.time_scale, args.serve_block, args.serve_slots)},
        "serving": runs,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--acc", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--fft", choices=["fp32", "split_fp16", "split_bf16", "gemm_fp16"], default="fp32",
                    help="transform arithmetic: plain FP32 (VALU) or split-precision matrix-core DFT-GEMMs")
    ap.add_argument("--time", type=int, default=0, help="samples per step (default: the full 16384)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tune the launch shape on the first 256 samples")
    ap.add_argument("--autotune-cache", metavar="FILE",
                    help="with --autotune: the persisted autotuner cache (a shape tuned before is reused)")
    ap.add_argument("--eager", action="store_true", help="launch kernel by kernel instead of replaying a HIP graph")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB device copy (PMC calibration)")
    ap.add_argument("--write-traffic", metavar="DIR", help="write profiles/traffic.json from the PMC runs under DIR")
    ap.add_argument("--calibrate-peaks", action="store_true",
                    help="measure the FP32 vector FMA and FP16 matrix-core issue rates, the FFT stage exchanges "
                         "and the row-to-column exchange's HBM access patterns (moff_probe)")
    ap.add_argument("--pipeline", choices=["two_pass", "stream"], default="two_pass",
                    help="row/column exchange of the fused path: two kernels through HBM, or one persistent "
                         "launch per grid size streaming through each XCD's cache")
    ap.add_argument("--jobs", type=int, default=256, help="serving: jobs in each trace")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrival rate of the first trace, jobs/s")
    ap.add_argument("--trace-seed", type=int, default=4000, help="serving: seed of the first trace")
    ap.add_argument("--serve-block", type=int, default=64, help="serving: samples per block")
    ap.add_argument("--serve-slots", type=int, default=8, help="serving: jobs admitted at once")
    ap.add_argument("--time-scale", type=float, default=1.0 / 64, help="serving: integration-length factor")
    ap.add_argument("--capacity-trace", action="store_true",
                    help="serving: a second trace at 0.7 of the capacity measured on the first")
    ap.add_argument("--workload", choices=["headline", "batched", "serving"], default="headline",
                    help="headline: 2048 antennas, 256^2 grids; batched: 4096 antennas, 256 channels over "
                         "50-200 MHz with per-channel grid sizes (128^2..384^2), 6x6 kernels")
    args = ap.parse_args()

    if args.write_traffic:
        print(json.dumps(write_traffic(args.write_traffic), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py: the MOFF hot path runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is described in the design notes, not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0812_3669_amd import api, configs, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)       # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        # what plain device kernels reach on this GPU's HBM: the same copy (read + write), a fill (write only)
        # and a sum (read only), 10 launches each, timed with events
        nbytes = a.numel() * 4
        rates = {}
        for name, fn, moved in (("copy", lambda: b.copy_(a), 2 * nbytes), ("fill", lambda: b.fill_(0.5), nbytes),
                                ("read", lambda: torch.sum(a), nbytes)):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                fn()
            e1.record()
            e1.synchronize()
            rates[name] = round(10 * moved / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3, "hbm_gbps": rates}))
        return

    if args.calibrate_peaks:
        # measured ceilings beside the published ones: 8 x 256 workgroups per kind, 10 timed launches each
        out = torch.empty(2048 * 256, dtype=torch.float32, device=dev)
        res = {}
        for kind, name, iters in ((0, "fp32_vector_fma_tflops", 4096), (1, "f16_mfma_tflops", 2048)):
            api.probe(kind, 2048, iters, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            flops = sum(api.probe(kind, 2048, iters, out) for _ in range(10))
            e1.record()
            e1.synchronize()
            res[name] = round(flops / (e0.elapsed_time(e1) * 1e-3) / 1e12, 1)
        # the two exchanges between the stages of a 256-point transform: through LDS (radix-16 stages, the
        # library's scheme) and across lanes (radix-2 stages with DPP / swizzle / permute), 2048 x 16 transforms
        # of a random batch, 64 repeats per launch
        data = torch.randn(2048 * 16 * 256, dtype=torch.complex64, device=dev)
        for kind, name in ((2, "fft256_lds_exchange"), (3, "fft256_crosslane_exchange")):
            api.probe(kind, 2048, 64, data)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            flops = sum(api.probe(kind, 2048, 64, data) for _ in range(10))
            e1.record()
            e1.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            res[name] = {"tflops": round(flops / sec / 1e12, 1),
                         "transforms_per_s": round(flops / (5 * 256 * 8) / sec / 1e9, 3) * 1e9}
        del data
        # the row-to-column exchange's HBM access patterns alone, over one headline launch's 8192 channel-samples
        # (8 GiB): the row pass's tile stores and the column pass's tile loads, 5 timed launches each
        xbuf = torch.zeros(8192 * 2 * 65536, dtype=torch.complex64, device=dev)
        for kind, name in ((5, "exchange_store_tbs"), (6, "exchange_load_tbs")):
            api.probe(kind, 8192, 1, xbuf)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            moved = sum(api.probe(kind, 8192, 1, xbuf) for _ in range(5))
            e1.record()
            e1.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            res[name] = round(moved / sec / 1e12, 3)
            res[name.replace("_tbs", "_ms_per_launch")] = round(sec / 5 * 1e3, 3)
        print(json.dumps(res))
        return

    if args.workload == "serving":
        serving_bench(args, dev)
        return
    cfg = configs.HEADLINE if args.workload == "headline" else configs.BATCHED
    T = args.time or cfg.n_time
    print(f"bench: building workload {cfg.name} (T={T})", file=sys.stderr, flush=True)
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    sk = synth.sky(cfg)
    kern_np = synth.kernels(geo, g, cfg.n_pol)
    volts = synth.DeviceVoltages(cfg, geo, g, sk, dev, chunk=64).all(T)
    acc_mode = api.ACC_FP64_COMP if args.acc == "fp64" else api.ACC_FP32
    fft_mode = {"fp32": api.FFT_FP32, "split_fp16": api.FFT_SPLIT_FP16, "split_bf16": api.FFT_SPLIT_BF16,
                "gemm_fp16": api.FFT_GEMM_FP16}[args.fft]
    plan = api.plan_for(cfg, geo, acc_mode=acc_mode, fft_mode=fft_mode)
    # room for every shape the autotuner tries, up to 16384 channel-samples per launch
    room = max(plan.workspace_bytes_for(tb, cpb) for tb in (8, 16, 32, 64, 128, 256)
               for cpb in (4, 8, 16, 32, 64, 128) if tb * cpb <= 16384) if args.autotune else None
    plan.bind(dev, workspace_bytes=room)
    plan.set_kernels(torch.from_numpy(kern_np).to(dev))
    plan.set_pipeline(api.PIPELINE_STREAM if args.pipeline == "stream" else api.PIPELINE_TWO_PASS)
    acc = plan.new_accumulator()
    tuned = None
    if args.autotune:
        tuned = plan.autotune(volts, acc, n_t=min(T, 256), cache=args.autotune_cache)
        print(f"bench: autotuned launch shape {tuned}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print("bench: workload resident; warmup", file=sys.stderr, flush=True)

    run = plan.correlate if args.eager else plan.correlate_graph

    def step():
        acc.zero_()
        run(volts, acc, n_t=T)
        return plan.read_image(acc, n_samples=T, split=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(bool(args.eager))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        img = step()
    e1.record()
    torch.cuda.synchronize()
    plan.profile(False)
    ms = e0.elapsed_time(e1) / args.steps
    if not args.eager:
        # kernel timing needs the eager path (events cannot be recorded inside the replayed graph): one extra,
        # untimed step with per-launch events
        plan.profile(True)
        acc.zero_()
        plan.correlate(volts, acc, n_t=T)
        torch.cuda.synchronize()
        plan.profile(False)
    cs = cfg.n_chan * T
    value = cs / (ms / 1e3)
    if args.pipeline == "stream":
        status = plan.stream_status()
        if status != 0:
            raise SystemExit(f"bench: streaming form reported status {status}; the timed result is not valid")
    print(f"bench: {ms:.2f} ms/step", file=sys.stderr, flush=True)

    # per-kernel event timing over the profiled step; algorithmic flops per channel-sample of each pass
    P, K, A = cfg.n_pol, cfg.ksize, cfg.n_ant

    def pass_flops(kind, n):
        fft_half = 5.0 * n * n * math.log2(n) * P          # half of the 2-D transform (rows or columns)
        if kind == 2:
            return cfg.flops_per_cs(n)                       # streaming form: the whole path in one kernel
        return 8.0 * A * P * K * K + fft_half if kind == 0 else fft_half + 16.0 * n * n

    names = {0: "k_rowgemm" if args.fft == "gemm_fp16" else "k_rows", 1: "k_cols", 2: "k_stream"}
    split = args.fft in SPLIT_PRODUCTS
    mfma_step = {}
    if split:
        # the matrix-core passes transform every row of the touched bands and every column (256^2, two pols)
        names = {0: "k_rows_mfma", 1: "k_cols_mfma"}
        _, band_ptr, _, band_rows = plan.debug_tiles()
        if len(set(band_rows.tolist())) != 1 or set(plan.grid_n) != {256}:
            raise SystemExit("bench: the matrix-core flop count assumes 256^2 grids with one band height")
        per_transform = MFMA_FLOPS_PER_TRANSFORM * SPLIT_PRODUCTS[args.fft]
        mfma_step = {0: (len(band_ptr) - 1) * int(band_rows[0]) * P * T * per_transform,
                     1: cfg.n_chan * 256 * P * T * per_transform}
    elif args.fft == "gemm_fp16":
        mfma_step = {0: T * sum(rowgemm_mfma_flops(geo, cfg, c, n) for c, n in enumerate(plan.grid_n))}
    kt = {}
    for kind in (0, 1, 2):
        tot_ms, launches, kcs = plan.profile_read(kind)
        if launches == 0:
            continue
        # the profiled step covers every channel for T samples; split its channel-samples by grid size
        step_flops = sum(T * pass_flops(kind, n) for n in plan.grid_n)
        frac_cs = kcs / (T * cfg.n_chan)
        kt[kind] = dict(ms=tot_ms, launches=launches, cs=kcs, flops=step_flops * frac_cs,
                        mfma_flops=mfma_step.get(kind, 0.0) * frac_cs)
    dom = max(kt, key=lambda k: kt[k]["ms"])
    d = kt[dom]
    nl = max(d["launches"], 1)
    avg_ms = d["ms"] / nl
    launch_cs = round(d["cs"] / nl)
    tot_ms_all = sum(v["ms"] for v in kt.values())
    traffic = _traffic(args.fft, names[dom], launch_cs) if args.workload == "headline" else None
    if d["mfma_flops"] > 0:
        # a matrix-core kernel: its own split-FP16/BF16 products against the dense matrix-core peak
        achieved = d["mfma_flops"] / nl / (avg_ms / 1e3)
        roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_MFMA_16 / 1e12, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_MFMA_16, "traffic": traffic,
                    "measured_ceiling": {"what": "FP16 matrix-core instruction rate (moff_probe)",
                                         "value": MEASURED_MFMA_16 / 1e12, "frac": achieved / MEASURED_MFMA_16}}
    else:
        # algorithmically the path is arithmetic-bound (12 MFLOP per 8.4 KB of voltages at the headline): the FP32
        # vector units, whose published peak assumes packed FP32 instructions (disabled in this build)
        achieved = d["flops"] / nl / (avg_ms / 1e3)
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                    "measured_ceiling": {"what": "FP32 FMA issue rate of this build (moff_probe)",
                                         "value": MEASURED_FP32_FMA / 1e12, "frac": achieved / MEASURED_FP32_FMA}}
    roofline.update({"kernel": names[dom], "avg_launch_ms": avg_ms, "channel_samples_per_launch": launch_cs,
                     "kernel_share": {names[k]: kt[k]["ms"] / tot_ms_all for k in kt}})
    if traffic:
        # what the kernel as built moves: the row-to-column exchange, far above the algorithmic bytes.  Its
        # arithmetic intensity against the ridge (peak flops / 8 TB/s) says which roof binds it.
        gbs = traffic / (avg_ms / 1e3)
        peak = PEAK_MFMA_16 if d["mfma_flops"] > 0 else PEAK_FP32_VECTOR
        intensity = (d["mfma_flops"] if d["mfma_flops"] > 0 else d["flops"]) / nl / traffic
        attainable = min(peak, intensity * PEAK_HBM)   # the roofline at the measured intensity
        roofline["limiter"] = {
            "measured_bytes_per_launch": traffic,
            "algorithmic_bytes_per_launch": launch_cs * cfg.volt_bytes_per_cs(),
            "achieved_gbs": gbs / 1e9, "frac_hbm_peak": gbs / PEAK_HBM, "frac_measured_copy": gbs / MEASURED_COPY,
            "flop_per_byte": intensity, "ridge_flop_per_byte": peak / PEAK_HBM,
            "lower_roof": "hbm" if intensity * PEAK_HBM < peak else roofline["bound"],
            "attainable_tflops": attainable / 1e12, "frac_of_attainable": achieved / attainable}
        if names[dom] == "k_rows":
            # against what the row pass's own store pattern reaches with no arithmetic around it
            roofline["limiter"]["exchange_pattern"] = {
                "what": "the row pass's exchange tile stores alone (moff_probe kind 5)",
                "value_gbs": MEASURED_EXCHANGE_STORE / 1e9, "frac": gbs / MEASURED_EXCHANGE_STORE}
            # both passes against the time their exchange traffic takes at the access patterns' own rates
            cols_traffic = _traffic(args.fft, "k_cols", launch_cs)
            if 1 in kt and cols_traffic:
                pair_ms = avg_ms + kt[1]["ms"] / max(kt[1]["launches"], 1)
                floor_ms = (traffic / MEASURED_EXCHANGE_STORE + cols_traffic / MEASURED_EXCHANGE_LOAD) * 1e3
                roofline["limiter"]["two_pass_exchange_floor"] = {
                    "floor_ms_per_launch": floor_ms, "measured_ms_per_launch": pair_ms, "frac": floor_ms / pair_ms}
    algo_flops_step = sum(T * cfg.flops_per_cs(n) for n in plan.grid_n)
    if args.workload == "headline":
        metric = "channel-samples imaged/s (N=2048, 256^2 grid), "
        workload = ("headline: 2048 antennas, 200-lambda disk, 128 channels 100-130 MHz, 2 pols, 4x4 kernels, "
                    "256^2 grid, %d samples, int8" % T)
    else:
        metric = "channel-samples imaged/s (N=4096, per-channel grids 128^2..384^2), "
        sizes = sorted(set(plan.grid_n))
        workload = ("batched: 4096 antennas, 376-lambda disk at 200 MHz, 256 channels 50-200 MHz, 2 pols, 6x6 "
                    "kernels, per-channel grids %s, %d samples, int8" % ("/".join(map(str, sizes)), T))

    out = {
        "metric": metric + ("plain FP32 path" if args.fft == "fp32" else f"{args.fft} matrix-core transform"),
        "value": value, "unit": "channel-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "split_fp16": "f16x2->f32", "split_bf16": "bf16x3->f32",
                  "gemm_fp16": "f16x2->f32 (row GEMM) + f32"}[args.fft],
        "data": "synthetic (seeded point sources + noise, int8 voltages)",
        "config": {"workload": workload,
                   "channel_samples_per_step": cs, "accumulator": args.acc,
                   "fft": args.fft,
                   "launch_shape": dict(zip(("time_block", "chans_per_block", "time_group"), plan.launch_shape())),
                   "graph_replay": not args.eager,
                   "pipeline": args.pipeline,
                   "algorithmic_flops_per_cs": algo_flops_step / cs,
                   "achieved_algorithmic_tflops": algo_flops_step / (ms / 1e3) / 1e12,
                   "whole_path_frac_fp32_peak": algo_flops_step / (ms / 1e3) / PEAK_FP32_VECTOR,
                   "whole_path_frac_measured_fma": algo_flops_step / (ms / 1e3) / MEASURED_FP32_FMA},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, geo, kern_np, volts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
