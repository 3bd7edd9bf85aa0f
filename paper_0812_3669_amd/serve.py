"""Serving form of the MOFF hot path: continuous batching of correlation jobs on one GPU.

Jobs arrive as a seeded Poisson stream.  Each job has its own array (antenna count), channel count, integration
length and grid size; it is admitted when a slot is free and its projected HBM (workspace + accumulator +
kernels + one time block of voltages) fits the budget, otherwise it waits in arrival order.  Admitted jobs
advance one time block at a time, each on its own HIP stream, so the kernels of different jobs overlap on the
device; a job's accumulator stays resident until its integration is complete, when its image is read out and
its latency (completion - arrival) recorded.  Results are deterministic per job: the same job gives the same
image alone or in a mix.

The scheduler (``Scheduler``) is independent of the device: ``GpuExecutor`` runs jobs through the C ABI,
``ModelExecutor`` stands in for it with a modelled duration (used by CPU tests of admission, queueing and
budget handling).
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import configs

ANTENNAS = (256, 1024, 4096, 8192)
CHANNELS = (16, 64, 256)
SAMPLES = (1024, 8192, 65536)
GRIDS = (128, 256, 512)
MODES = ("fp32", "split_fp16")


@dataclass
class JobSpec:
    job_id: int
    arrival: float          # seconds from trace start
    n_ant: int
    n_chan: int
    n_time: int
    grid_n: int
    mode: str = "fp32"
    seed: int = 0

    def site_config(self) -> configs.Config:
        """The array a job observes with: band 100-130 MHz, 4x4 kernels, the disk filling the grid at the top
        channel (diameter n - K - 2 wavelengths), int8 voltages, 5 point sources.  Positions, gains and kernels
        depend on the array shape (antennas, channels, grid) only, as an instrument's do; the sky and the
        voltages come from ``config()``, which differs per job."""
        K = 4
        site = 7919 * self.n_ant + 131 * self.n_chan + self.grid_n
        return configs.Config(f"site{site}", 10_000 + site, n_ant=self.n_ant, n_pol=2, n_chan=self.n_chan,
                              ksize=K, f_lo=100e6, f_hi=130e6, disk_lambda=float(self.grid_n - K - 2),
                              disk_ref_hz=130e6, grid_n=self.grid_n, n_time=self.n_time, n_src=5)

    def config(self) -> configs.Config:
        """The job's own seeds (sky and voltages), same shapes as ``site_config``."""
        return configs.scaled(self.site_config(), name=f"job{self.job_id}", index=1000 + self.seed)

    @property
    def fft_mode(self) -> str:
        """The split-precision transform is built for 256^2 grids; other sizes run the FP32 transform."""
        return self.mode if self.grid_n == 256 else "fp32"

    def chans_per_launch(self, block: int, cap_bytes: int = 1 << 30) -> int:
        """Channels per launch so that the row-transform buffer (block samples x channels x 2 pols x n^2 x 8 B)
        stays under ``cap_bytes``: concurrent jobs then leave room for each other."""
        per = block * 2 * self.grid_n ** 2 * 8
        return int(max(1, min(self.n_chan, 64, cap_bytes // per)))

    @property
    def channel_samples(self) -> int:
        return self.n_chan * self.n_time


def make_trace(seed: int = 4000, n_jobs: int = 256, rate: float = 200.0, time_scale: float = 1.0,
               max_ant: int = 8192) -> List[JobSpec]:
    """Seeded Poisson trace.  Each job draws antennas, channels, samples and grid uniformly and independently
    from the serving workload's sets; ``time_scale`` shrinks every integration length (a stated reduction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    ants = [a for a in ANTENNAS if a <= max_ant]
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        T = int(rng.choice(SAMPLES))
        out.append(JobSpec(j, t, int(rng.choice(ants)), int(rng.choice(CHANNELS)),
                           max(1, int(round(T * time_scale))), int(rng.choice(GRIDS)),
                           str(rng.choice(MODES)), seed=int(rng.integers(0, 1 << 30))))
    return out


def hbm_bytes(spec: JobSpec, block: int, plan_ws: Optional[int] = None) -> int:
    """Projected device memory of a job: accumulator (4 FP32 reals per pixel), image, kernels, one block of
    voltages, and the plan workspace (tap tables + row-transform buffer of one launch block)."""
    pix = spec.n_chan * spec.grid_n ** 2
    acc = pix * 4 * 4
    img = pix * 4 * 8
    kern = spec.n_chan * spec.n_ant * 2 * 16 * 8
    volt = block * spec.n_chan * spec.n_ant * 2 * 2
    ws = plan_ws if plan_ws is not None else (kern + min(16, spec.n_chan) * 16 * 2 * spec.grid_n ** 2 * 8)
    return int(acc + img + kern + volt + ws)


@dataclass
class JobState:
    spec: JobSpec
    admitted: float = 0.0
    done_samples: int = 0
    finished: float = 0.0
    hbm: int = 0
    handle: object = None


@dataclass
class Stats:
    latencies: List[float] = field(default_factory=list)
    admitted: int = 0
    rejected: int = 0
    peak_concurrent: int = 0
    channel_samples: int = 0
    wall: float = 0.0
    results: Dict[int, object] = field(default_factory=dict)

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"jobs_completed": len(self.latencies), "admitted": self.admitted, "rejected": self.rejected,
                "peak_concurrent": self.peak_concurrent,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "channel_samples": self.channel_samples, "wall_s": self.wall,
                "channel_samples_per_s": self.channel_samples / self.wall if self.wall > 0 else 0.0}


class Scheduler:
    """Admission by HBM budget and slots, arrival-order queue, one time block per active job per round."""

    def __init__(self, executor, hbm_budget: int, max_slots: int = 8, block: int = 64,
                 keep_results: bool = False, progress=None):
        self.progress = progress        # optional callable(completed, total), called as jobs complete
        self.ex = executor
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.block = block
        self.keep = keep_results

    def run(self, trace: List[JobSpec], realtime: bool = True) -> Stats:
        st = Stats()
        pending = sorted(trace, key=lambda s: s.arrival)
        queue: List[JobSpec] = []
        active: List[JobState] = []
        used = 0
        t_start = self.ex.now()
        i = 0
        while i < len(pending) or queue or active:
            now = self.ex.now() - t_start
            if not realtime and not queue and not active and i < len(pending):
                self.ex.advance_to(t_start + pending[i].arrival)
                now = self.ex.now() - t_start
            while i < len(pending) and pending[i].arrival <= now:
                spec = pending[i]
                i += 1
                self.ex.prefetch(spec, self.block)   # host set-up (instrument, plan) starts in the background
                queue.append(spec)
            # admit in arrival order while a slot and memory are free; a job whose set-up is still running holds
            # the head of the queue; one that can never fit is rejected when it reaches the head
            while queue and len(active) < self.max_slots and self.ex.ready(queue[0]):
                spec = queue[0]
                need = self.ex.hbm(spec, self.block)
                if need > self.budget:
                    queue.pop(0)
                    st.rejected += 1
                    self.ex.discard(spec)
                    continue
                if used + need > self.budget:
                    break
                queue.pop(0)
                js = JobState(spec, admitted=now, hbm=need)
                js.handle = self.ex.start(spec, self.block)
                used += need
                active.append(js)
                st.admitted += 1
            st.peak_concurrent = max(st.peak_concurrent, len(active))
            if not active:
                if queue:
                    self.ex.sleep(0.001)            # the head job's set-up is still running
                elif i < len(pending):
                    wait = t_start + pending[i].arrival - self.ex.now()
                    if wait > 0:
                        self.ex.sleep(wait)
                continue
            # one block of every active job, enqueued back to back (their streams overlap on the device)
            for js in active:
                if js.done_samples < js.spec.n_time:
                    nt = min(self.block, js.spec.n_time - js.done_samples)
                    self.ex.step(js.handle, js.done_samples, nt)
                    js.done_samples += nt
            self.ex.wait_round([js.handle for js in active])
            finished = [js for js in active if js.done_samples >= js.spec.n_time]
            for js in finished:
                img = self.ex.finish(js.handle)
                js.finished = self.ex.now() - t_start
                st.latencies.append(js.finished - js.spec.arrival)
                st.channel_samples += js.spec.channel_samples
                if self.progress:
                    self.progress(len(st.latencies), len(pending))
                if self.keep:
                    st.results[js.spec.job_id] = img
                used -= js.hbm
                active.remove(js)
        st.wall = self.ex.now() - t_start
        return st


class ModelExecutor:
    """Device stand-in: a job block takes cs / rate seconds of modelled time (no GPU, no real sleeping)."""

    def __init__(self, cs_per_s: float = 2e6, hbm_scale: float = 1.0):
        self.t = 0.0
        self.rate = cs_per_s
        self.hbm_scale = hbm_scale
        self.started: List[int] = []
        self._round = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)

    def advance_to(self, t):
        self.t = max(self.t, t)

    def hbm(self, spec, block):
        return int(hbm_bytes(spec, block) * self.hbm_scale)

    def prefetch(self, spec, block):
        pass

    def ready(self, spec):
        return True

    def discard(self, spec):
        pass

    def start(self, spec, block):
        self.started.append(spec.job_id)
        return {"spec": spec}

    def step(self, h, t0, nt):
        cost = h["spec"].n_chan * nt * (h["spec"].grid_n / 256.0) ** 2 / self.rate
        self._round += cost

    def wait_round(self, handles):
        self.t += self._round
        self._round = 0.0

    def finish(self, h):
        return None


class GpuExecutor:
    """Runs each job through the C ABI on its own stream; voltages are drawn per block on the device.

    A job's host set-up (its instrument's kernels, cached per array shape, and its plan) starts on a worker
    thread when it arrives, so it overlaps the device work of the jobs already running (numpy and the plan
    builder release the interpreter lock).  Admission uses the exact device footprint of the built plan:
    workspace + accumulator + image + kernels + one block of voltages.
    """

    def __init__(self, device="cuda:0", workers: int = 8):
        import threading
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.torch = torch
        self.device = torch.device(device)
        self._pool = ThreadPoolExecutor(max_workers=workers)
        self._lock = threading.Lock()
        self._plans = {}          # job id -> future of the plan
        self._sites = {}          # array shape -> future of the instrument (geometry, gains, kernels)
        self._site_dev = {}       # array shape -> [device kernels, active users]

    def now(self):
        return time.perf_counter()

    def sleep(self, dt):
        time.sleep(max(dt, 0.0))

    def advance_to(self, t):
        self.sleep(t - self.now())

    @staticmethod
    def _make_site(spec):
        from . import synth
        scfg = spec.site_config()
        geo = synth.geometry(scfg)
        g = synth.gains(scfg)
        return {"geo": geo, "g": g, "kern_np": synth.kernels(geo, g, 2)}

    def _site(self, spec):
        """The instrument of this job's shape: the first thread to ask builds it (never a nested pool task, so
        workers cannot all block waiting on each other); the others wait for its result."""
        from concurrent.futures import Future
        key = (spec.n_ant, spec.n_chan, spec.grid_n)
        with self._lock:
            fut = self._sites.get(key)
            mine = fut is None
            if mine:
                fut = self._sites[key] = Future()
        if mine:
            try:
                fut.set_result(self._make_site(spec))
            except BaseException as e:  # pragma: no cover - surfaced to every waiter
                fut.set_exception(e)
        return fut.result()

    def _prepare(self, spec, block):
        from . import api
        site = self._site(spec)
        fft = {"fp32": api.FFT_FP32, "split_fp16": api.FFT_SPLIT_FP16}[spec.fft_mode]
        return api.plan_for(spec.site_config(), site["geo"], fft_mode=fft, time_block=block,
                            chans_per_block=spec.chans_per_launch(block))

    def prefetch(self, spec, block):
        with self._lock:
            if spec.job_id not in self._plans:
                self._plans[spec.job_id] = self._pool.submit(self._prepare, spec, block)

    def ready(self, spec):
        fut = self._plans.get(spec.job_id)
        return fut is not None and fut.done()

    def _plan(self, spec, block):
        self.prefetch(spec, block)
        return self._plans[spec.job_id].result()

    def hbm(self, spec, block):
        plan = self._plan(spec, block)
        kern = spec.n_chan * spec.n_ant * 2 * 16 * 8
        volt = block * spec.n_chan * spec.n_ant * 2 * 2
        return int(plan.workspace_bytes + plan.acc_bytes + plan.image_bytes + kern + volt)

    def discard(self, spec):
        self._plans.pop(spec.job_id, None)

    def start(self, spec, block):
        from . import synth
        torch = self.torch
        site = self._site(spec)
        plan = self._plan(spec, block)
        cfg = spec.config()
        sk = synth.sky(cfg)
        key = (spec.n_ant, spec.n_chan, spec.grid_n)
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            dev = self._site_dev.get(key)
            if dev is None:
                dev = self._site_dev[key] = [torch.from_numpy(site["kern_np"]).to(self.device), 0]
            dev[1] += 1
            plan.bind(self.device, stream=stream)
            plan.set_kernels(dev[0], stream=stream)
            acc = plan.new_accumulator()
            gen = synth.DeviceVoltages(cfg, site["geo"], site["g"], sk, self.device, chunk=block)
            vbuf = torch.empty((block, cfg.n_chan, cfg.n_ant, cfg.n_pol, 2), dtype=torch.int8, device=self.device)
        ev = torch.cuda.Event()
        return {"spec": spec, "plan": plan, "acc": acc, "gen": gen, "vbuf": vbuf, "stream": stream, "ev": ev,
                "site_key": key, "block": block}

    def step(self, h, t0, nt):
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            v = h["vbuf"][:nt]
            h["gen"].chunk_into(t0 // h["block"], v)
            h["plan"].correlate(v, h["acc"], n_t=nt, stream=h["stream"])
            h["ev"].record(h["stream"])

    def wait_round(self, handles):
        for h in handles:
            h["ev"].synchronize()

    def finish(self, h):
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            img = h["plan"].read_image(h["acc"], n_samples=h["spec"].n_time, stream=h["stream"], split=False)
        h["stream"].synchronize()
        dev = self._site_dev[h["site_key"]]
        dev[1] -= 1
        if dev[1] == 0:
            del self._site_dev[h["site_key"]]   # free the device copy; the host copy stays cached
        self._plans.pop(h["spec"].job_id, None)
        return img
