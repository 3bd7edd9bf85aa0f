"""Serving form of the MOFF hot path: continuous batching of correlation jobs on one GPU.

Jobs arrive as a seeded Poisson stream.  Each job has its own array (antenna count), channel count, integration
length and grid size.  A job is admitted when a slot is free and its projected HBM fits the budget: workspace,
accumulator, image, kernels, and the voltage blocks in flight.  Admitted jobs advance independently.  Each keeps up
to ``depth`` time blocks enqueued on its own HIP stream and enqueues the next block as soon as one completes, so a
small job never waits for a large job's block and the kernels of different jobs overlap on the device.

A job's accumulator stays resident until its integration is complete; then its image is read out and its latency
(completion - arrival) is recorded.  Admission is re-checked on every pass of the loop.  While the head of the
queue waits for memory, later jobs that fit are admitted in its place (backfill), for at most ``max_head_wait``
seconds; after that nothing overtakes the head until it has been admitted.  A job whose set-up, launch or read-out
raises is marked failed and its memory released, and serving continues.  Results are deterministic per job: the
same job gives the same image alone or in a mix.

The scheduler (``Scheduler``) is independent of the device.  ``GpuExecutor`` runs jobs through the C ABI.
``ModelExecutor`` stands in for it with a modelled device (one FIFO queue of blocks, each taking its channel-samples
/ rate seconds), used by CPU tests of admission, backfill, failure handling and latency accounting.
"""
from __future__ import annotations

import math
import time
from collections import deque
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
        """"fp32" (scatter gridding, FP32 transform) or "split_fp16" (gridding and the row transform as one
        split-FP16 matrix-core GEMM; any grid size)."""
        return self.mode

    def chans_per_launch(self, block: int, cap_bytes: int = 1 << 30) -> int:
        """Channels per launch (at most 64) so that the row-transform buffer (block samples x channels x 2 pols x
        n^2 x 8 B) stays under ``cap_bytes``: concurrent jobs then leave room for each other, and one launch of a
        large job does not hold a hardware queue long in front of the others' blocks."""
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


def hbm_bytes(spec: JobSpec, block: int, plan_ws: Optional[int] = None, depth: int = 1) -> int:
    """Projected device memory of a job: accumulator (4 FP32 reals per pixel), image, kernels, ``depth`` blocks of
    voltages, and the plan workspace (tap tables + row-transform buffer of one launch block)."""
    pix = spec.n_chan * spec.grid_n ** 2
    acc = pix * 4 * 4
    img = pix * 4 * 8
    kern = spec.n_chan * spec.n_ant * 2 * 16 * 8
    volt = depth * block * spec.n_chan * spec.n_ant * 2 * 2
    ws = plan_ws if plan_ws is not None else (kern + min(16, spec.n_chan) * 16 * 2 * spec.grid_n ** 2 * 8)
    return int(acc + img + kern + volt + ws)


@dataclass
class JobState:
    spec: JobSpec
    admitted: float = 0.0
    enqueued: int = 0          # samples enqueued so far
    finished: float = 0.0
    hbm: int = 0
    handle: object = None


@dataclass
class Stats:
    latencies: List[float] = field(default_factory=list)
    admitted: int = 0
    rejected: int = 0
    failed: int = 0
    backfilled: int = 0
    peak_concurrent: int = 0
    channel_samples: int = 0
    wall: float = 0.0
    results: Dict[int, object] = field(default_factory=dict)
    errors: Dict[int, str] = field(default_factory=dict)
    order: List[int] = field(default_factory=list)      # job ids in admission order
    times: Dict[int, tuple] = field(default_factory=dict)  # job id -> (arrival, admitted, finished), trace seconds

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"jobs_completed": len(self.latencies), "admitted": self.admitted, "rejected": self.rejected,
                "failed": self.failed, "backfilled": self.backfilled, "peak_concurrent": self.peak_concurrent,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "channel_samples": self.channel_samples, "wall_s": self.wall,
                "channel_samples_per_s": self.channel_samples / self.wall if self.wall > 0 else 0.0}


class Scheduler:
    """Admission by HBM budget and slots with bounded backfill; every job advances on its own completions."""

    def __init__(self, executor, hbm_budget: int, max_slots: int = 8, block: int = 64, depth: int = 2,
                 max_head_wait: float = 2.0, keep_results: bool = False, progress=None):
        self.progress = progress        # optional callable(completed, total), called as jobs complete
        self.ex = executor
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.block = block
        self.depth = depth              # time blocks a job keeps enqueued when every slot is busy
        self.max_head_wait = max_head_wait
        self.keep = keep_results

    def _fail(self, st: Stats, spec: JobSpec, err: BaseException):
        st.failed += 1
        st.errors[spec.job_id] = f"{type(err).__name__}: {err}"

    def run(self, trace: List[JobSpec], realtime: bool = True) -> Stats:
        st = Stats()
        ex = self.ex
        pending = sorted(trace, key=lambda s: s.arrival)
        queue: List[JobSpec] = []
        active: List[JobState] = []
        used = 0
        t_start = ex.now()
        head_since: Optional[float] = None    # when the current head of the queue started waiting for memory
        head_id: Optional[int] = None
        i = 0
        while i < len(pending) or queue or active:
            now = ex.now() - t_start
            if not realtime and not queue and not active and i < len(pending):
                ex.advance_to(t_start + pending[i].arrival)
                now = ex.now() - t_start
            while i < len(pending) and pending[i].arrival <= now:
                spec = pending[i]
                i += 1
                ex.prefetch(spec, self.block)   # host set-up (instrument, plan) starts in the background
                queue.append(spec)
            progressed, waiting = self._admit(st, queue, active, now, head_since)
            # the head waits for memory: note since when (backfill past it stops after max_head_wait)
            if waiting is None:
                head_since, head_id = None, None
            elif waiting != head_id:
                head_since, head_id = now, waiting
            st.peak_concurrent = max(st.peak_concurrent, len(active))
            # advance every active job on its own completions; with few jobs running each keeps up to twice as
            # many blocks enqueued (they share its voltage buffer in stream order, so depth costs no memory; more
            # would hold the hardware queues that other jobs' streams share)
            depth = min(2 * self.depth, max(self.depth, -(-self.max_slots * self.depth // max(len(active), 1))))
            for js in list(active):
                try:
                    ex.poll(js.handle)
                    while js.enqueued < js.spec.n_time and ex.in_flight(js.handle) < depth:
                        nt = min(self.block, js.spec.n_time - js.enqueued)
                        ex.step(js.handle, js.enqueued, nt)
                        js.enqueued += nt
                        progressed = True
                    if js.enqueued >= js.spec.n_time and ex.in_flight(js.handle) == 0:
                        img = ex.finish(js.handle)
                        js.finished = ex.now() - t_start
                        st.latencies.append(js.finished - js.spec.arrival)
                        st.times[js.spec.job_id] = (js.spec.arrival, js.admitted, js.finished)
                        st.channel_samples += js.spec.channel_samples
                        if self.keep:
                            st.results[js.spec.job_id] = img
                        active.remove(js)
                        progressed = True
                        if self.progress:
                            self.progress(len(st.latencies), len(pending))
                except Exception as e:    # the job fails; the others keep running
                    self._fail(st, js.spec, e)
                    ex.release(js.handle)
                    active.remove(js)
                    progressed = True
            if progressed:
                continue
            if active:
                ex.wait_any([js.handle for js in active])
            elif queue:
                ex.sleep(0.001)            # a queued job's set-up is still running
            elif i < len(pending):
                wait = t_start + pending[i].arrival - ex.now()
                if wait > 0:
                    ex.sleep(wait)
        st.wall = ex.now() - t_start
        return st

    def _need(self, spec, st, queue):
        """Projected HBM of a job whose set-up is done, or None (set-up failed: the job is failed and dropped)."""
        try:
            return self.ex.hbm(spec, self.block, self.depth)
        except Exception as e:
            self._fail(st, spec, e)
            queue.remove(spec)
            self.ex.discard(spec)
            return None

    def _admit(self, st, queue, active, now, head_since):
        """One admission pass in arrival order.  The first job in the queue that is ready is the head; it is
        admitted if a slot and its memory are free.  While it waits for memory, later ready jobs that fit are
        admitted in its place (backfill) unless it has waited max_head_wait seconds.  Jobs whose set-up is still
        running are skipped; a job that can never fit the budget is rejected when reached.  Returns (progressed,
        job id of the head if it is waiting for memory, else None)."""
        ex = self.ex
        progressed = False
        used = sum(js.hbm for js in active)
        waiting = None                 # the head, when it waits for memory
        for spec in list(queue):
            if len(active) >= self.max_slots:
                break
            if not ex.ready(spec):
                continue
            need = self._need(spec, st, queue)
            if need is None:
                progressed = True
                continue
            if need > self.budget:
                queue.remove(spec)
                st.rejected += 1
                ex.discard(spec)
                progressed = True
                continue
            if used + need > self.budget:
                if waiting is None:
                    waiting = spec.job_id
                    if head_since is not None and now - head_since >= self.max_head_wait:
                        break          # the head has waited long enough: nothing overtakes it
                continue
            queue.remove(spec)
            try:
                handle = ex.start(spec, self.block)
            except Exception as e:
                self._fail(st, spec, e)
                ex.discard(spec)
                progressed = True
                continue
            active.append(JobState(spec, admitted=now, hbm=need, handle=handle))
            used += need
            st.admitted += 1
            st.order.append(spec.job_id)
            if waiting is not None:
                st.backfilled += 1
            progressed = True
        return progressed, waiting


class ModelExecutor:
    """Device stand-in: one FIFO queue of blocks, each taking its channel-samples / rate seconds of modelled time
    (grids scaled by (n / 256)^2), with no GPU and no real sleeping.  ``fail`` maps job ids to the call that raises
    for them ("prepare", "start", "step" or "finish"), to test failure handling."""

    def __init__(self, cs_per_s: float = 2e6, hbm_scale: float = 1.0, fail: Optional[Dict[int, str]] = None):
        self.t = 0.0
        self.rate = cs_per_s
        self.hbm_scale = hbm_scale
        self.fail = dict(fail or {})
        self.started: List[int] = []
        self.released: List[int] = []
        self.device_free = 0.0
        self.max_inflight: Dict[int, int] = {}    # job id -> most blocks it had enqueued at once

    def _maybe_fail(self, spec, where):
        if self.fail.get(spec.job_id) == where:
            raise RuntimeError(f"modelled {where} failure of job {spec.job_id}")

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)

    def advance_to(self, t):
        self.t = max(self.t, t)

    def hbm(self, spec, block, depth=1):
        self._maybe_fail(spec, "prepare")
        return int(hbm_bytes(spec, block, depth=depth) * self.hbm_scale)

    def prefetch(self, spec, block):
        pass

    def ready(self, spec):
        return True

    def discard(self, spec):
        pass

    def start(self, spec, block):
        self._maybe_fail(spec, "start")
        self.started.append(spec.job_id)
        return {"spec": spec, "inflight": deque()}

    def step(self, h, t0, nt):
        self._maybe_fail(h["spec"], "step")
        cost = h["spec"].n_chan * nt * (h["spec"].grid_n / 256.0) ** 2 / self.rate
        begin = max(self.device_free, self.t)
        self.device_free = begin + cost
        h["inflight"].append(self.device_free)
        h["max_inflight"] = max(h.get("max_inflight", 0), len(h["inflight"]))
        self.max_inflight[h["spec"].job_id] = h["max_inflight"]

    def poll(self, h):
        while h["inflight"] and h["inflight"][0] <= self.t:
            h["inflight"].popleft()

    def in_flight(self, h):
        return len(h["inflight"])

    def wait_any(self, handles):
        due = [h["inflight"][0] for h in handles if h["inflight"]]
        if due:
            self.t = max(self.t, min(due))

    def finish(self, h):
        self._maybe_fail(h["spec"], "finish")
        return None

    def release(self, h):
        self.released.append(h["spec"].job_id)


class GpuExecutor:
    """Runs each job through the C ABI on its own stream; voltages are drawn per block on the device.

    A job's host set-up (its instrument's kernels, cached per array shape, and its plan) starts on a worker
    thread when it arrives, so it overlaps the device work of the jobs already running (numpy and the plan
    builder release the interpreter lock).  Plans are reused: when a job ends its plan is unbound (its device
    workspace freed) and kept, at most ``idle_per_shape`` per job shape (antennas, channels, grid, arithmetic form,
    launch shape), for the next job of that shape, which then skips the plan build.  Admission uses the exact
    device footprint of the built plan: workspace + accumulator + image + kernels + one block of voltages.
    """

    def __init__(self, device="cuda:0", workers: int = 8, idle_per_shape: int = 2):
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
        self._idle = {}           # plan key -> unbound plans of finished jobs
        self._models = {}         # job id -> future of (sky, host voltage-model response)
        self.idle_per_shape = idle_per_shape
        self.plans_built = 0
        self.plans_reused = 0

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

    @staticmethod
    def _plan_key(spec, block):
        return (spec.n_ant, spec.n_chan, spec.grid_n, spec.fft_mode, block, spec.chans_per_launch(block))

    def _prepare(self, spec, block):
        from . import api
        key = self._plan_key(spec, block)
        with self._lock:
            idle = self._idle.get(key)
            if idle:
                self.plans_reused += 1
                return idle.pop()
        site = self._site(spec)
        fft = {"fp32": api.FFT_FP32, "split_fp16": api.FFT_GEMM_FP16}[spec.fft_mode]
        plan = api.plan_for(spec.site_config(), site["geo"], fft_mode=fft, time_block=block,
                            chans_per_block=spec.chans_per_launch(block))
        with self._lock:
            self.plans_built += 1
        return plan

    def _keep(self, spec, block, plan):
        """An unbound plan back to the idle pool of its job shape (dropped beyond idle_per_shape)."""
        plan.unbind()
        with self._lock:
            idle = self._idle.setdefault(self._plan_key(spec, block), [])
            if len(idle) < self.idle_per_shape:
                idle.append(plan)

    def _voltage_model(self, spec):
        """The job's sky and the host side of its voltage generator (numpy, released interpreter lock): built on a
        worker thread when the job arrives, so admission does not stall the loop that feeds the running jobs."""
        from . import synth
        site = self._site(spec)
        cfg = spec.config()
        sk = synth.sky(cfg)
        return sk, synth.source_response(cfg, site["geo"], site["g"], sk)

    def prefetch(self, spec, block):
        with self._lock:
            if spec.job_id not in self._plans:
                fut = self._pool.submit(self._prepare, spec, block)
                fut.block = block
                self._plans[spec.job_id] = fut
                self._models[spec.job_id] = self._pool.submit(self._voltage_model, spec)

    def ready(self, spec):
        fut, mod = self._plans.get(spec.job_id), self._models.get(spec.job_id)
        return fut is not None and fut.done() and mod is not None and mod.done()

    def _plan(self, spec, block):
        self.prefetch(spec, block)
        return self._plans[spec.job_id].result()

    def hbm(self, spec, block, depth=1):
        """Device footprint of a job: its blocks are ordered on one stream and share one voltage buffer, so the
        blocks in flight add no memory."""
        plan = self._plan(spec, block)
        kern = spec.n_chan * spec.n_ant * 2 * 16 * 8
        volt = block * spec.n_chan * spec.n_ant * 2 * 2
        return int(plan.workspace_bytes + plan.acc_bytes + plan.image_bytes + kern + volt)

    def discard(self, spec):
        self._models.pop(spec.job_id, None)
        fut = self._plans.pop(spec.job_id, None)
        if fut is not None and fut.done() and fut.exception() is None:
            self._keep(spec, getattr(fut, "block", 64), fut.result())

    def start(self, spec, block):
        from . import synth
        torch = self.torch
        site = self._site(spec)
        plan = self._plan(spec, block)
        cfg = spec.config()
        mod = self._models.pop(spec.job_id, None)
        sk, resp = mod.result() if mod is not None else self._voltage_model(spec)
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
            gen = synth.DeviceVoltages(cfg, site["geo"], site["g"], sk, self.device, chunk=block, resp=resp)
            vbuf = torch.empty((block, cfg.n_chan, cfg.n_ant, cfg.n_pol, 2), dtype=torch.int8, device=self.device)
        return {"spec": spec, "plan": plan, "acc": acc, "gen": gen, "vbuf": vbuf, "stream": stream,
                "events": deque(), "site_key": key, "block": block}

    def step(self, h, t0, nt):
        """Enqueues one block (voltage synthesis, then the correlation) on the job's stream; an event marks its end.
        Blocks of one job are ordered by its stream, so they share the voltage buffer."""
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            v = h["vbuf"][:nt]
            h["gen"].chunk_into(t0 // h["block"], v)
            h["plan"].correlate(v, h["acc"], n_t=nt, stream=h["stream"])
            ev = torch.cuda.Event()
            ev.record(h["stream"])
        h["events"].append(ev)

    def poll(self, h):
        while h["events"] and h["events"][0].query():
            h["events"].popleft()

    def in_flight(self, h):
        return len(h["events"])

    def wait_any(self, handles):
        """Returns once some job's oldest block has finished (polling every 0.2 ms, so the loop never blocks on one
        job while another could be fed)."""
        while True:
            for h in handles:
                if h["events"] and h["events"][0].query():
                    return
            if not any(h["events"] for h in handles):
                return
            time.sleep(0.0002)

    def _drop(self, h):
        dev = self._site_dev.get(h["site_key"])
        if dev is not None:
            dev[1] -= 1
            if dev[1] == 0:
                del self._site_dev[h["site_key"]]   # free the device copy; the host copy stays cached
        self._plans.pop(h["spec"].job_id, None)
        self._keep(h["spec"], h["block"], h["plan"])   # the job's stream is synchronised: nothing uses it now

    def finish(self, h):
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            img = h["plan"].read_image(h["acc"], n_samples=h["spec"].n_time, stream=h["stream"], split=False)
        h["stream"].synchronize()
        self._drop(h)
        return img

    def release(self, h):
        """A failed job: wait for what its stream holds (an error there is the job's own), then free its memory."""
        try:
            h["stream"].synchronize()
        except Exception:
            pass
        h["events"].clear()
        self._drop(h)
