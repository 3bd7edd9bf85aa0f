"""CPU tests of the serving scheduler with a modelled executor: admission by HBM budget and slots, arrival-order
queueing with bounded backfill, rejection of jobs that can never fit, per-job failure handling, jobs advancing on
their own completions, latency accounting."""
import numpy as np

from paper_0812_3669_amd import serve
from paper_0812_3669_amd.serve import JobSpec, ModelExecutor, Scheduler, hbm_bytes, make_trace


def test_trace_is_seeded_and_drawn_from_the_sets():
    a = make_trace(seed=7, n_jobs=64)
    b = make_trace(seed=7, n_jobs=64)
    assert [(j.arrival, j.n_ant, j.n_chan, j.n_time, j.grid_n, j.mode) for j in a] == \
           [(j.arrival, j.n_ant, j.n_chan, j.n_time, j.grid_n, j.mode) for j in b]
    assert all(j.n_ant in (256, 1024, 4096, 8192) and j.n_chan in (16, 64, 256) for j in a)
    assert all(j.grid_n in (128, 256, 512) and j.n_time in (1024, 8192, 65536) for j in a)
    gaps = np.diff([0.0] + [j.arrival for j in make_trace(seed=1, n_jobs=4000)])
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0     # Poisson stream, mean 200 jobs/s


def _jobs(n, T=256, chans=16, grid=128, spacing=0.0):
    return [JobSpec(i, i * spacing, 256, chans, T, grid) for i in range(n)]


def test_all_jobs_complete_and_latency_includes_queueing():
    ex = ModelExecutor(cs_per_s=1e6)
    sch = Scheduler(ex, hbm_budget=1 << 40, max_slots=2, block=64)
    st = sch.run(_jobs(6), realtime=False)
    s = st.summary()
    assert s["jobs_completed"] == 6 and s["admitted"] == 6 and s["rejected"] == 0
    assert s["peak_concurrent"] == 2
    lat = sorted(st.latencies)
    assert lat[-1] > 2.5 * lat[0]            # the last jobs waited for slots
    assert st.channel_samples == 6 * 16 * 256


def test_budget_limits_concurrency_and_rejects_oversized_jobs():
    job = JobSpec(0, 0.0, 256, 16, 128, 128)
    need = hbm_bytes(job, 64, depth=2)
    ex = ModelExecutor(cs_per_s=1e6)
    sch = Scheduler(ex, hbm_budget=int(2.5 * need), max_slots=8, block=64)
    jobs = _jobs(5, T=128) + [JobSpec(99, 0.0, 8192, 256, 128, 512)]   # the last can never fit
    st = sch.run(jobs, realtime=False)
    assert st.rejected == 1 and st.admitted == 5
    assert st.peak_concurrent == 2


def test_arrivals_in_the_future_wait_for_their_time():
    ex = ModelExecutor(cs_per_s=1e9)
    sch = Scheduler(ex, hbm_budget=1 << 40, max_slots=4, block=64)
    st = sch.run(_jobs(3, T=64, spacing=5.0), realtime=False)
    assert st.summary()["jobs_completed"] == 3
    assert st.wall >= 10.0
    assert max(st.latencies) < 0.01


def test_job_site_shared_by_shape_and_launch_cap():
    a = serve.JobSpec(0, 0.0, 1024, 64, 128, 256, "split_fp16", seed=1)
    b = serve.JobSpec(1, 0.5, 1024, 64, 4096, 256, "fp32", seed=2)
    assert a.site_config().index == b.site_config().index          # same instrument
    assert a.config().index != b.config().index                    # own sky and voltages
    assert a.config().n_ant == a.site_config().n_ant and a.config().grid_n == 256
    big = serve.JobSpec(2, 0.0, 8192, 256, 1024, 512, "split_fp16")
    assert big.fft_mode == "split_fp16" and a.fft_mode == "split_fp16"
    cpl = big.chans_per_launch(64)
    assert cpl == 4 and 64 * cpl * 2 * 512 ** 2 * 8 <= (1 << 30)


def test_gpu_executor_prepares_jobs_in_background():
    """Host set-up of queued jobs runs on worker threads (fewer workers than jobs, jobs sharing instruments)
    and completes: no worker waits on work queued behind it.  Plans are host-only, so this runs on the CPU."""
    import time
    ex = serve.GpuExecutor("cuda:0", workers=2)
    specs = [serve.JobSpec(j, 0.0, 256, 16, 64, 128 if j % 2 else 64 + 64, "fp32", seed=j) for j in range(6)]
    for sp in specs:
        ex.prefetch(sp, 64)
    t0 = time.time()
    while not all(ex.ready(sp) for sp in specs):
        assert time.time() - t0 < 60, "set-up did not finish"
        time.sleep(0.01)
    sizes = [ex.hbm(sp, 64) for sp in specs]
    assert all(s > 0 for s in sizes)
    assert len(ex._sites) == 1          # one instrument shape shared by every job


def test_small_job_is_not_held_by_a_large_one():
    """Jobs advance on their own completions: a small job admitted next to a large one finishes long before it
    (in lockstep rounds it would wait for the large job's block every round)."""
    big = JobSpec(0, 0.0, 4096, 256, 4096, 512)
    small = JobSpec(1, 0.0, 256, 16, 256, 128)
    ex = ModelExecutor(cs_per_s=1e6)
    st = Scheduler(ex, hbm_budget=1 << 45, max_slots=4, block=64).run([big, small], realtime=False)
    assert st.summary()["jobs_completed"] == 2
    # latencies are recorded in completion order: the small job completes first
    assert st.latencies[0] < 0.1 * st.latencies[1]


def test_backfill_admits_jobs_that_fit_while_the_head_waits():
    """Job 0 runs; job 1 (the head) needs more memory than is left and waits; the later jobs 2, 3 fit and are
    admitted before it (backfill); job 1 is admitted once job 0 has finished."""
    big = JobSpec(0, 0.0, 1024, 64, 1024, 256)
    head = JobSpec(1, 0.0, 1024, 64, 512, 256)
    smalls = [JobSpec(2 + k, 0.0, 256, 16, 128, 128) for k in range(2)]
    ex = ModelExecutor(cs_per_s=1e6)
    need_big = ex.hbm(big, 64, 2)
    need_small = ex.hbm(smalls[0], 64, 2)
    budget = need_big + 2 * need_small + need_small // 2      # job 1 cannot run beside job 0, the smalls can
    st = Scheduler(ex, hbm_budget=budget, max_slots=8, block=64, max_head_wait=1e9).run([big, head] + smalls,
                                                                                        realtime=False)
    assert st.summary()["jobs_completed"] == 4
    assert st.order == [0, 2, 3, 1], st.order
    assert st.backfilled == 2


def test_backfill_stops_once_the_head_has_waited_long_enough():
    """With a short head-wait bound, small jobs that keep arriving stop overtaking the waiting head: it is admitted
    before the last of them."""
    big = JobSpec(0, 0.0, 1024, 64, 2048, 256)
    head = JobSpec(1, 0.001, 1024, 64, 512, 256)
    smalls = [JobSpec(2 + k, 0.002 + 0.05 * k, 256, 16, 64, 128) for k in range(60)]
    ex = ModelExecutor(cs_per_s=1e6)
    need_big = ex.hbm(big, 64, 2)
    budget = need_big + ex.hbm(smalls[0], 64, 2) * 2
    st = Scheduler(ex, hbm_budget=budget, max_slots=8, block=64, max_head_wait=0.05).run([big, head] + smalls,
                                                                                         realtime=False)
    assert st.summary()["jobs_completed"] == 62
    pos = st.order.index(1)
    assert pos < len(st.order) - 10, st.order      # the head did not wait for every later small job
    assert st.backfilled >= 1


def test_failed_jobs_release_their_memory_and_serving_continues():
    """A job that fails while being set up, started, stepped or read out is counted failed, its memory returns to
    the budget, and every other job completes.  With a budget of one job at a time, a failure that kept its
    memory would stall every later job."""
    jobs = [JobSpec(i, 0.0, 256, 16, 256, 128) for i in range(8)]
    ex = ModelExecutor(cs_per_s=1e6, fail={1: "prepare", 3: "start", 4: "step", 6: "finish"})
    need = ex.hbm(jobs[0], 64, 2)
    st = Scheduler(ex, hbm_budget=need, max_slots=4, block=64).run(jobs, realtime=False)
    s = st.summary()
    assert s["failed"] == 4 and s["jobs_completed"] == 4, (s, st.errors)
    assert set(st.errors) == {1, 3, 4, 6}
    assert sorted(ex.released) == [4, 6]
    assert "step" in st.errors[4]


def test_depth_doubles_only_while_slots_are_free():
    """A job running alone keeps up to twice the block depth enqueued; with every slot busy each keeps the
    configured depth (more would hold the hardware queues other jobs' streams share)."""
    alone = serve.JobSpec(0, 0.0, 256, 16, 64 * 20, 128, "fp32")
    ex = ModelExecutor()
    Scheduler(ex, hbm_budget=1 << 40, max_slots=4, block=64, depth=2).run([alone], realtime=False)
    assert ex.max_inflight[0] == 4
    busy = [serve.JobSpec(j, 0.0, 256, 16, 64 * 20, 128, "fp32") for j in range(4)]
    ex = ModelExecutor()
    Scheduler(ex, hbm_budget=1 << 40, max_slots=4, block=64, depth=2).run(busy, realtime=False)
    # while all four run each keeps two; the last one left alone may go to four
    assert all(ex.max_inflight[j] <= 4 for j in range(4)) and min(ex.max_inflight.values()) == 2
