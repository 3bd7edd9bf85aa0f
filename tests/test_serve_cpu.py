"""CPU tests of the serving scheduler with a modelled executor: admission by HBM budget and slots, arrival-order
queueing, rejection of jobs that can never fit, latency accounting."""
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
    need = hbm_bytes(job, 64)
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
    assert big.fft_mode == "fp32" and a.fft_mode == "split_fp16"
    cpl = big.chans_per_launch(64)
    assert cpl >= 1 and 64 * cpl * 2 * 512 ** 2 * 8 <= (1 << 30)


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
