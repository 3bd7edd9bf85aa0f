"""Serving form on the GPU: jobs admitted by HBM budget, overlapping on their own streams; each job's image is
the same alone and in a mix (bit for bit); small FP32 and split-FP16 jobs match the oracle; a job whose set-up
fails (forced on the host) is counted failed while the others complete."""
import time

import numpy as np
import pytest
import torch

from oracle import moff_oracle as ora
from paper_0812_3669_amd import serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5

JOBS = [
    serve.JobSpec(0, 0.0, 256, 16, 128, 128, "fp32", seed=11),
    serve.JobSpec(1, 0.0, 256, 16, 96, 256, "split_fp16", seed=12),
    serve.JobSpec(2, 0.0, 1024, 16, 64, 128, "fp32", seed=13),
]
OTHERS = [
    serve.JobSpec(3, 0.0, 1024, 64, 192, 256, "fp32", seed=14),
    serve.JobSpec(4, 0.001, 256, 64, 128, 512, "fp32", seed=15),
    serve.JobSpec(5, 0.002, 4096, 16, 64, 256, "split_fp16", seed=16),
]


def _run(trace, slots, ex=None):
    ex = ex or serve.GpuExecutor(DEV)
    # every job's host set-up is finished before the trace starts, so admission is bounded by the slots alone and
    # the mix overlaps however fast the jobs run
    for j in trace:
        ex.prefetch(j, 64)
    t_end = time.time() + 120
    while not all(ex.ready(j) for j in trace):
        assert time.time() < t_end, "job set-up did not finish"
        time.sleep(0.005)
    sch = serve.Scheduler(ex, hbm_budget=64 << 30, max_slots=slots, block=64, keep_results=True)
    st = sch.run(trace, realtime=False)
    torch.cuda.synchronize()
    return st


def test_each_job_same_alone_and_in_the_mix():
    alone = {}
    for j in JOBS:
        st = _run([j], 1)
        alone[j.job_id] = st.results[j.job_id].cpu()
    mix = JOBS + OTHERS
    st = _run(mix, 4)
    assert st.peak_concurrent >= 3, st.summary()
    assert len(st.latencies) == len(mix)
    for j in JOBS:
        assert torch.equal(alone[j.job_id], st.results[j.job_id].cpu()), j


@pytest.mark.parametrize("j", [JOBS[0], serve.JobSpec(7, 0.0, 256, 16, 80, 128, "split_fp16", seed=17)],
                         ids=["fp32", "split_fp16"])
def test_small_job_against_oracle(j):
    st = _run([j], 1)
    img = st.results[j.job_id].cpu().numpy().astype(np.complex128)
    cfg, scfg = j.config(), j.site_config()
    geo = synth.geometry(scfg)
    g = synth.gains(scfg)
    kern = synth.kernels(geo, g, 2)
    volts = synth.DeviceVoltages(cfg, geo, g, synth.sky(cfg), torch.device(DEV), chunk=64).all(j.n_time)
    n = j.grid_n
    sel = [0, j.n_chan - 1]
    ref = ora.image(volts[:, sel].cpu().numpy(), kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel],
                    scfg.cell_lambda)
    for k, c in enumerate(sel):
        got = img[c * 4 * n * n:(c + 1) * 4 * n * n].reshape(4, n, n)
        e = ora.relative_errors(got, ref[k])
        assert np.all(e <= TOL), (c, e)


class _FailingSetup(serve.GpuExecutor):
    """Host-side failure: the plan of one job cannot be built (as a plan the library rejects would be)."""

    def _prepare(self, spec, block):
        if spec.job_id == 99:
            raise RuntimeError("plan rejected for job 99")
        return super()._prepare(spec, block)


def test_failed_job_does_not_stop_the_others():
    mix = JOBS + [serve.JobSpec(99, 0.0, 256, 16, 64, 128, "fp32", seed=99)]
    st = _run(mix, 4, ex=_FailingSetup(DEV))
    s = st.summary()
    assert s["failed"] == 1 and 99 in st.errors and s["jobs_completed"] == len(JOBS), (s, st.errors)
    alone = _run([JOBS[0]], 1)
    assert torch.equal(alone.results[0].cpu(), st.results[0].cpu())


def test_plans_reused_across_jobs_of_one_shape():
    """Jobs of one shape run one after another reuse the first job's plan (unbound when it ends, bound again for
    the next): one plan built for three jobs, and each image equals the one a fresh executor computes alone."""
    same = [serve.JobSpec(20 + k, 0.0, 256, 16, 64 + 16 * k, 128, "fp32", seed=30 + k) for k in range(3)]
    ex = serve.GpuExecutor(DEV)
    got = {}
    for j in same:
        st = _run([j], 1, ex)
        got[j.job_id] = st.results[j.job_id].cpu()
    assert ex.plans_built == 1 and ex.plans_reused == 2, (ex.plans_built, ex.plans_reused)
    for j in same:
        fresh = _run([j], 1)
        assert torch.equal(fresh.results[j.job_id].cpu(), got[j.job_id]), j
