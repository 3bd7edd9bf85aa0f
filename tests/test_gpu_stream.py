"""The streaming form of the fused path (one persistent launch per grid size, row-transformed samples passed
through a per-XCD ring in cache) against the two-pass form, bit for bit, and against the oracle."""
import numpy as np
import pytest
import torch

from oracle import moff_oracle as ora
from paper_0812_3669_amd import api, configs, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _small(n, P=2, A=40, C=2, T=9, K=4, seed=0, int8=True):
    return configs.scaled(configs.PLAIN, index=300 + seed, n_ant=A, n_pol=P, n_chan=C, n_time=T, ksize=K,
                          grid_n=n, disk_lambda=0.6 * n, int8=int8)


def _same(a1, a2, plan):
    """Streaming and two-pass accumulators: equal up to FP32 rounding of the same sums (the two kernels are
    compiled separately, so the compiler may contract multiply-adds differently); report how many differ."""
    d = (a1 - a2).abs()
    scale = max(float(a2.abs().max()), 1e-30)
    nd = int((d > 0).sum())
    print(f"stream vs two-pass: {nd} of {a1.numel()} differ, max rel {float(d.max()) / scale:.3g}", flush=True)
    assert float(d.max()) <= 1e-6 * scale


def _both(cfg, geo, kern, volts, **kw):
    plan = api.plan_for(cfg, geo, **kw).bind(DEV)
    plan.set_kernels(torch.from_numpy(np.ascontiguousarray(kern)).to(DEV))
    v = torch.from_numpy(np.ascontiguousarray(volts)).to(DEV)
    a2 = plan.new_accumulator()
    plan.correlate(v, a2)
    plan.set_pipeline(api.PIPELINE_STREAM)
    a1 = plan.new_accumulator()
    print(f"stream: n={plan.grid_n[0]} C={cfg.n_chan} T={volts.shape[0]}", flush=True)
    plan.correlate(v, a1)
    torch.cuda.synchronize()
    assert plan.stream_status() == 0
    return plan, a1, a2


@pytest.mark.parametrize("n,P,K,A,C,T,tb,acc", [
    (64, 2, 4, 40, 9, 37, 8, api.ACC_FP32),
    (64, 1, 4, 40, 9, 37, 8, api.ACC_FP32),
    (128, 2, 6, 70, 3, 19, 0, api.ACC_FP32),
    (128, 1, 6, 70, 3, 19, 0, api.ACC_FP32),
    (256, 2, 4, 90, 10, 20, 0, api.ACC_FP64_COMP),
    (512, 2, 4, 31, 2, 5, 0, api.ACC_FP32),
])
def test_stream_matches_two_pass(n, P, K, A, C, T, tb, acc):
    cfg = _small(n, P=P, A=A, C=C, T=T, K=K, seed=n)
    geo, kern, volts = synth.workload(cfg)
    plan, a1, a2 = _both(cfg, geo, kern, volts, time_block=tb, acc_mode=acc)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    errs = {}
    for name, a in (("stream", a1), ("two-pass", a2)):
        imgs = [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(a)]
        errs[name] = max(float(ora.relative_errors(imgs[c], ref[c]).max()) for c in range(cfg.n_chan))
    print(f"oracle errors: {errs}", flush=True)
    assert errs["two-pass"] <= 1e-5 and errs["stream"] <= 1e-5, errs
    _same(a1, a2, plan)


def test_stream_against_oracle_and_jones():
    cfg = _small(128, A=50, C=3, T=11, seed=5)
    geo, kern, volts = synth.workload(cfg)
    plan, a1, _ = _both(cfg, geo, kern, volts)
    imgs = [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(a1)]
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    for c in range(cfg.n_chan):
        assert np.all(ora.relative_errors(imgs[c], ref[c]) <= 1e-5), c
    rng = np.random.default_rng(3)
    J = np.zeros(kern.shape[:2] + (2, 2) + kern.shape[3:], dtype=np.complex64)
    for p in range(2):
        J[:, :, p, p] = kern[:, :, p]
        J[:, :, p, 1 - p] = 0.3 * (rng.standard_normal(kern[:, :, p].shape) +
                                   1j * rng.standard_normal(kern[:, :, p].shape))
    plan, a1, a2 = _both(cfg, geo, J, volts, kernel_mode=api.KERNEL_JONES)
    _same(a1, a2, plan)


def test_stream_several_grid_sizes_and_graph_replay():
    cfg = configs.scaled(configs.BATCHED, n_ant=48, n_chan=12, n_time=21)
    geo, kern, volts = synth.workload(cfg)
    plan, a1, a2 = _both(cfg, geo, kern, volts, time_block=8)
    assert len(set(plan.grid_n)) >= 4
    _same(a1, a2, plan)
    v = torch.from_numpy(volts).to(DEV)
    a3 = plan.new_accumulator()
    for _ in range(2):
        a3.zero_()
        plan.correlate_graph(v, a3)
        torch.cuda.synchronize()
        assert plan.stream_status() == 0
        assert torch.equal(a3, a1)


def test_stream_headline_slice():
    """2048 antennas, 128 channels, 256^2, 256 device-drawn samples: streaming equals two-pass."""
    cfg = configs.HEADLINE
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    kern = synth.kernels(geo, g, cfg.n_pol)
    volts = synth.DeviceVoltages(cfg, geo, g, synth.sky(cfg), torch.device(DEV), chunk=64).all(256)
    plan = api.plan_for(cfg, geo).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    a2 = plan.new_accumulator()
    plan.correlate(volts, a2)
    plan.set_pipeline(api.PIPELINE_STREAM)
    a1 = plan.new_accumulator()
    plan.correlate(volts, a1)
    torch.cuda.synchronize()
    assert plan.stream_status() == 0
    _same(a1, a2, plan)
