"""The no-alloc entry point (moff_correlate_noalloc) against moff_correlate, through the C ABI.

Two calls in a row on fresh accumulators, the second with a smaller input; each compared with moff_correlate on
the same plan and samples, per image (channel x product) to the parity tolerance (max |a - b| / max |b| <= 1e-5,
cross products scaled by sqrt(max XX max YY)): the fixed exchange buffer changes the launch blocks and so the FP32
summation order, nothing else.  Cases: 128^2 grids, 35 channels and 300 samples (blocks of 32 channels x 8 samples
and 3 channels x 85 samples); 512^2 grids, 20 channels (16 channels x 1 sample, 4 channels x 4 samples); the split
FP16 transform at 256^2 (3 channels x 21 samples).
"""
import numpy as np
import pytest
import torch

from oracle import moff_oracle as ora
from paper_0812_3669_amd import api, configs, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
DEV = "cuda:0"


def _case(n, C, T, A, fft=api.FFT_FP32, seed=0):
    cfg = configs.scaled(configs.PLAIN, index=300 + seed, n_ant=A, n_chan=C, n_time=T, grid_n=n,
                         disk_lambda=0.5 * n)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=fft).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    return cfg, plan, torch.from_numpy(volts).to(DEV)


def _images(plan, acc):
    return [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(acc)]


@pytest.mark.parametrize("n,C,T,A,fft,T2", [(128, 35, 300, 50, api.FFT_FP32, 37), (512, 20, 5, 30, api.FFT_FP32, 2),
                                            (256, 3, 70, 40, api.FFT_SPLIT_FP16, 9)])
def test_noalloc_matches_correlate_on_two_calls(n, C, T, A, fft, T2):
    cfg, plan, v = _case(n, C, T, A, fft=fft, seed=n)
    for nt in (T, T2):
        ref = plan.new_accumulator()
        plan.correlate(v, ref, n_t=nt)
        got = plan.new_accumulator()
        plan.correlate_noalloc(v, got, n_t=nt)
        a, b = _images(plan, got), _images(plan, ref)
        torch.cuda.synchronize()
        worst = 0.0
        for c in range(cfg.n_chan):
            e = ora.relative_errors(a[c], b[c])
            worst = max(worst, float(e.max()))
            assert np.all(e <= TOL), (n, nt, c, e)
        print(f"noalloc n={n} fft={fft} samples={nt}: worst per-image difference from moff_correlate {worst:.2e}",
              flush=True)


def test_noalloc_rejects_bad_arguments(lib):
    cfg, plan, v = _case(64, 2, 4, 20)
    acc = plan.new_accumulator()
    assert lib.moff_correlate_noalloc(None, None, 0, None, None) == api._lib.MOFF_E_INVALID
    assert lib.moff_correlate_noalloc(plan._h, None, 4, api._ptr(acc), None) == api._lib.MOFF_E_INVALID
    assert lib.moff_correlate_noalloc(plan._h, api._ptr(v), -1, api._ptr(acc), None) == api._lib.MOFF_E_INVALID
