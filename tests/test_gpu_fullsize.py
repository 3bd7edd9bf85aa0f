"""The plain workload at full size against the FP64 oracle: 256 antennas in a 60-wavelength disk, 32 channels over
100-130 MHz (uv scaled per channel), 2 pols, 4x4 kernels, 128^2 grids, all 4096 samples of int8 voltages with
5 point sources, through the default launch shape and graph replay; every channel and every pixel, with the FP32
and the compensated FP64 (sum, carry) accumulator.  The oracle is evaluated once for the module (about three
minutes on 16 host threads)."""
import os
import time

import numpy as np
import pytest
import torch

from oracle import moff_oracle as ora
from paper_0812_3669_amd import api, configs, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
DEV = "cuda:0"


@pytest.fixture(scope="module")
def plain():
    cfg = configs.PLAIN
    geo, kern, volts = synth.workload(cfg)
    t0 = time.perf_counter()
    print(f"\nplain: FP64 oracle for {cfg.n_chan} channels x {cfg.n_time} samples on "
          f"{len(os.sched_getaffinity(0))} host threads", flush=True)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda, t_batch=512)
    print(f"plain: oracle done in {time.perf_counter() - t0:.1f} s", flush=True)
    return cfg, geo, kern, volts, ref


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("acc", [api.ACC_FP32, api.ACC_FP64_COMP], ids=["acc32", "acc64"])
def test_plain_every_channel_every_pixel(plain, acc):
    cfg, geo, kern, volts, ref = plain
    plan = api.plan_for(cfg, geo, acc_mode=acc).bind(DEV)
    assert plan.launch_shape() == (256, 32, 32)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    v = torch.from_numpy(volts).to(DEV)
    a = plan.new_accumulator()
    print(f"plain [acc {acc}]: correlate {cfg.n_chan} channels x {cfg.n_time} samples", flush=True)
    plan.correlate_graph(v, a)
    imgs = [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(a)]
    torch.cuda.synchronize()
    errs = np.array([ora.relative_errors(imgs[c], ref[c]) for c in range(cfg.n_chan)])
    print(f"plain [acc {acc}]: worst per-image error XX {errs[:, 0].max():.2e}  YY {errs[:, 1].max():.2e}  "
          f"XY {errs[:, 2].max():.2e}  YX {errs[:, 3].max():.2e} over {cfg.n_chan} channels", flush=True)
    assert np.all(errs <= TOL), errs.max()
