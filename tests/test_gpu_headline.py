"""The headline workload at full size against the FP64 oracle, every pixel.

2048 antennas in a 200-wavelength disk, 128 channels over 100-130 MHz, two pols, 4x4 kernels, 256^2 grids and all
16384 samples of device-drawn int8 voltages, run through the C ABI in the launch configuration the benchmark times
(default launch shape, graph replay, every channel of the plan).  The lowest and the highest channel are checked
pixel by pixel against the oracle evaluated over the whole integration (computed once for the module), in six
arithmetic forms: FP32 transform with the FP32 accumulator, FP32 transform with the FP64 (sum, carry) accumulator,
the split FP16 and split BF16 matrix-core transforms with the FP64 (sum, carry) accumulator, and the matrix-core
row pass (gridding + row DFT as one split-FP16 GEMM) with either accumulator.  The per-image
errors (XX, YY, XY, YX of each checked channel; max|gpu - oracle| / max|oracle|, the cross products scaled by
sqrt(max XX max YY)) are printed as a table.
"""
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

MODES = [
    ("fp32 transform, fp32 accumulator", api.FFT_FP32, api.ACC_FP32),
    ("fp32 transform, fp64 (sum, carry) accumulator", api.FFT_FP32, api.ACC_FP64_COMP),
    ("split fp16 transform, fp64 (sum, carry) accumulator", api.FFT_SPLIT_FP16, api.ACC_FP64_COMP),
    ("split bf16 transform, fp64 (sum, carry) accumulator", api.FFT_SPLIT_BF16, api.ACC_FP64_COMP),
    ("gemm fp16 row pass, fp32 accumulator", api.FFT_GEMM_FP16, api.ACC_FP32),
    ("gemm fp16 row pass, fp64 (sum, carry) accumulator", api.FFT_GEMM_FP16, api.ACC_FP64_COMP),
]


@pytest.fixture(scope="module")
def headline():
    cfg = configs.HEADLINE
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    sk = synth.sky(cfg)
    kern = synth.kernels(geo, g, cfg.n_pol)
    dev = torch.device(DEV)
    print(f"\nheadline: drawing {cfg.n_time} samples of int8 voltages on the device", flush=True)
    volts = synth.DeviceVoltages(cfg, geo, g, sk, dev, chunk=64).all(cfg.n_time)
    sel = [0, cfg.n_chan - 1]
    v_host = volts[:, sel].cpu().numpy()
    t0 = time.perf_counter()
    print(f"headline: FP64 oracle for channels {sel} x {cfg.n_time} samples on {len(os.sched_getaffinity(0))} "
          "host threads", flush=True)
    ref = ora.image(v_host, kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel], cfg.cell_lambda,
                    t_batch=256)
    print(f"headline: oracle done in {time.perf_counter() - t0:.1f} s", flush=True)
    return cfg, geo, kern, volts, sel, ref


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("label,fft,acc", MODES, ids=["fp32", "fp32_acc64", "split_fp16_acc64", "split_bf16_acc64",
                                                     "gemm_fp16", "gemm_fp16_acc64"])
def test_headline_every_pixel(headline, label, fft, acc):
    cfg, geo, kern, volts, sel, ref = headline
    dev = torch.device(DEV)
    plan = api.plan_for(cfg, geo, fft_mode=fft, acc_mode=acc).bind(dev)
    assert plan.launch_shape() == (256, 32, 32)
    plan.set_kernels(torch.from_numpy(kern).to(dev))
    accb = plan.new_accumulator()
    print(f"headline [{label}]: correlate {cfg.n_chan} channels x {cfg.n_time} samples", flush=True)
    plan.correlate_graph(volts, accb)
    imgs = plan.read_image(accb)
    rows = []
    for k, c in enumerate(sel):
        got = imgs[c].cpu().numpy().astype(np.complex128)
        e = ora.relative_errors(got, ref[k])
        rows.append((c, e))
    torch.cuda.synchronize()
    for c, e in rows:
        print(f"headline [{label}] channel {c:3d}: XX {e[0]:.2e}  YY {e[1]:.2e}  XY {e[2]:.2e}  YX {e[3]:.2e}",
              flush=True)
    for c, e in rows:
        assert np.all(e <= TOL), (label, c, e)
    del plan, accb, imgs
    torch.cuda.empty_cache()
