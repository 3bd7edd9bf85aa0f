"""CPU tests of the Python binding's buffer checks: every pointer handed to the C ABI is a contiguous tensor on
the plan's device, of the right dtype and at least the size the call reads or writes.  A bad buffer raises
ValueError (also under ``python -O``) before anything reaches the library.  The plan's device is set to torch's
``meta`` device, so the checks run here without a GPU; no call below reaches the device."""
import numpy as np
import pytest
import torch

from paper_0812_3669_amd import api, configs, synth

META = torch.device("meta")


def _plan(acc_mode=api.ACC_FP32, n_tap=0, fft_mode=api.FFT_FP32):
    cfg = configs.scaled(configs.PLAIN, n_ant=20, n_chan=2, grid_n=64, disk_lambda=30.0, n_time=8)
    geo = synth.geometry(cfg)
    plan = api.plan_for(cfg, geo, acc_mode=acc_mode, n_tap=n_tap, fft_mode=fft_mode)
    plan.device = META          # stands in for a bound device: only the checks run
    return cfg, plan


def _volts(cfg, T, device=META):
    return torch.empty((T, cfg.n_chan, cfg.n_ant, cfg.n_pol, 2), dtype=torch.int8, device=device)


def _acc(plan, dtype=torch.float32, device=META, short=0):
    elems = plan.acc_bytes // (8 if dtype == torch.float64 else 4) - short
    return torch.empty(elems, dtype=dtype, device=device)


def test_unbound_plan_rejects_buffers():
    cfg, plan = _plan()
    plan.device = None
    with pytest.raises(ValueError, match="not bound"):
        plan.correlate(_volts(cfg, 4), _acc(plan))


def test_accumulator_dtype_must_match_the_accumulator_mode():
    cfg, plan = _plan(acc_mode=api.ACC_FP64_COMP)
    with pytest.raises(ValueError, match="dtype"):
        plan.correlate(_volts(cfg, 4), _acc(plan, torch.float32))
    with pytest.raises(ValueError, match="dtype"):
        plan.correlate_graph(_volts(cfg, 4), _acc(plan, torch.float32))
    with pytest.raises(ValueError, match="dtype"):
        plan.read_image(_acc(plan, torch.float32))


@pytest.mark.parametrize("acc_mode,dt", [(api.ACC_FP32, torch.float32), (api.ACC_FP64_COMP, torch.float64)])
def test_accumulator_too_small(acc_mode, dt):
    cfg, plan = _plan(acc_mode=acc_mode)
    with pytest.raises(ValueError, match="bytes"):
        plan.correlate(_volts(cfg, 4), _acc(plan, dt, short=1))
    with pytest.raises(ValueError, match="bytes"):
        plan.read_image(_acc(plan, dt, short=1))
    with pytest.raises(ValueError, match="bytes"):
        plan.autotune(_volts(cfg, 4), _acc(plan, dt, short=1), n_t=4)


def test_voltages_checked_for_dtype_size_layout_and_device():
    cfg, plan = _plan()
    acc = _acc(plan)
    with pytest.raises(ValueError, match="bytes"):
        plan.correlate(_volts(cfg, 3), acc, n_t=4)
    with pytest.raises(ValueError, match="dtype"):
        plan.correlate(_volts(cfg, 4).to(torch.int16), acc)
    v = torch.empty((4, cfg.n_chan, cfg.n_ant, cfg.n_pol, 4), dtype=torch.int8, device=META)[..., :2]
    with pytest.raises(ValueError, match="contiguous"):
        plan.correlate(v, acc)
    with pytest.raises(ValueError, match="must be on"):
        plan.correlate(_volts(cfg, 4, device="cpu"), acc)
    with pytest.raises(ValueError, match="must be on"):
        plan.correlate(_volts(cfg, 4), _acc(plan, device="cpu"))
    with pytest.raises(ValueError, match="n_t"):
        plan.correlate(_volts(cfg, 4), acc, n_t=-1)


def test_staged_buffers_checked():
    cfg, plan = _plan()
    T = 3
    grid_elems = T * cfg.n_pol * plan.pix_total
    with pytest.raises(ValueError, match="bytes"):
        plan.fft(torch.empty(grid_elems - 1, dtype=torch.complex64, device=META), T)
    with pytest.raises(ValueError, match="dtype"):
        plan.fft(torch.empty(grid_elems, dtype=torch.float32, device=META), T)
    with pytest.raises(ValueError, match="bytes"):
        plan.grid(_volts(cfg, T), out=torch.empty(grid_elems - 1, dtype=torch.complex64, device=META))
    with pytest.raises(ValueError, match="bytes"):
        plan.accumulate(torch.empty(grid_elems - 1, dtype=torch.complex64, device=META), T, _acc(plan))
    with pytest.raises(ValueError, match="bytes"):
        plan.accumulate(torch.empty(grid_elems, dtype=torch.complex64, device=META), T, _acc(plan, short=1))
    with pytest.raises(ValueError, match="bytes"):
        plan.debug_unpack(torch.empty(cfg.n_chan * cfg.n_ant * cfg.n_pol * 2 - 1, dtype=torch.int8, device=META))


def test_kernel_and_phase_shapes_checked():
    cfg, plan = _plan()
    K = cfg.ksize
    with pytest.raises(ValueError, match="shape"):
        plan.set_kernels(torch.empty((cfg.n_chan, cfg.n_ant, cfg.n_pol, K * K), dtype=torch.complex64, device=META))
    with pytest.raises(ValueError, match="dtype"):
        plan.set_kernels(torch.empty((cfg.n_chan, cfg.n_ant, cfg.n_pol, K, K), dtype=torch.complex128,
                                     device=META))
    kern = torch.empty((cfg.n_chan, cfg.n_ant, cfg.n_pol, K, K), dtype=torch.complex64, device=META)
    with pytest.raises(ValueError, match="phase"):
        plan.set_kernels(kern, phase=torch.empty((cfg.n_chan, cfg.n_ant, 1), dtype=torch.complex64, device=META))


def test_tap_and_calibration_buffers_checked():
    cfg, plan = _plan(n_tap=2)
    T = 4
    tap = torch.empty((T, cfg.n_chan, 2, cfg.n_pol), dtype=torch.complex64, device=META)
    with pytest.raises(ValueError, match="bytes"):
        plan.correlate_tap(_volts(cfg, T), _acc(plan), tap[:T - 1])
    with pytest.raises(ValueError, match="bytes"):
        plan.cal_accumulate(_volts(cfg, T), tap, torch.empty(plan.cal_bytes // 8 - 1, dtype=torch.float64,
                                                                 device=META))
    with pytest.raises(ValueError, match="dtype"):
        plan.cal_solve(torch.empty(plan.cal_bytes // 4, dtype=torch.float32, device=META),
                       torch.empty((cfg.n_chan, cfg.n_ant, cfg.n_pol, cfg.ksize, cfg.ksize), dtype=torch.complex64,
                                   device=META))
    with pytest.raises(ValueError, match="shape"):
        plan.set_taps(np.zeros((cfg.n_chan, 3, 2), dtype=np.int32))


def test_probe_buffer_checked():
    with pytest.raises(ValueError):
        api.probe(0, 4, 1, torch.empty(4 * 256, dtype=torch.float32))


def test_autotune_key_names_every_input_of_the_shape_choice():
    """Identical plans share the autotuner cache key; a different transform, accumulator, grid size, antenna count
    or channel count changes it.  Host only (the compute-unit count is 0 until the plan is bound)."""
    cfg = configs.scaled(configs.PLAIN, n_ant=20, n_chan=2, grid_n=64, disk_lambda=30.0, n_time=8)
    geo = synth.geometry(cfg)
    k0 = api.plan_for(cfg, geo).autotune_key
    assert k0 == api.plan_for(cfg, geo).autotune_key
    assert "\t" not in k0 and "\n" not in k0 and k0.startswith("cu=0 ")
    others = [api.plan_for(cfg, geo, fft_mode=api.FFT_GEMM_FP16).autotune_key,
              api.plan_for(cfg, geo, acc_mode=api.ACC_FP64_COMP).autotune_key]
    for kw in (dict(grid_n=128), dict(n_ant=21), dict(n_chan=3)):
        c2 = configs.scaled(configs.PLAIN, **{**dict(n_ant=20, n_chan=2, grid_n=64, disk_lambda=30.0, n_time=8),
                                               **kw})
        others.append(api.plan_for(c2, synth.geometry(c2)).autotune_key)
    assert len(set(others + [k0])) == len(others) + 1


def test_unbind_releases_the_device_and_blocks_calls():
    """An unbound plan (its workspace released for reuse by a later job) refuses every device call until it is
    bound again; its host-side queries still work."""
    cfg, plan = _plan()
    ws = plan.workspace_bytes
    plan.unbind()
    assert plan.device is None and plan.workspace_bytes == ws
    with pytest.raises(ValueError, match="not bound"):
        plan.correlate(_volts(cfg, 4), _acc(plan))
    with pytest.raises(ValueError, match="not bound"):
        plan.set_kernels(torch.empty((cfg.n_chan, cfg.n_ant, cfg.n_pol, cfg.ksize, cfg.ksize),
                                     dtype=torch.complex64, device=META))
