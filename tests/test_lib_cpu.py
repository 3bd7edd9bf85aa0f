"""CPU tests of the C-ABI library: it loads, exports every declared function, validates plans, and its host
plan (footprints, row bands) matches an independent recompute bit for bit.  No compute calls (no GPU here)."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_0812_3669_amd import _lib, configs, synth
from paper_0812_3669_amd.api import MoffError, Plan


def test_library_exports_every_declared_function(lib):
    names = _lib.header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib._SIGS), set(names) ^ set(_lib._SIGS)


def test_status_strings(lib):
    assert lib.moff_status_str(0) == b"MOFF_OK"
    assert lib.moff_status_str(1) == b"MOFF_E_INVALID"
    assert lib.moff_status_str(4) == b"MOFF_E_UNSUPPORTED"


def test_probe_rejects_bad_arguments(lib):
    """moff_probe validates on the host before anything is enqueued (MOFF_E_INVALID = 1)."""
    out = C.c_void_p(256)   # never dereferenced: every call below fails validation
    assert lib.moff_probe(7, 1, 1, out, None) == 1
    assert lib.moff_probe(-1, 1, 1, out, None) == 1
    assert lib.moff_probe(0, 0, 1, out, None) == 1
    assert lib.moff_probe(1, 1, 0, out, None) == 1
    assert lib.moff_probe(0, 1, 1, None, None) == 1


def _geo(cfg):
    return synth.geometry(cfg)


@pytest.mark.parametrize("name", ["tiny", "plain", "headline"])
def test_footprints_and_bands_match_independent_recompute(name):
    cfg = configs.CONFIGS[name]
    if name == "headline":
        cfg = configs.scaled(cfg, n_chan=6)
    geo = _geo(cfg)
    plan = Plan(geo.ant_xy_m, geo.freqs_hz, geo.grid_n, n_pol=cfg.n_pol, ksize=cfg.ksize)
    origin, ptr, ant, rows = plan.debug_tiles()
    K = cfg.ksize
    band = 0
    for c in range(cfg.n_chan):
        n = int(geo.grid_n[c])
        s = geo.freqs_hz[c] / configs.C_LIGHT / cfg.cell_lambda
        X = geo.ant_xy_m[:, 0] * s + n / 2
        Y = geo.ant_xy_m[:, 1] * s + n / 2
        i0 = np.floor(X).astype(np.int64) - K // 2 + 1
        j0 = np.floor(Y).astype(np.int64) - K // 2 + 1
        assert np.array_equal(origin[c, :, 0], j0)
        assert np.array_equal(origin[c, :, 1], i0)
        h = rows[c]
        assert h in (4, 8, 16) and cfg.n_pol * h * n * 8 <= (32768 if n & (n - 1) == 0 else 16384)
        jmin, jmax = j0.min(), j0.max() + K - 1
        for b in range(jmin // h, jmax // h + 1):
            lo, hi = b * h, min(n, b * h + h) - 1
            expect = np.nonzero((j0 <= hi) & (j0 + K - 1 >= lo))[0]
            got = ant[ptr[band]:ptr[band + 1]]
            assert np.array_equal(got, expect), (c, b)
            band += 1
    assert band == len(ptr) - 1


def test_boundary_antennas_listed_in_both_bands():
    # an antenna whose 4 x 4 footprint straddles a band boundary belongs to both bands (module-boundary copy)
    xy = np.array([[0.0, -0.5], [3.0, 2.0]])  # footprint rows of antenna 0 around the grid centre
    plan = Plan(xy, [configs.C_LIGHT], [32], n_pol=1, ksize=4)
    origin, ptr, ant, rows = plan.debug_tiles()
    h = rows[0]
    j0 = origin[0, 0, 0]
    bands_of_0 = [b for b in range(len(ptr) - 1) if 0 in ant[ptr[b]:ptr[b + 1]]]
    assert len(bands_of_0) == len({j0 // h, (j0 + 3) // h})


@pytest.mark.parametrize("kw,status", [
    (dict(ksize=3), 1), (dict(ksize=10), 1), (dict(n_pol=3), 1), (dict(grid_n=[48]), 4),
    (dict(grid_n=[16]), 4), (dict(cell_lambda=0.0), 1), (dict(fft_mode=7), 1), (dict(acc_mode=5), 1),
    (dict(kernel_mode=2), 1), (dict(kernel_mode=1, n_pol=1), 1),
    (dict(kernel_mode=1, grid_n=[256], fft_mode=1), 4),
])
def test_plan_validation(kw, status):
    xy = np.array([[1.0, 2.0], [-3.0, 4.0], [5.0, -6.0]])
    args = dict(ant_xy_m=xy, freqs_hz=[configs.C_LIGHT], grid_n=[32], n_pol=2, ksize=4)
    args.update(kw)
    with pytest.raises(MoffError) as ei:
        Plan(**args)
    assert ei.value.status == status


def test_antenna_count_limits():
    """Antenna fields are 16 bits wide: 65534 antennas plan, 65535 do not; the matrix-core row pass rejects rows
    whose antenna lists outgrow its LDS (MOFF_E_UNSUPPORTED) instead of launching them."""
    rng = np.random.default_rng(5)
    r = 0.3 * 256 * np.sqrt(rng.random(65535))
    phi = 2 * np.pi * rng.random(65535)
    xy = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)
    args = dict(freqs_hz=[configs.C_LIGHT], grid_n=[256], n_pol=2, ksize=4)
    Plan(ant_xy_m=xy[:65534], **args)
    with pytest.raises(MoffError) as ei:
        Plan(ant_xy_m=xy, **args)
    assert ei.value.status == 1
    with pytest.raises(MoffError) as ei:
        Plan(ant_xy_m=xy[:65534], fft_mode=3, **args)
    assert ei.value.status == 4


def test_footprint_outside_grid_is_invalid():
    xy = np.array([[14.0, 0.0]])     # X = 30 on a 32 grid: footprint 29..32 leaves the grid
    with pytest.raises(MoffError) as ei:
        Plan(xy, [configs.C_LIGHT], [32], n_pol=1, ksize=4)
    assert ei.value.status == 1
    assert "leaves" in str(ei.value)
    Plan(np.array([[13.0, 0.0]]), [configs.C_LIGHT], [32], n_pol=1, ksize=4)   # X = 29: cells 28..31 fit


def test_auto_grid_size_and_offsets():
    cfg = configs.BATCHED
    cfg = configs.scaled(cfg, n_ant=64, n_chan=8)
    geo = _geo(cfg)
    plan = Plan(geo.ant_xy_m, geo.freqs_hz, None, n_pol=2, ksize=cfg.ksize)
    assert all(n in configs.ALLOWED_GRID_SIZES for n in plan.grid_n)
    assert plan.grid_n == sorted(plan.grid_n)
    off = 0
    for c, n in enumerate(plan.grid_n):
        assert plan.pix_off[c] == off
        off += n * n
    assert plan.acc_bytes == off * 4 * 4
    assert plan.image_bytes == off * 4 * 8
    assert plan.workspace_bytes > 0


def test_state_errors_without_bind(lib):
    xy = np.array([[1.0, 2.0]])
    plan = Plan(xy, [configs.C_LIGHT], [32], n_pol=1, ksize=4)
    st = lib.moff_correlate(plan._h, C.c_void_p(1), 1, C.c_void_p(1), None)
    assert st == 5  # MOFF_E_STATE
    assert lib.moff_grid(plan._h, None, -1, None, None) == 1
    small = C.c_size_t(16)
    assert lib.moff_bind(plan._h, C.c_void_p(256), small, None) == 2   # MOFF_E_BUDGET, nothing enqueued


def test_cost_model_counts():
    # Discussion: MWA FX load = 31 MHz x 125,000 baselines x 4 pols = 15.5e12 cmacs/s
    assert 31e6 * 125000 * 4 == pytest.approx(15.5e12)
    # algorithmic flops per channel-sample of the headline workload (5 n^2 log2 n^2 per pol FFT)
    f = configs.HEADLINE.flops_per_cs()
    assert f == pytest.approx(2 * 5 * 65536 * 16 + 8 * 2048 * 2 * 16 + 16 * 65536)
    assert f / 1e6 == pytest.approx(12.06, abs=0.01)


def test_split_precision_transform_needs_256_grids_and_two_pols():
    xy = np.array([[1.0, 2.0], [-3.0, 4.0]])
    for kw in (dict(grid_n=[128], n_pol=2), dict(grid_n=[256], n_pol=1)):
        with pytest.raises(MoffError) as ei:
            Plan(xy, [configs.C_LIGHT], fft_mode=1, ksize=4, **kw)
        assert ei.value.status == 4
    Plan(xy, [configs.C_LIGHT], [256], n_pol=2, ksize=4, fft_mode=1)
    Plan(xy, [configs.C_LIGHT], [256], n_pol=2, ksize=4, fft_mode=2)


def test_jones_kernels_pack_four_planes():
    xy = np.array([[1.0, 2.0], [-3.0, 4.0]])
    diag = Plan(xy, [configs.C_LIGHT], [32], n_pol=2, ksize=4)
    jones = Plan(xy, [configs.C_LIGHT], [32], n_pol=2, ksize=4, kernel_mode=1)
    assert jones._kernel_shape() == (1, 2, 2, 2, 4, 4)
    assert diag._kernel_shape() == (1, 2, 2, 4, 4)
    # the packed kernel table doubles (four planes instead of two); nothing else in the workspace changes
    assert jones.workspace_bytes > diag.workspace_bytes
    assert jones.acc_bytes == diag.acc_bytes


def test_pipeline_validation():
    xy = np.array([[1.0, 2.0], [-3.0, 4.0]])
    plan = Plan(xy, [configs.C_LIGHT], [256], n_pol=2, ksize=4, fft_mode=1)
    with pytest.raises(MoffError) as ei:
        plan.set_pipeline(1)
    assert ei.value.status == 4
    plan = Plan(xy, [configs.C_LIGHT], [32], n_pol=2, ksize=4)
    with pytest.raises(MoffError) as ei:
        plan.set_pipeline(5)
    assert ei.value.status == 1
    plan.set_pipeline(1)
    plan.set_pipeline(0)


def test_tap_validation_and_sizes():
    xy = np.array([[1.0, 2.0], [-3.0, 4.0], [5.0, -6.0]])
    with pytest.raises(MoffError) as ei:
        Plan(xy, [configs.C_LIGHT], [32], n_pol=2, ksize=4, n_tap=9)
    assert ei.value.status == 1
    plain = Plan(xy, [configs.C_LIGHT, 2 * configs.C_LIGHT], [32, 64], n_pol=2, ksize=4)
    taps = Plan(xy, [configs.C_LIGHT, 2 * configs.C_LIGHT], [32, 64], n_pol=2, ksize=4, n_tap=3)
    # tap twiddles (n per tap per channel), indices, pixels and footprint origins live in the workspace
    assert taps.workspace_bytes >= plain.workspace_bytes + 3 * (32 + 64) * 8 + 2 * 3 * 8 * 2 + 2 * 3 * 8
    b = C.c_size_t()
    assert taps.lib.moff_cal_size(taps._h, C.byref(b)) == 0
    assert b.value == 2 * 3 * 3 * 2 * 16 + 2 * 3 * 2 * 8 + 2 * 3 * 2 * 8
    # taps need a bound plan made with n_tap > 0
    assert taps.lib.moff_correlate_tap(taps._h, C.c_void_p(1), 1, C.c_void_p(1), C.c_void_p(1), None) == 5
    assert plain.lib.moff_cal_accumulate(plain._h, C.c_void_p(1), C.c_void_p(1), 1, C.c_void_p(1), None) == 5


def test_plan_builder_under_host_sanitizers(tmp_path):
    """The host plan builder compiled with g++ -fsanitize=address,undefined (host code only, no HIP) builds
    plans for several layouts without a memory or undefined-behaviour report."""
    import os
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "plan_sanitizer")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(root, "include"), "-I" + os.path.join(root, "paper_0812_3669_amd", "csrc"),
           os.path.join(root, "tests", "plan_sanitizer_driver.cpp"),
           os.path.join(root, "paper_0812_3669_amd", "csrc", "plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "leaves the 32^2 grid" in r.stdout
