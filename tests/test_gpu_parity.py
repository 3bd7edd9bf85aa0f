"""GPU parity of the HIP path against the FP64 oracle, element by element, through the C ABI.

Tolerance (per image = channel x product): max|gpu - oracle| / max|oracle| <= 1e-5 for XX and YY, and for XY,
YX the same divided by sqrt(max XX * max YY).  Integer work (voltage unpacking) is bit-exact.
"""
import numpy as np
import pytest
import torch

from oracle import moff_oracle as ora
from paper_0812_3669_amd import api, configs, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
DEV = "cuda:0"


def _setup(cfg, acc_mode=api.ACC_FP32, time_block=0, chans=None, n_time=None):
    geo, kern, volts = synth.workload(cfg, n_time=n_time, chans=chans)
    plan = api.plan_for(cfg, geo, acc_mode=acc_mode, time_block=time_block).bind(DEV)
    plan.set_kernels(torch.from_numpy(np.ascontiguousarray(kern)).to(DEV))
    return geo, kern, volts, plan


def _run_fused(plan, volts, n_time=None):
    acc = plan.new_accumulator()
    v = torch.from_numpy(np.ascontiguousarray(volts)).to(DEV)
    plan.correlate(v, acc, n_t=n_time)
    imgs = [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(acc)]
    torch.cuda.synchronize()
    return imgs, acc


def _check_images(imgs, ref, tol=TOL, label="", report=False):
    worst = 0.0
    for c in range(len(ref)):
        e = ora.relative_errors(imgs[c], ref[c])
        worst = max(worst, float(e.max()))
        if report:
            print(f"{label} channel {c}: per-image errors " + " ".join(f"{x:.2e}" for x in np.ravel(e)), flush=True)
        assert np.all(e <= tol), f"{label} channel {c}: per-product errors {e}"
    return worst


def _small(n, P=2, A=40, C=2, T=9, K=4, seed=0, disk=None, int8=True):
    disk = disk if disk is not None else 0.6 * n
    return configs.scaled(configs.PLAIN, index=100 + seed, n_ant=A, n_pol=P, n_chan=C, n_time=T, ksize=K,
                          grid_n=n, disk_lambda=disk, int8=int8)


# ---------------------------------------------------------------------------------------------------------
# bit-exact integer work
# ---------------------------------------------------------------------------------------------------------
def test_unpack_bit_exact():
    cfg = _small(64, C=3, A=37)
    geo = synth.geometry(cfg)
    plan = api.plan_for(cfg, geo).bind(DEV)
    rng = np.random.default_rng(3)
    v = rng.integers(-128, 128, size=(cfg.n_chan, cfg.n_ant, 2, 2), dtype=np.int64).astype(np.int8)
    v[0, 0, 0] = (-128, 127)
    out = plan.debug_unpack(torch.from_numpy(v).to(DEV)).cpu().numpy()
    assert np.array_equal(out, v.astype(np.float32))


# ---------------------------------------------------------------------------------------------------------
# staged path: each step against the oracle's step
# ---------------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,K", [(64, 4), (128, 6), (256, 4)])
def test_staged_grid(n, K):
    cfg = _small(n, C=2, A=53, T=5, K=K)
    geo, kern, volts, plan = _setup(cfg)
    g = plan.grid(torch.from_numpy(volts).to(DEV))
    grids = [x.cpu().numpy() for x in plan.split_grids(g, cfg.n_time)]
    e = ora.unpack(volts)
    for c in range(cfg.n_chan):
        origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[c], cfg.cell_lambda, n, K)
        for p in range(cfg.n_pol):
            ref = ora.grid_many(e[:, c, :, p], kern[c, :, p], origin, n)
            err = np.abs(grids[c][:, p] - ref).max() / np.abs(ref).max()
            assert err < 1e-6, (c, p, err)


@pytest.mark.parametrize("n", [32, 64, 96, 128, 160, 192, 256, 320, 384, 512])
def test_staged_fft_every_size(n):
    """moff_fft on oracle-made grids (rounded to complex64) against the oracle's direct DFT."""
    cfg = _small(n, C=1, A=24, T=2, disk=0.5 * n)
    geo, kern, volts, plan = _setup(cfg)
    e = ora.unpack(volts)
    origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, n, cfg.ksize)
    G = np.stack([ora.grid_many(e[:, 0, :, p], kern[0, :, p], origin, n) for p in range(2)], axis=1)  # [T,P,n,n]
    G64 = G.astype(np.complex64)
    buf = torch.from_numpy(np.ascontiguousarray(G64.reshape(-1))).to(DEV)
    plan.fft(buf, cfg.n_time)
    ef = plan.split_grids(buf, cfg.n_time)[0].cpu().numpy()                 # FFT pixel order
    ref = ora.efield_image(G64.astype(np.complex128))                         # centred
    got = np.fft.fftshift(ef, axes=(-2, -1))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


@pytest.mark.parametrize("n", [64, 192, 256, 384])
def test_staged_fft_full_random_grid(n):
    """moff_fft on random grids with data in every cell (rows and columns no footprint touches included)
    against the oracle's direct DFT: the staged transform covers the whole grid, not the footprint rows only."""
    cfg = _small(n, C=2, A=12, T=3, disk=0.3 * n, seed=n + 1)
    geo, kern, volts, plan = _setup(cfg)
    rng = np.random.default_rng(n)
    G = (rng.standard_normal((cfg.n_time, 2 * plan.pix_total)) +
         1j * rng.standard_normal((cfg.n_time, 2 * plan.pix_total))).astype(np.complex64)
    buf = torch.from_numpy(np.ascontiguousarray(G.reshape(-1))).to(DEV)
    plan.fft(buf, cfg.n_time)
    ef = plan.split_grids(buf, cfg.n_time)
    for c in range(cfg.n_chan):
        o = 2 * plan.pix_off[c]
        g = G[:, o:o + 2 * n * n].reshape(cfg.n_time, 2, n, n).astype(np.complex128)
        ref = ora.efield_image(g)
        got = np.fft.fftshift(ef[c].cpu().numpy(), axes=(-2, -1))
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 2e-6, (c, err)


def test_staged_fft_more_samples_than_one_grid_dimension():
    """moff_fft over 70000 samples of random 32^2 grids, more than the 65535 workgroups one launch dimension
    holds: samples on both sides of 65535 against the oracle's direct DFT."""
    n, T = 32, 70000
    cfg = _small(n, C=1, A=8, T=4, disk=0.4 * n, seed=77)
    geo, kern, volts, plan = _setup(cfg)
    gen = torch.Generator(device=DEV).manual_seed(77)
    buf = torch.randn(T * 2 * plan.pix_total, dtype=torch.complex64, device=DEV, generator=gen)
    keep = [0, 1, 65534, 65535, 65536, T - 1]
    src = buf.view(T, -1)[keep].cpu().numpy()
    plan.fft(buf, T)
    got = buf.view(T, -1)[keep].cpu().numpy()
    for k, t in enumerate(keep):
        ref = ora.efield_image(src[k].reshape(2, n, n).astype(np.complex128))
        out = np.fft.fftshift(got[k].reshape(2, n, n), axes=(-2, -1))
        err = np.abs(out - ref).max() / np.abs(ref).max()
        assert err < 2e-6, (t, err)


def test_staged_accumulate_and_readout():
    n = 64
    cfg = _small(n, C=2, A=20, T=6)
    geo, kern, volts, plan = _setup(cfg)
    rng = np.random.default_rng(1)
    ef = (rng.standard_normal((cfg.n_time, 2 * plan.pix_total)) +
          1j * rng.standard_normal((cfg.n_time, 2 * plan.pix_total))).astype(np.complex64)
    acc = plan.new_accumulator()
    plan.accumulate(torch.from_numpy(ef.reshape(-1)).to(DEV), cfg.n_time, acc)
    imgs = [im.cpu().numpy() for im in plan.read_image(acc, n_samples=cfg.n_time, normalize=True)]
    e128 = ef.astype(np.complex128)
    for c in range(cfg.n_chan):
        o = 2 * plan.pix_off[c]
        ex = np.fft.fftshift(e128[:, o:o + n * n].reshape(-1, n, n), axes=(-2, -1))
        ey = np.fft.fftshift(e128[:, o + n * n:o + 2 * n * n].reshape(-1, n, n), axes=(-2, -1))
        ref = np.stack([p.sum(0) for p in ora.pol_products(ex, ey)]) / cfg.n_time
        assert np.all(ora.relative_errors(imgs[c].astype(np.complex128), ref) < TOL)


def test_staged_chain_matches_fused():
    cfg = _small(128, C=2, A=60, T=7)
    geo, kern, volts, plan = _setup(cfg)
    v = torch.from_numpy(volts).to(DEV)
    g = plan.grid(v)
    plan.fft(g, cfg.n_time)
    acc_s = plan.new_accumulator()
    plan.accumulate(g, cfg.n_time, acc_s)
    acc_f = plan.new_accumulator()
    plan.correlate(v, acc_f)
    a, b = acc_s.cpu().numpy(), acc_f.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


# ---------------------------------------------------------------------------------------------------------
# fused path against the whole oracle
# ---------------------------------------------------------------------------------------------------------
def test_tiny_workload_full():
    """64 antennas, 1 channel, 1 pol, complex64 voltages, 64^2 grid, 256 samples: every pixel."""
    cfg = configs.TINY
    geo, kern, volts, plan = _setup(cfg)
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label="tiny")


@pytest.mark.parametrize("n,P,K,A,C,T,int8", [
    (32, 2, 4, 12, 2, 5, True), (64, 1, 4, 50, 2, 11, True), (96, 2, 4, 30, 1, 3, True),
    (128, 2, 6, 70, 3, 19, True), (160, 2, 4, 33, 1, 4, True), (192, 1, 8, 41, 1, 5, False),
    (256, 2, 4, 90, 2, 6, True), (320, 2, 2, 25, 1, 3, True), (384, 2, 6, 44, 1, 3, True),
    (512, 2, 4, 31, 1, 2, True),
])
def test_fused_every_size(n, P, K, A, C, T, int8):
    cfg = _small(n, P=P, A=A, C=C, T=T, K=K, int8=int8, seed=n)
    geo, kern, volts, plan = _setup(cfg)
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"n={n}")


# ---------------------------------------------------------------------------------------------------------
# gridding + row transform as one split-FP16 matrix-core GEMM over time samples (MOFF_FFT_GEMM_FP16)
# ---------------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,P,K,A,C,T,acc", [
    (32, 2, 4, 12, 2, 5, api.ACC_FP32), (64, 1, 4, 50, 2, 11, api.ACC_FP32), (96, 2, 2, 30, 1, 3, api.ACC_FP64_COMP),
    (128, 2, 6, 70, 3, 19, api.ACC_FP32), (160, 2, 4, 33, 1, 4, api.ACC_FP32), (192, 1, 8, 41, 1, 5, api.ACC_FP32),
    (256, 2, 4, 90, 2, 40, api.ACC_FP32), (256, 2, 4, 300, 2, 33, api.ACC_FP64_COMP), (320, 2, 2, 25, 1, 3, api.ACC_FP32),
    (384, 2, 6, 44, 1, 3, api.ACC_FP32), (512, 2, 4, 31, 1, 2, api.ACC_FP32),
])
def test_gemm_row_pass_every_size(n, P, K, A, C, T, acc):
    """The matrix-core row pass (gridding + row DFT as a split-FP16 GEMM) against the oracle, every pixel.  The
    300-antenna 256^2 case puts 60-odd antennas on the middle rows (several K chunks) and 33 samples span three
    16-sample tiles, the last one ragged."""
    cfg = _small(n, P=P, A=A, C=C, T=T, K=K, seed=n + 2000 + A)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, acc_mode=acc, fft_mode=api.FFT_GEMM_FP16).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"gemm row pass n={n} P={P} K={K}", report=True)


def test_gemm_row_pass_default_shape_phases_edges():
    """The matrix-core row pass at the default launch shape with ragged time and channel blocks (300 samples, 33
    channels), with phase-centre phases folded into its kernels, and with footprints on the grid edges."""
    cfg = _small(64, A=30, C=33, T=300, seed=41)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=api.FFT_GEMM_FP16).bind(DEV)
    assert plan.launch_shape() == (256, 32, 32)
    ph = _phases(cfg, 4)
    plan.set_kernels(torch.from_numpy(kern).to(DEV), phase=torch.from_numpy(ph).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    sel = [0, cfg.n_chan - 1]
    ref = ora.image(ora.apply_phases(volts, ph)[:, sel], kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel],
                    cfg.cell_lambda)
    _check_images([imgs[c] for c in sel], ref, label="gemm default shape, phased")
    cfg, geo, kern, volts = _edge_setup(256, 4, T=40, seed=5)
    plan = api.plan_for(cfg, geo, fft_mode=api.FFT_GEMM_FP16).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    _check_images(imgs, ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda),
                  label="gemm edges", report=True)


def test_gemm_row_pass_batched_sizes_and_graph():
    """Per-channel grid sizes 128^2-384^2 with 6x6 kernels (the batched workload's shape, 48 antennas), eager and
    graph-replayed (bit-identical)."""
    cfg = configs.scaled(configs.BATCHED, n_ant=48, n_chan=6, n_time=21)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=api.FFT_GEMM_FP16).bind(DEV)
    assert len(set(plan.grid_n)) >= 4, plan.grid_n
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, acc = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label="gemm per-channel sizes", report=True)
    v = torch.from_numpy(volts).to(DEV)
    g = plan.new_accumulator()
    for _ in range(2):
        g.zero_()
        plan.correlate_graph(v, g)
        torch.cuda.synchronize()
        assert torch.equal(g, acc)


def test_ragged_time_blocks_and_fp64_accumulator():
    cfg = _small(64, C=3, A=45, T=37)
    for mode in (api.ACC_FP32, api.ACC_FP64_COMP):
        geo, kern, volts, plan = _setup(cfg, acc_mode=mode, time_block=8)
        imgs, _ = _run_fused(plan, volts)
        ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
        _check_images(imgs, ref, label=f"acc mode {mode}")


def test_default_shape_ragged_blocks():
    """The library's default launch shape (256-sample x 32-channel blocks, 32-sample row groups) with a ragged
    last time block (300 = 256 + 44 samples; its last row group holds 12) and a ragged last channel block
    (35 = 32 + 3 channels): every pixel of every channel against the oracle."""
    cfg = _small(64, C=35, A=30, T=300, seed=11)
    geo, kern, volts, plan = _setup(cfg)
    assert plan.launch_shape() == (256, 32, 32)
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label="default shape, ragged blocks")


def test_plain_workload_channels():
    """The plain workload (256 antennas, 32 channels, 128^2, dual pol): all channels through the fused path,
    lowest and highest channel checked pixel by pixel over the first 512 samples."""
    cfg = configs.PLAIN
    geo, kern, volts, plan = _setup(cfg, n_time=512)
    imgs, _ = _run_fused(plan, volts)
    sel = [0, cfg.n_chan - 1]
    ref = ora.image(volts[:, sel], kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel], cfg.cell_lambda)
    _check_images([imgs[c] for c in sel], ref, label="plain")


# ---------------------------------------------------------------------------------------------------------
# degenerate cases and properties
# ---------------------------------------------------------------------------------------------------------
def test_zero_samples_leave_accumulator_untouched():
    cfg = _small(64, C=1, A=10, T=3)
    geo, kern, volts, plan = _setup(cfg)
    acc = plan.new_accumulator().fill_(3.5)
    plan.correlate(torch.from_numpy(volts).to(DEV), acc, n_t=0)
    torch.cuda.synchronize()
    assert torch.all(acc == 3.5)


def test_single_antenna_and_stacked_antennas():
    n = 64
    for xy in (np.array([[2.3, -4.1]]), np.tile(np.array([[1.2, 0.7]]), (9, 1))):
        geo = synth.Geometry(xy, np.array([configs.C_LIGHT]), np.array([n], dtype=np.int32), 1.0, 8)
        cfg = configs.scaled(configs.PLAIN, n_ant=xy.shape[0], n_chan=1, ksize=8, grid_n=n, n_time=5)
        rng = np.random.default_rng(2)
        kern = (rng.standard_normal((1, xy.shape[0], 2, 8, 8)) + 1j * rng.standard_normal((1, xy.shape[0], 2, 8, 8)))
        kern = kern.astype(np.complex64)
        volts = rng.integers(-127, 128, size=(5, 1, xy.shape[0], 2, 2)).astype(np.int8)
        plan = api.plan_for(cfg, geo).bind(DEV)
        plan.set_kernels(torch.from_numpy(kern).to(DEV))
        imgs, _ = _run_fused(plan, volts)
        ref = ora.image(volts, kern, xy, geo.freqs_hz, geo.grid_n, 1.0)
        _check_images(imgs, ref, label=f"{xy.shape[0]} antennas")


@pytest.mark.parametrize("n,K,fft", [(256, 4, api.FFT_FP32), (512, 4, api.FFT_FP32), (512, 8, api.FFT_FP32),
                                     (512, 4, api.FFT_GEMM_FP16)])
def test_maximum_antenna_count(n, K, fft):
    """65534 antennas (the largest count a plan takes: tap metadata and row lists hold 16-bit antenna fields) in a
    disk of 0.6 n cells: thousands of antennas per row band, tens of taps on each cell, band voltage tables of
    several thousand records and (matrix-core form) about 70 K chunks per row."""
    cfg = configs.scaled(configs.PLAIN, index=900 + n + K, n_ant=65534, n_pol=2, n_chan=1, n_time=3, ksize=K,
                         grid_n=n, disk_lambda=0.6 * n, int8=True)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=fft).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"65534 antennas n={n} K={K} fft={fft}", report=True)


def test_deterministic_and_split_integration():
    """Same input twice -> bit-identical accumulators; an integration split at a time-block boundary equals
    the unsplit one bit for bit (accumulation is linear in time: checkpoint and resume)."""
    cfg = _small(128, C=2, A=64, T=32)
    geo, kern, volts, plan = _setup(cfg, time_block=8)
    v = torch.from_numpy(volts).to(DEV)
    a1, a2, a3 = plan.new_accumulator(), plan.new_accumulator(), plan.new_accumulator()
    plan.correlate(v, a1)
    plan.correlate(v, a2)
    plan.correlate(v[:16].contiguous(), a3)
    plan.correlate(v[16:].contiguous(), a3)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)
    assert torch.equal(a1, a3)


def _edge_setup(n, K, T, A_inner=24, seed=0):
    """One channel at f = c (one metre = one wavelength, cell 1): eight antennas whose footprints touch grid
    rows and columns 0 and n - 1 (the four corners and the four edge midpoints), plus random interior antennas;
    random complex kernels and random int8 voltages."""
    rng = np.random.default_rng(seed)
    lo, hi, mid = K // 2 - 1 + 0.3, n - 1 - K // 2 + 0.6, n / 2 + 0.45    # floor(X) = K/2 - 1, n - 1 - K/2
    edge = [(x, y) for x in (lo, mid, hi) for y in (lo, mid, hi) if (x, y) != (mid, mid)]
    inner = rng.uniform(K + 2, n - K - 2, size=(A_inner, 2))
    XY = np.concatenate([np.array(edge), inner])
    xy = XY - n / 2                                                        # metres east, north
    geo = synth.Geometry(xy, np.array([configs.C_LIGHT]), np.array([n], dtype=np.int32), 1.0, K)
    origin = ora.footprint_origin(xy, configs.C_LIGHT, 1.0, n, K)
    assert origin[:, 0].min() == 0 and origin[:, 1].min() == 0
    assert origin[:, 0].max() + K == n and origin[:, 1].max() + K == n
    A = xy.shape[0]
    kern = (rng.standard_normal((1, A, 2, K, K)) + 1j * rng.standard_normal((1, A, 2, K, K))).astype(np.complex64)
    volts = rng.integers(-127, 128, size=(T, 1, A, 2, 2)).astype(np.int8)
    cfg = configs.scaled(configs.PLAIN, n_ant=A, n_chan=1, ksize=K, grid_n=n, n_time=T)
    return cfg, geo, kern, volts


@pytest.mark.parametrize("n,K,fft", [(256, 4, api.FFT_FP32), (384, 6, api.FFT_FP32), (256, 4, api.FFT_SPLIT_FP16),
                                     (256, 4, api.FFT_SPLIT_BF16)])
def test_footprints_on_grid_edges(n, K, fft):
    """Footprints on grid rows and columns 0 and n - 1: the first and last bands, the row-range masks of the
    column pass and the grid borders of the scatter; 40 samples (a row group of 32 and a ragged one)."""
    cfg, geo, kern, volts = _edge_setup(n, K, T=40, seed=n + fft)
    plan = api.plan_for(cfg, geo, fft_mode=fft).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"edges n={n} fft={fft}", report=True)
    if fft == api.FFT_FP32:
        g = plan.grid(torch.from_numpy(volts).to(DEV))
        grids = plan.split_grids(g, cfg.n_time)[0].cpu().numpy()
        origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[0], 1.0, n, K)
        e = ora.unpack(volts)
        for p in range(2):
            r = ora.grid_many(e[:, 0, :, p], kern[0, :, p], origin, n)
            assert np.abs(grids[:, p] - r).max() <= 1e-6 * np.abs(r).max(), p
            assert np.abs(r[:, 0, :]).max() > 0 and np.abs(r[:, n - 1, :]).max() > 0
            assert np.abs(r[:, :, 0]).max() > 0 and np.abs(r[:, :, n - 1]).max() > 0


def test_hermitian_products_and_positivity():
    cfg = _small(64, C=1, A=30, T=8)
    geo, kern, volts, plan = _setup(cfg)
    imgs, _ = _run_fused(plan, volts)
    im = imgs[0]
    assert np.array_equal(im[3], np.conj(im[2]))
    assert im[0].real.min() >= 0 and im[1].real.min() >= 0
    assert np.all(np.abs(im[2]) ** 2 <= im[0].real * im[1].real * (1 + 1e-4) + 1e-3)


# ---------------------------------------------------------------------------------------------------------
# batching: per-channel grid sizes, graph replay, launch shapes, autotuner
# ---------------------------------------------------------------------------------------------------------
def test_per_channel_grid_sizes_against_oracle():
    """Channels spanning 50-200 MHz get grids from 128^2 to 384^2 (6x6 kernels), all in one correlate call."""
    cfg = configs.scaled(configs.BATCHED, n_ant=48, n_chan=6, n_time=5)
    geo, kern, volts, plan = _setup(cfg)
    assert len(set(plan.grid_n)) >= 4, plan.grid_n
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label="per-channel sizes")


@pytest.mark.parametrize("fft", [api.FFT_FP32, api.FFT_GEMM_FP16])
def test_interleaved_grid_sizes_fused_and_staged(fft):
    """Grid sizes chosen per channel and interleaved (96, 256, 96, 192, 192, 128, 256): seven channels make six
    launch blocks of consecutive equal sizes.  The fused path against the oracle pixel by pixel, and the staged
    chain (grid, 2-D FFT, accumulate) against the fused accumulator."""
    cfg = _small(96, C=7, A=36, T=11, disk=50.0, seed=23)
    geo, kern, volts = synth.workload(cfg)
    sizes = np.array([96, 256, 96, 192, 192, 128, 256], dtype=np.int32)
    geo = synth.Geometry(geo.ant_xy_m, geo.freqs_hz, sizes, geo.cell_lambda, geo.ksize)
    plan = api.plan_for(cfg, geo, fft_mode=fft).bind(DEV)
    assert list(plan.grid_n) == sizes.tolist()
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, acc_f = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"interleaved sizes fft={fft}")
    if fft == api.FFT_FP32:
        v = torch.from_numpy(volts).to(DEV)
        g = plan.grid(v)
        plan.fft(g, cfg.n_time)
        acc_s = plan.new_accumulator()
        plan.accumulate(g, cfg.n_time, acc_s)
        a, b = acc_s.cpu().numpy(), acc_f.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


def test_graph_replay_shapes_and_autotune():
    cfg = _small(128, C=5, A=64, T=40)
    geo, kern, volts, plan = _setup(cfg)
    big = max(plan.workspace_bytes_for(tb, cpb) for tb in (8, 16, 32, 64) for cpb in (4, 8, 16, 32, 64, 128))
    plan.bind(DEV, workspace_bytes=big)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    v = torch.from_numpy(volts).to(DEV)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    a_ref = plan.new_accumulator()
    plan.correlate(v, a_ref)
    a_g = plan.new_accumulator()
    for _ in range(3):                       # capture once, replay; eager work in between
        a_g.zero_()
        plan.correlate_graph(v, a_g)
        torch.cuda.synchronize()
        assert torch.equal(a_g, a_ref)
    plan.set_launch_shape(8, 2, 2)
    assert plan.launch_shape() == (8, 2, 2)
    a2 = plan.new_accumulator()
    plan.correlate(v, a2)
    _check_images([im.cpu().numpy().astype(np.complex128) for im in plan.read_image(a2)], ref, label="shape")
    best = plan.autotune(v, plan.new_accumulator(), n_t=16)
    assert best["ms"] > 0 and plan.launch_shape() == (best["time_block"], best["chans_per_block"],
                                                      best["time_group"])
    a3 = plan.new_accumulator()
    plan.correlate(v, a3)
    _check_images([im.cpu().numpy().astype(np.complex128) for im in plan.read_image(a3)], ref, label="tuned")


def test_autotune_cache(tmp_path):
    """The persisted autotuner cache: the first call tunes and appends its shape under the plan's key; a second
    plan with the same signature applies it without timing; a plan with another signature (a different transform)
    tunes again and adds its own line; results stay correct under the cached shape."""
    cfg = _small(128, C=5, A=64, T=40)
    geo, kern, volts = synth.workload(cfg)
    v = torch.from_numpy(volts).to(DEV)
    cache = str(tmp_path / "tune.txt")
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)

    def bound(**kw):
        plan = api.plan_for(cfg, geo, **kw)
        big = max(plan.workspace_bytes_for(tb, cpb) for tb in (8, 16, 32, 64) for cpb in (4, 8, 16, 32, 64, 128))
        plan.bind(DEV, workspace_bytes=big)
        plan.set_kernels(torch.from_numpy(kern).to(DEV))
        return plan

    p1 = bound()
    first = p1.autotune(v, p1.new_accumulator(), n_t=16, cache=cache)
    assert not first["cached"] and first["ms"] > 0
    lines = open(cache).read().splitlines()
    assert lines == [f"{p1.autotune_key}\t{first['time_block']} {first['chans_per_block']} {first['time_group']} "
                     f"{first['ms']:g}"] or (len(lines) == 1 and lines[0].startswith(p1.autotune_key + "\t"))
    p2 = bound()
    assert p2.autotune_key == p1.autotune_key
    second = p2.autotune(v, p2.new_accumulator(), n_t=16, cache=cache)
    assert second["cached"]
    assert p2.launch_shape() == (first["time_block"], first["chans_per_block"], first["time_group"])
    acc = p2.new_accumulator()
    p2.correlate(v, acc)
    _check_images([im.cpu().numpy().astype(np.complex128) for im in p2.read_image(acc)], ref, label="cached shape")
    p3 = bound(fft_mode=api.FFT_GEMM_FP16)
    third = p3.autotune(v, p3.new_accumulator(), n_t=16, cache=cache)
    assert not third["cached"] and len(open(cache).read().splitlines()) == 2
    # a malformed line and a shape that does not fit the bound workspace are not applied: the plan tunes again,
    # keeps a shape that fits, and appends it (the last line for a key wins)
    p4 = bound()
    with open(cache, "a") as fh:
        fh.write(f"{p4.autotune_key}\tnot numbers\n")
        fh.write(f"{p4.autotune_key}\t4096 4096 64 0.1\n")
    fourth = p4.autotune(v, p4.new_accumulator(), n_t=16, cache=cache)
    assert not fourth["cached"]
    assert p4.launch_shape() == (fourth["time_block"], fourth["chans_per_block"], fourth["time_group"])
    assert open(cache).read().splitlines()[-1].startswith(p4.autotune_key + "\t")
    p5 = bound()
    fifth = p5.autotune(v, p5.new_accumulator(), n_t=16, cache=cache)
    assert fifth["cached"] and p5.launch_shape() == p4.launch_shape()



# ---------------------------------------------------------------------------------------------------------
# precision form: both FFT stages on the matrix cores with split FP16 / BF16 products
# ---------------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [api.FFT_FP32, api.FFT_SPLIT_FP16, api.FFT_SPLIT_BF16])
@pytest.mark.parametrize("acc_mode", [api.ACC_FP32, api.ACC_FP64_COMP])
def test_split_precision_transform(mode, acc_mode):
    """The split FP16 / BF16 matrix-core transform against the oracle, beside the FP32 transform on the same
    inputs; prints the per-image errors (XX, YY, XY, YX of each channel)."""
    cfg = _small(256, C=2, A=90, T=6, seed=7)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=mode, acc_mode=acc_mode).bind(DEV)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    worst = _check_images(imgs, ref, label=f"fft mode {mode} acc {acc_mode}", report=True)
    print(f"fft mode {mode} acc {acc_mode}: worst per-image error {worst:.2e}")


@pytest.mark.parametrize("mode", [api.FFT_SPLIT_FP16, api.FFT_SPLIT_BF16])
def test_split_precision_default_shape_ragged(mode):
    """The matrix-core forms at the default launch shape with a ragged last time block (260 = 256 + 4 samples)
    and a ragged last channel block (33 = 32 + 1 channels); the first channel and the one in the ragged block
    against the oracle, every pixel."""
    cfg = _small(256, C=33, A=40, T=260, seed=13)
    geo, kern, volts = synth.workload(cfg)
    plan = api.plan_for(cfg, geo, fft_mode=mode).bind(DEV)
    assert plan.launch_shape() == (256, 32, 32)
    plan.set_kernels(torch.from_numpy(kern).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    sel = [0, cfg.n_chan - 1]
    ref = ora.image(volts[:, sel], kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel], cfg.cell_lambda)
    _check_images([imgs[c] for c in sel], ref, label=f"split mode {mode}, ragged blocks", report=True)


# ---------------------------------------------------------------------------------------------------------
# the headline workload at full size, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------------------------------------
def test_headline_full_size_sampled_pixels():
    """2048 antennas, 128 channels, 256^2, all 16384 samples (device-drawn int8 voltages), default launch shape,
    graph replay.  Sampled pixels of the lowest and highest channel against the oracle evaluated pixel by
    pixel over the whole integration.  Scale per product: the largest |oracle| over the sampled pixels, which
    include the centre pixel (the autocorrelation peak)."""
    cfg = configs.HEADLINE
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    sk = synth.sky(cfg)
    kern = synth.kernels(geo, g, cfg.n_pol)
    dev = torch.device(DEV)
    volts = synth.DeviceVoltages(cfg, geo, g, sk, dev, chunk=64).all(cfg.n_time)
    plan = api.plan_for(cfg, geo).bind(dev)
    plan.set_kernels(torch.from_numpy(kern).to(dev))
    acc = plan.new_accumulator()
    plan.correlate_graph(volts, acc)
    imgs = plan.read_image(acc)
    n = cfg.grid_n
    pix = np.array([[n // 2, n // 2], [n // 2 + 1, n // 2], [3, 250], [200, 17], [128, 77], [255, 0]])
    for c in (0, cfg.n_chan - 1):
        got = imgs[c].cpu().numpy()[:, pix[:, 0], pix[:, 1]].astype(np.complex128)
        v = volts[:, c:c + 1].cpu().numpy()
        ref = ora.image_pixels(v, kern[c], geo.ant_xy_m, geo.freqs_hz[c], n, cfg.cell_lambda, pix, t_batch=512)
        sxx, syy = np.abs(ref[0]).max(), np.abs(ref[1]).max()
        scale = np.array([sxx, syy, np.sqrt(sxx * syy), np.sqrt(sxx * syy)])[:, None]
        err = (np.abs(got - ref) / scale).max(axis=1)
        assert np.all(err <= TOL), (c, err)


# ---------------------------------------------------------------------------------------------------------
# phase-centre tracking and full-polarisation (Jones) kernels
# ---------------------------------------------------------------------------------------------------------
def _phases(cfg, seed):
    rng = np.random.default_rng(seed)
    return np.exp(2j * np.pi * rng.random((cfg.n_chan, cfg.n_ant, cfg.n_pol))).astype(np.complex64)


def test_phase_tracking_per_time_block():
    """Each antenna's voltage times a phase before gridding, the phases changing between two blocks of samples;
    then back to no phase.  Against the oracle on the phased voltages."""
    cfg = _small(128, C=2, A=48, T=14, seed=7)
    geo, kern, volts, plan = _setup(cfg)
    ph1, ph2 = _phases(cfg, 1), _phases(cfg, 2)
    kd = torch.from_numpy(np.ascontiguousarray(kern)).to(DEV)
    v = torch.from_numpy(volts).to(DEV)
    acc = plan.new_accumulator()
    plan.set_kernels(kd, phase=torch.from_numpy(ph1).to(DEV))
    plan.correlate(v[:6].contiguous(), acc)
    plan.set_kernels(kd, phase=torch.from_numpy(ph2).to(DEV))
    plan.correlate(v[6:].contiguous(), acc)
    imgs = [im.cpu().numpy().astype(np.complex128) for im in plan.read_image(acc)]
    args = (kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    r1 = ora.image(ora.apply_phases(volts[:6], ph1), *args)
    r2 = ora.image(ora.apply_phases(volts[6:], ph2), *args)
    _check_images(imgs, [a + b for a, b in zip(r1, r2)], label="phased")
    plan.set_kernels(kd)
    imgs, _ = _run_fused(plan, volts)
    _check_images(imgs, ora.image(volts, *args), label="unphased again")


def _jones_kernels(kern, seed, leak=0.3):
    """Diagonal kernels [C, A, 2, K, K] plus random off-diagonal leakage -> [C, A, 2, 2, K, K]."""
    rng = np.random.default_rng(seed)
    C, A, P, K, _ = kern.shape
    J = np.zeros((C, A, 2, 2, K, K), dtype=np.complex64)
    for p in range(2):
        J[:, :, p, p] = kern[:, :, p]
        q = 1 - p
        J[:, :, p, q] = leak * (rng.standard_normal((C, A, K, K)) + 1j * rng.standard_normal((C, A, K, K)))
    return J


@pytest.mark.parametrize("n,K,A,C,T,tb", [(64, 4, 40, 2, 9, 0), (128, 6, 61, 2, 13, 4), (256, 4, 75, 1, 5, 0),
                                          (64, 4, 30, 33, 300, 0)])
def test_jones_kernels_fused(n, K, A, C, T, tb):
    """tb = 0: the library's default launch shape; the last case ends in ragged time and channel blocks."""
    cfg = _small(n, A=A, C=C, T=T, K=K, seed=20 + n)
    geo, kern, volts = synth.workload(cfg)
    J = _jones_kernels(kern, seed=n)
    plan = api.plan_for(cfg, geo, kernel_mode=api.KERNEL_JONES, time_block=tb).bind(DEV)
    plan.set_kernels(torch.from_numpy(J).to(DEV))
    imgs, _ = _run_fused(plan, volts)
    ref = ora.image_jones(volts, J, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)
    _check_images(imgs, ref, label=f"jones n={n}")


def test_jones_staged_grid_and_phase():
    """Staged gridding with Jones kernels (both pols into each grid), with phases folded in."""
    cfg = _small(64, A=33, C=2, T=4, seed=31)
    geo, kern, volts = synth.workload(cfg)
    J = _jones_kernels(kern, seed=5)
    ph = _phases(cfg, 9)
    plan = api.plan_for(cfg, geo, kernel_mode=api.KERNEL_JONES).bind(DEV)
    plan.set_kernels(torch.from_numpy(J).to(DEV), phase=torch.from_numpy(ph).to(DEV))
    g = plan.grid(torch.from_numpy(volts).to(DEV))
    grids = [x.cpu().numpy() for x in plan.split_grids(g, cfg.n_time)]
    e = ora.apply_phases(volts, ph)
    n = cfg.grid_n
    for c in range(cfg.n_chan):
        origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[c], cfg.cell_lambda, n, cfg.ksize)
        for p in range(2):
            ref = sum(ora.grid_many(e[:, c, :, q], J[c, :, p, q], origin, n) for q in range(2))
            err = np.abs(grids[c][:, p] - ref).max() / np.abs(ref).max()
            assert err < 1e-6, (c, p, err)


def test_batched_workload_every_grid_size():
    """The batching workload at full size (4096 antennas, 256 channels over 50-200 MHz, per-channel grids,
    6x6 kernels) for 256 device-drawn samples through one graph-replayed correlate; the first channel of every
    distinct grid size (128^2 .. 384^2) and the highest channel checked pixel by pixel against the oracle."""
    cfg = configs.scaled(configs.BATCHED, n_time=256)
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    sk = synth.sky(cfg)
    kern = synth.kernels(geo, g, cfg.n_pol)
    dev = torch.device(DEV)
    volts = synth.DeviceVoltages(cfg, geo, g, sk, dev, chunk=64).all(cfg.n_time)
    plan = api.plan_for(cfg, geo).bind(dev)
    plan.set_kernels(torch.from_numpy(kern).to(dev))
    acc = plan.new_accumulator()
    plan.correlate_graph(volts, acc)
    imgs = plan.read_image(acc)
    sizes = plan.grid_n
    sel = sorted({sizes.index(n) for n in set(sizes)} | {cfg.n_chan - 1})
    assert len(set(sizes)) == 6, sorted(set(sizes))
    print(f"batched: channels {sel}, grids {[sizes[c] for c in sel]}", flush=True)
    v = volts[:, sel].cpu().numpy()
    ref = ora.image(v, kern[sel], geo.ant_xy_m, geo.freqs_hz[sel], geo.grid_n[sel], cfg.cell_lambda)
    _check_images([imgs[c].cpu().numpy().astype(np.complex128) for c in sel], ref, label="batched")


def test_overlapped_and_serial_two_pass_agree():
    """The overlapped two-pass form (row pass of the next block on an internal stream, two exchange buffers)
    gives the same accumulator as the serial one, bit for bit, eager and graph-replayed."""
    import os
    cfg = _small(128, C=5, A=50, T=37, seed=9)
    geo, kern, volts = synth.workload(cfg)
    accs = []
    for ov in ("1", "0"):
        old = os.environ.get("MOFF_OVERLAP")
        os.environ["MOFF_OVERLAP"] = ov
        try:
            plan = api.plan_for(cfg, geo, time_block=8, chans_per_block=2).bind(DEV)
        finally:
            if old is None:
                del os.environ["MOFF_OVERLAP"]
            else:
                os.environ["MOFF_OVERLAP"] = old
        plan.set_kernels(torch.from_numpy(np.ascontiguousarray(kern)).to(DEV))
        v = torch.from_numpy(volts).to(DEV)
        a = plan.new_accumulator()
        plan.correlate(v, a)
        g = plan.new_accumulator()
        for _ in range(3):                       # replays on a cleared accumulator, each checked
            g.zero_()
            plan.correlate_graph(v, g)
            torch.cuda.synchronize()
            assert torch.equal(g, a), ov
        accs.append(a)
    assert torch.equal(accs[0], accs[1])
