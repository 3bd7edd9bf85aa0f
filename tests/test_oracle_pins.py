"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics (CPU only).

Each test would fail for a plausible mistake in the oracle: a dropped autocorrelation or a wrong conjugation
(FX identity), a wrong DFT sign or pixel axis (lone point source, numpy ifft2 reduction), a wrong
normalisation (Parseval), a mirrored image or swapped products (invariants).
"""
import math

import numpy as np
import pytest

from oracle import moff_oracle as ora
from paper_0812_3669_amd import configs, synth
from tests.fx_pin import direct_imaging, fx_image, fx_image_jones

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _origin(ant_xy, f, cell, n, K):
    # independent recompute of the footprint convention: cells floor(X)-K/2+1 .. floor(X)+K/2
    X = ant_xy[:, 0] * f / configs.C_LIGHT / cell + n / 2
    Y = ant_xy[:, 1] * f / configs.C_LIGHT / cell + n / 2
    return np.stack([np.floor(Y).astype(int) - K // 2 + 1, np.floor(X).astype(int) - K // 2 + 1], axis=1)


def _small(P, A=24, n=32, T=8, K=4, seed=7, disk=14.0):
    cfg = configs.scaled(configs.TINY, index=50 + seed, n_ant=A, n_pol=P, grid_n=n, n_time=T, ksize=K,
                         disk_lambda=disk, int8=(P == 2))
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    sk = synth.sky(cfg)
    kern = synth.kernels(geo, g, P)
    volts = synth.voltages_host(cfg, geo, g, sk)
    return cfg, geo, kern, volts


def _peak_err(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# ---------------------------------------------------------------------------------------------------------
# 1. FX brute force (Eqs. visDef, Bdef, m1-m6): MOFF image == software-holography image of all visibilities
# ---------------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("P", [1, 2])
def test_fx_identity(P):
    cfg, geo, kern, volts = _small(P)
    img = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    e = ora.unpack(volts)[:, 0]                                                # [T, A, P]
    origin = _origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, cfg.grid_n, cfg.ksize)
    fx = fx_image(e, kern[0], origin, cfg.grid_n)
    for k in range(img.shape[0]):
        assert _peak_err(img[k], fx[k]) < 1e-12, k


def test_fx_identity_k6_odd_sizes():
    cfg, geo, kern, volts = _small(2, A=13, n=40, T=5, K=6, seed=3, disk=20.0)
    img = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    origin = _origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, cfg.grid_n, cfg.ksize)
    fx = fx_image(ora.unpack(volts)[:, 0], kern[0], origin, cfg.grid_n)
    for k in range(4):
        assert _peak_err(img[k], fx[k]) < 1e-12


def test_fx_identity_catches_dropped_autocorrelations():
    """A plausible oracle mistake (only cross pairs) is far outside the FX pin's tolerance."""
    cfg, geo, kern, volts = _small(1)
    img = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    e = ora.unpack(volts)[:, 0]
    origin = _origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, cfg.grid_n, cfg.ksize)
    auto_only = np.zeros_like(e)
    auto_only[:, 0] = e[:, 0]
    # the single-antenna image is the autocorrelation term of antenna 0; removing it changes the image
    fx_auto = fx_image(auto_only, kern[0], origin, cfg.grid_n)
    assert np.abs(fx_auto).max() / np.abs(img).max() > 1e-3


# ---------------------------------------------------------------------------------------------------------
# 2. Parseval: the DFT normalisation (sum over pixels = n^2 * grid energy)
# ---------------------------------------------------------------------------------------------------------
def test_parseval():
    cfg, geo, kern, volts = _small(2, T=6)
    n, K = cfg.grid_n, cfg.ksize
    img = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, n, K)
    e = ora.unpack(volts)[:, 0]
    G = [ora.grid_many(e[:, :, p], kern[0, :, p], origin, n) for p in range(2)]
    assert abs(img[0].sum() - n * n * np.sum(np.abs(G[0]) ** 2)) / abs(img[0].sum()) < 1e-12
    assert abs(img[1].sum() - n * n * np.sum(np.abs(G[1]) ** 2)) / abs(img[1].sum()) < 1e-12
    cross = n * n * np.sum(G[0] * np.conj(G[1]))
    assert abs(img[2].sum() - cross) / abs(img[0].sum()) < 1e-12


def test_grid_many_matches_scatter():
    cfg, geo, kern, volts = _small(2, T=3)
    origin = ora.footprint_origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, cfg.grid_n, cfg.ksize)
    e = ora.unpack(volts)[:, 0]
    Gm = ora.grid_many(e[:, :, 1], kern[0, :, 1], origin, cfg.grid_n)
    for t in range(3):
        Gs = ora.grid(e[t, :, 1], kern[0, :, 1], origin, cfg.grid_n)
        assert np.abs(Gm[t] - Gs).max() < 1e-12 * np.abs(Gs).max()


# ---------------------------------------------------------------------------------------------------------
# 3. Lone point source: sign of the imaging transform, kernel conjugation and pixel axes
# ---------------------------------------------------------------------------------------------------------
def _lone_source_delta(n=32, A=10, T=4, dq=(-3, 5), seed=1):
    """Delta kernels (one unit tap at (K/2-1, K/2-1)), antennas on integer cells, unit gains, no noise."""
    rng = np.random.default_rng(seed)
    K, cell, f = 4, 1.0, configs.C_LIGHT      # f = c -> one metre is one wavelength
    cells = rng.choice(np.arange(8, n - 8), size=(A, 2))
    ant_xy = np.stack([cells[:, 1] - n / 2, cells[:, 0] - n / 2], axis=1).astype(np.float64)  # x=east, y=north
    qs, ps = n // 2 + dq[0], n // 2 + dq[1]
    l_s, m_s = (ps - n / 2) / (n * cell), (qs - n / 2) / (n * cell)
    s = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    e = s[:, None] * np.exp(-2j * np.pi * (ant_xy[:, 0] * l_s + ant_xy[:, 1] * m_s))[None, :]
    kern = np.zeros((1, A, 1, K, K), dtype=np.complex64)
    kern[0, :, 0, K // 2 - 1, K // 2 - 1] = 1.0
    volts = e[:, None, :, None].astype(np.complex128)
    return volts, kern, ant_xy, f, n, cells, s, (qs, ps)


def test_point_source_closed_form():
    volts, kern, ant_xy, f, n, cells, s, (qs, ps) = _lone_source_delta()
    img = ora.image(volts, kern, ant_xy, [f], [n], 1.0)[0][0].real
    A = cells.shape[0]
    pw = np.sum(np.abs(s) ** 2)
    assert np.unravel_index(np.argmax(img), img.shape) == (qs, ps)
    assert abs(img[qs, ps] - A * A * pw) < 1e-9 * A * A * pw
    # everywhere: the array PSF centred on the source, sum_t|s|^2 |sum_a w^{r_a.(q - q_s)}|^2
    q = np.arange(n)
    phase = (cells[:, 0][:, None, None] * (q[None, :, None] - qs) +
             cells[:, 1][:, None, None] * (q[None, None, :] - ps)) / n
    psf = np.abs(np.exp(2j * np.pi * phase).sum(axis=0)) ** 2 * pw
    assert np.abs(img - psf).max() < 1e-9 * A * A * pw


@pytest.mark.parametrize("dq", [(5, -3), (-7, 2), (0, 6)])
def test_point_source_gaussian_kernels(dq):
    """Generator kernels (sigma 1 cell Gaussians with random gains): the peak lands on the source pixel."""
    cfg = configs.scaled(configs.TINY, n_ant=64, n_time=16, n_src=1)
    geo = synth.geometry(cfg)
    g = synth.gains(cfg)
    kern = synth.kernels(geo, g, 1)
    n = cfg.grid_n
    qs, ps = n // 2 + dq[0], n // 2 + dq[1]
    sk = synth.Sky(np.array([2.0]), np.array([[(ps - n / 2) / n, (qs - n / 2) / n]]))
    lam = geo.freqs_hz[0] / configs.C_LIGHT
    rng = np.random.default_rng(0)
    s = rng.standard_normal(cfg.n_time) + 1j * rng.standard_normal(cfg.n_time)
    ph = np.exp(-2j * np.pi * lam * (geo.ant_xy_m[:, 0] * sk.lm[0, 0] + geo.ant_xy_m[:, 1] * sk.lm[0, 1]))
    e = s[:, None] * np.conj(g[:, 0])[None, :] * ph[None, :]
    img = ora.image(e[:, None, :, None], kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, 1.0)[0][0].real
    assert np.unravel_index(np.argmax(img), img.shape) == (qs, ps)


def test_point_source_mirrored_sign_fails():
    """The e^{-2 pi i} transform (the paper's F^T read literally) would put the source at -(l, m)."""
    volts, kern, ant_xy, f, n, cells, s, (qs, ps) = _lone_source_delta(dq=(4, 6))
    img = ora.image(volts, kern, ant_xy, [f], [n], 1.0)[0][0].real
    assert img[qs, ps] > 10 * img[n - qs, n - ps]


# ---------------------------------------------------------------------------------------------------------
# 3b. int8 voltages (Eq. Ea and its footnote: the A/D quantisation folded into the noise term)
# ---------------------------------------------------------------------------------------------------------
def _quantised_quarter_source(n, dq, amps, seed=3, A=12):
    """A lone source at a quarter-grid pixel offset seen by delta-kernel antennas on integer cells: every
    antenna's phase exp(-2 pi i (x l + y m)) is a power of i, so quantising s_t times it is exact per
    component (one of re, im is 0, the other +-Q(s_t)), with Q(s) = clip(rint(s), -127, 127)."""
    rng = np.random.default_rng(seed)
    K = 4
    cells = rng.choice(np.arange(6, n - 6), size=(A, 2))
    ant_xy = np.stack([cells[:, 1] - n / 2, cells[:, 0] - n / 2], axis=1).astype(np.float64)
    qs, ps = n // 2 + dq[0], n // 2 + dq[1]
    l_s, m_s = (ps - n / 2) / n, (qs - n / 2) / n
    ph = np.exp(-2j * np.pi * (ant_xy[:, 0] * l_s + ant_xy[:, 1] * m_s))          # powers of i
    x = np.asarray(amps, dtype=np.float64)[:, None] * ph[None, :]                # [T, A]
    q = np.zeros(x.shape + (2,), dtype=np.int8)
    q[..., 0] = np.clip(np.rint(x.real), -127, 127).astype(np.int8)
    q[..., 1] = np.clip(np.rint(x.imag), -127, 127).astype(np.int8)
    kern = np.zeros((1, A, 1, K, K), dtype=np.complex64)
    kern[0, :, 0, K // 2 - 1, K // 2 - 1] = 1.0
    return q[:, None, :, None, :], kern, ant_xy, (qs, ps)


@pytest.mark.parametrize("dq", [(0, 8), (8, -8), (-8, 0)])
def test_int8_quarter_pixel_source_closed_form(dq):
    """int8 (re, im) pairs read as re + i im: the quantised lone source images at its own pixel with the
    closed-form power sum_t (A Q(s_t))^2 (rounding half to even and the clip at 127 included).  Reading the
    pair as im + i re, or conjugating it, mirrors the image and moves the peak off the source pixel."""
    n = 32
    amps = [100.4, 37.5, 38.5, -64.49, 300.0, 127.6]          # rint: 100, 38, 38, -64; clipped: 127, 127
    volts, kern, ant_xy, (qs, ps) = _quantised_quarter_source(n, dq, amps)
    img = ora.image(volts, kern, ant_xy, [configs.C_LIGHT], [n], 1.0)[0][0].real
    A = ant_xy.shape[0]
    q_amp = np.clip(np.rint(np.asarray(amps)), -127, 127)
    assert list(q_amp) == [100, 38, 38, -64, 127, 127]
    expect = float(np.sum((A * q_amp) ** 2))
    assert np.unravel_index(np.argmax(img), img.shape) == (qs, ps)
    assert img[qs, ps] == expect                                  # integer arithmetic, exact in FP64
    swapped = volts[..., ::-1].copy()
    img_sw = ora.image(swapped, kern, ant_xy, [configs.C_LIGHT], [n], 1.0)[0][0].real
    conj = volts.copy()
    conj[..., 1] = -conj[..., 1]
    img_cj = ora.image(conj, kern, ant_xy, [configs.C_LIGHT], [n], 1.0)[0][0].real
    for wrong in (img_sw, img_cj):
        assert wrong[qs, ps] < 0.5 * expect
        assert np.unravel_index(np.argmax(wrong), wrong.shape) == ((n - qs) % n, (n - ps) % n)


def test_int8_equals_the_same_values_as_complex64():
    """The int8 branch of the unpack step gives exactly the complex values re + i im: an image from int8
    voltages equals, bit for bit, the image from those values stored as complex64 (including -128)."""
    cfg, geo, kern, volts = _small(2, A=18, T=5, seed=12)
    assert volts.dtype == np.int8
    volts = volts.copy()
    volts[0, 0, 0, 0] = (-128, 127)
    volts[1, 0, 3, 1] = (5, -128)
    c64 = (volts[..., 0].astype(np.float32) + 1j * volts[..., 1].astype(np.float32)).astype(np.complex64)
    assert np.array_equal(ora.unpack(volts), c64.astype(np.complex128))
    a = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    b = ora.image(c64, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------------------------------------
# 4. Reduction to the direct-imaging correlator and numpy's inverse FFT
# ---------------------------------------------------------------------------------------------------------
def test_delta_kernels_reduce_to_ifft2():
    rng = np.random.default_rng(11)
    n, A, T, K = 32, 16, 5, 4
    cells = np.stack([rng.integers(4, n - 4, A), rng.integers(4, n - 4, A)], axis=1)
    ant_xy = np.stack([cells[:, 1] - n / 2 + 0.25, cells[:, 0] - n / 2 + 0.75], axis=1)   # sub-cell offsets
    e = rng.standard_normal((T, A)) + 1j * rng.standard_normal((T, A))
    kern = np.zeros((1, A, 1, K, K), dtype=np.complex64)
    kern[0, :, 0, K // 2 - 1, K // 2 - 1] = 1.0
    img = ora.image(e[:, None, :, None], kern, ant_xy, [configs.C_LIGHT], [n], 1.0)[0][0]
    ref = direct_imaging(e, cells, n)
    assert _peak_err(img, ref) < 1e-12


# ---------------------------------------------------------------------------------------------------------
# 5. Single antenna: its power beam; centre pixel |sum_k K(k)|^2 sum_t |E_t|^2
# ---------------------------------------------------------------------------------------------------------
def test_single_antenna_beam():
    rng = np.random.default_rng(5)
    n, K, T = 32, 4, 7
    ant_xy = np.array([[1.3, -2.6]])
    kern = (rng.standard_normal((1, 1, 1, K, K)) + 1j * rng.standard_normal((1, 1, 1, K, K))).astype(np.complex64)
    e = rng.standard_normal((T, 1)) + 1j * rng.standard_normal((T, 1))
    img = ora.image(e[:, None, :, None], kern, ant_xy, [configs.C_LIGHT], [n], 1.0)[0][0]
    pw = np.sum(np.abs(e) ** 2)
    k128 = kern[0, 0, 0].astype(np.complex128)
    assert abs(img[n // 2, n // 2] - pw * abs(k128.sum()) ** 2) < 1e-10 * pw * abs(k128.sum()) ** 2
    # whole image = |2-D DTFT of the kernel|^2 * power (shift-invariant, so the footprint origin drops out)
    ft = np.fft.fftshift(np.fft.ifft2(np.pad(k128, ((0, n - K), (0, n - K))))) * n * n
    assert _peak_err(img, pw * np.abs(ft) ** 2) < 1e-12


# ---------------------------------------------------------------------------------------------------------
# 6. Invariants
# ---------------------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def dual():
    cfg, geo, kern, volts = _small(2, A=20, n=32, T=6, seed=9)
    img = ora.image(volts, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    return cfg, geo, kern, volts, img


def test_invariant_integer_shift(dual):
    cfg, geo, kern, volts, img = dual
    shifted = geo.ant_xy_m + np.array([3.0, -2.0]) * configs.C_LIGHT / geo.freqs_hz[0] * cfg.cell_lambda
    img2 = ora.image(volts, kern, shifted, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    for k in range(4):
        assert _peak_err(img2[k], img[k]) < 1e-11


def test_invariant_scale(dual):
    cfg, geo, kern, volts, img = dual
    e = ora.unpack(volts) * (0.5 - 2.0j)
    img2 = ora.image(e, kern, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    assert _peak_err(img2, img * abs(0.5 - 2.0j) ** 2) < 1e-12


def test_invariant_pol_swap(dual):
    cfg, geo, kern, volts, img = dual
    img2 = ora.image(volts[:, :, :, ::-1], kern[:, :, ::-1], geo.ant_xy_m, geo.freqs_hz, geo.grid_n,
                     cfg.cell_lambda)[0]
    for a, b in [(0, 1), (1, 0), (2, 3), (3, 2)]:
        assert _peak_err(img2[a], img[b]) < 1e-12


def test_invariant_hermitian_and_cauchy_schwarz(dual):
    img = dual[4]
    assert _peak_err(img[3], np.conj(img[2])) < 1e-13
    assert np.abs(img[0].imag).max() < 1e-12 * np.abs(img[0]).max()
    assert img[0].real.min() >= 0 and img[1].real.min() >= 0
    assert np.all(np.abs(img[2]) ** 2 <= img[0].real * img[1].real * (1 + 1e-9) + 1e-9)


def test_invariant_conjugate_mirrors(dual):
    cfg, geo, kern, volts, img = dual
    n = cfg.grid_n
    e = np.conj(ora.unpack(volts))
    img2 = ora.image(e, np.conj(kern), geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    mirror = (n - np.arange(n)) % n
    for a, b in [(0, 0), (1, 1), (2, 3), (3, 2)]:
        assert _peak_err(img2[a], img[b][np.ix_(mirror, mirror)]) < 1e-12


def test_footprint_outside_grid_rejected():
    with pytest.raises(ValueError):
        ora.footprint_origin(np.array([[40.0, 0.0]]), configs.C_LIGHT, 1.0, 64, 4)


def test_pixel_route_matches_full_image(dual):
    cfg, geo, kern, volts, img = dual
    pix = np.array([[0, 0], [16, 16], [3, 29], [31, 7]])
    got = ora.image_pixels(volts, kern[0], geo.ant_xy_m, geo.freqs_hz[0], cfg.grid_n, cfg.cell_lambda, pix,
                           t_batch=4)
    for k in range(4):
        ref = img[k][pix[:, 0], pix[:, 1]]
        assert np.abs(got[k] - ref).max() < 1e-11 * np.abs(img[k]).max()


# ---------------------------------------------------------------------------------------------------------
# 7. Full-polarisation (Jones) kernels and phase-centre tracking
# ---------------------------------------------------------------------------------------------------------
def _jones_kern(kern, rng, leak=0.3):
    """[C, A, 2, K, K] diagonal kernels -> [C, A, 2, 2, K, K] with random leakage terms."""
    C, A, P, K, _ = kern.shape
    J = np.zeros((C, A, 2, 2, K, K), dtype=np.complex64)
    J[:, :, 0, 0], J[:, :, 1, 1] = kern[:, :, 0], kern[:, :, 1]
    J[:, :, 0, 1] = leak * (rng.standard_normal((C, A, K, K)) + 1j * rng.standard_normal((C, A, K, K)))
    J[:, :, 1, 0] = leak * (rng.standard_normal((C, A, K, K)) + 1j * rng.standard_normal((C, A, K, K)))
    return J


def test_jones_fx_identity():
    cfg, geo, kern, volts = _small(2, A=10, n=24, T=4, seed=4, disk=10.0)
    J = _jones_kern(kern, np.random.default_rng(0))
    img = ora.image_jones(volts, J, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    origin = _origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, cfg.grid_n, cfg.ksize)
    fx = fx_image_jones(ora.unpack(volts)[:, 0], J[0], origin, cfg.grid_n)
    for k in range(4):
        assert _peak_err(img[k], fx[k]) < 1e-12


def test_jones_with_diagonal_kernels_is_the_diagonal_image(dual):
    cfg, geo, kern, volts, img = dual
    J = _jones_kern(kern, np.random.default_rng(0), leak=0.0)
    img2 = ora.image_jones(volts, J, geo.ant_xy_m, geo.freqs_hz, geo.grid_n, cfg.cell_lambda)[0]
    assert _peak_err(img2, img) < 1e-13


def test_phase_tracking_moves_the_source_to_the_phase_centre():
    """Phases exp(+2 pi i (u l_s + v m_s)) per antenna (a delay towards the source) move a lone source to the
    image centre; the image then equals that of a source at the centre."""
    volts, kern, ant_xy, f, n, cells, s, (qs, ps) = _lone_source_delta(dq=(5, -3))
    l_s, m_s = (ps - n / 2) / n, (qs - n / 2) / n
    phase = np.exp(2j * np.pi * (ant_xy[:, 0] * l_s + ant_xy[:, 1] * m_s))[None, :, None]
    img = ora.image(ora.apply_phases(volts[:, :, :, :], phase), kern, ant_xy, [f], [n], 1.0)[0][0].real
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2, n // 2)
    A = cells.shape[0]
    assert abs(img[n // 2, n // 2] - A * A * np.sum(np.abs(s) ** 2)) < 1e-9 * A * A * np.sum(np.abs(s) ** 2)


# ---------------------------------------------------------------------------------------------------------
# Electric-field tap and feedback calibration (Section 6)
# ---------------------------------------------------------------------------------------------------------
def _tap_setup(A=30, n=32, T=12, K=4, seed=3, M=3):
    cfg, geo, kern, volts = _small(1, A=A, n=n, T=T, K=K, seed=seed)
    origin = _origin(geo.ant_xy_m, geo.freqs_hz[0], cfg.cell_lambda, n, K)
    e = ora.unpack(volts)[:, 0, :, 0]                                  # [T, A]
    rng = np.random.default_rng(seed)
    pix = rng.integers(0, n, size=(M, 2))
    pix[0] = (n // 2, n // 2)
    return cfg, geo, kern[0, :, 0], origin, e, pix, n


def test_antenna_beam_closed_form_for_a_delta_kernel():
    """One antenna, a single unit tap at (y0, x0): its beam is exp(+2 pi i (row (q - n/2) + col (p - n/2)) / n)
    at the tap's grid cell (row, col) = origin + (y0, x0), written here with numpy's exp."""
    n, K = 32, 4
    kern = np.zeros((1, K, K), dtype=np.complex64)
    kern[0, 1, 2] = 1.0
    origin = np.array([[9, 17]])
    pix = np.array([[3, 30], [16, 16], [21, 5]])
    B = ora.antenna_beams(kern, origin, n, pix)[:, 0]
    row, col = 9 + 1, 17 + 2
    ref = np.exp(2j * np.pi * (row * (pix[:, 0] - n // 2) + col * (pix[:, 1] - n // 2)) / n)
    assert np.abs(B - ref).max() < 1e-12


def test_tap_is_the_sum_of_antenna_beams():
    """E~ at a pixel from the grid-and-transform route equals sum_a B_a E_a (linearity of W^T and F^T)."""
    cfg, geo, kern, origin, e, pix, n = _tap_setup()
    tap = ora.efield_pixels(ora.grid_many(e, kern, origin, n), pix)   # [T, M]
    B = ora.antenna_beams(kern, origin, n, pix)                        # [M, A]
    assert _peak_err(e @ B.T, tap) < 1e-12


def test_feedback_sums_partition_the_calibrator_power():
    """sum_i S_i = <|E(theta)|^2>: the per-antenna correlations of Eq. FBeq2 add up to Eq. FBeq1, and
    <|E(theta)|^2> is the image pixel itself."""
    cfg, geo, kern, origin, e, pix, n = _tap_setup()
    tap = ora.efield_pixels(ora.grid_many(e, kern, origin, n), pix)
    R, Pw, V = ora.feedback_sums(e, tap)
    B = ora.antenna_beams(kern, origin, n, pix)
    S, X, u = ora.feedback_solve(R, Pw, V, B)
    assert np.abs(S.sum(axis=1) - Pw).max() < 1e-12 * Pw.max()
    img = ora.image(ora.unpack(_small(1, A=30, n=32, T=12, K=4, seed=3)[3]), kern[None, :, None],
                    geo.ant_xy_m, geo.freqs_hz, [n], cfg.cell_lambda)[0][0]
    assert np.abs(img[pix[:, 0], pix[:, 1]].real - Pw).max() < 1e-9 * Pw.max()


def test_exclusion_sum_against_brute_force_visibilities():
    """X_i = sum over j, k != i of g_j g_k* v_jk, from the visibility matrix v_jk = sum_t E_j conj(E_k)."""
    cfg, geo, kern, origin, e, pix, n = _tap_setup(A=12, T=9)
    tap = ora.efield_pixels(ora.grid_many(e, kern, origin, n), pix)
    R, Pw, V = ora.feedback_sums(e, tap)
    B = ora.antenna_beams(kern, origin, n, pix)
    S, X, u = ora.feedback_solve(R, Pw, V, B)
    vis = e.T @ np.conj(e)                                             # v_jk
    A = e.shape[1]
    for m in range(pix.shape[0]):
        g = B[m]
        for i in range(A):
            keep = np.arange(A) != i
            ref = np.sum(g[keep][:, None] * np.conj(g[keep])[None, :] * vis[np.ix_(keep, keep)])
            assert abs(X[m, i] - ref) < 1e-10 * abs(Pw[m])
    # the printed Eq. FBeq3 (total minus S_i only) differs from the exact exclusion
    assert np.abs((Pw[:, None] - S) - X).max() > 1e-3 * Pw.max()


def test_gain_update_is_stationary_when_calibrated_and_corrects_errors():
    """One calibrator, no noise: antenna i's voltage is a_i s(t).  With every g_i a_i = 1 the update factor
    is exactly 1 (with the printed factor 2N it would be -1); with a few antennas off by (1 + d_i), one update
    g_i -> u_i g_i leaves them off by O(d^2 + d / N)."""
    rng = np.random.default_rng(11)
    A, T, n, K = 64, 16, 32, 4
    kern = (rng.standard_normal((A, K, K)) + 1j * rng.standard_normal((A, K, K))).astype(np.complex64)
    origin = rng.integers(2, n - K - 2, size=(A, 2))
    pix = np.array([[n // 2 + 3, n // 2 - 5]])
    B = ora.antenna_beams(kern, origin, n, pix)[0]                     # g_i toward the calibrator
    s = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    for d_scale in (0.0, 0.05):
        d = np.zeros(A, dtype=np.complex128)
        bad = rng.choice(A, 8, replace=False)
        d[bad] = d_scale * (rng.standard_normal(8) + 1j * rng.standard_normal(8)) / np.sqrt(2)
        a = (1 + d) / B                                                # true responses: g_i a_i = 1 + d_i
        e = s[:, None] * a[None, :]
        tap = ora.efield_pixels(ora.grid_many(e, kern, origin, n), pix)
        R, Pw, V = ora.feedback_sums(e, tap)
        S, X, u = ora.feedback_solve(R, Pw, V, B[None, :])
        if d_scale == 0.0:
            assert np.abs(u - 1).max() < 1e-9
        else:
            before = np.abs(B * a - 1).max()
            after = np.abs(u[0] * B * a - 1).max()
            assert before > 0.02 and after < 0.2 * before, (before, after)
