"""Seeded synthetic inputs for the MOFF hot path: antenna layout, gains, sky, kernels and voltages.

This module is shared by the tests, the benchmark and the oracle checks.  It holds only the *input model*
(the antenna voltage model of Eq. Ea and the sky of the measurement equation), never the correlator's
arithmetic (gridding, the spatial transform, squaring).

Recipe (all draws from numpy PCG64; seed base = 1000 * config index):

* positions (seed base+0): uniform in a disk of diameter D, r = (D/2) sqrt(U), phi = 2 pi U'.
* gains (seed base+1): g[a, p] = exp(i phi), phi ~ U[0, 2 pi).
* sources (seed base+2): flux S ~ U[1, 5], direction (l, m) ~ U(-0.5, 0.5)^2.
* voltages (seed base+3): E[t, c, a, p] = conj(g[a, p]) sum_s sqrt(S_s / P) z[t, c, s, p] exp(-2 pi i (u l_s + v m_s))
  + n[t, c, a, p], with z and n unit complex Gaussians (E|z|^2 = 1) independent per (t, c, s, p) and
  (t, c, a, p).  The gains cancel against the kernels, which carry g (calibrated data).
* int8 quantisation: alpha = 16 / sqrt(P_tot / 2) with P_tot = sum_s S_s / P + 1 the expected power per
  pol, q = clip(rint(alpha x), -127, 127) per component, interleaved (re, im).
* kernels: K[c, a, p, y, x] = g[a, p] exp(-((i0 + x - X)^2 + (j0 + y - Y)^2) / 2), a Gaussian of one cell
  sigma sampled at the antenna's sub-cell offset, where X = u / cell + n / 2 and the K x K footprint starts
  at i0 = floor(X) - K/2 + 1 (and likewise in Y).  Stored as complex64.

Large workloads draw their voltages on the GPU with torch's Philox generator (``voltages_device``): same
model, a different random stream, chunked over time so any chunk can be regenerated alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from .configs import C_LIGHT, Config


@dataclass
class Geometry:
    ant_xy_m: np.ndarray      # float64 [A, 2]  (east, north) metres
    freqs_hz: np.ndarray      # float64 [C]
    grid_n: np.ndarray        # int32 [C]
    cell_lambda: float
    ksize: int


@dataclass
class Sky:
    flux: np.ndarray          # float64 [S]
    lm: np.ndarray            # float64 [S, 2]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def positions(cfg: Config, n_ant: Optional[int] = None) -> np.ndarray:
    """Antenna positions uniform in the array disk (metres), float64 [A, 2]."""
    n_ant = cfg.n_ant if n_ant is None else n_ant
    rng = _rng(cfg.seed_base + 0)
    r = 0.5 * cfg.disk_m() * np.sqrt(rng.random(n_ant))
    phi = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)


def geometry(cfg: Config) -> Geometry:
    return Geometry(positions(cfg), np.asarray(cfg.freqs(), dtype=np.float64),
                    np.asarray(cfg.grid_sizes(), dtype=np.int32), cfg.cell_lambda, cfg.ksize)


def gains(cfg: Config) -> np.ndarray:
    """Unit-modulus random-phase complex gains, complex128 [A, P]."""
    rng = _rng(cfg.seed_base + 1)
    return np.exp(1j * 2.0 * np.pi * rng.random((cfg.n_ant, cfg.n_pol)))


def sky(cfg: Config) -> Sky:
    rng = _rng(cfg.seed_base + 2)
    flux = rng.uniform(1.0, 5.0, cfg.n_src)
    lm = rng.uniform(-0.5, 0.5, (cfg.n_src, 2))
    return Sky(flux, lm)


def kernels(geo: Geometry, g: np.ndarray, n_pol: int) -> np.ndarray:
    """Per-antenna K x K Gaussian kernels at each channel's sub-cell offset, complex64 [C, A, P, K, K]."""
    K = geo.ksize
    C, A = len(geo.freqs_hz), geo.ant_xy_m.shape[0]
    out = np.empty((C, A, n_pol, K, K), dtype=np.complex64)
    taps = np.arange(K, dtype=np.float64)
    g64 = g[:, :n_pol].astype(np.complex64)
    for c in range(C):
        lam_cells = geo.freqs_hz[c] / C_LIGHT / geo.cell_lambda
        X = geo.ant_xy_m[:, 0] * lam_cells + geo.grid_n[c] / 2
        Y = geo.ant_xy_m[:, 1] * lam_cells + geo.grid_n[c] / 2
        dx = np.floor(X)[:, None] - K // 2 + 1 + taps[None, :] - X[:, None]   # [A, K]
        dy = np.floor(Y)[:, None] - K // 2 + 1 + taps[None, :] - Y[:, None]
        env = np.exp(-(dy[:, :, None] ** 2 + dx[:, None, :] ** 2) / 2.0)      # [A, K(y), K(x)]
        np.multiply(g64[:, :, None, None], env.astype(np.float32)[:, None, :, :], out=out[c])
    return out


def quant_scale(cfg: Config, sk: Sky) -> float:
    p_tot = float(np.sum(sk.flux)) / cfg.n_pol + 1.0
    return 16.0 / math.sqrt(p_tot / 2.0)


def _source_phases(geo: Geometry, sk: Sky) -> np.ndarray:
    """exp(-2 pi i (u l + v m)) per (channel, antenna, source), complex128 [C, A, S]."""
    lam = geo.freqs_hz / C_LIGHT                                            # [C] 1/m
    ph = (geo.ant_xy_m[None, :, None, 0] * sk.lm[None, None, :, 0] +
          geo.ant_xy_m[None, :, None, 1] * sk.lm[None, None, :, 1]) * lam[:, None, None]
    return np.exp(-2j * np.pi * ph)


def voltages_host(cfg: Config, geo: Geometry, g: np.ndarray, sk: Sky, n_time: Optional[int] = None,
                  chans: Optional[Sequence[int]] = None) -> np.ndarray:
    """Voltages drawn on the host.

    Returns int8 [T, C, A, P, 2] for int8 workloads, complex64 [T, C, A, P] otherwise.  ``chans`` restricts the
    draw to a subset of channels (the random stream is drawn for all channels, so subsets are consistent).
    """
    T = cfg.n_time if n_time is None else n_time
    C, A, P, S = len(geo.freqs_hz), geo.ant_xy_m.shape[0], cfg.n_pol, len(sk.flux)
    rng = _rng(cfg.seed_base + 3)
    z = (rng.standard_normal((T, C, S, P)) + 1j * rng.standard_normal((T, C, S, P))) / math.sqrt(2.0)
    nz = (rng.standard_normal((T, C, A, P)) + 1j * rng.standard_normal((T, C, A, P))) / math.sqrt(2.0)
    amp = np.sqrt(sk.flux / P)                                              # [S]
    ph = _source_phases(geo, sk)                                            # [C, A, S]
    sig = np.einsum("cas,tcsp->tcap", ph * amp[None, None, :], z)
    x = np.conj(g)[None, None, :, :] * sig + nz
    if chans is not None:
        x = x[:, list(chans)]
    if not cfg.int8:
        return x.astype(np.complex64)
    alpha = quant_scale(cfg, sk)
    q = np.empty(x.shape + (2,), dtype=np.int8)
    q[..., 0] = np.clip(np.rint(alpha * x.real), -127, 127).astype(np.int8)
    q[..., 1] = np.clip(np.rint(alpha * x.imag), -127, 127).astype(np.int8)
    return q


def source_response(cfg: Config, geo: Geometry, g: np.ndarray, sk: Sky) -> np.ndarray:
    """Per-(channel, antenna, source, pol) response of the voltage model with conj(g) folded in, complex64
    [C, A, S, P] (host side of ``DeviceVoltages``; it can be built ahead of the device generator)."""
    ph = _source_phases(geo, sk) * np.sqrt(sk.flux / cfg.n_pol)[None, None, :]
    return (ph[:, :, :, None] * np.conj(g)[None, :, None, :]).astype(np.complex64)


class DeviceVoltages:
    """int8 voltages drawn on a torch device, chunk by chunk in time, from the same model.

    Chunk k (samples [k*chunk, (k+1)*chunk)) uses a Philox generator seeded with (seed base + 3) * 1_000_003 + k,
    so any chunk can be redrawn alone.  Output layout int8 [T, C, A, P, 2].
    """

    def __init__(self, cfg: Config, geo: Geometry, g: np.ndarray, sk: Sky, device, chunk: int = 64,
                 resp: Optional[np.ndarray] = None):
        import torch
        self.torch = torch
        self.cfg, self.device, self.chunk = cfg, device, chunk
        if resp is None:
            resp = source_response(cfg, geo, g, sk)
        self.resp = torch.from_numpy(resp).to(device)
        self.alpha = quant_scale(cfg, sk)
        self.C, self.A, self.S, self.P = resp.shape[0], resp.shape[1], resp.shape[2], resp.shape[3]

    def chunk_into(self, k: int, out) -> None:
        """Fill ``out`` (int8 view [chunk', C, A, P, 2]) with chunk k."""
        torch = self.torch
        t = out.shape[0]
        gen = torch.Generator(device=self.device)
        gen.manual_seed((self.cfg.seed_base + 3) * 1_000_003 + k)
        z = torch.randn((t, self.C, self.S, self.P), dtype=torch.complex64, device=self.device, generator=gen)
        x = torch.einsum("casp,tcsp->tcap", self.resp, z)
        x += torch.randn((t, self.C, self.A, self.P), dtype=torch.complex64, device=self.device, generator=gen)
        xr = torch.view_as_real(x) * self.alpha
        out.copy_(torch.clamp(torch.round(xr), -127, 127).to(torch.int8))

    def all(self, n_time: int):
        torch = self.torch
        v = torch.empty((n_time, self.C, self.A, self.P, 2), dtype=torch.int8, device=self.device)
        for k in range((n_time + self.chunk - 1) // self.chunk):
            t0 = k * self.chunk
            self.chunk_into(k, v[t0:min(n_time, t0 + self.chunk)])
        return v


def workload(cfg: Config, n_time: Optional[int] = None, chans: Optional[Sequence[int]] = None):
    """Convenience bundle for host-sized workloads: (geometry, kernels, voltages)."""
    geo = geometry(cfg)
    g = gains(cfg)
    sk = sky(cfg)
    kern = kernels(geo, g, cfg.n_pol)
    volts = voltages_host(cfg, geo, g, sk, n_time=n_time, chans=chans)
    if chans is not None:
        geo = Geometry(geo.ant_xy_m, geo.freqs_hz[list(chans)], geo.grid_n[list(chans)], geo.cell_lambda,
                       geo.ksize)
        kern = kern[list(chans)]
    return geo, kern, volts
