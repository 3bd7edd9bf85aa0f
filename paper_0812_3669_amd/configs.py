"""Workload descriptions for the MOFF hot path (grid -> 2-D FFT -> square/accumulate).

Every number here is a property of a synthetic array shaped like the compact radio-cosmology layouts the
paper targets (Introduction; Discussion, filling-factor argument Eqs. Eff1-Eff2).  The paper itself prints no
array layout, so the five workloads below are stated concretely:

* ``tiny``     64 antennas, 30 wavelength disk, 1 channel, 1 pol, 64^2 grid, 256 samples, complex64 voltages.
* ``plain``    256 antennas, 60 wavelength disk at 130 MHz, 32 channels over 100-130 MHz, 2 pols, 128^2 grid,
               4096 samples, int8 voltages.
* ``headline`` 2048 antennas, 200 wavelength disk at 130 MHz, 128 channels over 100-130 MHz, 2 pols, 256^2
               grid, 16384 samples, int8 voltages.
* ``batched``  4096 antennas, 376 wavelength disk at 200 MHz, 256 channels over 50-200 MHz, 2 pols, 6x6
               kernels, per-channel grids between 128^2 and 384^2, 4096 samples in 64-sample blocks.
* ``serving``  Poisson stream of jobs (see ``serve.py``).

Conventions fixed here (the paper leaves them open; the readings are listed in the design notes):
channel centres f_c = f_lo + (c + 1/2)(f_hi - f_lo)/C; the quoted disk diameter in wavelengths holds at the
reference frequency ``disk_ref_hz`` (the top of the band), so every channel's footprint fits its grid; the
cell size is one wavelength; the uv coordinate of an antenna scales with frequency, u = x f / c_light.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

C_LIGHT = 299792458.0

# Allowed grid sizes: 2^a * {1, 3, 5}, multiples of 32 (tile multiple of the FFT kernels).
ALLOWED_GRID_SIZES = (32, 64, 96, 128, 160, 192, 256, 320, 384, 512)


@dataclass(frozen=True)
class Config:
    name: str
    index: int              # seed base = 1000 * index
    n_ant: int
    n_pol: int              # 1 or 2
    n_chan: int
    ksize: int              # kernel footprint K (even)
    f_lo: float             # Hz
    f_hi: float             # Hz
    disk_lambda: float      # array diameter in wavelengths at disk_ref_hz
    disk_ref_hz: float
    grid_n: Optional[int]   # fixed grid size for every channel, or None for per-channel sizing
    n_time: int
    n_src: int
    int8: bool = True
    time_block: int = 64
    cell_lambda: float = 1.0

    @property
    def seed_base(self) -> int:
        return 1000 * self.index

    def freqs(self) -> List[float]:
        """Channel centre frequencies f_c = f_lo + (c + 1/2)(f_hi - f_lo)/C."""
        if self.n_chan == 1:
            return [0.5 * (self.f_lo + self.f_hi)]
        bw = (self.f_hi - self.f_lo) / self.n_chan
        return [self.f_lo + (c + 0.5) * bw for c in range(self.n_chan)]

    def disk_m(self) -> float:
        """Array diameter in metres."""
        return self.disk_lambda * C_LIGHT / self.disk_ref_hz

    def grid_sizes(self) -> List[int]:
        """Per-channel grid size: the fixed size, or the smallest allowed size >= ceil(D_lambda(f_c)) + K + 2."""
        if self.grid_n is not None:
            return [self.grid_n] * self.n_chan
        out = []
        for f in self.freqs():
            need = math.ceil(self.disk_lambda * f / self.disk_ref_hz / self.cell_lambda) + self.ksize + 2
            out.append(min(s for s in ALLOWED_GRID_SIZES if s >= need))
        return out

    def volt_bytes_per_cs(self) -> int:
        """Algorithmic input bytes per channel-sample: every antenna's voltage in each pol (int8 or complex64)."""
        return self.n_ant * self.n_pol * (2 if self.int8 else 8)

    def flops_per_cs(self, n: Optional[int] = None) -> float:
        """Algorithmic flops per channel-sample: 5 n^2 log2(n^2) per pol FFT + 8 N_a P K^2 gridding + products."""
        n = n if n is not None else (self.grid_n or max(self.grid_sizes()))
        fft = 5.0 * n * n * math.log2(n * n) * self.n_pol
        grid = 8.0 * self.n_ant * self.n_pol * self.ksize ** 2
        prod = (16.0 if self.n_pol == 2 else 4.0) * n * n
        return fft + grid + prod


TINY = Config("tiny", 0, n_ant=64, n_pol=1, n_chan=1, ksize=4, f_lo=150e6, f_hi=150e6, disk_lambda=30.0,
              disk_ref_hz=150e6, grid_n=64, n_time=256, n_src=3, int8=False)
PLAIN = Config("plain", 1, n_ant=256, n_pol=2, n_chan=32, ksize=4, f_lo=100e6, f_hi=130e6, disk_lambda=60.0,
               disk_ref_hz=130e6, grid_n=128, n_time=4096, n_src=5)
HEADLINE = Config("headline", 2, n_ant=2048, n_pol=2, n_chan=128, ksize=4, f_lo=100e6, f_hi=130e6,
                  disk_lambda=200.0, disk_ref_hz=130e6, grid_n=256, n_time=16384, n_src=5)
BATCHED = Config("batched", 3, n_ant=4096, n_pol=2, n_chan=256, ksize=6, f_lo=50e6, f_hi=200e6,
                 disk_lambda=376.0, disk_ref_hz=200e6, grid_n=None, n_time=4096, n_src=8)

CONFIGS = {c.name: c for c in (TINY, PLAIN, HEADLINE, BATCHED)}


def scaled(cfg: Config, **kw) -> Config:
    """A copy of ``cfg`` with some fields replaced (used for the small parity variants)."""
    d = {f: getattr(cfg, f) for f in cfg.__dataclass_fields__}
    d.update(kw)
    return Config(**d)
