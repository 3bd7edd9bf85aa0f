"""Python binding of the MOFF hot path: torch for device memory and streams, every step in ``libmoff.so``.

    plan = Plan(ant_xy_m, freqs_hz, grid_n, n_pol=2, ksize=4)        # host-only plan
    plan.bind()                                                       # device workspace + twiddles
    plan.set_kernels(kern)                                            # complex64 [C, A, P, K, K] on the GPU
    acc = plan.new_accumulator()
    plan.correlate(volts, acc)                                        # int8 [T, C, A, P, 2] on the GPU
    images = plan.read_image(acc, n_samples=T)                        # list of complex64 [M, n, n]
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (ACC_FP32, ACC_FP64_COMP, FFT_FP32, FFT_GEMM_FP16, FFT_SPLIT_BF16, FFT_SPLIT_FP16,  # noqa: F401
                   KERNEL_DIAG, KERNEL_JONES, PIPELINE_STREAM, PIPELINE_TWO_PASS, VOLT_C64, VOLT_INT8)


class MoffError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        lib = _lib.load()
        name = lib.moff_status_str(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


def _check(status: int, where: str):
    if status != 0:
        lib = _lib.load()
        raise MoffError(status, where, lib.moff_last_error().decode())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _check_buffer(t, name: str, device, dtypes, nbytes: int):
    """The C ABI takes raw pointers and trusts their extent, so every buffer passed to it is checked here first:
    a torch tensor on the plan's device, contiguous, of one of ``dtypes`` and holding at least ``nbytes`` bytes.
    Raises ValueError (TypeError for a non-tensor); nothing is enqueued then."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if device is None:
        raise ValueError(f"{name}: the plan is not bound to a device (call bind() first)")
    if t.device != torch.device(device):
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    dtypes = dtypes if isinstance(dtypes, (tuple, list)) else (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{name} holds {have} bytes, the call needs {nbytes}")


class Plan:
    """A MOFF correlation plan (geometry, band binning, workspace) for one array and channel set."""

    def __init__(self, ant_xy_m, freqs_hz, grid_n=None, n_pol: int = 2, ksize: int = 4, cell_lambda: float = 1.0,
                 fft_mode: int = FFT_FP32, acc_mode: int = ACC_FP32, time_block: int = 0,
                 volt_format: int = VOLT_INT8, chans_per_block: int = 0, time_group: int = 0,
                 kernel_mode: int = KERNEL_DIAG, n_tap: int = 0):
        self.lib = _lib.load()
        xy = np.ascontiguousarray(ant_xy_m, dtype=np.float64)
        fr = np.ascontiguousarray(freqs_hz, dtype=np.float64)
        self.n_ant, self.n_chan, self.n_pol, self.ksize = xy.shape[0], fr.shape[0], n_pol, ksize
        self.acc_mode, self.volt_format, self.kernel_mode, self.n_tap = acc_mode, volt_format, kernel_mode, n_tap
        gn = None
        if grid_n is not None:
            gn = np.ascontiguousarray(np.broadcast_to(np.asarray(grid_n, dtype=np.int32), (self.n_chan,)))
        d = _lib.PlanDesc()
        d.n_ant, d.n_pol, d.n_chan, d.ksize = self.n_ant, n_pol, self.n_chan, ksize
        d.ant_xy_m = xy.ctypes.data_as(C.POINTER(C.c_double))
        d.freq_hz = fr.ctypes.data_as(C.POINTER(C.c_double))
        d.grid_n = gn.ctypes.data_as(C.POINTER(C.c_int32)) if gn is not None else None
        d.cell_lambda = cell_lambda
        d.fft_mode, d.acc_mode, d.time_block, d.volt_format = fft_mode, acc_mode, time_block, volt_format
        d.chans_per_block, d.time_group, d.kernel_mode, d.n_tap = chans_per_block, time_group, kernel_mode, n_tap
        h = C.c_void_p()
        _check(self.lib.moff_plan(C.byref(d), C.byref(h)), "moff_plan")
        self._h = h
        self._ws = None
        self._kern_ref = None
        self.device = None
        self.grid_n = []
        self.pix_off = []
        for c in range(self.n_chan):
            n = C.c_int32()
            o = C.c_int64()
            _check(self.lib.moff_grid_n(h, c, C.byref(n)), "moff_grid_n")
            _check(self.lib.moff_chan_offset(h, c, C.byref(o)), "moff_chan_offset")
            self.grid_n.append(n.value)
            self.pix_off.append(o.value)
        self.pix_total = self.pix_off[-1] + self.grid_n[-1] ** 2
        self.n_prod = 4 if n_pol == 2 else 1

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.moff_plan_destroy(h)
            self._h = None

    # ---- sizes -------------------------------------------------------------------------------------------------
    def _size(self, fn) -> int:
        b = C.c_size_t()
        _check(fn(self._h, C.byref(b)), fn.__name__)
        return b.value

    @property
    def workspace_bytes(self) -> int:
        return self._size(self.lib.moff_workspace_size)

    @property
    def acc_bytes(self) -> int:
        return self._size(self.lib.moff_acc_size)

    @property
    def image_bytes(self) -> int:
        return self._size(self.lib.moff_image_size)

    # ---- device state --------------------------------------------------------------------------------------------
    def workspace_bytes_for(self, time_block: int, chans_per_block: int) -> int:
        b = C.c_size_t()
        _check(self.lib.moff_workspace_size_for(self._h, time_block, chans_per_block, C.byref(b)),
               "moff_workspace_size_for")
        return b.value

    def bind(self, device="cuda", stream=None, workspace_bytes: Optional[int] = None):
        """Allocates the device workspace (at least ``workspace_bytes``, e.g. room for the autotuner) and binds."""
        import torch
        n = max(self.workspace_bytes, workspace_bytes or 0, 256)
        self._ws = torch.empty(n + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        _check(self.lib.moff_bind(self._h, C.c_void_p(aligned), C.c_size_t(n), _stream_handle(stream)),
               "moff_bind")
        self.device = self._ws.device
        return self

    def unbind(self):
        """Releases the device workspace.  The plan keeps its host state (footprints, bands, tap groups, row lists)
        and can be bound again, after which its kernels must be set again; until then every call that needs the
        device raises (the buffer checks find no bound device)."""
        self._ws = None
        self._kern_ref = None
        self.device = None
        return self

    def _kernel_shape(self):
        if self.kernel_mode == KERNEL_JONES:
            return (self.n_chan, self.n_ant, 2, 2, self.ksize, self.ksize)
        return (self.n_chan, self.n_ant, self.n_pol, self.ksize, self.ksize)

    def set_kernels(self, kern, stream=None, phase=None):
        """kern: complex64 on the device, [C, A, P, K, K] (diagonal) or [C, A, 2, 2, K, K] (Jones; [.., p, q, ..]
        maps voltage pol q into grid p), the noise weight folded in.  phase: optional complex64 [C, A, P] that
        multiplies each voltage before gridding (phase-centre tracking)."""
        import torch
        shape = self._kernel_shape()
        _check_buffer(kern, "kern", self.device, torch.complex64, int(np.prod(shape)) * 8)
        if tuple(kern.shape) != shape:
            raise ValueError(f"kern must have shape {shape}, got {tuple(kern.shape)}")
        if phase is None:
            _check(self.lib.moff_set_kernels(self._h, _ptr(kern), _stream_handle(stream)), "moff_set_kernels")
        else:
            pshape = (self.n_chan, self.n_ant, self.n_pol)
            _check_buffer(phase, "phase", self.device, torch.complex64, int(np.prod(pshape)) * 8)
            if tuple(phase.shape) != pshape:
                raise ValueError(f"phase must have shape {pshape}, got {tuple(phase.shape)}")
            _check(self.lib.moff_set_kernels_phased(self._h, _ptr(kern), _ptr(phase), _stream_handle(stream)),
                   "moff_set_kernels_phased")
        self._kern_ref = (kern, phase)   # keep alive until the packing kernel has run
        return self

    def new_accumulator(self):
        import torch
        dt = torch.float64 if self.acc_mode == ACC_FP64_COMP else torch.float32
        elems = self.acc_bytes // (8 if dt == torch.float64 else 4)
        return torch.zeros(elems, dtype=dt, device=self.device)

    def _sample_bytes(self) -> int:
        """Bytes of one time sample of voltages (all channels, antennas and pols)."""
        return self.n_chan * self.n_ant * self.n_pol * (2 if self.volt_format == VOLT_INT8 else 8)

    def _check_volts(self, volts, n_t):
        import torch
        if n_t < 0:
            raise ValueError(f"n_t must be >= 0, got {n_t}")
        dt = torch.int8 if self.volt_format == VOLT_INT8 else torch.complex64
        _check_buffer(volts, "volts", self.device, dt, n_t * self._sample_bytes())

    def _check_acc(self, acc, name="acc"):
        import torch
        dt = torch.float64 if self.acc_mode == ACC_FP64_COMP else torch.float32
        _check_buffer(acc, name, self.device, dt, self.acc_bytes)

    def _grid_bytes(self, n_t: int) -> int:
        """Bytes of n_t staged grids or E-field images (complex64, P * sum_c n_c^2 per sample)."""
        return n_t * self.n_pol * self.pix_total * 8

    # ---- the hot path ---------------------------------------------------------------------------------------------
    def correlate(self, volts, acc, n_t: Optional[int] = None, stream=None):
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        self._check_acc(acc)
        _check(self.lib.moff_correlate(self._h, _ptr(volts), n_t, _ptr(acc), _stream_handle(stream)),
               "moff_correlate")

    def correlate_graph(self, volts, acc, n_t: Optional[int] = None, stream=None):
        """Same as correlate, replayed from a captured HIP graph (captured on first use per buffer set)."""
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        self._check_acc(acc)
        _check(self.lib.moff_correlate_graph(self._h, _ptr(volts), n_t, _ptr(acc), _stream_handle(stream)),
               "moff_correlate_graph")

    def correlate_noalloc(self, volts, acc, n_t: Optional[int] = None, stream=None):
        """Same as correlate, with the row-transformed grids in the library's fixed exchange buffer (allocates no
        device memory; for callers that cannot)."""
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        self._check_acc(acc)
        _check(self.lib.moff_correlate_noalloc(self._h, _ptr(volts), n_t, _ptr(acc), _stream_handle(stream)),
               "moff_correlate_noalloc")

    # ---- E-field taps and feedback calibration ---------------------------------------------------------------------
    def set_taps(self, pix, stream=None):
        """pix int [C, n_tap, 2] (or [n_tap, 2] for every channel): centred (row, col) pixels of each channel."""
        pix = np.asarray(pix, dtype=np.int32)
        if pix.ndim == 2:
            pix = np.broadcast_to(pix, (self.n_chan,) + pix.shape)
        pix = np.ascontiguousarray(pix)
        if pix.shape != (self.n_chan, self.n_tap, 2):
            raise ValueError(f"pix must have shape {(self.n_chan, self.n_tap, 2)}, got {pix.shape}")
        self._tap_pix = pix
        _check(self.lib.moff_set_taps(self._h, pix.ctypes.data_as(C.POINTER(C.c_int32)), _stream_handle(stream)),
               "moff_set_taps")
        return self

    def new_tap_buffer(self, n_t: int):
        import torch
        return torch.empty((n_t, self.n_chan, self.n_tap, self.n_pol), dtype=torch.complex64, device=self.device)

    def correlate_tap(self, volts, acc, tap, n_t: Optional[int] = None, stream=None):
        """correlate plus the E-field image at the tapped pixels of every sample: tap complex64 [T, C, n_tap, P]."""
        import torch
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        self._check_acc(acc)
        _check_buffer(tap, "tap", self.device, torch.complex64, n_t * self.n_chan * self.n_tap * self.n_pol * 8)
        _check(self.lib.moff_correlate_tap(self._h, _ptr(volts), n_t, _ptr(acc), _ptr(tap), _stream_handle(stream)),
               "moff_correlate_tap")

    @property
    def cal_bytes(self) -> int:
        return self._size(self.lib.moff_cal_size)

    def new_cal(self):
        import torch
        return torch.zeros(self.cal_bytes // 8, dtype=torch.float64, device=self.device)

    def cal_accumulate(self, volts, tap, cal, n_t: Optional[int] = None, stream=None):
        import torch
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        _check_buffer(tap, "tap", self.device, torch.complex64, n_t * self.n_chan * self.n_tap * self.n_pol * 8)
        _check_buffer(cal, "cal", self.device, torch.float64, self.cal_bytes)
        _check(self.lib.moff_cal_accumulate(self._h, _ptr(volts), _ptr(tap), n_t, _ptr(cal), _stream_handle(stream)),
               "moff_cal_accumulate")

    def split_cal(self, cal):
        """-> R complex128 [C, n_tap, A, P], Pw float64 [C, n_tap, P], V float64 [C, A, P] (views)."""
        import torch
        Cc, M, A, P = self.n_chan, self.n_tap, self.n_ant, self.n_pol
        nr = Cc * M * A * P
        R = torch.view_as_complex(cal[:2 * nr].view(nr, 2)).view(Cc, M, A, P)
        Pw = cal[2 * nr:2 * nr + Cc * M * P].view(Cc, M, P)
        V = cal[2 * nr + Cc * M * P:2 * nr + Cc * M * P + Cc * A * P].view(Cc, A, P)
        return R, Pw, V

    def cal_solve(self, cal, kern, stream=None):
        """-> (S, X, u), each complex128 [C, n_tap, A, P]: the per-antenna correlation with its gain applied,
        the sum of all visibilities not involving the antenna, and the gain-update factor."""
        import torch
        _check_buffer(cal, "cal", self.device, torch.float64, self.cal_bytes)
        kshape = (self.n_chan, self.n_ant, self.n_pol, self.ksize, self.ksize)
        _check_buffer(kern, "kern", self.device, torch.complex64, int(np.prod(kshape)) * 8)
        shape = (3, self.n_chan, self.n_tap, self.n_ant, self.n_pol)
        out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        _check(self.lib.moff_cal_solve(self._h, _ptr(cal), _ptr(kern), _ptr(out), _stream_handle(stream)),
               "moff_cal_solve")
        return out[0], out[1], out[2]

    def set_pipeline(self, pipeline: int):
        """PIPELINE_TWO_PASS (row and column kernels) or PIPELINE_STREAM (one persistent launch per grid size)."""
        _check(self.lib.moff_set_pipeline(self._h, int(pipeline)), "moff_set_pipeline")
        return self

    def stream_status(self) -> int:
        """Status code of the streaming form's last call (0 = fine); synchronises the device."""
        code = C.c_int32()
        _check(self.lib.moff_stream_status(self._h, C.byref(code)), "moff_stream_status")
        return code.value

    def launch_shape(self):
        tb, cpb, tg = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib.moff_get_launch_shape(self._h, C.byref(tb), C.byref(cpb), C.byref(tg)), "launch shape")
        return tb.value, cpb.value, tg.value

    def set_launch_shape(self, time_block: int, chans_per_block: int, time_group: int):
        _check(self.lib.moff_set_launch_shape(self._h, time_block, chans_per_block, time_group), "set launch shape")

    def autotune(self, volts, acc, n_t: Optional[int] = None, stream=None, cache: Optional[str] = None):
        """Times candidate launch shapes on this input (acc is scratch); keeps and returns the fastest.  With
        ``cache`` (a text file, created if missing) a shape tuned earlier for the same plan signature
        (``autotune_key``) is applied without timing (``"cached": True``); a new result is appended to it."""
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        self._check_acc(acc)
        tb, cpb, tg, ms, hit = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double(), C.c_int32(0)
        if cache is None:
            _check(self.lib.moff_autotune(self._h, _ptr(volts), n_t, _ptr(acc), _stream_handle(stream),
                                          C.byref(tb), C.byref(cpb), C.byref(tg), C.byref(ms)), "moff_autotune")
        else:
            _check(self.lib.moff_autotune_cached(self._h, os.fsencode(cache), _ptr(volts), n_t, _ptr(acc),
                                                 _stream_handle(stream), C.byref(tb), C.byref(cpb), C.byref(tg),
                                                 C.byref(ms), C.byref(hit)), "moff_autotune_cached")
        return {"time_block": tb.value, "chans_per_block": cpb.value, "time_group": tg.value, "ms": ms.value,
                "cached": bool(hit.value)}

    @property
    def autotune_key(self) -> str:
        """The autotuner cache's key for this plan (every input of the launch-shape choice)."""
        buf = C.create_string_buffer(1024)
        _check(self.lib.moff_autotune_key(self._h, buf, len(buf)), "moff_autotune_key")
        return buf.value.decode()

    def grid(self, volts, n_t: Optional[int] = None, out=None, stream=None):
        import torch
        n_t = volts.shape[0] if n_t is None else n_t
        self._check_volts(volts, n_t)
        if out is None:
            out = torch.empty(n_t * self.n_pol * self.pix_total, dtype=torch.complex64, device=self.device)
        _check_buffer(out, "out", self.device, torch.complex64, self._grid_bytes(n_t))
        _check(self.lib.moff_grid(self._h, _ptr(volts), n_t, _ptr(out), _stream_handle(stream)), "moff_grid")
        return out

    def fft(self, grid, n_t: int, stream=None):
        import torch
        if n_t < 0:
            raise ValueError(f"n_t must be >= 0, got {n_t}")
        _check_buffer(grid, "grid", self.device, torch.complex64, self._grid_bytes(n_t))
        _check(self.lib.moff_fft(self._h, _ptr(grid), n_t, _stream_handle(stream)), "moff_fft")
        return grid

    def accumulate(self, efield, n_t: int, acc, stream=None):
        import torch
        if n_t < 0:
            raise ValueError(f"n_t must be >= 0, got {n_t}")
        _check_buffer(efield, "efield", self.device, torch.complex64, self._grid_bytes(n_t))
        self._check_acc(acc)
        _check(self.lib.moff_accumulate(self._h, _ptr(efield), n_t, _ptr(acc), _stream_handle(stream)),
               "moff_accumulate")

    def read_image(self, acc, n_samples: int = 0, normalize: bool = False, stream=None, split: bool = True):
        import torch
        self._check_acc(acc)
        img = torch.empty(self.n_prod * self.pix_total, dtype=torch.complex64, device=self.device)
        _check(self.lib.moff_read_image(self._h, _ptr(acc), n_samples, int(bool(normalize)), _ptr(img),
                                        _stream_handle(stream)), "moff_read_image")
        if not split:
            return img
        return self.split_images(img)

    def split_images(self, flat) -> List:
        out = []
        for c in range(self.n_chan):
            n = self.grid_n[c]
            o = self.n_prod * self.pix_off[c]
            out.append(flat[o:o + self.n_prod * n * n].view(self.n_prod, n, n))
        return out

    def split_grids(self, flat, n_t: int) -> List:
        """Staged grid/E-field buffer -> list over channels of [n_t, P, n, n] views."""
        per = self.n_pol * self.pix_total
        v = flat[: n_t * per].view(n_t, per)
        out = []
        for c in range(self.n_chan):
            n = self.grid_n[c]
            o = self.n_pol * self.pix_off[c]
            out.append(v[:, o:o + self.n_pol * n * n].view(n_t, self.n_pol, n, n))
        return out

    # ---- kernel timing ------------------------------------------------------------------------------------------------
    def profile(self, enable: bool):
        _check(self.lib.moff_profile(self._h, int(bool(enable))), "moff_profile")

    def profile_read(self, kind: int):
        """(total ms, launches, channel-samples) of kind 0 (row pass) or 1 (column pass); syncs the events."""
        ms, n, cs = C.c_double(), C.c_int64(), C.c_int64()
        _check(self.lib.moff_profile_read(self._h, kind, C.byref(ms), C.byref(n), C.byref(cs)), "moff_profile_read")
        return ms.value, n.value, cs.value

    # ---- test hooks ------------------------------------------------------------------------------------------------
    def debug_unpack(self, volt_sample, stream=None):
        import torch
        dt = torch.int8 if self.volt_format == VOLT_INT8 else torch.complex64
        _check_buffer(volt_sample, "volt_sample", self.device, dt, self._sample_bytes())
        out = torch.empty(self.n_chan * self.n_ant * self.n_pol * 2, dtype=torch.float32, device=self.device)
        _check(self.lib.moff_debug_unpack(self._h, _ptr(volt_sample), _ptr(out), _stream_handle(stream)),
               "moff_debug_unpack")
        return out.view(self.n_chan, self.n_ant, self.n_pol, 2)

    def debug_tiles(self):
        nb, ne = C.c_int64(), C.c_int64()
        rows = np.zeros(self.n_chan, dtype=np.int32)
        _check(self.lib.moff_debug_tile_counts(self._h, C.byref(nb), C.byref(ne),
                                               rows.ctypes.data_as(C.POINTER(C.c_int32))), "tile counts")
        origin = np.zeros((self.n_chan, self.n_ant, 2), dtype=np.int32)
        ptr = np.zeros(nb.value + 1, dtype=np.int32)
        ant = np.zeros(max(ne.value, 1), dtype=np.int32)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
        _check(self.lib.moff_debug_tiles(self._h, ip(origin), ip(ptr), ip(ant)), "moff_debug_tiles")
        return origin, ptr, ant[: ne.value], rows


def probe(kind: int, blocks: int, iters: int, out, stream=None):
    """Enqueues a probe (``moff_probe``): kind 0 FP32 vector FMAs, kind 1 FP16 matrix-core instructions (``out`` a
    device float32 tensor of blocks x 256 elements); kinds 2 and 3 the exchange probes, 256-point transforms with
    an LDS transpose or cross-lane exchanges (``out`` a device complex64 tensor of blocks x 16 x 256 elements,
    transformed in place); kind 4 the XCD of each workgroup; kinds 5 and 6 the exchange's store and load patterns
    over ``blocks`` channel-samples (``out`` a device complex64 tensor of blocks x 2 x 256 x 256 elements).  Returns
    the flops it performs (5 N log2 N per transform for kinds 2 and 3), or for kinds 5 and 6 the bytes it moves."""
    import torch
    lib = _lib.load()
    if not isinstance(out, torch.Tensor) or not out.is_cuda:
        raise ValueError("out must be a device tensor")
    if kind in (0, 1):
        _check_buffer(out, "out", out.device, torch.float32, blocks * 256 * 4)
    elif kind in (2, 3):
        _check_buffer(out, "out", out.device, torch.complex64, blocks * 16 * 256 * 8)
    elif kind == 4:
        _check_buffer(out, "out", out.device, torch.float32, blocks * 4)
    elif kind in (5, 6):
        _check_buffer(out, "out", out.device, torch.complex64, blocks * 2 * 65536 * 8)
    else:
        raise ValueError(f"unknown probe kind {kind}")
    _check(lib.moff_probe(kind, blocks, iters, _ptr(out), _stream_handle(stream)), "probe")
    if kind == 0:
        return blocks * 256 * iters * 16
    if kind == 1:
        return blocks * 4 * iters * 4 * 16384
    if kind == 4:
        return 0
    if kind in (5, 6):
        return blocks * 2 * 65536 * 8
    return blocks * 16 * iters * 5 * 256 * 8


def plan_for(cfg, geo, **kw) -> "Plan":
    """Plan for a workload description (``configs.Config``) and its geometry (``synth.Geometry``)."""
    return Plan(geo.ant_xy_m, geo.freqs_hz, geo.grid_n, n_pol=cfg.n_pol, ksize=cfg.ksize,
                cell_lambda=cfg.cell_lambda, volt_format=VOLT_INT8 if cfg.int8 else VOLT_C64, **kw)
