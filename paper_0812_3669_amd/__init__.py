"""MI355X-native MOFF correlator hot path (gridding -> 2-D FFT -> polarisation products, accumulated).

The compute path is the HIP library ``libmoff.so`` (C ABI declared in ``include/moff.h``); ``api`` is a thin
ctypes binding over it.  Nothing here falls back to a CPU implementation.
"""
__all__ = ["configs", "synth"]
