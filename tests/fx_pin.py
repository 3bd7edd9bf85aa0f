"""Independent formulations used to pin the FP64 oracle (no code shared with it beyond numpy itself).

* ``fx_image``: the FX route.  Visibilities of all ordered antenna pairs (autocorrelations included,
  Eq. visDef), gridded with the two antennas' kernel cross-correlation (Eq. Bdef: B~ = S[W * W^*]) onto a
  wrapped visibility grid, then transformed with numpy's inverse FFT (software holography, Eq. RBeamEq).
  Eqs. m1-m6 state that this equals the MOFF image; wrapping modulo n is exact at integer pixels.
* ``direct_imaging``: the direct-imaging correlator (Section 2) -- delta kernels at integer cells reduce
  the image to sum_t |n^2 ifft2(G_t)|^2 after an fftshift.
"""
from __future__ import annotations

import numpy as np

PRODUCT_PAIRS = {1: [(0, 0)], 2: [(0, 0), (1, 1), (0, 1), (1, 0)]}


def fx_image(e: np.ndarray, kern: np.ndarray, origin: np.ndarray, n: int) -> np.ndarray:
    """e complex128 [T, A, P]; kern [A, P, K, K]; origin int [A, 2] (j0, i0). Returns [n_prod, n, n]."""
    T, A, P = e.shape
    K = kern.shape[-1]
    kern = kern.astype(np.complex128)
    out = []
    for (pp, qq) in PRODUCT_PAIRS[P]:
        vis = np.einsum("ta,tb->ab", e[:, :, pp], np.conj(e[:, :, qq]))          # v_ab over all ordered pairs
        V = np.zeros((n, n), dtype=np.complex128)
        a_idx, b_idx = np.meshgrid(np.arange(A), np.arange(A), indexing="ij")
        a_idx, b_idx = a_idx.ravel(), b_idx.ravel()
        for ky in range(K):
            for kx in range(K):
                for ly in range(K):
                    for lx in range(K):
                        w = kern[a_idx, pp, ky, kx] * np.conj(kern[b_idx, qq, ly, lx]) * vis[a_idx, b_idx]
                        dj = (origin[a_idx, 0] + ky - origin[b_idx, 0] - ly) % n
                        di = (origin[a_idx, 1] + kx - origin[b_idx, 1] - lx) % n
                        np.add.at(V, (dj, di), w)
        img = (n * n) * np.fft.fftshift(np.fft.ifft2(V), axes=(-2, -1))
        out.append(img)
    return np.stack(out)


def fx_image_jones(e: np.ndarray, kern: np.ndarray, origin: np.ndarray, n: int) -> np.ndarray:
    """FX route with 2 x 2 Jones kernels: A_PQ = sum_{a,b,q,r} v_ab^{qr} sum_{taps} K_{a,Pq} conj(K_{b,Qr}),
    visibilities v_ab^{qr} = sum_t E_{a,q} conj(E_{b,r}); kern [A, 2 (P), 2 (q), K, K]."""
    T, A, _ = e.shape
    K = kern.shape[-1]
    kern = kern.astype(np.complex128)
    a_idx, b_idx = np.meshgrid(np.arange(A), np.arange(A), indexing="ij")
    a_idx, b_idx = a_idx.ravel(), b_idx.ravel()
    out = []
    for (PP, QQ) in PRODUCT_PAIRS[2]:
        V = np.zeros((n, n), dtype=np.complex128)
        for q in range(2):
            for r in range(2):
                vis = np.einsum("ta,tb->ab", e[:, :, q], np.conj(e[:, :, r]))[a_idx, b_idx]
                for ky in range(K):
                    for kx in range(K):
                        for ly in range(K):
                            for lx in range(K):
                                w = kern[a_idx, PP, q, ky, kx] * np.conj(kern[b_idx, QQ, r, ly, lx]) * vis
                                dj = (origin[a_idx, 0] + ky - origin[b_idx, 0] - ly) % n
                                di = (origin[a_idx, 1] + kx - origin[b_idx, 1] - lx) % n
                                np.add.at(V, (dj, di), w)
        out.append((n * n) * np.fft.fftshift(np.fft.ifft2(V), axes=(-2, -1)))
    return np.stack(out)


def direct_imaging(e: np.ndarray, cells: np.ndarray, n: int) -> np.ndarray:
    """Delta kernels: antenna a puts E_a on cell (j, i) = cells[a]. e [T, A] -> XX image [n, n]."""
    T = e.shape[0]
    G = np.zeros((T, n, n), dtype=np.complex128)
    for a in range(cells.shape[0]):
        G[:, cells[a, 0], cells[a, 1]] += e[:, a]
    Ef = (n * n) * np.fft.fftshift(np.fft.ifft2(G, axes=(-2, -1)), axes=(-2, -1))
    return np.sum(np.abs(Ef) ** 2, axis=0)
