"""FP64 CPU oracle for the MOFF hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import this
module.  The product (the HIP library and its Python binding) never calls it, and it shares no code with
them: it takes plain numpy arrays produced by the seeded input generator and nothing else.

What it computes is the plain definition of the MOFF image (Section 4, Eq. m6; the direct-imaging
correlator's I = <|E(theta)|^2>_t, Section 2):

    I'(theta) = < | F^T(theta, r) W^T(r, a) N~(a, a) E'(a) |^2 >_t

step by step and in the paper's order, in float64/complex128:

1. E'(a): the channelised voltages, int8 (re, im) pairs converted exactly (Eq. Ea; its footnote folds the
   A/D quantisation into the noise term).
2. N~: a diagonal per-antenna, per-pol weight (Eq. m4 defines N^-1 = N~^T N~).  The workloads fold it into
   the kernels, so the oracle applies the kernels as given.
3. W^T(r, a): every antenna's channelised voltage is spread onto the regular grid r through its own K x K
   complex kernel (Eq. m6 step 2; Section 4, grid spacing free, item 2 of the MOFF properties).  The
   kernel is multiplied as given, with no conjugation.  Footprint convention: cell centres are integers,
   X = u / cell + n / 2, and the footprint covers cells floor(X) - K/2 + 1 ... floor(X) + K/2.
4. F^T(theta, r): a direct DFT, no FFT factorisation:
       E~[q, p] = sum_{j, i} D[j, q] G[j, i] D[i, p],  D[k, q] = exp(+2 pi i ((k (q - n/2)) mod n) / n)
   with the angle reduced in integers before cos/sin.  The sign is +, the adjoint of the e^{-2 pi i u.theta}
   of the voltage model (Eq. Ea), so a source at (l, m) images at +(l, m).  Pixel (q, p) <-> direction
   (m, l) = ((q - n/2), (p - n/2)) / (n cell).  Evaluated separably as two complex128 matrix products, which
   is the same double sum for every pixel.
5. |.|^2 and <.>_t: polarisation products XX = |E_X|^2, YY = |E_Y|^2, XY = E_X conj(E_Y) and
   YX = E_Y conj(E_X) (computed on its own, not as a conjugate) summed -- not averaged -- over time
   (Eq. m6; Discussion, four polarisations).  Single-pol data gives one product, |E|^2.

Output: complex128 [C, n_prod, n, n] with products ordered XX, YY, XY, YX (n_prod = 4) or XX (n_prod = 1).
"""
from __future__ import annotations

import math
from typing import Iterable, List, Optional, Sequence

import numpy as np

C_LIGHT = 299792458.0


# ---------------------------------------------------------------------------------------------------------
# Step 1: voltages (Eq. Ea)
# ---------------------------------------------------------------------------------------------------------
def unpack(volts: np.ndarray) -> np.ndarray:
    """int8 [..., 2] (re, im) -> complex128 [...], exactly; complex64 input is promoted."""
    if volts.dtype == np.int8:
        return volts[..., 0].astype(np.float64) + 1j * volts[..., 1].astype(np.float64)
    return volts.astype(np.complex128)


# ---------------------------------------------------------------------------------------------------------
# Geometry (Section 4: free grid spacing; ground-fixed grid axes)
# ---------------------------------------------------------------------------------------------------------
def cell_coords(ant_xy_m: np.ndarray, freq_hz: float, cell_lambda: float, n: int):
    """Fractional cell coordinates (X, Y) = (u, v) / cell + n / 2 with (u, v) = (x, y) f / c, in float64."""
    scale = freq_hz / C_LIGHT / cell_lambda
    X = ant_xy_m[:, 0] * scale + n / 2
    Y = ant_xy_m[:, 1] * scale + n / 2
    return X, Y


def footprint_origin(ant_xy_m: np.ndarray, freq_hz: float, cell_lambda: float, n: int, K: int) -> np.ndarray:
    """First covered cell (j0, i0) per antenna, int64 [A, 2]; raises if any footprint leaves the grid."""
    X, Y = cell_coords(ant_xy_m, freq_hz, cell_lambda, n)
    i0 = np.floor(X).astype(np.int64) - K // 2 + 1
    j0 = np.floor(Y).astype(np.int64) - K // 2 + 1
    if np.any(i0 < 0) or np.any(j0 < 0) or np.any(i0 + K > n) or np.any(j0 + K > n):
        raise ValueError("an antenna footprint leaves the grid")
    return np.stack([j0, i0], axis=1)


# ---------------------------------------------------------------------------------------------------------
# Step 3: gridding W^T (Eq. m6, step 2)
# ---------------------------------------------------------------------------------------------------------
def grid(e: np.ndarray, kern: np.ndarray, origin: np.ndarray, n: int) -> np.ndarray:
    """G[j0 + y, i0 + x] += K_a[y, x] * E_a for every antenna a and tap (y, x).

    e: complex128 [A] one pol's voltages at one (t, c); kern: complex [A, K, K]; origin: [A, 2] (j0, i0).
    Returns complex128 [n, n] indexed [j (north, v), i (east, u)].
    """
    A, K = kern.shape[0], kern.shape[1]
    G = np.zeros((n, n), dtype=np.complex128)
    contrib = kern.astype(np.complex128) * e[:, None, None]                  # [A, K, K]
    jj = origin[:, 0][:, None, None] + np.arange(K)[None, :, None]
    ii = origin[:, 1][:, None, None] + np.arange(K)[None, None, :]
    np.add.at(G, (np.broadcast_to(jj, (A, K, K)), np.broadcast_to(ii, (A, K, K))), contrib)
    return G


def grid_many(e: np.ndarray, kern: np.ndarray, origin: np.ndarray, n: int) -> np.ndarray:
    """The same gridding for a batch of samples: e complex128 [T, A] -> G complex128 [T, n, n].

    The sum for each cell is the sum of step 3, accumulated as a (cells x antennas) sparse weight matrix
    applied to the voltage batch with one library matrix product.
    """
    import scipy.sparse as sp
    A, K = kern.shape[0], kern.shape[1]
    jj = origin[:, 0][:, None, None] + np.arange(K)[None, :, None]
    ii = origin[:, 1][:, None, None] + np.arange(K)[None, None, :]
    cell = (np.broadcast_to(jj, (A, K, K)) * n + np.broadcast_to(ii, (A, K, K))).ravel()
    ant = np.broadcast_to(np.arange(A)[:, None, None], (A, K, K)).ravel()
    W = sp.csr_matrix((kern.astype(np.complex128).ravel(), (cell, ant)), shape=(n * n, A))
    return np.ascontiguousarray(np.asarray((W @ e.T).T)).reshape(e.shape[0], n, n)


# ---------------------------------------------------------------------------------------------------------
# Step 4: spatial transform F^T as a direct DFT (Eq. m6, step 3)
# ---------------------------------------------------------------------------------------------------------
def dft_matrix(n: int) -> np.ndarray:
    """D[k, q] = exp(+2 pi i ((k (q - n/2)) mod n) / n), angle reduced in integers, complex128 [n, n]."""
    k = np.arange(n, dtype=np.int64)[:, None]
    q = np.arange(n, dtype=np.int64)[None, :]
    r = np.mod(k * (q - n // 2), n)
    ang = 2.0 * np.pi * r.astype(np.float64) / n
    return np.cos(ang) + 1j * np.sin(ang)


def efield_image(G: np.ndarray, D: Optional[np.ndarray] = None) -> np.ndarray:
    """E~[q, p] = sum_{j, i} D[j, q] G[j, i] D[i, p] for G [..., n, n]."""
    n = G.shape[-1]
    D = dft_matrix(n) if D is None else D
    return np.matmul(np.matmul(D.T, G), D)


def efield_pixels(G: np.ndarray, pix: np.ndarray) -> np.ndarray:
    """E~ at selected pixels only: pix int [M, 2] (q, p); G [T, n, n] -> complex128 [T, M].

    The same double sum for each pixel, summed over the column index i first (a matrix product with the
    selected columns of D), then over the row index j.
    """
    n = G.shape[-1]
    D = dft_matrix(n)
    GD = np.matmul(G, D[:, pix[:, 1]])                     # [T, n (j), M]: sum over i of G[j, i] D[i, p_m]
    return np.einsum("tjm,jm->tm", GD, D[:, pix[:, 0]])    # sum over j of D[j, q_m] (...)


# ---------------------------------------------------------------------------------------------------------
# Step 5: polarisation products, summed over time (Eq. m6; Discussion)
# ---------------------------------------------------------------------------------------------------------
def pol_products(ex: np.ndarray, ey: Optional[np.ndarray]) -> List[np.ndarray]:
    """[XX, YY, XY, YX] for dual pol, [XX] for single pol; inputs complex128 of any shape."""
    if ey is None:
        return [(ex * np.conj(ex))]
    return [ex * np.conj(ex), ey * np.conj(ey), ex * np.conj(ey), ey * np.conj(ex)]


# ---------------------------------------------------------------------------------------------------------
# The whole definition
# ---------------------------------------------------------------------------------------------------------
def image(volts: np.ndarray, kern: np.ndarray, ant_xy_m: np.ndarray, freqs_hz: Sequence[float],
          grid_n: Sequence[int], cell_lambda: float, t_batch: int = 16) -> List[np.ndarray]:
    """The MOFF image for every channel.

    volts: int8 [T, C, A, P, 2] or complex [T, C, A, P]; kern: complex64 [C, A, P, K, K].
    Returns a list over channels of complex128 [n_prod, n_c, n_c] (sums over the T samples).
    """
    e_all = unpack(volts)
    T, C, A, P = e_all.shape
    K = kern.shape[-1]
    out = []
    for c in range(C):
        n = int(grid_n[c])
        origin = footprint_origin(ant_xy_m, freqs_hz[c], cell_lambda, n, K)
        D = dft_matrix(n)
        acc = np.zeros((4 if P == 2 else 1, n, n), dtype=np.complex128)
        for t0 in range(0, T, t_batch):
            t1 = min(T, t0 + t_batch)
            ef = []
            for p in range(P):
                G = grid_many(e_all[t0:t1, c, :, p], kern[c, :, p], origin, n)    # [t, n, n]
                ef.append(efield_image(G, D))
            prods = pol_products(ef[0], ef[1] if P == 2 else None)
            for k, pr in enumerate(prods):
                acc[k] += pr.sum(axis=0)
        out.append(acc)
    return out


def image_jones(volts: np.ndarray, kern: np.ndarray, ant_xy_m: np.ndarray, freqs_hz: Sequence[float],
                grid_n: Sequence[int], cell_lambda: float, t_batch: int = 16) -> List[np.ndarray]:
    """The MOFF image with full-polarisation (2 x 2 Jones) kernels: grid p receives every pol q of each antenna,
    G_p = sum_a sum_q K_{a,pq} E_{a,q} (the polarimetric form of Eq. m6 step 2); the rest as in ``image``.

    kern: complex [C, A, 2 (p), 2 (q), K, K].  Returns a list over channels of complex128 [4, n_c, n_c].
    """
    e_all = unpack(volts)
    T, C, A, P = e_all.shape
    K = kern.shape[-1]
    out = []
    for c in range(C):
        n = int(grid_n[c])
        origin = footprint_origin(ant_xy_m, freqs_hz[c], cell_lambda, n, K)
        D = dft_matrix(n)
        acc = np.zeros((4, n, n), dtype=np.complex128)
        for t0 in range(0, T, t_batch):
            t1 = min(T, t0 + t_batch)
            ef = []
            for p in range(2):
                G = sum(grid_many(e_all[t0:t1, c, :, q], kern[c, :, p, q], origin, n) for q in range(2))
                ef.append(efield_image(G, D))
            for k, pr in enumerate(pol_products(ef[0], ef[1])):
                acc[k] += pr.sum(axis=0)
        out.append(acc)
    return out


def apply_phases(volts: np.ndarray, phase: np.ndarray) -> np.ndarray:
    """Phase-centre tracking (Section 4): each antenna's channelised voltage times its phase, before gridding.
    volts int8 [T, C, A, P, 2] or complex [T, C, A, P]; phase complex [C, A, P] -> complex128 [T, C, A, P]."""
    return unpack(volts) * phase.astype(np.complex128)[None]


def image_pixels(volts: np.ndarray, kern: np.ndarray, ant_xy_m: np.ndarray, freq_hz: float, n: int,
                 cell_lambda: float, pix: np.ndarray, chan: int = 0, t_batch: int = 256) -> np.ndarray:
    """Selected pixels of one channel's image (same definition, evaluated pixel by pixel).

    volts: int8 [T, C', A, P, 2] (channel ``chan`` used); pix int [M, 2]. Returns complex128 [n_prod, M].
    """
    T, P = volts.shape[0], volts.shape[3]
    K = kern.shape[-1]
    origin = footprint_origin(ant_xy_m, freq_hz, cell_lambda, n, K)
    acc = np.zeros((4 if P == 2 else 1, pix.shape[0]), dtype=np.complex128)
    for t0 in range(0, T, t_batch):
        t1 = min(T, t0 + t_batch)
        e = unpack(volts[t0:t1, chan])
        ef = [efield_pixels(grid_many(e[:, :, p], kern[:, p], origin, n), pix) for p in range(P)]
        prods = pol_products(ef[0], ef[1] if P == 2 else None)
        for k, pr in enumerate(prods):
            acc[k] += pr.sum(axis=0)
    return acc


# ---------------------------------------------------------------------------------------------------------
# Electric-field image tap and feedback calibration (Section 6; Eqs. FBeq1-FBeq3 and the gain update)
# ---------------------------------------------------------------------------------------------------------
def antenna_beams(kern: np.ndarray, origin: np.ndarray, n: int, pix: np.ndarray) -> np.ndarray:
    """B_a(q, p) = sum_{y, x} K_a[y, x] D[j0 + y, q] D[i0 + x, p]: the E-field image of a unit voltage on
    antenna a alone, at centred pixels pix int [M, 2] (q, p).  kern [A, K, K] -> complex128 [M, A].
    By linearity the image pixel is E~(q, p) = sum_a B_a(q, p) E_a: each antenna's calibrated gain toward
    that direction, the g_i of the feedback-calibration equations."""
    A, K = kern.shape[0], kern.shape[1]
    D = dft_matrix(n)
    rows = origin[:, 0][:, None] + np.arange(K)[None, :]          # [A, K] grid rows j0 + y
    cols = origin[:, 1][:, None] + np.arange(K)[None, :]          # [A, K] grid columns i0 + x
    out = np.empty((pix.shape[0], A), dtype=np.complex128)
    k128 = kern.astype(np.complex128)
    for m, (q, p) in enumerate(pix):
        dr = D[rows, q]                                            # [A, K]
        dc = D[cols, p]                                            # [A, K]
        out[m] = np.einsum("ayx,ay,ax->a", k128, dr, dc)
    return out


def feedback_sums(e: np.ndarray, e_tap: np.ndarray):
    """The correlations of the feedback loop over T samples of one channel and pol, as sums over t.

    e complex [T, A] (antenna voltages), e_tap complex [T, M] (E-field image at the calibrator pixels).
    Returns R [M, A] = sum_t E(theta_m, t) conj(E_a(t)), Pw [M] = sum_t |E(theta_m, t)|^2 (Eq. FBeq1's left
    side) and V [A] = sum_t |E_a(t)|^2 (the antenna autocorrelations v_aa)."""
    e = e.astype(np.complex128)
    e_tap = e_tap.astype(np.complex128)
    R = e_tap.T @ np.conj(e)
    Pw = np.sum(np.abs(e_tap) ** 2, axis=0)
    V = np.sum(np.abs(e) ** 2, axis=0)
    return R, Pw, V


def feedback_solve(R: np.ndarray, Pw: np.ndarray, V: np.ndarray, B: np.ndarray):
    """Feedback-calibration quantities per calibrator m and antenna i (Section 6), with g_i = B_i(theta_m):

    * S_i = < E(theta) g_i* E_i* >_t = conj(g_i) R_i (Eq. FBeq2's left side; its right side as printed,
      sum_j g_i g_j* v_ij, is conj(S_i): the reading kept here is the left side).  sum_i S_i = Pw.
    * X_i = sum over j, k both != i of g_j g_k* v_jk = Pw - S_i - conj(S_i) + |g_i|^2 v_ii: the sum of all
      visibilities not involving antenna i (Eq. FBeq3 subtracts only S_i; the exact exclusion also removes
      the column k = i and adds back the doubly removed v_ii term).
    * u_i = 1 + dg_i / g_i = 2 - N conj(S_i) / Pw: the gain update of the single-calibrator case with the
      factor N (not 2N, which would give dg_i = -g_i for a perfectly calibrated array; with N it vanishes
      there), applied as g_i -> u_i g_i, i.e. antenna i's kernel multiplied by u_i.
    R [M, A], Pw [M], V [A], B [M, A] -> (S, X, u), each complex128 [M, A]."""
    N = R.shape[1]
    S = np.conj(B) * R
    X = Pw[:, None] - S - np.conj(S) + (np.abs(B) ** 2) * V[None, :]
    u = 2.0 - N * np.conj(S) / Pw[:, None]
    return S, X, u


def relative_errors(gpu: np.ndarray, ora: np.ndarray) -> np.ndarray:
    """Per-product peak-normalised error of one channel's image [n_prod, n, n].

    XX, YY: max|gpu - ora| / max|ora|.  XY, YX: divided by sqrt(max XX * max YY) (Cauchy-Schwarz scale).
    """
    n_prod = ora.shape[0]
    err = np.abs(gpu - ora).reshape(n_prod, -1).max(axis=1)
    if n_prod == 1:
        return err / np.abs(ora[0]).max()
    sxx, syy = np.abs(ora[0]).max(), np.abs(ora[1]).max()
    scale = np.array([sxx, syy, math.sqrt(sxx * syy), math.sqrt(sxx * syy)])
    return err / scale
