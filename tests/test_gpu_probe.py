"""The issue-rate probes behind the measured ceilings (``moff_probe``): each kernel performs the work it reports.
The FMA probe's per-thread result is replayed in float32 on the host; the matrix-core probe's against the
16x16x32 product of its operands in the documented lane layout (A: lane l holds row l % 16, k = 8 (l / 16) + i;
B: lane l holds column l % 16, k = 8 (l / 16) + i; D: lane l holds rows 4 (l / 16) + i of column l % 16)."""
import numpy as np
import pytest
import torch

from paper_0812_3669_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(kind, blocks, iters):
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float32, device=DEV)
    print(f"probe kind={kind} blocks={blocks} iters={iters}", flush=True)
    flops = api.probe(kind, blocks, iters, out)
    torch.cuda.synchronize()
    return flops, out.cpu().numpy()


def test_fma_probe_matches_a_float32_replay():
    blocks, iters = 3, 37
    flops, got = _run(0, blocks, iters)
    assert flops == blocks * 256 * iters * 16
    tid = np.arange(256, dtype=np.int64)
    b = np.float32(0.5) + np.float32(1e-3) * (tid & 7).astype(np.float32)
    c = np.float32(1e-6) * (1 + (tid & 3)).astype(np.float32)
    bc = b.astype(np.float64) * c.astype(np.float64)              # exact product of two float32
    a = (tid[:, None] + np.arange(8)[None, :]).astype(np.float32)
    for _ in range(iters):
        a = (a.astype(np.float64) + bc[:, None]).astype(np.float32)
    s = np.zeros(256, dtype=np.float32)
    for k in range(8):
        s = s + a[:, k]
    want = np.tile(s, blocks)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)


def test_mfma_probe_matches_the_tile_product():
    blocks = 2
    flops1, got1 = _run(1, blocks, 1)
    flops3, got3 = _run(1, blocks, 3)
    assert flops1 == blocks * 4 * 1 * 4 * 16384 and flops3 == 3 * flops1
    lane = np.arange(64)
    x = np.array([[np.float16(np.float32(0.001) * np.float32((l + k) & 7)) for k in range(8)] for l in lane])
    y = np.array([[np.float16(np.float32(0.002) * np.float32((3 * l + k) & 7)) for k in range(8)] for l in lane])
    A = np.zeros((16, 32))
    B = np.zeros((32, 16))
    for l in lane:
        for i in range(8):
            A[l % 16, 8 * (l // 16) + i] = float(x[l, i])
            B[8 * (l // 16) + i, l % 16] = float(y[l, i])
    D = A @ B
    per_lane = np.array([4 * sum(D[4 * (l // 16) + i, l % 16] for i in range(4)) for l in lane])
    want1 = np.tile(per_lane, 4 * blocks)
    np.testing.assert_allclose(got1, want1, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(got3, 3 * want1, rtol=1e-5, atol=1e-9)


def _bitrev8(n):
    return int(f"{n:08b}"[::-1], 2)


@pytest.mark.parametrize("kind", [2, 3])
def test_exchange_probes_transform(kind):
    """Both exchange probes compute X[k] = (1/256) sum_n x[n] e^(+2 pi i n k / 256) (numpy's inverse FFT): kind 2 in
    natural order, kind 3 with position n holding X[bitrev8(n)]; one and two repeats (the second transforms the
    first's output as it lies in memory)."""
    blocks = 3
    rng = np.random.default_rng(kind)
    x = (rng.standard_normal((blocks * 16, 256)) + 1j * rng.standard_normal((blocks * 16, 256))).astype(np.complex64)
    perm = np.arange(256) if kind == 2 else np.array([_bitrev8(n) for n in range(256)])
    for iters in (1, 2):
        d = torch.from_numpy(x.ravel()).to(DEV)
        print(f"exchange probe kind={kind} blocks={blocks} iters={iters}", flush=True)
        flops = api.probe(kind, blocks, iters, d)
        torch.cuda.synchronize()
        assert flops == blocks * 16 * iters * 5 * 256 * 8
        want = x.astype(np.complex128)
        for _ in range(iters):
            want = np.fft.ifft(want, axis=1)[:, perm]
        got = d.cpu().numpy().reshape(blocks * 16, 256)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err < 1e-5, (kind, iters, err)


def test_xcd_ids():
    """Every workgroup reads an XCD number in [0, 8) and all eight XCDs appear; printed beside b % 8, the
    dispatcher's round-robin placement that the fused passes' channel-to-XCD mapping assumes."""
    blocks = 4096
    out = torch.full((blocks,), -1.0, dtype=torch.float32, device=DEV)
    api.probe(4, blocks, 1, out)
    torch.cuda.synchronize()
    x = out.cpu().numpy().astype(int)
    assert x.min() >= 0 and x.max() < 8 and len(set(x.tolist())) == 8
    same = float(np.mean(x == (np.arange(blocks) % 8)))
    print(f"XCD ids: counts {np.bincount(x, minlength=8).tolist()}, equal to b % 8 for {same:.3f} of workgroups")


def test_exchange_pattern_probes_move_what_they_report():
    """Kind 5 stores every element of 40 channel-samples of column-group tiles (a ragged second run of samples),
    each value naming its channel-sample and output block (u, q // 16); kind 6 reads them all back in the column
    pass's order, and each thread's sum over its run equals the closed form 16 (sum u + n_u (q // 16))."""
    ncs = 40
    buf = torch.full((ncs * 2 * 65536,), complex(-1.0, -1.0), dtype=torch.complex64, device=DEV)
    print(f"exchange pattern probes ncs={ncs}", flush=True)
    assert api.probe(5, ncs, 1, buf) == ncs * 2 * 65536 * 8
    torch.cuda.synchronize()
    h = buf.cpu().numpy().reshape(ncs, 2, 32, 256, 8)
    u = np.arange(ncs)[:, None, None, None, None]
    q = (np.arange(32)[:, None, None] * 8 + np.arange(8)[None, None, :])[None, None]
    assert np.array_equal(h.real, np.broadcast_to(u, h.shape).astype(np.float32))
    assert np.array_equal(h.imag, np.broadcast_to(q // 16, h.shape).astype(np.float32))
    assert api.probe(6, ncs, 1, buf) == ncs * 2 * 65536 * 8
    torch.cuda.synchronize()
    g = buf.cpu().numpy().reshape(ncs, 2, 32, 256, 8)
    expect = 16 * (np.arange(ncs).sum() + ncs * (q[0, 0, :, 0, :] // 16))      # [tile, col]
    for p in range(2):
        for j in range(16):
            assert np.array_equal(g[ncs - 1, p, :, j + 240, :].real, expect.astype(np.float32)), (p, j)
    # everything else is what kind 5 wrote
    g[ncs - 1, :, :, 240:, :] = h[ncs - 1, :, :, 240:, :]
    assert np.array_equal(g, h)
