"""Gradient sums over more entries than the gradient steps address with buffer
loads (2^29 entries, byte offsets below 2^31): such a call reads its entries
with global loads instead.  A 256 x 256 frame with every one of 8193 bins
active (65536 x 8193 > 2^29 entries) is checked on sampled pixels against the
same pixels in a small call (buffer loads; the same summation order, so the
sums agree bit for bit) and against the oracle's gradients (Methods, the
Poisson likelihood of the observation model)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_06700_amd import rt3d, synth
from gpu_util import oracle_to_device, to_dev_u32

pytestmark = pytest.mark.gpu

T = 8193
ROWS = COLS = 256
BUF_ENTRIES = 1 << 29


def _counts():
    """Counts of the 8193 bins (every bin active), the same in every pixel."""
    b = np.arange(T)
    return 1 + (b * 7919 % 5)


def _state(P, seed):
    rng = np.random.default_rng(seed)
    s = oracle.State(1, 1, P, 4)
    s.cnt[:] = rng.integers(1, 3, P)
    s.t[:, 0] = rng.uniform(50.0, T - 60.0, P)
    s.t[:, 1] = np.minimum(s.t[:, 0] + rng.uniform(200.0, 900.0, P), T - 1.0)
    s.r[:, :2] = rng.uniform(5.0, 60.0, (P, 2))
    s.t[s.cnt < 2, 1] = 0.0
    s.r[s.cnt < 2, 1] = 0.0
    s.b[:] = rng.uniform(0.5, 2.0, P)
    return s


def test_gradients_past_buffer_range():
    irf = synth.exgauss_irf(1.2, 3.0, -6, 40)
    P = ROWS * COLS
    assert P * T > BUF_ENTRIES
    print(f"[big-entries] {ROWS}x{COLS}x{T}, {P * T} entries", flush=True)
    ctx = rt3d.Context(irf.probs, T, r_init=1, lanes_per_pixel=4)   # the same lanes at both sizes
    cnt = _counts()
    row = torch.from_numpy(((np.arange(T, dtype=np.int64) << 16) | cnt).astype(np.uint32).view(np.int32)).cuda()
    ent = row.repeat(P)
    off = torch.arange(0, P + 1, dtype=torch.int64, device="cuda").mul_(T).to(torch.int32)
    s = _state(P, 11)
    s.rows, s.cols = ROWS, COLS
    dgt, dgr, dgb = ctx.gradients(oracle_to_device(s), off, ent)
    torch.cuda.synchronize()
    del ent
    pick = np.array([0, 1, 4097, 33333, P - 2, P - 1])
    dgt = dgt.cpu().numpy()[:, pick]
    dgr = dgr.cpu().numpy()[:, pick]
    dgb = dgb.cpu().numpy()[pick]

    # the same pixels alone: buffer loads, the same sums
    n = len(pick)
    sm = oracle.State(1, 1, n, 4)
    for a in ("t", "r", "cnt", "b"):
        getattr(sm, a)[:] = getattr(s, a)[pick]
    off_o = (np.arange(n + 1, dtype=np.int64) * T).astype(np.uint32)
    ent_o = np.tile(((np.arange(T, dtype=np.int64) << 16) | cnt).astype(np.uint32), n)
    sgt, sgr, sgb = ctx.gradients(oracle_to_device(sm), to_dev_u32(off_o), to_dev_u32(ent_o))
    np.testing.assert_array_equal(dgt, sgt.cpu().numpy())
    np.testing.assert_array_equal(dgr, sgr.cpu().numpy())
    np.testing.assert_array_equal(dgb, sgb.cpu().numpy())

    # and the oracle
    O = oracle.Oracle(oracle.Model(irf.probs, T), oracle.Params(r_init=1))
    (gt, gr, gb), (at, ar, ab) = O.grad(off_o, ent_o, sm)
    live = np.arange(4)[None, :] < sm.cnt[:, None]
    for g_gpu, g_or, a in ((dgt[:4].T.astype(np.float64), gt, at), (dgr[:4].T.astype(np.float64), gr, ar)):
        err = np.abs(g_gpu - g_or)[live]
        assert np.all(err <= 1e-4 * a[live] + 1e-30), (err.max(), (err / a[live]).max())
    assert np.all(np.abs(dgb - gb) <= 1e-4 * ab + 1e-30)
