"""Pins of the learned-denoiser oracle (oracle/cnn.py).

The convolution is pinned to torch's conv2d in float64 (a library routine
with a different formulation: NCHW, OIHW), the backward pass to central
finite differences of the loss, Adam to torch.optim.Adam, and the features
and target matching to hand-built cases.
"""
import numpy as np
import pytest
import torch

from oracle import cnn


def test_conv3x3_equals_torch_conv2d():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 7, 4))
    W = rng.normal(size=(3, 3, 4, 6))
    b = rng.normal(size=6)
    y = cnn.conv3x3(x, W, b)
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    wt = torch.from_numpy(W).permute(3, 2, 0, 1)          # [cout, cin, ky, kx]
    yt = torch.nn.functional.conv2d(xt, wt, torch.from_numpy(b), padding=1).permute(0, 2, 3, 1)
    np.testing.assert_allclose(y, yt.numpy(), rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    F, H, W = 1, 5, 6
    x = rng.normal(size=(F, H, W, 16))
    w = cnn.he_init(3).astype(np.float64)
    w += rng.normal(0, 0.05, w.shape)                     # non-zero biases, padding weights
    target = rng.normal(size=(F, H, W, 3))
    mask = rng.random((F, H, W, 3)) < 0.6
    loss, g = cnn.loss_and_grad(x, w, target, mask)
    idx = rng.choice(len(w), 60, replace=False)
    eps = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (cnn.loss_and_grad(x, wp, target, mask)[0] - cnn.loss_and_grad(x, wm, target, mask)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_adam_equals_torch():
    rng = np.random.default_rng(2)
    w0 = rng.normal(size=50)
    wt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        opt.zero_grad()
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = cnn.adam(w, g, m, v, step, 1e-2)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_hand_cases():
    F, H, W, K = 1, 3, 3, 4
    t = np.zeros((9, K))
    r = np.zeros((9, K))
    cnt = np.ones(9, dtype=int)
    t[:, 0] = 100.0
    r[:, 0] = np.e - 1.0
    t[4, 0] = 104.0                                   # centre sits 4 bins deeper
    x = cnn.features(t, r, cnt, 2.0, F, H, W)        # gate = 3 x 2 = 6 bins
    assert x.shape == (1, 3, 3, 16)
    # the 5 x 5 window of any pixel of a 3 x 3 image holds all nine pixels, all
    # within the gate of each other: mean 904 / 9
    np.testing.assert_allclose(x[0, 1, 1, 0], (104.0 - 904.0 / 9) / 2.0)
    np.testing.assert_allclose(x[0, 0, 0, 0], (100.0 - 904.0 / 9) / 2.0)
    np.testing.assert_allclose(x[..., 1], 1.0)
    np.testing.assert_allclose(x[..., 2], 1.0)
    np.testing.assert_allclose(x[..., 3], 9.0 / 25.0)
    assert np.all(x[..., 4:] == 0)
    # a centre 10 bins deeper is outside every neighbour's gate: alone on its surface
    t[4, 0] = 110.0
    x = cnn.features(t, r, cnt, 2.0, F, H, W)
    assert x[0, 1, 1, 0] == 0.0 and x[0, 1, 1, 3] == 1.0 / 25.0
    np.testing.assert_allclose(x[0, 0, 0, 0], 0.0)
    np.testing.assert_allclose(x[0, 0, 0, 3], 8.0 / 25.0)
    # a second point of a pixel joins the neighbours of the slot whose gate it
    # falls in, whatever its own slot; a four-point pixel feeds its first three slots
    cnt[0] = 4
    t[0, :] = [95.0, 101.0, 200.0, 300.0]
    r[0, :] = np.e - 1.0
    x = cnn.features(t, r, cnt, 2.0, F, H, W)
    # pixel (0, 1), slot 0 at 100: neighbours 95 and 101 of pixel 0 and the six
    # other 100s (the centre at 110 is out): 9 points, mean (95 + 101 + 700) / 9
    np.testing.assert_allclose(x[0, 0, 1, 0], (100.0 - 896.0 / 9) / 2.0)
    np.testing.assert_allclose(x[0, 0, 1, 3], 9.0 / 25.0)
    assert x[0, 0, 0, 6] == 1.0 and x[0, 0, 0, 10] == 1.0
    assert x[0, 0, 0, 8] == 0.0 and x[0, 0, 0, 11] == 1.0 / 25.0   # slot 2 at 200 is alone
    assert np.all(x[0, 0, 0, 12:] == 0)


def test_target_matching():
    t = np.array([[10.0, 50.0, 0, 0], [5.0, 0, 0, 0]])
    cnt = np.array([2, 1])
    truth = np.array([[11.0, np.nan], [48.0, 30.0]])      # [S, P]
    tgt, msk = cnn.targets(t, cnt, truth, sigma_h=1.0)
    assert msk.tolist() == [[True, True, False], [False, False, False]]
    np.testing.assert_allclose(tgt[0, :2], [1.0, -2.0])


def test_training_reduces_loss_on_a_toy():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(1, 8, 8, 16))
    x[..., cnn.LIVE_IN:] = 0
    target = np.tanh(x[..., :3])
    mask = np.ones_like(target, dtype=bool)
    w = cnn.he_init(0).astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    l0, _ = cnn.loss_and_grad(x, w, target, mask)
    for step in range(1, 41):
        loss, g = cnn.loss_and_grad(x, w, target, mask)
        w, m, v = cnn.adam(w, g, m, v, step, 3e-3)
    assert loss < 0.5 * l0


# ---------------------------------------------------------------- the network inside the loop

def _loop_case(k_init):
    import oracle
    from paper_1905_06700_amd import synth
    sc = synth.layers_scene(5, rows=20, cols=22, T=1024, signal=6.0, sbr=0.2)
    prm = dict(dz=sc.meta["dz"], r_min=sc.meta["r_min"], r_init=1, k_init=k_init)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**prm))
    off, ent = oracle.compact(sc.Z[None])
    s = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    O.iterate(off, ent, s)
    return sc, prm, O, off, ent, s


def test_zero_network_iteration_is_the_plain_iteration_without_denoiser():
    """With every weight zero the network moves nothing; when no pixel holds
    four points (three peaks sought) no APSS runs either, so an iteration with
    the learned denoiser equals the loop's iteration with no depth denoiser,
    bit for bit."""
    import oracle
    sc, prm, O, off, ent, s = _loop_case(3)
    assert s.cnt.max() <= 3 and (s.cnt > 0).mean() > 0.5
    a = O.iterate_cnn(off, ent, s.copy(), np.zeros(cnn.N_PARAMS))
    plain = oracle.Oracle(O.m, oracle.Params(**prm, use_apss=0))
    b = plain.iterate(off, ent, s.copy())
    for name in ("t", "r", "n", "cnt", "b"):
        np.testing.assert_array_equal(getattr(a, name), getattr(b, name), err_msg=name)


def test_four_point_pixels_take_apss_and_others_stay_under_a_zero_network():
    """Pixels with four points (more than the network's slots) take exactly
    the APSS result, which reads the whole pre-denoiser state; the others keep
    depth and normals when the network outputs zero."""
    sc, prm, O, off, ent, s = _loop_case(3)
    s = s.copy()
    rng = np.random.default_rng(3)
    pick = np.nonzero(s.cnt >= 1)[0][::7][:20]          # points added 60-80 bins behind the last
    assert pick.size == 20
    for q in pick:
        c = s.cnt[q]
        while c < 4:
            s.t[q, c] = s.t[q, c - 1] + 60.0 + rng.uniform(0, 20)
            s.r[q, c] = 1.0
            s.n[q, c] = (0.0, 0.0, -1.0)
            c += 1
        s.cnt[q] = 4
    ref = O.apss(s.copy())
    out = O.cnn_denoise(s.copy(), np.zeros(cnn.N_PARAMS))
    four = s.cnt == 4
    assert four.sum() >= 20
    np.testing.assert_array_equal(out.t[four], ref.t[four])
    np.testing.assert_array_equal(out.n[four], ref.n[four])
    np.testing.assert_array_equal(out.t[~four], s.t[~four])
    np.testing.assert_array_equal(out.n[~four], s.n[~four])
    assert np.any(ref.t[four] != s.t[four])             # APSS did move them


def test_bias_only_network_moves_each_slot_by_sigma_h_times_its_output():
    """A network whose only non-zero parameters are the last layer's biases
    outputs those biases everywhere (every hidden activation is ReLU(0) = 0):
    slot k < cnt of a pixel with at most three points moves by sigma_h c_k,
    clamped to [0, T - 1]; slots past the count stay.  c = (0.25, -0.5, 60)
    (exact in FP16) sends every third slot past the last bin."""
    sc, prm, O, off, ent, s = _loop_case(3)
    w = np.zeros(cnn.N_PARAMS)
    c = np.array([0.25, -0.5, 60.0])
    w[-3:] = c
    sig = float(np.sqrt(O.m.sigma2))
    out = O.cnn_denoise(s.copy(), w)
    T = O.m.T
    for k in range(4):
        mv = (s.cnt > k) & (s.cnt <= 3) & (k < 3)
        want = np.clip(s.t[mv, k] + sig * c[k], 0, T - 1) if k < 3 else s.t[mv, k]
        np.testing.assert_allclose(out.t[mv, k], want, rtol=0, atol=1e-12)
        np.testing.assert_array_equal(out.t[~mv, k], s.t[~mv, k])
    assert np.all(out.t[(s.cnt > 2), 2] == T - 1)
    np.testing.assert_array_equal(out.n, s.n)
