"""GPU parity and gain of the learned depth denoiser, through the C ABI.

Forward: the FP16-MFMA network against the FP64 oracle with the same FP16
rounding points (features, weights, each layer's stored output), element by
element within 2e-3 of the output scale.  Training: each weight gradient
element of one step within 1e-2 of its layer's largest against the oracle's
backward pass, and the Adam update against the oracle's Adam.  In the loop:
one iteration with the network as the depth denoiser (APSS for pixels with
four points) against the oracle's iteration with the same network, and a
short reconstruction.  Gain: a network trained on the GPU by
the library's own kernels, on depth-block inputs recorded from plain-APSS
runs of multi-layer scenes, reconstructs held-out scenes with a lower depth
error than the method with no depth denoiser.
"""
import numpy as np
import pytest

from gpu_util import device_to_oracle, oracle_to_device, to_dev_hist, to_dev_u32, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from oracle import cnn  # noqa: E402
from paper_1905_06700_amd import rt3d, synth, train  # noqa: E402

ROWS, COLS, T = 40, 72, 1024      # two 64-pixel tiles per row, the second ragged


def params(sc, **kw):
    m = sc.meta
    p = dict(dz=m["dz"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
    p.update(kw)
    return p


_cache = {}


def setup():
    if "s" not in _cache:
        sc = synth.layers_scene(3, rows=ROWS, cols=COLS, T=T)
        O = oracle.Oracle(oracle.Model(sc.irf.probs, T), oracle.Params(**params(sc)))
        off, ent = oracle.compact(sc.Z[None])
        s = O.init(off, ent, oracle.State(1, ROWS, COLS, 4))
        for _ in range(2):
            O.iterate(off, ent, s)
        O.depth_step(off, ent, s)
        ctx = rt3d.Context(sc.irf.probs, T, denoiser=rt3d.DENOISE_CNN, **params(sc))
        ctx.workspace(1, ROWS, COLS, ROWS * COLS * 200)
        _cache.update(sc=sc, O=O, s=s, ctx=ctx, sig=float(np.sqrt(O.m.sigma2)))
    return _cache


def weights(seed):
    w = cnn.he_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    w += rng.normal(0, 0.02, w.shape)
    return w.astype(np.float32)


def test_cnn_forward_matches_oracle():
    c = setup()
    s, ctx = c["s"], c["ctx"]
    w = weights(1)
    ctx.cnn_set_weights(w)
    np.testing.assert_array_equal(ctx.cnn_get_weights(), w)
    y = ctx.cnn_forward(oracle_to_device(s)).cpu().numpy()           # [3, P]
    x = cnn.features(s.t, s.r, s.cnt, c["sig"], 1, ROWS, COLS)
    yo, _ = cnn.forward(x, w.astype(np.float64), fp16=True)
    yo = yo.reshape(-1, 3).T
    scale = max(1.0, np.abs(yo).max())
    err = np.abs(y - yo).max()
    print(f"[gpu-cnn] forward max |gpu - oracle| = {err:.3e} (output scale {scale:.2f})", flush=True)
    assert err <= 2e-3 * scale


def test_cnn_train_step_gradient_and_adam_match_oracle():
    c = setup()
    s, ctx, sc = c["s"], c["ctx"], c["sc"]
    w = weights(2)
    ctx.cnn_set_weights(w)
    truth = sc.depth.reshape(3, -1).astype(np.float32)
    loss = ctx.cnn_train_step(oracle_to_device(s), torch.from_numpy(truth).cuda(), lr=1e-3)
    torch.cuda.synchronize()
    g = ctx.cnn_last_gradient().astype(np.float64)
    x = cnn.features(s.t, s.r, s.cnt, c["sig"], 1, ROWS, COLS)
    tgt, msk = cnn.targets(s.t, s.cnt, truth.astype(np.float64), c["sig"])
    lo, go = cnn.loss_and_grad(x, w.astype(np.float64), tgt.reshape(1, ROWS, COLS, 3),
                               msk.reshape(1, ROWS, COLS, 3), fp16=True)
    lg = loss.cpu().numpy()
    assert int(lg[1]) == int(msk.sum())
    assert abs(lg[0] - lo) <= 1e-2 * lo
    at = 0
    for li, (ci, co) in enumerate(zip(cnn.CIN, cnn.COUT)):
        n = 9 * ci * co + co
        a, b = g[at:at + n], go[at:at + n]
        rel = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
        print(f"[gpu-cnn] layer {li} weight-gradient max element error {rel:.2e} of the layer's largest",
              flush=True)
        assert rel <= 1e-2
        at += n
    w1, _, _ = cnn.adam(w.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    np.testing.assert_allclose(ctx.cnn_get_weights(), w1, rtol=1e-5, atol=1e-6)


_loop = {}


def loop_setup():
    """A multi-layer scene (four peaks sought, so some pixels hold four points)
    after the initialisation and two plain iterations, and a CNN context."""
    if "s" not in _loop:
        sc = synth.layers_scene(4, rows=ROWS, cols=COLS, T=T, signal=6.0, sbr=0.2)
        prm = params(sc)
        O = oracle.Oracle(oracle.Model(sc.irf.probs, T), oracle.Params(**prm))
        off, ent = oracle.compact(sc.Z[None])
        s = O.init(off, ent, oracle.State(1, ROWS, COLS, 4))
        for _ in range(2):
            O.iterate(off, ent, s)
        ctx = rt3d.Context(sc.irf.probs, T, denoiser=rt3d.DENOISE_CNN, **prm)
        ctx.workspace(1, ROWS, COLS, ROWS * COLS * 200)
        _loop.update(sc=sc, O=O, s=s, off=off, ent=ent, ctx=ctx, sig=float(np.sqrt(O.m.sigma2)), prm=prm)
    return _loop


def _net_scale(O, s, off, ent, w, sig):
    """Largest |network output| on the state the depth block hands the network."""
    s1 = O.depth_step(off, ent, s.copy())
    x = cnn.features(s1.t, s1.r, s1.cnt, sig, 1, ROWS, COLS)
    yo, _ = cnn.forward(x, w, fp16=True)
    return max(1.0, float(np.abs(yo).max()))


def test_cnn_iteration_matches_oracle():
    """One whole iteration with the learned denoiser in the depth block: the
    depth step, APSS for pixels with four points, the network's move of the
    other pixels' slots, then merge, intensity step, intensity low-pass and
    background steps, against the oracle's iteration with the same network
    from the same state.  Bars derived from the steps': counts equal on
    >= 99.9% of pixels; depths within 2e-4 bin (the depth step's bar) plus
    sigma_h x 2e-3 x the output scale (the forward bar, moved by sigma_h)."""
    c = loop_setup()
    O, s, ctx, sig = c["O"], c["s"], c["ctx"], c["sig"]
    w = weights(4)
    ctx.cnn_set_weights(w)
    w64 = w.astype(np.float64)
    assert (s.cnt == 4).sum() > 0 and (s.cnt == 2).sum() > 0
    so = O.iterate_cnn(c["off"], c["ent"], s.copy(), w64)
    sg = device_to_oracle(ctx.step(rt3d.STEP_ITERATION, oracle_to_device(s), to_dev_u32(c["off"]),
                                   to_dev_u32(c["ent"])), 4)
    scale = _net_scale(O, s, c["off"], c["ent"], w64, sig)
    same = sg.cnt == so.cnt
    lv = (np.arange(4)[None, :] < so.cnt[:, None]) & same[:, None]
    dt = np.abs(sg.t - so.t)[lv].max()
    dr = (np.abs(sg.r - so.r) / np.maximum(so.r, 1e-6))[lv].max()
    bar = 2e-4 + sig * 2e-3 * scale
    print(f"[gpu-cnn] iteration: count agreement {same.mean():.5f}, max depth err {dt:.2e} bins (bar {bar:.2e}), "
          f"max intensity err {dr:.2e} relative, four-point pixels {(s.cnt == 4).sum()}", flush=True)
    assert same.mean() >= 0.999
    assert dt <= bar
    # background: the step's bar (1e-5 relative) plus twice the oracle's own
    # response to FP16 rounding in the network, away from the filter's reach
    # of a pixel whose point count differs
    resp = _bg_rounding_response(O, s, c["off"], c["ent"], w64)
    reach = _reach((~same).reshape(ROWS, COLS)).reshape(-1)
    assert (~reach).mean() > 0.8
    rel = np.abs(sg.b - so.b) / np.maximum(so.b, 1e-12)
    print(f"[gpu-cnn] background: max relative err {rel[~reach].max():.2e} (bar {1e-5 + resp:.2e})", flush=True)
    assert rel[~reach].max() <= 1e-5 + resp


def _reach(bad, radius=8):
    """Pixels within the background filter's reach (ceil(4 sigma_b) = 8) of a flagged pixel (circular)."""
    reach = np.zeros_like(bad)
    for di in range(-radius, radius + 1):
        for dj in range(-radius, radius + 1):
            reach |= np.roll(np.roll(bad, di, 0), dj, 1)
    return reach


def _bg_rounding_response(O, s, off, ent, w):
    """Twice the largest relative difference of the oracle's end-of-iteration
    background between the network with FP16 storage points and the same
    network in FP64, away from the reach of pixels whose point count the two
    give differently.  The background step reads the depths the network
    moved, so output rounding in the network reaches the background; the
    GPU's network rounds (in another order) at the same points."""
    a = O.iterate_cnn(off, ent, s.copy(), w, fp16=True)
    b = O.iterate_cnn(off, ent, s.copy(), w, fp16=False)
    far = ~_reach((a.cnt != b.cnt).reshape(ROWS, COLS)).reshape(-1)
    return 2.0 * float((np.abs(a.b - b.b) / np.maximum(b.b, 1e-12))[far].max())


def test_cnn_reconstruction_matches_oracle():
    """A short reconstruction (initialisation and three iterations) with the
    learned denoiser against the oracle's.  Each iteration adds at most the
    one-iteration bar, so depths stay within three times it."""
    c = loop_setup()
    O, ctx, sig, sc = c["O"], c["ctx"], c["sig"], c["sc"]
    w = weights(5)
    w64 = w.astype(np.float64)
    prm = dict(c["prm"], n_iter=3)
    O3 = oracle.Oracle(O.m, oracle.Params(**prm))
    so = O3.reconstruct_cnn(c["off"], c["ent"], oracle.State(1, ROWS, COLS, 4), w64)
    net = rt3d.Context(sc.irf.probs, T, denoiser=rt3d.DENOISE_CNN, **prm)
    net.cnn_set_weights(w)
    res = net.reconstruct(to_dev_hist(sc.Z)[None], max_entries=ROWS * COLS * 200)
    assert net.query().device_error == 0
    pt = u32(res.pt_off).astype(np.int64)
    cnt = np.diff(pt)
    same = cnt == so.cnt
    depth = res.depth.cpu().numpy()
    errs = [np.abs(depth[pt[p]:pt[p] + so.cnt[p]] - so.t[p, :so.cnt[p]]).max()
            for p in np.nonzero(same & (so.cnt > 0))[0]]
    s0 = O3.init(c["off"], c["ent"], oracle.State(1, ROWS, COLS, 4))
    bar = 3 * (2e-4 + sig * 2e-3 * _net_scale(O3, s0, c["off"], c["ent"], w64, sig))
    print(f"[gpu-cnn] reconstruction (3 iterations): count agreement {same.mean():.5f}, "
          f"max depth err {max(errs):.2e} bins (bar {bar:.2e})", flush=True)
    assert same.mean() >= 0.999
    assert max(errs) <= bar


def _scores(scenes, res, sig, R, C):
    """Depth error over true surfaces (each matched to the nearest estimated
    point of its pixel, capped at 3 sigma_h): (RMSE over the surfaces found
    within the cap, fraction found)."""
    pt = u32(res.pt_off).astype(np.int64)
    depth = res.depth.cpu().numpy()
    P1 = R * C
    errs = []
    for f, sc in enumerate(scenes):
        truth = sc.depth.reshape(sc.depth.shape[0], -1)
        for p in range(P1):
            est = depth[pt[f * P1 + p]:pt[f * P1 + p + 1]]
            for sfc in range(truth.shape[0]):
                d = truth[sfc, p]
                if np.isfinite(d):
                    errs.append(np.abs(est - d).min() if est.size else np.inf)
    e = np.asarray(errs)
    found = e < 3 * sig
    return float(np.sqrt(np.mean(e[found] ** 2))), float(found.mean())


def test_trained_network_beats_no_denoiser():
    """Train on the GPU (the library's own kernels) by the training recipe --
    depth-block inputs recorded at iterations 1, 2, 5, 10 and 20 of plain-APSS
    runs of multi-layer scenes (6 signal photons per pixel, SBR 0.2), random
    crops -- then reconstruct held-out scenes: the network's depth error over
    the surfaces found is lower than with no depth denoiser, at the same
    detection rate."""
    R, C_, T_, n_scenes = 96, 96, 1024, 24
    sc0 = synth.layers_scene(0, rows=8, cols=8, T=T_)
    p = params(sc0)
    apss = rt3d.Context(sc0.irf.probs, T_, **p)
    net = rt3d.Context(sc0.irf.probs, T_, denoiser=rt3d.DENOISE_CNN, **p)
    none = rt3d.Context(sc0.irf.probs, T_, denoiser=rt3d.DENOISE_NONE, **p)
    lists = (train.scene_lists((s, R, C_, T_, 6.0, 0.2)) for s in range(n_scenes))
    hist = train.train_recipe(net, apss, lists, n_scenes, steps=600, rows=R, cols=C_, frames_per_batch=8,
                              crop=64, batch=16, seed=7, log=lambda m: print("[gpu-cnn]", m, flush=True))
    test = [synth.layers_scene(100 + s, rows=R, cols=C_, T=T_, signal=6.0, sbr=0.2) for s in range(2)]
    sig = float(np.sqrt(net.sigma2))
    Zt = torch.cat([to_dev_hist(s.Z)[None] for s in test])
    r = {}
    for name, ctx in (("apss", apss), ("cnn", net), ("none", none)):
        ctx.workspace(2, R, C_, 2 * R * C_ * 200)
        res = ctx.make_output(2 * R * C_)
        ctx.reconstruct_into(res, 2, R, C_, hist=Zt)
        r[name] = _scores(test, res, sig, R, C_)
    print(f"[gpu-cnn] held-out (RMSE over found surfaces, found fraction): {r}; training loss {hist}", flush=True)
    assert r["cnn"][0] < 0.95 * r["none"][0]
    assert r["cnn"][1] >= r["none"][1] - 0.02


@pytest.mark.parametrize("regime", ["config4", "bright"])
def test_trained_checkpoint_within_ten_percent_of_apss(regime):
    """The committed checkpoints of the training recipe (trained on the GPU by
    the library's kernels on scenes of seeds 0..1999) against plain APSS on
    held-out scenes (seeds 10000..10003) of their regime: depth RMSE (true
    surfaces matched greedily within 3 sigma_h, a miss counted 3 sigma_h) within
    10% of APSS's, at the same fraction of surfaces found.  config4: 2 signal
    photons/px at SBR 0.05 (about a third of the surfaces found); bright: 6
    photons/px at SBR 0.2 (about 90% found)."""
    import os
    from paper_1905_06700_amd import train as tr
    sig_ph, sbr, name = (2.0, 0.05, "denoiser_c4") if regime == "config4" else (6.0, 0.2, "denoiser_bright")
    path = os.path.join(os.path.dirname(tr.__file__), "weights", name + ".rt3dcnn")
    R = C_ = 256
    T_ = 1024
    test = [synth.layers_scene(10000 + s, rows=R, cols=C_, T=T_, signal=sig_ph, sbr=sbr) for s in range(4)]
    p = params(test[0])
    apss = rt3d.Context(test[0].irf.probs, T_, **p)
    net = rt3d.Context(test[0].irf.probs, T_, denoiser=rt3d.DENOISE_CNN, **p)
    net.denoiser_load(path)
    sig = float(np.sqrt(net.sigma2))
    Z = torch.cat([to_dev_hist(s.Z)[None] for s in test])
    r = {}
    for nm, ctx in (("apss", apss), ("cnn", net)):
        ctx.workspace(4, R, C_, 4 * R * C_ * 200)
        res = ctx.make_output(4 * R * C_)
        ctx.reconstruct_into(res, 4, R, C_, hist=Z)
        assert ctx.query().device_error == 0
        pt = u32(res.pt_off).astype(np.int64)
        dep = res.depth.cpu().numpy()
        errs, nts, nfs = [], [], []
        for f, sc in enumerate(test):
            sl = pt[f * R * C_:(f + 1) * R * C_ + 1] - pt[f * R * C_]
            e, nt, nf = tr.match_surfaces(sc.depth.reshape(3, -1), sl, dep[pt[f * R * C_]:], 3 * sig)
            errs.append(e)
            nts.append(nt)
            nfs.append(nf)
        r[nm] = tr.depth_scores(errs, nts, nfs, 4 * R * C_, 3 * sig)
    print(f"[gpu-cnn] {regime} held-out: {r}", flush=True)
    assert r["cnn"]["depth_rmse_bins"] <= 1.10 * r["apss"]["depth_rmse_bins"]
    assert r["cnn"]["found"] >= r["apss"]["found"] - 0.01
