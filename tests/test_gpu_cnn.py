"""GPU parity and gain of the learned depth denoiser, through the C ABI.

Forward: the FP16-MFMA network against the FP64 oracle with the same FP16
rounding points (features, weights, each layer's stored output).  Training:
the weight gradient of one step against the oracle's backward pass, and the
Adam update against the oracle's Adam.  Gain: a network trained on the GPU by
the library's own kernels, on depth-block inputs recorded from plain-APSS
runs of multi-layer scenes, reconstructs held-out scenes with a lower depth
error than the method with no depth denoiser.
"""
import numpy as np
import pytest

from gpu_util import oracle_to_device, to_dev_hist, to_dev_u32, u32

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
    assert err <= 2e-2 * scale


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
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"[gpu-cnn] layer {li} weight-gradient relative error {rel:.2e}", flush=True)
        assert rel <= 2e-2
        at += n
    w1, _, _ = cnn.adam(w.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    np.testing.assert_allclose(ctx.cnn_get_weights(), w1, rtol=1e-5, atol=1e-6)


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
    """Train on the GPU (the library's own kernels) on depth-block inputs
    recorded from plain-APSS runs of multi-layer scenes (6 signal photons per
    pixel, SBR 0.2), then reconstruct held-out scenes: the network's depth
    error over the surfaces found is lower than with no depth denoiser, at the
    same detection rate."""
    R, C_, F, T_ = 96, 96, 6, 1024
    trn = [synth.layers_scene(s, rows=R, cols=C_, T=T_, signal=6.0, sbr=0.2) for s in range(F)]
    p = params(trn[0])
    apss = rt3d.Context(trn[0].irf.probs, T_, **p)
    net = rt3d.Context(trn[0].irf.probs, T_, denoiser=rt3d.DENOISE_CNN, **p)
    none = rt3d.Context(trn[0].irf.probs, T_, denoiser=rt3d.DENOISE_NONE, **p)
    Z = torch.cat([to_dev_hist(s.Z)[None] for s in trn])
    recorded = train.record_depth_inputs(apss, Z, iters=(0, 1, 2, 4, 7, 11), n_iter=12)
    truth = torch.from_numpy(np.concatenate([s.depth.reshape(3, -1) for s in trn], axis=1)
                             .astype(np.float32)).cuda()
    net.workspace(F, R, C_, F * R * C_ * 200)
    hist = train.train(net, [(recorded, truth)], steps=600, lr=2e-3, seed=7, log_every=100,
                       log=lambda m: print("[gpu-cnn]", m, flush=True))
    del recorded
    test = [synth.layers_scene(100 + s, rows=R, cols=C_, T=T_, signal=6.0, sbr=0.2) for s in range(2)]
    sig = float(np.sqrt(net.sigma2))
    Zt = torch.cat([to_dev_hist(s.Z)[None] for s in test])
    r = {}
    for name, ctx in (("apss", apss), ("cnn", net), ("none", none)):
        ctx.workspace(2, R, C_, 2 * R * C_ * 200)
        res = ctx.make_output(2 * R * C_)
        ctx.reconstruct_into(res, 2, R, C_, hist=Zt)
        r[name] = _scores(test, res, sig, R, C_)
    print(f"[gpu-cnn] held-out (matched RMSE bins, found fraction): {r}; training loss {hist}", flush=True)
    assert r["cnn"][0] < 0.95 * r["none"][0]
    assert r["cnn"][1] >= r["none"][1] - 0.02
