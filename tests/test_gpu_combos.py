"""Combinations of the observation-model options, through the C ABI: graph
replay with per-pixel IRF classes (the class lists are built inside the
recorded call), super-resolution with the pinhole camera, IRF classes with
the pinhole camera (both against the oracle with the same options), and a
warm start under super-resolution (against the oracle iterating from the
state the previous call left)."""
import numpy as np
import pytest

from gpu_util import intensity_err, params_for, to_dev_hist, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402


def compare(res, so, rows, cols, name):
    pt = u32(res.pt_off).astype(np.int64)
    cnt = np.diff(pt)
    same = cnt == so.cnt
    bad = (~same).reshape(-1, rows, cols)
    nb = np.zeros_like(bad)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            nb |= np.roll(np.roll(bad, di, 1), dj, 2)
    depth = res.depth.cpu().numpy()
    good = np.nonzero(~nb.reshape(-1) & (so.cnt > 0))[0]
    errs = [np.abs(depth[pt[p]:pt[p] + so.cnt[p]] - so.t[p, :so.cnt[p]]).max() for p in good]
    ierr = intensity_err(res.intensity, pt, so, good)
    print(f"[gpu-combos] {name}: count agreement {same.mean():.5f}, max depth err {max(errs):.2e} bins, "
          f"max intensity err {ierr:.2e} relative", flush=True)
    assert same.mean() >= 0.999
    assert len(errs) >= 0.9 * (so.cnt > 0).sum() and max(errs) <= 1e-3
    assert ierr <= 2e-5


def test_graph_replay_with_irf_classes():
    sc, irfs, cls = synth.irf_class_scene(1, rows=19, cols=26)
    ctx = rt3d.Context(irfs[0].probs, sc.T, **params_for(sc))
    for i in irfs[1:]:
        ctx.add_irf(i.probs)
    P = sc.rows * sc.cols
    Z = to_dev_hist(sc.Z)[None]
    c = torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda()
    ctx.workspace(1, sc.rows, sc.cols, P * 64)
    direct = ctx.make_output(P)
    ctx.reconstruct_into(direct, 1, sc.rows, sc.cols, hist=Z, irf_class=c)
    replayed = ctx.make_output(P)
    print("[gpu-combos] graph with IRF classes", flush=True)
    g = ctx.graph(replayed, 1, sc.rows, sc.cols, hist=Z, irf_class=c)
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
        assert ctx.query().device_error == 0
        n = int(direct.pt_off[-1].item())
        assert torch.equal(direct.pt_off, replayed.pt_off)
        assert torch.equal(direct.depth[:n], replayed.depth[:n])
        assert torch.equal(direct.background, replayed.background)
        replayed.depth.zero_()
    del g


def test_super_resolution_with_pinhole_camera_matches_oracle():
    sc = synth.sr_scene(4, rows=12, cols=10, s=3)
    m = sc.meta
    p = dict(dz=m["dz"], p_xy=0.6, r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"], persp=0.02)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**p))
    ctx = rt3d.Context(sc.irf.probs, sc.T, sr=3, **p)
    off, ent = oracle.compact(sc.Z[None])
    so = O.sr_reconstruct(off, ent, oracle.SRState(1, 12, 10, 3, 4))
    print("[gpu-combos] super-resolution with the pinhole camera", flush=True)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None])
    assert ctx.query().device_error == 0
    compare(res, so, 36, 30, "sr + pinhole")
    np.testing.assert_allclose(res.background.cpu().numpy(), so.b, rtol=1e-3, atol=1e-9)


def test_irf_classes_with_pinhole_camera_matches_oracle():
    sc, irfs, cls = synth.irf_class_scene(2, rows=22, cols=20)
    p = dict(params_for(sc), persp=0.004, p_xy=0.9)
    models = [oracle.Model(i.probs, sc.T) for i in irfs]
    O = oracle.Oracle(models[0], oracle.Params(**p), irf_models=models[1:], irf_class=cls.reshape(-1))
    ctx = rt3d.Context(irfs[0].probs, sc.T, **p)
    for i in irfs[1:]:
        ctx.add_irf(i.probs)
    off, ent = oracle.compact(sc.Z[None])
    so = O.reconstruct(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    print("[gpu-combos] IRF classes with the pinhole camera", flush=True)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None], irf_class=torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda())
    assert ctx.query().device_error == 0
    compare(res, so, sc.rows, sc.cols, "classes + pinhole")


def test_super_resolution_warm_start_matches_oracle_iterations():
    s = 3
    sa = synth.sr_scene(5, rows=10, cols=12, s=s)
    sb = synth.sr_scene(6, rows=10, cols=12, s=s)          # the next video frame
    m = sa.meta
    p = dict(dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
    O = oracle.Oracle(oracle.Model(sa.irf.probs, sa.T), oracle.Params(**p))
    ctx = rt3d.Context(sa.irf.probs, sa.T, sr=s, **p)
    R, C = 10 * s, 12 * s
    a = ctx.reconstruct(to_dev_hist(sa.Z)[None])
    assert ctx.query().device_error == 0
    # the state the call left, read back from its output (slot order = ascending depth)
    st = oracle.SRState(1, 10, 12, s, 4)
    pt = u32(a.pt_off).astype(np.int64)
    d, r, nrm = a.depth.cpu().numpy(), a.intensity.cpu().numpy(), a.normal.cpu().numpy().astype(np.float64)
    st.cnt[:] = np.diff(pt)
    for q in range(R * C):
        c = st.cnt[q]
        st.t[q, :c], st.r[q, :c], st.n[q, :c] = d[pt[q]:pt[q] + c], r[pt[q]:pt[q] + c], nrm[pt[q]:pt[q] + c]
    st.b[:] = a.background.cpu().numpy()
    b = ctx.make_output(R * C, n_bg=10 * 12)
    print("[gpu-combos] super-resolution warm start", flush=True)
    ctx.reconstruct_into(b, 1, 10, 12, hist=to_dev_hist(sb.Z)[None], warm_start=True)
    assert ctx.query().device_error == 0
    off, ent = oracle.compact(sb.Z[None])
    for _ in range(O.p.n_iter):
        O.sr_iterate(off, ent, st)
    compare(b, st, R, C, "sr warm start")
