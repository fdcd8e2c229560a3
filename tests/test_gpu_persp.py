"""Perspective camera in the map f (Results, "Observation model": camera
parameters such as the focal length), through the C ABI, against the oracle
with the same camera: a tilted world plane and a sphere in front of it seen
by a pinhole camera.  Initial normals, APSS and the intensity graph (the
steps that use world positions) and whole reconstructions, with the bars of
the orthographic tests; the refusals."""
import numpy as np
import pytest

from gpu_util import intensity_err, device_to_oracle, oracle_to_device, to_dev_hist, to_dev_u32, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

_SC = {}


def scene(k=0):
    if k not in _SC:
        _SC[k] = synth.persp_scene(k) if k == 0 else synth.persp_scene(k, rows=29, cols=37, a=0.04)
    return _SC[k]


def pair_persp(sc):
    m = sc.meta
    p = dict(dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"],
             persp=m["persp"])
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**p))
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    return O, ctx


def test_persp_init_normals_match_oracle():
    sc = scene()
    O, ctx = pair_persp(sc)
    off, ent = oracle.compact(sc.Z[None])
    so = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    print(f"[gpu-persp] init {sc.rows}x{sc.cols}x{sc.T}", flush=True)
    d = ctx.step(rt3d.STEP_INIT, None, to_dev_u32(off), to_dev_u32(ent), shape=(1, sc.rows, sc.cols))
    sg = device_to_oracle(d, 4)
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    np.testing.assert_array_equal(sg.t, so.t)
    np.testing.assert_allclose(sg.n, so.n, atol=2e-6)


def test_persp_apss_and_intensity_graph_match_oracle():
    sc = scene()
    O, ctx = pair_persp(sc)
    off, ent = oracle.compact(sc.Z[None])
    s0 = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    for _ in range(2):
        O.iterate(off, ent, s0)
    din = oracle_to_device(s0)
    live = np.arange(4)[None, :] < s0.cnt[:, None]
    print("[gpu-persp] apss, intensity filter", flush=True)
    so = O.apss(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_APSS, din), 4)
    assert np.abs(sg.t - so.t)[live].max() <= 1e-3
    assert np.abs(sg.n - so.n)[live].max() <= 1e-3
    moved = np.abs(so.t - s0.t)[live].max()
    assert moved > 1e-3                                   # the step does something to compare

    so = O.intensity_filter(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_IFILTER, din), 4)
    same = sg.cnt == so.cnt
    assert same.mean() >= 0.999
    lv = (np.arange(4)[None, :] < so.cnt[:, None]) & same[:, None]
    np.testing.assert_allclose(sg.r[lv], so.r[lv], rtol=1e-5)


@pytest.mark.parametrize("k", [0, 1])
def test_persp_reconstruction_matches_oracle(k):
    sc = scene(k)
    O, ctx = pair_persp(sc)
    off, ent = oracle.compact(sc.Z[None])
    so = O.reconstruct(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    print(f"[gpu-persp] reconstruct scene {k}: {sc.rows}x{sc.cols}, persp {sc.meta['persp']}", flush=True)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None])
    assert ctx.query().device_error == 0
    pt = u32(res.pt_off).astype(np.int64)
    cnt = np.diff(pt)
    same = cnt == so.cnt
    bad = (~same).reshape(sc.rows, sc.cols)
    nb = np.zeros_like(bad)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            nb |= np.roll(np.roll(bad, di, 0), dj, 1)
    depth = res.depth.cpu().numpy()
    good = np.nonzero(~nb.reshape(-1) & (so.cnt > 0))[0]
    errs = [np.abs(depth[pt[p]:pt[p] + so.cnt[p]] - so.t[p, :so.cnt[p]]).max() for p in good]
    ierr = intensity_err(res.intensity, pt, so, good)
    print(f"[gpu-persp] scene {k}: count agreement {same.mean():.5f}, max depth err {max(errs):.2e} bins, "
          f"max intensity err {ierr:.2e} relative", flush=True)
    assert same.mean() >= 0.999
    assert max(errs) <= 1e-3
    assert ierr <= 2e-5
    np.testing.assert_allclose(res.background.cpu().numpy(), so.b, rtol=1e-3, atol=1e-9)


def test_persp_refusals():
    sc = scene()
    with pytest.raises(rt3d.Rt3dError) as e:
        rt3d.Context(sc.irf.probs, sc.T, persp=-0.1)
    assert e.value.status == rt3d.E_INVALID
    with pytest.raises(rt3d.Rt3dError) as e:      # R = ceil(2 / 0.3) = 7: the tile does not fit
        rt3d.Context(sc.irf.probs, sc.T, persp=0.05, p_xy=0.3)
    assert e.value.status == rt3d.E_UNSUPPORTED
