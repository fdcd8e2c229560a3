"""Initialisation of pixels whose pooled window holds many active bins
(Methods, initialisation: the log-matched filter over the pooled photons of
the window around each pixel).  One frame whose background rises across the
columns from 20 to 330 photons per pixel at T = 4613 puts pools of every size
in one launch: up to 608 photons (scored from registers and LDS), 609 to
1536 (listed and scored from LDS by the second kernel, which stages them in
passes over HBM), and more (the HBM path).  Through the C ABI against the
oracle: the initial state exactly (counts and depths) or within rounding
(intensities, background, normals), whole reconstructions to the bars of the
plain model, and a batch of two such frames equal to each alone."""
import numpy as np
import pytest

from gpu_util import intensity_err, device_to_oracle, to_dev_hist, to_dev_u32, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

_SC = {}


def scene(k=0):
    if k not in _SC:
        _SC[k] = synth.ramp_background_scene(k, cols=44 if k == 0 else 37)
    return _SC[k]


def params(sc):
    m = sc.meta
    return dict(dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])


def pools(sc):
    """Pooled active bins of each pixel's (2 r_init + 1)^2 window."""
    nz = (sc.Z != 0).sum(-1)
    pad = np.pad(nz, 1)
    return sum(pad[1 + di:1 + di + sc.rows, 1 + dj:1 + dj + sc.cols] for di in (-1, 0, 1) for dj in (-1, 0, 1))


def test_scene_spans_every_pool_regime():
    sc = scene()
    pl = pools(sc).reshape(-1)
    assert (pl <= 608).sum() >= 100 and ((pl > 608) & (pl <= 1536)).sum() >= 100 and (pl > 1536).sum() >= 100


def test_wide_pools_init_matches_oracle():
    sc = scene()
    p = params(sc)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**p))
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    off, ent = oracle.compact(sc.Z[None])
    so = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    print(f"[gpu-wide] init {sc.rows}x{sc.cols}x{sc.T}, {len(ent)} entries", flush=True)
    d = ctx.step(rt3d.STEP_INIT, None, to_dev_u32(off), to_dev_u32(ent), shape=(1, sc.rows, sc.cols))
    assert ctx.query().device_error == 0
    sg = device_to_oracle(d, 4)
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    np.testing.assert_array_equal(sg.t, so.t)
    np.testing.assert_allclose(sg.r, so.r, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sg.b, so.b, rtol=2e-6, atol=1e-12)
    np.testing.assert_allclose(sg.n, so.n, atol=2e-6)
    assert (so.cnt > 0).mean() > 0.9


def test_wide_pools_reconstruction_matches_oracle():
    sc = scene()
    p = params(sc)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**p))
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    off, ent = oracle.compact(sc.Z[None])
    so = O.reconstruct(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    print("[gpu-wide] reconstruct", flush=True)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None], max_entries=len(ent) + 4096)
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
    errs = [np.abs(depth[pt[q]:pt[q] + so.cnt[q]] - so.t[q, :so.cnt[q]]).max() for q in good]
    ierr = intensity_err(res.intensity, pt, so, good)
    print(f"[gpu-wide] count agreement {same.mean():.5f}, max depth err {max(errs):.2e} bins "
          f"over {len(errs)} pixels, max intensity err {ierr:.2e} relative", flush=True)
    assert same.mean() >= 0.999
    assert len(errs) > 0.5 * so.npix and max(errs) <= 1e-3
    assert ierr <= 2e-5
    np.testing.assert_allclose(res.background.cpu().numpy(), so.b, rtol=1e-3, atol=1e-9)


def test_wide_pools_batch_equals_frames_alone():
    sa, sb = scene(0), scene(1)
    ctx = rt3d.Context(sa.irf.probs, sa.T, **params(sa))
    alone = []
    for sc in (sa, sb):
        r = ctx.reconstruct(to_dev_hist(sc.Z)[None], max_entries=sc.rows * sc.cols * 400)
        alone.append((u32(r.pt_off).astype(np.int64), r.depth.cpu(), r.background.cpu()))
    Z = torch.cat([to_dev_hist(sa.Z).reshape(-1, sa.T), to_dev_hist(sb.Z).reshape(-1, sb.T)]).contiguous()
    P = int(Z.shape[0])
    ctx.workspace(1, 1, P, P * 400)
    out = ctx.make_output(P)
    print("[gpu-wide] uneven batch", flush=True)
    ctx.reconstruct_into(out, 2, 1, 1, hist=Z, frame_shapes=[(sa.rows, sa.cols), (sb.rows, sb.cols)])
    assert ctx.query().device_error == 0
    pt = u32(out.pt_off).astype(np.int64)
    n0 = sa.rows * sa.cols
    for f, (b, n) in enumerate(((0, n0), (n0, sb.rows * sb.cols))):
        po, dep, bg = alone[f]
        np.testing.assert_array_equal(pt[b:b + n + 1] - pt[b], po, err_msg=f"frame {f}")
        assert torch.equal(out.depth[pt[b]:pt[b + n]].cpu(), dep[:int(po[-1])]), f"frame {f} depth"
        assert torch.equal(out.background[b:b + n].cpu(), bg), f"frame {f} background"


def test_wide_pools_with_irf_classes_match_oracle():
    """Two IRF classes in 4 x 4 pixel blocks: one init launch per class, each
    listing only its own class's large pools for the wide kernel."""
    sc = scene()
    p = params(sc)
    irfs = [sc.irf, synth.gaussian_irf(2.0, 12)]
    i, j = np.mgrid[0:sc.rows, 0:sc.cols]
    cls = (((i // 4) + (j // 4)) % 2).astype(np.uint8).reshape(-1)
    models = [oracle.Model(f.probs, sc.T) for f in irfs]
    O = oracle.Oracle(models[0], oracle.Params(**p), irf_models=models[1:], irf_class=cls)
    O._keep = models
    ctx = rt3d.Context(irfs[0].probs, sc.T, **p)
    ctx.add_irf(irfs[1].probs)
    off, ent = oracle.compact(sc.Z[None])
    so = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    ctx.debug_irf_class(torch.from_numpy(cls).cuda())
    print("[gpu-wide] init with two IRF classes", flush=True)
    d = ctx.step(rt3d.STEP_INIT, None, to_dev_u32(off), to_dev_u32(ent), shape=(1, sc.rows, sc.cols))
    assert ctx.query().device_error == 0
    sg = device_to_oracle(d, 4)
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    np.testing.assert_array_equal(sg.t, so.t)
    np.testing.assert_allclose(sg.r, so.r, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sg.b, so.b, rtol=2e-6, atol=1e-12)
