"""Warm start (video): a reconstruction that starts from the previous call's
final state instead of the initialisation, through the C ABI, against the
oracle running the same iterations from that state (the previous call's
output, read back)."""
import numpy as np
import pytest

from gpu_util import intensity_err, pair, to_dev_hist, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402


def next_frame(sc, seed):
    """The same scene with new photon counts (the next frame of a static scene)."""
    Z = synth.render(np.random.default_rng(seed), sc.irf, sc.T, sc.depth, sc.intensity, sc.background)
    return synth.Scene(Z, sc.irf, sc.T, sc.depth, sc.intensity, sc.background, sc.meta)


def state_from_output(res, rows, cols):
    """The point state a reconstruction left, rebuilt from its output (points
    in slot order, which is ascending depth)."""
    s = oracle.State(1, rows, cols, 4)
    pt = u32(res.pt_off).astype(np.int64)
    depth, inten = res.depth.cpu().numpy(), res.intensity.cpu().numpy()
    normal = res.normal.cpu().numpy().astype(np.float64)
    s.cnt[:] = np.diff(pt)
    for p in range(rows * cols):
        c = s.cnt[p]
        s.t[p, :c] = depth[pt[p]:pt[p] + c]
        s.r[p, :c] = inten[pt[p]:pt[p] + c]
        s.n[p, :c] = normal[pt[p]:pt[p] + c]
    s.b[:] = res.background.cpu().numpy()
    return s


def test_warm_start_matches_oracle_iterations():
    sa = synth.plane_scene(0)
    sb = next_frame(sa, 77)
    O, ctx = pair(sa)
    R, C = sa.rows, sa.cols
    a = ctx.reconstruct(to_dev_hist(sa.Z)[None])
    assert ctx.query().device_error == 0
    s0 = state_from_output(a, R, C)
    b = ctx.make_output(R * C)
    ctx.reconstruct_into(b, 1, R, C, hist=to_dev_hist(sb.Z)[None], warm_start=True)
    assert ctx.query().device_error == 0
    off_o, ent_o = oracle.compact(sb.Z.reshape(1, R, C, sb.T))
    so = s0.copy()
    for _ in range(O.p.n_iter):
        O.iterate(off_o, ent_o, so)
    pt = u32(b.pt_off).astype(np.int64)
    cnt = np.diff(pt)
    same = cnt == so.cnt
    print(f"[gpu-warm] count agreement {same.mean():.5f} over {R * C} pixels", flush=True)
    assert same.mean() >= 0.999
    depth = b.depth.cpu().numpy()
    err = max(float(np.abs(depth[pt[p]:pt[p] + cnt[p]] - so.t[p, :cnt[p]]).max(initial=0))
              for p in np.nonzero(same)[0])
    ierr = intensity_err(b.intensity, pt, so, np.nonzero(same)[0])
    print(f"[gpu-warm] max depth err {err:.2e} bins, max intensity err {ierr:.2e} relative", flush=True)
    assert err <= 1e-3
    assert ierr <= 2e-5
    np.testing.assert_allclose(b.background.cpu().numpy(), so.b, rtol=1e-4, atol=1e-9)


def test_warm_start_needs_a_matching_previous_state():
    sa = synth.plane_scene(0)
    O, ctx = pair(sa)
    R, C = sa.rows, sa.cols
    Z = to_dev_hist(sa.Z)[None]
    ctx.workspace(1, R, C, R * C * 64)
    out = ctx.make_output(R * C)
    with pytest.raises(rt3d.Rt3dError) as e:          # nothing reconstructed yet
        ctx.reconstruct_into(out, 1, R, C, hist=Z, warm_start=True)
    assert e.value.status == rt3d.E_STATE
    ctx.reconstruct_into(out, 1, R, C, hist=Z)
    ctx.reconstruct_into(out, 1, R, C, hist=Z, warm_start=True)     # same frames: accepted
    assert ctx.query().device_error == 0
    half = Z[:, :R // 2].contiguous()
    with pytest.raises(rt3d.Rt3dError) as e:          # different frame size
        ctx.reconstruct_into(ctx.make_output(half.shape[1] * C), 1, R // 2, C, hist=half, warm_start=True)
    assert e.value.status == rt3d.E_STATE
