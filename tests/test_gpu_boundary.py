"""The C ABI's output and error contract on the GPU: the world Z output of
the observation model's map f, gains outside the model's range, non-finite
values reaching the output, and checkpoints of the learned denoiser that let
training resume exactly."""
import ctypes as C
import os

import numpy as np
import pytest

from gpu_util import oracle_to_device, params_for, to_dev_hist, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from oracle import cnn  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

FLT_MIN = float(np.finfo(np.float32).tiny)


def _points(res):
    pt = u32(res.pt_off).astype(np.int64)
    return pt, res.depth.cpu().numpy()


def _ray_z(persp, rows, cols):
    """z component of each pixel's unit ray under the pinhole camera (pixel-major)."""
    i, j = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    u = persp * (j - 0.5 * (cols - 1))
    w = persp * (i - 0.5 * (rows - 1))
    return (1.0 / np.sqrt(1.0 + u * u + w * w)).reshape(-1)


def test_world_z_orthographic_and_old_output_struct():
    sc = synth.plane_scene(0)
    p = params_for(sc, n_iter=3)
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    Zd = to_dev_hist(sc.Z)[None]
    res = ctx.reconstruct(Zd, world_z=True)
    assert ctx.query().device_error == 0
    pt, depth = _points(res)
    n = int(pt[-1])
    assert n > 0
    np.testing.assert_array_equal(res.world_z.cpu().numpy()[:n], depth[:n] * p["dz"])
    # a caller built before world_z existed passes the shorter struct and gets the same output
    old = ctx.make_output(sc.rows * sc.cols)
    inp, o = ctx._io(old, 1, sc.rows, sc.cols, hist=Zd)
    o.struct_size = rt3d.Output.world_z.offset
    o.world_z = 12345                                   # past the caller's struct: must not be used
    ctx._check(rt3d.lib().rt3d_reconstruct(ctx._h, C.byref(inp), C.byref(o), rt3d._stream()))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(old.pt_off), u32(res.pt_off))
    np.testing.assert_array_equal(old.depth.cpu().numpy()[:n], depth[:n])
    o.struct_size = rt3d.Output.world_z.offset + 4
    assert rt3d.lib().rt3d_reconstruct(ctx._h, C.byref(inp), C.byref(o), rt3d._stream()) == rt3d.E_INVALID


@pytest.mark.parametrize("sr", [1, 2])
def test_world_z_pinhole_camera(sr):
    sc = synth.persp_scene(0) if sr == 1 else synth.persp_scene(0, rows=16, cols=14)
    p = params_for(sc, n_iter=2, persp=sc.meta["persp"], sr=sr)
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None], world_z=True)
    assert ctx.query().device_error == 0
    pt, depth = _points(res)
    vz = _ray_z(p["persp"], sc.rows * sr, sc.cols * sr)
    wz = res.world_z.cpu().numpy()
    cnt = np.diff(pt)
    want = np.repeat(vz, cnt) * depth[:pt[-1]] * p["dz"]
    assert pt[-1] > 0
    np.testing.assert_allclose(wz[:pt[-1]], want, rtol=1e-13, atol=0)


def test_invalid_gains_count_as_dead_pixels_and_are_reported():
    sc = synth.plane_scene(1)
    p = params_for(sc, n_iter=4)
    P = sc.rows * sc.cols
    g = np.ones(P, dtype=np.float32)
    bad = [3, 100, 517, 1000]
    g_bad = g.copy()
    g_bad[bad] = [np.nan, -1.0, np.inf, -np.inf]
    g_dead = g.copy()
    g_dead[bad] = 0.0
    Zd = to_dev_hist(sc.Z)[None]
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    r_bad = ctx.reconstruct(Zd, gain=torch.from_numpy(g_bad).cuda())
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_INVALID
    ctx2 = rt3d.Context(sc.irf.probs, sc.T, **p)
    r_dead = ctx2.reconstruct(Zd, gain=torch.from_numpy(g_dead).cuda())
    assert ctx2.query().device_error == 0
    np.testing.assert_array_equal(u32(r_bad.pt_off), u32(r_dead.pt_off))
    n = int(u32(r_dead.pt_off)[-1])
    np.testing.assert_array_equal(r_bad.depth.cpu().numpy()[:n], r_dead.depth.cpu().numpy()[:n])
    np.testing.assert_array_equal(r_bad.intensity.cpu().numpy()[:n], r_dead.intensity.cpu().numpy()[:n])
    np.testing.assert_array_equal(r_bad.background.cpu().numpy(), r_dead.background.cpu().numpy())
    assert np.all(np.diff(u32(r_dead.pt_off).astype(np.int64))[bad] == 0)


def test_intensity_beyond_fp32_range_is_reported_as_nonfinite():
    """A pixel with the smallest normal FP32 gain: its initial intensity (the
    window's signal photons over g sum h) passes the FP32 range.  With no
    iteration the value reaches the output, and the call reports E_NONFINITE."""
    sc = synth.plane_scene(2)
    p = params_for(sc, n_iter=0)
    off, ent = oracle.compact(sc.Z[None])
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**p))
    s0 = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    r0 = np.where(s0.cnt > 0, s0.r[:, 0], 0.0)
    big = np.nonzero(r0 > 8.0)[0][:5]                   # r0 / FLT_MIN > FLT_MAX for these
    assert len(big) == 5
    g = np.ones(sc.rows * sc.cols, dtype=np.float32)
    g[big] = FLT_MIN
    ctx = rt3d.Context(sc.irf.probs, sc.T, **p)
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None], gain=torch.from_numpy(g).cuda())
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_NONFINITE
    pt = u32(res.pt_off).astype(np.int64)
    inten = res.intensity.cpu().numpy()
    assert all(np.isinf(inten[pt[q]]) for q in big)
    ok = np.setdiff1d(np.arange(sc.rows * sc.cols), big)
    assert all(np.all(np.isfinite(inten[pt[q]:pt[q + 1]])) for q in ok)


def _cnn_state():
    sc = synth.layers_scene(3, rows=24, cols=40, T=512)
    prm = params_for(sc)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, sc.T), oracle.Params(**prm))
    off, ent = oracle.compact(sc.Z[None])
    s = O.init(off, ent, oracle.State(1, sc.rows, sc.cols, 4))
    O.depth_step(off, ent, s)
    return sc, prm, s


def test_denoiser_checkpoint_resumes_training_bit_identically(tmp_path):
    sc, prm, s = _cnn_state()
    truth = torch.from_numpy(sc.depth.reshape(sc.depth.shape[0], -1).astype(np.float32)).cuda()
    st = oracle_to_device(s)

    def ctx_():
        c = rt3d.Context(sc.irf.probs, sc.T, denoiser=rt3d.DENOISE_CNN, **prm)
        c.workspace(1, sc.rows, sc.cols, sc.rows * sc.cols * 64)
        return c

    a = ctx_()
    a.cnn_set_weights(cnn.he_init(21).astype(np.float32))
    for _ in range(3):
        a.cnn_train_step(st, truth, lr=2e-3)
    path = str(tmp_path / "net.rt3dcnn")
    a.denoiser_save(path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"RT3DCNN\0" and len(raw) == 8 + 4 * 11 + 8 + 12 * rt3d.CNN_PARAMS + 8
    assert int.from_bytes(raw[52:60], "little") == 3              # Adam step
    for _ in range(2):
        a.cnn_train_step(st, truth, lr=2e-3)
    wa = a.cnn_get_weights()
    b = ctx_()
    b.denoiser_load(path)
    for _ in range(2):
        b.cnn_train_step(st, truth, lr=2e-3)
    np.testing.assert_array_equal(b.cnn_get_weights(), wa)
    np.testing.assert_array_equal(b.cnn_last_gradient(), a.cnn_last_gradient())
    # damaged files leave the context as it was
    wb = b.cnn_get_weights()
    for name, data in [("short", raw[:-9]), ("long", raw + b"\0"),
                       ("flipped", raw[:100] + bytes([raw[100] ^ 1]) + raw[101:]),
                       ("magic", b"RT3DCNX\0" + raw[8:])]:
        q = str(tmp_path / name)
        open(q, "wb").write(data)
        with pytest.raises(rt3d.Rt3dError) as e:
            b.denoiser_load(q)
        assert e.value.status == rt3d.E_INVALID, name
    np.testing.assert_array_equal(b.cnn_get_weights(), wb)
    plain = rt3d.Context(sc.irf.probs, sc.T, **prm)
    with pytest.raises(rt3d.Rt3dError) as e:
        plain.denoiser_load(path)
    assert e.value.status == rt3d.E_STATE
