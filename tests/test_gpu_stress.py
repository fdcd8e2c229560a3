"""The stress configuration at its full sizes: multi-layer scenes of 128^2,
256^2 and 512^2 pixels x 2000 bins (1 signal photon per pixel at SBR 0.01,
~98 active bins per pixel, 15% of the pixels empty), in one uneven batch.

The oracle cannot run 20 iterations over 344 k pixels, so the checks are the
ones that hold at any size or that the oracle can compute piece by piece:
compaction of the whole batch bit-exact; the initialisation and the raw
gradients of a full 512^2 frame, launched over the whole frame, against the
oracle on sampled windows (each pixel's initialisation depends only on the
pooled window around it, its initial normal on the APSS window beyond that,
its gradients on its own state and photons); and whole reconstructions of
the uneven batch equal to each frame alone, to the bit, twice."""
import numpy as np
import pytest

from gpu_util import device_to_oracle, oracle_to_device, to_dev_hist, to_dev_u32, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

SIDES = [128, 256, 512]
_SC = {}


def scenes():
    for k, n in enumerate(SIDES):
        if n not in _SC:
            print(f"[gpu-stress] generating {n}x{n}x2000", flush=True)
            _SC[n] = synth.stress_scene(k, side=n)
    return [_SC[n] for n in SIDES]


def params(sc):
    m = sc.meta
    return dict(dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])


def test_stress_compaction_bit_exact():
    scs = scenes()
    T = scs[0].T
    Z = np.concatenate([sc.Z.reshape(-1, T) for sc in scs])
    off_o, ent_o = oracle.compact(Z)
    ctx = rt3d.Context(scs[0].irf.probs, T, **params(scs[0]))
    print(f"[gpu-stress] compaction of {Z.shape[0]} pixels, {len(ent_o)} entries", flush=True)
    off, ent = ctx.compact(torch.from_numpy(Z.view(np.int16)).cuda(), capacity=len(ent_o) + 1024)
    assert ctx.query().device_error == 0
    np.testing.assert_array_equal(u32(off), off_o)
    np.testing.assert_array_equal(u32(ent)[:len(ent_o)], ent_o)


WINDOWS = [(0, 0), (0, 488), (250, 130), (490, 490), (300, 500)]   # top-left corners of 24 x 24 windows
MARGIN = 3          # pooling radius 1 + APSS radius 2 of the initial normals


def test_stress_full_frame_init_and_gradients_on_sampled_windows():
    sc = scenes()[-1]
    n, T = sc.rows, sc.T
    p = params(sc)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, T), oracle.Params(**p))
    ctx = rt3d.Context(sc.irf.probs, T, **p)
    off_o, ent_o = oracle.compact(sc.Z[None])
    off, ent = to_dev_u32(off_o), to_dev_u32(ent_o)
    print(f"[gpu-stress] init and gradients of a {n}x{n}x{T} frame", flush=True)
    d = ctx.step(rt3d.STEP_INIT, None, off, ent, shape=(1, n, n))
    full = device_to_oracle(d, 4)
    gt, gr, gb = ctx.gradients(d, off, ent)
    gt = gt.cpu().numpy()[:4].T.astype(np.float64)
    gr = gr.cpu().numpy()[:4].T.astype(np.float64)
    gb = gb.cpu().numpy().astype(np.float64)
    assert ctx.query().device_error == 0
    for (i0, j0) in WINDOWS:
        i0, j0 = min(i0, n - 24), min(j0, n - 24)
        a0, a1 = max(0, i0 - MARGIN), min(n, i0 + 24 + MARGIN)
        b0, b1 = max(0, j0 - MARGIN), min(n, j0 + 24 + MARGIN)
        crop = np.ascontiguousarray(sc.Z[a0:a1, b0:b1])
        co, ce = oracle.compact(crop[None])
        so = O.init(co, ce, oracle.State(1, a1 - a0, b1 - b0, 4))
        # the window's pixels in the crop and in the frame
        ci, cj = np.mgrid[i0 - a0:i0 - a0 + 24, j0 - b0:j0 - b0 + 24]
        qc = (ci * (b1 - b0) + cj).reshape(-1)
        qf = ((ci + a0) * n + (cj + b0)).reshape(-1)
        np.testing.assert_array_equal(full.cnt[qf], so.cnt[qc], err_msg=f"window {(i0, j0)} counts")
        np.testing.assert_array_equal(full.t[qf], so.t[qc], err_msg=f"window {(i0, j0)} depths")
        np.testing.assert_allclose(full.r[qf], so.r[qc], rtol=2e-6, atol=1e-6)
        np.testing.assert_allclose(full.b[qf], so.b[qc], rtol=2e-6, atol=1e-12)
        np.testing.assert_allclose(full.n[qf], so.n[qc], atol=2e-6)
        # gradients of the GPU's state on the window's pixels
        sw = oracle.State(1, 24, 24, 4)
        for a in ("t", "r", "n", "cnt", "b"):
            getattr(sw, a)[:] = getattr(full, a)[qf]
        wz = np.ascontiguousarray(sc.Z[i0:i0 + 24, j0:j0 + 24])
        wo, we = oracle.compact(wz[None])
        (ot, orr, ob), (at, ar, ab) = O.grad(wo, we, sw)
        live = np.arange(4)[None, :] < sw.cnt[:, None]
        for g_gpu, g_or, sc_ in ((gt[qf], ot, at), (gr[qf], orr, ar)):
            err = np.abs(g_gpu - g_or)[live]
            assert np.all(err <= 1e-4 * sc_[live] + 1e-30), (i0, j0, err.max())
        assert np.all(np.abs(gb[qf] - ob) <= 1e-4 * ab + 1e-30)
        print(f"[gpu-stress] window {(i0, j0)}: {int(so.cnt[qc].sum())} points agree", flush=True)


def test_stress_uneven_batch_equals_frames_alone_and_repeats():
    scs = scenes()
    T = scs[0].T
    # bit equality across batches needs a fixed lanes-per-pixel mapping (the
    # default follows the batch's size)
    ctx = rt3d.Context(scs[0].irf.probs, T, lanes_per_pixel=4, **params(scs[0]))
    alone = []
    for sc in scs:
        r = ctx.reconstruct(to_dev_hist(sc.Z)[None], max_entries=sc.rows * sc.cols * 110)
        assert ctx.query().device_error == 0
        alone.append((u32(r.pt_off).astype(np.int64), r.depth.cpu(), r.intensity.cpu(), r.background.cpu()))
    Z = torch.cat([to_dev_hist(sc.Z).reshape(-1, T) for sc in scs]).contiguous()
    P = int(Z.shape[0])
    shapes = [(sc.rows, sc.cols) for sc in scs]
    ctx.workspace(1, 1, P, P * 110)
    print(f"[gpu-stress] uneven batch {SIDES} ({P} pixels) in one call", flush=True)
    outs = []
    for _ in range(2):
        out = ctx.make_output(P)
        ctx.reconstruct_into(out, len(scs), 1, 1, hist=Z, frame_shapes=shapes)
        assert ctx.query().device_error == 0
        outs.append(out)
    a, b = outs
    assert torch.equal(a.pt_off, b.pt_off) and torch.equal(a.background, b.background)
    npts = int(a.pt_off[-1].item())
    assert torch.equal(a.depth[:npts], b.depth[:npts]) and torch.equal(a.intensity[:npts], b.intensity[:npts])
    pt = u32(a.pt_off).astype(np.int64)
    base = 0
    for f, (sc, (po, dep, inten, bg)) in enumerate(zip(scs, alone)):
        m = sc.rows * sc.cols
        np.testing.assert_array_equal(pt[base:base + m + 1] - pt[base], po, err_msg=f"frame {f} point offsets")
        k = int(po[-1])
        assert torch.equal(a.depth[pt[base]:pt[base] + k].cpu(), dep[:k]), f"frame {f} depth"
        assert torch.equal(a.intensity[pt[base]:pt[base] + k].cpu(), inten[:k]), f"frame {f} intensity"
        assert torch.equal(a.background[base:base + m].cpu(), bg), f"frame {f} background"
        base += m
    print(f"[gpu-stress] {npts} points over {P} pixels, batch equals frames alone", flush=True)
