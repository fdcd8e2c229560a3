"""Frames of different sizes in one reconstruction call, through the C ABI:
every frame's result must equal, to the bit, what a call on that frame alone
returns (per-pixel steps run once over the whole batch, steps that read
neighbouring pixels once per group of equally sized frames).  The single-frame
calls are themselves held to the oracle by test_gpu_parity.py."""
import numpy as np
import pytest

from gpu_util import params_for, to_dev_hist

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1905_06700_amd import rt3d, synth  # noqa: E402

# two frames of one size (one group), then two other sizes, then the first
# size again (a group of its own: groups are runs of consecutive frames)
SHAPES = [(37, 23), (37, 23), (20, 31), (9, 40), (37, 23)]
T = 777


def scenes():
    return [synth.head_scene(40 + f, rows=r, cols=c, T=T, signal=8.0, sbr=0.5) for f, (r, c) in enumerate(SHAPES)]


def alone(ctx, sc):
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None])
    st = ctx.query()
    assert st.device_error == 0
    return res


def frame_slices(res, bases, sizes):
    """Per frame: (pt_off relative to the frame's first point, depth, intensity, normal, background)."""
    pt = res.pt_off.cpu().numpy().view(np.uint32).astype(np.int64)
    out = []
    for b, n in zip(bases, sizes):
        p0, p1 = pt[b], pt[b + n]
        out.append((pt[b:b + n + 1] - p0, res.depth[p0:p1].cpu(), res.intensity[p0:p1].cpu(),
                    res.normal[p0:p1].cpu(), res.background[b:b + n].cpu()))
    return out


def test_uneven_batch_equals_frames_alone():
    scs = scenes()
    # frames alone take the per-step kernels too (not the one-launch loop of small
    # frames, whose sums round in another order), so the results compare to the bit
    ctx = rt3d.Context(scs[0].irf.probs, T, **params_for(scs[0]), fused_loop=0)
    sizes = [r * c for r, c in SHAPES]
    bases = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    P = int(sum(sizes))
    ref = [frame_slices(alone(ctx, sc), [0], [sc.rows * sc.cols])[0] for sc in scs]
    Z = torch.cat([to_dev_hist(sc.Z).reshape(-1, T) for sc in scs]).contiguous()
    ctx.workspace(1, 1, P, P * 64)
    out = ctx.make_output(P)
    print(f"[gpu-uneven] {len(SHAPES)} frames {SHAPES}, {P} pixels in one call", flush=True)
    ctx.reconstruct_into(out, len(SHAPES), 1, 1, hist=Z, frame_shapes=SHAPES)
    st = ctx.query()
    assert st.device_error == 0
    got = frame_slices(out, bases, sizes)
    for f, (a, b) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(a[0], b[0], err_msg=f"frame {f} point offsets")
        for name, x, y in zip(("depth", "intensity", "normal", "background"), a[1:], b[1:]):
            assert torch.equal(x, y), f"frame {f} {name}"
    assert int(out.pt_off[-1].item()) == sum(int(r[0][-1]) for r in ref)


def test_uneven_batch_graph_replay():
    scs = scenes()[:3]
    shapes = SHAPES[:3]
    ctx = rt3d.Context(scs[0].irf.probs, T, **params_for(scs[0]))
    sizes = [r * c for r, c in shapes]
    P = int(sum(sizes))
    Z = torch.cat([to_dev_hist(sc.Z).reshape(-1, T) for sc in scs]).contiguous()
    ctx.workspace(1, 1, P, P * 64)
    direct = ctx.make_output(P)
    ctx.reconstruct_into(direct, len(shapes), 1, 1, hist=Z, frame_shapes=shapes)
    replayed = ctx.make_output(P)
    g = ctx.graph(replayed, len(shapes), 1, 1, hist=Z, frame_shapes=shapes)
    g.launch()
    torch.cuda.synchronize()
    assert ctx.query().device_error == 0
    for name in ("pt_off", "background"):
        assert torch.equal(getattr(direct, name), getattr(replayed, name)), name
    n = int(direct.pt_off[-1].item())
    for name in ("depth", "intensity", "normal"):
        assert torch.equal(getattr(direct, name)[:n], getattr(replayed, name)[:n]), name
    del g


def test_uneven_batch_with_learned_denoiser_equals_frames_alone():
    """The learned denoiser runs once per group of equal-size frames; each
    frame of the batch equals the frame reconstructed alone, to the bit."""
    from oracle import cnn
    scs = scenes()
    w = cnn.he_init(3).astype(np.float32)
    rng = np.random.default_rng(4)
    w += rng.normal(0, 0.02, w.shape).astype(np.float32)
    prm = dict(params_for(scs[0]), denoiser=rt3d.DENOISE_CNN, fused_loop=0, n_iter=4)
    ctx = rt3d.Context(scs[0].irf.probs, T, **prm)
    ctx.cnn_set_weights(w)
    sizes = [r * c for r, c in SHAPES]
    bases = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    P = int(sum(sizes))
    ref = [frame_slices(alone(ctx, sc), [0], [sc.rows * sc.cols])[0] for sc in scs]
    Z = torch.cat([to_dev_hist(sc.Z).reshape(-1, T) for sc in scs]).contiguous()
    ctx.workspace(1, 1, P, P * 64)
    out = ctx.make_output(P)
    print(f"[gpu-uneven] learned denoiser, {len(SHAPES)} frames {SHAPES} in one call", flush=True)
    ctx.reconstruct_into(out, len(SHAPES), 1, 1, hist=Z, frame_shapes=SHAPES)
    assert ctx.query().device_error == 0
    got = frame_slices(out, bases, sizes)
    for f, (a, b) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(a[0], b[0], err_msg=f"frame {f} point offsets")
        for name, x, y in zip(("depth", "intensity", "normal", "background"), a[1:], b[1:]):
            assert torch.equal(x, y), f"frame {f} {name}"
