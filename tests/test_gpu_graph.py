"""Replay of a recorded reconstruction (rt3d_graph_*), through the C ABI: each
replay reproduces, bit for bit, a direct call on the inputs the buffers hold at
that moment, with other GPU work and synchronisations between replays."""
import numpy as np
import pytest

from gpu_util import params_for, to_dev_hist

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1905_06700_amd import rt3d, synth  # noqa: E402


def _snapshot(res):
    """Offsets, background and the live part of the per-point arrays (the
    arrays' tail beyond the last point keeps whatever an earlier call left)."""
    n = int(res.pt_off[-1].item())
    return [res.pt_off.clone(), res.background.clone(), res.depth[:n].clone(), res.intensity[:n].clone(),
            res.normal[:n].clone()]


def test_graph_replays_equal_direct_calls():
    scenes = [synth.plane_scene(s) for s in range(3)]
    sc = scenes[0]
    F, R, C, T = 4, sc.rows, sc.cols, sc.T
    batches = [torch.stack([to_dev_hist(scenes[(k + f) % 3].Z) for f in range(F)]) for k in range(3)]
    ctx = rt3d.Context(sc.irf.probs, T, **params_for(sc))
    ctx.workspace(F, R, C, F * R * C * T)
    P = F * R * C
    buf = batches[0].clone()
    out_g = ctx.make_output(P)
    g = ctx.graph(out_g, F, R, C, hist=buf)
    for rep, k in enumerate((0, 1, 2, 0, 1)):
        buf.copy_(batches[k])
        g.launch()
        torch.cuda.synchronize()
        got = _snapshot(out_g)
        noise = torch.randn(1 << 16, device="cuda").sum()        # unrelated work between replays
        out_e = ctx.make_output(P)
        ctx.reconstruct_into(out_e, F, R, C, hist=buf)
        want = _snapshot(out_e)
        assert ctx.query().device_error == 0
        print(f"[gpu-graph] replay {rep} (batch {k}): {int(got[0][-1].item())} points, noise {float(noise):.2f}",
              flush=True)
        for a, b in zip(got, want):
            assert torch.equal(a, b)
    del g
