"""rt3d_compact_noalloc (the compaction for callers that cannot allocate)
against rt3d_debug_compact on the same histograms: identical lists, bit for
bit, on two calls in a row (the second smaller, into the same buffers), with
the capacity overflow reported the same way."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_06700_amd import rt3d, synth
from gpu_util import to_dev_hist, u32

pytestmark = pytest.mark.gpu


def _lists_existing(ctx, Zd, cap):
    off, ent = ctx.compact(Zd, capacity=cap)
    torch.cuda.synchronize()
    return u32(off), u32(ent)


def test_noalloc_compaction_equals_existing_entry_point_twice():
    sc = synth.head_scene(0, rows=48, cols=40)          # T = 4613, ~54 active bins per pixel, some > 128
    Z = sc.Z.reshape(-1, sc.T)
    rng = np.random.default_rng(7)
    Z2 = rng.poisson(0.05, (37, sc.T)).astype(np.uint16)   # second call: fewer pixels, ragged
    Z2[5] = 0                                               # an empty pixel
    ref = rt3d.Context(sc.irf.probs, sc.T)
    fresh = rt3d.Context(sc.irf.probs, sc.T)              # never given a workspace
    P1 = Z.shape[0]
    cap = int(np.count_nonzero(Z)) + 64
    off = torch.full((P1 + 1,), -1, dtype=torch.int32, device="cuda")
    ent = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for call, Zc in enumerate((Z, Z2)):
        Zd = to_dev_hist(np.ascontiguousarray(Zc))
        P = Zc.shape[0]
        fresh.compact_noalloc(Zd, off, ent, err)
        torch.cuda.synchronize()
        off_e, ent_e = _lists_existing(ref, Zd, cap)
        off_o, ent_o = oracle.compact(Zc)
        got_off = u32(off)[:P + 1]
        E = int(got_off[-1])
        print(f"[no-alloc] call {call}: {P} pixels x {sc.T} bins, {E} entries", flush=True)
        np.testing.assert_array_equal(got_off, off_e[:P + 1])
        np.testing.assert_array_equal(u32(ent)[:E], ent_e[:E])
        np.testing.assert_array_equal(got_off, off_o)
        np.testing.assert_array_equal(u32(ent)[:E], ent_o)
        assert int(err.item()) == 0
    assert fresh.query().device_error == 0


def test_noalloc_capacity_overflow_matches_existing_entry_point():
    rng = np.random.default_rng(3)
    T = 301
    Z = rng.poisson(0.4, (300, T)).astype(np.uint16)
    ctx = rt3d.Context([1.0, 2.0, 1.0], T)
    ref = rt3d.Context([1.0, 2.0, 1.0], T)
    cap = int(np.count_nonzero(Z)) // 2
    Zd = to_dev_hist(Z)
    for P in (300, 211):                                    # two calls, the second smaller
        off = torch.zeros(P + 1, dtype=torch.int32, device="cuda")
        ent = torch.zeros(cap, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.compact_noalloc(Zd[:P], off, ent, err)
        torch.cuda.synchronize()
        assert int(err.item()) == rt3d.E_CAPACITY
        off_e, ent_e = _lists_existing(ref, Zd[:P], cap)
        with pytest.raises(rt3d.Rt3dError):
            ref.query()
        np.testing.assert_array_equal(u32(off), off_e[:P + 1])
        assert int(u32(off)[-1]) == cap
        np.testing.assert_array_equal(u32(ent), ent_e[:cap])


def test_noalloc_rejects_sizes_past_its_array_on_the_host():
    ctx = rt3d.Context([1.0, 2.0, 1.0], 8)
    t = torch.zeros(16, dtype=torch.int32, device="cuda")
    L = rt3d.lib()
    st = L.rt3d_compact_noalloc(ctx._h, rt3d._ptr(t), rt3d.NOALLOC_MAX_PIXELS + 1, rt3d._ptr(t),
                                rt3d._ptr(t), 16, None, rt3d._stream())
    assert st == rt3d.E_INVALID
    assert b"RT3D_NOALLOC_MAX_PIXELS" in L.rt3d_last_error(ctx._h)
