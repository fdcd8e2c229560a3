"""GPU parity of photon-event ingest, through the C ABI: unordered (pixel, bin)
events counted into the active-bin lists, bit-exact against the oracle, and a
whole reconstruction from events identical to one from the histograms the
events add up to."""
import numpy as np
import pytest

from gpu_util import params_for, to_dev_hist, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402


def events_of(Z: np.ndarray, seed: int):
    """The photons of histograms Z [..., T] as shuffled (pixel, bin) events."""
    T = Z.shape[-1]
    flat = Z.reshape(-1)
    idx = np.flatnonzero(flat)
    key = np.repeat(idx, flat[idx].astype(np.int64))
    key = key[np.random.default_rng(seed).permutation(key.size)]
    return (key // T).astype(np.int32), (key % T).astype(np.int64)


def dev_events(pix, bins):
    return (torch.from_numpy(np.ascontiguousarray(pix, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(bins, dtype=np.uint16).view(np.int16)).cuda())


def check_csr(ctx, pix, bins, npix, T, label):
    dp, db = dev_events(pix, bins)
    print(f"[gpu-events] {label}: {pix.size} events, {npix} pixels x {T} bins", flush=True)
    off, ent = ctx.compact_events(dp, db, npix)
    assert ctx.query().device_error == 0
    oo, oe = oracle.compact_events(pix, bins, npix, T)
    o = u32(off)
    np.testing.assert_array_equal(o, oo)
    np.testing.assert_array_equal(u32(ent)[:o[-1]], oe)


@pytest.mark.parametrize("which", ["plane", "ragged"])
def test_events_compaction_bit_exact(which):
    if which == "plane":
        sc = synth.plane_scene(0)
    else:
        sc = synth.head_scene(0, rows=37, cols=23, T=777, signal=8.0, sbr=0.5)
    T = sc.T
    ctx = rt3d.Context(sc.irf.probs, T)
    pix, bins = events_of(sc.Z, 11)
    check_csr(ctx, pix, bins, sc.rows * sc.cols, T, which)


def test_events_long_segments_and_edges():
    """Segments around the LDS sort limit (2048 events) and far beyond it (the
    in-place global-memory sort), a bin at the maximum count, empty pixels."""
    T = 300
    rng = np.random.default_rng(5)
    sizes = [0, 1, 63, 64, 65, 2047, 2048, 2049, 5000, 70000, 0, 3]
    pix, bins = [], []
    for p, n in enumerate(sizes):
        if n == 70000:                       # 65535 photons in one bin + 4465 spread
            b = np.concatenate([np.full(65535, 17), rng.integers(18, T, n - 65535)])
        else:
            b = rng.integers(0, T if n < 3000 else 40, n)
        pix.append(np.full(b.size, p))
        bins.append(b)
    pix, bins = np.concatenate(pix), np.concatenate(bins)
    perm = rng.permutation(pix.size)
    irf = synth.gaussian_irf(1.5, 9).probs
    ctx = rt3d.Context(irf, T)
    check_csr(ctx, pix[perm], bins[perm], len(sizes), T, "long segments")
    check_csr(ctx, pix[:0], bins[:0], 5, T, "no events")


def test_events_invalid_and_saturated_flagged():
    T = 50
    irf = synth.gaussian_irf(1.5, 9).probs
    ctx = rt3d.Context(irf, T)
    pix = np.array([0, 1, 7, 1], dtype=np.int32)       # pixel 7 does not exist (npix = 4)
    bins = np.array([3, 4, 5, 60])                     # bin 60 >= T
    dp, db = dev_events(pix, bins)
    off, ent = ctx.compact_events(dp, db, 4)
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_INVALID
    o = u32(off)
    np.testing.assert_array_equal(o, [0, 1, 2, 2, 2])   # the two valid events are kept
    np.testing.assert_array_equal(u32(ent)[:2], [(3 << 16) | 1, (4 << 16) | 1])
    dp, db = dev_events(np.zeros(65537, dtype=np.int32), np.full(65537, 9))
    off, ent = ctx.compact_events(dp, db, 2)
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_INVALID
    assert u32(ent)[0] == (9 << 16) | 0xFFFF


def test_reconstruction_from_events_equals_from_histograms():
    sc = synth.head_scene(0, rows=37, cols=23, T=777, signal=8.0, sbr=0.5)
    T = sc.T
    ctx = rt3d.Context(sc.irf.probs, T, **params_for(sc))
    a = ctx.reconstruct(to_dev_hist(sc.Z)[None])
    pix, bins = events_of(sc.Z, 12)
    dp, db = dev_events(pix, bins)
    scratch = torch.empty(pix.size, dtype=torch.int32, device="cuda")
    P = sc.rows * sc.cols
    b = ctx.make_output(P)
    ctx.reconstruct_into(b, 1, sc.rows, sc.cols, events=(dp, db, scratch))
    st = ctx.query()
    assert st.device_error == 0 and st.entries == int(np.count_nonzero(sc.Z))
    print(f"[gpu-events] reconstruction from {pix.size} events, {st.entries} entries", flush=True)
    for name in ("pt_off", "depth", "intensity", "normal", "background"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
