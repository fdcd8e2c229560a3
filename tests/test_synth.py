"""The seeded generators: determinism and the photon levels they promise."""
import numpy as np

from paper_1905_06700_amd import synth


def test_plane_scene_is_deterministic_and_levels():
    a = synth.plane_scene(3)
    b = synth.plane_scene(3)
    np.testing.assert_array_equal(a.Z, b.Z)
    assert a.Z.shape == (32, 32, 300) and a.Z.dtype == np.uint16
    d = a.depth[0]
    assert d.min() == 50.0 and d.max() == 250.0
    photons = a.Z.sum() / (32 * 32)
    assert abs(photons - 11.0) < 0.6           # 10 signal + 1 background on average
    assert not np.array_equal(a.Z, synth.plane_scene(4).Z)


def test_head_scene_shape_occluder_and_levels():
    sc = synth.head_scene(0, rows=47, cols=47, T=1200, signal=5.0, sbr=0.1)
    assert sc.Z.shape == (47, 47, 1200)
    M = sc.meta["occluder"]
    assert M.sum() == round(0.3 * 47 * 47)
    assert np.allclose(sc.depth[1][M > 0] - sc.depth[0][M > 0], 200.0)
    sig = np.nansum(np.where(np.isfinite(sc.depth), sc.intensity, 0), 0).mean()
    assert abs(sig - 5.0) < 0.2
    assert abs(sc.background * 1200 - 50.0) < 1e-9


def test_irf_probabilities():
    g = synth.gaussian_irf(1.5, 9)
    assert g.origin == 9 and abs(g.probs.sum() - 1) < 1e-6
    e = synth.exgauss_irf(3.0, 10.0, -18, 118)
    assert abs(e.probs.sum() - 1) < 1e-4 and 0 < e.shift < 10
