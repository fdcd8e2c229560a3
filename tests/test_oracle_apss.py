"""Pins of the oracle's APSS depth denoiser and initial normals.

APSS fits algebraic spheres to oriented points (the depth update of the
paper's Results, "Reconstruction algorithm"; the APSS method it cites).
Points sampled exactly on a plane or a sphere, with their exact normals, are
fixed points of the fit-and-project step; a weighted plane fit recovers the
normal of planar samples; the fit is translation covariant; and the pixel
window search finds the same neighbours as a search over every point.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def grid_state(oracle, rows, cols, K=2):
    s = oracle.State(1, rows, cols, K)
    s.cnt[:] = 1
    return s


def test_plane_is_fixed_point(oracle_lib):
    rows, cols, dz = 12, 14, 0.1
    p = oracle_lib.Params(dz=dz, k_max=2)
    s = grid_state(oracle_lib, rows, cols)
    i, j = np.mgrid[0:rows, 0:cols]
    a, bx, by = 30.0, 0.37, -0.21                # world plane Z = a + bx X + by Y
    Zw = a + bx * j + by * i
    s.t[:, 0] = (Zw / dz).reshape(-1)
    n = np.array([bx, by, -1.0]) / np.linalg.norm([bx, by, -1.0])
    s.n[:, 0, :] = n
    t0 = s.t.copy()
    oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=1000), p).apss(s)
    np.testing.assert_allclose(s.t[:, 0], t0[:, 0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(s.n[:, 0, :], np.broadcast_to(n, (rows * cols, 3)), atol=1e-12)


def test_sphere_front_cap_is_fixed_point(oracle_lib):
    rows = cols = 15
    dz = 0.05
    p = oracle_lib.Params(dz=dz, k_max=2, h_apss=2.5)
    s = grid_state(oracle_lib, rows, cols)
    i, j = np.mgrid[0:rows, 0:cols].astype(float)
    c = np.array([7.3, 6.8, 40.0])
    rad = 12.0
    Zw = c[2] - np.sqrt(rad ** 2 - (j - c[0]) ** 2 - (i - c[1]) ** 2)   # near side
    s.t[:, 0] = (Zw / dz).reshape(-1)
    pts = np.stack([j, i, Zw], -1).reshape(-1, 3)
    nrm = (pts - c) / rad                                              # faces the sensor
    s.n[:, 0, :] = nrm
    t0 = s.t.copy()
    oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=2000), p).apss(s)
    np.testing.assert_allclose(s.t[:, 0] * dz, t0[:, 0] * dz, rtol=0, atol=1e-10)
    np.testing.assert_allclose(s.n[:, 0, :], nrm, atol=1e-10)


def test_two_separated_planes_do_not_mix(oracle_lib):
    rows, cols, dz = 10, 10, 0.1
    p = oracle_lib.Params(dz=dz, k_max=2)
    s = oracle_lib.State(1, rows, cols, 2)
    s.cnt[:] = 2
    i, j = np.mgrid[0:rows, 0:cols]
    front = 20.0 + 0.1 * j
    back = 35.0 - 0.2 * i
    s.t[:, 0] = (front / dz).reshape(-1)
    s.t[:, 1] = (back / dz).reshape(-1)
    nf = np.array([0.1, 0.0, -1.0]) / np.linalg.norm([0.1, 0.0, -1.0])
    nb = np.array([0.0, -0.2, -1.0]) / np.linalg.norm([0.0, -0.2, -1.0])
    s.n[:, 0, :] = nf
    s.n[:, 1, :] = nb
    t0 = s.t.copy()
    oracle_lib.Oracle(oracle_lib.Model([1.0], T=1000), p).apss(s)
    np.testing.assert_allclose(s.t, t0, atol=1e-10)


def test_plane_fit_normals_recover_plane(oracle_lib):
    rows, cols, dz = 9, 11, 0.2
    p = oracle_lib.Params(dz=dz, k_max=2)
    s = grid_state(oracle_lib, rows, cols)
    i, j = np.mgrid[0:rows, 0:cols]
    bx, by = -0.3, 0.45
    s.t[:, 0] = ((10.0 + bx * j + by * i) / dz).reshape(-1)
    O = oracle_lib.Oracle(oracle_lib.Model([1.0], T=1000), p)
    O.init_normals(s)
    n = np.array([bx, by, -1.0]) / np.linalg.norm([bx, by, -1.0])
    np.testing.assert_allclose(s.n[:, 0, :], np.broadcast_to(n, (rows * cols, 3)), atol=1e-12)
    # and then APSS keeps the plane
    t0 = s.t.copy()
    O.apss(s)
    np.testing.assert_allclose(s.t, t0, atol=1e-10)


def test_isolated_point_keeps_default_normal_and_depth(oracle_lib):
    p = oracle_lib.Params(dz=0.1, k_max=1)
    s = oracle_lib.State(1, 3, 3, 1)
    s.cnt[4] = 1
    s.t[4, 0] = 123.4
    s.n[4, 0, :] = [0.3, 0.0, -np.sqrt(1 - 0.09)]
    O = oracle_lib.Oracle(oracle_lib.Model([1.0], T=1000), p)
    O.apss(s)
    assert s.t[4, 0] == 123.4
    O.init_normals(s)
    np.testing.assert_array_equal(s.n[4, 0], [0.0, 0.0, -1.0])


def test_translation_covariance(oracle_lib):
    rng = np.random.default_rng(3)
    rows, cols, dz = 8, 9, 0.1
    p = oracle_lib.Params(dz=dz, k_max=2)
    s = grid_state(oracle_lib, rows, cols)
    i, j = np.mgrid[0:rows, 0:cols]
    s.t[:, 0] = ((20 + 0.2 * j + 0.1 * i + 0.02 * (i - 4) ** 2) / dz).reshape(-1) + rng.normal(0, 1.0, rows * cols)
    O = oracle_lib.Oracle(oracle_lib.Model([1.0], T=5000), p)
    O.init_normals(s)
    a = s.copy()
    b = s.copy()
    delta = 37.25
    b.t[:, 0] += delta
    O.apss(a)
    O.apss(b)
    np.testing.assert_allclose(b.t[:, 0] - delta, a.t[:, 0], atol=1e-9)
    np.testing.assert_allclose(b.n, a.n, atol=1e-12)
    assert np.abs(a.t - s.t).max() > 1e-3       # the step did move points


def test_window_neighbours_equal_brute_force(oracle_lib):
    rng = np.random.default_rng(11)
    rows, cols, K = 7, 8, 3
    for h_apss, p_xy, dz in ((2.0, 1.0, 0.1), (1.5, 0.7, 0.3), (3.0, 1.0, 1.0)):
        p = oracle_lib.Params(dz=dz, p_xy=p_xy, h_apss=h_apss, k_max=K)
        s = oracle_lib.State(1, rows, cols, K)
        s.cnt[:] = rng.integers(0, K + 1, rows * cols)
        for q in range(rows * cols):
            s.t[q, :s.cnt[q]] = np.sort(rng.uniform(100, 130, s.cnt[q]))
        O = oracle_lib.Oracle(oracle_lib.Model([1.0], T=1000), p)
        # brute force in numpy over every point of the frame
        pts, idx = [], []
        for q in range(rows * cols):
            for k in range(s.cnt[q]):
                pts.append([(q % cols) * p_xy, (q // cols) * p_xy, s.t[q, k] * dz])
                idx.append(q * K + k)
        pts, idx = np.array(pts), np.array(idx)
        for a in range(len(idx)):
            d2 = ((pts - pts[a]) ** 2).sum(1)
            expect = sorted(idx[d2 < h_apss ** 2])
            got = sorted(O.apss_neighbours(s, idx[a]))
            got_bf = sorted(O.apss_neighbours(s, idx[a], brute_force=True))
            assert got == expect == got_bf
