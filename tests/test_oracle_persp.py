"""Pins of the oracle's perspective camera (Observation model: the map f takes
the camera's parameters, such as its focal length).  Reading: a pinhole at
the origin looking along +Z; pixel (i, j) sees along the unit ray of
(a (j - cx), a (i - cy), 1), cx = (cols - 1)/2, cy = (rows - 1)/2, and depth t
is the range t dz along that ray.

The points below are placed by the test itself where each pixel's ray meets
a world plane or sphere (an independent statement of the geometry): APSS must
leave them and their normals in place (its algebraic sphere reproduces planes
and spheres exactly), the initial normals of plane points must be the
plane's normal facing the sensor, and the windowed neighbour search must
equal brute force.  A wrong ray direction, range convention or principal
point moves the points off the surface in the oracle's geometry and fails
these tests.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")

A = 0.05       # tangent of one pixel's angle
DZ = 0.1


def rays(rows, cols, a=A):
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    v = np.stack([a * (j - (cols - 1) / 2), a * (i - (rows - 1) / 2), np.ones_like(i)], axis=-1)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def state_from(oracle, rho, normals, rows, cols):
    s = oracle.State(1, rows, cols, 4)
    s.cnt[:] = 1
    s.t[:, 0] = (rho / DZ).reshape(-1)
    s.r[:, 0] = 5.0
    s.n[:, 0] = normals.reshape(-1, 3)
    return s


def plane_points(rows, cols):
    nrm = np.array([0.3, -0.2, -1.0])
    nrm /= np.linalg.norm(nrm)                 # faces the sensor (n_z < 0)
    d0 = -20.0 / np.sqrt(1 + 0.3 ** 2 + 0.2 ** 2)  # n . x = d0: the plane passes near (0, 0, 20)
    v = rays(rows, cols)
    rho = d0 / (v @ nrm)
    return rho, np.broadcast_to(nrm, v.shape).copy(), v


def sphere_points(rows, cols, C=np.array([0.4, -0.3, 30.0]), Rs=20.0):
    v = rays(rows, cols)
    b = v @ C
    disc = b * b - C @ C + Rs * Rs
    assert np.all(disc > 0)                      # every ray meets the sphere
    rho = b - np.sqrt(disc)                      # the near intersection
    x = rho[..., None] * v
    return rho, (x - C) / Rs, v


def params(oracle, **kw):
    return oracle.Params(k_max=4, dz=DZ, p_xy=0.7, h_apss=2.0, persp=A, **kw)


@pytest.mark.parametrize("surface", ["plane", "sphere"])
def test_perspective_apss_keeps_points_on_planes_and_spheres(oracle_lib, surface):
    rows, cols = 19, 23
    rho, normals, v = (plane_points if surface == "plane" else sphere_points)(rows, cols)
    s = state_from(oracle_lib, rho, normals, rows, cols)
    O = oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=400), params(oracle_lib))
    s0 = s.copy()
    O.apss(s)
    np.testing.assert_allclose(s.t[:, 0], s0.t[:, 0], atol=1e-7)
    np.testing.assert_allclose(s.n[:, 0], s0.n[:, 0], atol=1e-7)
    # sanity of the setting: the fit moves points that are off the surface
    s1 = s0.copy()
    s1.t[200, 0] += 3.0
    O.apss(s1)
    assert abs(s1.t[200, 0] - s0.t[200, 0]) < 2.5      # pulled back towards the surface


def test_perspective_initial_normals_of_a_plane(oracle_lib):
    rows, cols = 19, 23
    rho, normals, v = plane_points(rows, cols)
    s = state_from(oracle_lib, rho, np.zeros_like(normals), rows, cols)
    O = oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=400), params(oracle_lib))
    O.init_normals(s)
    np.testing.assert_allclose(s.n[:, 0], normals.reshape(-1, 3), atol=1e-9)
    assert np.all(np.einsum("pc,pc->p", s.n[:, 0], v.reshape(-1, 3)) < 0)


def test_perspective_windowed_neighbours_equal_brute_force(oracle_lib):
    rows, cols = 15, 17
    rho, normals, _ = sphere_points(rows, cols)
    s = state_from(oracle_lib, rho, normals, rows, cols)
    rng = np.random.default_rng(3)
    s.cnt[rng.random(rows * cols) < 0.3] = 2               # a second surface 1.5 world units behind
    s.t[:, 1] = s.t[:, 0] + 15.0
    # a pixel's footprint here is at least ~0.6 world units: R = ceil(2 / 0.45) = 5 pixels cover h
    O = oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=400),
                          oracle_lib.Params(k_max=4, dz=DZ, p_xy=0.45, h_apss=2.0, persp=A))
    for q in range(0, rows * cols * 4, 7):
        if q % 4 >= s.cnt[q // 4]:
            continue
        a = set(O.apss_neighbours(s, q).tolist())
        b = set(O.apss_neighbours(s, q, brute_force=True).tolist())
        assert a == b, q
    # and with the orthographic map the same depths give other neighbourhoods
    Oo = oracle_lib.Oracle(oracle_lib.Model([1.0, 2.0, 1.0], T=400),
                           oracle_lib.Params(k_max=4, dz=DZ, p_xy=0.45, h_apss=2.0))
    q = (7 * cols + 8) * 4
    assert set(Oo.apss_neighbours(s, q).tolist()) != set(O.apss_neighbours(s, q).tolist())
