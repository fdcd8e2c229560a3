"""Pins of the oracle's super-resolved observation model (Results, dynamic
scenes; Discussion): the map f sends the s x s point-grid pixels of a block
to one lidar pixel, whose Poisson intensity adds all their points.

The NLL is pinned to the Poisson pmf summed over every bin with the
point-grid-to-lidar mapping written independently (a numpy reshape), the
gradients to central differences, s = 1 to the plain model, the scatter of
the lidar pixel's residual back to its points to the plain step of one point
carrying the block's whole intensity, and the intensity step to the photon
balance of expectation-maximisation.
"""
import numpy as np
import pytest
from scipy.stats import norm, poisson

pytestmark = pytest.mark.usefixtures("oracle_lib")


def sr_problem(oracle, seed=0, s=2, rows=2, cols=3, T=60, K=3, dead=True):
    """Random points on the (rows s) x (cols s) point grid and photon counts
    on the rows x cols lidar grid."""
    rng = np.random.default_rng(1000 + seed)
    m = oracle.Model(norm.pdf(np.arange(-9, 10), scale=1.5), T=T)
    st = oracle.SRState(1, rows, cols, s, K)
    st.g[:] = rng.uniform(0.5, 1.5, rows * cols)
    if dead:
        st.g[1] = 0.0
    for q in range(st.npix):
        c = rng.integers(0, K + 1)
        st.cnt[q] = c
        ts = np.sort(rng.choice(np.arange(12, T - 12), c, replace=False)).astype(float)
        st.t[q, :c] = ts + rng.uniform(0.05, 0.95, c)
        st.r[q, :c] = rng.uniform(0.5, 3.0, c)
    st.b[:] = rng.uniform(0.01, 0.2, rows * cols)
    Z = (rng.poisson(3.0, (rows, cols, T)) * (rng.random((rows, cols, T)) < 0.3)).astype(np.uint16)
    off, ent = oracle.compact(Z)
    return m, st, Z, off, ent


def blocks(st):
    """Point-grid pixel numbers of each lidar pixel, [lidar pixels, s^2]."""
    R, C, s = st.rows, st.cols, st.s
    idx = np.arange(st.F * R * C).reshape(st.F, st.lrows, s, st.lcols, s)
    return idx.transpose(0, 1, 3, 2, 4).reshape(-1, s * s)


@pytest.mark.parametrize("s", [2, 3])
def test_sr_nll_equals_dense_poisson_over_blocks(oracle_lib, s):
    m, st, Z, off, ent = sr_problem(oracle_lib, seed=s, s=s)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3))
    T = m.T
    total = 0.0
    for p, qs in enumerate(blocks(st)):
        if st.g[p] <= 0:
            continue
        lam = np.full(T, st.b[p])
        for q in qs:
            for k in range(st.cnt[q]):
                lam += st.r[q, k] * m.h(np.arange(T) - st.t[q, k])[0]
        total -= poisson.logpmf(Z.reshape(-1, T)[p], st.g[p] * lam).sum()
    assert abs(O.sr_nll(off, ent, st) - total) <= 1e-10 * abs(total)


@pytest.mark.parametrize("seed", [0, 1])
def test_sr_gradients_match_central_differences(oracle_lib, seed):
    m, st, Z, off, ent = sr_problem(oracle_lib, seed=seed, s=2)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3))
    (gt, gr, gb), (at, ar, ab) = O.sr_grad(off, ent, st)

    def central(arr, idx, eps):
        x0 = arr[idx]
        arr[idx] = x0 + eps
        fp = O.sr_nll(off, ent, st)
        arr[idx] = x0 - eps
        fm = O.sr_nll(off, ent, st)
        arr[idx] = x0
        return (fp - fm) / (2 * eps)

    for q in range(st.npix):
        for k in range(st.cnt[q]):
            fd = central(st.t, (q, k), 1e-6)
            assert abs(fd - gt[q, k]) <= 1e-6 * at[q, k] + 1e-6, (q, k, fd, gt[q, k])
            fd = central(st.r, (q, k), 1e-7 * st.r[q, k])
            assert abs(fd - gr[q, k]) <= 1e-6 * ar[q, k] + 1e-6, (q, k, fd, gr[q, k])
    for p in range(st.b.size):
        fd = central(st.b, p, 1e-7 * st.b[p])
        assert abs(fd - gb[p]) <= 1e-6 * ab[p] + 1e-6, (p, fd, gb[p])
    dead = blocks(st)[1]
    assert gb[1] == 0 and np.all(gt[dead] == 0) and np.all(gr[dead] == 0)


def test_sr_with_one_point_grid_pixel_per_lidar_pixel_is_the_plain_model(oracle_lib):
    m, st, Z, off, ent = sr_problem(oracle_lib, seed=5, s=1, rows=3, cols=4)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3))
    plain = oracle_lib.State(1, 3, 4, 3, st.g.copy())
    for a in ("t", "r", "n", "cnt", "b"):
        setattr(plain, a, getattr(st, a).copy())
    assert O.sr_nll(off, ent, st) == O.nll(off, ent, plain)
    for x, y in zip(O.sr_grad(off, ent, st)[0], O.grad(off, ent, plain)[0]):
        np.testing.assert_array_equal(x, y)
    a, b = st.copy(), plain.copy()
    for sr_step, step in ((O.sr_depth_step, O.depth_step), (O.sr_intensity_step, O.intensity_step),
                          (O.sr_bg_step, O.bg_step)):
        sr_step(off, ent, a)
        step(off, ent, b)
        for name in ("t", "r", "b"):
            np.testing.assert_array_equal(getattr(a, name), getattr(b, name), err_msg=sr_step.__name__)
    O.sr_iterate(off, ent, a)
    O.iterate(off, ent, b)
    for name in ("t", "r", "n", "cnt", "b"):
        np.testing.assert_array_equal(getattr(a, name), getattr(b, name), err_msg=name)


@pytest.mark.parametrize("s", [2, 3])
def test_sr_points_copied_over_a_block_step_like_one_point(oracle_lib, s):
    """Every point-grid pixel of a block holding the same points, with 1/s^2 of
    the intensity each, gives the lidar pixel the lambda of one pixel holding
    the points at full intensity: the depth and background steps are then the
    plain ones, the intensity step the plain one divided by s^2."""
    m, plain, Z, off, ent = sr_problem(oracle_lib, seed=7, s=1, rows=2, cols=3)
    P = oracle_lib.Params(k_max=3)
    O = oracle_lib.Oracle(m, P)
    st = oracle_lib.SRState(1, 2, 3, s, 3, plain.g.copy())
    O.sr_expand(plain, st)
    np.testing.assert_array_equal(st.b, plain.b)
    for p, qs in enumerate(blocks(st)):
        for q in qs:
            assert st.cnt[q] == plain.cnt[p]
            np.testing.assert_array_equal(st.t[q], plain.t[p])
            np.testing.assert_allclose(st.r[q], plain.r[p] / s ** 2, rtol=1e-15)
    a, b = st.copy(), plain.copy()
    O.sr_depth_step(off, ent, a)
    O.depth_step(off, ent, b)
    O.sr_intensity_step(off, ent, a)
    O.intensity_step(off, ent, b)
    O.sr_bg_step(off, ent, a)
    O.bg_step(off, ent, b)
    for p, qs in enumerate(blocks(a)):
        for q in qs:
            np.testing.assert_allclose(a.t[q], b.t[p], rtol=1e-13, atol=1e-12)
            np.testing.assert_allclose(a.r[q], b.r[p] / s ** 2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(a.b, b.b, rtol=1e-12)


def test_sr_intensity_step_balances_photons(oracle_lib):
    """At beta_r = 1 the step is expectation-maximisation: for a lidar pixel
    with gain 1, sum over its points of r_new S(t) = sum_e z (lambda_e - b)/lambda_e
    (lambda from the old intensities)."""
    m, st, Z, off, ent = sr_problem(oracle_lib, seed=3, s=2, dead=False)
    st.g[:] = 1.0
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3, beta_r=1.0))
    before = st.copy()
    O.sr_intensity_step(off, ent, st)
    T = m.T
    for p, qs in enumerate(blocks(st)):
        lam = np.full(T, before.b[p])
        lhs = 0.0
        for q in qs:
            for k in range(st.cnt[q]):
                lam += before.r[q, k] * m.h(np.arange(T) - before.t[q, k])[0]
                lhs += st.r[q, k] * m.S(np.array([st.t[q, k]]))[0][0]
        z = Z.reshape(-1, T)[p].astype(float)
        rhs = np.sum(z * (lam - before.b[p]) / lam)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, rhs), (p, lhs, rhs)


def test_sr_reconstruction_resolves_below_the_lidar_pixel(oracle_lib):
    """Strong noiseless-background data of a tilted plane seen by 12 x 12 lidar
    pixels: the super-resolved cloud on the 36 x 36 point grid follows the
    plane's slope inside each lidar pixel, which one depth per lidar pixel
    cannot."""
    from paper_1905_06700_amd import synth
    sc = synth.sr_scene(0, rows=12, cols=12, s=3, T=120, signal=9 * 400.0, sbr=1e6, theta=0.5)
    m = oracle_lib.Model(sc.irf.probs, sc.T)
    off, ent = oracle_lib.compact(sc.Z)
    me = sc.meta
    # one surface only: the disc is moved out of this frame's interior checks
    truth = sc.depth[0]
    P = oracle_lib.Params(dz=me["dz"], p_xy=me["p_xy"], r_min=me["r_min"], k_init=1, k_max=4)
    O = oracle_lib.Oracle(m, P)
    st = O.sr_reconstruct(off, ent, oracle_lib.SRState(1, 12, 12, 3, 4))
    first = np.where(st.cnt > 0, st.t[:, 0], np.nan).reshape(36, 36)
    # compare away from the disc edge (two surfaces in one lidar pixel) and the frame border
    i, j = np.mgrid[0:36, 0:36]
    edge = np.zeros((36, 36), bool)
    d = truth
    for di in (-4, 0, 4):
        for dj in (-4, 0, 4):
            edge |= np.abs(np.roll(np.roll(d, di, 0), dj, 1) - d) > 10
    keep = ~edge & (i >= 4) & (i < 32) & (j >= 4) & (j < 32) & (st.cnt.reshape(36, 36) > 0)
    assert keep.sum() > 200
    err_sr = np.abs(first - truth)[keep]
    # the same data with one depth per lidar pixel, repeated over its block
    Oc = oracle_lib.Oracle(m, oracle_lib.Params(dz=0.1, p_xy=1.0, r_min=me["r_min"] * 9, k_init=1, k_max=4))
    sc_state = Oc.reconstruct(off, ent, oracle_lib.State(1, 12, 12, 4))
    coarse = np.where(sc_state.cnt > 0, sc_state.t[:, 0], np.nan).reshape(12, 12)
    err_coarse = np.abs(np.kron(coarse, np.ones((3, 3))) - truth)[keep]
    print(f"sr rms {np.sqrt(np.mean(err_sr ** 2)):.3f} bins, coarse rms {np.sqrt(np.mean(err_coarse ** 2)):.3f}")
    assert np.sqrt(np.mean(err_sr ** 2)) < 0.6 * np.sqrt(np.mean(err_coarse ** 2))
