"""Pins of the oracle's per-pixel IRFs (Results, "Observation model": the
response h_ij is known per pixel).  Pixel p's likelihood uses its own IRF.

The NLL is pinned to the Poisson pmf summed over every bin with each pixel's
own h, the gradients to central differences.  Per-pixel work is independent,
so a map of two IRF classes must reproduce, pixel by pixel, the plain model
run with each class's IRF everywhere.  The merge distance follows the pixel's
own IRF width.
"""
import numpy as np
import pytest
from scipy.stats import norm, poisson

pytestmark = pytest.mark.usefixtures("oracle_lib")

T = 70


def models(oracle):
    """Class 0: Gaussian sigma 1.2 bins; class 1: sigma 3 bins with an
    exponential tail (another length and origin)."""
    a = oracle.Model(norm.pdf(np.arange(-7, 8), scale=1.2), T=T)
    x = np.arange(-12, 30)
    tail = np.exp(-np.clip(x, 0, None) / 6.0) * (x >= 0)
    b = oracle.Model(np.convolve(norm.pdf(np.arange(-9, 10), scale=3.0), tail)[:50] + 1e-4, T=T)
    return a, b


def problem(oracle, seed=0, rows=3, cols=4, K=3):
    rng = np.random.default_rng(2000 + seed)
    st = oracle.State(1, rows, cols, K)
    npix = rows * cols
    st.g = rng.uniform(0.5, 1.5, npix)
    st.g[5] = 0.0
    for p in range(npix):
        c = rng.integers(0, K + 1)
        st.cnt[p] = c
        ts = np.sort(rng.choice(np.arange(15, T - 25), c, replace=False)).astype(float)
        st.t[p, :c] = ts + rng.uniform(0.05, 0.95, c)
        st.r[p, :c] = rng.uniform(1.0, 6.0, c)
    st.b[:] = rng.uniform(0.01, 0.2, npix)
    Z = (rng.poisson(2.0, (rows, cols, T)) * (rng.random((rows, cols, T)) < 0.3)).astype(np.uint16)
    cls = rng.integers(0, 2, npix).astype(np.uint8)
    cls[0], cls[1] = 0, 1
    off, ent = oracle.compact(Z)
    return st, Z, off, ent, cls


def test_per_pixel_irf_nll_equals_dense_poisson(oracle_lib):
    a, b = models(oracle_lib)
    st, Z, off, ent, cls = problem(oracle_lib)
    O = oracle_lib.Oracle(a, oracle_lib.Params(k_max=3), irf_models=[b], irf_class=cls)
    total = 0.0
    for p in range(st.npix):
        if st.g[p] <= 0:
            continue
        m = (a, b)[cls[p]]
        lam = np.full(T, st.b[p])
        for k in range(st.cnt[p]):
            lam += st.r[p, k] * m.h(np.arange(T) - st.t[p, k])[0]
        total -= poisson.logpmf(Z.reshape(-1, T)[p], st.g[p] * lam).sum()
    assert abs(O.nll(off, ent, st) - total) <= 1e-10 * abs(total)
    assert abs(O.nll_dense(Z, st) - total) <= 1e-10 * abs(total)


def test_per_pixel_irf_gradients_match_central_differences(oracle_lib):
    a, b = models(oracle_lib)
    st, Z, off, ent, cls = problem(oracle_lib, seed=1)
    O = oracle_lib.Oracle(a, oracle_lib.Params(k_max=3), irf_models=[b], irf_class=cls)
    (gt, gr, gb), (at, ar, ab) = O.grad(off, ent, st)

    def central(arr, idx, eps):
        x0 = arr[idx]
        arr[idx] = x0 + eps
        fp = O.nll(off, ent, st)
        arr[idx] = x0 - eps
        fm = O.nll(off, ent, st)
        arr[idx] = x0
        return (fp - fm) / (2 * eps)

    for p in range(st.npix):
        for k in range(st.cnt[p]):
            fd = central(st.t, (p, k), 1e-6)
            assert abs(fd - gt[p, k]) <= 1e-6 * at[p, k] + 1e-6, (p, k, fd, gt[p, k])
            fd = central(st.r, (p, k), 1e-7 * st.r[p, k])
            assert abs(fd - gr[p, k]) <= 1e-6 * ar[p, k] + 1e-6, (p, k, fd, gr[p, k])
        fd = central(st.b, p, 1e-7 * st.b[p])
        assert abs(fd - gb[p]) <= 1e-6 * ab[p] + 1e-6, (p, fd, gb[p])


def test_per_pixel_irf_steps_equal_the_plain_model_of_each_class(oracle_lib):
    st, Z, off, ent, cls = problem(oracle_lib, seed=2, rows=5, cols=6)
    P = oracle_lib.Params(k_max=3, r_init=0, k_init=2)
    a, b = models(oracle_lib)
    mixed = oracle_lib.Oracle(a, P, irf_models=[b], irf_class=cls)
    plain = []
    for m in models(oracle_lib):
        plain.append(oracle_lib.Oracle(m, P))

    def run(O, s, name):
        s = s.copy()
        if name == "init":
            return O.init(off, ent, s, normals=False)
        getattr(O, name)(off, ent, s)
        return s

    for name in ("init", "depth_step", "intensity_step", "bg_step"):
        got = run(mixed, st, name)
        ref = [run(O, st, name) for O in plain]
        for p in range(st.npix):
            want = ref[cls[p]]
            assert got.cnt[p] == want.cnt[p], (name, p)
            np.testing.assert_array_equal(got.t[p], want.t[p], err_msg=f"{name} t {p}")
            np.testing.assert_array_equal(got.r[p], want.r[p], err_msg=f"{name} r {p}")
            assert got.b[p] == want.b[p], (name, p)
    # a class number past the models counts as class 0
    far = cls.copy()
    far[cls == 1] = 9
    O9 = oracle_lib.Oracle(models(oracle_lib)[0], P, irf_models=[models(oracle_lib)[1]], irf_class=far)
    got = run(O9, st, "depth_step")
    np.testing.assert_array_equal(got.t, run(plain[0], st, "depth_step").t)


def test_merge_distance_follows_each_pixel_irf(oracle_lib):
    a, b = models(oracle_lib)
    da, db = max(1.0, np.sqrt(a.sigma2)), max(1.0, np.sqrt(b.sigma2))
    assert db > da + 1.0
    st = oracle_lib.State(1, 1, 2, 2)
    gap = 0.5 * (da + db)                     # apart for the narrow IRF, coincident for the wide one
    st.cnt[:] = 2
    st.t[:, 0], st.t[:, 1] = 30.0, 30.0 + gap
    st.r[:] = 2.0
    O = oracle_lib.Oracle(a, oracle_lib.Params(k_max=2), irf_models=[b], irf_class=np.array([0, 1], np.uint8))
    O.merge(st)
    assert list(st.cnt) == [2, 1]
    assert st.t[1, 0] == pytest.approx(30.0 + gap / 2) and st.r[1, 0] == 4.0
