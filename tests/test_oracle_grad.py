"""Pins of the oracle's Poisson negative log-likelihood and its gradients.

The observation model and the negative log-likelihood are those of the
paper's Results, "Observation model".  The oracle evaluates the NLL over
active bins only; these tests pin it to the Poisson pmf summed over every bin
(scipy), to a hand-built case, to central finite differences (the gradients),
and to the closed-form stationary points of the background and of a single
intensity.
"""
import numpy as np
import pytest
from scipy.stats import norm, poisson

pytestmark = pytest.mark.usefixtures("oracle_lib")


def small_problem(oracle, seed=0, rows=3, cols=4, T=60, dead=True):
    rng = np.random.default_rng(seed)
    irf = norm.pdf(np.arange(-9, 10), scale=1.5)
    m = oracle.Model(irf, T=T)
    K = 3
    s = oracle.State(1, rows, cols, K)
    npix = rows * cols
    s.g = rng.uniform(0.5, 1.5, npix)
    if dead:
        s.g[1] = 0.0
    for p in range(npix):
        c = rng.integers(0, K + 1)
        s.cnt[p] = c
        # depths away from the fine-table knots (multiples of 1/32)
        ts = np.sort(rng.choice(np.arange(12, T - 12), c, replace=False)).astype(float)
        ts += (rng.integers(0, 32, c) + rng.uniform(0.2, 0.8, c)) / 32.0
        s.t[p, :c] = ts
        s.r[p, :c] = rng.uniform(1.0, 6.0, c)
    s.b[:] = rng.uniform(0.01, 0.2, npix)
    Z = rng.poisson(2.0, (rows, cols, T)) * (rng.random((rows, cols, T)) < 0.3)
    Z = Z.astype(np.uint16)
    off, ent = oracle.compact(Z)
    return m, s, Z, off, ent


def test_nll_sparse_equals_scipy_dense(oracle_lib):
    m, s, Z, off, ent = small_problem(oracle_lib)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3))
    val = O.nll(off, ent, s)
    # independent dense evaluation: lambda from the model's h, pmf from scipy
    T = m.T
    total = 0.0
    for p in range(s.npix):
        if s.g[p] <= 0:
            continue
        lam = np.full(T, s.b[p])
        for k in range(s.cnt[p]):
            lam += s.r[p, k] * m.h(np.arange(T) - s.t[p, k])[0]
        lam *= s.g[p]
        total -= poisson.logpmf(Z.reshape(-1, T)[p], lam).sum()
    assert abs(val - total) <= 1e-10 * abs(total)
    assert abs(O.nll_dense(Z, s) - total) <= 1e-10 * abs(total)


def test_nll_hand_case(oracle_lib):
    # unit spike IRF: a point at integer depth 2 puts all its light in bin 2
    m = oracle_lib.Model([1.0], T=5, origin=0)
    s = oracle_lib.State(1, 1, 1, 1)
    s.cnt[0] = 1
    s.t[0, 0] = 2.0
    s.r[0, 0] = 3.0
    s.b[0] = 0.5
    s.g[0] = 2.0
    Z = np.array([[[0, 1, 4, 0, 2]]], dtype=np.uint16)
    off, ent = oracle_lib.compact(Z)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1))
    lam = np.array([1.0, 1.0, 7.0, 1.0, 1.0])  # 2 * (3 * [0,0,1,0,0] + 0.5)
    expect = -poisson.logpmf([0, 1, 4, 0, 2], lam).sum()
    assert abs(O.nll(off, ent, s) - expect) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradients_match_central_differences(oracle_lib, seed):
    m, s, Z, off, ent = small_problem(oracle_lib, seed=seed)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3))
    (gt, gr, gb), (at, ar, ab) = O.grad(off, ent, s)
    for p in range(s.npix):
        for k in range(s.cnt[p]):
            for arr, g_an, scale, eps in ((s.t, gt, at, 1e-6), (s.r, gr, ar, 1e-7 * s.r[p, k])):
                x0 = arr[p, k]
                arr[p, k] = x0 + eps
                fp = O.nll(off, ent, s)
                arr[p, k] = x0 - eps
                fm = O.nll(off, ent, s)
                arr[p, k] = x0
                fd = (fp - fm) / (2 * eps)
                # the FD error of a sum of ~1e3 terms is ~1e-9 relative
                assert abs(fd - g_an[p, k]) <= 1e-6 * scale[p, k] + 1e-6, (p, k, fd, g_an[p, k])
        eps = 1e-7 * s.b[p]
        b0 = s.b[p]
        s.b[p] = b0 + eps
        fp = O.nll(off, ent, s)
        s.b[p] = b0 - eps
        fm = O.nll(off, ent, s)
        s.b[p] = b0
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - gb[p]) <= 1e-6 * ab[p] + 1e-6, (p, fd, gb[p])
    # dead pixels have zero gradients
    assert gb[1] == 0 and np.all(gt[1] == 0) and np.all(gr[1] == 0)


def test_background_stationary_point(oracle_lib):
    # no points: dNLL/db = g (T - Z/b) vanishes at b* = Z/(g T)
    m = oracle_lib.Model([1.0, 2.0, 1.0], T=40)
    s = oracle_lib.State(1, 1, 2, 1)
    s.g[:] = [1.3, 0.7]
    Z = np.zeros((1, 2, 40), dtype=np.uint16)
    Z[0, 0, [3, 9, 20]] = [1, 2, 4]
    Z[0, 1, [0, 39]] = [5, 1]
    off, ent = oracle_lib.compact(Z)
    s.b[:] = Z.reshape(2, -1).sum(1) / (s.g * 40)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1))
    (_, _, gb), _ = O.grad(off, ent, s)
    np.testing.assert_allclose(gb, 0.0, atol=1e-12)


def test_single_intensity_stationary_point(oracle_lib):
    # one point, no background, photons inside its support:
    # dNLL/dr = g S - Z / r vanishes at r* = Z / (g S)
    irf = norm.pdf(np.arange(-6, 7), scale=1.2)
    m = oracle_lib.Model(irf, T=50)
    s = oracle_lib.State(1, 1, 1, 1)
    s.cnt[0] = 1
    s.t[0, 0] = 24.37
    s.g[0] = 0.8
    s.b[0] = 0.0
    Z = np.zeros((1, 1, 50), dtype=np.uint16)
    Z[0, 0, [21, 23, 24, 25, 27]] = [1, 3, 5, 2, 1]
    off, ent = oracle_lib.compact(Z)
    S, _ = m.S(np.array([24.37]))
    s.r[0, 0] = 12.0 / (0.8 * S[0])
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1))
    (_, gr, _), (_, ar, _) = O.grad(off, ent, s)
    assert abs(gr[0, 0]) < 1e-12 * ar[0, 0]
