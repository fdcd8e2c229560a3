"""Pins of the oracle's impulse-response model against closed forms.

The paper takes the per-pixel IRF h as known (Results, Observation model).
The oracle's continuous h is the Catmull-Rom interpolant of the samples; these
tests pin it to facts that do not go through the oracle's own formula: the
Keys cubic-convolution kernel (Catmull-Rom is its a = -1/2 case), exact
reproduction of quadratics, interpolation at the samples, Sheppard's
correction for a binned Gaussian, and finite differences for derivatives.
"""
import numpy as np
import pytest
from scipy.stats import norm

pytestmark = pytest.mark.usefixtures("oracle_lib")


def keys(x, a=-0.5):
    x = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros_like(x)
    m1 = x <= 1
    m2 = (x > 1) & (x < 2)
    out[m1] = (a + 2) * x[m1] ** 3 - (a + 3) * x[m1] ** 2 + 1
    out[m2] = a * x[m2] ** 3 - 5 * a * x[m2] ** 2 + 8 * a * x[m2] - 4 * a
    return out


def test_spike_is_keys_kernel(oracle_lib):
    m = oracle_lib.Model([0.0, 0.0, 1.0, 0.0, 0.0], T=50, origin=2)
    tau = np.arange(-3 * 32, 3 * 32 + 1) / 32.0
    h, _ = m.h(tau)
    expect = np.maximum(keys(tau), 0.0)  # negative lobe of the kernel clamps to zero
    np.testing.assert_allclose(h, expect, atol=1e-15)


def test_quadratic_reproduced_between_interior_samples(oracle_lib):
    k = np.arange(21, dtype=np.float64)
    irf = 100.0 - (k - 10.0) ** 2
    m = oracle_lib.Model(irf, T=100, origin=10)
    s = irf.sum()
    pos = np.arange(1 * 32, 19 * 32 + 1) / 32.0          # sample positions 1..19
    h, _ = m.h(pos - 10.0)
    np.testing.assert_allclose(h, (100.0 - (pos - 10.0) ** 2) / s, rtol=0, atol=1e-14)


def test_interpolates_samples_and_origin(oracle_lib):
    rng = np.random.default_rng(7)
    irf = rng.uniform(0.1, 1.0, 13)
    m = oracle_lib.Model(irf, T=80)
    assert m.origin == int(np.argmax(irf))
    h, _ = m.h(np.arange(13) - m.origin)
    np.testing.assert_allclose(h, irf / irf.sum(), rtol=1e-15, atol=1e-17)
    h_out, hp_out = m.h(np.array([-m.origin - 1.0 - 1e-9, 13 - m.origin + 1e-9, 500.0]))
    assert np.all(h_out == 0) and np.all(hp_out == 0)


def test_derivatives_match_finite_differences(oracle_lib):
    irf = norm.pdf(np.arange(-9, 10), scale=1.5)
    m = oracle_lib.Model(irf, T=200)
    rng = np.random.default_rng(1)
    # positions strictly inside a fine-table segment (h and S are linear there)
    tau = (np.floor(rng.uniform(-8, 8, 50) * 32) + 0.5) / 32.0
    eps = 1e-5
    hp_fd = (m.h(tau + eps)[0] - m.h(tau - eps)[0]) / (2 * eps)
    np.testing.assert_allclose(m.h(tau)[1], hp_fd, rtol=1e-7, atol=1e-9)
    ts = (np.floor(rng.uniform(20, 180, 50) * 32) + 0.5) / 32.0
    S, Sp = m.S(ts)
    Sp_fd = (m.S(ts + eps)[0] - m.S(ts - eps)[0]) / (2 * eps)
    np.testing.assert_allclose(Sp, Sp_fd, rtol=1e-6, atol=1e-9)


def test_S_is_unit_at_interior_integers_and_falls_at_edges(oracle_lib):
    irf = norm.pdf(np.arange(-9, 10), scale=1.5)
    m = oracle_lib.Model(irf, T=100)
    S, _ = m.S(np.arange(12, 88, dtype=np.float64))
    np.testing.assert_allclose(S, 1.0, atol=1e-13)
    # at the first bin only the right half of the IRF falls inside the histogram
    S0, _ = m.S(np.array([0.0]))
    half = irf[9:].sum() / irf.sum()
    assert abs(S0[0] - half) < 1e-13


def test_variance_sheppard_and_two_point(oracle_lib):
    m2 = oracle_lib.Model([1.0, 1.0], T=10)
    assert abs(m2.sigma2 - 0.25) < 1e-15
    sig = 1.5
    lags = np.arange(-9, 10)
    binned = norm.cdf((lags + 0.5) / sig) - norm.cdf((lags - 0.5) / sig)
    mg = oracle_lib.Model(binned, T=300)
    assert abs(mg.sigma2 - (sig ** 2 + 1.0 / 12.0)) < 2e-4


def test_peak_window_from_cumulative_mass(oracle_lib):
    sig = 1.5
    lags = np.arange(-9, 10)
    binned = norm.cdf((lags + 0.5) / sig) - norm.cdf((lags - 0.5) / sig)
    m = oracle_lib.Model(binned, T=300)
    cdf_upper = norm.cdf((lags + 0.5) / sig)  # mass up to and including each lag
    lo = lags[np.argmax(cdf_upper >= 0.05)]
    hi = lags[np.argmax(cdf_upper >= 0.95)]
    assert m.window() == (-lo, hi)


def test_lmf_weights_zero_off_support_and_monotone(oracle_lib):
    irf = np.array([0.0, 1.0, 3.0, 2.0, 0.0])
    m = oracle_lib.Model(irf, T=64)
    q = m.lmf_table(1.0)
    assert q[0] == 0 and q[4] == 0
    assert q[2] > q[3] > q[1] > 0
    # log(1 + h T) at 16 fractional bits
    assert abs(q[2] / 65536.0 - np.log1p(0.5 * 64)) < 1e-4


def test_invalid_irf_rejected(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.Model([0.0, 0.0], T=10)
    with pytest.raises(ValueError):
        oracle_lib.Model([1.0, -1.0, 2.0], T=10)
    with pytest.raises(ValueError):
        oracle_lib.Model(np.ones(11), T=10)


def test_fisher_information_of_binned_gaussian(oracle_lib):
    # Fisher information about the shift theta of a binned Gaussian,
    # p_k(theta) = Phi((k + 1/2 - theta)/s) - Phi((k - 1/2 - theta)/s),
    # I(theta) = sum_k p_k'(theta)^2 / p_k(theta), averaged over theta in [0, 1)
    sig = 2.5
    lags = np.arange(-15, 16)
    binned = norm.cdf((lags + 0.5) / sig) - norm.cdf((lags - 0.5) / sig)
    m = oracle_lib.Model(binned, T=400)
    vals = []
    for th in np.arange(64) / 64.0:
        p = norm.cdf((lags + 0.5 - th) / sig) - norm.cdf((lags - 0.5 - th) / sig)
        dp = (norm.pdf((lags - 0.5 - th) / sig) - norm.pdf((lags + 0.5 - th) / sig)) / sig
        vals.append(np.sum(dp ** 2 / p))
    exact = np.mean(vals)
    assert abs(m.fisher / exact - 1) < 2e-2
    # and a wider Gaussian approaches the continuous value 1/sigma^2
    assert abs(exact * sig ** 2 - 1) < 0.02
