"""Pins of the oracle's per-step functions.

Each test fixes a step of the reconstruction loop (Results, "Reconstruction
algorithm"; Methods) to something outside the oracle: numpy for compaction,
exhaustive float64 search for the log-matched-filter peak, closed-form
expectation-maximisation fixed points for the intensity and background
steps, hand-built cases for merge and the intensity graph, and numpy's FFT
for the circular background filter.
"""
import numpy as np
import pytest
from scipy.stats import norm

from paper_1905_06700_amd import synth

pytestmark = pytest.mark.usefixtures("oracle_lib")


# ---------------------------------------------------------------- compaction

def test_compaction_equals_numpy_nonzero(oracle_lib):
    rng = np.random.default_rng(0)
    for shape in [(1, 1, 7), (5, 3, 64), (2, 4, 4, 301)]:
        Z = (rng.poisson(0.4, shape) * (rng.random(shape) < 0.5)).astype(np.uint16)
        Z.reshape(-1)[:3] = [65534, 1, 0]
        off, ent = oracle_lib.compact(Z)
        T = shape[-1]
        Zf = Z.reshape(-1, T)
        for p in range(Zf.shape[0]):
            nz = np.nonzero(Zf[p])[0]
            e = ent[off[p]:off[p + 1]]
            np.testing.assert_array_equal(e >> 16, nz)
            np.testing.assert_array_equal(e & 0xFFFF, Zf[p, nz])
        assert off[-1] == np.count_nonzero(Z)
        assert int((ent & 0xFFFF).sum()) == int(Z.sum())


def test_compaction_empty(oracle_lib):
    off, ent = oracle_lib.compact(np.zeros((3, 10), dtype=np.uint16))
    assert ent.size == 0 and np.all(off == 0)


def test_compaction_of_events_hand_case(oracle_lib):
    # photons of 3 pixels x 5 bins: pixel 0 gets bin 3 twice and bin 1 once,
    # pixel 1 nothing, pixel 2 bin 0 once -- in scrambled order
    off, ent = oracle_lib.compact_events([0, 2, 0, 0], [3, 0, 1, 3], 3, 5)
    np.testing.assert_array_equal(off, [0, 2, 2, 3])
    np.testing.assert_array_equal(ent, [(1 << 16) | 1, (3 << 16) | 2, (0 << 16) | 1])


def test_compaction_of_events_is_order_free_and_conserves_photons(oracle_lib):
    rng = np.random.default_rng(3)
    npix, T = 40, 97
    pix = rng.integers(0, npix, 3000)
    bins = rng.integers(0, T, 3000)
    off, ent = oracle_lib.compact_events(pix, bins, npix, T)
    perm = rng.permutation(pix.size)
    off2, ent2 = oracle_lib.compact_events(pix[perm], bins[perm], npix, T)
    np.testing.assert_array_equal(off, off2)
    np.testing.assert_array_equal(ent, ent2)
    assert int((ent & 0xFFFF).sum()) == pix.size
    for p in range(npix):                       # per pixel: distinct bins ascending, counts by brute force
        e = ent[off[p]:off[p + 1]]
        mine = bins[pix == p]
        np.testing.assert_array_equal(e >> 16, np.unique(mine))
        np.testing.assert_array_equal(e & 0xFFFF, [(mine == b).sum() for b in np.unique(mine)])


# ---------------------------------------------------------------- initialisation

def gauss_model(oracle, T, sig=1.5, half=9):
    lags = np.arange(-half, half + 1)
    return oracle.Model(norm.cdf((lags + 0.5) / sig) - norm.cdf((lags - 0.5) / sig), T=T)


def test_lmf_single_photon_peaks_at_its_bin(oracle_lib):
    m = gauss_model(oracle_lib, 100)
    for tb in (0, 7, 50, 99):
        Z = np.zeros((1, 1, 100), dtype=np.uint16)
        Z[0, 0, tb] = 1
        off, ent = oracle_lib.compact(Z)
        s = oracle_lib.State(1, 1, 1, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(n_min=1, kappa=0.0, k_init=1))
        O.init(off, ent, s)
        assert s.cnt[0] == 1 and s.t[0, 0] == tb


def test_lmf_noiseless_template_recovers_depth(oracle_lib):
    irf = np.array([1.0, 2.0, 4.0, 7.0, 5.0, 3.0, 2.0, 1.0])
    m = oracle_lib.Model(irf, T=200)
    for d in (3, 60, 196):
        Z = np.zeros((1, 1, 200), dtype=np.uint16)
        for k, v in enumerate(irf):
            tb = d + k - 3
            if 0 <= tb < 200:
                Z[0, 0, tb] = int(v * 100)
        off, ent = oracle_lib.compact(Z)
        s = oracle_lib.State(1, 1, 1, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=1))
        O.init(off, ent, s)
        assert s.cnt[0] == 1 and s.t[0, 0] == d


def test_lmf_argmax_matches_exhaustive_float_search(oracle_lib):
    """Peak = argmax over tau of sum z log(h(t - tau) + eps), by brute force."""
    rng = np.random.default_rng(5)
    T = 150
    m = gauss_model(oracle_lib, T)
    hbar = m.h(np.arange(-9, 10))[0]
    eps = 1.0 / T
    for trial in range(20):
        Z = rng.poisson(0.05, (1, 1, T)).astype(np.uint16)
        d = rng.integers(10, 140)
        Z[0, 0, d - 2:d + 3] += rng.poisson(3.0, 5).astype(np.uint16)
        off, ent = oracle_lib.compact(Z)
        z = Z[0, 0].astype(float)
        score = np.array([sum(z[t] * (np.log(m.h(t - tau)[0][0] + eps) - np.log(eps))
                              for t in np.nonzero(z)[0]) for tau in range(T)])
        best = int(np.argmax(score))
        srt = np.sort(score)
        if srt[-1] - srt[-2] < 1e-3:
            continue                                   # near tie: fixed point rounding decides
        s = oracle_lib.State(1, 1, 1, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(n_min=1, kappa=0.0, k_init=1))
        O.init(off, ent, s)
        assert s.cnt[0] == 1 and s.t[0, 0] == best
        assert hbar is not None


def test_lmf_intensity_and_background_closed_form(oracle_lib):
    # one surface, no background photons: r0 = photons / (g * IRF mass in window),
    # background = b_min
    irf = np.array([1.0, 3.0, 6.0, 3.0, 1.0])
    m = oracle_lib.Model(irf, T=100)
    wl, wr = m.window()
    Z = np.zeros((1, 1, 100), dtype=np.uint16)
    Z[0, 0, 40:45] = [2, 6, 12, 6, 2]
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 1, 4, g=np.array([0.5]))
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=2, b_min=1e-8))
    O.init(off, ent, s, normals=False)
    assert s.cnt[0] == 1 and s.t[0, 0] == 42
    mass = irf[2 - wl:2 + wr + 1].sum() / irf.sum()
    n_win = Z[0, 0, 42 - wl:42 + wr + 1].sum()
    assert abs(s.r[0, 0] - n_win / (0.5 * mass)) < 1e-12
    assert s.b[0] == 1e-8


def test_lmf_empty_dead_and_background_only_pixels(oracle_lib):
    m = gauss_model(oracle_lib, 80)
    Z = np.zeros((1, 3, 80), dtype=np.uint16)
    Z[0, 1, [5, 30, 60]] = 1
    Z[0, 2, [10, 11]] = [3, 3]
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 3, 4, g=np.array([1.0, 2.0, 0.0]))
    O = oracle_lib.Oracle(m, oracle_lib.Params(b_min=1e-8))
    O.init(off, ent, s)
    assert list(s.cnt) == [0, 0, 0]
    assert s.b[0] == 1e-8                      # no photons
    assert abs(s.b[1] - 3.0 / (2.0 * 80)) < 1e-15   # Z/(g T)
    assert s.b[2] == 1e-8                      # dead pixel


# ---------------------------------------------------------------- depth step

def test_depth_step_moves_towards_the_data(oracle_lib):
    m = gauss_model(oracle_lib, 100)
    irf = m.h(np.arange(-9, 10))[0]
    Z = np.zeros((1, 1, 100), dtype=np.uint16)
    Z[0, 0, 41:60] = np.round(irf * 1000).astype(np.uint16)   # surface at 50
    off, ent = oracle_lib.compact(Z)
    # beta_t = 1 with strong, background-free data: the Fisher-scaled step is
    # close to a Newton step
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1, dmax=5.0, beta_t=1.0))
    for start in (48.3, 50.6, 51.9):
        s = oracle_lib.State(1, 1, 1, 1)
        s.cnt[0] = 1
        s.t[0, 0] = start
        s.r[0, 0] = 1000.0
        s.b[0] = 1e-3
        O.depth_step(off, ent, s)
        assert abs(s.t[0, 0] - 50.0) < 0.2 * abs(start - 50.0)


def test_depth_step_is_fisher_scaled_gradient(oracle_lib):
    # the step is -beta (dNLL/dt)/(g r I_h), I_h the shift Fisher information of
    # one photon, with dNLL/dt pinned by finite differences in test_oracle_grad
    from test_oracle_grad import small_problem
    m, s, Z, off, ent = small_problem(oracle_lib, seed=4)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=3, dmax=1e9, beta_t=0.7))
    (gt, _, _), _ = O.grad(off, ent, s)
    t0 = s.t.copy()
    O.depth_step(off, ent, s)
    for p in range(s.npix):
        for k in range(s.cnt[p]):
            if s.g[p] > 0:
                expect = np.clip(t0[p, k] - 0.7 * gt[p, k] / (s.g[p] * s.r[p, k] * m.fisher), 0, m.T - 1)
                assert abs(s.t[p, k] - expect) < 1e-9 * max(1.0, abs(expect))
            else:
                assert s.t[p, k] == t0[p, k]


def test_depth_step_clip_and_clamp(oracle_lib):
    m = gauss_model(oracle_lib, 60)
    Z = np.zeros((1, 1, 60), dtype=np.uint16)
    Z[0, 0, 0] = 200
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 1, 1)
    s.cnt[0], s.t[0, 0], s.r[0, 0], s.b[0] = 1, 0.3, 50.0, 1e-3
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1, dmax=0.25))
    O.depth_step(off, ent, s)
    assert abs(s.t[0, 0] - 0.05) < 1e-12           # clipped to 0.25
    O.depth_step(off, ent, s)
    assert s.t[0, 0] == 0.0                        # clamped at the first bin


# ---------------------------------------------------------------- merge

def test_merge_hand_case(oracle_lib):
    m = gauss_model(oracle_lib, 100)
    s = oracle_lib.State(1, 1, 1, 4)
    s.cnt[0] = 3
    s.t[0, :3] = [30.0, 10.0, 10.8]                 # unsorted on purpose
    s.r[0, :3] = [2.0, 1.0, 3.0]
    s.n[0, 0] = [0, 0, -1]
    s.n[0, 1] = [0.6, 0, -0.8]
    s.n[0, 2] = [0, 0.6, -0.8]
    O = oracle_lib.Oracle(m, oracle_lib.Params(d_merge=1.0))
    O.merge(s)
    assert s.cnt[0] == 2
    assert abs(s.t[0, 0] - (1.0 * 10.0 + 3.0 * 10.8) / 4.0) < 1e-12
    assert s.r[0, 0] == 4.0
    nn = np.array([0.6, 1.8, -3.2])
    np.testing.assert_allclose(s.n[0, 0], nn / np.linalg.norm(nn), atol=1e-15)
    assert s.t[0, 1] == 30.0 and s.r[0, 1] == 2.0
    # chains merge into the running point
    s.cnt[0] = 3
    s.t[0, :3] = [5.0, 5.9, 6.3]
    s.r[0, :3] = [1.0, 1.0, 1.0]
    O.merge(s)
    assert s.cnt[0] == 1 and abs(s.t[0, 0] - ((5.0 + 5.9) / 2 * 2 + 6.3) / 3) < 1e-12


# ---------------------------------------------------------------- intensity

def test_intensity_step_single_point_em_closed_form(oracle_lib):
    m = gauss_model(oracle_lib, 80)
    Z = np.zeros((1, 1, 80), dtype=np.uint16)
    Z[0, 0, [37, 39, 40, 41, 44]] = [1, 2, 5, 3, 1]
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 1, 1, g=np.array([1.7]))
    s.cnt[0], s.t[0, 0], s.r[0, 0], s.b[0] = 1, 40.3, 3.0, 0.0
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1))
    O.intensity_step(off, ent, s)
    S, _ = m.S(np.array([40.3]))
    assert abs(s.r[0, 0] - 12.0 / (1.7 * S[0])) < 1e-12


def test_intensity_filter_constant_field_and_graph(oracle_lib):
    rows, cols = 5, 6
    p = oracle_lib.Params(k_max=2, dz=0.1, h_int=2.0, r_min=0.0)
    s = oracle_lib.State(1, rows, cols, 2)
    s.cnt[:] = 1
    s.t[:, 0] = 100.0
    s.r[:, 0] = 3.0
    O = oracle_lib.Oracle(gauss_model(oracle_lib, 500), p)
    O.intensity_filter(s)
    np.testing.assert_allclose(s.r[:, 0], 3.0, rtol=1e-15)  # constant field, borders too
    # hand case: centre pixel of 3x3; neighbour set picks the nearest point per pixel
    s = oracle_lib.State(1, 3, 3, 2)
    s.cnt[:] = 1
    s.t[:, 0] = 50.0
    s.r[:, 0] = np.arange(9, dtype=float)
    s.t[0, 0] = 80.0                     # 3 world units away: not a neighbour
    s.cnt[2] = 2
    s.t[2, :2] = [40.0, 51.0]            # nearest of the two is slot 1 (0.1 away)
    s.r[2, :2] = [100.0, 20.0]
    O.intensity_filter(s)
    expect = (4.0 + 1 + 20.0 + 3 + 5 + 6 + 7 + 8) / 9.0
    assert abs(s.r[4, 0] - expect) < 1e-12
    # corner pixel (0,0) sits alone at depth 80: its 3 surrounding pixels hold no
    # point within h_int, so its intensity is divided by 1 + 3
    assert abs(s.r[0, 0] - 0.0 / 4) < 1e-15


def test_intensity_threshold_removes_and_compacts(oracle_lib):
    p = oracle_lib.Params(k_max=3, dz=0.1, h_int=0.5, r_min=1.0)
    s = oracle_lib.State(1, 1, 1, 3)
    s.cnt[0] = 3
    s.t[0, :3] = [10.0, 20.0, 30.0]
    s.r[0, :3] = [5.0, 0.5, 2.0]
    s.n[0, 2] = [0.6, 0.0, -0.8]
    O = oracle_lib.Oracle(gauss_model(oracle_lib, 500), p)
    O.intensity_filter(s)
    assert s.cnt[0] == 2
    np.testing.assert_array_equal(s.t[0], [10.0, 30.0, 0.0])
    np.testing.assert_array_equal(s.r[0], [5.0, 2.0, 0.0])
    np.testing.assert_array_equal(s.n[0, 1], [0.6, 0.0, -0.8])


# ---------------------------------------------------------------- background

def test_background_step_closed_form(oracle_lib):
    m = gauss_model(oracle_lib, 50)
    Z = np.zeros((1, 2, 50), dtype=np.uint16)
    Z[0, 0, [1, 20, 33]] = [1, 2, 2]
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 2, 1, g=np.array([0.9, 1.0]))
    s.b[:] = [0.4, 0.3]
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_max=1, b_min=1e-8))
    O.bg_step(off, ent, s)
    assert abs(s.b[0] - 5.0 / (0.9 * 50)) < 1e-15   # no points: one EM step reaches Z/(g T)
    assert s.b[1] == 1e-8                           # no photons: the floor


def test_background_filter_equals_fft(oracle_lib):
    rng = np.random.default_rng(2)
    for (F, rows, cols, sig) in [(1, 16, 20, 2.0), (2, 9, 7, 1.3), (1, 5, 4, 2.0)]:
        b = rng.uniform(0.1, 1.0, (F, rows, cols))
        p = oracle_lib.Params(sigma_b=sig, b_min=0.0)
        s = oracle_lib.State(F, rows, cols, 1)
        s.b[:] = b.reshape(-1)
        oracle_lib.Oracle(gauss_model(oracle_lib, 50), p).bg_filter(s)
        rb = int(np.ceil(4 * sig))
        d = np.arange(-rb, rb + 1)
        w = np.exp(-d ** 2 / (2 * sig ** 2))
        w /= w.sum()
        for f in range(F):
            kr = np.zeros(rows)
            kc = np.zeros(cols)
            np.add.at(kr, d % rows, w)
            np.add.at(kc, d % cols, w)
            Kf = np.fft.fft(kr)[:, None] * np.fft.fft(kc)[None, :]
            # correlation with a symmetric kernel = convolution
            expect = np.real(np.fft.ifft2(np.fft.fft2(b[f]) * np.conj(Kf)))
            np.testing.assert_allclose(s.b.reshape(F, rows, cols)[f], expect, rtol=0, atol=1e-12)


def test_background_filter_identity_and_constants(oracle_lib):
    s = oracle_lib.State(1, 6, 6, 1)
    s.b[:] = np.linspace(0.0, 1.0, 36)
    b0 = s.b.copy()
    oracle_lib.Oracle(gauss_model(oracle_lib, 50), oracle_lib.Params(sigma_b=0.0, b_min=0.0)).bg_filter(s)
    np.testing.assert_array_equal(s.b, b0)
    s.b[:] = 0.25
    oracle_lib.Oracle(gauss_model(oracle_lib, 50), oracle_lib.Params(sigma_b=2.0, b_min=0.0)).bg_filter(s)
    np.testing.assert_allclose(s.b, 0.25, rtol=1e-14)


# ---------------------------------------------------------------- whole loop

def test_whole_loop_recovers_plane_from_strong_noiseless_data(oracle_lib):
    sc = synth.plane_scene(0, signal=2000.0, bkg_photons=0.0, theta=0.4)
    m = oracle_lib.Model(sc.irf.probs, sc.T)
    off, ent = oracle_lib.compact(sc.Z)
    O = oracle_lib.Oracle(m, oracle_lib.Params(dz=0.1, r_min=50.0))
    s = O.reconstruct(off, ent, oracle_lib.State(1, sc.rows, sc.cols, 4))
    assert np.all(s.cnt == 1)
    err = (s.t[:, 0] - sc.depth[0].reshape(-1)).reshape(sc.rows, sc.cols)
    # one-sided APSS neighbourhoods bias the image border slightly
    assert np.sqrt(np.mean(err[2:-2, 2:-2] ** 2)) < 0.05
    assert np.sqrt(np.mean(err ** 2)) < 0.15
    # the intensity low-pass smooths the reflectivity field but keeps its level
    assert abs(s.r[:, 0].mean() / sc.intensity[0].mean() - 1) < 0.03
