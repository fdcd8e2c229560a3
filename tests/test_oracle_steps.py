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
    """Peak = argmax over tau of sum z log(h(t - tau) + eps) - log eps, by
    brute force in float64.  The oracle scores with weights rounded to 16
    fractional bits (exact integer sums), so each score is off by at most
    0.5 sum(z) / 2^16; wherever the float top-two margin exceeds twice that
    bound, the integer argmax must be the float argmax."""
    rng = np.random.default_rng(5)
    T = 150
    m = gauss_model(oracle_lib, T)
    eps = 1.0 / T
    checked = 0
    for trial in range(40):
        Z = rng.poisson(0.05, (1, 1, T)).astype(np.uint16)
        d = rng.integers(10, 140)
        Z[0, 0, d - 2:d + 3] += rng.poisson(3.0 if trial % 2 else 1.0, 5).astype(np.uint16)
        off, ent = oracle_lib.compact(Z)
        z = Z[0, 0].astype(float)
        nz = np.nonzero(z)[0]
        score = np.array([sum(z[t] * (np.log(m.h(t - tau)[0][0] + eps) - np.log(eps)) for t in nz)
                          for tau in range(T)])
        best = int(np.argmax(score))
        srt = np.sort(score)
        bound = 0.5 * z.sum() / 2.0 ** 16
        if srt[-1] - srt[-2] <= 2.0 * bound:
            continue                                   # the rounding may decide this one
        s = oracle_lib.State(1, 1, 1, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(n_min=1, kappa=0.0, k_init=1))
        O.init(off, ent, s)
        assert s.cnt[0] == 1 and s.t[0, 0] == best
        checked += 1
    assert checked >= 36


def test_lmf_weights_are_rounded_log_filter(oracle_lib):
    """q_k = round(2^16 log(1 + h_k T sbr_guess)): within half a unit of the
    float weight of the log-matched filter at each integer lag."""
    T = 150
    m = gauss_model(oracle_lib, T)
    for sbr in (1.0, 0.1):
        q = m.lmf_table(sbr)
        h = m.h(np.arange(m.L) - m.origin)[0]
        exact = 2.0 ** 16 * np.log1p(h * T * sbr)
        assert np.all(np.abs(q - exact) <= 0.5)


def test_lmf_pooled_window_hand_case(oracle_lib):
    """r_init = 1 pools the photons of the 3 x 3 window (clipped at the frame
    edge, not wrapped).  5 x 5 frame, 40 bins, IRF (1, 2, 1):
      - centre (2, 2): own 3 photons at bin 10 and 2 at bin 25;
      - its 8 neighbours: 2 photons each at bin 25;
      - the outer ring: 4 photons each at bin 10, except (4, 4): 100 at bin 33.
    Centre, own photons only (r_init 0): argmax 10.  Pooled 3 x 3: bin 10
    holds 3, bin 25 holds 18, so the peak is 25 (a 5 x 5 pool would pick 33,
    then 10).  Its window 24..26 holds 2 own photons; background from the 3
    others over the 37 unclaimed bins: r0 = 2 - 3 * 3/37, b0 = 3/37.
    Corner (0, 0) pools (0,0), (0,1), (1,0): 4 + 4 + 4 at bin 10 and (1,1):
    2 at bin 25; a wrapped window would reach (4, 4)'s 100 at bin 33."""
    T = 40
    m = oracle_lib.Model(np.array([1.0, 2.0, 1.0]), T=T)
    assert m.window() == (1, 1)
    Z = np.zeros((1, 5, 5, T), dtype=np.uint16)
    for i in range(5):
        for j in range(5):
            if max(abs(i - 2), abs(j - 2)) == 2:
                Z[0, i, j, 10] = 4
            elif max(abs(i - 2), abs(j - 2)) == 1:
                Z[0, i, j, 25] = 2
    Z[0, 4, 4, 10] = 0
    Z[0, 4, 4, 33] = 100
    Z[0, 2, 2, 10] = 3
    Z[0, 2, 2, 25] = 2
    off, ent = oracle_lib.compact(Z)
    for r_init, t_centre in ((0, 10), (1, 25)):
        s = oracle_lib.State(1, 5, 5, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=1, r_init=r_init, n_min=1, kappa=3.0, b_min=1e-8))
        O.init(off, ent, s, normals=False)
        c = 2 * 5 + 2
        assert s.cnt[c] == 1 and s.t[c, 0] == t_centre
        if r_init == 1:
            assert abs(s.r[c, 0] - (2.0 - 3.0 * 3.0 / 37.0)) < 1e-12
            assert abs(s.b[c] - 3.0 / 37.0) < 1e-15
            assert s.cnt[0] == 1 and s.t[0, 0] == 10           # corner: not wrapped
        else:
            # own photons: 3 at bin 10 (window 9..11), 2 others over 37 bins
            assert abs(s.r[c, 0] - (3.0 - 2.0 * 3.0 / 37.0)) < 1e-12
            assert abs(s.b[c] - 2.0 / 37.0) < 1e-15


def test_lmf_second_round_claims_and_keep_test_hand_case(oracle_lib):
    """Pixel (1, 1) of the pooled-window case with k_init = 2: its 3 x 3 pool
    holds 23 photons at bin 10 (five ring pixels and the centre) and 8 at bin
    25, its own photons are the 2 at bin 25.  Round 1 takes 10 (accepted on
    the pool, claims bins 9..11), round 2 scores the unclaimed photons and
    takes 25 (claims 24..26).  The keep test uses the pixel's own photons: the
    peak at 10 holds none and is dropped; the peak at 25 keeps
    r0 = 2 - 0 * 3/34 = 2 and the background has no unclaimed photon left
    (b0 = b_min).  With k_init = 1 only the dropped peak is found: no point."""
    T = 40
    m = oracle_lib.Model(np.array([1.0, 2.0, 1.0]), T=T)
    Z = np.zeros((1, 5, 5, T), dtype=np.uint16)
    for i in range(5):
        for j in range(5):
            if max(abs(i - 2), abs(j - 2)) == 2:
                Z[0, i, j, 10] = 4
            elif max(abs(i - 2), abs(j - 2)) == 1:
                Z[0, i, j, 25] = 2
    Z[0, 4, 4, 10] = 0
    Z[0, 4, 4, 33] = 100
    Z[0, 2, 2, 10] = 3
    Z[0, 2, 2, 25] = 2
    off, ent = oracle_lib.compact(Z)
    q = 1 * 5 + 1
    for k_init, cnt in ((1, 0), (2, 1)):
        s = oracle_lib.State(1, 5, 5, 4)
        O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=k_init, r_init=1, n_min=1, kappa=3.0, b_min=1e-8))
        O.init(off, ent, s, normals=False)
        assert s.cnt[q] == cnt
        if cnt:
            assert s.t[q, 0] == 25 and abs(s.r[q, 0] - 2.0) < 1e-15
            assert s.b[q] == 1e-8


def test_lmf_later_rounds_score_unclaimed_photons_hand_case(oracle_lib):
    """One pixel, 100 bins, IRF (1, 2, 4, 8, 4, 2, 1)/22 (window -2..+2,
    suppression half width 3), no background: noiseless templates x20 at
    depth 30 (440 photons) and x4 at depth 60 (88 photons).  After round 1
    takes 30 and claims bins 28..32, round 2 scores the unclaimed photons
    only: the first template's tails (20 photons at bins 27 and 33) score
    20 q(4/22) at tau = 26 and 34, below the second template's score at 60.
    Scoring every photon instead would put 288 > 261 (in units of log) at
    tau = 26 and 34, just outside the suppression, and reject it.  Round 3
    (tau = 26, tie with 34, smallest first) is rejected.  Own photons in the
    claimed windows 400 and 80, the other 48 over 90 bins; the IRF mass in a
    window is 20/22."""
    T = 100
    irf = np.array([1.0, 2.0, 4.0, 8.0, 4.0, 2.0, 1.0])
    m = oracle_lib.Model(irf, T=T)
    assert m.window() == (2, 2)
    Z = np.zeros((1, 1, T), dtype=np.uint16)
    Z[0, 0, 27:34] += (20 * irf).astype(np.uint16)
    Z[0, 0, 57:64] += (4 * irf).astype(np.uint16)
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 1, 4)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=3, r_init=0, n_min=2, kappa=3.0, b_min=1e-8))
    O.init(off, ent, s, normals=False)
    assert s.cnt[0] == 2
    np.testing.assert_array_equal(s.t[0, :2], [30.0, 60.0])
    H = 20.0 / 22.0
    assert abs(s.b[0] - 48.0 / 90.0) < 1e-15
    assert abs(s.r[0, 0] - (400.0 - 5.0 * 48.0 / 90.0) / H) < 1e-10
    assert abs(s.r[0, 1] - (80.0 - 5.0 * 48.0 / 90.0) / H) < 1e-10


def test_lmf_two_surfaces_on_background_hand_case(oracle_lib):
    """One pixel, 100 bins, IRF (1, 2, 4, 2, 1)/10 (window -2..+2, suppression
    half width ceil(2 sigma_h) = 3): noiseless templates of 100 photons at
    depth 30 and 50 photons at depth 70 on one background photon per bin,
    except bins 0..4, which are empty.
      round 1: the larger template, 30 (symmetric data and filter), accepted;
      round 2: on the unclaimed photons, 70, accepted;
      round 3: the flat background's first full window is tau = 7 (window
               5..9, 5 photons against 245 * 5/100 expected): rejected, stop.
    Own photons (r_init = 0): 105 and 55 in the two claimed windows, the other
    85 over the 90 unclaimed bins, so b0 = 85/90 (a claimed rejected window
    would give 80/85, an unclaimed denominator 85/100) and
    r0 = 105 - 5 * 85/90, 55 - 5 * 85/90 (the IRF mass in each window is 1)."""
    T = 100
    irf = np.array([1.0, 2.0, 4.0, 2.0, 1.0])
    m = oracle_lib.Model(irf, T=T)
    assert m.window() == (2, 2)
    Z = np.ones((1, 1, T), dtype=np.uint16)
    Z[0, 0, :5] = 0
    Z[0, 0, 28:33] += (10 * irf).astype(np.uint16)
    Z[0, 0, 68:73] += (5 * irf).astype(np.uint16)
    assert int(Z.sum()) == 95 + 150
    off, ent = oracle_lib.compact(Z)
    s = oracle_lib.State(1, 1, 1, 4)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=3, r_init=0, n_min=2, kappa=3.0, b_min=1e-8))
    O.init(off, ent, s, normals=False)
    assert s.cnt[0] == 2
    np.testing.assert_array_equal(s.t[0, :2], [30.0, 70.0])
    assert abs(s.b[0] - 85.0 / 90.0) < 1e-15
    assert abs(s.r[0, 0] - (105.0 - 5.0 * 85.0 / 90.0)) < 1e-12
    assert abs(s.r[0, 1] - (55.0 - 5.0 * 85.0 / 90.0)) < 1e-12
    # k_init = 1 stops after the first peak: the second template's photons
    # count as background
    s = oracle_lib.State(1, 1, 1, 4)
    O = oracle_lib.Oracle(m, oracle_lib.Params(k_init=1, r_init=0, n_min=2, kappa=3.0, b_min=1e-8))
    O.init(off, ent, s, normals=False)
    assert s.cnt[0] == 1 and s.t[0, 0] == 30.0
    assert abs(s.b[0] - 140.0 / 95.0) < 1e-15
    assert abs(s.r[0, 0] - (105.0 - 5.0 * 140.0 / 95.0)) < 1e-12


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


def _graph_case(oracle_lib):
    # centre pixel of 3x3; the neighbour set picks the nearest point per pixel
    s = oracle_lib.State(1, 3, 3, 2)
    s.cnt[:] = 1
    s.t[:, 0] = 50.0
    s.r[:, 0] = np.arange(9, dtype=float) + 1.0
    s.t[0, 0] = 80.0                     # 3 world units away: not a neighbour
    s.cnt[2] = 2
    s.t[2, :2] = [40.0, 51.0]            # nearest of the two is slot 1 (0.1 away)
    s.r[2, :2] = [100.0, 20.0]
    return s


@pytest.mark.parametrize("ilp_box", [0, 1])
def test_intensity_filter_constant_field_and_graph(oracle_lib, ilp_box):
    rows, cols = 5, 6
    p = oracle_lib.Params(k_max=2, dz=0.1, h_int=2.0, r_min=0.0, ilp_box=ilp_box)
    s = oracle_lib.State(1, rows, cols, 2)
    s.cnt[:] = 1
    s.t[:, 0] = 100.0
    s.r[:, 0] = 3.0
    O = oracle_lib.Oracle(gauss_model(oracle_lib, 500), p)
    O.intensity_filter(s)
    # a constant field is invariant (the box reading only inside the image)
    inner = np.zeros((rows, cols), bool)
    inner[1:-1, 1:-1] = True
    np.testing.assert_allclose(s.r[:, 0][inner.reshape(-1) | (ilp_box == 0)], 3.0, rtol=1e-15)
    s = _graph_case(oracle_lib)
    O.intensity_filter(s)
    found = [2.0, 20.0, 4, 6, 7, 8, 9]       # pixel 0 (depth 80) is not on the surface
    if ilp_box == 0:
        # mean over the point and the seven neighbours on its surface
        expect = (5.0 + sum(found)) / 8.0
        # the corner (0,0) sits alone at depth 80: no neighbour, its intensity stays
        expect_corner = 1.0
    else:
        # 3 x 3 box: the missing neighbour counts as zero
        expect = (5.0 + sum(found)) / 9.0
        expect_corner = 1.0 / 4
    assert abs(s.r[4, 0] - expect) < 1e-12
    assert abs(s.r[0, 0] - expect_corner) < 1e-15
    # border pixel (0,1): neighbours (0,0) [not on the surface], (0,2) slot 1,
    # (1,0), (1,1), (1,2); five pixels inside the image
    s = _graph_case(oracle_lib)
    O.intensity_filter(s)
    nb = [20.0, 4, 5, 6]
    assert abs(s.r[1, 0] - (2.0 + sum(nb)) / (1 + (5 if ilp_box else 4))) < 1e-12


def test_intensity_filter_surface_mean_keeps_an_isolated_point(oracle_lib):
    """The reading of the paper's low-pass (only points of one surface are
    correlated): a point whose surrounding pixels hold no point of its surface
    keeps its intensity and survives the threshold, while the 3 x 3 box reading
    divides it by 9 and removes it."""
    s = oracle_lib.State(1, 3, 3, 2)
    s.cnt[:] = 1
    s.t[:, 0] = 50.0
    s.r[:, 0] = 4.0
    s.t[4, 0] = 200.0                    # centre point far from its neighbours' surface
    s.r[4, 0] = 3.0
    for ilp_box, kept in ((0, True), (1, False)):
        O = oracle_lib.Oracle(gauss_model(oracle_lib, 500),
                              oracle_lib.Params(k_max=2, dz=0.1, h_int=2.0, r_min=1.0, ilp_box=ilp_box))
        c = s.copy()
        O.intensity_filter(c)
        assert (c.cnt[4] == 1) == kept
        if kept:
            assert c.t[4, 0] == 200.0 and c.r[4, 0] == 3.0


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
