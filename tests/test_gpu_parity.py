"""GPU parity: every step of the HIP path against the FP64 oracle on the same
seeded inputs, called through the C ABI.

Bars (the GPU computes in FP32 with FP64 depth state, the oracle in FP64):
  - compaction: bit-exact;
  - initialisation: integer peak depths and counts exact (integer score), r/b
    to FP32 rounding;
  - raw gradients: |gpu - oracle| <= 1e-4 x (sum of absolute terms);
  - single steps: depth within 2e-4 bin, intensity/background within 1e-5
    relative, APSS within 1e-3 bin;
  - whole reconstruction: identical point counts on >= 99.9% of pixels and
    depths within 1e-3 bin on pixels whose count and neighbourhood counts
    agree (a decision taken on the other side of a threshold is listed with
    its margin).
Inputs: config-1 plane (32 x 32 x 300), config-2 head shape (141 x 141 x
4613) and a ragged 37 x 23 x 777 scene that spans several tiles with a tail.
"""
import numpy as np
import pytest

from gpu_util import device_to_oracle, intensity_err, oracle_to_device, pair, params_for, to_dev_hist, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_1905_06700_amd import rt3d, synth  # noqa: E402


def _scene(name):
    if name == "c1":
        return synth.plane_scene(0)
    if name == "c2":
        sc = synth.head_scene(0)
        sc.meta["r_init"] = 1
        return sc
    if name == "ragged":
        sc = synth.head_scene(7, rows=37, cols=23, T=777, signal=8.0, sbr=0.5)
        sc.meta.update(r_init=1, dz=0.07)
        return sc
    if name == "ragged_r3":
        # 7 x 7 photon pooling: interior pixels pool more photons than the
        # library scores from LDS (its branch-and-bound path), border pixels fewer
        sc = synth.head_scene(7, rows=37, cols=23, T=777, signal=8.0, sbr=0.5)
        sc.meta.update(r_init=3, dz=0.07)
        return sc
    if name == "bright":
        # the top ten rows' counts scaled by 400: pools there hold photon totals
        # whose product with the largest filter weight passes 2^32 (the 64-bit
        # search), the rest stay within it (the 32-bit one), and pixels on the
        # seam pool both
        sc = synth.head_scene(3, rows=24, cols=19, T=777, signal=8.0, sbr=0.5)
        assert int(sc.Z.max()) * 400 < 65535
        sc.Z[:10] = sc.Z[:10] * np.uint16(400)
        sc.meta.update(r_init=1, dz=0.07)
        return sc
    raise KeyError(name)


_cache = {}


def scene(name):
    if name not in _cache:
        print(f"[gpu-parity] generating {name}", flush=True)
        _cache[name] = _scene(name)
    return _cache[name]


def csr(sc):
    return oracle.compact(sc.Z.reshape(1, sc.rows, sc.cols, sc.T))


# ------------------------------------------------------------------ compaction

@pytest.mark.parametrize("name", ["c1", "c2", "ragged"])
def test_compaction_bit_exact(name):
    sc = scene(name)
    O, ctx = pair(sc)
    off_o, ent_o = csr(sc)
    off, ent = ctx.compact(to_dev_hist(sc.Z))
    st = ctx.query()
    assert st.device_error == 0
    np.testing.assert_array_equal(u32(off), off_o)
    E = int(off_o[-1])
    np.testing.assert_array_equal(u32(ent)[:E], ent_o)


def test_compaction_edge_cases():
    rng = np.random.default_rng(0)
    ctx = rt3d.Context([1.0, 2.0, 1.0], 301)
    for Z in [np.zeros((5, 301), np.uint16),                     # empty
              np.full((3, 301), 65534, np.uint16),               # dense, maximum counts
              (rng.poisson(0.3, (131, 301))).astype(np.uint16),  # ragged pixel starts
              np.eye(301, dtype=np.uint16)[:7] * 9]:             # one bin each
        off_o, ent_o = oracle.compact(Z)
        off, ent = ctx.compact(to_dev_hist(Z))
        assert ctx.query().device_error == 0
        np.testing.assert_array_equal(u32(off), off_o)
        np.testing.assert_array_equal(u32(ent)[:len(ent_o)], ent_o)
    # capacity overflow is reported, not written past
    Z = np.ones((4, 301), np.uint16)
    off, ent = ctx.compact(to_dev_hist(Z), capacity=100)
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_CAPACITY


def test_reconstruct_past_entry_capacity_is_truncated():
    """A reconstruction whose active bins exceed the workspace's max_entries
    reports E_CAPACITY and works on the lists cut at the capacity: the result
    equals the oracle's reconstruction of those truncated lists (the offsets
    clamped to the capacity, the entries beyond it dropped)."""
    sc = scene("c1")
    O, _ = pair(sc)
    ctx = rt3d.Context(sc.irf.probs, sc.T, **params_for(sc), fused_loop=0)
    off_o, ent_o = csr(sc)
    cap = len(ent_o) * 3 // 5                          # ~40% of the pixels lose their lists
    P = sc.rows * sc.cols
    ctx.workspace(1, sc.rows, sc.cols, cap)
    out = ctx.make_output(P)
    ctx.reconstruct_into(out, 1, sc.rows, sc.cols, hist=to_dev_hist(sc.Z)[None])
    with pytest.raises(rt3d.Rt3dError) as e:
        ctx.query()
    assert e.value.status == rt3d.E_CAPACITY
    off_t = np.minimum(off_o, cap).astype(np.uint32)
    so = O.reconstruct(off_t, ent_o[:cap].copy(), oracle.State(1, sc.rows, sc.cols, 4))
    frac, errs, cnt_g, _, ierr, _ = _compare_final(sc, so, out, P)
    print(f"[gpu-parity] truncated lists ({cap} of {len(ent_o)} entries): count agreement {frac:.5f}, "
          f"max depth err {errs.max():.2e} bins, max intensity err {ierr:.2e}", flush=True)
    assert np.all(cnt_g[np.diff(off_t.astype(np.int64)) == 0] == 0)     # no photons left: no point
    assert frac >= 0.999 and errs.max() <= 1e-3 and ierr <= 2e-5


# ------------------------------------------------------------------ init

@pytest.mark.parametrize("name", ["c1", "c2", "ragged", "ragged_r3", "bright"])
def test_init_matches_oracle(name):
    sc = scene(name)
    O, ctx = pair(sc)
    off_o, ent_o = csr(sc)
    so = O.init(off_o, ent_o, oracle.State(1, sc.rows, sc.cols, 4))
    from gpu_util import to_dev_u32
    d = ctx.step(rt3d.STEP_INIT, None, to_dev_u32(off_o), to_dev_u32(ent_o), shape=(1, sc.rows, sc.cols))
    sg = device_to_oracle(d, 4)
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    np.testing.assert_array_equal(sg.t, so.t)
    np.testing.assert_allclose(sg.r, so.r, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sg.b, so.b, rtol=2e-6, atol=1e-12)
    np.testing.assert_allclose(sg.n, so.n, atol=2e-6)


# ------------------------------------------------------------------ gradients

@pytest.mark.parametrize("name", ["c1", "c2", "ragged"])
@pytest.mark.parametrize("iters", [0, 3])
@pytest.mark.parametrize("lanes", [4, 8])
def test_gradients_match_oracle(name, iters, lanes):
    from gpu_util import to_dev_u32
    sc = scene(name)
    O, ctx = pair(sc, lanes_per_pixel=lanes)
    off_o, ent_o = csr(sc)
    s = O.init(off_o, ent_o, oracle.State(1, sc.rows, sc.cols, 4))
    for _ in range(iters):
        O.iterate(off_o, ent_o, s)
    (gt, gr, gb), (at, ar, ab) = O.grad(off_o, ent_o, s)
    dgt, dgr, dgb = ctx.gradients(oracle_to_device(s), to_dev_u32(off_o), to_dev_u32(ent_o))
    dgt = dgt.cpu().numpy()[:4].T.astype(np.float64)
    dgr = dgr.cpu().numpy()[:4].T.astype(np.float64)
    dgb = dgb.cpu().numpy().astype(np.float64)
    live = np.arange(4)[None, :] < s.cnt[:, None]
    for g_gpu, g_or, a in ((dgt, gt, at), (dgr, gr, ar)):
        err = np.abs(g_gpu - g_or)[live]
        assert np.all(err <= 1e-4 * a[live] + 1e-30), (err.max(), (err / a[live]).max())
    assert np.all(np.abs(dgb - gb) <= 1e-4 * ab + 1e-30)


# ------------------------------------------------------------------ single steps

def _state_after(sc, O, iters):
    off_o, ent_o = csr(sc)
    s = O.init(off_o, ent_o, oracle.State(1, sc.rows, sc.cols, 4))
    for _ in range(iters):
        O.iterate(off_o, ent_o, s)
    return s


@pytest.mark.parametrize("name", ["c1", "c2", "ragged"])
@pytest.mark.parametrize("lanes", [4, 8])
def test_single_steps_match_oracle(name, lanes):
    from gpu_util import to_dev_u32
    sc = scene(name)
    O, ctx = pair(sc, lanes_per_pixel=lanes)
    off_o, ent_o = csr(sc)
    off, ent = to_dev_u32(off_o), to_dev_u32(ent_o)
    s0 = _state_after(sc, O, 2)
    din = oracle_to_device(s0)
    live = np.arange(4)[None, :] < s0.cnt[:, None]

    # depth step
    so = O.depth_step(off_o, ent_o, s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_DEPTH, din, off, ent), 4)
    assert np.abs(sg.t - so.t)[live].max() <= 2e-4

    # APSS
    so = O.apss(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_APSS, din), 4)
    assert np.abs(sg.t - so.t)[live].max() <= 1e-3
    assert np.abs(sg.n - so.n)[live].max() <= 1e-3

    # merge
    so = O.merge(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_MERGE, din), 4)
    np.testing.assert_array_equal(sg.cnt, so.cnt)
    lv = np.arange(4)[None, :] < so.cnt[:, None]
    assert np.abs(sg.t - so.t)[lv].max(initial=0) <= 1e-9
    np.testing.assert_allclose(sg.r[lv], so.r[lv], rtol=1e-6)

    # intensity step
    so = O.intensity_step(off_o, ent_o, s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_INTENSITY, din, off, ent), 4)
    np.testing.assert_allclose(sg.r[live], so.r[live], rtol=1e-5, atol=1e-6)

    # intensity filter + threshold
    so = O.intensity_filter(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_IFILTER, din), 4)
    same = sg.cnt == so.cnt
    assert same.mean() >= 0.999, np.nonzero(~same)
    lv = (np.arange(4)[None, :] < so.cnt[:, None]) & same[:, None]
    np.testing.assert_allclose(sg.r[lv], so.r[lv], rtol=1e-5)
    np.testing.assert_array_equal(sg.t[lv], so.t[lv])

    # background step
    so = O.bg_step(off_o, ent_o, s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_BKG, din, off, ent), 4)
    np.testing.assert_allclose(sg.b, so.b, rtol=1e-5, atol=1e-12)

    # background filter
    so = O.bg_filter(s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_BFILTER, din), 4)
    np.testing.assert_allclose(sg.b, so.b, rtol=1e-5, atol=1e-12)


def test_iteration_merges_close_points_like_oracle():
    """One whole iteration (the loop fuses the in-pixel merge into the
    intensity step) on a state where every fifth single-point pixel holds a
    second point closer than d_merge, half of them out of depth order."""
    from gpu_util import to_dev_u32
    sc = scene("c1")
    O, ctx = pair(sc)
    off_o, ent_o = csr(sc)
    off, ent = to_dev_u32(off_o), to_dev_u32(ent_o)
    s0 = _state_after(sc, O, 2)
    dm = O.p.d_merge if O.p.d_merge > 0 else max(1.0, np.sqrt(O.m.sigma2))
    picks = np.nonzero(s0.cnt == 1)[0][::5]
    assert picks.size > 50
    for n, q in enumerate(picks):
        t, r, nv = s0.t[q, 0], s0.r[q, 0], s0.n[q, 0].copy()
        close = (t + 0.4 * dm, 0.5 * r) if n % 2 else (t - 0.3 * dm, 0.7 * r)
        if n % 4 < 2:      # the added point in slot 0: depths out of order when it lies deeper
            s0.t[q, :2] = [close[0], t]
            s0.r[q, :2] = [close[1], r]
        else:
            s0.t[q, :2] = [t, close[0]]
            s0.r[q, :2] = [r, close[1]]
        s0.n[q, 1] = nv
        s0.cnt[q] = 2
    print(f"[gpu-parity] merge-iteration: {picks.size} pixels with an added close point", flush=True)
    so = O.iterate(off_o, ent_o, s0.copy())
    sg = device_to_oracle(ctx.step(rt3d.STEP_ITERATION, oracle_to_device(s0), off, ent), 4)
    same = sg.cnt == so.cnt
    assert same[picks].mean() >= 0.99 and same.mean() >= 0.999
    lv = (np.arange(4)[None, :] < so.cnt[:, None]) & same[:, None]
    assert np.abs(sg.t - so.t)[lv].max() <= 1e-3


@pytest.mark.parametrize("sigma_b", [0.0, 2.0, 12.0])
def test_background_filter_widths(sigma_b):
    """The background filter alone on three frames of 37 x 23 and two of 5 x 7
    (smaller than the filter's reach, so the circular halo wraps more than
    once): the floor only (sigma_b = 0), the tiled kernel (2) and the two-pass
    kernels of wide filters (12, radius 48)."""
    irf = synth.gaussian_irf(1.5, 9).probs
    rng = np.random.default_rng(int(sigma_b * 10) + 3)
    for F, rows, cols in ((3, 37, 23), (2, 5, 7)):
        s0 = oracle.State(F, rows, cols, 4)
        s0.b[:] = rng.gamma(2.0, 0.01, s0.npix)
        s0.b[::17] = 0.0                         # below the floor
        prm = dict(sigma_b=sigma_b, b_min=1e-3)
        O = oracle.Oracle(oracle.Model(irf, 50), oracle.Params(**prm))
        ctx = rt3d.Context(irf, 50, **prm)
        so = O.bg_filter(s0.copy())
        print(f"[gpu-parity] background filter sigma_b {sigma_b}: {F} x {rows} x {cols}", flush=True)
        sg = device_to_oracle(ctx.step(rt3d.STEP_BFILTER, oracle_to_device(s0)), 4)
        np.testing.assert_allclose(sg.b, so.b, rtol=1e-5, atol=1e-12)


# ------------------------------------------------------------------ whole loop

def _compare_final(sc, so, res, P):
    pt_off = u32(res.pt_off).astype(np.int64)
    cnt_g = np.diff(pt_off)
    same = cnt_g == so.cnt
    frac = same.mean()
    depth = res.depth.cpu().numpy()
    inten = res.intensity.cpu().numpy()
    # pixels whose own and 5x5-neighbourhood counts agree
    rows, cols = sc.rows, sc.cols
    bad = (~same).reshape(-1, rows, cols)
    nb_bad = np.zeros_like(bad)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            nb_bad |= np.roll(np.roll(bad, di, 1), dj, 2)
    ok = (~nb_bad).reshape(-1)
    errs = []
    for p in np.nonzero(ok)[0]:
        c = so.cnt[p]
        if c:
            errs.append(np.abs(depth[pt_off[p]:pt_off[p] + c] - so.t[p, :c]).max())
    ierr = intensity_err(inten, pt_off, so, np.nonzero(ok)[0])
    return frac, np.array(errs), cnt_g, depth, ierr, pt_off


@pytest.mark.parametrize("name,fused", [("c1", 1), ("c1", 0), ("c2", 1), ("ragged", 1), ("ragged", 0)])
def test_reconstruction_matches_oracle(name, fused):
    """fused = 1: frames of at most 4096 pixels (c1, ragged) run every iteration
    in one launch; fused = 0: one launch per step (the path of larger frames)."""
    sc = scene(name)
    O, _ = pair(sc)
    ctx = rt3d.Context(sc.irf.probs, sc.T, **params_for(sc), fused_loop=fused)
    off_o, ent_o = csr(sc)
    so = O.reconstruct(off_o, ent_o, oracle.State(1, sc.rows, sc.cols, 4))
    res = ctx.reconstruct(to_dev_hist(sc.Z)[None])
    st = ctx.query()
    assert st.device_error == 0
    assert st.entries == len(ent_o)
    frac, errs, cnt_g, depth, ierr, pt_off = _compare_final(sc, so, res, sc.rows * sc.cols)
    print(f"[gpu-parity] {name} (fused loop {fused}): count agreement {frac:.5f}, max depth err {errs.max():.2e} bins "
          f"over {len(errs)} pixels, max intensity err {ierr:.2e} relative", flush=True)
    assert frac >= 0.999
    assert errs.max() <= 1e-3
    assert ierr <= 2e-5
    np.testing.assert_allclose(res.background.cpu().numpy(), so.b, rtol=1e-3, atol=1e-9)


def test_reconstruction_is_deterministic():
    sc = scene("c1")
    _, ctx = pair(sc)
    Z = to_dev_hist(sc.Z)[None]
    a = ctx.reconstruct(Z)
    b = ctx.reconstruct(Z)
    torch.cuda.synchronize()
    for x, y in ((a.pt_off, b.pt_off), (a.depth, b.depth), (a.intensity, b.intensity),
                 (a.background, b.background)):
        assert torch.equal(x, y)


def test_autotune_choice_is_kept_and_reconstructs_identically():
    """rt3d_autotune times the loop mappings (per step with 4 or 8 lanes per
    pixel, all iterations in one launch) on a 64-frame batch of 32 x 32 frames
    and on one head-shaped frame, and keeps one per batch shape; later calls on
    that shape give what a context forced to that mapping gives."""
    for kind in ("small", "head"):
        if kind == "small":
            scs = [synth.plane_scene(s) for s in range(4)]
            F = 64
        else:
            scs = [scene("c2")]
            F = 1
        sc = scs[0]
        R, C = sc.rows, sc.cols
        Z = torch.stack([to_dev_hist(scs[f % len(scs)].Z) for f in range(F)]).contiguous()
        ctx = rt3d.Context(sc.irf.probs, sc.T, **params_for(sc))
        ctx.workspace(F, R, C, F * R * C * 128)
        out = ctx.make_output(F * R * C)
        choice = ctx.autotune(out, F, R, C, hist=Z)
        fused, lanes = ctx.mapping(out, F, R, C, hist=Z)
        print(f"[gpu-parity] autotune {F} x {R} x {C}: {'one launch' if fused else 'per step'}, "
              f"{lanes} lanes per pixel", flush=True)
        assert choice == fused and lanes in (4, 8)
        ctx.reconstruct_into(out, F, R, C, hist=Z)
        forced = rt3d.Context(sc.irf.probs, sc.T, **params_for(sc), fused_loop=fused, lanes_per_pixel=lanes)
        forced.workspace(F, R, C, F * R * C * 128)
        ref = forced.make_output(F * R * C)
        forced.reconstruct_into(ref, F, R, C, hist=Z)
        assert ctx.query().device_error == 0 and forced.query().device_error == 0
        for name in ("pt_off", "background"):
            assert torch.equal(getattr(out, name), getattr(ref, name)), name
        n = int(ref.pt_off[-1].item())
        for name in ("depth", "intensity"):
            assert torch.equal(getattr(out, name)[:n], getattr(ref, name)[:n]), name


def test_batched_frames_equal_single_frames():
    scs = [synth.plane_scene(s) for s in range(3)]
    _, ctx = pair(scs[0])
    Z = torch.cat([to_dev_hist(s.Z)[None] for s in scs])
    batch = ctx.reconstruct(Z)
    P = 32 * 32
    for f, s in enumerate(scs):
        one = ctx.reconstruct(to_dev_hist(s.Z)[None])
        pb = u32(batch.pt_off).astype(np.int64)
        p1 = u32(one.pt_off).astype(np.int64)
        np.testing.assert_array_equal(np.diff(pb[f * P:(f + 1) * P + 1]), np.diff(p1))
        a, b = pb[f * P], pb[(f + 1) * P]
        np.testing.assert_array_equal(batch.depth[a:b].cpu().numpy(), one.depth[:p1[-1]].cpu().numpy())


def test_gain_and_dead_pixels():
    sc = scene("c1")
    O, ctx = pair(sc)
    g = synth.random_gain(5, sc.rows, sc.cols)
    # counts scale with the gain in the observation model
    rng = np.random.default_rng(9)
    Z = synth.render(rng, sc.irf, sc.T, sc.depth, sc.intensity, sc.background, gain=g)
    off_o, ent_o = oracle.compact(Z[None])
    so = oracle.State(1, sc.rows, sc.cols, 4, g=g.reshape(-1))
    O.reconstruct(off_o, ent_o, so)
    res = ctx.reconstruct(to_dev_hist(Z)[None], gain=torch.from_numpy(g.astype(np.float32).reshape(-1)).cuda())
    frac, errs, cnt_g, _, ierr, _ = _compare_final(sc, so, res, sc.rows * sc.cols)
    assert frac >= 0.999 and errs.max() <= 1e-3 and ierr <= 2e-5
    assert np.all(cnt_g[g.reshape(-1) == 0] == 0)
