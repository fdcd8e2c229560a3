"""Seeded synthetic single-photon lidar scenes.

This module only simulates data: photon arrival times are drawn from a
continuous impulse response and binned, background photons are uniform over
the histogram, and every count is Poisson (the observation model of the
paper's Results, "Observation model").  It contains none of the
reconstruction's arithmetic and is shared by the GPU tests, the oracle tests
and the benchmark, which all take their inputs from here.

Seeds: numpy PCG64 with seed = 1905067000 + 1000 * config + scene.  Draw
order inside a scene: geometry, then reflectivities, then photons.

Scenes stand in for the paper's two datasets (a 141 x 141 x 4613 raster scan
of a head at 40 m and 32 x 32 x 153 array video at 320 m), which are not
available; shapes, photon levels and signal-to-background ratios follow the
paper's descriptions.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import erf, sqrt

import numpy as np

SEED_BASE = 1905067000


def seed_of(config: int, scene: int = 0) -> int:
    return SEED_BASE + 1000 * config + scene


# --------------------------------------------------------------------------
# impulse responses (binned probabilities of a continuous arrival jitter)
# --------------------------------------------------------------------------

def _norm_cdf(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + np.vectorize(erf)(x / sqrt(2.0)))


@dataclass
class IRF:
    """Binned impulse response: probs[k] = P(round(X) = lags[k]) for the jitter X;
    origin = argmax index.  A surface at depth d (bins) puts its photons at
    round(d - lags[origin] + X)."""
    lags: np.ndarray
    probs: np.ndarray
    kind: str
    sigma: float
    tau: float = 0.0

    @property
    def origin(self) -> int:
        return int(np.argmax(self.probs))

    @property
    def shift(self) -> int:
        return int(self.lags[self.origin])

    def draw(self, rng: np.random.Generator, n: int) -> np.ndarray:
        x = rng.normal(0.0, self.sigma, n)
        if self.tau > 0:
            x = x + rng.exponential(self.tau, n)
        return x


def gaussian_irf(sigma: float, half: int) -> IRF:
    lags = np.arange(-half, half + 1)
    probs = _norm_cdf((lags + 0.5) / sigma) - _norm_cdf((lags - 0.5) / sigma)
    return IRF(lags, probs, "gaussian", sigma)


def exgauss_irf(sigma: float, tau: float, lo: int, hi: int) -> IRF:
    """Gaussian(0, sigma) convolved with an exponential tail of mean tau."""
    lags = np.arange(lo, hi + 1)

    def cdf(x):
        x = np.asarray(x, dtype=np.float64)
        lam = 1.0 / tau
        return _norm_cdf(x / sigma) - np.exp(-lam * x + 0.5 * (lam * sigma) ** 2) * \
            _norm_cdf(x / sigma - lam * sigma)

    probs = cdf(lags + 0.5) - cdf(lags - 0.5)
    return IRF(lags, np.maximum(probs, 0.0), "exgauss", sigma, tau)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

@dataclass
class Scene:
    Z: np.ndarray            # uint16 [rows, cols, T]
    irf: IRF
    T: int
    depth: np.ndarray        # float64 [S, rows, cols], true depth in bins (nan = absent)
    intensity: np.ndarray    # float64 [S, rows, cols], expected signal photons
    background: float        # expected background photons per bin
    meta: dict = field(default_factory=dict)

    @property
    def rows(self):
        return self.Z.shape[0]

    @property
    def cols(self):
        return self.Z.shape[1]


def render(rng, irf: IRF, T: int, depth, intensity, b: float, gain=None) -> np.ndarray:
    """Poisson photon counts for surfaces (depth, intensity) [S, rows, cols] on a
    uniform background b per bin.  Photons outside [0, T) are lost."""
    S, rows, cols = depth.shape
    npix = rows * cols
    g = np.ones(npix) if gain is None else np.asarray(gain, dtype=np.float64).reshape(-1)
    pix_all, bin_all = [], []
    for s in range(S):
        d = depth[s].reshape(-1)
        lam = np.where(np.isfinite(d), intensity[s].reshape(-1), 0.0) * g
        n = rng.poisson(lam)
        pix = np.repeat(np.arange(npix), n)
        x = irf.draw(rng, pix.size)
        tb = np.floor(d[pix] - irf.shift + x + 0.5).astype(np.int64)
        keep = (tb >= 0) & (tb < T)
        pix_all.append(pix[keep])
        bin_all.append(tb[keep])
    nb = rng.poisson(b * T * g)
    pix = np.repeat(np.arange(npix), nb)
    pix_all.append(pix)
    bin_all.append(rng.integers(0, T, pix.size))
    pix = np.concatenate(pix_all)
    tb = np.concatenate(bin_all)
    idx, cnt = np.unique(pix * T + tb, return_counts=True)
    assert cnt.max(initial=0) < 65535, "count overflow for uint16 histograms"
    Z = np.zeros(npix * T, dtype=np.uint16)
    Z[idx] = cnt
    return Z.reshape(rows, cols, T)


def _blur_circular(field_, sigma):
    rows, cols = field_.shape
    fy = np.fft.fftfreq(rows)[:, None]
    fx = np.fft.fftfreq(cols)[None, :]
    H = np.exp(-2.0 * (np.pi * sigma) ** 2 * (fx ** 2 + fy ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(field_) * H))


def plane_scene(scene: int = 0, rows: int = 32, cols: int = 32, T: int = 300,
                signal: float = 10.0, bkg_photons: float = 1.0, theta=None) -> Scene:
    """Config 1: one tilted plane with depths spanning bins 50..250, Gaussian
    IRF sigma 1.5 bins, mean `signal` photons/pixel, reflectivity U[0.5, 1],
    `bkg_photons` background photons per pixel."""
    rng = np.random.default_rng(seed_of(1, scene))
    irf = gaussian_irf(1.5, 9)
    th = rng.uniform(0.0, np.pi / 2) if theta is None else float(theta)
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    u = j * np.cos(th) + i * np.sin(th)
    span = u.max() - u.min()
    d = 50.0 + 200.0 * (u - u.min()) / (span if span > 0 else 1.0)
    rho = rng.uniform(0.5, 1.0, (rows, cols))
    r = rho * signal / 0.75
    b = bkg_photons / T
    Z = render(rng, irf, T, d[None], r[None], b)
    return Scene(Z, irf, T, d[None], r[None], b,
                 dict(config=1, dz=0.1, p_xy=1.0, mean_signal=signal, r_min=0.2 * signal,
                      r_init=0, k_init=3))


def head_scene(scene: int = 0, rows: int = 141, cols: int = 141, T: int = 4613,
               signal: float = 5.0, sbr: float = 0.1) -> Scene:
    """Config 2 (the paper's raster-scan shape, 141 x 141 x 4613): a smooth bumpy
    back surface and a foreground occluder 200 bins nearer over 30% of the
    pixels (a thresholded smooth random field), ex-Gaussian IRF (sigma 3 bins,
    exponential tail 10 bins), mean `signal` photons/pixel at the given SBR."""
    rng = np.random.default_rng(seed_of(2, scene))
    irf = exgauss_irf(3.0, 10.0, -18, 118)
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    ci = (rows - 1) / 2.0
    d_bg = (T / 2.0 - 6.5) + 100.0 * np.sin(2 * np.pi * i / 47) * np.sin(2 * np.pi * j / 47) \
        + 2.0 * (i - ci)
    noise = rng.normal(0.0, 1.0, (rows, cols))
    sm = _blur_circular(noise, 6.0)
    n_occ = int(round(0.3 * rows * cols))
    order = np.argsort(sm.reshape(-1), kind="stable")[::-1]
    M = np.zeros(rows * cols)
    M[order[:n_occ]] = 1.0
    M = M.reshape(rows, cols)
    d_fg = d_bg - 200.0
    rho_bg = rng.uniform(0.5, 1.0, (rows, cols))
    rho_fg = rng.uniform(0.5, 1.0, (rows, cols))
    a = signal / 0.75
    r_bg = a * rho_bg * (1.0 - 0.5 * M)
    r_fg = a * rho_fg * 0.5 * M
    depth = np.stack([np.where(M > 0, d_fg, np.nan), d_bg])
    inten = np.stack([np.where(M > 0, r_fg, 0.0), r_bg])
    b = signal / sbr / T
    Z = render(rng, irf, T, depth, inten, b)
    return Scene(Z, irf, T, depth, inten, b,
                 dict(config=2, dz=0.05, p_xy=1.0, mean_signal=signal, r_min=0.2 * signal,
                      r_init=1, k_init=3, occluder=M))


def layers_scene(scene: int = 0, rows: int = 256, cols: int = 256, T: int = 1024, signal: float = 2.0,
                 sbr: float = 0.05, config: int = 4) -> Scene:
    """Config 4 (learned-denoiser scenes): up to three piecewise-smooth depth
    layers (base depths at 0.68 T, 0.44 T and 0.20 T): each a random plane
    (tilt <= 0.5 bin/pixel) plus 40 x a unit-variance field blurred at 16 px
    plus offsets U[-30, 30] on 8 Voronoi cells.  Layer 0 covers every pixel,
    layer 1 half of them and layer 2 a fifth (thresholded smooth fields); a
    front layer takes half of the signal left behind it.  Reflectivity
    U[0.5, 1], mean `signal` photons/pixel, ex-Gaussian IRF of config 2."""
    rng = np.random.default_rng(seed_of(config, scene))
    irf = exgauss_irf(3.0, 10.0, -18, 118)
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    depth = np.full((3, rows, cols), np.nan)
    base = (0.68 * T, 0.44 * T, 0.20 * T)
    fields = []
    for s in range(3):
        ti, tj = rng.uniform(-0.5, 0.5, 2)
        f = _blur_circular(rng.normal(0, 1, (rows, cols)), 16.0)
        f /= f.std() + 1e-12
        cells = rng.uniform(0, 1, (8, 2)) * [rows, cols]
        offs = rng.uniform(-30, 30, 8)
        lab = np.argmin((i[..., None] - cells[:, 0]) ** 2 + (j[..., None] - cells[:, 1]) ** 2, axis=-1)
        d = base[s] + ti * (i - rows / 2) + tj * (j - cols / 2) + 40.0 * f + offs[lab]
        fields.append(np.clip(d, 20, T - 40))
    pres = [np.ones((rows, cols), bool)]
    for frac in (0.5, 0.8):
        g = _blur_circular(rng.normal(0, 1, (rows, cols)), 8.0)
        pres.append(g > np.quantile(g, frac))
    for s in range(3):
        depth[s] = np.where(pres[s], fields[s], np.nan)
    rho = rng.uniform(0.5, 1.0, (3, rows, cols))
    a = signal / 0.75
    share = np.zeros((3, rows, cols))
    left = np.ones((rows, cols))
    for s in (2, 1, 0):                       # nearest layer first
        take = np.where(pres[s], 0.5 * left if s > 0 else left, 0.0)
        share[s] = take
        left = left - take
    inten = a * rho * share
    b = signal / sbr / T
    Z = render(rng, irf, T, depth, np.where(np.isfinite(depth), inten, 0.0), b)
    return Scene(Z, irf, T, depth, inten, b,
                 dict(config=config, dz=0.1, p_xy=1.0, mean_signal=signal, r_min=0.2 * signal,
                      r_init=1, k_init=4))


def sr_scene(scene: int = 0, rows: int = 32, cols: int = 32, s: int = 3, T: int = 153, signal: float = 3.0,
             sbr: float = 0.5, theta=None, config: int = 3) -> Scene:
    """Super-resolution scene (the paper's 32 x 32 x 153 array video, whose
    point cloud is estimated on a grid three times finer): the truth lives on
    the (rows s) x (cols s) point grid -- a tilted background plane spanning
    bins 0.45 T .. 0.75 T and a disc (radius a quarter of the frame) 25 bins
    nearer whose centre moves with `scene` (video frames) -- and each lidar
    pixel collects the photons of its s x s point-grid pixels.  Gaussian IRF
    sigma 1.5 bins; mean `signal` photons per lidar pixel at the given SBR;
    reflectivity U[0.5, 1].  `depth` / `intensity` are the point grid's;
    Z [rows, cols, T] is the lidar's.  meta p_xy = 1 world unit per
    point-grid pixel, dz = 0.1 s (the lidar pixel pitch s world units)."""
    rng = np.random.default_rng(seed_of(config, 500 + scene))
    irf = gaussian_irf(1.5, 9)
    R, C = rows * s, cols * s
    th = rng.uniform(0.0, np.pi / 2) if theta is None else float(theta)
    i, j = np.mgrid[0:R, 0:C].astype(np.float64)
    u = j * np.cos(th) + i * np.sin(th)
    span = u.max() - u.min()
    plane = T * (0.45 + 0.30 * (u - u.min()) / (span if span > 0 else 1.0))
    ph = 2.0 * np.pi * scene / 50.0
    ci, cj = R * (0.5 + 0.2 * np.sin(ph)), C * (0.5 + 0.2 * np.cos(ph))
    disc = (i - ci) ** 2 + (j - cj) ** 2 < (0.25 * min(R, C)) ** 2
    depth = np.where(disc, plane - 25.0, plane)[None]
    rho = rng.uniform(0.5, 1.0, (1, R, C))
    inten = rho * (signal / (s * s)) / 0.75
    b = signal / sbr / T
    Zf = render(rng, irf, T, depth, inten, b / (s * s))
    Z = Zf.reshape(rows, s, cols, s, T).sum(axis=(1, 3), dtype=np.int64)
    assert Z.max(initial=0) < 65535
    return Scene(Z.astype(np.uint16), irf, T, depth, inten, b,
                 dict(config=config, sr=s, dz=0.1 * s, p_xy=1.0, mean_signal=signal,
                      r_min=0.2 * signal / (s * s), r_init=0, k_init=3))


def irf_class_scene(scene: int = 0, rows: int = 40, cols: int = 36, T: int = 777, signal: float = 8.0,
                    sbr: float = 0.5, config: int = 6):
    """Per-pixel IRFs (the observation model's h_ij): three detector classes
    -- Gaussian sigma 1.5 bins, Gaussian sigma 3 bins, and the ex-Gaussian of
    config 2 -- assigned to pixels in seeded random blocks of 4 x 4 (a
    detector array whose tiles differ), over the head-shaped geometry (bumpy
    surface and a 30% occluder 200 bins nearer, scaled to T).  Each pixel's
    photons follow its own IRF.  Returns (scene with irf = class 0's IRF,
    [IRF of every class], uint8 class map [rows, cols])."""
    rng = np.random.default_rng(seed_of(config, scene))
    irfs = [gaussian_irf(1.5, 9), gaussian_irf(3.0, 12), exgauss_irf(3.0, 10.0, -18, 118)]
    bi, bj = (rows + 3) // 4, (cols + 3) // 4
    cls = np.kron(rng.integers(0, len(irfs), (bi, bj)), np.ones((4, 4), np.int64))[:rows, :cols].astype(np.uint8)
    base = head_scene(5000 + scene, rows=rows, cols=cols, T=T, signal=signal, sbr=sbr)
    Z = np.zeros_like(base.Z)
    for k, irf in enumerate(irfs):
        Zk = render(rng, irf, T, base.depth, base.intensity, base.background)
        Z[cls == k] = Zk[cls == k]
    sc = Scene(Z, irfs[0], T, base.depth, base.intensity, base.background,
               dict(base.meta, config=config, r_init=0))
    return sc, irfs, cls


def persp_scene(scene: int = 0, rows: int = 32, cols: int = 28, T: int = 600, a: float = 0.05,
                signal: float = 10.0, sbr: float = 1.0, config: int = 7) -> Scene:
    """Perspective camera (a pinhole at the origin looking along +Z; pixel
    (i, j) sees along the unit ray of (a (j - cx), a (i - cy), 1), depth =
    range / dz along it, dz = 0.1): a tilted world plane through (0, 0, 30)
    with normal (0.1, -0.05, -1) and, in front of it, a sphere of radius 5
    centred at (1, -0.5, 22) that takes half of the signal of the rays it
    meets (two surfaces there).  Gaussian IRF sigma 1.5 bins, mean `signal`
    photons/pixel at the given SBR, reflectivity U[0.5, 1].  meta: persp = a,
    p_xy = 0.6 (below the smallest pixel footprint, so the APSS window covers
    h = 2)."""
    rng = np.random.default_rng(seed_of(config, scene))
    irf = gaussian_irf(1.5, 9)
    dz = 0.1
    i, j = np.mgrid[0:rows, 0:cols].astype(np.float64)
    v = np.stack([a * (j - (cols - 1) / 2), a * (i - (rows - 1) / 2), np.ones_like(i)], axis=-1)
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    n0 = np.array([0.1, -0.05, -1.0])
    n0 /= np.linalg.norm(n0)
    rho_plane = (n0 @ np.array([0.0, 0.0, 30.0])) / (v @ n0)
    C, Rs = np.array([1.0, -0.5, 22.0]), 5.0
    b = v @ C
    disc = b * b - C @ C + Rs * Rs
    hit = disc > 0
    rho_sphere = np.where(hit, b - np.sqrt(np.where(hit, disc, 0.0)), np.nan)
    depth = np.stack([rho_sphere / dz, rho_plane / dz])
    rho = rng.uniform(0.5, 1.0, (2, rows, cols))
    amp = signal / 0.75
    inten = np.stack([np.where(hit, 0.5 * amp * rho[0], 0.0), np.where(hit, 0.5, 1.0) * amp * rho[1]])
    bkg = signal / sbr / T
    Z = render(rng, irf, T, depth, inten, bkg)
    return Scene(Z, irf, T, depth, inten, bkg,
                 dict(config=config, dz=dz, p_xy=0.6, persp=a, mean_signal=signal, r_min=0.2 * signal,
                      r_init=0, k_init=3))


def stress_scene(scene: int = 0, side: int = 512, T: int = 2000, signal: float = 1.0, sbr: float = 0.01,
                 empty: float = 0.15) -> Scene:
    """Config 5 (stress): the multi-layer geometry of config 4 at side x side x
    T, mean `signal` photons per pixel at the given SBR (1 photon, SBR 0.01:
    100 background photons per pixel), and a fraction `empty` of the pixels
    (a thresholded smooth field) with no surface at all."""
    base_rng = np.random.default_rng(seed_of(5, 1000 + scene))
    g = _blur_circular(base_rng.normal(0, 1, (side, side)), 8.0)
    hole = g > np.quantile(g, 1.0 - empty)
    sc = layers_scene(scene, rows=side, cols=side, T=T, signal=signal, sbr=sbr, config=5)
    depth = np.where(hole[None], np.nan, sc.depth)
    inten = np.where(hole[None], 0.0, sc.intensity)
    rng = np.random.default_rng(seed_of(5, 2000 + scene))
    Z = render(rng, sc.irf, T, depth, inten, sc.background)
    meta = dict(sc.meta, config=5, empty=hole)
    return Scene(Z, sc.irf, T, depth, inten, sc.background, meta)


def ramp_background_scene(scene: int = 0, rows: int = 36, cols: int = 44, T: int = 4613, signal: float = 5.0,
                          bkg_lo: float = 20.0, bkg_hi: float = 330.0) -> Scene:
    """Config-2 geometry and IRF with the background photons per pixel rising
    linearly across the columns from bkg_lo to bkg_hi (the execution-time
    sweep's range of active bins per pixel in one frame).  The per-pixel
    background level is returned as the `background` array; every pixel has
    unit gain."""
    sc = head_scene(scene, rows=rows, cols=cols, T=T, signal=signal)
    bph = np.broadcast_to(np.linspace(bkg_lo, bkg_hi, cols)[None, :], (rows, cols))
    g = bph / bph.max()
    rng = np.random.default_rng(seed_of(2, 3000 + scene))
    # render's gain scales signal and background alike: divide the signal back out
    Z = render(rng, sc.irf, T, sc.depth, sc.intensity / g[None], bph.max() / T, gain=g)
    return Scene(Z, sc.irf, T, sc.depth, sc.intensity, bph / T, dict(sc.meta))


def random_gain(rng_seed: int, rows: int, cols: int, dead_frac: float = 0.02) -> np.ndarray:
    """Per-pixel detector gain in [0.5, 1.5] with a fraction of dead (0) pixels."""
    rng = np.random.default_rng(rng_seed)
    g = rng.uniform(0.5, 1.5, (rows, cols))
    g[rng.random((rows, cols)) < dead_frac] = 0.0
    return g
