"""Training driver of the learned depth denoiser (orchestration only: every
step runs in librt3d.so's kernels).

The network is trained on the inputs the depth denoiser sees in the plain
method: the states after the depth gradient step, recorded at several
iterations of APSS reconstructions of synthetic multi-layer scenes, with the
scenes' true depths as targets (slot-to-surface matching and the masked
squared error are done by the library's training step).  Weights start from
a seeded He initialisation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rt3d

RECORD_ITERS = (0, 1, 2, 4, 7, 11, 15, 19)


LIVE_IN = 12   # feature channels that carry data


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (zero biases) in the library's layout, from a seed;
    the last layer starts at zero, so training starts from the identity (no
    depth correction)."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(((16, 32), (32, 32), (32, 32), (32, 3))):
        live_in = LIVE_IN if ci == 16 else ci
        w = rng.normal(0.0, np.sqrt(2.0 / (9 * live_in)), (3, 3, ci, co))
        if ci == 16:
            w[:, :, LIVE_IN:, :] = 0.0
        if li == 3:
            w[:] = 0.0
        parts += [w.reshape(-1), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def record_depth_inputs(ctx: rt3d.Context, Z: torch.Tensor, iters=RECORD_ITERS, n_iter: int = 20):
    """Runs the plain reconstruction step by step on histograms Z [F, R, C, T]
    and returns the states after the depth step at the given iterations."""
    F, R, C, T = Z.shape
    ctx.workspace(F, R, C, F * R * C * 256)
    off, ent = ctx.compact(Z.reshape(-1, T))
    st = ctx.step(rt3d.STEP_INIT, None, off, ent, shape=(F, R, C))
    out = []
    for it in range(n_iter):
        st = ctx.step(rt3d.STEP_DEPTH, st, off, ent)
        if it in iters:
            out.append(st)
        st = ctx.step(rt3d.STEP_APSS, st)
        st = ctx.step(rt3d.STEP_MERGE, st)
        st = ctx.step(rt3d.STEP_INTENSITY, st, off, ent)
        st = ctx.step(rt3d.STEP_IFILTER, st)
        st = ctx.step(rt3d.STEP_BKG, st, off, ent)
        st = ctx.step(rt3d.STEP_BFILTER, st)
    return out


def train(net: rt3d.Context, batches, steps: int, lr: float = 2e-3, seed: int = 0, log_every: int = 0,
          log=print):
    """batches: list of (states, truth [S, P] cuda float) pairs.  Returns the
    loss history sampled every log_every steps (and the last)."""
    net.cnn_set_weights(he_init(seed))
    pairs = [(st, tr) for states, tr in batches for st in states]
    hist = []
    loss = torch.zeros(2, dtype=torch.float32, device="cuda")
    for step in range(steps):
        st, tr = pairs[step % len(pairs)]
        net.cnn_train_step(st, tr, lr=lr, loss=loss)
        if (log_every and step % log_every == 0) or step == steps - 1:
            v = float(loss[0].item())
            hist.append(v)
            if log_every:
                log(f"[train] step {step} loss {v:.4f}")
    return hist


def depth_rmse(depth_true: np.ndarray, pt_off: np.ndarray, depth: np.ndarray, cap: float):
    """Depth RMSE over true surfaces (each matched to the nearest estimated
    point of its pixel, errors capped at `cap`, a miss counting `cap`) and the
    fraction of surfaces found within `cap`.  depth_true [S, P] (NaN = absent)."""
    errs = []
    for p in range(depth_true.shape[1]):
        est = depth[pt_off[p]:pt_off[p + 1]]
        for s in range(depth_true.shape[0]):
            d = depth_true[s, p]
            if not np.isfinite(d):
                continue
            e = float(np.abs(est - d).min()) if est.size else np.inf
            errs.append(min(e, cap))
    e = np.asarray(errs)
    return float(np.sqrt(np.mean(e ** 2))), float(np.mean(e < cap))
