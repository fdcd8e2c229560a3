"""Training and evaluation driver of the learned depth denoiser
(orchestration only: every step of the reconstruction and of training runs
in librt3d.so's kernels; torch holds device memory and cuts crops).

Recipe: config-4 multi-layer scenes (seeds 0 .. n-1, generated on the host by
a pool of worker processes as active-bin lists), reconstructed by the plain
method (APSS) step by step on the GPU; the states after the depth gradient
step at iterations 1, 2, 5, 10 and 20 -- the inputs the depth denoiser sees
-- are kept in a buffer of recent scenes, and each training step takes a
batch of random 64 x 64 crops from it with the scenes' true depths as
targets (slot-to-surface matching and the masked squared error are the
library's training step).  Weights start from a seeded He initialisation;
the result is written as a checkpoint (rt3d_denoiser_save).

    python -m paper_1905_06700_amd.train --scenes 2000 --out net.rt3dcnn
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

RECORD_ITERS = (0, 1, 4, 9, 19)    # iterations 1, 2, 5, 10 and 20 (0-based)
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


# ---------------------------------------------------------------------------
# scenes as active-bin lists (host worker processes)

def scene_lists(args):
    """One config-4 scene (seed index s) as (off uint32 [P + 1], ent uint32
    [E] with entry = bin << 16 | count, true depths float32 [3, P])."""
    from . import synth
    s, rows, cols, T, signal, sbr = args
    sc = synth.layers_scene(s, rows=rows, cols=cols, T=T, signal=signal, sbr=sbr)
    Z = sc.Z.reshape(-1, T)
    pix, tb = np.nonzero(Z)
    ent = (tb.astype(np.uint32) << np.uint32(16)) | Z[pix, tb].astype(np.uint32)
    off = np.zeros(Z.shape[0] + 1, dtype=np.uint32)
    off[1:] = np.cumsum(np.bincount(pix, minlength=Z.shape[0]))
    return off, ent, sc.depth.reshape(3, -1).astype(np.float32)


def batch_lists(items):
    """Concatenated lists of several frames (pixel-major, frame after frame)."""
    offs, ents, truths = zip(*items)
    base = np.cumsum([0] + [len(e) for e in ents[:-1]])
    off = np.concatenate([o[:-1] + b for o, b in zip(offs, base)] + [[int(base[-1]) + len(ents[-1])]])
    return off.astype(np.uint32), np.concatenate(ents), np.concatenate(truths, axis=1)


# ---------------------------------------------------------------------------
# GPU side

def record_depth_inputs(ctx, off, ent, shape, iters=RECORD_ITERS, n_iter: int = 20):
    """Runs the plain reconstruction step by step on active-bin lists (device
    int32 tensors) of `shape` = (F, R, C) frames and returns the states after
    the depth step at the given iterations."""
    from . import rt3d
    st = ctx.step(rt3d.STEP_INIT, None, off, ent, shape=shape)
    out = []
    for it in range(n_iter):
        if it not in iters:
            st = ctx.step(rt3d.STEP_ITERATION, st, off, ent)
            continue
        st = ctx.step(rt3d.STEP_DEPTH, st, off, ent)
        out.append(st)
        for k in (rt3d.STEP_APSS, rt3d.STEP_MERGE):
            st = ctx.step(k, st)
        st = ctx.step(rt3d.STEP_INTENSITY, st, off, ent)
        st = ctx.step(rt3d.STEP_IFILTER, st)
        st = ctx.step(rt3d.STEP_BKG, st, off, ent)
        st = ctx.step(rt3d.STEP_BFILTER, st)
    return out


def crop_batch(pool, n, size, rng):
    """n random size x size crops from the (state, truth) pairs in `pool`,
    as one state of n frames and its true depths [3, n size^2]."""
    import torch
    from . import rt3d
    parts = {k: [] for k in ("t", "r", "n", "cnt", "b", "tr")}
    for _ in range(n):
        st, tr = pool[int(rng.integers(len(pool)))]
        F, R, C = st.frames, st.rows, st.cols
        f, y, x = int(rng.integers(F)), int(rng.integers(R - size + 1)), int(rng.integers(C - size + 1))
        win = (slice(f, f + 1), slice(y, y + size), slice(x, x + size))
        parts["t"].append(st.t.view(4, F, R, C)[(slice(None),) + win])
        parts["r"].append(st.r.view(4, F, R, C)[(slice(None),) + win])
        parts["n"].append(st.n.view(3, 4, F, R, C)[(slice(None), slice(None)) + win])
        parts["cnt"].append(st.cnt.view(F, R, C)[win])
        parts["b"].append(st.b.view(F, R, C)[win])
        parts["tr"].append(tr.view(3, F, R, C)[(slice(None),) + win])
    cat = lambda k, d: torch.cat(parts[k], dim=d)
    P = n * size * size
    st = rt3d.DeviceState(n, size, size, cat("t", 1).reshape(4, P).contiguous(),
                          cat("r", 1).reshape(4, P).contiguous(), cat("n", 2).reshape(3, 4, P).contiguous(),
                          cat("cnt", 0).reshape(P).contiguous(), cat("b", 0).reshape(P).contiguous())
    return st, cat("tr", 1).reshape(3, P).contiguous()


def train_recipe(net, apss, lists, n_scenes: int, steps: int, rows=256, cols=256, frames_per_batch=16,
                 crop=64, batch=32, lr=2e-3, lr_final=2e-4, buffer_batches=4, seed=0, log=print):
    """Trains `net` (a context with the learned denoiser) on depth-block inputs
    recorded by `apss` (a plain context) from scenes yielded by `lists` (an
    iterator of scene_lists results, n_scenes of them).  The learning rate
    decays geometrically from lr to lr_final.  Returns the loss history
    (every 50 steps and the last)."""
    import torch
    net.cnn_set_weights(he_init(seed))
    net.workspace(batch, crop, crop, batch * crop * crop * 8)
    rng = np.random.default_rng(seed + 1)
    n_batches = (n_scenes + frames_per_batch - 1) // frames_per_batch
    per_batch = max(1, steps // n_batches)
    pool, hist, done = [], [], 0
    loss = torch.zeros(2, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for b in range(n_batches):
        k = min(frames_per_batch, n_scenes - b * frames_per_batch)
        off, ent, truth = batch_lists([next(lists) for _ in range(k)])
        doff = torch.from_numpy(off.view(np.int32)).cuda()
        dent = torch.from_numpy(ent.view(np.int32)).cuda()
        dtr = torch.from_numpy(truth).cuda()
        apss.workspace(k, rows, cols, len(ent) + 1)
        recs = record_depth_inputs(apss, doff, dent, (k, rows, cols))
        pool = pool[-(buffer_batches - 1) * len(RECORD_ITERS):] if buffer_batches > 1 else []
        pool += [(st, dtr) for st in recs]
        n_here = per_batch if b < n_batches - 1 else steps - done
        for _ in range(n_here):
            a = lr * (lr_final / lr) ** (done / max(steps - 1, 1))
            st, tr = crop_batch(pool, batch, crop, rng)
            net.cnn_train_step(st, tr, lr=a, loss=loss)
            if done % 50 == 0 or done == steps - 1:
                v = float(loss[0].item())
                hist.append((done, v))
                log(f"[train] step {done} scenes {b * frames_per_batch + k} loss {v:.4f} lr {a:.2e} "
                    f"({time.perf_counter() - t0:.0f} s)")
            done += 1
    return hist


# ---------------------------------------------------------------------------
# evaluation

def match_surfaces(depth_true: np.ndarray, pt_off: np.ndarray, depth: np.ndarray, cap: float):
    """Each true surface of a pixel is matched greedily (nearest pair first)
    to an unused estimated point of that pixel within `cap` bins.
    depth_true [S, P] (NaN = absent); the estimated points of pixel p are
    depth[pt_off[p] : pt_off[p + 1]] (at most 4).  Returns (errors of the
    matched surfaces, number of true surfaces, number of unmatched points)."""
    S, P = depth_true.shape
    cnt = np.diff(pt_off).astype(np.int64)
    K = 4
    est = np.full((P, K), np.nan)
    idx = pt_off[:-1, None].astype(np.int64) + np.arange(K)[None, :]
    live = np.arange(K)[None, :] < np.minimum(cnt, K)[:, None]
    est[live] = depth[idx[live]]
    d = np.abs(depth_true.T[:, :, None] - est[:, None, :])          # [P, S, K]
    d = np.where(np.isfinite(d), d, np.inf)
    errs = []
    for _ in range(min(S, K)):
        flat = d.reshape(P, -1)
        j = np.argmin(flat, axis=1)
        best = flat[np.arange(P), j]
        ok = best <= cap
        errs.append(best[ok])
        s_i, k_i = j // K, j % K
        rows = np.nonzero(ok)[0]
        d[rows, s_i[ok], :] = np.inf
        d[rows, :, k_i[ok]] = np.inf
    e = np.concatenate(errs) if errs else np.zeros(0)
    n_true = int(np.isfinite(depth_true).sum())
    return e, n_true, int(cnt.sum()) - e.size


def depth_scores(errs, n_true, n_false, n_pix, cap):
    """Depth RMSE over all true surfaces (a miss counts cap), over the found
    ones, the fraction found and the unmatched points per pixel."""
    e = np.concatenate(errs)
    nt, nf = sum(n_true), sum(n_false)
    se = float(np.sum(e ** 2)) + (nt - e.size) * cap * cap
    return {"depth_rmse_bins": round(float(np.sqrt(se / max(nt, 1))), 4),
            "depth_rmse_found_bins": round(float(np.sqrt(np.mean(e ** 2))) if e.size else 0.0, 4),
            "found": round(e.size / max(nt, 1), 4),
            "false_points_per_px": round(nf / max(n_pix, 1), 4)}


def depth_rmse(depth_true: np.ndarray, pt_off: np.ndarray, depth: np.ndarray, cap: float):
    """(RMSE over the true surfaces with misses counted at cap, fraction found)."""
    e, nt, _ = match_surfaces(depth_true, pt_off, depth, cap)
    s = depth_scores([e], [nt], [0], 1, cap)
    return s["depth_rmse_bins"], s["found"]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--scenes", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--rows", type=int, default=256)
    ap.add_argument("--cols", type=int, default=256)
    ap.add_argument("--bins", type=int, default=1024)
    ap.add_argument("--signal", type=float, default=2.0)
    ap.add_argument("--sbr", type=float, default=0.05)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=2e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True, help="checkpoint path")
    a = ap.parse_args(argv)
    import multiprocessing as mp
    # the workers start before this process touches the GPU
    ctx = mp.get_context("spawn")
    with ctx.Pool(a.workers) as workers:
        jobs = ((s, a.rows, a.cols, a.bins, a.signal, a.sbr) for s in range(a.scenes))
        lists = workers.imap(scene_lists, jobs, chunksize=1)
        import torch
        from . import rt3d, synth
        sc = synth.layers_scene(0, rows=8, cols=8, T=a.bins)
        m = sc.meta
        p = dict(dz=m["dz"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
        apss = rt3d.Context(sc.irf.probs, a.bins, **p)
        net = rt3d.Context(sc.irf.probs, a.bins, denoiser=rt3d.DENOISE_CNN, **p)
        t0 = time.perf_counter()
        hist = train_recipe(net, apss, lists, a.scenes, a.steps, rows=a.rows, cols=a.cols, lr=a.lr,
                            lr_final=a.lr_final, seed=a.seed,
                            log=lambda s: print(s, file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        net.denoiser_save(a.out)
        print(f"[train] {a.scenes} scenes, {a.steps} steps, loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}, "
              f"{time.perf_counter() - t0:.0f} s; checkpoint {a.out}", flush=True)


if __name__ == "__main__":
    main()
