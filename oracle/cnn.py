"""FP64 oracle of the learned depth denoiser (TEST INFRASTRUCTURE ONLY).

The paper's formulation lets any denoiser play the proximal step of the depth
block (Results, "Reconstruction algorithm"; Discussion: other point-cloud
denoisers can be plugged in to trade quality for speed).  This module defines
the small convolutional denoiser the GPU library implements, in plain numpy
float64: features, four 3x3 convolutions, ReLU, masked squared error, the
backward pass and Adam.  Only the tests, the smoke check and the benchmark's
CPU leg use it; it shares no code with the GPU library.

Reading (not in the paper; it only says denoisers are interchangeable):
  features, per pixel and slot k < 3 (valid_k = k < min(cnt, 3)):
    neighbours of slot k: the points (any slot) of the 5 x 5 window (same
          frame, inside the image, the point itself included) whose depth
          lies within GATE sigma_h of t_k -- the same surface, as the 3-D
          support of APSS selects it;
    d_k = clip((t_k - mean_k) / sigma_h, -8, 8), mean_k = their mean depth;
    a_k = log(1 + r_k);  v_k = 1;  n_k = their number / 25;
          (all four are 0 when slot k is invalid)
  channels [d0 a0 v0 n0 d1 a1 v1 n1 d2 a2 v2 n2] padded with zeros to 16;
  net: conv3x3(16->32)+ReLU, conv3x3(32->32)+ReLU, conv3x3(32->32)+ReLU,
       conv3x3(32->3), zero padding ("same"), weights w[ky][kx][cin][cout];
  output y_k = correction of slot k's depth in units of sigma_h;
  loss: sum over masked (pixel, slot) of (y_k - y*_k)^2 / max(1, count),
        y*_k = clip((t_true - t_k) / sigma_h, -8, 8);
  optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
Optional FP16 rounding points mirror the GPU's storage: features, weights,
activations after each layer, and the backward's incoming gradients.
"""
from __future__ import annotations

import numpy as np

CIN = (16, 32, 32, 32)
LIVE_IN = 12                      # feature channels that carry data (the rest pad to 16)
GATE = 3.0                        # neighbour depth gate in units of sigma_h
COUT = (32, 32, 32, 3)
N_PARAMS = sum(9 * ci * co + co for ci, co in zip(CIN, COUT))


def unflatten(w: np.ndarray):
    """Flat parameter vector -> [(W [3,3,cin,cout], b [cout]) x 4]."""
    out, at = [], 0
    for ci, co in zip(CIN, COUT):
        W = w[at:at + 9 * ci * co].reshape(3, 3, ci, co)
        at += 9 * ci * co
        b = w[at:at + co]
        at += co
        out.append((W, b))
    assert at == len(w)
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (float32), drawn from a seed."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in zip(CIN, COUT):
        fan_in = 9 * (LIVE_IN if ci == 16 else ci)  # the first layer has LIVE_IN live channels
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), 9 * ci * co))
        parts.append(np.zeros(co))
    w = np.concatenate(parts).astype(np.float32)
    w_layers = unflatten(w)
    w_layers[0][0][:, :, LIVE_IN:, :] = 0.0         # padding channels carry nothing
    return w


def f16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def features(t, r, cnt, sigma_h, F, H, W):
    """t, r: [P, K] (pixel-major, K >= 3); cnt [P] -> x [F, H, W, 16]."""
    K = np.asarray(t).shape[-1]
    t = np.asarray(t, dtype=np.float64).reshape(F, H, W, K)
    r = np.asarray(r, dtype=np.float64).reshape(F, H, W, K)
    call = np.minimum(np.asarray(cnt).reshape(F, H, W), K)
    c = np.minimum(call, 3)
    x = np.zeros((F, H, W, 16))
    for k in range(3):
        valid = c > k
        tk = np.where(valid, t[..., k], 0.0)
        s = np.zeros((F, H, W))
        n = np.zeros((F, H, W))
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                y0, y1 = max(0, -dy), min(H, H - dy)
                x0, x1 = max(0, -dx), min(W, W - dx)
                for k2 in range(K):
                    tm = t[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, k2]
                    ok = (call[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx] > k2) & \
                        (np.abs(tm - tk[:, y0:y1, x0:x1]) <= GATE * sigma_h)
                    s[:, y0:y1, x0:x1] += np.where(ok, tm, 0.0)
                    n[:, y0:y1, x0:x1] += ok
        mean = s / np.maximum(n, 1)
        x[..., 4 * k] = np.where(valid, np.clip((tk - mean) / sigma_h, -8, 8), 0.0)
        x[..., 4 * k + 1] = np.where(valid, np.log1p(np.where(valid, r[..., k], 0.0)), 0.0)
        x[..., 4 * k + 2] = valid
        x[..., 4 * k + 3] = np.where(valid, n / 25.0, 0.0)
    return x


def conv3x3(x, W, b):
    """'Same' 3x3 convolution (cross-correlation), zero padding, NHWC."""
    F, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (F, H, Wd, W.shape[3])).copy()
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[ky, kx]
    return y


def conv3x3_grads(x, W, dy):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    F, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, W.shape[2])
            dW[ky, kx] = xs.T @ dy.reshape(-1, W.shape[3])
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dy @ W[ky, kx].T
    return dxp[:, 1:H + 1, 1:Wd + 1, :], dW, dy.sum(axis=(0, 1, 2))


def forward(x, w, fp16=False):
    """Returns (y [F,H,W,3], activations list with the input first)."""
    layers = unflatten(np.asarray(w, dtype=np.float64))
    rnd = f16 if fp16 else (lambda a: a)
    acts = [rnd(x)]
    h = acts[0]
    for li, (W, b) in enumerate(layers):
        h = conv3x3(h, rnd(W), b)
        if li < 3:
            h = np.maximum(h, 0.0)
        h = rnd(h)
        acts.append(h)
    return h, acts


def loss_and_grad(x, w, target, mask, fp16=False):
    """Masked squared error and its gradient w.r.t. the flat weights.
    target, mask: [F, H, W, 3]."""
    layers = unflatten(np.asarray(w, dtype=np.float64))
    rnd = f16 if fp16 else (lambda a: a)
    y, acts = forward(x, w, fp16)
    m = mask.astype(np.float64)
    count = max(1.0, m.sum())
    diff = (y - target) * m
    loss = float((diff ** 2).sum() / count)
    g = rnd(2.0 * diff)                            # gradient of the sum, scaled below
    grads = [None] * 4
    for li in range(3, -1, -1):
        W, _ = layers[li]
        if li < 3:
            g = g * (acts[li + 1] > 0)
        dx, dW, db = conv3x3_grads(acts[li], rnd(W), g)
        grads[li] = (dW / count, db / count)
        g = rnd(dx)
    return loss, flatten(grads)


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def targets(t, cnt, truth, sigma_h, K=3):
    """Matched targets: slot k of a pixel (k < min(cnt, 3)) takes the nearest
    true depth of that pixel within 3 sigma_h; truth [S, P] (nan = absent).
    Returns (y* [P, 3], mask [P, 3])."""
    P = len(cnt)
    tgt = np.zeros((P, K))
    msk = np.zeros((P, K), dtype=bool)
    for p in range(P):
        for k in range(min(int(cnt[p]), K)):
            d = np.abs(truth[:, p] - t[p, k])
            d = np.where(np.isfinite(d), d, np.inf)
            s = int(np.argmin(d))
            if d[s] <= 3 * sigma_h:
                tgt[p, k] = np.clip((truth[s, p] - t[p, k]) / sigma_h, -8, 8)
                msk[p, k] = True
    return tgt, msk
