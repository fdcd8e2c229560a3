#!/usr/bin/env python3
"""Throughput of the whole reconstruction at the paper's raster-scan shape.

Workload: synthetic scenes of 141 x 141 pixels x 4613 bins shaped like the
paper's head scan (a bumpy back surface plus a 30%-coverage occluder 200 bins
nearer, ex-Gaussian IRF, 5 signal photons/pixel, SBR 0.1), uint16 histograms
resident in HBM.  One step = one call of the library's reconstruction on a
batch of frames: compaction of the histograms into active bins,
log-matched-filter initialisation, 20 iterations of depth / intensity /
background updates with APSS, the intensity low-pass + threshold and the
background filter, and output packing.

Prints one JSON line: frames/s (value), Gbin/s and photon-bins/s, the time
of every kernel group per call, the roofline of the group taking the most time
(timed live with HIP events over the timed region; HBM bytes from stored
FETCH_SIZE / WRITE_SIZE counters when they match the current sources), and the
FP64 CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s & Gbin/s RT3D at 141x141x4613; learned-vs-APSS at matched depth RMSE"
HBM_PEAK_GBS = 8000.0
ROWS, COLS, BINS = 141, 141, 4613


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """Thread count and CPU model of this host (the oracle's timing context):
    /proc/cpuinfo's model name and lscpu's model lines.  Call it before the
    GPU is initialised (it starts lscpu as a child process)."""
    import subprocess
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    lscpu = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "BIOS Model name", "Socket(s)", "Core(s) per socket",
                             "Thread(s) per core", "CPU(s)", "CPU max MHz"):
                lscpu[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"threads_available": n, "model": model, "lscpu": lscpu}


# The oracle on all host cores: one frame per process, the processes started
# (spawned, before the GPU is initialised) and released together.
_BARRIER = None


def _pool_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_frame(s):
    import oracle
    from paper_1905_06700_amd import synth
    sc = synth.head_scene(s)
    O = oracle.Oracle(oracle.Model(sc.irf.probs, BINS), oracle.Params(**scene_params(sc)))
    _BARRIER.wait()
    t0 = time.time()
    off, ent = oracle.compact(sc.Z[None])
    t1 = time.time()
    st = O.init(off, ent, oracle.State(1, ROWS, COLS, 4))
    t2 = time.time()
    for _ in range(20):
        O.iterate(off, ent, st)
    return t0, t1, t2, time.time()


def oracle_all_cores(workers=16):
    """Frames/s of the FP64 oracle with `workers` frames in parallel processes."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    n = max(1, min(workers, host_cpu()["threads_available"]))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(n)
    with ctx.Pool(n, initializer=_pool_init, initargs=(barrier,)) as pool:
        times = pool.map(_oracle_frame, range(n))
    wall = max(t[3] for t in times) - min(t[0] for t in times)
    per = [t[3] - t[0] for t in times]
    return {"value": round(n / wall, 4), "unit": "frames/s", "cores": n, "kind": "oracle",
            "sample": f"{n} full {ROWS}x{COLS}x{BINS} frames (compaction + init + 20 iterations), one per "
                      f"process on {n} host threads, {wall:.1f} s wall",
            "seconds_per_frame_median": round(sorted(per)[len(per) // 2], 2)}


def scene_params(sc):
    m = sc.meta
    return dict(dz=m["dz"], r_min=m["r_min"], r_init=1, k_init=m["k_init"])


# The init's integer score arithmetic (32-bit multiply-adds, 2 ops each) runs
# on the vector ALU: 64 lanes per CU per clock x 2 ops x 256 CUs x 2.4 GHz.
ALU_INT_PEAK_TOPS = 64 * 2 * 256 * 2.4e9 / 1e12

# Kernel groups timed one at a time by the library's event timer.
GROUPS = ["compact", "init", "normals", "depth", "apss", "intensity", "ifilter", "bkg", "bfilter", "output"]

# Library sources each group's code lives in (for matching stored byte counters).
GROUP_SOURCES = {"compact": ["k_compact.hip"], "init": ["k_init.hip"], "normals": ["k_init.hip"],
                 "depth": ["k_steps.hip"], "intensity": ["k_steps.hip"], "bkg": ["k_steps.hip"],
                 "apss": ["k_apss.hip"], "merge": ["k_apss.hip"], "ifilter": ["k_filter.hip"],
                 "bfilter": ["k_filter.hip"], "output": ["k_filter.hip", "k_compact.hip"]}


def algorithmic_bytes(kernel, F, N, T, E, pts):
    """Bytes a kernel group must move per launch over F frames of N pixels:
    E active entries, pts live points (see the design notes for each row)."""
    FN = F * N
    if kernel == "compact":
        return 2 * FN * T + 4 * E + 4 * (FN + 1)
    if kernel in ("depth", "intensity"):
        # entries + offsets + count + background, point depth (f64) and intensity read,
        # updated depth or intensity written (the intensity group also merges, which
        # for points in depth order and apart reads nothing more)
        wr = 8 if kernel == "depth" else 4
        return 4 * E + 4 * (FN + 1) + FN + 4 * FN + 12 * pts + wr * pts
    if kernel == "bkg":
        return 4 * E + 4 * (FN + 1) + FN + 8 * FN + 12 * pts
    if kernel == "apss":
        # read the count of every pixel and t (f64), n of every point once; write t, n
        return pts * (8 + 12) * 2 + FN
    if kernel == "merge":
        return 2 * pts * (8 + 4 + 12) + 2 * FN
    if kernel == "ifilter":
        return 24 * pts + 2 * FN
    if kernel == "bfilter":
        return 16 * FN
    if kernel == "normals":
        return 8 * pts + FN + 12 * pts
    if kernel == "output":
        return pts * (8 + 4 + 12) + 4 * (FN + 1) + 4 * FN + FN + 8 * pts
    raise KeyError(kernel)


def roofline_of(kernel, F, N, T, E, pooled, L, pts, avg_ms):
    """Roofline object of one kernel group from its average launch time: HBM
    bound with algorithmic bytes, except the init, which is bound by its
    integer score arithmetic: 2 ops x L lags per pooled active entry (the
    exact log-matched filter over every tau)."""
    if kernel == "init":
        ops = 2.0 * pooled * L
        achieved = ops / (avg_ms / 1e3) / 1e12
        return {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 3), "peak": ALU_INT_PEAK_TOPS,
                "unit": "TOP/s", "frac": round(achieved / ALU_INT_PEAK_TOPS, 4), "traffic": None,
                "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_ops_per_launch": int(ops)}
    abytes = algorithmic_bytes(kernel, F, N, T, E, pts)
    achieved = abytes / (avg_ms / 1e3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "avg_launch_us": round(avg_ms * 1e3, 2),
            "algorithmic_bytes_per_launch": int(abytes)}


def stored_traffic(kernel, frames):
    """HBM bytes per launch measured with FETCH_SIZE / WRITE_SIZE counters
    (profiles/traffic_<kernel>_head141x141x4613.md), or None when the
    kernel's sources changed since the counters were taken or the counters
    were taken at another number of frames per launch."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_head141x141x4613.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("traffic "):
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
    if not rec:
        return None
    h = hashlib.sha256()
    for f in GROUP_SOURCES[kernel] + ["rt3d_dev.h"]:
        h.update(open(os.path.join(ROOT, "paper_1905_06700_amd", "csrc", f), "rb").read())
    if rec.get("sources_sha256") != h.hexdigest() or int(rec.get("frames", 0)) != frames:
        return None
    return int(float(rec["bytes_per_launch"]))


def small_frames(F=64, reps=5):
    """Batches of small frames (config 1 plane scenes, 32 x 32 x 300), where
    the ~140 launches of a call dominate: direct calls against replays of a
    recorded graph."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    scenes = [synth.plane_scene(s) for s in range(4)]
    sc = scenes[0]
    R, C, T = sc.rows, sc.cols, sc.T
    Z = torch.stack([torch.from_numpy(scenes[f % 4].Z.view(np.int16)) for f in range(F)]).cuda()
    m = sc.meta
    ctx = rt3d.Context(sc.irf.probs, T, dz=m["dz"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
    ctx.workspace(F, R, C, F * R * C * 64)
    out = ctx.make_output(F * R * C)
    res = {"workload": f"{F} frames of {R}x{C}x{T} (tilted plane, 10 signal + 1 background photon/px) per call"}
    g = ctx.graph(out, F, R, C, hist=Z)
    for name, run in (("direct", lambda: ctx.reconstruct_into(out, F, R, C, hist=Z)), ("graph", g.launch)):
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"call_ms_{name}"] = round(ms, 3)
        res[f"frames_per_s_{name}"] = round(F / (ms / 1e3), 1)
    del g
    return res


def uneven_frames(reps=3):
    """Eight scenes of different sizes (sides 48 .. 160 pixels, 1024 bins,
    head-shaped generator with the config-2 IRF, 3 signal photons/px at SBR
    0.5): one call over all of them (neighbour steps per size group) against
    one call per scene, back to back on the stream."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    sides = [48, 64, 80, 96, 112, 128, 144, 160]
    T = 1024
    scs = [synth.head_scene(64 + k, rows=n, cols=n, T=T, signal=3.0, sbr=0.5) for k, n in enumerate(sides)]
    m = scs[0].meta
    ctx = rt3d.Context(scs[0].irf.probs, T, dz=m["dz"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
    Zs = [torch.from_numpy(np.ascontiguousarray(sc.Z).view(np.int16)).cuda() for sc in scs]
    Z = torch.cat([z.reshape(-1, T) for z in Zs]).contiguous()
    P = int(Z.shape[0])
    ctx.workspace(1, 1, P, P * 64)
    out = ctx.make_output(P)
    outs = [ctx.make_output(n * n) for n in sides]
    shapes = [(n, n) for n in sides]

    def one_call():
        ctx.reconstruct_into(out, len(sides), 1, 1, hist=Z, frame_shapes=shapes)

    def per_scene():
        for n, z, o in zip(sides, Zs, outs):
            ctx.reconstruct_into(o, 1, n, n, hist=z)

    res = {"workload": f"8 scenes of {sides[0]}^2 .. {sides[-1]}^2 pixels x {T} bins ({P} pixels), one call "
                       "against one call per scene"}
    for name, run in (("one_call", one_call), ("per_scene", per_scene)):
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"ms_{name}"] = round(ms, 3)
        res[f"scenes_per_s_{name}"] = round(len(sides) / (ms / 1e3), 1)
    return res


def hbm_regime(scenes, F=64):
    """The gradient-step and APSS kernels where their data no longer fits the
    256 MB MALL: F head-shaped frames per call (the entries alone take 4.3 MB
    per frame).  Per kernel group: average launch time, algorithmic bytes per
    launch and the fraction of the 8 TB/s HBM peak they make."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d

    sc0 = scenes[0]
    n = len(scenes)
    Z = torch.stack([torch.from_numpy(scenes[f % n].Z.view(np.int16)) for f in range(F)]).cuda()
    ctx = rt3d.Context(sc0.irf.probs, BINS, **scene_params(sc0))
    ctx.workspace(F, ROWS, COLS, int(F * ROWS * COLS * 200))
    P = F * ROWS * COLS
    out = ctx.make_output(P)
    ctx.reconstruct_into(out, F, ROWS, COLS, hist=Z)
    st = ctx.query()
    E, pts = int(st.entries), int(out.pt_off[-1].item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.reconstruct_into(out, F, ROWS, COLS, hist=Z)
    e1.record()
    torch.cuda.synchronize()
    res = {"workload": f"{F} frames of {ROWS}x{COLS}x{BINS} per call (entries {E * 4 / 1e6:.0f} MB, past the MALL)",
           "frames_per_s": round(F / (e0.elapsed_time(e1) / 1e3), 1)}
    for g in ("depth", "intensity", "bkg", "apss"):
        ctx.profile(g)
        ctx.reconstruct_into(out, F, ROWS, COLS, hist=Z)
        torch.cuda.synchronize()
        ms, nl = ctx.profile_read()
        ctx.profile(None)
        avg = ms / max(int(nl), 1)
        ab = algorithmic_bytes(g, F, ROWS * COLS, BINS, E, pts)
        gbs = ab / (avg / 1e3) / 1e9
        res[g] = {"avg_launch_us": round(avg * 1e3, 2), "algorithmic_bytes_per_launch": int(ab),
                  "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        if g == "apss":
            res[g].update(apss_valu(pts, avg))
    del Z
    return res


# APSS arithmetic: 40 flop per neighbour evaluation over the (2R+1)^2 window
# (R = ceil(h_apss / p_xy) = 2) and the live points of each window pixel.
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector peak (counts packed FP32 instructions)
FP32_NONPACKED_TFLOPS = 78.6      # without packed FP32 instructions, as this library is built


def apss_valu(pts, avg_ms, R=2, N=ROWS * COLS, F=64):
    """APSS flops per launch (40 (2R+1)^2 K flop per point, K = live points per
    pixel) against the FP32 vector peaks."""
    K = pts / (F * N)
    flops = 40.0 * (2 * R + 1) ** 2 * K * pts
    tf = flops / (avg_ms / 1e3) / 1e12
    return {"algorithmic_flops_per_launch": int(flops), "achieved_TFLOPs": round(tf, 2),
            "frac_valu": round(tf / FP32_PEAK_TFLOPS, 4), "frac_valu_nonpacked": round(tf / FP32_NONPACKED_TFLOPS, 4)}


def stress_batch(reps=3):
    """The stress configuration: one uneven batch of 8 multi-layer scenes with
    sides 128 .. 512 pixels x 2000 bins (1 signal photon per pixel at SBR
    0.01, ~98 active bins per pixel, 15% of the pixels empty), 857 k pixels
    and 3.4 GB of histograms per call, a working set well past the 256 MB
    MALL.  Call time, and per kernel group the average launch time and the
    fraction of the 8 TB/s HBM peak its algorithmic bytes make."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    sides = (128, 160, 192, 256, 320, 384, 448, 512)
    parts, sc0 = [], None
    for k, n in enumerate(sides):
        log(f"[bench] stress: generating {n}x{n}x2000")
        sc = synth.stress_scene(k, side=n)
        sc0 = sc0 or sc
        parts.append(torch.from_numpy(sc.Z.view(np.int16).reshape(-1, sc.T)).cuda())
        del sc
    Z = torch.cat(parts).contiguous()
    del parts
    P, T = int(Z.shape[0]), int(Z.shape[1])
    shapes = [(n, n) for n in sides]
    m = sc0.meta
    ctx = rt3d.Context(sc0.irf.probs, T, dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"], r_init=m["r_init"],
                       k_init=m["k_init"])
    ctx.workspace(1, 1, P, P * 130)
    out = ctx.make_output(P)
    run = lambda: ctx.reconstruct_into(out, len(sides), 1, 1, hist=Z, frame_shapes=shapes)
    run()
    torch.cuda.synchronize()
    st = ctx.query()
    assert st.device_error == 0
    E, pts = int(st.entries), int(out.pt_off[-1].item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"workload": f"8 scenes {sides[0]}^2..{sides[-1]}^2 x {T} bins in one call ({P} pixels, "
                       f"{E / P:.1f} active bins/px, 1 signal photon/px, SBR 0.01)",
           "call_ms": round(ms, 3), "frames_per_s": round(len(sides) / (ms / 1e3), 1),
           "gbin_per_s": round(P * T / (ms / 1e3) / 1e9, 1), "points": pts}
    for g in GROUPS:
        ctx.profile(g)
        run()
        torch.cuda.synchronize()
        gms, nl = ctx.profile_read()
        ctx.profile(None)
        nl = max(int(nl), 1)
        avg = gms / nl
        r = {"ms_per_call": round(gms, 3), "launches": nl, "avg_launch_us": round(avg * 1e3, 1)}
        if g != "init":
            ab = algorithmic_bytes(g, 1, P, T, E, pts)
            r["frac_hbm"] = round(ab / (avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        res[g] = r
    del Z, out, ctx
    torch.cuda.empty_cache()
    return res


def super_resolution(reps=5):
    """The paper's array-video mode: 32 x 32 x 153 lidar frames (a moving disc
    over a tilted plane, 3 signal photons/px at SBR 0.5) reconstructed on a
    96 x 96 point grid (s = 3): one frame per call, direct and replayed from a
    recorded graph (the paper's per-frame latency), and 64 frames per call."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    s, R, C = 3, 32, 32
    scs = [synth.sr_scene(k, rows=R, cols=C, s=s) for k in range(8)]
    sc, m = scs[0], scs[0].meta
    ctx = rt3d.Context(sc.irf.probs, sc.T, sr=s, dz=m["dz"], p_xy=m["p_xy"], r_min=m["r_min"],
                       r_init=m["r_init"], k_init=m["k_init"])
    res = {"workload": f"{R}x{C}x{sc.T} lidar frames on a {R * s}x{C * s} point grid (moving disc over a plane, "
                       "3 signal photons/px, SBR 0.5), 20 iterations, APSS",
           "paper_context": {"ms_per_frame": 20, "hardware": "NVIDIA Titan Xp", "data": "real 32x32x153 array "
                             "video at 320 m reconstructed on 96x96"}}

    def timed(run):
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for F in (1, 64):
        Z = torch.stack([torch.from_numpy(scs[f % len(scs)].Z.view(np.int16)) for f in range(F)]).cuda()
        ctx.workspace(F, R, C, F * R * C * sc.T)
        out = ctx.make_output(F * R * C * s * s, n_bg=F * R * C)
        ms = timed(lambda: ctx.reconstruct_into(out, F, R, C, hist=Z))
        res[f"call_ms_{F}_frames"] = round(ms, 3)
        res[f"frames_per_s_{F}_frames"] = round(F / (ms / 1e3), 1)
        if F == 1:
            g = ctx.graph(out, F, R, C, hist=Z)
            ms = timed(g.launch)
            res["call_ms_1_frame_graph"] = round(ms, 3)
            del g
        else:
            ctx.profile("depth")
            ctx.reconstruct_into(out, F, R, C, hist=Z)
            torch.cuda.synchronize()
            kms, n = ctx.profile_read()
            ctx.profile(None)
            res["depth_step_us_64_frames"] = round(kms / max(int(n), 1) * 1e3, 2)
        assert ctx.query().device_error == 0
    return res


def observation_model(scenes, F=16, reps=3):
    """Cost of the observation-model options on the head-shaped frames (16
    per call): three per-pixel IRF classes (the scene's ex-Gaussian and two
    Gaussians, on seeded 4 x 4 pixel blocks; each IRF-dependent kernel runs
    once per class) and the pinhole camera (persp = 1/115, a pixel footprint
    of about one world unit at the scene's ~115-unit range, p_xy = 0.9),
    against the default single IRF and orthographic map.  Timing only: the
    photons come from the scene's one IRF and orthographic geometry."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    n = len(scenes)
    sc0 = scenes[0]
    Z = torch.stack([torch.from_numpy(scenes[f % n].Z.view(np.int16)) for f in range(F)]).cuda()
    P = F * ROWS * COLS
    rng = np.random.default_rng(synth.seed_of(6, 99))
    blocks = rng.integers(0, 3, (F, (ROWS + 3) // 4, (COLS + 3) // 4))
    cls = np.kron(blocks, np.ones((1, 4, 4), np.int64))[:, :ROWS, :COLS].astype(np.uint8)
    cls_d = torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda()
    base = scene_params(sc0)
    variants = {"single_irf": (rt3d.Context(sc0.irf.probs, BINS, **base), None),
                "three_irf_classes": (rt3d.Context(sc0.irf.probs, BINS, **base), cls_d),
                "pinhole_camera": (rt3d.Context(sc0.irf.probs, BINS, **dict(base, persp=1 / 115.0, p_xy=0.9)), None)}
    for i in (synth.gaussian_irf(1.5, 9), synth.gaussian_irf(3.0, 12)):
        variants["three_irf_classes"][0].add_irf(i.probs)
    res = {"workload": f"{F} frames of {ROWS}x{COLS}x{BINS} (head-shaped) per call"}
    for name, (ctx, c) in variants.items():
        ctx.workspace(F, ROWS, COLS, int(P * 200))
        out = ctx.make_output(P)

        def run():
            ctx.reconstruct_into(out, F, ROWS, COLS, hist=Z, irf_class=c)

        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        r = {"call_ms": round(ms, 3), "frames_per_s": round(F / (ms / 1e3), 1)}
        for g in ("init", "depth", "apss", "ifilter"):
            ctx.profile(g)
            run()
            torch.cuda.synchronize()
            kms, nl = ctx.profile_read()
            ctx.profile(None)
            r[f"{g}_ms_per_call"] = round(kms, 4)
        assert ctx.query().device_error == 0
        res[name] = r
    del Z
    return res


def video_and_scenes(reps=5):
    """Batched video with scenes in one launch: 64 frames of 32 x 32 x 153 (a
    disc moving over a plane, 3 signal photons/px at SBR 0.5, zero-padded to
    1024 bins, the video camera's Gaussian IRF as a second IRF class) with 16
    head-shaped scenes of 96 x 96 x 1024 (3 signal photons/px, SBR 0.5)."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    T = 1024
    video = [synth.sr_scene(k, rows=32, cols=32, s=1, T=153) for k in range(64)]
    scenes = [synth.head_scene(700 + k, rows=96, cols=96, T=T, signal=3.0, sbr=0.5) for k in range(16)]
    frames = []
    for sc in video:
        z = np.zeros((32, 32, T), np.uint16)
        z[..., :sc.T] = sc.Z
        frames.append(z)
    frames += [sc.Z for sc in scenes]
    shapes = [(32, 32)] * 64 + [(96, 96)] * 16
    cls = torch.from_numpy(np.concatenate([np.full(32 * 32, 1, np.uint8)] * 64 +
                                          [np.zeros(96 * 96, np.uint8)] * 16)).cuda()
    Z = torch.cat([torch.from_numpy(z.view(np.int16)).cuda().reshape(-1, T) for z in frames]).contiguous()
    P = int(Z.shape[0])
    ctx = rt3d.Context(scenes[0].irf.probs, T, dz=scenes[0].meta["dz"], r_min=0.6, r_init=1, k_init=3)
    ctx.add_irf(video[0].irf.probs)
    ctx.workspace(1, 1, P, P * 64)
    out = ctx.make_output(P)

    def run():
        ctx.reconstruct_into(out, len(frames), 1, 1, hist=Z, frame_shapes=shapes, irf_class=cls)

    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert ctx.query().device_error == 0
    return {"workload": "64 frames of 32x32x153 (padded to 1024 bins, second IRF class) + 16 scenes of "
                        "96x96x1024 in one call", "call_ms": round(ms, 3),
            "frames_per_s": round(len(frames) / (ms / 1e3), 1)}


def execution_time_sweep(reps=5):
    """Time per frame as the frame grows and as the active bins per pixel grow
    (Results, execution time of the method: pixel counts 32^2 .. 400^2 at about
    4 active bins per pixel; 141 x 141 frames with the background raised until
    2 .. 128 bins per pixel are active).  Head-shaped scenes, T = 4613, the
    config-2 IRF.  Each point is timed two ways: one frame per call (the
    paper's per-frame time), and frames batched up to ~16 x 141^2 pixels per
    call (copies of the one frame), the per-frame cost when the GPU is full."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    def point(sc):
        n = sc.rows * sc.cols
        F = max(1, min(16, round(16 * ROWS * COLS / n), int(3e9 // (n * BINS * 2))))
        Z1 = torch.from_numpy(sc.Z.view(np.int16)).cuda()
        a_est = float((sc.Z != 0).sum()) / n
        ctx = rt3d.Context(sc.irf.probs, BINS, **scene_params(sc))
        ctx.workspace(F, sc.rows, sc.cols, int(F * n * (1.5 * a_est + 64)))
        res = {}
        for tag, f in (("single", 1), ("batched", F)):
            Z = Z1[None].expand(f, -1, -1, -1).contiguous()
            out = ctx.make_output(f * n)
            for _ in range(2):
                ctx.reconstruct_into(out, f, sc.rows, sc.cols, hist=Z)
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ctx.reconstruct_into(out, f, sc.rows, sc.cols, hist=Z)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            st = ctx.query()
            assert st.device_error == 0
            res[f"ms_per_frame_{tag}"] = round(float(np.median(ms)) / f, 4)
            if tag == "batched":
                res["frames_per_batch"] = f
            res["active_bins_per_px"] = round(st.entries / (f * n), 2)
            del Z, out
        del ctx, Z1
        torch.cuda.empty_cache()
        return res

    pixels = []
    for k, side in enumerate((32, 64, 96, 141, 200, 283, 400)):
        sc = synth.head_scene(50 + k, rows=side, cols=side, signal=3.0, sbr=2.5)
        log(f"[bench] sweep: {side}x{side}x{BINS}")
        pixels.append(dict(pixels=side * side, side=side, **point(sc)))
    bins = []
    for k, A in enumerate((2, 4, 8, 16, 32, 64, 128)):
        sig = min(3.0, 0.75 * A)
        sc = synth.head_scene(60 + k, signal=sig, sbr=sig / (A - sig))
        log(f"[bench] sweep: {ROWS}x{COLS}x{BINS}, about {A} active bins/px")
        bins.append(dict(target_active_bins=A, **point(sc)))
    return {"workload": "head-shaped scenes, T=4613, config-2 IRF; (a) sides 32..400 at ~3 signal + "
                        "1.2 background photons/px; (b) 141x141 with background raised to 2..128 "
                        "active bins/px",
            "pixels": pixels, "active_bins": bins}


DENOISER_CHECKPOINT = os.path.join(ROOT, "paper_1905_06700_amd", "weights", "denoiser_c4.rt3dcnn")
# the same recipe on scenes of the brighter regime (6 signal photons/px, SBR 0.2)
DENOISER_CHECKPOINT_BRIGHT = os.path.join(ROOT, "paper_1905_06700_amd", "weights", "denoiser_bright.rt3dcnn")


def _evaluate(ctx, scenes, rows, cols, bins, sig, batch=16):
    """Reconstructs `scenes` in calls of `batch` frames; returns frames/s (of
    the first full call, timed over 3 repeats) and the depth scores of
    S33-style greedy matching within 3 sigma_h."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import train

    P1 = rows * cols
    errs, n_true, n_false, fps = [], [], [], None
    for b0 in range(0, len(scenes), batch):
        part = scenes[b0:b0 + batch]
        F = len(part)
        Z = torch.stack([torch.from_numpy(s.Z.view(np.int16)) for s in part]).cuda()
        ctx.workspace(F, rows, cols, F * P1 * 200)
        res = ctx.make_output(F * P1)
        ctx.reconstruct_into(res, F, rows, cols, hist=Z)
        torch.cuda.synchronize()
        if fps is None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                ctx.reconstruct_into(res, F, rows, cols, hist=Z)
            e1.record()
            torch.cuda.synchronize()
            fps = 3 * F / (e0.elapsed_time(e1) / 1e3)
        pt = res.pt_off.cpu().numpy().view(np.uint32).astype(np.int64)
        dep = res.depth.cpu().numpy()
        for f, sc in enumerate(part):
            sl = pt[f * P1:(f + 1) * P1 + 1] - pt[f * P1]
            e, nt, nf = train.match_surfaces(sc.depth.reshape(sc.depth.shape[0], -1), sl, dep[pt[f * P1]:], 3 * sig)
            errs.append(e)
            n_true.append(nt)
            n_false.append(nf)
        del Z, res
    out = {"frames_per_s": round(fps, 2)}
    out.update(train.depth_scores(errs, n_true, n_false, len(scenes) * P1, 3 * sig))
    return out


def learned_vs_apss(rows=256, cols=256, bins=1024, n_eval=50, n_high=16):
    """Learned denoiser against plain APSS: the network of the committed
    checkpoint (trained on the GPU by paper_1905_06700_amd/train.py's recipe:
    config-4 scenes, inputs recorded at iterations 1, 2, 5, 10, 20 of APSS runs,
    64 x 64 crops, batch 32), else a short training run here.  Both paths
    reconstruct the held-out config-4 scenes (seeds 10000 .. 10000 + n_eval - 1,
    2 signal photons/px, SBR 0.05) and a brighter regime (6 photons/px, SBR
    0.2) where most surfaces are found; depth scores by greedy matching within
    3 sigma_h (misses count 3 sigma_h), frames/s on 16-frame calls."""
    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth, train

    sc0 = synth.layers_scene(0, rows=8, cols=8, T=bins)
    m = sc0.meta
    p = dict(dz=m["dz"], r_min=m["r_min"], r_init=m["r_init"], k_init=m["k_init"])
    apss = rt3d.Context(sc0.irf.probs, bins, **p)
    net = rt3d.Context(sc0.irf.probs, bins, denoiser=rt3d.DENOISE_CNN, **p)
    if os.path.exists(DENOISER_CHECKPOINT):
        net.denoiser_load(DENOISER_CHECKPOINT)
        training = {"checkpoint": os.path.relpath(DENOISER_CHECKPOINT, ROOT)}
    else:
        n_train = 64
        log(f"[bench] learned denoiser: no checkpoint, training on {n_train} scenes here")
        lists = (train.scene_lists((s, rows, cols, bins, 2.0, 0.05)) for s in range(n_train))
        t0 = time.perf_counter()
        hist = train.train_recipe(net, apss, lists, n_train, steps=800, rows=rows, cols=cols, log=log)
        training = {"scenes": n_train, "steps": 800, "first_loss": round(hist[0][1], 4),
                    "final_loss": round(hist[-1][1], 4), "seconds_incl_data": round(time.perf_counter() - t0, 1)}
    sig = float(np.sqrt(apss.sigma2))
    log(f"[bench] learned denoiser: generating {n_eval} held-out config-4 scenes")
    ev = [synth.layers_scene(10000 + s, rows=rows, cols=cols, T=bins) for s in range(n_eval)]
    out = {"workload": f"{rows}x{cols}x{bins} multi-layer scenes (up to 3 surfaces, 2 signal photons/px, SBR 0.05), "
                       f"held-out seeds 10000..{10000 + n_eval - 1}, 16 frames per call",
           "training": training}
    for name, ctx in (("apss", apss), ("cnn", net)):
        out[name] = _evaluate(ctx, ev, rows, cols, bins, sig)
    del ev
    hi = [synth.layers_scene(10000 + s, rows=rows, cols=cols, T=bins, signal=6.0, sbr=0.2) for s in range(n_high)]
    out["bright"] = {"workload": f"{rows}x{cols}x{bins} multi-layer scenes, 6 signal photons/px, SBR 0.2, "
                                 f"held-out seeds 10000..{10000 + n_high - 1}"}
    out["bright"]["apss"] = _evaluate(apss, hi, rows, cols, bins, sig)
    out["bright"]["cnn_config4_weights"] = _evaluate(net, hi, rows, cols, bins, sig)
    if os.path.exists(DENOISER_CHECKPOINT_BRIGHT):
        net.denoiser_load(DENOISER_CHECKPOINT_BRIGHT)
        out["bright"]["training"] = {"checkpoint": os.path.relpath(DENOISER_CHECKPOINT_BRIGHT, ROOT)}
    out["bright"]["cnn"] = _evaluate(net, hi, rows, cols, bins, sig)
    for d in (out, out["bright"]):
        d["rmse_ratio_cnn_over_apss"] = round(d["cnn"]["depth_rmse_bins"] / d["apss"]["depth_rmse_bins"], 4)
        d["rmse_found_ratio_cnn_over_apss"] = round(d["cnn"]["depth_rmse_found_bins"] /
                                                    max(d["apss"]["depth_rmse_found_bins"], 1e-9), 4)
        d["speedup_cnn_over_apss"] = round(d["cnn"]["frames_per_s"] / d["apss"]["frames_per_s"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=32,
                    help="frames per reconstruction call (32: where frames/s levels off)")
    ap.add_argument("--kernel", default="", help="kernel group for the roofline object (default: the one "
                                                  "taking the most time per call)")
    ap.add_argument("--cpu-frames", type=int, default=2, help="frames the oracle times (0 = skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-APSS leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the execution-time sweep")
    ap.add_argument("--no-stress", action="store_true", help="skip the stress batch (8 scenes up to 512^2 x "
                                                             "2000; about a minute of scene generation)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy kernel of known size, the "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); frames are "
              "independent, so N GPUs would each take whole frames (see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    # the oracle on every host core first: its worker processes start before
    # this process touches the GPU
    cpu_all = oracle_all_cores() if args.cpu_frames > 0 else None
    host = host_cpu()

    import numpy as np
    import torch

    from paper_1905_06700_amd import rt3d, synth

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nbytes} bytes done")
        del src, dst

    F = args.frames
    n_distinct = min(F, 8)
    log(f"[bench] generating {n_distinct} distinct {ROWS}x{COLS}x{BINS} scenes")
    scenes = [synth.head_scene(s) for s in range(n_distinct)]
    sc0 = scenes[0]
    Zs = [torch.from_numpy(s.Z.view(np.int16)) for s in scenes]
    Z = torch.stack([Zs[f % n_distinct] for f in range(F)]).cuda()
    torch.cuda.synchronize()
    log(f"[bench] {F} frames resident on the GPU ({Z.numel() * 2 / 1e9:.2f} GB)")

    ctx = rt3d.Context(sc0.irf.probs, BINS, **scene_params(sc0))
    max_entries = int(F * ROWS * COLS * 200)
    ctx.workspace(F, ROWS, COLS, max_entries)
    P = F * ROWS * COLS
    out = ctx.make_output(P)

    def step():
        ctx.reconstruct_into(out, F, ROWS, COLS, hist=Z)

    for _ in range(args.warmup):
        step()
    st = ctx.query()
    E = int(st.entries)
    pts = int(out.pt_off[-1].item())
    log(f"[bench] warmup done: {E} active entries, {pts} points")

    # time of each kernel group per call (one call each, events around its launches);
    # the roofline object follows the group that takes the most, timed again live
    # over the timed region below
    group = {}
    for g in GROUPS:
        ctx.profile(g)
        step()
        torch.cuda.synchronize()
        ms, n = ctx.profile_read()
        ctx.profile(None)
        group[g] = (ms, int(n))
    gtotal = sum(v[0] for v in group.values())
    kernel = args.kernel or max(group, key=lambda g: group[g][0])
    log(f"[bench] kernel groups per call: " + ", ".join(f"{g} {group[g][0]:.3f} ms" for g in GROUPS))

    ctx.profile(kernel)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kms, klaunch = ctx.profile_read()
    ctx.profile(None)
    ctx.query()

    ms_per_step = gpu_ms / args.steps
    fps = F * args.steps / (gpu_ms / 1e3)
    gbin = F * ROWS * COLS * BINS * args.steps / (gpu_ms / 1e3) / 1e9
    pbin = E * args.steps / (gpu_ms / 1e3)

    # single-frame latency
    out1 = ctx.make_output(ROWS * COLS)
    Z1 = Z[:1].contiguous()
    for _ in range(2):
        ctx.reconstruct_into(out1, 1, ROWS, COLS, hist=Z1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.reconstruct_into(out1, 1, ROWS, COLS, hist=Z1)
    e1.record()
    torch.cuda.synchronize()
    latency_ms = e0.elapsed_time(e1) / 5
    # the same frame replayed from a recorded graph (one launch per call)
    g1 = ctx.graph(out1, 1, ROWS, COLS, hist=Z1)
    for _ in range(2):
        g1.launch()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        g1.launch()
    e1.record()
    torch.cuda.synchronize()
    latency_graph_ms = e0.elapsed_time(e1) / 5
    del g1

    # pooled active entries (the init's (2 r_init + 1)^2 windows, r_init = 1)
    nz = (Z != 0).sum(dim=-1, dtype=torch.int64)
    pad = torch.nn.functional.pad(nz, (1, 1, 1, 1))
    pooled = int(sum(pad[:, 1 + di:ROWS + 1 + di, 1 + dj:COLS + 1 + dj].sum().item()
                     for di in (-1, 0, 1) for dj in (-1, 0, 1)))
    avg_ms = kms / max(klaunch, 1)
    roofline = roofline_of(kernel, F, ROWS * COLS, BINS, E, pooled, len(sc0.irf.probs), pts, avg_ms)
    roofline["launches"] = int(klaunch)
    traffic = stored_traffic(kernel, F)
    if traffic is not None:
        roofline["traffic"] = traffic
    kernels = {g: {"ms_per_call": round(group[g][0], 4), "launches_per_call": group[g][1],
                   "share": round(group[g][0] / gtotal, 4)} for g in GROUPS}
    # the whole call against HBM: histogram bins at 2 bytes each read once
    # (the compaction's floor), and every HBM-bound group's algorithmic bytes
    # (the init, bound by its integer arithmetic, counts its pooled reads of
    # L2-resident entries as 4 bytes per own entry)
    call_bytes = sum(algorithmic_bytes(g, F, ROWS * COLS, BINS, E, pts) * group[g][1]
                     for g in GROUPS if g != "init") + 4 * E
    call_roofline = {
        "histogram_bins_per_s": round(gbin * 1e9, 1),
        "bins_per_s_at_hbm_peak": HBM_PEAK_GBS * 1e9 / 2,
        "frac_bins": round(gbin * 1e9 / (HBM_PEAK_GBS * 1e9 / 2), 4),
        "algorithmic_bytes_per_call": int(call_bytes),
        "achieved_GBs": round(call_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "frac_hbm": round(call_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    cpu = None
    if args.cpu_frames > 0:
        import oracle
        oracle.build(force=False)
        m = oracle.Model(sc0.irf.probs, BINS)
        O = oracle.Oracle(m, oracle.Params(**scene_params(sc0)))
        nf = args.cpu_frames
        log(f"[bench] timing the FP64 oracle on {nf} full frames (1 thread)")
        split = {"compaction": 0.0, "init": 0.0, "iterations": 0.0}
        for f in range(nf):
            t0 = time.perf_counter()
            off, ent = oracle.compact(scenes[f % n_distinct].Z[None])
            t1 = time.perf_counter()
            s = O.init(off, ent, oracle.State(1, ROWS, COLS, 4))
            t2 = time.perf_counter()
            for _ in range(20):
                O.iterate(off, ent, s)
            t3 = time.perf_counter()
            split["compaction"] += t1 - t0
            split["init"] += t2 - t1
            split["iterations"] += t3 - t2
        el = sum(split.values())
        single = {"value": round(nf / el, 4), "unit": "frames/s", "cores": 1,
                  "sample": f"{nf} full {ROWS}x{COLS}x{BINS} frames (compaction + init + 20 iterations), "
                            f"{el:.1f} s on one host thread",
                  "gbin_per_s": round(nf * ROWS * COLS * BINS / el / 1e9, 4),
                  "ms_per_frame_split": {k: round(v * 1e3 / nf, 1) for k, v in split.items()}}
        cpu = dict(cpu_all, single_thread=single, host=host)

    res = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "141x141x4613 head-shaped synthetic scene (bumpy surface + 30% occluder, "
                               "ex-Gaussian IRF, 5 signal photons/px, SBR 0.1), 20 iterations, APSS",
                   "frames_per_step": F, "rows": ROWS, "cols": COLS, "bins": BINS, "iterations": 20},
        "gbin_per_s": round(gbin, 2), "photon_bins_per_s": round(pbin, 1),
        "active_entries_per_frame": E // F, "points_per_frame": pts // F,
        "single_frame_latency_ms": round(latency_ms, 3), "single_frame_latency_graph_ms": round(latency_graph_ms, 3),
        "small_frames": small_frames(), "uneven_frames": uneven_frames(), "hbm_regime": hbm_regime(scenes),
        "super_resolution": super_resolution(), "observation_model": observation_model(scenes),
        "video_and_scenes": video_and_scenes(),
        "execution_time_sweep": None if args.no_sweep else execution_time_sweep(),
        "stress_batch": None if args.no_stress else stress_batch(),
        "wall_s": round(wall, 3),
        "roofline": roofline, "call_roofline": call_roofline, "kernels": kernels, "cpu_baseline": cpu,
        "learned_vs_apss": None if args.no_learned else learned_vs_apss(),
        "paper_context": {"frames_per_s": 76.9, "ms_per_frame": 13, "hardware": "NVIDIA Titan Xp",
                          "data": "real head scan, ~3 photons/px, SBR 13"},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
