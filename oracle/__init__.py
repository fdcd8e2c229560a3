"""FP64 CPU oracle (test infrastructure only).

The C library ``rt3d_oracle.c`` is the plain, slow reference the GPU library
is checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the GPU
library.  This module builds the C file with gcc and wraps it with ctypes;
every array is numpy float64 / int32 in the pixel-major layout documented in
``rt3d_oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt3d_oracle.c")
_LIB = os.path.join(_HERE, "librt3d_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, no fast-math, single threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Params(C.Structure):
    _fields_ = [("n_iter", C.c_int), ("k_max", C.c_int), ("k_init", C.c_int),
                ("p_xy", C.c_double), ("dz", C.c_double), ("h_apss", C.c_double),
                ("h_int", C.c_double), ("beta_t", C.c_double), ("dmax", C.c_double),
                ("beta_r", C.c_double), ("beta_b", C.c_double), ("r_min", C.c_double),
                ("d_merge", C.c_double), ("sigma_b", C.c_double), ("b_min", C.c_double),
                ("sbr_guess", C.c_double), ("r_init", C.c_int), ("n_min", C.c_int),
                ("kappa", C.c_double), ("w_nms", C.c_int), ("m_min", C.c_int),
                ("use_apss", C.c_int), ("persp", C.c_double), ("ilp_box", C.c_int)]


@dataclass
class Params:
    """Algorithm parameters (defaults as read from the paper; see the header)."""
    n_iter: int = 20
    k_max: int = 4
    k_init: int = 3
    p_xy: float = 1.0
    dz: float = 0.1
    h_apss: float = 2.0
    h_int: float = 2.0
    beta_t: float = 0.5
    dmax: float = 0.0
    beta_r: float = 1.0
    beta_b: float = 1.0
    r_min: float = 1.0
    d_merge: float = 0.0
    sigma_b: float = 2.0
    b_min: float = 1e-8
    sbr_guess: float = 1.0
    r_init: int = 0
    n_min: int = 2
    kappa: float = 3.0
    w_nms: int = 0
    m_min: int = 3
    use_apss: int = 1
    persp: float = 0.0
    ilp_box: int = 0

    def c(self) -> _Params:
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)})


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_P = C.POINTER(_Params)
_I64 = C.c_int64


def _declare(L):
    L.or_model_new.restype = C.c_void_p
    L.or_model_new.argtypes = [_dp, C.c_int, C.c_int, C.c_int]
    L.or_model_free.argtypes = [C.c_void_p]
    L.or_model_set_classes.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    L.or_model_origin.restype = C.c_int
    L.or_model_origin.argtypes = [C.c_void_p]
    L.or_model_sigma2.restype = C.c_double
    L.or_model_sigma2.argtypes = [C.c_void_p]
    L.or_model_fisher.restype = C.c_double
    L.or_model_fisher.argtypes = [C.c_void_p]
    L.or_model_window.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.or_h.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
    L.or_S.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
    L.or_lmf_table.argtypes = [C.c_void_p, C.c_double, _i64p]
    L.or_compact.restype = _I64
    L.or_compact.argtypes = [_u16p, _I64, C.c_int, _u32p, _u32p]
    L.or_nll.restype = C.c_double
    L.or_nll.argtypes = [C.c_void_p, _I64, _u32p, _u32p, C.c_int, _dp, _dp, _ip, _dp, _dp]
    L.or_nll_dense.restype = C.c_double
    L.or_nll_dense.argtypes = [C.c_void_p, _I64, _u16p, C.c_int, _dp, _dp, _ip, _dp, _dp]
    L.or_grad.argtypes = [C.c_void_p, _I64, _u32p, _u32p, C.c_int, _dp, _dp, _ip, _dp, _dp,
                          _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_init.argtypes = [C.c_void_p, _P, C.c_int, C.c_int, C.c_int, _u32p, _u32p, _dp,
                          _dp, _dp, _dp, _ip, _dp]
    L.or_init_normals.argtypes = [_P, C.c_int, C.c_int, C.c_int, _dp, _ip, _dp]
    L.or_depth_step.argtypes = [C.c_void_p, _P, _I64, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_apss.argtypes = [_P, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _ip]
    L.or_apss_neighbours.argtypes = [_P, C.c_int, C.c_int, C.c_int, _dp, _ip, _I64, C.c_int,
                                     _i64p, C.c_int]
    L.or_merge.argtypes = [C.c_void_p, _P, _I64, _dp, _dp, _dp, _ip]
    L.or_intensity_step.argtypes = [C.c_void_p, _P, _I64, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_intensity_filter.argtypes = [_P, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _ip]
    L.or_bg_step.argtypes = [C.c_void_p, _P, _I64, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_bg_filter.argtypes = [_P, C.c_int, C.c_int, C.c_int, _dp]
    for name in ("or_iterate", "or_reconstruct"):
        getattr(L, name).argtypes = [C.c_void_p, _P, C.c_int, C.c_int, C.c_int, _u32p, _u32p,
                                     _dp, _dp, _dp, _dp, _ip, _dp]
    _i = C.c_int
    L.or_sr_nll.restype = C.c_double
    L.or_sr_nll.argtypes = [C.c_void_p, _i, _i, _i, _i, _u32p, _u32p, _i, _dp, _dp, _ip, _dp, _dp]
    L.or_sr_grad.argtypes = [C.c_void_p, _i, _i, _i, _i, _u32p, _u32p, _i, _dp, _dp, _ip, _dp, _dp,
                             _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_sr_depth_step.argtypes = [C.c_void_p, _P, _i, _i, _i, _i, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_sr_intensity_step.argtypes = [C.c_void_p, _P, _i, _i, _i, _i, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_sr_bg_step.argtypes = [C.c_void_p, _P, _i, _i, _i, _i, _u32p, _u32p, _dp, _dp, _dp, _ip, _dp]
    L.or_sr_expand.argtypes = [_i, _i, _i, _i, _i, _dp, _dp, _ip, _dp, _dp, _dp, _ip]
    for name in ("or_sr_iterate", "or_sr_reconstruct"):
        getattr(L, name).argtypes = [C.c_void_p, _P, _i, _i, _i, _i, _u32p, _u32p,
                                     _dp, _dp, _dp, _dp, _ip, _dp]


class Model:
    """IRF model (normalised samples, Catmull-Rom interpolant, sigma_h^2, Fisher information)."""

    def __init__(self, irf, T: int, origin: int = -1):
        self.irf = np.ascontiguousarray(irf, dtype=np.float64)
        self.T = int(T)
        self.L = len(self.irf)
        self._h = lib().or_model_new(self.irf, self.L, int(origin), self.T)
        if not self._h:
            raise ValueError("invalid IRF")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_model_free(self._h)
            self._h = None

    @property
    def origin(self) -> int:
        return lib().or_model_origin(self._h)

    @property
    def sigma2(self) -> float:
        return lib().or_model_sigma2(self._h)

    @property
    def fisher(self) -> float:
        return lib().or_model_fisher(self._h)

    def window(self):
        wl, wr = C.c_int(), C.c_int()
        lib().or_model_window(self._h, C.byref(wl), C.byref(wr))
        return wl.value, wr.value

    def h(self, tau):
        tau = np.ascontiguousarray(np.atleast_1d(tau), dtype=np.float64)
        h, hp = np.zeros_like(tau), np.zeros_like(tau)
        lib().or_h(self._h, len(tau), tau, h, hp)
        return h, hp

    def S(self, tau):
        tau = np.ascontiguousarray(np.atleast_1d(tau), dtype=np.float64)
        s, sp = np.zeros_like(tau), np.zeros_like(tau)
        lib().or_S(self._h, len(tau), tau, s, sp)
        return s, sp

    def lmf_table(self, sbr_guess: float = 1.0) -> np.ndarray:
        q = np.zeros(self.L, dtype=np.int64)
        lib().or_lmf_table(self._h, float(sbr_guess), q)
        return q


def compact(Z: np.ndarray):
    """Histograms [..., T] uint16 -> (off uint32 [npix+1], ent uint32 [E])."""
    Z = np.ascontiguousarray(Z, dtype=np.uint16)
    T = Z.shape[-1]
    npix = Z.size // T
    nnz = int(np.count_nonzero(Z))
    off = np.zeros(npix + 1, dtype=np.uint32)
    ent = np.zeros(max(nnz, 1), dtype=np.uint32)
    e = lib().or_compact(Z, npix, T, off, ent)
    assert e == nnz
    return off, ent[:e].copy() if e else np.zeros(0, dtype=np.uint32)


def compact_events(pix, bins, npix: int, T: int):
    """Photon events (pixel, bin), any order -> the active-bin lists of their
    histogram: the count of each (pixel, bin) is the number of events that name
    it (the observation model's z), then `compact`.  Counts above 65535 do not
    fit the entry format and raise."""
    key = np.asarray(pix, dtype=np.int64) * T + np.asarray(bins, dtype=np.int64)
    assert key.size == 0 or (key.min() >= 0 and key.max() < npix * T)
    Z = np.bincount(key, minlength=npix * T)
    assert Z.max(initial=0) <= 65535
    return compact(Z.astype(np.uint16).reshape(npix, T))


def _ent(ent):
    ent = np.ascontiguousarray(ent, dtype=np.uint32)
    return ent if ent.size else np.zeros(1, dtype=np.uint32)


class State:
    """Pixel-major point state: t, r [npix, K]; n [npix, K, 3]; cnt, b, g [npix]."""

    def __init__(self, F, rows, cols, K, g=None):
        self.F, self.rows, self.cols, self.K = F, rows, cols, K
        npix = F * rows * cols
        self.t = np.zeros((npix, K))
        self.r = np.zeros((npix, K))
        self.n = np.zeros((npix, K, 3))
        self.n[..., 2] = -1.0
        self.cnt = np.zeros(npix, dtype=np.int32)
        self.b = np.zeros(npix)
        self.g = np.ones(npix) if g is None else np.ascontiguousarray(g, dtype=np.float64).reshape(-1)

    @property
    def npix(self):
        return self.F * self.rows * self.cols

    def copy(self) -> "State":
        s = State(self.F, self.rows, self.cols, self.K, self.g.copy())
        for a in ("t", "r", "n", "cnt", "b"):
            setattr(s, a, getattr(self, a).copy())
        return s


class SRState(State):
    """Super-resolved state (Results, dynamic scenes): the point arrays t, r, n,
    cnt of `State` on the point grid of (rows s) x (cols s) pixels per frame,
    while b and g belong to the rows x cols lidar pixels."""

    def __init__(self, F, rows, cols, s, K, g=None):
        super().__init__(F, rows * s, cols * s, K)
        self.s, self.lrows, self.lcols = s, rows, cols
        nl = F * rows * cols
        self.b = np.zeros(nl)
        self.g = np.ones(nl) if g is None else np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        assert self.g.size == nl

    def copy(self) -> "SRState":
        c = SRState(self.F, self.lrows, self.lcols, self.s, self.K, self.g.copy())
        for a in ("t", "r", "n", "cnt", "b"):
            setattr(c, a, getattr(self, a).copy())
        return c


class Oracle:
    """The oracle's steps bound to one IRF model and parameter set.

    Per-pixel IRFs (the observation model's h_ij): irf_class[p] names pixel
    p's model, 0 = `model`, k >= 1 = irf_models[k - 1] (numbers past the list
    count as 0).  The class table is attached to `model` while this oracle
    lives."""

    def __init__(self, model: Model, params: Params, irf_models=None, irf_class=None):
        self.m, self.p = model, params
        self._pc = params.c()
        self._cls = None
        if irf_class is not None:
            self._models = [model] + list(irf_models or [])
            self._marr = (C.c_void_p * len(self._models))(*[mm._h for mm in self._models])
            self._cls = np.ascontiguousarray(irf_class, dtype=np.uint8).reshape(-1)
            lib().or_model_set_classes(model._h, len(self._models), self._marr,
                                       self._cls.ctypes.data_as(C.c_void_p))

    def __del__(self):
        if getattr(self, "_cls", None) is not None and _lib is not None and getattr(self.m, "_h", None):
            _lib.or_model_set_classes(self.m._h, 0, None, None)

    @property
    def _P(self):
        self._pc = self.p.c()
        return C.byref(self._pc)

    def nll(self, off, ent, s: State) -> float:
        return lib().or_nll(self.m._h, s.npix, off, _ent(ent), s.K, s.t, s.r, s.cnt, s.b, s.g)

    def nll_dense(self, Z, s: State) -> float:
        Z = np.ascontiguousarray(Z, dtype=np.uint16)
        return lib().or_nll_dense(self.m._h, s.npix, Z, s.K, s.t, s.r, s.cnt, s.b, s.g)

    def grad(self, off, ent, s: State):
        gt, gr = np.zeros_like(s.t), np.zeros_like(s.r)
        at, ar = np.zeros_like(s.t), np.zeros_like(s.r)
        gb, ab = np.zeros_like(s.b), np.zeros_like(s.b)
        lib().or_grad(self.m._h, s.npix, off, _ent(ent), s.K, s.t, s.r, s.cnt, s.b, s.g,
                      gt, gr, gb, at, ar, ab)
        return (gt, gr, gb), (at, ar, ab)

    def init(self, off, ent, s: State, normals: bool = True) -> State:
        lib().or_init(self.m._h, self._P, s.F, s.rows, s.cols, off, _ent(ent), s.g,
                      s.t, s.r, s.n, s.cnt, s.b)
        if normals:
            self.init_normals(s)
        return s

    def init_normals(self, s: State) -> State:
        lib().or_init_normals(self._P, s.F, s.rows, s.cols, s.t, s.cnt, s.n)
        return s

    def depth_step(self, off, ent, s: State) -> State:
        lib().or_depth_step(self.m._h, self._P, s.npix, off, _ent(ent), s.g, s.t, s.r, s.cnt, s.b)
        return s

    def apss(self, s: State) -> State:
        lib().or_apss(self._P, s.F, s.rows, s.cols, self.m.T, s.t, s.n, s.cnt)
        return s

    def apss_neighbours(self, s: State, q: int, brute_force: bool = False, cap: int = 4096):
        out = np.zeros(cap, dtype=np.int64)
        lib().or_apss_neighbours(self._P, s.F, s.rows, s.cols, s.t, s.cnt, int(q),
                                 int(brute_force), out, cap)
        return out[1:1 + out[0]].copy()

    def merge(self, s: State) -> State:
        lib().or_merge(self.m._h, self._P, s.npix, s.t, s.r, s.n, s.cnt)
        return s

    def intensity_step(self, off, ent, s: State) -> State:
        lib().or_intensity_step(self.m._h, self._P, s.npix, off, _ent(ent), s.g, s.t, s.r,
                                s.cnt, s.b)
        return s

    def intensity_filter(self, s: State) -> State:
        lib().or_intensity_filter(self._P, s.F, s.rows, s.cols, s.t, s.r, s.n, s.cnt)
        return s

    def bg_step(self, off, ent, s: State) -> State:
        lib().or_bg_step(self.m._h, self._P, s.npix, off, _ent(ent), s.g, s.t, s.r, s.cnt, s.b)
        return s

    def bg_filter(self, s: State) -> State:
        lib().or_bg_filter(self._P, s.F, s.rows, s.cols, s.b)
        return s

    def iterate(self, off, ent, s: State) -> State:
        lib().or_iterate(self.m._h, self._P, s.F, s.rows, s.cols, off, _ent(ent), s.g,
                         s.t, s.r, s.n, s.cnt, s.b)
        return s

    def reconstruct(self, off, ent, s: State) -> State:
        lib().or_reconstruct(self.m._h, self._P, s.F, s.rows, s.cols, off, _ent(ent), s.g,
                             s.t, s.r, s.n, s.cnt, s.b)
        return s

    # -- the learned denoiser in the depth block ----------------------------
    def cnn_denoise(self, s: State, w, fp16: bool = True) -> State:
        """Depth denoiser with the learned network (the loop's depth block with
        another plugged-in denoiser; Results, "Reconstruction algorithm"):
        pixels holding more than the network's three slots take the APSS step
        (their fit reads every point of the pre-denoiser state, as APSS alone
        does); the network then reads the features of the resulting state and
        moves slot k < cnt of every pixel with at most three points by
        sigma_h y_k, kept inside [0, T - 1].  Normals of those pixels stay.
        fp16: the FP16 storage points of the network (features, weights,
        activations, output) as the GPU keeps them."""
        from . import cnn
        sigma_h = float(np.sqrt(self.m.sigma2))
        fitted = self.apss(s.copy())
        four = s.cnt > 3
        s.t[four] = fitted.t[four]
        s.n[four] = fitted.n[four]
        x = cnn.features(s.t, s.r, s.cnt, sigma_h, s.F, s.rows, s.cols)
        y, _ = cnn.forward(x, w, fp16=fp16)
        y = y.reshape(s.npix, 3)
        for k in range(3):
            mv = (s.cnt <= 3) & (s.cnt > k)
            s.t[mv, k] = np.clip(s.t[mv, k] + sigma_h * y[mv, k], 0.0, self.m.T - 1)
        return s

    def iterate_cnn(self, off, ent, s: State, w, fp16: bool = True) -> State:
        """One iteration of the loop with the learned depth denoiser in place of
        APSS: depth step, cnn_denoise, merge, intensity step, intensity
        low-pass and threshold, background step, background filter."""
        self.depth_step(off, ent, s)
        self.cnn_denoise(s, w, fp16)
        self.merge(s)
        self.intensity_step(off, ent, s)
        self.intensity_filter(s)
        self.bg_step(off, ent, s)
        self.bg_filter(s)
        return s

    def reconstruct_cnn(self, off, ent, s: State, w, fp16: bool = True) -> State:
        """Initialisation, then n_iter iterations with the learned depth denoiser."""
        self.init(off, ent, s)
        for _ in range(self.p.n_iter):
            self.iterate_cnn(off, ent, s, w, fp16)
        return s

    # -- super-resolution (s x s point-grid pixels per lidar pixel) ----------
    def _sr(self, s: SRState):
        return (s.s, s.F, s.lrows, s.lcols)

    def sr_nll(self, off, ent, s: SRState) -> float:
        return lib().or_sr_nll(self.m._h, *self._sr(s), off, _ent(ent), s.K, s.t, s.r, s.cnt, s.b, s.g)

    def sr_grad(self, off, ent, s: SRState):
        gt, gr = np.zeros_like(s.t), np.zeros_like(s.r)
        at, ar = np.zeros_like(s.t), np.zeros_like(s.r)
        gb, ab = np.zeros_like(s.b), np.zeros_like(s.b)
        lib().or_sr_grad(self.m._h, *self._sr(s), off, _ent(ent), s.K, s.t, s.r, s.cnt, s.b, s.g,
                         gt, gr, gb, at, ar, ab)
        return (gt, gr, gb), (at, ar, ab)

    def sr_depth_step(self, off, ent, s: SRState) -> SRState:
        lib().or_sr_depth_step(self.m._h, self._P, *self._sr(s), off, _ent(ent), s.g, s.t, s.r, s.cnt, s.b)
        return s

    def sr_intensity_step(self, off, ent, s: SRState) -> SRState:
        lib().or_sr_intensity_step(self.m._h, self._P, *self._sr(s), off, _ent(ent), s.g, s.t, s.r, s.cnt, s.b)
        return s

    def sr_bg_step(self, off, ent, s: SRState) -> SRState:
        lib().or_sr_bg_step(self.m._h, self._P, *self._sr(s), off, _ent(ent), s.g, s.t, s.r, s.cnt, s.b)
        return s

    def sr_expand(self, coarse: State, s: SRState) -> SRState:
        """The lidar-grid initialisation `coarse` spread over the point grid (normals facing the sensor)."""
        lib().or_sr_expand(s.K, *self._sr(s), coarse.t, coarse.r, coarse.cnt, s.t, s.r, s.n, s.cnt)
        s.b[:] = coarse.b
        return s

    def sr_iterate(self, off, ent, s: SRState) -> SRState:
        lib().or_sr_iterate(self.m._h, self._P, *self._sr(s), off, _ent(ent), s.g, s.t, s.r, s.n, s.cnt, s.b)
        return s

    def sr_reconstruct(self, off, ent, s: SRState) -> SRState:
        lib().or_sr_reconstruct(self.m._h, self._P, *self._sr(s), off, _ent(ent), s.g, s.t, s.r, s.n, s.cnt,
                                s.b)
        return s
