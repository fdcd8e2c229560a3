"""ctypes binding of librt3d.so (the C ABI in include/rt3d.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the stream (the current torch
stream).  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt3d.so")
K_MAX = 4
NOALLOC_MAX_PIXELS = 4194304   # RT3D_NOALLOC_MAX_PIXELS

OK, E_INVALID, E_NOMEM, E_DEVICE, E_CAPACITY, E_STATE, E_UNSUPPORTED, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
DENOISE_NONE, DENOISE_APSS = 0, 1
IN_HIST_U16, IN_PHOTON_CSR, IN_PHOTON_EVENTS = 0, 1, 2
STEP_INIT, STEP_DEPTH, STEP_APSS, STEP_MERGE, STEP_INTENSITY, STEP_IFILTER, STEP_BKG, STEP_BFILTER, \
    STEP_ITERATION = range(9)

EXPORTS = ["rt3d_params_default", "rt3d_create", "rt3d_destroy", "rt3d_last_error", "rt3d_sigma2",
           "rt3d_workspace_bytes", "rt3d_set_workspace", "rt3d_reconstruct", "rt3d_query",
           "rt3d_profile", "rt3d_profile_read", "rt3d_graph_create", "rt3d_graph_launch", "rt3d_graph_destroy",
           "rt3d_autotune", "rt3d_mapping", "rt3d_add_irf", "rt3d_debug_irf_class",
           "rt3d_debug_compact", "rt3d_compact_noalloc", "rt3d_debug_compact_events", "rt3d_debug_step", "rt3d_debug_gradients",
           "rt3d_cnn_set_weights", "rt3d_cnn_get_weights", "rt3d_cnn_last_gradient",
           "rt3d_cnn_forward", "rt3d_cnn_train_step", "rt3d_denoiser_save", "rt3d_denoiser_load"]
KERNELS = ["compact", "init", "normals", "depth", "apss", "merge", "intensity", "ifilter", "bkg",
           "bfilter", "output", "cnn", "loop"]
DENOISE_CNN = 2
FLAG_WARM_START = 1
CNN_PARAMS = 24003


class Adam(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class Rt3dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rt3d status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_iter", C.c_int32), ("k_max", C.c_int32),
                ("k_init", C.c_int32), ("p_xy", C.c_double), ("dz", C.c_double),
                ("h_apss", C.c_double), ("h_int", C.c_double), ("beta_t", C.c_double),
                ("dmax", C.c_double), ("beta_r", C.c_double), ("beta_b", C.c_double),
                ("r_min", C.c_double), ("d_merge", C.c_double), ("sigma_b", C.c_double),
                ("b_min", C.c_double), ("sbr_guess", C.c_double), ("r_init", C.c_int32),
                ("n_min", C.c_int32), ("kappa", C.c_double), ("w_nms", C.c_int32),
                ("m_min", C.c_int32), ("denoiser", C.c_int32), ("fused_loop", C.c_int32),
                ("sr", C.c_int32), ("persp", C.c_double), ("ilp_box", C.c_int32),
                ("lanes_per_pixel", C.c_int32)]


class Input(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("kind", C.c_int32), ("frames", C.c_uint32),
                ("rows", C.c_uint32), ("cols", C.c_uint32), ("hist", C.c_void_p),
                ("off", C.c_void_p), ("ent", C.c_void_p), ("gain", C.c_void_p),
                ("ev_pixel", C.c_void_p), ("ev_bin", C.c_void_p), ("ev_scratch", C.c_void_p),
                ("n_events", C.c_uint64), ("frame_rows", C.c_void_p), ("frame_cols", C.c_void_p),
                ("flags", C.c_uint32), ("irf_class", C.c_void_p)]


class Output(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("capacity", C.c_uint32), ("pt_off", C.c_void_p),
                ("depth", C.c_void_p), ("intensity", C.c_void_p), ("normal", C.c_void_p),
                ("background", C.c_void_p), ("world_z", C.c_void_p)]


class State(C.Structure):
    _fields_ = [("frames", C.c_uint32), ("rows", C.c_uint32), ("cols", C.c_uint32),
                ("t", C.c_void_p), ("r", C.c_void_p), ("n", C.c_void_p), ("cnt", C.c_void_p),
                ("b", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("device_error", C.c_int32),
                ("entries", C.c_uint64), ("points", C.c_uint64)]


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(or python paper_1905_06700_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int32
        L.rt3d_params_default.argtypes = [C.POINTER(Params)]
        L.rt3d_create.argtypes = [C.POINTER(C.c_double), C.c_uint32, C.c_int32, C.c_uint32,
                                  C.POINTER(Params), C.POINTER(vp)]
        L.rt3d_create.restype = st
        L.rt3d_destroy.argtypes = [vp]
        L.rt3d_last_error.argtypes = [vp]
        L.rt3d_last_error.restype = C.c_char_p
        L.rt3d_sigma2.argtypes = [vp]
        L.rt3d_sigma2.restype = C.c_double
        L.rt3d_workspace_bytes.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        L.rt3d_workspace_bytes.restype = C.c_size_t
        L.rt3d_set_workspace.argtypes = [vp, vp, C.c_size_t, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_uint64]
        L.rt3d_set_workspace.restype = st
        L.rt3d_reconstruct.argtypes = [vp, C.POINTER(Input), C.POINTER(Output), vp]
        L.rt3d_reconstruct.restype = st
        L.rt3d_query.argtypes = [vp, vp, C.POINTER(Stats)]
        L.rt3d_query.restype = st
        L.rt3d_profile.argtypes = [vp, C.c_int32]
        L.rt3d_profile.restype = st
        L.rt3d_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.rt3d_profile_read.restype = st
        L.rt3d_autotune.argtypes = [vp, C.POINTER(Input), C.POINTER(Output), vp, C.POINTER(C.c_int32)]
        L.rt3d_autotune.restype = st
        L.rt3d_mapping.argtypes = [vp, C.POINTER(Input), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.rt3d_mapping.restype = st
        L.rt3d_graph_create.argtypes = [vp, C.POINTER(Input), C.POINTER(Output), C.POINTER(vp)]
        L.rt3d_graph_create.restype = st
        L.rt3d_graph_launch.argtypes = [vp, vp]
        L.rt3d_graph_launch.restype = st
        L.rt3d_graph_destroy.argtypes = [vp]
        L.rt3d_graph_destroy.restype = None
        L.rt3d_debug_compact.argtypes = [vp, vp, C.c_uint32, vp, vp, C.c_uint64, vp]
        L.rt3d_debug_compact.restype = st
        L.rt3d_compact_noalloc.argtypes = [vp, vp, C.c_uint32, vp, vp, C.c_uint64, vp, vp]
        L.rt3d_compact_noalloc.restype = st
        L.rt3d_debug_compact_events.argtypes = [vp, vp, vp, C.c_uint64, C.c_uint32, vp, vp, vp, C.c_uint64, vp]
        L.rt3d_debug_compact_events.restype = st
        L.rt3d_debug_step.argtypes = [vp, C.c_int32, vp, vp, vp, C.POINTER(State), C.POINTER(State), vp]
        L.rt3d_debug_step.restype = st
        L.rt3d_debug_gradients.argtypes = [vp, vp, vp, vp, C.POINTER(State), vp, vp, vp, vp]
        L.rt3d_debug_gradients.restype = st
        L.rt3d_add_irf.argtypes = [vp, C.POINTER(C.c_double), C.c_uint32, C.c_int32, C.POINTER(C.c_int32)]
        L.rt3d_add_irf.restype = st
        L.rt3d_debug_irf_class.argtypes = [vp, vp]
        L.rt3d_debug_irf_class.restype = st
        fp = C.POINTER(C.c_float)
        for name in ("rt3d_cnn_set_weights", "rt3d_cnn_get_weights", "rt3d_cnn_last_gradient"):
            getattr(L, name).argtypes = [vp, fp, C.c_size_t]
            getattr(L, name).restype = st
        L.rt3d_cnn_forward.argtypes = [vp, C.POINTER(State), vp, vp]
        L.rt3d_cnn_forward.restype = st
        L.rt3d_cnn_train_step.argtypes = [vp, C.POINTER(State), vp, C.c_uint32, C.POINTER(Adam), vp, vp]
        L.rt3d_cnn_train_step.restype = st
        for f in (L.rt3d_denoiser_save, L.rt3d_denoiser_load):
            f.argtypes = [vp, C.c_char_p]
            f.restype = st
        _lib = L
    return _lib


def default_params(**kw) -> Params:
    p = Params()
    lib().rt3d_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k) or k == "struct_size":
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class DeviceState:
    """Slot-major point state on the device (see rt3d_state)."""
    frames: int
    rows: int
    cols: int
    t: torch.Tensor      # float64 [K_MAX, P]
    r: torch.Tensor      # float32 [K_MAX, P]
    n: torch.Tensor      # float32 [3, K_MAX, P]
    cnt: torch.Tensor    # uint8 [P]
    b: torch.Tensor      # float32 [P]

    @classmethod
    def empty(cls, frames, rows, cols, device="cuda"):
        P = frames * rows * cols
        return cls(frames, rows, cols,
                   torch.zeros(K_MAX, P, dtype=torch.float64, device=device),
                   torch.zeros(K_MAX, P, dtype=torch.float32, device=device),
                   torch.zeros(3, K_MAX, P, dtype=torch.float32, device=device),
                   torch.zeros(P, dtype=torch.uint8, device=device),
                   torch.zeros(P, dtype=torch.float32, device=device))

    def c(self) -> State:
        for x in (self.t, self.r, self.n, self.cnt, self.b):
            assert x.is_cuda and x.is_contiguous()
        return State(self.frames, self.rows, self.cols, self.t.data_ptr(), self.r.data_ptr(),
                     self.n.data_ptr(), self.cnt.data_ptr(), self.b.data_ptr())


@dataclass
class Result:
    pt_off: torch.Tensor     # uint32-valued int64 view [P+1] (stored as int32 on device)
    depth: torch.Tensor      # float64 [capacity]
    intensity: torch.Tensor  # float32 [capacity]
    normal: torch.Tensor     # float32 [capacity, 3]
    background: torch.Tensor  # float32 [P]
    world_z: torch.Tensor | None = None  # float64 [capacity] or None


class Graph:
    """A recorded reconstruction (keeps its buffers alive); launch() replays it
    on the current torch stream."""

    def __init__(self, ctx, handle, keep):
        self._ctx, self._h, self._keep = ctx, handle, keep

    def launch(self):
        self._ctx._check(lib().rt3d_graph_launch(self._h, _stream()))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.rt3d_graph_destroy(self._h)
            self._h = None


class Context:
    """One rt3d context: an IRF, a bin count and parameters."""

    def __init__(self, irf, bins: int, origin: int = -1, **params):
        self.params = default_params(**params)
        irf = [float(x) for x in irf]
        arr = (C.c_double * len(irf))(*irf)
        h = C.c_void_p()
        s = lib().rt3d_create(arr, len(irf), int(origin), int(bins), C.byref(self.params), C.byref(h))
        if s != OK:
            raise Rt3dError(s, "rt3d_create failed")
        self._h = h
        self.bins = int(bins)
        self._ws = None
        self._ws_shape = None
        self._debug_cls = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.rt3d_destroy(h)
            self._h = None

    def _check(self, s):
        if s != OK:
            raise Rt3dError(s, lib().rt3d_last_error(self._h).decode())

    @property
    def sigma2(self) -> float:
        return lib().rt3d_sigma2(self._h)

    def workspace(self, frames: int, rows: int, cols: int, max_entries: int):
        """Allocate (torch) and bind a workspace for up to this batch shape."""
        shape = (frames, rows, cols, max_entries)
        if self._ws_shape == shape:
            return
        nb = lib().rt3d_workspace_bytes(self._h, frames, rows, cols, max_entries)
        self._ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(lib().rt3d_set_workspace(self._h, C.c_void_p(aligned), nb, frames, rows, cols,
                                             max_entries))
        self._ws_shape = shape

    def profile(self, kernel: str | None):
        """Time every later launch of one kernel group with HIP events (None = off)."""
        kid = -1 if kernel is None else KERNELS.index(kernel)
        self._check(lib().rt3d_profile(self._h, kid))

    def profile_read(self):
        """(total milliseconds, launches) of the timed kernel since the last read."""
        ms, n = C.c_double(), C.c_uint64()
        self._check(lib().rt3d_profile_read(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def query(self) -> Stats:
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        self._check(lib().rt3d_query(self._h, _stream(), C.byref(st)))
        return st

    # -- whole reconstruction ------------------------------------------------
    def make_output(self, P: int, capacity: int | None = None, normals: bool = True,
                    n_bg: int | None = None, world_z: bool = False) -> Result:
        """Output buffers for P (point-grid) pixels and n_bg (lidar) background values (default P)."""
        cap = P * K_MAX if capacity is None else capacity
        dev = "cuda"
        return Result(torch.zeros(P + 1, dtype=torch.int32, device=dev),
                      torch.zeros(cap, dtype=torch.float64, device=dev),
                      torch.zeros(cap, dtype=torch.float32, device=dev),
                      torch.zeros(cap, 3, dtype=torch.float32, device=dev) if normals else None,
                      torch.zeros(P if n_bg is None else n_bg, dtype=torch.float32, device=dev),
                      torch.zeros(cap, dtype=torch.float64, device=dev) if world_z else None)

    def add_irf(self, irf, origin: int = -1) -> int:
        """Add a per-pixel IRF class (rt3d_add_irf); returns its number."""
        irf = [float(x) for x in irf]
        arr = (C.c_double * len(irf))(*irf)
        k = C.c_int32()
        self._check(lib().rt3d_add_irf(self._h, arr, len(irf), int(origin), C.byref(k)))
        return k.value

    def debug_irf_class(self, cls):
        """Per-pixel IRF classes (cuda uint8 [P] or None) of the step-by-step calls."""
        assert cls is None or (cls.is_cuda and cls.dtype == torch.uint8 and cls.is_contiguous())
        self._debug_cls = cls                         # alive while the library uses it
        self._check(lib().rt3d_debug_irf_class(self._h, _ptr(cls)))

    def _io(self, out: Result, frames: int, rows: int, cols: int, hist=None, off=None, ent=None, gain=None,
            events=None, frame_shapes=None, warm_start=False, irf_class=None):
        inp = Input()
        inp.flags = FLAG_WARM_START if warm_start else 0
        inp.struct_size = C.sizeof(Input)
        inp.frames, inp.rows, inp.cols = frames, rows, cols
        if frame_shapes is not None:
            assert len(frame_shapes) == frames
            fr = (C.c_uint32 * frames)(*[int(r) for r, _ in frame_shapes])
            fc = (C.c_uint32 * frames)(*[int(q) for _, q in frame_shapes])
            inp.frame_rows, inp.frame_cols = C.addressof(fr), C.addressof(fc)
            inp._shape_arrays = (fr, fc)           # alive while the call reads them
        if hist is not None:
            assert hist.dtype == torch.uint16 or hist.dtype == torch.int16
            assert hist.is_cuda and hist.is_contiguous()
            inp.kind = IN_HIST_U16
            inp.hist = hist.data_ptr()
        elif events is not None:
            pix, bins, scratch = events
            assert pix.numel() == bins.numel() <= scratch.numel()
            inp.kind = IN_PHOTON_EVENTS
            inp.ev_pixel, inp.ev_bin, inp.ev_scratch = pix.data_ptr(), bins.data_ptr(), scratch.data_ptr()
            inp.n_events = pix.numel()
        else:
            inp.kind = IN_PHOTON_CSR
            inp.off, inp.ent = off.data_ptr(), ent.data_ptr()
        inp.gain = gain.data_ptr() if gain is not None else None
        npix = sum(int(r) * int(q) for r, q in frame_shapes) if frame_shapes is not None else frames * rows * cols
        if irf_class is not None:
            assert irf_class.is_cuda and irf_class.dtype == torch.uint8 and irf_class.is_contiguous()
            assert irf_class.numel() >= npix, "irf_class smaller than the batch"
            inp.irf_class = irf_class.data_ptr()
        # the library trusts these sizes: point-grid pixels for pt_off, lidar pixels for background
        sr = self.params.sr
        assert out.pt_off.numel() >= npix * sr * sr + 1 and out.background.numel() >= npix, \
            "output buffers smaller than the batch"
        o = Output()
        o.struct_size = C.sizeof(Output)
        o.capacity = out.depth.numel()
        o.pt_off, o.depth, o.intensity = out.pt_off.data_ptr(), out.depth.data_ptr(), out.intensity.data_ptr()
        o.normal = out.normal.data_ptr() if out.normal is not None else None
        o.background = out.background.data_ptr()
        o.world_z = out.world_z.data_ptr() if out.world_z is not None else None
        return inp, o

    def reconstruct_into(self, out: Result, frames: int, rows: int, cols: int, hist=None, off=None,
                         ent=None, gain=None, events=None, frame_shapes=None, warm_start=False, irf_class=None):
        """Enqueue one reconstruction on the current torch stream (no sync).
        Input: hist, or (off, ent), or events = (pixel int32, bin int16, scratch int32).
        frame_shapes: [(rows, cols)] per frame for frames of different sizes, whose
        pixels follow one another (rows and cols are then ignored).
        warm_start: start from the previous call's final state (same frames).
        irf_class: cuda uint8 [P], each pixel's IRF class (see add_irf)."""
        inp, o = self._io(out, frames, rows, cols, hist, off, ent, gain, events, frame_shapes, warm_start,
                          irf_class)
        self._check(lib().rt3d_reconstruct(self._h, C.byref(inp), C.byref(o), _stream()))
        return out

    def autotune(self, out: Result, frames: int, rows: int, cols: int, hist=None, off=None, ent=None, gain=None,
                 events=None, frame_shapes=None, irf_class=None) -> int:
        """Time both loop mappings on this input (synchronises) and keep the faster
        for this batch shape; returns 1 (all iterations in one launch) or 0 (per step)."""
        inp, o = self._io(out, frames, rows, cols, hist, off, ent, gain, events, frame_shapes, irf_class=irf_class)
        fused = C.c_int32(0)
        self._check(lib().rt3d_autotune(self._h, C.byref(inp), C.byref(o), _stream(), C.byref(fused)))
        return int(fused.value)

    def mapping(self, out: Result, frames: int, rows: int, cols: int, hist=None, frame_shapes=None):
        """(fused, lanes per pixel) that reconstruct_into would use for this input."""
        inp, _ = self._io(out, frames, rows, cols, hist, frame_shapes=frame_shapes)
        fused, lanes = C.c_int32(0), C.c_int32(0)
        self._check(lib().rt3d_mapping(self._h, C.byref(inp), C.byref(fused), C.byref(lanes)))
        return int(fused.value), int(lanes.value)

    def graph(self, out: Result, frames: int, rows: int, cols: int, hist=None, off=None, ent=None, gain=None,
              events=None, frame_shapes=None, irf_class=None) -> "Graph":
        """Record reconstruct_into with these buffers as a replayable graph."""
        inp, o = self._io(out, frames, rows, cols, hist, off, ent, gain, events, frame_shapes, irf_class=irf_class)
        h = C.c_void_p()
        self._check(lib().rt3d_graph_create(self._h, C.byref(inp), C.byref(o), C.byref(h)))
        return Graph(self, h, (out, hist, off, ent, gain, events, irf_class))

    def reconstruct(self, hist, gain=None, max_entries=None, irf_class=None, world_z=False) -> Result:
        """hist: cuda uint16 [frames, rows, cols, bins] (or [rows, cols, bins]);
        world_z: also return each point's world Z coordinate."""
        if hist.dim() == 3:
            hist = hist.unsqueeze(0)
        F, R, Cc, T = hist.shape
        assert T == self.bins
        P = F * R * Cc
        me = int(max_entries) if max_entries is not None else min(P * T, 2 ** 32 - 1)
        self.workspace(F, R, Cc, me)
        sr = self.params.sr
        out = self.make_output(P * sr * sr, n_bg=P, world_z=world_z)
        self.reconstruct_into(out, F, R, Cc, hist=hist, gain=gain, irf_class=irf_class)
        return out

    # -- step-by-step entry points -----------------------------------------
    def compact(self, hist, capacity=None):
        hist = hist.contiguous()
        T = hist.shape[-1]
        P = hist.numel() // T
        cap = int(capacity) if capacity is not None else max(1, P * T)
        off = torch.zeros(P + 1, dtype=torch.int32, device="cuda")
        ent = torch.zeros(cap, dtype=torch.int32, device="cuda")
        if self._ws_shape is None or self._ws_shape[0] * self._ws_shape[1] * self._ws_shape[2] < P:
            self.workspace(1, 1, P, 1)
        self._check(lib().rt3d_debug_compact(self._h, _ptr(hist), P, _ptr(off), _ptr(ent), cap, _stream()))
        return off, ent

    def compact_noalloc(self, hist, off, ent, err=None):
        """rt3d_compact_noalloc into caller buffers (cuda int32 off [P + 1],
        ent [capacity], optional err int32 [1]); no workspace, no allocation."""
        hist = hist.contiguous()
        T = hist.shape[-1]
        P = hist.numel() // T
        assert off.dtype == torch.int32 and off.numel() >= P + 1 and ent.dtype == torch.int32
        self._check(lib().rt3d_compact_noalloc(self._h, _ptr(hist), P, _ptr(off), _ptr(ent), ent.numel(),
                                               _ptr(err) if err is not None else None, _stream()))

    def compact_events(self, pix, bins, npix: int, capacity=None):
        """Photon events (cuda int32 pixel, int16 bin, any order) -> (off, ent)."""
        pix, bins = pix.contiguous(), bins.contiguous()
        assert pix.dtype == torch.int32 and bins.dtype in (torch.int16, torch.uint16)
        n = pix.numel()
        cap = int(capacity) if capacity is not None else max(1, n)
        off = torch.zeros(npix + 1, dtype=torch.int32, device="cuda")
        ent = torch.zeros(cap, dtype=torch.int32, device="cuda")
        scratch = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        if self._ws_shape is None or self._ws_shape[0] * self._ws_shape[1] * self._ws_shape[2] < npix:
            self.workspace(1, 1, npix, 1)
        self._check(lib().rt3d_debug_compact_events(self._h, _ptr(pix), _ptr(bins), n, npix, _ptr(scratch),
                                                    _ptr(off), _ptr(ent), cap, _stream()))
        return off, ent

    def step(self, step: int, st_in: DeviceState | None, off=None, ent=None, gain=None,
             shape=None) -> DeviceState:
        if st_in is not None:
            F, R, Cc = st_in.frames, st_in.rows, st_in.cols
        else:
            F, R, Cc = shape
        out = DeviceState.empty(F, R, Cc)
        cin = st_in.c() if st_in is not None else None
        cout = out.c()
        sr = self.params.sr
        if step in (STEP_BFILTER, STEP_ITERATION, STEP_INIT):
            P = F * R * Cc // (sr * sr)          # the workspace is sized in lidar pixels
            if self._ws_shape is None or self._ws_shape[0] * self._ws_shape[1] * self._ws_shape[2] < P:
                self.workspace(1, 1, P, 1)
        self._check(lib().rt3d_debug_step(self._h, step, _ptr(off), _ptr(ent), _ptr(gain),
                                          C.byref(cin) if cin is not None else None, C.byref(cout),
                                          _stream()))
        return out

    # -- learned denoiser -------------------------------------------------
    def cnn_set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == CNN_PARAMS
        self._check(lib().rt3d_cnn_set_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def _host_vec(self, fn):
        import numpy as np
        out = np.zeros(CNN_PARAMS, dtype=np.float32)
        self._check(fn(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def cnn_get_weights(self):
        return self._host_vec(lib().rt3d_cnn_get_weights)

    def denoiser_save(self, path: str):
        """Checkpoint of the network, its Adam moments and step (rt3d_denoiser_save)."""
        self._check(lib().rt3d_denoiser_save(self._h, os.fsencode(path)))

    def denoiser_load(self, path: str):
        self._check(lib().rt3d_denoiser_load(self._h, os.fsencode(path)))

    def cnn_last_gradient(self):
        return self._host_vec(lib().rt3d_cnn_last_gradient)

    def cnn_forward(self, st: DeviceState) -> torch.Tensor:
        """Network output [3, P] (slot corrections in sigma_h units)."""
        P = st.frames * st.rows * st.cols
        y = torch.zeros(3, P, dtype=torch.float32, device="cuda")
        cs = st.c()
        self._check(lib().rt3d_cnn_forward(self._h, C.byref(cs), _ptr(y), _stream()))
        return y

    def cnn_train_step(self, st: DeviceState, truth: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999,
                       eps=1e-8, loss: torch.Tensor | None = None) -> torch.Tensor:
        """One Adam step on a state and its true depths [S, P] (NaN = absent).
        Returns the device tensor (loss, matched slots), filled asynchronously."""
        if loss is None:
            loss = torch.zeros(2, dtype=torch.float32, device="cuda")
        truth = truth.contiguous()
        opt = Adam(C.sizeof(Adam), lr, beta1, beta2, eps)
        cs = st.c()
        self._check(lib().rt3d_cnn_train_step(self._h, C.byref(cs), _ptr(truth), truth.shape[0],
                                              C.byref(opt), _ptr(loss), _stream()))
        return loss

    def gradients(self, st: DeviceState, off, ent, gain=None):
        P = st.frames * st.rows * st.cols
        gt = torch.zeros(K_MAX, P, dtype=torch.float32, device="cuda")
        gr = torch.zeros(K_MAX, P, dtype=torch.float32, device="cuda")
        gb = torch.zeros(P // self.params.sr ** 2, dtype=torch.float32, device="cuda")
        cs = st.c()
        self._check(lib().rt3d_debug_gradients(self._h, _ptr(off), _ptr(ent), _ptr(gain), C.byref(cs),
                                               _ptr(gt), _ptr(gr), _ptr(gb), _stream()))
        return gt, gr, gb
