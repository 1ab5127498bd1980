"""Python binding of libhough (argument marshalling only).

Every step of the vote and peak search runs in the HIP kernels of
``libhough.so``; this module loads the library, checks shapes and passes
device pointers.  PyTorch supplies device memory and streams.  There is no
fallback: if the library is missing, importing this module's entry points
raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhough.so")

HOUGH_OK, HOUGH_EINVAL, HOUGH_ENOMEM, HOUGH_EDEVICE = 0, -1, -2, -3
ACC_I32, ACC_U16 = 0, 1

SYMBOLS = (
    "hough_ctx_create", "hough_ctx_destroy", "hough_vote", "hough_peaks", "hough_event_batch",
    "hough_event_batch_packed",
    "hough_vote_batch", "hough_vertices", "hough_associate", "hough_event_noalloc",
    "hough_set_launch", "hough_get_launch", "hough_set_timing", "hough_get_timing", "hough_get_work",
    "hough_autotune", "hough_tune_lookup",
    "hough_server_create", "hough_server_destroy", "hough_server_clock", "hough_server_submit",
    "hough_server_replay", "hough_server_poll", "hough_server_stats",
    "hough_selftest_divide", "hough_selftest_angles", "hough_selftest_near", "hough_diag_rates", "hough_status_str", "hough_last_error", "hough_version",
)


class HoughError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        lib = _lib_or_none()
        msg = lib.hough_status_str(status).decode() if lib else str(status)
        detail = lib.hough_last_error().decode() if lib else ""
        super().__init__(f"{what}: {msg}" + (f" ({detail})" if detail else ""))


class _Grid(ctypes.Structure):
    _fields_ = [("n_d0", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("n_kappa", ctypes.c_int32),
                ("kappa_min", ctypes.c_float), ("kappa_scale", ctypes.c_float),
                ("cos_phi", ctypes.c_void_p), ("sin_phi", ctypes.c_void_p), ("d0", ctypes.c_void_p),
                ("acc_type", ctypes.c_int32), ("family", ctypes.c_int32), ("forward", ctypes.c_int32)]


class _VertexGrid(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32), ("x_min", ctypes.c_float),
                ("x_scale", ctypes.c_float), ("y_min", ctypes.c_float), ("y_scale", ctypes.c_float),
                ("x_centre", ctypes.c_void_p), ("y_centre", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("max_events", ctypes.c_int32), ("max_hits", ctypes.c_int64), ("tune_cache", ctypes.c_char_p)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("n_grids", ctypes.c_int32), ("grids", ctypes.c_void_p), ("thresholds", ctypes.c_void_p),
                ("lanes", ctypes.c_int32), ("batch_events", ctypes.c_void_p), ("batch_hits", ctypes.c_void_p),
                ("event_candidates", ctypes.c_void_p), ("deadline_ms", ctypes.c_double),
                ("queue_limit", ctypes.c_int32), ("keep_candidates", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("batch_timeout_ms", ctypes.c_double)]


class _Served(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("grid", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_hits", ctypes.c_int32), ("n_found", ctypes.c_int32), ("n_stored", ctypes.c_int32),
                ("batch_events", ctypes.c_int32), ("n_votes", ctypes.c_uint64), ("cand_offset", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


_LIB = None


def _lib_or_none():
    return _LIB


def load(path: str = LIB_PATH):
    """Load libhough.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1311_2769_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.hough_ctx_create.restype = i32
    lib.hough_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Grid), ctypes.POINTER(_Opts)]
    lib.hough_ctx_destroy.restype = None
    lib.hough_ctx_destroy.argtypes = [vp]
    lib.hough_vote.restype = i32
    lib.hough_vote.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.hough_peaks.restype = i32
    lib.hough_peaks.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    lib.hough_event_batch.restype = i32
    lib.hough_event_batch.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.hough_event_noalloc.restype = i32
    lib.hough_event_noalloc.argtypes = [ctypes.POINTER(_Grid), vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.hough_event_batch_packed.restype = i32
    lib.hough_event_batch_packed.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.hough_vote_batch.restype = i32
    lib.hough_vote_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.hough_set_launch.restype = i32
    lib.hough_set_launch.argtypes = [vp, i32, i32, i32, i32]
    lib.hough_get_launch.restype = i32
    lib.hough_get_launch.argtypes = [vp, i32] + [ctypes.POINTER(i32)] * 3
    lib.hough_set_timing.restype = i32
    lib.hough_set_timing.argtypes = [vp, i32]
    lib.hough_get_timing.restype = i32
    lib.hough_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    lib.hough_get_work.restype = i32
    lib.hough_get_work.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.hough_autotune.restype = i32
    lib.hough_autotune.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, i32, ctypes.c_char_p, vp,
                                   ctypes.POINTER(ctypes.c_float)]
    lib.hough_tune_lookup.restype = i32
    lib.hough_tune_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_Grid), i32, i64,
                                      ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
    lib.hough_server_create.restype = i32
    lib.hough_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_ServerOpts)]
    lib.hough_server_destroy.restype = None
    lib.hough_server_destroy.argtypes = [vp]
    lib.hough_server_clock.restype = ctypes.c_double
    lib.hough_server_clock.argtypes = [vp]
    lib.hough_server_submit.restype = i32
    lib.hough_server_submit.argtypes = [vp, i64, i32, vp, vp, i32, ctypes.c_double]
    lib.hough_server_replay.restype = i32
    lib.hough_server_replay.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.hough_server_poll.restype = i32
    lib.hough_server_poll.argtypes = [vp, ctypes.POINTER(_Served), i32, vp, i64, ctypes.POINTER(i32), i32]
    lib.hough_server_stats.restype = i32
    lib.hough_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.hough_diag_rates.restype = i32
    lib.hough_diag_rates.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.hough_associate.restype = i32
    lib.hough_associate.argtypes = [vp, vp, vp, i32, vp, vp, i32, i32, vp, i64, vp, vp]
    lib.hough_vertices.restype = i32
    lib.hough_vertices.argtypes = [vp, ctypes.POINTER(_VertexGrid), i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp,
                                   vp]
    lib.hough_selftest_divide.restype = i32
    lib.hough_selftest_divide.argtypes = [i64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_uint64)]
    lib.hough_selftest_angles.restype = i32
    lib.hough_selftest_angles.argtypes = [i64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float)]
    lib.hough_selftest_near.restype = i32
    lib.hough_selftest_near.argtypes = [i64, ctypes.c_uint64, ctypes.c_float, ctypes.c_float, i32, i32,
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(ctypes.c_uint64)]
    lib.hough_status_str.restype = ctypes.c_char_p
    lib.hough_status_str.argtypes = [i32]
    lib.hough_last_error.restype = ctypes.c_char_p
    lib.hough_last_error.argtypes = []
    lib.hough_version.restype = ctypes.c_char_p
    lib.hough_version.argtypes = []
    _LIB = lib
    return lib


def _check(status, what):
    if status != HOUGH_OK:
        raise HoughError(status, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclasses.dataclass
class GridSpec:
    """The binned parameter space, with fp32 bin tables (host arrays)."""
    n_d0: int
    n_phi: int
    n_kappa: int
    kappa_min: float
    kappa_scale: float
    cos_phi: np.ndarray
    sin_phi: np.ndarray
    d0: np.ndarray | None
    acc_u16: bool
    straight: bool = False     # the (phi0, d0) straight-line family; the kappa fields describe d0
    forward: bool = False      # forward-hemisphere option: only phi0 with x cos + y sin > 0

    @classmethod
    def from_grid(cls, g):
        """From any object with the fields of a grid (n_d0, n_phi, ..., acc_type "i32"/"u16",
        optionally family "curved"/"straight" and forward)."""
        return cls(int(g.n_d0), int(g.n_phi), int(g.n_kappa), float(g.kappa_min), float(g.kappa_scale),
                   np.asarray(g.cos_phi, np.float32), np.asarray(g.sin_phi, np.float32),
                   None if g.d0 is None else np.asarray(g.d0, np.float32), g.acc_type == "u16",
                   getattr(g, "family", "curved") == "straight", bool(getattr(g, "forward", False)))

    @property
    def cells(self):
        return self.n_d0 * self.n_phi * self.n_kappa

    @property
    def acc_dtype(self):
        return torch.int16 if self.acc_u16 else torch.int32

    def max_candidates(self):
        """Upper bound on candidates of one event: no two candidates are neighbours."""
        return ((self.n_d0 + 1) // 2 if self.n_d0 > 1 else 1) * (self.n_phi // 2) * ((self.n_kappa + 1) // 2)


class DeviceGrid:
    """A grid's fp32 bin tables on a device and the hough_grid that points at them
    (for the calls that take a grid rather than a context)."""

    def __init__(self, grid, device="cuda"):
        self.spec = grid if isinstance(grid, GridSpec) else GridSpec.from_grid(grid)
        self.device = torch.device(device)
        s = self.spec
        self.cos_phi = torch.from_numpy(s.cos_phi.copy()).to(self.device)
        self.sin_phi = torch.from_numpy(s.sin_phi.copy()).to(self.device)
        self.d0 = None if s.d0 is None else torch.from_numpy(s.d0.copy()).to(self.device)
        self.struct = _Grid(s.n_d0, s.n_phi, s.n_kappa, s.kappa_min, s.kappa_scale, self.cos_phi.data_ptr(),
                            self.sin_phi.data_ptr(), None if self.d0 is None else self.d0.data_ptr(),
                            ACC_U16 if s.acc_u16 else ACC_I32, 1 if s.straight else 0, 1 if s.forward else 0)


def event_noalloc(dgrid, x, y, threshold, acc, out, n_found, n_votes=None, stream=None):
    """hough_event_noalloc: one event's vote, peaks and sort with the library's fixed
    scratch (no context).  dgrid: a DeviceGrid; acc, out [cap, 2] int32, n_found [1]
    int32 and n_votes [1] int64 (or None) are the caller's device tensors."""
    lib = load()
    n = int(x.numel())
    if y.numel() != n or x.dtype != torch.float32 or y.dtype != torch.float32:
        raise ValueError("x, y must be fp32 tensors of equal length")
    if acc.numel() != dgrid.spec.cells or acc.element_size() != (2 if dgrid.spec.acc_u16 else 4):
        raise ValueError("accumulator has the wrong size or type")
    cap = int(out.shape[0]) if out is not None else 0
    _check(lib.hough_event_noalloc(ctypes.byref(dgrid.struct), _ptr(x), _ptr(y), n, int(threshold), _ptr(acc),
                                   _ptr(out) if cap else None, cap, _ptr(n_found), _ptr(n_votes),
                                   _stream_handle(stream)), "hough_event_noalloc")
    return acc, out, n_found, n_votes


class VertexGridSpec:
    """A binned (x, y) vertex grid (Section 5) with its fp32 centre tables on a device."""

    def __init__(self, vgrid, device="cuda"):
        self.n_x, self.n_y = int(vgrid.n_x), int(vgrid.n_y)
        self.device = torch.device(device)
        self.x_centre = torch.from_numpy(np.asarray(vgrid.x_centre, np.float32).copy()).to(self.device)
        self.y_centre = torch.from_numpy(np.asarray(vgrid.y_centre, np.float32).copy()).to(self.device)
        self.struct = _VertexGrid(self.n_x, self.n_y, float(vgrid.x_min), float(vgrid.x_scale),
                                  float(vgrid.y_min), float(vgrid.y_scale), self.x_centre.data_ptr(),
                                  self.y_centre.data_ptr())

    @property
    def cells(self):
        return self.n_x * self.n_y

    def max_candidates(self):
        """No two vertex candidates are neighbours."""
        return ((self.n_x + 1) // 2) * ((self.n_y + 1) // 2)


class HoughContext:
    """One grid on one device: owns the library context and the device bin tables."""

    def __init__(self, grid, *, device="cuda", max_events: int = 1, max_hits: int = 1 << 20,
                 tune_cache: str | None = None):
        self.lib = load()
        self.spec = grid if isinstance(grid, GridSpec) else GridSpec.from_grid(grid)
        self.device = torch.device(device)
        s = self.spec
        self.cos_phi = torch.from_numpy(s.cos_phi.copy()).to(self.device)
        self.sin_phi = torch.from_numpy(s.sin_phi.copy()).to(self.device)
        self.d0 = None if s.d0 is None else torch.from_numpy(s.d0.copy()).to(self.device)
        g = _Grid(s.n_d0, s.n_phi, s.n_kappa, s.kappa_min, s.kappa_scale, self.cos_phi.data_ptr(),
                  self.sin_phi.data_ptr(), None if self.d0 is None else self.d0.data_ptr(),
                  ACC_U16 if s.acc_u16 else ACC_I32, 1 if s.straight else 0, 1 if s.forward else 0)
        opts = _Opts(int(max_events), int(max_hits), tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.hough_ctx_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(opts)),
                   "hough_ctx_create")
        self.handle = h
        self.max_events = int(max_events)
        self.max_hits = int(max_hits)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.hough_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- allocation helpers ------------------------------------------------------------
    def new_acc(self, n_events=None):
        shape = (self.spec.n_d0, self.spec.n_phi, self.spec.n_kappa)
        if n_events is not None:
            shape = (n_events,) + shape
        return torch.empty(shape, dtype=self.spec.acc_dtype, device=self.device)

    # -- entry points -------------------------------------------------------------------
    def vote(self, x, y, acc=None, n_votes=None, stream=None):
        n = int(x.numel())
        if y.numel() != n or x.dtype != torch.float32 or y.dtype != torch.float32:
            raise ValueError("x, y must be fp32 tensors of equal length")
        if not (x.is_contiguous() and y.is_contiguous()):
            raise ValueError("x, y must be contiguous")
        if acc is None:
            acc = self.new_acc()
        if acc.numel() != self.spec.cells or acc.element_size() != (2 if self.spec.acc_u16 else 4):
            raise ValueError("accumulator has the wrong size or type")
        if n_votes is None:
            n_votes = torch.empty(1, dtype=torch.int64, device=self.device)
        _check(self.lib.hough_vote(self.handle, _ptr(x), _ptr(y), n, _ptr(acc), _ptr(n_votes),
                                   _stream_handle(stream)), "hough_vote")
        return acc, n_votes

    def peaks(self, acc, threshold, cap=None, out=None, n_found=None, stream=None):
        if cap is None:
            cap = self.spec.max_candidates() if out is None else out.shape[0]
        if out is None:
            out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
        if n_found is None:
            n_found = torch.empty(1, dtype=torch.int32, device=self.device)
        if acc.numel() != self.spec.cells:
            raise ValueError("accumulator has the wrong size")
        _check(self.lib.hough_peaks(self.handle, _ptr(acc), int(threshold), _ptr(out) if cap else None,
                                    int(cap), _ptr(n_found), _stream_handle(stream)), "hough_peaks")
        return out, n_found

    def vertices(self, vgrid, cands, cand_off, n_found, track_threshold, vertex_threshold, vout=None,
                 vout_off=None, n_vertices=None, vacc=None, want_acc=False, sorted_lists=True, stream=None):
        """Second transform of this context's candidates (hough_vertices).  cand_off and
        vout_off are host or device int64 offsets; sorted_lists: the lists are sorted by
        votes descending, as this context writes them.  Returns (vout, vout_off, n_vertices, vacc)."""
        if not isinstance(vgrid, VertexGridSpec):
            vgrid = VertexGridSpec(vgrid, self.device)
        off = torch.as_tensor(np.asarray(cand_off, np.int64) if not torch.is_tensor(cand_off) else cand_off,
                              dtype=torch.int64).to(self.device)
        n_events = off.numel() - 1
        if vout_off is None:
            vout_off = np.arange(n_events + 1, dtype=np.int64) * vgrid.max_candidates()
        voff = torch.as_tensor(np.asarray(vout_off, np.int64) if not torch.is_tensor(vout_off) else vout_off,
                               dtype=torch.int64).to(self.device)
        if vout is None:
            vout = torch.empty((max(int(voff[-1].item()), 1), 2), dtype=torch.int32, device=self.device)
        if n_vertices is None:
            n_vertices = torch.empty(n_events, dtype=torch.int32, device=self.device)
        if vacc is None and want_acc:
            vacc = torch.empty((n_events, vgrid.n_x, vgrid.n_y), dtype=torch.int32, device=self.device)
        _check(self.lib.hough_vertices(self.handle, ctypes.byref(vgrid.struct), n_events, _ptr(cands), _ptr(off),
                                       _ptr(n_found), 1 if sorted_lists else 0, int(track_threshold),
                                       int(vertex_threshold), _ptr(vout), _ptr(voff), _ptr(n_vertices), _ptr(vacc),
                                       _stream_handle(stream)),
               "hough_vertices")
        return vout, voff, n_vertices, vacc

    def associate(self, x, y, cands, n_cands, min_votes, cap=None, pairs=None, n_pairs=None, stream=None):
        """Hit association of one event (hough_associate): the (candidate index, hit
        index) pairs of candidates with at least min_votes votes.  cands [n, 2] int32
        and n_cands [1] int32 on the device (hough_peaks' outputs).  Returns
        (pairs [cap, 2] int32, n_pairs [1] int64); pairs are unordered.  cap (or
        pairs) must be given: n_pairs reports the full count when it is too small."""
        if cap is None:
            if pairs is None:
                raise ValueError("associate needs cap or a pairs buffer")
            cap = pairs.shape[0]
        if pairs is None:
            pairs = torch.empty((max(int(cap), 1), 2), dtype=torch.int32, device=self.device)
        if n_pairs is None:
            n_pairs = torch.empty(1, dtype=torch.int64, device=self.device)
        _check(self.lib.hough_associate(self.handle, _ptr(x), _ptr(y), int(x.numel()), _ptr(cands), _ptr(n_cands),
                                        int(cands.shape[0]), int(min_votes), _ptr(pairs), int(cap), _ptr(n_pairs),
                                        _stream_handle(stream)), "hough_associate")
        return pairs, n_pairs

    def event_batch(self, hit_off, x, y, threshold, cand_off=None, cands=None, n_found=None,
                    n_votes=None, acc=None, want_votes=True, stream=None):
        hit_off = np.ascontiguousarray(hit_off, dtype=np.int64)
        n_events = hit_off.shape[0] - 1
        if cand_off is None:
            cap = self.spec.max_candidates()
            cand_off = np.arange(n_events + 1, dtype=np.int64) * cap
        cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
        if cands is None:
            cands = torch.empty((max(int(cand_off[-1]), 1), 2), dtype=torch.int32, device=self.device)
        if n_found is None:
            n_found = torch.empty(n_events, dtype=torch.int32, device=self.device)
        if n_votes is None and want_votes:
            n_votes = torch.empty(n_events, dtype=torch.int64, device=self.device)
        _check(self.lib.hough_event_batch(
            self.handle, n_events, hit_off.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(y), int(threshold),
            _ptr(acc), _ptr(cands), cand_off.ctypes.data_as(ctypes.c_void_p), _ptr(n_found), _ptr(n_votes),
            _stream_handle(stream)), "hough_event_batch")
        return cands, cand_off, n_found, n_votes

    def event_batch_packed(self, hit_off, x, y, threshold, cand_off=None, cands=None, cand_start=None,
                           n_found=None, n_votes=None, acc=None, want_votes=True, stream=None):
        """hough_event_batch_packed: as event_batch, with event e's stored list at
        cands[cand_start[e]] and the lists back to back.  Returns (cands, cand_start,
        n_found, n_votes); cand_start[-1] is the total stored."""
        hit_off = np.ascontiguousarray(hit_off, dtype=np.int64)
        n_events = hit_off.shape[0] - 1
        if cand_off is None:
            cand_off = np.arange(n_events + 1, dtype=np.int64) * self.spec.max_candidates()
        cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
        if cands is None:
            cands = torch.empty((max(int(cand_off[-1]), 1), 2), dtype=torch.int32, device=self.device)
        if cand_start is None:
            cand_start = torch.empty(n_events + 1, dtype=torch.int64, device=self.device)
        if n_found is None:
            n_found = torch.empty(n_events, dtype=torch.int32, device=self.device)
        if n_votes is None and want_votes:
            n_votes = torch.empty(n_events, dtype=torch.int64, device=self.device)
        _check(self.lib.hough_event_batch_packed(
            self.handle, n_events, hit_off.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(y), int(threshold),
            _ptr(acc), _ptr(cands), cand_off.ctypes.data_as(ctypes.c_void_p), _ptr(cand_start), _ptr(n_found),
            _ptr(n_votes), _stream_handle(stream)), "hough_event_batch_packed")
        return cands, cand_start, n_found, n_votes

    def vote_batch(self, hit_off, x, y, acc=None, n_votes=None, stream=None):
        hit_off = np.ascontiguousarray(hit_off, dtype=np.int64)
        n_events = hit_off.shape[0] - 1
        if acc is None:
            acc = self.new_acc(n_events)
        if acc.numel() != n_events * self.spec.cells:
            raise ValueError("accumulator has the wrong size")
        if n_votes is None:
            n_votes = torch.empty(n_events, dtype=torch.int64, device=self.device)
        _check(self.lib.hough_vote_batch(self.handle, n_events, hit_off.ctypes.data_as(ctypes.c_void_p),
                                         _ptr(x), _ptr(y), _ptr(acc), _ptr(n_votes), _stream_handle(stream)),
               "hough_vote_batch")
        return acc, n_votes

    def set_launch(self, which, rows, threads, split=1):
        _check(self.lib.hough_set_launch(self.handle, which, rows, threads, split), "hough_set_launch")

    def autotune(self, which, hit_off, x, y, threshold=1, *, acc=None, cand_off=None, cands=None,
                 n_found=None, reps=5, cache=None, stream=None):
        """Time the launch shapes of `which` (0 single-event vote of event 0,
        1 whole batch) on these resident hits, keep the fastest on this
        context and, with a cache path (or $HOUGH_TUNE_CACHE), record it.
        Returns (rows, threads, split, best_ms)."""
        hit_off = np.ascontiguousarray(hit_off, dtype=np.int64)
        n_events = hit_off.shape[0] - 1
        if which == 0 and acc is None:
            acc = self.new_acc()
        if which == 1:
            if cand_off is None:
                cand_off = np.arange(n_events + 1, dtype=np.int64) * self.spec.max_candidates()
            cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
            if cands is None:
                cands = torch.empty((max(int(cand_off[-1]), 1), 2), dtype=torch.int32, device=self.device)
            if n_found is None:
                n_found = torch.empty(n_events, dtype=torch.int32, device=self.device)
        best = ctypes.c_float()
        _check(self.lib.hough_autotune(
            self.handle, int(which), n_events, hit_off.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(y),
            int(threshold), _ptr(acc), _ptr(cands),
            None if cand_off is None else cand_off.ctypes.data_as(ctypes.c_void_p), _ptr(n_found), int(reps),
            cache.encode() if cache else None, _stream_handle(stream), ctypes.byref(best)), "hough_autotune")
        return self.get_launch(which) + (best.value,)

    def set_timing(self, enable):
        """0/False: graphs; 1/True: timed direct launches; 2: timed and counting
        the vote's evaluated pairs (get_work)."""
        mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        _check(self.lib.hough_set_timing(self.handle, mode), "hough_set_timing")

    def get_timing(self):
        """(vote_ms, total_ms) of the last timed batch (waits for it)."""
        v, t = ctypes.c_float(), ctypes.c_float()
        _check(self.lib.hough_get_timing(self.handle, ctypes.byref(v), ctypes.byref(t)), "hough_get_timing")
        return v.value, t.value

    def get_work(self):
        """(hit, phi0 row) pairs the last timed batch's vote evaluated (waits for it)."""
        v = ctypes.c_uint64()
        _check(self.lib.hough_get_work(self.handle, ctypes.byref(v)), "hough_get_work")
        return int(v.value)

    def get_launch(self, which):
        vals = [ctypes.c_int32() for _ in range(3)]
        _check(self.lib.hough_get_launch(self.handle, which, *[ctypes.byref(v) for v in vals]),
               "hough_get_launch")
        return tuple(v.value for v in vals)


def selftest_divide(n: int, seed: int = 1):
    """(mismatches, checked) of the device division self-test."""
    lib = load()
    bad, used = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.hough_selftest_divide(int(n), int(seed), ctypes.byref(bad), ctypes.byref(used)),
           "hough_selftest_divide")
    return bad.value, used.value


def selftest_angles(n: int, seed: int = 1):
    """(max |atan2f - atan2|, max |asinf - asin|) in radians over n device draws."""
    lib = load()
    ea, es = ctypes.c_float(), ctypes.c_float()
    _check(lib.hough_selftest_angles(int(n), int(seed), ctypes.byref(ea), ctypes.byref(es)),
           "hough_selftest_angles")
    return ea.value, es.value


def selftest_near(n: int, kappa_min: float, kappa_scale: float, n_kappa: int, form: int = 0, seed: int = 1):
    """(mismatches, redone, checked) of the device check of the approximate bins
    (form 0: 3D one-reciprocal quotient, 1: 2D scaled hit reciprocal)."""
    lib = load()
    bad, redo, used = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.hough_selftest_near(int(n), int(seed), float(kappa_min), float(kappa_scale), int(n_kappa), int(form),
                                   ctypes.byref(bad), ctypes.byref(redo), ctypes.byref(used)),
           "hough_selftest_near")
    return bad.value, redo.value, used.value


def acc_to_numpy(acc, spec: GridSpec):
    """Accumulator tensor to an int64 numpy array (uint16 cells widened without sign)."""
    a = acc.detach().cpu()
    if spec.acc_u16:
        return a.numpy().view(np.uint16).astype(np.int64).reshape(acc.shape)
    return a.numpy().astype(np.int64)


def cands_to_numpy(out, n_found, cap=None):
    n = int(n_found)
    m = n if cap is None else min(n, cap)
    c = out[:m].detach().cpu().numpy()
    return c[:, 0].astype(np.int64), c[:, 1].astype(np.int64), n


def tune_lookup(cache, device, grid, which, hits):
    """Host-only: the (rows, threads, split) a tuning cache records for this
    device tag, grid and hit count, or None."""
    lib = load()
    spec = grid if isinstance(grid, GridSpec) else GridSpec.from_grid(grid)
    g = _Grid(spec.n_d0, spec.n_phi, spec.n_kappa, spec.kappa_min, spec.kappa_scale, None, None, None,
              ACC_U16 if spec.acc_u16 else ACC_I32)
    found, r, t, sp = (ctypes.c_int32() for _ in range(4))
    _check(lib.hough_tune_lookup(cache.encode() if cache else None, device.encode(), ctypes.byref(g), int(which),
                                 int(hits), ctypes.byref(found), ctypes.byref(r), ctypes.byref(t),
                                 ctypes.byref(sp)), "hough_tune_lookup")
    return (r.value, t.value, sp.value) if found.value else None


def diag_rates():
    """(LDS atomic adds/s, plain fp32 VALU ops/s) measured on the current device."""
    lib = load()
    a, v = ctypes.c_double(), ctypes.c_double()
    _check(lib.hough_diag_rates(ctypes.byref(a), ctypes.byref(v)), "hough_diag_rates")
    return a.value, v.value


HOUGH_EBUSY = -4


class Server:
    """The served stream (a trigger-farm node) of libhough: continuous
    batching over per-grid lanes with device-resident pools.  Events are host
    fp32 arrays; results come back through poll()."""

    def __init__(self, grids, thresholds, *, device="cuda", lanes=2, batch_events=None, batch_hits=None,
                 event_candidates=None, deadline_ms=2.0, queue_limit=4096, keep_candidates=True,
                 tune_cache=None, batch_timeout_ms=0.0):
        self.lib = load()
        self.device = torch.device(device)
        self.specs = [g if isinstance(g, GridSpec) else GridSpec.from_grid(g) for g in grids]
        n = len(self.specs)
        self._tables = []
        structs = (_Grid * n)()
        for i, sp in enumerate(self.specs):
            c = torch.from_numpy(sp.cos_phi.copy()).to(self.device)
            sn = torch.from_numpy(sp.sin_phi.copy()).to(self.device)
            d0 = None if sp.d0 is None else torch.from_numpy(sp.d0.copy()).to(self.device)
            self._tables.append((c, sn, d0))
            structs[i] = _Grid(sp.n_d0, sp.n_phi, sp.n_kappa, sp.kappa_min, sp.kappa_scale, c.data_ptr(),
                               sn.data_ptr(), None if d0 is None else d0.data_ptr(),
                               ACC_U16 if sp.acc_u16 else ACC_I32, 1 if sp.straight else 0,
                               1 if sp.forward else 0)
        self._keep = [structs]
        thr = (ctypes.c_int32 * n)(*[int(t) for t in thresholds])

        def arr(vals, ct):
            if vals is None:
                return None
            a = (ct * n)(*[int(v) for v in vals])
            self._keep.append(a)
            return ctypes.cast(a, ctypes.c_void_p)

        opts = _ServerOpts(n, ctypes.cast(structs, ctypes.c_void_p), ctypes.cast(thr, ctypes.c_void_p), int(lanes),
                           arr(batch_events, ctypes.c_int32), arr(batch_hits, ctypes.c_int64),
                           arr(event_candidates, ctypes.c_int64), float(deadline_ms), int(queue_limit),
                           1 if keep_candidates else 0, tune_cache.encode() if tune_cache else None,
                           float(batch_timeout_ms))
        self._keep.append(thr)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.hough_server_create(ctypes.byref(h), ctypes.byref(opts)), "hough_server_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.hough_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self):
        return self.lib.hough_server_clock(self.handle)

    def submit(self, tag, grid, x, y, t_submit=-1.0):
        """Hand over one event (host arrays).  False when the queue is full."""
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        st = self.lib.hough_server_submit(self.handle, int(tag), int(grid), x.ctypes.data_as(ctypes.c_void_p),
                                          y.ctypes.data_as(ctypes.c_void_p), int(x.size), float(t_submit))
        if st == HOUGH_EBUSY:
            return False
        _check(st, "hough_server_submit")
        return True

    def replay(self, arrival_s, pick, pool_grid, pool_hit_off, pool_x, pool_y):
        """Open-loop replay: arrival i is pool event pick[i], submitted at
        arrival_s[i] seconds from now (blocks until every event is submitted;
        poll from another thread meanwhile).  Returns each submit's status."""
        arrival_s = np.ascontiguousarray(arrival_s, np.float64)
        pick = np.ascontiguousarray(pick, np.int32)
        pool_grid = np.ascontiguousarray(pool_grid, np.int32)
        pool_hit_off = np.ascontiguousarray(pool_hit_off, np.int64)
        pool_x = np.ascontiguousarray(pool_x, np.float32)
        pool_y = np.ascontiguousarray(pool_y, np.float32)
        n = arrival_s.size
        status = np.zeros(n, np.int32)
        vp = ctypes.c_void_p
        _check(self.lib.hough_server_replay(self.handle, n, arrival_s.ctypes.data_as(vp), pick.ctypes.data_as(vp),
                                            pool_grid.size, pool_grid.ctypes.data_as(vp),
                                            pool_hit_off.ctypes.data_as(vp), pool_x.ctypes.data_as(vp),
                                            pool_y.ctypes.data_as(vp), status.ctypes.data_as(vp)),
               "hough_server_replay")
        return status

    def poll(self, max_out=4096, cand_cap=1 << 22, wait_ms=0, with_cands=True):
        """Finished events: a list of dicts (tag, grid, status, n_hits,
        n_found, n_votes, batch_events, t_submit, t_launch, t_done and the
        candidates as an int32 [n, 2] array of (votes, cell), unless
        with_cands is false).  After a device failure the failed events come
        back with status HOUGH_EDEVICE."""
        out = (_Served * max_out)()
        buf = np.empty((max(cand_cap, 1), 2), np.int32)
        n = ctypes.c_int32()
        st = self.lib.hough_server_poll(self.handle, out, max_out, buf.ctypes.data_as(ctypes.c_void_p),
                                        int(cand_cap), ctypes.byref(n), int(wait_ms))
        res = []
        for k in range(n.value):
            r = out[k]
            res.append({"tag": r.tag, "grid": r.grid, "status": r.status, "n_hits": r.n_hits,
                        "n_found": r.n_found, "n_votes": r.n_votes, "batch_events": r.batch_events,
                        "t_submit": r.t_submit, "t_launch": r.t_launch, "t_done": r.t_done,
                        "n_stored": r.n_stored,
                        "cands": buf[r.cand_offset:r.cand_offset + r.n_stored].copy() if with_cands else None})
        if st != HOUGH_EDEVICE:
            _check(st, "hough_server_poll")
        return res

    def stats(self):
        p, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(self.lib.hough_server_stats(self.handle, ctypes.byref(p), ctypes.byref(r), ctypes.byref(b)),
               "hough_server_stats")
        return {"pending": p.value, "refused": r.value, "busy_lanes": b.value}
