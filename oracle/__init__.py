"""CPU oracle of the Hough track finder -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py`` may
import this package.  The product path (``paper_1311_2769_amd``) never does.

The arithmetic lives in ``hough_oracle.c`` (plain, single-threaded C, built
with gcc at -O2 and -ffp-contract=off so each expression is a sequence of
IEEE binary32 operations).  This module only builds the library and marshals
numpy arrays to it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hough_oracle.c")
LIB = os.path.join(HERE, "libhough_oracle.so")
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfpmath=sse",
          "-fexcess-precision=standard", "-fPIC", "-shared"]

_lock = threading.Lock()
_lib = None


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    cmd = ["gcc", *CFLAGS, *extra, "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    f32p = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.hough_oracle_vote.restype = ctypes.c_int64
    lib.hough_oracle_vote.argtypes = [ctypes.c_int64, f32p, f32p, ctypes.c_int32, f32p,
                                      ctypes.c_int32, f32p, f32p, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int32, i64p]
    lib.hough_oracle_peaks.restype = ctypes.c_int64
    lib.hough_oracle_peaks.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i64p,
                                       ctypes.c_int64, ctypes.c_int64, i64p, i64p]
    i32, f32 = ctypes.c_int32, ctypes.c_float
    lib.hough_oracle_vote_straight.restype = ctypes.c_int64
    lib.hough_oracle_vote_straight.argtypes = [ctypes.c_int64, f32p, f32p, i32, f32p, f32p, i32, f32, f32, i32,
                                               i64p]
    lib.hough_oracle_vertex_vote.restype = ctypes.c_int64
    lib.hough_oracle_vertex_vote.argtypes = [ctypes.c_int64, i64p, i64p, ctypes.c_int64,
                                             i32, f32p, i32, f32p, f32p, i32,
                                             i32, f32p, f32, f32, i32, f32p, f32, f32, i64p]
    lib.hough_oracle_associate.restype = ctypes.c_int64
    lib.hough_oracle_associate.argtypes = [ctypes.c_int64, f32p, f32p, i32, f32p, i32, f32p, f32p, i32, f32, f32,
                                           i32, i32, ctypes.c_int64, i64p, i64p, ctypes.c_int64, ctypes.c_int64,
                                           i64p, i64p]
    lib.hough_oracle_vertex_peaks.restype = ctypes.c_int64
    lib.hough_oracle_vertex_peaks.argtypes = [i32, i32, i64p, ctypes.c_int64, ctypes.c_int64, i64p, i64p]
    return lib


def load_library(path: str):
    return _bind(ctypes.CDLL(path))


def lib():
    """The oracle library, (re)built when missing or older than its source."""
    global _lib
    with _lock:
        if _lib is None:
            if (not os.path.exists(LIB)) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            _lib = load_library(LIB)
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def vote(x, y, grid, *, library=None):
    """Accumulator (int64, shape (n_d0, n_phi, n_kappa)) and the number of votes cast."""
    L = library or lib()
    x, y = _f32(x), _f32(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    acc = np.zeros(grid.cells, dtype=np.int64)
    cos_phi, sin_phi = _f32(grid.cos_phi), _f32(grid.sin_phi)
    d0 = None if grid.d0 is None else _f32(grid.d0)
    n = L.hough_oracle_vote(x.shape[0], _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                            grid.n_d0, None if d0 is None else _ptr(d0, ctypes.c_float),
                            grid.n_phi, _ptr(cos_phi, ctypes.c_float), _ptr(sin_phi, ctypes.c_float),
                            grid.n_kappa, float(grid.kappa_min), float(grid.kappa_scale),
                            int(bool(getattr(grid, "forward", False))), _ptr(acc, ctypes.c_int64))
    if n < 0:
        raise ValueError("oracle rejected the grid")
    return acc.reshape(grid.shape), int(n)


def peaks(acc, threshold, cap=None, *, library=None):
    """Sorted candidates (votes, cells) -- at most ``cap`` of them -- and n_found."""
    L = library or lib()
    acc = np.ascontiguousarray(acc, dtype=np.int64)
    if acc.ndim == 2:
        acc = acc[None]
    n_d0, n_phi, n_kappa = acc.shape
    if cap is None:
        cap = acc.size
    votes = np.zeros(max(cap, 1), dtype=np.int64)
    cells = np.zeros(max(cap, 1), dtype=np.int64)
    n = L.hough_oracle_peaks(n_d0, n_phi, n_kappa, _ptr(acc, ctypes.c_int64), int(threshold),
                             int(cap), _ptr(votes, ctypes.c_int64), _ptr(cells, ctypes.c_int64))
    if n < 0:
        raise ValueError("oracle rejected the peak search arguments")
    m = min(n, cap)
    return votes[:m].copy(), cells[:m].copy(), int(n)


def find(x, y, grid, threshold, cap=None, *, library=None):
    """Vote then peaks: (acc, n_votes, votes, cells, n_found)."""
    acc, n_votes = vote(x, y, grid, library=library)
    v, c, n = peaks(acc, threshold, cap, library=library)
    return acc, n_votes, v, c, n


def vertex_vote(cand_votes, cand_cells, track_threshold, grid, vgrid, *, library=None):
    """Second transform (Section 5): vertex accumulator int64 [n_x, n_y] and the votes cast."""
    L = library or lib()
    cv = np.ascontiguousarray(cand_votes, dtype=np.int64)
    cc = np.ascontiguousarray(cand_cells, dtype=np.int64)
    if cv.shape != cc.shape or cv.ndim != 1:
        raise ValueError("candidate votes and cells must be 1-D arrays of equal length")
    cos_phi, sin_phi = _f32(grid.cos_phi), _f32(grid.sin_phi)
    d0 = None if grid.d0 is None else _f32(grid.d0)
    xc, yc = _f32(vgrid.x_centre), _f32(vgrid.y_centre)
    vacc = np.zeros(vgrid.n_x * vgrid.n_y, dtype=np.int64)
    n = L.hough_oracle_vertex_vote(cv.shape[0], _ptr(cv, ctypes.c_int64), _ptr(cc, ctypes.c_int64),
                                   int(track_threshold), grid.n_d0,
                                   None if d0 is None else _ptr(d0, ctypes.c_float), grid.n_phi,
                                   _ptr(cos_phi, ctypes.c_float), _ptr(sin_phi, ctypes.c_float), grid.n_kappa,
                                   vgrid.n_x, _ptr(xc, ctypes.c_float), float(vgrid.x_min), float(vgrid.x_scale),
                                   vgrid.n_y, _ptr(yc, ctypes.c_float), float(vgrid.y_min), float(vgrid.y_scale),
                                   _ptr(vacc, ctypes.c_int64))
    if n < 0:
        raise ValueError("oracle rejected the vertex-vote arguments")
    return vacc.reshape(vgrid.n_x, vgrid.n_y), int(n)


def vertex_peaks(vacc, threshold, cap=None, *, library=None):
    """Sorted vertex candidates (votes, cells) -- at most ``cap`` -- and n_found."""
    L = library or lib()
    vacc = np.ascontiguousarray(vacc, dtype=np.int64)
    n_x, n_y = vacc.shape
    if cap is None:
        cap = vacc.size
    votes = np.zeros(max(cap, 1), dtype=np.int64)
    cells = np.zeros(max(cap, 1), dtype=np.int64)
    n = L.hough_oracle_vertex_peaks(n_x, n_y, _ptr(vacc, ctypes.c_int64), int(threshold), int(cap),
                                    _ptr(votes, ctypes.c_int64), _ptr(cells, ctypes.c_int64))
    if n < 0:
        raise ValueError("oracle rejected the vertex peak arguments")
    m = min(n, cap)
    return votes[:m].copy(), cells[:m].copy(), int(n)


def find_vertices(cand_votes, cand_cells, track_threshold, grid, vgrid, vertex_threshold, cap=None, *,
                  library=None):
    """Second transform then peaks: (vacc, n_votes, votes, cells, n_found)."""
    vacc, n = vertex_vote(cand_votes, cand_cells, track_threshold, grid, vgrid, library=library)
    v, c, nf = vertex_peaks(vacc, vertex_threshold, cap, library=library)
    return vacc, n, v, c, nf


def vote_straight(x, y, grid, *, library=None):
    """Straight-track accumulator (int64, shape (1, n_phi, n_d0)) and the votes cast.
    ``grid`` is a straight grid: its kappa fields describe the d0 axis."""
    L = library or lib()
    x, y = _f32(x), _f32(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    cos_phi, sin_phi = _f32(grid.cos_phi), _f32(grid.sin_phi)
    acc = np.zeros(grid.n_phi * grid.n_kappa, dtype=np.int64)
    n = L.hough_oracle_vote_straight(x.shape[0], _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), grid.n_phi,
                                     _ptr(cos_phi, ctypes.c_float), _ptr(sin_phi, ctypes.c_float), grid.n_kappa,
                                     float(grid.kappa_min), float(grid.kappa_scale),
                                     int(bool(getattr(grid, "forward", False))), _ptr(acc, ctypes.c_int64))
    if n < 0:
        raise ValueError("oracle rejected the straight grid")
    return acc.reshape(1, grid.n_phi, grid.n_kappa), int(n)


def find_straight(x, y, grid, threshold, cap=None, *, library=None):
    """Straight vote then peaks: (acc, n_votes, votes, cells, n_found)."""
    acc, n_votes = vote_straight(x, y, grid, library=library)
    v, c, n = peaks(acc, threshold, cap, library=library)
    return acc, n_votes, v, c, n


def associate(x, y, grid, cand_votes, cand_cells, min_votes, *, library=None):
    """Hit association (reading in hough_oracle.c): int64 arrays (candidate index,
    hit index) of every pair, in candidate order then hit order."""
    L = library or lib()
    x, y = _f32(x), _f32(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    cv = np.ascontiguousarray(cand_votes, dtype=np.int64)
    cc = np.ascontiguousarray(cand_cells, dtype=np.int64)
    cos_phi, sin_phi = _f32(grid.cos_phi), _f32(grid.sin_phi)
    d0 = None if grid.d0 is None else _f32(grid.d0)
    family = 1 if getattr(grid, "family", "curved") == "straight" else 0
    args = (x.shape[0], _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), grid.n_d0,
            None if d0 is None else _ptr(d0, ctypes.c_float), grid.n_phi, _ptr(cos_phi, ctypes.c_float),
            _ptr(sin_phi, ctypes.c_float), grid.n_kappa, float(grid.kappa_min), float(grid.kappa_scale), family,
            int(bool(getattr(grid, "forward", False))), cv.shape[0], _ptr(cv, ctypes.c_int64),
            _ptr(cc, ctypes.c_int64), int(min_votes))
    n = L.hough_oracle_associate(*args, 0, None, None)
    if n < 0:
        raise ValueError("oracle rejected the association arguments")
    out_c = np.zeros(max(n, 1), dtype=np.int64)
    out_h = np.zeros(max(n, 1), dtype=np.int64)
    L.hough_oracle_associate(*args, n, _ptr(out_c, ctypes.c_int64), _ptr(out_h, ctypes.c_int64))
    return out_c[:n].copy(), out_h[:n].copy()
