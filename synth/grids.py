"""Binned track-parameter grids (the Hough parameter space of Section 3).

A grid is an input to both the oracle and the HIP path: the phi0 bin-centre
cosines and sines, the d0 bin centres and the two fp32 constants that map a
curvature to a fractional kappa bin are computed here once (in fp64, rounded
to fp32) and handed to both sides, so neither evaluates a transcendental.

Bin placement (the paper gives none): bin ``i`` of a range ``[lo, hi)`` with
``n`` bins has centre ``lo + (i + 1/2) * (hi - lo) / n``; phi0 covers
``[0, 2*pi)`` and is periodic; kappa covers ``[-1/R, +1/R)`` in cm^-1 with
``R = 33 cm``; d0 covers ``[d0_lo, d0_hi)`` in cm.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

ACC_I32 = "i32"
ACC_U16 = "u16"


@dataclasses.dataclass(frozen=True)
class Grid:
    n_d0: int
    n_phi: int
    n_kappa: int
    kappa_min: np.float32        # fp32 lower edge of the kappa range
    kappa_scale: np.float32      # fp32 bins per unit of kappa
    cos_phi: np.ndarray          # fp32 [n_phi]
    sin_phi: np.ndarray          # fp32 [n_phi]
    d0: np.ndarray | None        # fp32 [n_d0] bin centres, None for the 2D grid
    acc_type: str                # "i32" or "u16"
    family: str = "curved"       # "straight": (phi0, d0) lines; the kappa fields then describe d0
    forward: bool = False        # forward-hemisphere option: only phi0 with x cos + y sin > 0

    @property
    def is_3d(self) -> bool:
        return self.d0 is not None

    @property
    def cells(self) -> int:
        return self.n_d0 * self.n_phi * self.n_kappa

    @property
    def shape(self) -> tuple:
        return (self.n_d0, self.n_phi, self.n_kappa)

    @property
    def acc_dtype(self):
        return np.int32 if self.acc_type == ACC_I32 else np.uint16

    def phi_centre(self, j) -> np.ndarray:
        """fp64 phi0 of bin centre ``j``."""
        return (np.asarray(j, dtype=np.float64) + 0.5) * (2.0 * math.pi / self.n_phi)

    def kappa_edges64(self) -> np.ndarray:
        """fp64 kappa bin edges implied by the fp32 constants (for tests)."""
        k = np.arange(self.n_kappa + 1, dtype=np.float64)
        return float(self.kappa_min) + k / float(self.kappa_scale)

    def kappa_centre(self, k) -> np.ndarray:
        return float(self.kappa_min) + (np.asarray(k, dtype=np.float64) + 0.5) / float(self.kappa_scale)

    def d0_centre(self, l) -> np.ndarray:
        if self.d0 is None:
            return np.zeros_like(np.asarray(l, dtype=np.float64))
        return self.d0.astype(np.float64)[np.asarray(l)]


def make_grid(n_phi: int, n_kappa: int, *, n_d0: int = 1, d0_range=None,
              kappa_half_range_inv_cm: float = 33.0, acc_type: str = ACC_I32,
              phi_table=None) -> Grid:
    """Build a grid.

    ``kappa_half_range_inv_cm`` is R in ``kappa in [-1/R, +1/R)``.  The bin
    scale ``n_kappa * R / 2`` is exact in fp32 for the configured sizes.
    ``phi_table`` (fp64 angles) replaces the bin centres when a test needs a
    table holding chosen angles; the peak finder still treats it as periodic.
    """
    if n_phi < 1 or n_kappa < 1 or n_d0 < 1:
        raise ValueError("grid dimensions must be positive")
    if phi_table is None:
        phi = (np.arange(n_phi, dtype=np.float64) + 0.5) * (2.0 * math.pi / n_phi)
    else:
        phi = np.asarray(phi_table, dtype=np.float64)
        if phi.shape != (n_phi,):
            raise ValueError("phi_table must have n_phi entries")
    cos_phi = np.cos(phi).astype(np.float32)
    sin_phi = np.sin(phi).astype(np.float32)
    R = float(kappa_half_range_inv_cm)
    kappa_min = np.float32(-1.0 / R)
    kappa_scale = np.float32(n_kappa * R / 2.0)
    if d0_range is None:
        if n_d0 != 1:
            raise ValueError("a 3D grid needs d0_range")
        d0 = None
    else:
        lo, hi = d0_range
        w = (hi - lo) / n_d0
        d0 = (lo + (np.arange(n_d0, dtype=np.float64) + 0.5) * w).astype(np.float32)
    return Grid(n_d0=n_d0, n_phi=n_phi, n_kappa=n_kappa, kappa_min=kappa_min,
                kappa_scale=kappa_scale, cos_phi=cos_phi, sin_phi=sin_phi, d0=d0,
                acc_type=acc_type)


def make_straight_grid(n_phi: int, n_d0: int, d0_range=(-32.0, 32.0), acc_type: str = ACC_I32) -> Grid:
    """Grid of the straight-line (phi0, d0) family: phi0 bin centres as for
    curved tracks, and ``n_d0`` d0 bins over ``d0_range`` held in the kappa
    fields (``kappa_min`` = lower d0 edge, ``kappa_scale`` = bins per cm)."""
    lo, hi = float(d0_range[0]), float(d0_range[1])
    if n_phi < 1 or n_d0 < 1 or not hi > lo:
        raise ValueError("bad straight grid")
    curved = make_grid(n_phi, n_d0, acc_type=acc_type)
    return dataclasses.replace(curved, kappa_min=np.float32(lo), kappa_scale=np.float32(n_d0 / (hi - lo)),
                               family="straight")


# The three grids of the workloads: 256 x 128 int32; 1024 x 512 int32;
# 64 d0 in [-30, 30) cm x 512 phi0 x 256 kappa uint16.
GRID_2D_SMALL = make_grid(256, 128)
GRID_2D = make_grid(1024, 512)
GRID_3D = make_grid(512, 256, n_d0=64, d0_range=(-30.0, 30.0), acc_type=ACC_U16)
# Straight lines: 1024 phi0 x 512 d0 bins of 0.125 cm over [-32, 32) cm, int32.
GRID_STRAIGHT = make_straight_grid(1024, 512)


@dataclasses.dataclass(frozen=True)
class VertexGrid:
    """Binned (x, y) vertex positions of the second transform (Section 5).

    Bin ``i`` of an axis has centre ``lo + (i + 1/2) * (hi - lo) / n``; a
    position p falls in bin ``(int)((p - min) * scale)`` when that is in
    ``[0, n)``.  Centres, ``min`` and ``scale`` are fp32 inputs of both sides.
    """
    n_x: int
    n_y: int
    x_centre: np.ndarray    # fp32 [n_x]
    y_centre: np.ndarray    # fp32 [n_y]
    x_min: np.float32
    x_scale: np.float32
    y_min: np.float32
    y_scale: np.float32

    @property
    def cells(self) -> int:
        return self.n_x * self.n_y


def make_vertex_grid(n_x: int, n_y: int, x_range=(-32.0, 32.0), y_range=(-32.0, 32.0)) -> VertexGrid:
    if n_x < 1 or n_y < 1:
        raise ValueError("a vertex grid needs at least one bin per axis")

    def axis(n, rng):
        lo, hi = float(rng[0]), float(rng[1])
        if not hi > lo:
            raise ValueError("empty vertex range")
        centre = (lo + (np.arange(n, dtype=np.float64) + 0.5) * ((hi - lo) / n)).astype(np.float32)
        return centre, np.float32(lo), np.float32(n / (hi - lo))

    xc, xm, xs = axis(n_x, x_range)
    yc, ym, ys = axis(n_y, y_range)
    return VertexGrid(n_x=n_x, n_y=n_y, x_centre=xc, y_centre=yc, x_min=xm, x_scale=xs, y_min=ym, y_scale=ys)


# 128 x 128 bins of 0.5 cm over [-32, 32)^2 cm: the displaced vertices of the
# displaced-vertex workload lie within 30 cm of the beam line.
VERTEX_GRID = make_vertex_grid(128, 128)
