"""The five workloads: grid, threshold and generator of each.

1: plain 2D, 40 prompt tracks, 256 phi0 x 128 kappa int32, threshold 7.
2: pileup-scale 2D, 5,000 prompt tracks, 1024 x 512 int32, threshold 7.
3: displaced 3D, 64 d0 x 512 phi0 x 256 kappa uint16, 3x3x3, threshold 5.
4: batch of 256 uneven 2D events (200-8,000 tracks), 1024 x 512 int32.
5: served stream, 80 % workload-4 style 2D and 20 % workload-3 style 3D.
6: straight lines (the kappa = 0 family), 2,000 tracks, 1024 phi0 x 512 d0 int32, threshold 7.
"""

from __future__ import annotations

import dataclasses

from .grids import Grid, GRID_2D_SMALL, GRID_2D, GRID_3D, GRID_STRAIGHT


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    id: int
    name: str
    grid: Grid
    threshold: int
    n_events: int
    grid_3d: Grid | None = None       # second grid of the mixed stream
    threshold_3d: int | None = None


CONFIGS = {
    1: WorkloadConfig(1, "plain2d_40trk_256x128", GRID_2D_SMALL, 7, 1),
    2: WorkloadConfig(2, "pileup2d_5000trk_1024x512", GRID_2D, 7, 1),
    3: WorkloadConfig(3, "displaced3d_35khits_64x512x256", GRID_3D, 5, 1),
    4: WorkloadConfig(4, "batch256_uneven2d_1024x512", GRID_2D, 7, 256),
    5: WorkloadConfig(5, "served_mix80x2d_20x3d", GRID_2D, 7, 0, GRID_3D, 5),
    6: WorkloadConfig(6, "straight2d_2000trk_1024x512", GRID_STRAIGHT, 7, 1),
}
