"""Seeded synthetic inputs for the Hough track finder.

This package is the only code shared by the CPU oracle (``oracle/``) and the
HIP path (``paper_1311_2769_amd/``).  It holds no arithmetic of the Hough
method itself: it places hits on known circles (the detector toy model of the
paper's Section 3, Figure 1 setup) and writes the binned parameter grids (the
shared cos/sin tables of the phi0 bin centres) that both sides take as inputs.
"""

from .grids import (Grid, make_grid, make_straight_grid, GRID_2D_SMALL, GRID_2D, GRID_3D, GRID_STRAIGHT,
                    VertexGrid, make_vertex_grid, VERTEX_GRID)
from .events import (
    Event, Batch, gen_config_event, gen_batch, gen_tracks_event,
    track_hits, LAYERS_CM, BASE_SEED, pack_events, poisson_arrivals,
)
from .configs import CONFIGS, WorkloadConfig
from .truth import match_candidates, efficiency

__all__ = [
    "Grid", "make_grid", "make_straight_grid", "GRID_2D_SMALL", "GRID_2D", "GRID_3D", "GRID_STRAIGHT",
    "VertexGrid", "make_vertex_grid", "VERTEX_GRID",
    "Event", "Batch", "gen_config_event", "gen_batch", "gen_tracks_event",
    "track_hits", "LAYERS_CM", "BASE_SEED", "pack_events", "poisson_arrivals", "CONFIGS", "WorkloadConfig",
    "match_candidates", "efficiency",
]
