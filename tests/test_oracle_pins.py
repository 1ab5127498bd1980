"""Pins of the CPU oracle to facts other than itself (CPU only).

Each test checks the oracle against something fixed by the geometry of the
track model (Section 3), a closed form, a library routine or a hand-derived
fixture -- never against a retyped copy of its own formula.
"""

import dataclasses
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth
from synth.grids import Grid, make_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")

# The library under test.  tests/test_oracle_mutants.py swaps in oracle builds with a
# planted mistake and checks that these pins catch it.
LIBRARY = [None]


def vote(x, y, grid):
    return oracle.vote(x, y, grid, library=LIBRARY[0])


def peaks(acc, threshold, cap=None):
    return oracle.peaks(acc, threshold, cap, library=LIBRARY[0])


def _grid_from_tables(n_phi, n_kappa, kappa_min, kappa_scale, cos_phi, sin_phi, d0=None, acc="i32"):
    return Grid(n_d0=1 if d0 is None else len(d0), n_phi=n_phi, n_kappa=n_kappa,
                kappa_min=np.float32(kappa_min), kappa_scale=np.float32(kappa_scale),
                cos_phi=np.asarray(cos_phi, np.float32), sin_phi=np.asarray(sin_phi, np.float32),
                d0=None if d0 is None else np.asarray(d0, np.float32), acc_type=acc)


# --------------------------------------------------------------------------------------
# Hand-derived exact fixture
# --------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_2d_votes_per_hit(golden):
    g = golden["grid_2d"]
    grid = _grid_from_tables(g["n_phi"], g["n_kappa"], g["kappa_min"], g["kappa_scale"],
                             g["cos_phi"], g["sin_phi"])
    for (x, y), row in zip(golden["hits_2d"], golden["votes_2d"]):
        acc, n = vote([x], [y], grid)
        expect = np.zeros(grid.shape, np.int64)
        for j, k in enumerate(row):
            if k is not None:
                expect[0, j, k] = 1
        np.testing.assert_array_equal(acc, expect, err_msg=f"hit {(x, y)}")
        assert n == sum(k is not None for k in row)


def test_golden_2d_accumulator_and_peaks(golden):
    g = golden["grid_2d"]
    grid = _grid_from_tables(g["n_phi"], g["n_kappa"], g["kappa_min"], g["kappa_scale"],
                             g["cos_phi"], g["sin_phi"])
    hx, hy = np.array(golden["hits_2d"], np.float32).T
    acc, n = vote(hx, hy, grid)
    expect = np.zeros(grid.shape, np.int64)
    for j, k, v in golden["acc_2d_nonzero"]:
        expect[0, j, k] = v
    np.testing.assert_array_equal(acc, expect)
    assert n == golden["n_votes_2d"]
    for key, t in (("T2", 2), ("T1", 1)):
        want = golden["peaks_2d"][key]
        v, c, nf = peaks(acc, t)
        assert nf == want["n_found"]
        assert v.tolist() == want["votes"]
        assert c.tolist() == want["cells"]


def test_golden_3d_votes(golden):
    g = golden["grid_3d"]
    grid = _grid_from_tables(g["n_phi"], g["n_kappa"], g["kappa_min"], g["kappa_scale"],
                             g["cos_phi"], g["sin_phi"], d0=g["d0"], acc="u16")
    total = np.zeros(grid.shape, np.int64)
    for (x, y), table in zip(golden["hits_3d"], golden["votes_3d"]):
        acc, n = vote([x], [y], grid)
        expect = np.zeros(grid.shape, np.int64)
        for l, row in enumerate(table):
            for j, k in enumerate(row):
                if k is not None:
                    expect[l, j, k] = 1
        np.testing.assert_array_equal(acc, expect, err_msg=f"hit {(x, y)}")
        total += expect
    hx, hy = np.array(golden["hits_3d"], np.float32).T
    acc, n = vote(hx, hy, grid)
    np.testing.assert_array_equal(acc, total)
    assert n == golden["n_votes_3d"]


# --------------------------------------------------------------------------------------
# Geometry: hits placed on known circles (circle-circle intersection, no Hough formula)
# --------------------------------------------------------------------------------------

def _edge_distance(kf):
    return np.abs(kf - np.round(kf))


@pytest.mark.parametrize("displaced", [False, True])
def test_known_circles_vote_their_own_kappa_bin(displaced):
    """A track's hits, evaluated at the track's own (d0, phi0), all land in the bin of its kappa."""
    rng = np.random.default_rng(11)
    n_kappa = 4096
    checked = 0
    for _ in range(120):
        phi0 = rng.uniform(0, 2 * math.pi)
        kappa = rng.uniform(-1 / 34, 1 / 34)
        d0 = float(np.float32(rng.uniform(-20, 20))) if displaced else 0.0
        ev = synth.gen_tracks_event([d0], [phi0], [kappa])
        r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
        keep = np.abs(r - abs(d0)) > 1.0           # well-conditioned chords only
        if keep.sum() < 3:
            continue
        tab = phi0 + np.array([0.0, 2 * math.pi / 3, 4 * math.pi / 3])
        grid = make_grid(3, n_kappa, phi_table=tab)
        if displaced:
            grid = Grid(**{**grid.__dict__, "d0": np.array([d0], np.float32), "acc_type": "u16"})
        kf = (kappa - float(grid.kappa_min)) * float(grid.kappa_scale)
        if _edge_distance(kf) < 0.05:
            continue
        acc, n = vote(ev.x[keep], ev.y[keep], grid)
        assert acc[0, 0, int(math.floor(kf))] == keep.sum(), (phi0, kappa, d0)
        checked += 1
    assert checked > 60


def _bin_centre_track(grid, l, j, k):
    phi0 = float(grid.phi_centre(j))
    kappa = float(grid.kappa_centre(k))
    d0 = float(grid.d0[l]) if grid.is_3d else 0.0
    return d0, phi0, kappa


@pytest.mark.parametrize("which", ["small2d", "big2d", "3d"])
def test_bin_centre_tracks_peak_at_their_bin(which):
    """Noise-free tracks at bin centres give #hits votes at the true cell and at the mirror cell
    (d0, phi0, kappa) -> (-d0, phi0 + pi, -kappa), and the candidate list holds them."""
    grid = {"small2d": synth.GRID_2D_SMALL, "big2d": synth.GRID_2D, "3d": synth.GRID_3D}[which]
    rng = np.random.default_rng(5)
    done = 0
    while done < 6:
        l = int(rng.integers(0, grid.n_d0))
        j = int(rng.integers(0, grid.n_phi))
        # |kappa| below 1/60 keeps every layer reachable
        k = int(rng.integers(int(grid.n_kappa * 0.25), int(grid.n_kappa * 0.75)))
        d0, phi0, kappa = _bin_centre_track(grid, l, j, k)
        if grid.is_3d and np.min(np.abs(synth.LAYERS_CM - abs(d0))) < 2.0:
            continue
        ev = synth.gen_tracks_event([d0], [phi0], [kappa])
        if ev.n_hits < 5:
            continue
        acc, n = vote(ev.x, ev.y, grid)
        mirror = (grid.n_d0 - 1 - l, (j + grid.n_phi // 2) % grid.n_phi, grid.n_kappa - 1 - k)
        assert acc[l, j, k] == ev.n_hits
        assert acc[mirror] == ev.n_hits
        assert acc.max() == ev.n_hits
        v, c, nf = peaks(acc, ev.n_hits)
        cells = set(c.tolist())
        for (a, b, cc) in ((l, j, k), mirror):
            cell = (a * grid.n_phi + b) * grid.n_kappa + cc
            if grid.is_3d:
                # a d0 neighbour may tie; the surviving cell is within one bin of the truth
                near = [x for x in cells
                        if abs(x // (grid.n_phi * grid.n_kappa) - a) <= 1
                        and (x // grid.n_kappa) % grid.n_phi == b and x % grid.n_kappa == cc]
                assert near, (which, l, j, k)
            else:
                assert cell in cells, (which, l, j, k)
        done += 1


def test_prompt_closed_form_single_hits():
    """At d0 = 0 the curvature is 2 sin(phi_h - phi0) / r (evaluated with atan2/sin in fp64):
    each single hit votes exactly once in each phi0 row where that value is in range."""
    grid = synth.GRID_2D_SMALL
    rng = np.random.default_rng(3)
    phis = grid.phi_centre(np.arange(grid.n_phi))
    for _ in range(40):
        r = rng.choice(synth.LAYERS_CM)
        ph = rng.uniform(0, 2 * math.pi)
        x, y = np.float32(r * math.cos(ph)), np.float32(r * math.sin(ph))
        acc, n = vote([x], [y], grid)
        rh = math.hypot(float(x), float(y))
        phh = math.atan2(float(y), float(x))
        kap = 2.0 * np.sin(phh - phis) / rh
        kf = (kap - float(grid.kappa_min)) * float(grid.kappa_scale)
        row_sums = acc[0].sum(axis=1)
        assert set(np.unique(row_sums)) <= {0, 1}
        sure = (kf > 1e-3) & (kf < grid.n_kappa - 1e-3) & (_edge_distance(kf) > 1e-3)
        out = (kf < -1e-3) | (kf > grid.n_kappa + 1e-3)
        for j in np.nonzero(sure)[0]:
            assert acc[0, j, int(math.floor(kf[j]))] == 1
        assert np.all(row_sums[out] == 0)
        assert n == row_sums.sum()


# --------------------------------------------------------------------------------------
# Invariants and special cases
# --------------------------------------------------------------------------------------

def test_vote_count_and_row_invariants():
    ev = synth.gen_config_event(1)
    grid = synth.GRID_2D_SMALL
    acc, n = vote(ev.x, ev.y, grid)
    assert acc.sum() == n
    assert np.all(acc[0].sum(axis=1) <= ev.n_hits)
    # one hit at a time: every (hit, row) receives at most one vote, and the
    # per-hit vote counts add up to the event's
    total = 0
    for i in range(0, ev.n_hits, 7):
        a1, n1 = vote(ev.x[i:i + 1], ev.y[i:i + 1], grid)
        assert np.all(a1[0].sum(axis=1) <= 1)
        total += n1
    assert total > 0


def test_hit_permutation_leaves_accumulator_unchanged():
    ev = synth.gen_config_event(1)
    grid = synth.GRID_2D_SMALL
    a1, n1 = vote(ev.x, ev.y, grid)
    p = np.random.default_rng(0).permutation(ev.n_hits)
    a2, n2 = vote(ev.x[p], ev.y[p], grid)
    np.testing.assert_array_equal(a1, a2)
    assert n1 == n2


def test_3d_slice_at_zero_d0_equals_2d():
    ev = synth.gen_config_event(1)
    g2 = synth.GRID_2D_SMALL
    g3 = Grid(**{**g2.__dict__, "n_d0": 3, "d0": np.array([-0.5, 0.0, 0.5], np.float32)})
    a2, _ = vote(ev.x, ev.y, g2)
    a3, _ = vote(ev.x, ev.y, g3)
    np.testing.assert_array_equal(a3[1], a2[0])
    assert not np.array_equal(a3[0], a2[0])


def test_nonfinite_and_origin_hits_cast_no_votes():
    grid = synth.GRID_2D_SMALL
    bad = np.array([[np.nan, 1.0], [1.0, np.nan], [np.inf, 2.0], [-np.inf, 0.0],
                    [0.0, 0.0], [np.inf, np.inf]], np.float32)
    acc, n = vote(bad[:, 0], bad[:, 1], grid)
    assert n == 0 and acc.sum() == 0
    acc3, n3 = vote(bad[:4, 0], bad[:4, 1], synth.GRID_3D)
    assert n3 == 0


def test_empty_event():
    acc, n = vote(np.zeros(0, np.float32), np.zeros(0, np.float32), synth.GRID_2D_SMALL)
    assert n == 0 and acc.sum() == 0
    v, c, nf = peaks(acc, 1)
    assert nf == 0 and len(v) == 0


# --------------------------------------------------------------------------------------
# Peak rule
# --------------------------------------------------------------------------------------

def _neighbour_max(acc, strict_centre):
    """Max over the 3x3(x3) neighbourhood (phi periodic, other edges ignored) via scipy."""
    a = acc.astype(np.int64)
    fp = np.ones((3, 3, 3), bool)
    if strict_centre:
        fp[1, 1, 1] = False
    big_neg = np.iinfo(np.int64).min // 2
    a = np.pad(a, ((0, 0), (1, 1), (0, 0)), mode="wrap")
    a = np.pad(a, ((1, 1), (0, 0), (1, 1)), mode="constant", constant_values=big_neg)
    m = ndi.maximum_filter(a, footprint=fp, mode="constant", cval=big_neg)
    return m[1:-1, 1:-1, 1:-1]


def _check_peak_bounds(acc, t):
    v, c, nf = peaks(acc, t)
    assert nf == len(c)
    flat = acc.reshape(-1)
    # sorted by (votes desc, cell asc); votes match the array
    assert v.tolist() == flat[c].tolist()
    assert list(zip((-v).tolist(), c.tolist())) == sorted(zip((-v).tolist(), c.tolist()))
    weak = (acc >= _neighbour_max(acc, False)) & (acc >= t)
    strict = (acc > _neighbour_max(acc, True)) & (acc >= t)
    cand = np.zeros(acc.size, bool)
    cand[c] = True
    cand = cand.reshape(acc.shape)
    assert np.all(cand <= weak)
    assert np.all(strict <= cand)
    # no two candidates are neighbours
    n_d0, n_phi, n_kappa = acc.shape
    idx = np.argwhere(cand)
    s = set(map(tuple, idx.tolist()))
    for (l, j, k) in idx.tolist():
        for od in (-1, 0, 1):
            for op in (-1, 0, 1):
                for ok in (-1, 0, 1):
                    if od == op == ok == 0:
                        continue
                    q = (l + od, (j + op) % n_phi, k + ok)
                    assert q not in s
    return v, c, nf


@pytest.mark.parametrize("shape,hi", [((1, 7, 9), 3), ((1, 16, 12), 6), ((4, 6, 5), 2), ((3, 5, 7), 9)])
def test_peaks_bounded_by_scipy_maximum_filter(shape, hi):
    rng = np.random.default_rng(hash(shape) % 2**32)
    for _ in range(20):
        acc = rng.integers(0, hi + 1, size=shape).astype(np.int64)
        _check_peak_bounds(acc, 1)
        _check_peak_bounds(acc, hi // 2 + 1)


def test_peak_special_cases():
    # delta
    acc = np.zeros((1, 8, 8), np.int64)
    acc[0, 3, 5] = 7
    v, c, n = peaks(acc, 7)
    assert n == 1 and c.tolist() == [3 * 8 + 5] and v.tolist() == [7]
    assert peaks(acc, 8)[2] == 0
    # constant field: every cell ties an earlier neighbour
    assert peaks(np.full((1, 5, 6), 9, np.int64), 1)[2] == 0
    assert peaks(np.full((3, 5, 6), 9, np.int64), 1)[2] == 0
    # two-cell plateaus keep the earlier cell (along kappa, phi0, d0)
    acc = np.zeros((1, 8, 8), np.int64)
    acc[0, 2, 3] = acc[0, 2, 4] = 5
    assert peaks(acc, 1)[1].tolist() == [2 * 8 + 3]
    acc = np.zeros((1, 8, 8), np.int64)
    acc[0, 2, 3] = acc[0, 3, 3] = 5
    assert peaks(acc, 1)[1].tolist() == [2 * 8 + 3]
    acc = np.zeros((3, 4, 4), np.int64)
    acc[0, 1, 1] = acc[1, 1, 1] = 5
    assert peaks(acc, 1)[1].tolist() == [0 * 16 + 1 * 4 + 1]
    # the phi0 seam: row n_phi - 1 precedes row 0 through the wrap offset +1
    acc = np.zeros((1, 8, 8), np.int64)
    acc[0, 0, 3] = acc[0, 7, 3] = 5
    assert peaks(acc, 1)[1].tolist() == [7 * 8 + 3]
    # kappa edges are not periodic
    acc = np.zeros((1, 8, 8), np.int64)
    acc[0, 4, 0] = 3
    acc[0, 4, 7] = 4
    assert sorted(peaks(acc, 1)[1].tolist()) == [4 * 8 + 0, 4 * 8 + 7]


def test_peaks_capacity_truncates_a_prefix():
    ev = synth.gen_config_event(1)
    acc, _ = vote(ev.x, ev.y, synth.GRID_2D_SMALL)
    v, c, n = peaks(acc, 3)
    assert n > 20
    v2, c2, n2 = peaks(acc, 3, cap=17)
    assert n2 == n and v2.tolist() == v[:17].tolist() and c2.tolist() == c[:17].tolist()
    v3, c3, n3 = peaks(acc, 3, cap=0)
    assert n3 == n and len(c3) == 0


def test_config1_tracks_found():
    """Physics sanity (not parity): with 256 phi0 bins against 128 kappa bins the phi0 bin
    width smears the small-radius hits over several kappa bins, so only about 60 % of the 40
    tracks of workload 1 leave a candidate within 1.6 phi0 bins and 6 kappa bins of the truth."""
    ev = synth.gen_config_event(1)
    grid = synth.GRID_2D_SMALL
    acc, n = vote(ev.x, ev.y, grid)
    v, c, nf = peaks(acc, 7)
    j = (c // grid.n_kappa) % grid.n_phi
    k = c % grid.n_kappa
    found = 0
    for p0, k0 in zip(ev.phi0, ev.kappa):
        jt = p0 / (2 * math.pi / grid.n_phi) - 0.5
        kt = (k0 - float(grid.kappa_min)) * float(grid.kappa_scale) - 0.5
        dj = (j - jt + grid.n_phi / 2) % grid.n_phi - grid.n_phi / 2
        if np.any((np.abs(dj) <= 1.6) & (np.abs(k - kt) <= 6)):
            found += 1
    assert found >= 20


# --------------------------------------------------------------------------------------
# Second transform: candidates to displaced vertices (Section 5)
# --------------------------------------------------------------------------------------

def vertex_vote(cv, cc, t, grid, vgrid):
    return oracle.vertex_vote(cv, cc, t, grid, vgrid, library=LIBRARY[0])


def vertex_peaks(vacc, threshold, cap=None):
    return oracle.vertex_peaks(vacc, threshold, cap, library=LIBRARY[0])


SMALL_VGRID = synth.make_vertex_grid(24, 20, (-6.0, 6.0), (-5.0, 5.0))


def _line_grid(angles_deg, d0_values, n_kappa=3):
    """A track grid whose phi0 rows are the given angles and whose d0 bins are the given values."""
    a = np.radians(np.asarray(angles_deg, np.float64))
    return _grid_from_tables(len(a), n_kappa, -0.03, 50.0, np.cos(a), np.sin(a), d0=d0_values)


def test_vertex_lines_through_a_cell_centre_meet_there():
    """Lines of several slopes (both voting modes) through one vertex put all
    their votes for it into that vertex's cell, and nowhere else as many."""
    vg = SMALL_VGRID
    a, b = 7, 13
    vx, vy = float(vg.x_centre[a]), float(vg.y_centre[b])
    angles = [5.0, 33.0, 61.0, 97.0, 128.0, 151.0, 178.0, 250.0]
    cs = np.cos(np.radians(angles)).astype(np.float32).astype(np.float64)
    sn = np.sin(np.radians(angles)).astype(np.float32).astype(np.float64)
    # line i: d0 bin i, phi0 row i (d0 = V_y c - V_x s, the sinusoid of V)
    d0 = (vy * cs - vx * sn).astype(np.float32)
    grid = _line_grid(angles, d0)
    n = len(angles)
    cells = np.array([(i * grid.n_phi + i) * grid.n_kappa + (i % grid.n_kappa) for i in range(n)], np.int64)
    vacc, nv = vertex_vote(np.full(n, 9), cells, 9, grid, vg)
    assert vacc[a, b] == n
    others = vacc.copy()
    others[a, b] = 0
    assert others.max() < n
    v, c, nf = vertex_peaks(vacc, n)
    assert nf == 1 and c.tolist() == [a * vg.n_y + b] and v.tolist() == [n]


def test_vertex_votes_once_per_column_or_row():
    """A shallow line votes once in every column, a steep one once in every row,
    when all its crossings of the dominant axis lie inside the grid."""
    vg = SMALL_VGRID
    for ang, steep in ((20.0, False), (160.0, False), (60.0, True), (115.0, True)):
        grid = _line_grid([ang], [0.3])
        vacc, nv = vertex_vote([5], [0], 1, grid, vg)
        if steep:
            assert nv == vg.n_y
            assert (vacc.sum(axis=0) == 1).all()
        else:
            assert nv == vg.n_x
            assert (vacc.sum(axis=1) == 1).all()


def test_vertex_axis_lines_closed_form():
    """phi0 = 0: the line y = d0 fills one row of cells; phi0 = 90 deg: x = -d0 fills one column."""
    vg = SMALL_VGRID
    g = _grid_from_tables(2, 1, -0.03, 50.0, [1.0, 0.0], [0.0, 1.0], d0=[1.2, 2.3])
    vacc, nv = vertex_vote([3], [0 * 2 + 0], 1, g, vg)            # d0 = 1.2, phi0 = 0
    iy = int((1.2 - vg.y_min) * vg.y_scale)
    expect = np.zeros((vg.n_x, vg.n_y), np.int64)
    expect[:, iy] = 1
    np.testing.assert_array_equal(vacc, expect)
    vacc, nv = vertex_vote([3], [1 * 2 + 1], 1, g, vg)            # d0 = 2.3, phi0 = 90 deg
    ix = int((-2.3 - vg.x_min) * vg.x_scale)
    expect = np.zeros((vg.n_x, vg.n_y), np.int64)
    expect[ix, :] = 1
    np.testing.assert_array_equal(vacc, expect)
    # the lower edges are inside, the upper edges outside
    g = _grid_from_tables(2, 1, -0.03, 50.0, [1.0, 0.0], [0.0, 1.0], d0=[-5.0, 5.0])
    vacc, nv = vertex_vote([3], [0], 1, g, vg)                    # y = -5 = y_min: row 0
    assert nv == vg.n_x and (vacc[:, 0] == 1).all()
    vacc, nv = vertex_vote([3], [1 * 2 + 0], 1, g, vg)            # y = 5 = y_max: no row
    assert nv == 0
    g = _grid_from_tables(2, 1, -0.03, 50.0, [0.0, 0.0], [1.0, -1.0], d0=[6.0, 6.0])
    vacc, nv = vertex_vote([3], [0], 1, g, vg)                    # x = -6 = x_min: column 0
    assert nv == vg.n_y and (vacc[0, :] == 1).all()
    vacc, nv = vertex_vote([3], [1 * 2 + 1], 1, g, vg)            # x = 6 = x_max: no column
    assert nv == 0


def test_vertex_transpose_symmetry():
    """Swapping the x and y axes maps the line (c, s, d0) to (s, c, -d0) and the
    accumulator to its transpose, bit for bit (the two voting modes trade places)."""
    vg = synth.make_vertex_grid(16, 16, (-4.0, 4.0), (-4.0, 4.0))
    rng = np.random.default_rng(5)
    ang = rng.uniform(0.0, 360.0, size=40)
    ang = ang[np.abs(np.abs(np.cos(np.radians(ang))) - np.abs(np.sin(np.radians(ang)))) > 1e-3]
    c = np.cos(np.radians(ang)).astype(np.float32)
    s = np.sin(np.radians(ang)).astype(np.float32)
    d = rng.uniform(-3.0, 3.0, size=ang.size).astype(np.float32)
    n = ang.size
    cells = np.array([(i * n + i) for i in range(n)], np.int64)
    g1 = _grid_from_tables(n, 1, -0.03, 50.0, c, s, d0=d)
    g2 = _grid_from_tables(n, 1, -0.03, 50.0, s, c, d0=-d)
    v1, n1 = vertex_vote(np.ones(n), cells, 1, g1, vg)
    v2, n2 = vertex_vote(np.ones(n), cells, 1, g2, vg)
    assert n1 == n2 > 0
    np.testing.assert_array_equal(v1, v2.T)


def test_vertex_track_threshold():
    """Candidates below the track threshold cast nothing; at it they vote."""
    vg = SMALL_VGRID
    grid = _line_grid([30.0], [0.5])
    assert vertex_vote([6], [0], 7, grid, vg)[1] == 0
    assert vertex_vote([7], [0], 7, grid, vg)[1] == vg.n_x


def _vertex_peaks_brute(vacc, t):
    n_x, n_y = vacc.shape
    out = []
    for ix in range(n_x):
        for iy in range(n_y):
            v = vacc[ix, iy]
            if v < t:
                continue
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    if (dx, dy) == (0, 0) or not (0 <= ix + dx < n_x and 0 <= iy + dy < n_y):
                        continue
                    w = vacc[ix + dx, iy + dy]
                    earlier = dx < 0 or (dx == 0 and dy < 0)
                    ok &= (v > w) if earlier else (v >= w)
            if ok:
                out.append((-int(v), ix * n_y + iy))
    out.sort()
    return [-a for a, _ in out], [b for _, b in out]


@pytest.mark.parametrize("shape,hi", [((5, 7), 3), ((9, 4), 6), ((1, 6), 2), ((12, 12), 9)])
def test_vertex_peaks_brute_force(shape, hi):
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    for _ in range(15):
        vacc = rng.integers(0, hi + 1, size=shape).astype(np.int64)
        for t in (1, hi // 2 + 1):
            v, c, n = vertex_peaks(vacc, t)
            bv, bc = _vertex_peaks_brute(vacc, t)
            assert n == len(bc) and v.tolist() == bv and c.tolist() == bc


def test_vertex_peak_edges_are_not_periodic():
    vacc = np.zeros((6, 5), np.int64)
    vacc[0, 2] = 4
    vacc[5, 2] = 5          # would hide (0, 2) if x wrapped
    vacc[3, 0] = 3
    vacc[3, 4] = 6          # would hide (3, 0) if y wrapped
    v, c, n = vertex_peaks(vacc, 1)
    assert sorted(c.tolist()) == sorted([0 * 5 + 2, 5 * 5 + 2, 3 * 5 + 0, 3 * 5 + 4])


# --------------------------------------------------------------------------------------
# Straight lines: the kappa = 0 family (phi0, d0)
# --------------------------------------------------------------------------------------

def vote_straight(x, y, grid):
    return oracle.vote_straight(x, y, grid, library=LIBRARY[0])


def test_straight_hits_on_a_line_vote_its_cell():
    """Noise-free hits of a line at a (phi0, d0) bin centre all vote that cell, and
    its mirror (d0 -> -d0, phi0 -> phi0 + pi) gets as many."""
    grid = synth.make_straight_grid(64, 48, (-12.0, 12.0))
    for j, k in ((5, 30), (40, 10), (17, 24)):
        phi0 = float(grid.phi_centre(j))
        d0 = -12.0 + (k + 0.5) * 0.5
        hx, hy, ok = synth.events.straight_hits([d0], [phi0])
        x, y = hx[ok].astype(np.float32), hy[ok].astype(np.float32)
        acc, n = vote_straight(x, y, grid)
        assert acc[0, j, k] == x.size > 5
        jm, km = (j + 32) % 64, 47 - k
        assert acc[0, jm, km] == x.size
        v, c, nf = peaks(acc, x.size)
        assert sorted(c.tolist()) == sorted([j * 48 + k, jm * 48 + km])


def test_straight_closed_form_single_hits():
    """A hit votes, in row j, the d0 bin of r sin(phi_h - phi0_j)."""
    grid = synth.make_straight_grid(96, 40, (-20.0, 20.0))
    rng = np.random.default_rng(9)
    phis = grid.phi_centre(np.arange(grid.n_phi))
    for _ in range(40):
        r = rng.uniform(1.0, 30.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        x, y = np.float32(r * math.cos(ph)), np.float32(r * math.sin(ph))
        acc, n = vote_straight([x], [y], grid)
        rr, pp = math.hypot(float(x), float(y)), math.atan2(float(y), float(x))
        for j in range(grid.n_phi):
            fd = (rr * math.sin(pp - phis[j]) + 20.0) * 1.0
            row = acc[0, j]
            if abs(fd - round(fd)) < 1e-3:
                continue                                  # too close to a bin edge to call
            if 0.0 <= fd < grid.n_kappa:
                assert row[int(fd)] == 1 and row.sum() == 1
            else:
                assert row.sum() == 0


def test_straight_one_vote_per_row_and_edges():
    grid = synth.make_straight_grid(32, 64, (-120.0, 120.0))
    ev = synth.gen_config_event(1)
    acc, n = vote_straight(ev.x, ev.y, grid)
    assert n == ev.n_hits * grid.n_phi
    assert (acc.sum(axis=2) == ev.n_hits).all()
    # phi0 = 0: u = y exactly; the lower d0 edge is inside, the upper outside
    g = _grid_from_tables(3, 8, -4.0, 1.0, [1.0, 0.0, -1.0], [0.0, 1.0, 0.0])   # d0 in [-4, 4)
    g = dataclasses.replace(g, family="straight")
    acc, n = vote_straight([0.0, 0.0], [-4.0, 0.0], g)
    assert acc[0, 0, 0] == 1 and acc[0, 0, 4] == 1
    acc, n = vote_straight([0.0], [4.0], g)             # u = 4 = upper edge at phi0 = 0
    assert acc[0, 0].sum() == 0 and acc[0, 2, 0] == 1   # and -4 at phi0 = pi


# --------------------------------------------------------------------------------------
# Forward-hemisphere option: a hit votes only where it lies ahead of P0
# --------------------------------------------------------------------------------------

def _forward(grid):
    return dataclasses.replace(grid, forward=True)


@pytest.mark.parametrize("which", ["small2d", "big2d", "3d"])
def test_forward_option_keeps_the_track_and_drops_its_mirror(which):
    """A noise-free bin-centre track moving away from the origin keeps its #hits votes at its
    own cell under the forward option; its mirror cell (-d0, phi0 + pi, -kappa), whose direction
    of travel puts every hit behind P0, gets none, and the candidates sit at the track."""
    grid = {"small2d": synth.GRID_2D_SMALL, "big2d": synth.GRID_2D, "3d": synth.GRID_3D}[which]
    fg = _forward(grid)
    rng = np.random.default_rng(8)
    done = 0
    while done < 6:
        l = int(rng.integers(0, grid.n_d0))
        j = int(rng.integers(0, grid.n_phi))
        k = int(rng.integers(int(grid.n_kappa * 0.25), int(grid.n_kappa * 0.75)))
        d0, phi0, kappa = _bin_centre_track(grid, l, j, k)
        if grid.is_3d and np.min(np.abs(synth.LAYERS_CM - abs(d0))) < 2.0:
            continue
        ev = synth.gen_tracks_event([d0], [phi0], [kappa])
        if ev.n_hits < 5:
            continue
        acc, n = vote(ev.x, ev.y, fg)
        full, n_full = vote(ev.x, ev.y, grid)
        mirror = (grid.n_d0 - 1 - l, (j + grid.n_phi // 2) % grid.n_phi, grid.n_kappa - 1 - k)
        assert acc[l, j, k] == ev.n_hits
        assert acc[mirror] == 0 and full[mirror] == ev.n_hits
        assert np.all(acc <= full) and 0 < n < n_full
        v, c, nf = peaks(acc, ev.n_hits)
        assert nf >= 1
        for cell in c.tolist():
            a, b, cc = cell // (grid.n_phi * grid.n_kappa), (cell // grid.n_kappa) % grid.n_phi, cell % grid.n_kappa
            assert b == j and cc == k and abs(a - l) <= (1 if grid.is_3d else 0), (which, cell)
        done += 1


def test_forward_option_votes_the_half_circle_ahead():
    """On a kappa range so wide that every (hit, phi0) pair votes, the full vote casts n_phi
    votes per hit, and the forward vote exactly the rows within 90 degrees of the hit's own
    direction (counted with fp64 angles): n_phi / 2 of the bin centres of an even n_phi."""
    grid = make_grid(64, 32, kappa_half_range_inv_cm=0.05)       # kappa in [-20, 20) cm^-1
    fg = _forward(grid)
    rng = np.random.default_rng(21)
    phis = grid.phi_centre(np.arange(grid.n_phi))
    checked = 0
    for _ in range(60):
        r = rng.uniform(0.5, 110.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        x, y = np.float32(r * math.cos(ph)), np.float32(r * math.sin(ph))
        ahead = np.cos(math.atan2(float(y), float(x)) - phis)
        if np.min(np.abs(ahead)) < 1e-5:
            continue                                     # a row too close to abreast to call
        a_full, n_full = vote([x], [y], grid)
        a_fwd, n_fwd = vote([x], [y], fg)
        assert n_full == grid.n_phi
        rows = a_fwd[0].sum(axis=1)
        np.testing.assert_array_equal(rows, (ahead > 0).astype(np.int64))
        assert n_fwd == grid.n_phi // 2
        checked += 1
    assert checked > 50


def test_forward_option_is_strict_and_the_same_for_every_d0():
    """Hand cases with hit (1, 0) and rows (cos, sin) = (0, 1), (1e-30, 1), (-1e-30, 1),
    (1, 0): x cos + y sin is 0, 1e-30, -1e-30 and 1, so the forward option keeps rows 1 and 3
    only (0 is not ahead), in every d0 slice; the full vote keeps all four."""
    c = [0.0, 1e-30, -1e-30, 1.0]
    s = [1.0, 1.0, 1.0, 0.0]
    for d0 in (None, [-0.5, 0.0, 0.5]):
        g = _grid_from_tables(4, 16, -20.0, 0.4, c, s, d0=d0)     # kappa in [-20, 20)
        a_full, _ = vote([1.0], [0.0], g)
        a_fwd, _ = vote([1.0], [0.0], _forward(g))
        for l in range(g.n_d0):
            assert a_full[l].sum(axis=1).tolist() == [1, 1, 1, 1]
            assert a_fwd[l].sum(axis=1).tolist() == [0, 1, 0, 1]


def test_forward_option_straight_lines():
    """Straight family: a line's hits keep its cell and lose its mirror (d0 -> -d0,
    phi0 -> phi0 + pi); on a d0 range wider than every hit radius, each hit votes exactly the
    rows within 90 degrees of its direction."""
    grid = _forward(synth.make_straight_grid(64, 48, (-12.0, 12.0)))
    for j, k in ((5, 30), (40, 10), (17, 24)):
        phi0 = float(grid.phi_centre(j))
        d0 = -12.0 + (k + 0.5) * 0.5
        hx, hy, ok = synth.events.straight_hits([d0], [phi0])
        x, y = hx[ok].astype(np.float32), hy[ok].astype(np.float32)
        acc, n = vote_straight(x, y, grid)
        assert acc[0, j, k] == x.size > 5
        assert acc[0, (j + 32) % 64, 47 - k] == 0
        v, c, nf = peaks(acc, x.size)
        assert c.tolist() == [j * 48 + k]
    wide = _forward(synth.make_straight_grid(32, 64, (-120.0, 120.0)))
    phis = wide.phi_centre(np.arange(wide.n_phi))
    ev = synth.gen_config_event(1)
    for i in range(0, ev.n_hits, 11):
        ahead = np.cos(math.atan2(float(ev.y[i]), float(ev.x[i])) - phis)
        if np.min(np.abs(ahead)) < 1e-5:
            continue
        acc, n = vote_straight(ev.x[i:i + 1], ev.y[i:i + 1], wide)
        np.testing.assert_array_equal(acc[0].sum(axis=1), (ahead > 0).astype(np.int64))


# --------------------------------------------------------------------------------------
# Hit association: the hits that vote inside a candidate's peak window
# --------------------------------------------------------------------------------------

def associate(x, y, grid, votes, cells, min_votes):
    return oracle.associate(x, y, grid, votes, cells, min_votes, library=LIBRARY[0])


def _window_members(grid, acc1, cell):
    """Does a single hit's accumulator acc1 (n_d0, n_phi, n_kappa) hold a vote in the
    3x3(x3) window of cell (phi periodic, d0 and kappa clipped)?"""
    l, j, k = cell // (grid.n_phi * grid.n_kappa), (cell // grid.n_kappa) % grid.n_phi, cell % grid.n_kappa
    rows = [(j + d) % grid.n_phi for d in (-1, 0, 1)]
    sl = acc1[max(l - 1, 0):l + 2][:, rows][:, :, max(k - 1, 0):k + 2]
    return sl.sum() > 0


@pytest.mark.parametrize("which", ["2d", "3d", "straight", "forward"])
def test_association_is_the_single_hit_votes_in_the_window(which):
    """A hit belongs to a candidate exactly when its own vote (the vote routine run on that
    hit alone) lands in the candidate's 3x3(x3) window -- checked pair by pair against
    window sums of single-hit accumulators."""
    if which == "3d":
        grid = make_grid(64, 32, n_d0=5, d0_range=(-10.0, 10.0))
        ev = synth.gen_config_event(3, 2)
        sel = np.arange(0, ev.n_hits, 200)
    elif which == "straight":
        grid = synth.make_straight_grid(64, 48, (-12.0, 12.0))
        ev = synth.gen_config_event(6, 0)
        sel = np.arange(0, ev.n_hits, 120)
    else:
        grid = synth.GRID_2D_SMALL if which == "2d" else _forward(synth.GRID_2D_SMALL)
        ev = synth.gen_config_event(1)
        sel = np.arange(ev.n_hits)
    x, y = ev.x[sel], ev.y[sel]
    one = vote_straight if grid.family == "straight" else vote
    acc, _ = one(x, y, grid)
    votes_all, cells_all, n = peaks(acc, 2)
    votes_all, cells_all = votes_all[:60], cells_all[:60]
    pc, ph = associate(x, y, grid, votes_all, cells_all, 3)
    got = set(zip(pc.tolist(), ph.tolist()))
    singles = [one(x[i:i + 1], y[i:i + 1], grid)[0] for i in range(len(x))]
    want = set()
    for c, (v, cell) in enumerate(zip(votes_all, cells_all)):
        if v < 3:
            continue
        for h, a1 in enumerate(singles):
            if _window_members(grid, a1, int(cell)):
                want.add((c, h))
    assert len(want) > 0
    assert got == want
    # candidate order, hits ascending within a candidate
    assert list(zip(pc.tolist(), ph.tolist())) == sorted(got)


def test_association_of_a_clean_track_is_its_hits():
    """A noise-free bin-centre track: its peak candidate (and, without the forward option,
    its mirror) holds exactly the track's hits; with the forward option the mirror is gone."""
    grid = synth.GRID_2D
    d0, phi0, kappa = _bin_centre_track(grid, 0, 300, 200)
    ev = synth.gen_tracks_event([d0], [phi0], [kappa])
    cell = 300 * grid.n_kappa + 200
    mirror = ((300 + grid.n_phi // 2) % grid.n_phi) * grid.n_kappa + grid.n_kappa - 1 - 200
    pc, ph = associate(ev.x, ev.y, grid, [ev.n_hits, ev.n_hits], [cell, mirror], 1)
    assert ph[pc == 0].tolist() == list(range(ev.n_hits))
    assert ph[pc == 1].tolist() == list(range(ev.n_hits))
    pc, ph = associate(ev.x, ev.y, _forward(grid), [ev.n_hits, ev.n_hits], [cell, mirror], 1)
    assert ph[pc == 0].tolist() == list(range(ev.n_hits)) and (pc == 1).sum() == 0


def test_association_threshold_and_empty_lists():
    ev = synth.gen_config_event(1)
    grid = synth.GRID_2D_SMALL
    acc, _ = vote(ev.x, ev.y, grid)
    v, c, n = peaks(acc, 5)
    pc, ph = associate(ev.x, ev.y, grid, v, c, int(v.max()) + 1)
    assert pc.size == 0
    pc, ph = associate(ev.x, ev.y, grid, v, c, int(v.max()))
    assert set(pc.tolist()) == set(np.nonzero(v == v.max())[0].tolist())
    pc, ph = associate(ev.x[:0], ev.y[:0], grid, v, c, 1)
    assert pc.size == 0
    pc, ph = associate(ev.x, ev.y, grid, v[:0], c[:0], 1)
    assert pc.size == 0


# --------------------------------------------------------------------------------------
# The binary32 operation order (reading 5 of the vote: one rounding per operation, in
# the order C parses the formula, no contraction, correctly rounded division)
# --------------------------------------------------------------------------------------

FP32_ORDER = os.path.join(os.path.dirname(__file__), "golden", "fp32_order.json")


def _fp32_cases():
    with open(FP32_ORDER) as f:
        return json.load(f)


def _hx(s):
    return np.float32(float.fromhex(s))


def _one_row_grid(case, g, family="curved"):
    """A grid of one phi0 row (and one d0 slice) holding the case's table values."""
    d0 = None
    if family == "curved" and float.fromhex(case["d0"]) != 0.0:
        d0 = [_hx(case["d0"])]
    if family == "curved":
        grid = _grid_from_tables(1, g["n_kappa"], _hx(g["kappa_min"]), _hx(g["kappa_scale"]),
                                 [_hx(case["cos"])], [_hx(case["sin"])], d0)
    else:
        grid = _grid_from_tables(1, g["n_d0"], _hx(g["d0_min"]), _hx(g["d0_scale"]),
                                 [_hx(case["cos"])], [_hx(case["sin"])])
        grid = dataclasses.replace(grid, family="straight")
    return grid


def _voted_bin(acc):
    nz = np.flatnonzero(acc.reshape(-1))
    assert len(nz) <= 1 and (len(nz) == 0 or acc.reshape(-1)[nz[0]] == 1)
    return int(nz[0]) if len(nz) else None


def test_fp32_order_curved_votes():
    """Hits whose kappa bin flips under a reordered, contracted, reciprocal or
    binary64 evaluation vote the bin that exact rational arithmetic with one
    binary32 rounding per operation gives (tests/golden/make_fp32_order.py)."""
    doc = _fp32_cases()
    wrong = []
    for i, case in enumerate(doc["curved"]):
        grid = _one_row_grid(case, doc["grids"][case["grid"]])
        acc, _ = vote([_hx(case["x"])], [_hx(case["y"])], grid)
        if _voted_bin(acc) != case["bin"]:
            wrong.append((i, _voted_bin(acc), case["bin"], sorted(case["separates"])))
    assert not wrong, wrong


def test_fp32_order_straight_votes():
    doc = _fp32_cases()
    wrong = []
    for i, case in enumerate(doc["straight"]):
        grid = _one_row_grid(case, doc["grids"][case["grid"]], family="straight")
        acc, _ = vote_straight([_hx(case["x"])], [_hx(case["y"])], grid)
        if _voted_bin(acc) != case["bin"]:
            wrong.append((i, _voted_bin(acc), case["bin"], sorted(case["separates"])))
    assert not wrong, wrong


def test_fp32_order_vertex_votes():
    """One line (a candidate of a one-cell track grid holding the case's d0,
    cos and sin) against one column (or row) centre of the vertex grid."""
    doc = _fp32_cases()
    wrong = []
    for i, case in enumerate(doc["vertex"]):
        g = doc["grids"][case["grid"]]
        tgrid = _grid_from_tables(1, 1, -1.0, 1.0, [_hx(case["cos"])], [_hx(case["sin"])], [_hx(case["d0"])])
        col = case["mode"] == "column"
        centre = [_hx(case["centre"])]
        vg = synth.VertexGrid(
            n_x=1 if col else g["n_x"], n_y=g["n_y"] if col else 1,
            x_centre=np.asarray(centre if col else np.zeros(g["n_x"]), np.float32),
            y_centre=np.asarray(np.zeros(g["n_y"]) if col else centre, np.float32),
            x_min=_hx(g["x_min"]), x_scale=_hx(g["x_scale"]), y_min=_hx(g["y_min"]), y_scale=_hx(g["y_scale"]))
        vacc, _ = vertex_vote([10], [0], 1, tgrid, vg)
        got = _voted_bin(vacc)
        if got != case["bin"]:
            wrong.append((i, got, case["bin"], sorted(case["separates"])))
    assert not wrong, wrong


def test_fp32_order_association():
    """The association recomputes the vote: a case's hit lies in the windows of
    candidates one bin below and one bin above its bin, and a bin flipped either
    way leaves one of the two windows."""
    doc = _fp32_cases()
    wrong = []
    for family in ("curved", "straight"):
        for i, case in enumerate(doc[family]):
            grid = _one_row_grid(case, doc["grids"][case["grid"]], family)
            b = case["bin"]
            c_idx, h_idx = associate([_hx(case["x"])], [_hx(case["y"])], grid, [9, 9], [b - 1, b + 1], 1)
            if list(c_idx) != [0, 1] or list(h_idx) != [0, 0]:
                wrong.append((family, i, list(c_idx), sorted(case["separates"])))
    assert not wrong, wrong
