"""The culling arcs on the CPU: every vote the oracle casts lies inside the
phi0 arcs that hit_prep gives its hit (no GPU).

hit_prep_kernel bounds, per hit and d0 slice, the sine of phi_h - phi0 for
which a vote is possible, turns the bound into two arcs of phi0 and widens
them (the derivation is in the comment above the kernel).  This test redoes
those steps in binary32 with numpy -- the same operations in the same order,
with the device's angle functions and reciprocal replaced by correctly rounded
ones (the kernel's widening covers the difference, which the device self-test
bounds) -- and checks that no row where the oracle votes falls outside the
arcs, over random hits spread across radii, angles and d0 slices, including
hits close to the d0 circles where the bound is tightest.
"""

import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth

F = np.float32
TWO_M18 = F(2.0 ** -18)
ARC_TOL = F(1e-4)
ROW_MARGIN = 1          # rows added on each side of an arc


def _kabs(grid):
    kmin = float(grid.kappa_min)
    kmax = kmin + grid.n_kappa / float(grid.kappa_scale)
    K = max(abs(kmin), abs(kmax)) * (1.0 + 1e-3)
    Kf = F(K)
    if float(Kf) < K:
        Kf = np.nextafter(Kf, F(np.inf))
    return Kf


def _pack_arc(phi_a, phi_b, n, sc):
    """Rows (start, count) whose centres lie in [phi_a, phi_b] widened by the
    tolerance and one row each side; count n is the full circle."""
    lo = F(np.ceil(F(F(phi_a - ARC_TOL) * sc) - F(0.5))) - F(ROW_MARGIN)
    hi = F(np.floor(F(F(phi_b + ARC_TOL) * sc) - F(0.5))) + F(ROW_MARGIN)
    if hi < lo:
        return None
    rows = hi - lo + F(1)
    if rows >= F(n):
        return (0, n)
    return (int(lo) % n, int(rows))


def _rows(arc, n):
    if arc is None:
        return set()
    start, count = arc
    return {(start + k) % n for k in range(count)}


def _arcs(slo, shi, ph, n, sc, fwd):
    pi = F(3.14159274)
    if not (np.isfinite(slo) and np.isfinite(shi)):
        return set(range(n))
    if slo > F(1) or shi < F(-1):
        return set()
    if not fwd and slo <= F(-1) and shi >= F(1):
        return set(range(n))
    alo = F(math.asin(float(max(slo, F(-1)))))
    ahi = F(math.asin(float(min(shi, F(1)))))
    pm = F(ph - pi)
    rows = _rows(_pack_arc(F(ph - ahi), F(ph - alo), n, sc), n)
    if not fwd:
        rows |= _rows(_pack_arc(F(pm + alo), F(pm + ahi), n, sc), n)
    return rows


def arc_rows(x, y, grid):
    """Rows per d0 slice where hit_prep lets the hit vote (a list of sets)."""
    x, y = F(x), F(y)
    n = grid.n_phi
    r2 = F(F(x * x) + F(y * y))
    r = F(np.sqrt(r2))
    r_ok = F(2.0 ** -30) <= r <= F(2.0 ** 30)
    inv_r = F(F(1) / (r if r_ok else F(1)))
    half_inv_r = F(F(0.5) * inv_r)
    ph = F(math.atan2(float(y), float(x)))
    sc = F(F(n) * F(0.159154943))
    fwd = bool(grid.forward)
    if grid.family == "straight":
        dlo = F(grid.kappa_min)
        dhi = F(float(grid.kappa_min) + grid.n_kappa / float(grid.kappa_scale))
        if not r_ok:
            return [set(range(n))]
        m = F(F(1e-5) + F(F(TWO_M18 * F(F(F(2) * abs(dlo)) + F(F(2) * abs(dhi)))) * inv_r))
        return [_arcs(F(F(dlo * inv_r) - m), F(F(dhi * inv_r) + m), ph, n, sc, fwd)]
    K = _kabs(grid)
    out = []
    for l in range(grid.n_d0):
        d = F(grid.d0[l]) if grid.d0 is not None else F(0)
        ad = abs(d)
        kd = F(K * ad)
        if r_ok and ad <= F(2.0 ** 30) and abs(F(r - ad)) >= F(F(0.0301) * F(r + ad)) and kd <= F(0.99):
            rr = F(r2 + F(d * d))
            a = F(K * rr)
            b = F(F(2) * d)
            s1 = F(F(F(b - a) * half_inv_r) * F(F(1) / F(F(1) - F(K * d))))
            s2 = F(F(F(b + a) * half_inv_r) * F(F(1) / F(F(1) + F(K * d))))
            w = F(F(1) / F(F(1) - kd))
            m = F(F(1e-5) + F(F(F(F(TWO_M18 * F(a + F(F(2) * ad))) * inv_r) * w) * w))
            out.append(_arcs(F(min(s1, s2) - m), F(max(s1, s2) + m), ph, n, sc, fwd))
        else:
            out.append(set(range(n)))
    return out


def _narrow(grid, n_kappa=8):
    """The grid with fewer kappa bins over the same kappa (or d0) range: the
    arcs depend only on the range, and the oracle runs faster."""
    scale = F(float(grid.kappa_scale) * n_kappa / grid.n_kappa)
    return dataclasses.replace(grid, n_kappa=n_kappa, kappa_scale=scale)


def _hits(rng, n, d0=None):
    r = np.exp(rng.uniform(math.log(0.5), math.log(200.0), size=n))
    if d0 is not None:              # half of them within 2 % of a d0 circle
        pick = rng.uniform(size=n) < 0.5
        r = np.where(pick, np.abs(rng.choice(d0, size=n)) * rng.uniform(0.98, 1.02, size=n) + 1e-3, r)
    phi = rng.uniform(0, 2 * math.pi, size=n)
    return (r * np.cos(phi)).astype(F), (r * np.sin(phi)).astype(F)


def _check(grid, x, y, vote):
    kept = total = 0
    for xi, yi in zip(x, y):
        acc, _ = vote(np.array([xi], F), np.array([yi], F), grid)
        acc = acc.reshape(grid.n_d0 if grid.family != "straight" else 1, grid.n_phi, -1)
        arcs = arc_rows(xi, yi, grid)
        for l, rows in enumerate(arcs):
            voted = set(np.flatnonzero(acc[l].sum(axis=1)).tolist())
            missing = voted - rows
            assert not missing, f"hit ({xi!r}, {yi!r}) slice {l}: votes outside its arcs in rows {sorted(missing)[:8]}"
            kept += len(rows)
            total += grid.n_phi
    return kept / total


@pytest.mark.parametrize("forward", [False, True])
def test_prompt_grid_votes_lie_in_their_arcs(forward):
    grid = dataclasses.replace(_narrow(synth.GRID_2D), forward=forward)
    x, y = _hits(np.random.default_rng(11 + forward), 3000)
    share = _check(grid, x, y, oracle.vote)
    assert share < (0.45 if forward else 0.8)     # the arcs do cull


def test_displaced_grid_votes_lie_in_their_arcs():
    grid = _narrow(synth.GRID_3D)
    x, y = _hits(np.random.default_rng(12), 400, d0=grid.d0)
    share = _check(grid, x, y, oracle.vote)
    assert share < 0.9


def test_straight_grid_votes_lie_in_their_arcs():
    grid = _narrow(synth.GRID_STRAIGHT)
    x, y = _hits(np.random.default_rng(13), 3000)
    _check(grid, x, y, oracle.vote_straight)


def test_the_emulation_is_not_vacuous():
    """Arcs without their row margin and angle tolerance miss votes on the same
    hits: the checks above can fail."""
    grid = _narrow(synth.GRID_2D)
    x, y = _hits(np.random.default_rng(14), 3000)
    global ARC_TOL, ROW_MARGIN
    saved = ARC_TOL, ROW_MARGIN
    ARC_TOL, ROW_MARGIN = F(-1e-4), 0
    try:
        with pytest.raises(AssertionError, match="outside its arcs"):
            _check(grid, x, y, oracle.vote)
    finally:
        ARC_TOL, ROW_MARGIN = saved
