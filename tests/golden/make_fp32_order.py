"""Write tests/golden/fp32_order.json: votes whose kappa bin depends on the
binary32 operation order.

The vote is specified as a fixed sequence of IEEE binary32 operations (the
formula of Section 3's vote in the reading that every operation rounds once to
nearest even, in the order C parses it, with no contraction).  A reordered or
contracted evaluation computes the same real number with different roundings,
so it lands in another bin only where the exact kf lies within a few units in
the last place of an integer.  This script finds such (hit, row) pairs on the
workload grids and records, for each, every intermediate value of the
canonical sequence and the bin it gives.

The values are derived here with exact rational arithmetic
(``fractions.Fraction``): each operation is computed exactly and then rounded
to the nearest binary32 number (ties to even), the definition of a binary32
operation.  A fused multiply-add rounds the exact a*b + c once.  Nothing here
calls the oracle or the HIP library; the bin tables and the hit positions come
from ``synth`` (shared inputs, no vote arithmetic).  numpy float32 only
proposes candidate pairs; every recorded value is recomputed exactly.

Each recorded case also lists the alternative orders it separates, with the
bin each alternative gives, so a reader can see why the case is there.

Run:  python tests/golden/make_fp32_order.py
"""

from __future__ import annotations

import json
import math
import os
import sys
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402  (bin tables only)

OUT = os.path.join(HERE, "fp32_order.json")
SEED = 20131112


# ---------------------------------------------------------------------------
# binary32 rounding from its definition
# ---------------------------------------------------------------------------

def rn(q: Fraction) -> Fraction:
    """Round an exact rational to the nearest binary32 number, ties to even.

    Normal numbers have 24 significant bits; below 2^-126 the quantum stays
    2^-149 (subnormals).  Overflow is an error here: no recorded case comes
    near it."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    # now 2^e <= a < 2^(e+1)
    quantum = Fraction(2) ** (max(e, -126) - 23)
    m = a / quantum
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    r = n * quantum
    if r >= Fraction(2) ** 128:
        raise OverflowError("binary32 overflow")
    return sign * r


def f32(v) -> Fraction:
    """An fp32 value (numpy float32 or Python float holding one) as an exact rational."""
    v = float(np.float32(v))
    assert math.isfinite(v)
    return Fraction(v)


def hexf(q: Fraction) -> str:
    return float(q).hex()


def floor_bin(kf: Fraction, n: int):
    """The bin a kf selects: floor(kf) when 0 <= kf < n, else None."""
    if kf >= 0 and kf < n:
        return kf.numerator // kf.denominator
    return None


# ---------------------------------------------------------------------------
# The canonical sequence and the alternatives
# ---------------------------------------------------------------------------

def curved_steps(x, y, d, c, s, kmin, kscale):
    """Section 3's vote, one binary32 rounding per operation, canonical order:
    r2 = x*x + y*y; u = y*c - x*s; num = 2*(u - d); den = (r2 - (2*d)*u) + d*d;
    kappa = num / den; kf = (kappa - kappa_min) * kappa_scale."""
    r2 = rn(rn(x * x) + rn(y * y))
    u = rn(rn(y * c) - rn(x * s))
    num = rn(2 * rn(u - d))
    den = rn(rn(r2 - rn(rn(2 * d) * u)) + rn(d * d))
    kappa = rn(num / den)
    kf = rn(rn(kappa - kmin) * kscale)
    return dict(r2=r2, u=u, num=num, den=den, kappa=kappa, kf=kf)


def _curved_alt(x, y, d, c, s, kmin, kscale, *, r2=None, u=None, den=None, kappa=None, kf=None):
    """The canonical sequence with chosen steps replaced by an alternative."""
    R2 = r2(x, y) if r2 else rn(rn(x * x) + rn(y * y))
    U = u(x, y, c, s) if u else rn(rn(y * c) - rn(x * s))
    NUM = rn(2 * rn(U - d))
    DEN = den(R2, U, d) if den else rn(rn(R2 - rn(rn(2 * d) * U)) + rn(d * d))
    KAPPA = kappa(NUM, DEN) if kappa else rn(NUM / DEN)
    KF = kf(KAPPA, kmin, kscale) if kf else rn(rn(KAPPA - kmin) * kscale)
    return KF


CURVED_ALTS = {
    # r2 with one product fused into the sum
    "r2_fma_x": dict(r2=lambda x, y: rn(x * x + rn(y * y))),
    "r2_fma_y": dict(r2=lambda x, y: rn(y * y + rn(x * x))),
    # u with one product fused into the difference
    "u_fma_yc": dict(u=lambda x, y, c, s: rn(y * c - rn(x * s))),
    "u_fma_xs": dict(u=lambda x, y, c, s: rn(rn(y * c) - x * s)),
    # the denominator reassociated or contracted (3D only: at d = 0 all equal r2)
    "den_reassociated": dict(den=lambda r2, u, d: rn(r2 + rn(rn(d * d) - rn(rn(2 * d) * u)))),
    "den_square_first": dict(den=lambda r2, u, d: rn(rn(r2 + rn(d * d)) - rn(rn(2 * d) * u))),
    "den_fma_cross": dict(den=lambda r2, u, d: rn(rn(r2 - rn(2 * d) * u) + rn(d * d))),
    "den_fma_square": dict(den=lambda r2, u, d: rn(d * d + rn(r2 - rn(rn(2 * d) * u)))),
    # division through a rounded reciprocal
    "kappa_by_reciprocal": dict(kappa=lambda num, den: rn(num * rn(1 / den))),
    # kf distributed or contracted
    "kf_distributed": dict(kf=lambda k, kmin, ks: rn(rn(k * ks) - rn(kmin * ks))),
    "kf_fma": dict(kf=lambda k, kmin, ks: rn(k * ks - rn(kmin * ks))),
}


def curved_in_double(x, y, d, c, s, kmin, kscale, n):
    """The whole vote evaluated in binary64 (Python floats are IEEE doubles)."""
    x, y, d, c, s, kmin, kscale = map(float, (x, y, d, c, s, kmin, kscale))
    u = y * c - x * s
    num = 2.0 * (u - d)
    den = x * x + y * y - 2.0 * d * u + d * d
    kappa = num / den
    kf = (kappa - kmin) * kscale
    return math.floor(kf) if 0.0 <= kf < n else None


def straight_steps(x, y, c, s, dmin, dscale):
    """The straight-line vote: u = y*c - x*s; fd = (u - d0_min) * d0_scale."""
    u = rn(rn(y * c) - rn(x * s))
    fd = rn(rn(u - dmin) * dscale)
    return dict(u=u, fd=fd)


STRAIGHT_ALTS = {
    "u_fma_yc": lambda x, y, c, s, dm, ds: rn(rn(rn(y * c - rn(x * s)) - dm) * ds),
    "u_fma_xs": lambda x, y, c, s, dm, ds: rn(rn(rn(rn(y * c) - x * s) - dm) * ds),
    "fd_distributed": lambda x, y, c, s, dm, ds: rn(rn(rn(rn(y * c) - rn(x * s)) * ds) - rn(dm * ds)),
    "fd_fma": lambda x, y, c, s, dm, ds: rn(rn(rn(y * c) - rn(x * s)) * ds - rn(dm * ds)),
}


def vertex_steps(mode, dt, c, s, centre, vmin, vscale):
    """Section 5's second transform for one line and one column (mode 'column':
    y = (d0 + x_c*s) / c) or row (mode 'row': x = (y_c*c - d0) / s); then
    f = (position - min) * scale."""
    if mode == "column":
        t = rn(centre * s)
        num = rn(dt + t)
        pos = rn(num / c)
    else:
        t = rn(centre * c)
        num = rn(t - dt)
        pos = rn(num / s)
    f = rn(rn(pos - vmin) * vscale)
    return dict(t=t, num=num, pos=pos, f=f)


def _vertex_alt(mode, dt, c, s, centre, vmin, vscale, which):
    if mode == "column":
        num = rn(centre * s + dt) if which == "num_fma" else rn(dt + rn(centre * s))
        den = c
    else:
        num = rn(centre * c - dt) if which == "num_fma" else rn(rn(centre * c) - dt)
        den = s
    pos = rn(num * rn(1 / den)) if which == "by_reciprocal" else rn(num / den)
    if which == "f_distributed":
        return rn(rn(pos * vscale) - rn(vmin * vscale))
    return rn(rn(pos - vmin) * vscale)


VERTEX_ALTS = ("num_fma", "by_reciprocal", "f_distributed")


# ---------------------------------------------------------------------------
# numpy proposals (float32 with numpy's correctly rounded single operations;
# fused forms through float64, which may double-round: proposals only)
# ---------------------------------------------------------------------------

F32 = np.float32


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def np_curved(x, y, d, c, s, kmin, kscale, alt=None):
    x, y, d, c, s = (np.asarray(v, F32) for v in (x, y, d, c, s))
    kmin, kscale = F32(kmin), F32(kscale)
    r2 = x * x + y * y
    if alt == "r2_fma_x":
        r2 = _fma32(x, x, y * y)
    if alt == "r2_fma_y":
        r2 = _fma32(y, y, x * x)
    u = y * c - x * s
    if alt == "u_fma_yc":
        u = _fma32(y, c, -(x * s))
    if alt == "u_fma_xs":
        u = _fma32(-x, s, y * c)
    num = F32(2) * (u - d)
    den = (r2 - (F32(2) * d) * u) + d * d
    if alt == "den_reassociated":
        den = r2 + (d * d - (F32(2) * d) * u)
    if alt == "den_square_first":
        den = (r2 + d * d) - (F32(2) * d) * u
    if alt == "den_fma_cross":
        den = _fma32(-(F32(2) * d), u, r2) + d * d
    if alt == "den_fma_square":
        den = _fma32(d, d, r2 - (F32(2) * d) * u)
    kappa = num / den
    if alt == "kappa_by_reciprocal":
        kappa = num * (F32(1) / den)
    kf = (kappa - kmin) * kscale
    if alt == "kf_distributed":
        kf = kappa * kscale - kmin * kscale
    if alt == "kf_fma":
        kf = _fma32(kappa, np.broadcast_to(kscale, kappa.shape), np.broadcast_to(-(kmin * kscale), kappa.shape))
    return kf


def np_bin(kf, n):
    ok = (kf >= 0) & (kf < n)
    return np.where(ok, np.floor(np.where(ok, kf, 0)).astype(np.int64), -1)


# ---------------------------------------------------------------------------
# Search
# ---------------------------------------------------------------------------

LAYERS = np.array([4, 7, 11, 16, 25, 35, 50, 65, 85, 110], dtype=np.float64)


def _hits(rng, n):
    r = rng.choice(LAYERS, size=n) * (1.0 + rng.uniform(-0.01, 0.01, size=n))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return (r * np.cos(phi)).astype(F32), (r * np.sin(phi)).astype(F32)


def _curved_case(grid, name, x, y, l, j, d_value=None):
    if d_value is not None:
        d = f32(d_value)
    else:
        d = f32(grid.d0[l]) if grid.d0 is not None else Fraction(0)
    c, s = f32(grid.cos_phi[j]), f32(grid.sin_phi[j])
    kmin, kscale = f32(grid.kappa_min), f32(grid.kappa_scale)
    X, Y = f32(x), f32(y)
    st = curved_steps(X, Y, d, c, s, kmin, kscale)
    b = floor_bin(st["kf"], grid.n_kappa)
    sep = {}
    for alt, kw in CURVED_ALTS.items():
        ab = floor_bin(_curved_alt(X, Y, d, c, s, kmin, kscale, **kw), grid.n_kappa)
        if ab != b:
            sep[alt] = ab
    db = curved_in_double(X, Y, d, c, s, kmin, kscale, grid.n_kappa)
    if db != b:
        sep["vote_in_double"] = db
    return dict(grid=name, l=None if d_value is not None else int(l), j=int(j), x=hexf(X), y=hexf(Y), d0=hexf(d), cos=hexf(c), sin=hexf(s),
                steps={k: hexf(v) for k, v in st.items()}, bin=b, separates=sep)


def search_curved(grid, name, alts, per_alt, rng, n_hits=4096, need_d=False, random_d0=False):
    """(hit, row) pairs of ``grid`` that the alternatives ``alts`` vote into
    another bin.  ``random_d0`` draws each hit's d0 from U[-30, 30] instead of
    the grid's bin centres, whose squares are exact in binary32 (there d0*d0
    fused into the sum rounds the same)."""
    cases, seen = [], set()
    got = {a: 0 for a in alts}
    n_l = grid.n_d0
    d0 = grid.d0 if grid.d0 is not None else np.zeros(1, F32)
    for _ in range(40):
        if all(v >= per_alt for v in got.values()):
            break
        x, y = _hits(rng, n_hits)
        ls = rng.integers(0, n_l, size=n_hits) if n_l > 1 else np.zeros(n_hits, np.int64)
        if need_d:
            ls = np.where(np.abs(d0[ls]) < 3.0, (ls + n_l // 4) % n_l, ls)
        dv = rng.uniform(-30.0, 30.0, size=n_hits).astype(F32) if random_d0 else d0[ls]
        X, Y, D = x[:, None], y[:, None], dv[:, None]
        C, S = grid.cos_phi[None, :], grid.sin_phi[None, :]
        base = np_bin(np_curved(X, Y, D, C, S, grid.kappa_min, grid.kappa_scale), grid.n_kappa)
        for alt in alts:
            if got[alt] >= per_alt:
                continue
            other = np_bin(np_curved(X, Y, D, C, S, grid.kappa_min, grid.kappa_scale, alt), grid.n_kappa)
            hi, jj = np.nonzero(base != other)
            for h, j in zip(hi[:64], jj[:64]):
                key = (int(h), int(j))
                if key in seen:
                    continue
                case = _curved_case(grid, name, x[h], y[h], ls[h], j, dv[h] if random_d0 else None)
                # keep cases inside the grid away from its first and last bins
                if case["bin"] is None or not (1 <= case["bin"] <= grid.n_kappa - 2):
                    continue
                if alt not in case["separates"]:
                    continue
                seen.add(key)
                cases.append(case)
                for a in case["separates"]:
                    if a in got:
                        got[a] += 1
                break
    missing = [a for a, v in got.items() if v == 0]
    if missing:
        raise RuntimeError(f"no separating case found for {missing} on {name}")
    return cases


def search_straight(grid, name, alts, per_alt, rng, n_hits=4096):
    """(hit, row) pairs of a straight-line grid that ``alts`` vote into another
    d0 bin.  On the workload grid (8 bins per cm, a power of two) the
    distributed and fused forms of fd round exactly as the canonical one, so
    they are searched on a grid whose scale is not a power of two."""
    cases, got = [], {a: 0 for a in alts}
    C, S = grid.cos_phi[None, :], grid.sin_phi[None, :]
    dm, ds = F32(grid.kappa_min), F32(grid.kappa_scale)
    for _ in range(40):
        if all(v >= per_alt for v in got.values()):
            break
        x, y = _hits(rng, n_hits)
        X, Y = x[:, None], y[:, None]
        u = Y * C - X * S
        base = np_bin((u - dm) * ds, grid.n_kappa)
        props = {
            "u_fma_yc": (_fma32(np.broadcast_to(Y, u.shape), np.broadcast_to(C, u.shape), -(X * S)) - dm) * ds,
            "u_fma_xs": (_fma32(np.broadcast_to(-X, u.shape), np.broadcast_to(S, u.shape), Y * C) - dm) * ds,
            "fd_distributed": u * ds - dm * ds,
            "fd_fma": _fma32(u, np.broadcast_to(ds, u.shape), np.broadcast_to(-(dm * ds), u.shape)),
        }
        for alt, kf in props.items():
            if alt not in got or got[alt] >= per_alt:
                continue
            hi, jj = np.nonzero(base != np_bin(kf, grid.n_kappa))
            for h, j in zip(hi[:64], jj[:64]):
                Xh, Yh = f32(x[h]), f32(y[h])
                c, s = f32(grid.cos_phi[j]), f32(grid.sin_phi[j])
                st = straight_steps(Xh, Yh, c, s, f32(dm), f32(ds))
                b = floor_bin(st["fd"], grid.n_kappa)
                if b is None or not (1 <= b <= grid.n_kappa - 2):
                    continue
                sep = {}
                for a, fn in STRAIGHT_ALTS.items():
                    ab = floor_bin(fn(Xh, Yh, c, s, f32(dm), f32(ds)), grid.n_kappa)
                    if ab != b:
                        sep[a] = ab
                if alt not in sep:
                    continue
                cases.append(dict(grid=name, j=int(j), x=hexf(Xh), y=hexf(Yh), cos=hexf(c), sin=hexf(s),
                                  steps={k: hexf(v) for k, v in st.items()}, bin=b, separates=sep))
                for a in sep:
                    if a in got:
                        got[a] += 1
                break
    missing = [a for a, v in got.items() if v == 0]
    if missing:
        raise RuntimeError(f"no separating straight case for {missing}")
    return cases


def search_vertex(vgrid, vname, alts, per_alt, rng, n_lines=65536):
    """Lines (d0, phi0) against the vertex grid's column (or row) centres.

    The lines are drawn at random (d0 U[-30, 30] cm, phi0 U[0, 2 pi)) rather
    than at the displaced grid's bin centres: with the centres' short binary
    fractions the alternatives below rarely reach another bin.  The workload's
    vertex grid has 2 bins per cm, a power of two, where the distributed f
    rounds as the canonical one; that form is searched on a grid of 1.5625
    bins per cm."""
    cases, got = [], {(m, a): 0 for m in ("column", "row") for a in alts}
    for _ in range(40):
        if all(v >= per_alt for v in got.values()):
            break
        dt = rng.uniform(-30.0, 30.0, size=n_lines).astype(F32)
        phi = rng.uniform(0.0, 2.0 * math.pi, size=n_lines)
        c, s = np.cos(phi).astype(F32), np.sin(phi).astype(F32)
        for mode in ("column", "row"):
            sel = np.abs(c) >= np.abs(s) if mode == "column" else np.abs(c) < np.abs(s)
            dtm, cm, sm = dt[sel], c[sel], s[sel]
            centres = vgrid.x_centre if mode == "column" else vgrid.y_centre
            vmin = F32(vgrid.y_min if mode == "column" else vgrid.x_min)
            vscale = F32(vgrid.y_scale if mode == "column" else vgrid.x_scale)
            nbin = vgrid.n_y if mode == "column" else vgrid.n_x
            D, CC, SS = dtm[:, None], cm[:, None], sm[:, None]
            Z = centres[None, :]
            if mode == "column":
                t = Z * SS
                num = D + t
                den = CC
                fused = _fma32(np.broadcast_to(Z, t.shape), np.broadcast_to(SS, t.shape),
                               np.broadcast_to(D, t.shape))
            else:
                t = Z * CC
                num = t - D
                den = SS
                fused = _fma32(np.broadcast_to(Z, t.shape), np.broadcast_to(CC, t.shape),
                               np.broadcast_to(-D, t.shape))
            pos = num / den
            base = np_bin((pos - vmin) * vscale, nbin)
            props = {
                "num_fma": ((fused / den) - vmin) * vscale,
                "by_reciprocal": ((num * (F32(1) / den)) - vmin) * vscale,
                "f_distributed": pos * vscale - vmin * vscale,
            }
            for alt, f in props.items():
                if (mode, alt) not in got or got[(mode, alt)] >= per_alt:
                    continue
                hi, zi = np.nonzero(base != np_bin(f, nbin))
                for h, z in zip(hi[:64], zi[:64]):
                    DT, C_, S_ = f32(dtm[h]), f32(cm[h]), f32(sm[h])
                    Zc = f32(centres[z])
                    st = vertex_steps(mode, DT, C_, S_, Zc, f32(vmin), f32(vscale))
                    b = floor_bin(st["f"], nbin)
                    if b is None or not (1 <= b <= nbin - 2):
                        continue
                    sep = {}
                    for a in VERTEX_ALTS:
                        ab = floor_bin(_vertex_alt(mode, DT, C_, S_, Zc, f32(vmin), f32(vscale), a), nbin)
                        if ab != b:
                            sep[a] = ab
                    if alt not in sep:
                        continue
                    cases.append(dict(grid=vname, mode=mode, centre_index=int(z), d0=hexf(DT), cos=hexf(C_),
                                      sin=hexf(S_), centre=hexf(Zc), steps={k: hexf(v) for k, v in st.items()},
                                      bin=b, separates=sep))
                    for a in sep:
                        if (mode, a) in got:
                            got[(mode, a)] += 1
                    break
    missing = [k for k, v in got.items() if v == 0]
    if missing:
        raise RuntimeError(f"no separating vertex case for {missing}")
    return cases


def main():
    rng = np.random.default_rng(SEED)
    g2, g3, gs = synth.GRID_2D, synth.GRID_3D, synth.GRID_STRAIGHT
    alts_2d = ["r2_fma_x", "r2_fma_y", "u_fma_yc", "u_fma_xs", "kappa_by_reciprocal", "kf_distributed", "kf_fma"]
    alts_3d = alts_2d + ["den_reassociated", "den_square_first", "den_fma_cross", "den_fma_square"]
    curved = search_curved(g2, "pileup_2d_1024x512", alts_2d, 3, rng)
    curved += search_curved(g3, "displaced_3d_64x512x256", alts_3d[:-1], 3, rng, need_d=True)
    curved += search_curved(g3, "displaced_3d_64x512x256", ["den_fma_square"], 2, rng, random_d0=True)
    if not any("vote_in_double" in c["separates"] for c in curved):
        raise RuntimeError("no case separates the binary64 evaluation")
    gs60 = synth.make_straight_grid(1024, 512, d0_range=(-30.0, 30.0))
    straight = search_straight(gs, "straight_1024x512", ["u_fma_yc", "u_fma_xs"], 3, rng)
    straight += search_straight(gs60, "straight_1024x512_60cm", ["fd_distributed", "fd_fma"], 3, rng)
    vg, vg100 = synth.VERTEX_GRID, synth.make_vertex_grid(100, 100)
    vertex = search_vertex(vg, "vertex_128x128", ["num_fma", "by_reciprocal"], 3, rng)
    vertex += search_vertex(vg100, "vertex_100x100", ["f_distributed"], 3, rng)
    doc = {
        "about": ("Votes whose bin depends on the binary32 operation order (the vote of Section 3 as a fixed "
                  "sequence of binary32 operations, each rounded once to nearest even, no contraction). "
                  "Every value is a binary32 number written as a hex float. 'steps' holds each "
                  "intermediate of the canonical sequence, derived with exact rational arithmetic and one "
                  "rounding per operation; 'bin' is the bin it selects (null: no vote). 'separates' lists "
                  "alternative orders that select another bin, with the bin each selects."),
        "written_by": "tests/golden/make_fp32_order.py (exact rationals; calls neither the oracle nor the HIP "
                      "library)",
        "curved_order": "r2 = x*x + y*y; u = y*cos - x*sin; num = 2*(u - d0); den = (r2 - (2*d0)*u) + d0*d0; "
                        "kappa = num / den; kf = (kappa - kappa_min) * kappa_scale; bin = floor(kf) if "
                        "0 <= kf < n_kappa",
        "straight_order": "u = y*cos - x*sin; fd = (u - d0_min) * d0_scale; bin = floor(fd) if 0 <= fd < n_d0",
        "vertex_order": "column: t = x_c*sin; num = d0 + t; pos = num / cos; row: t = y_c*cos; num = t - d0; "
                        "pos = num / sin; f = (pos - min) * scale; bin = floor(f) if 0 <= f < n",
        "grids": {
            "pileup_2d_1024x512": dict(n_kappa=g2.n_kappa, kappa_min=hexf(f32(g2.kappa_min)),
                                       kappa_scale=hexf(f32(g2.kappa_scale))),
            "displaced_3d_64x512x256": dict(n_kappa=g3.n_kappa, kappa_min=hexf(f32(g3.kappa_min)),
                                            kappa_scale=hexf(f32(g3.kappa_scale))),
            "straight_1024x512": dict(n_d0=gs.n_kappa, d0_min=hexf(f32(gs.kappa_min)),
                                      d0_scale=hexf(f32(gs.kappa_scale))),
            "straight_1024x512_60cm": dict(n_d0=gs60.n_kappa, d0_min=hexf(f32(gs60.kappa_min)),
                                           d0_scale=hexf(f32(gs60.kappa_scale))),
            **{name: dict(n_x=g.n_x, n_y=g.n_y, x_min=hexf(f32(g.x_min)), x_scale=hexf(f32(g.x_scale)),
                          y_min=hexf(f32(g.y_min)), y_scale=hexf(f32(g.y_scale)))
               for name, g in (("vertex_128x128", vg), ("vertex_100x100", vg100))},
        },
        "curved": curved,
        "straight": straight,
        "vertex": vertex,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}: {len(curved)} curved, {len(straight)} straight, {len(vertex)} vertex cases")


if __name__ == "__main__":
    main()
