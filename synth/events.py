"""Seeded toy events in the transverse plane (the detector model of Section 3).

Hits are placed geometrically, by intersecting each charged-particle circle
with the cylindrical layers; nothing here evaluates the Hough curvature
formula, so a generated track is an independent check of it.

Conventions (units cm, GeV, T):
* A track has a start point S, a direction angle psi at S and a signed
  curvature k (k > 0 turns counter-clockwise).  Its circle has centre
  ``C = S + (1/k) * (-sin psi, cos psi)`` and the point reached after arc
  length s is ``C + (1/k) * (sin(psi + k s), -cos(psi + k s))``.
* The track parameters (d0, phi0, kappa) are taken at the point of closest
  approach to the origin, ``P0 = (-d0 sin phi0, d0 cos phi0)``, where the
  direction of motion is ``(cos phi0, sin phi0)`` and kappa = k.
* A positive charge in a field along +z turns clockwise:
  ``kappa = -q * 0.299792458 * B / (100 * pT)``.
* Each track leaves one hit at its first forward crossing of each layer
  (loopers that never reach a layer leave none there), smeared along r*phi.
* Noise hits sit on a uniformly chosen layer at a uniform azimuth.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

LAYERS_CM = np.array([4.0, 7.0, 11.0, 16.0, 25.0, 35.0, 50.0, 65.0, 85.0, 110.0])
BASE_SEED = 13112769
B_TESLA = 3.8
C_LIGHT = 0.299792458          # GeV per (T m)
SMEAR_RPHI_CM = 20e-4          # 20 um Gaussian r-phi resolution
TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Event:
    x: np.ndarray                # fp32 [n_hits], cm
    y: np.ndarray                # fp32 [n_hits], cm
    label: np.ndarray            # int32 [n_hits]: track index, -1 for noise
    d0: np.ndarray               # fp64 [n_tracks] truth at closest approach
    phi0: np.ndarray             # fp64 [n_tracks] in [0, 2 pi)
    kappa: np.ndarray            # fp64 [n_tracks], cm^-1
    kind: str = "2d"             # "2d" (prompt grid) or "3d" (displaced grid)

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class Batch:
    x: np.ndarray                # fp32, all events packed
    y: np.ndarray
    hit_off: np.ndarray          # int64 [n_events + 1] CSR offsets
    events: list

    @property
    def n_events(self) -> int:
        return len(self.events)

    @property
    def n_hits(self) -> int:
        return int(self.hit_off[-1])


def kappa_from_pt(pt, q, b_tesla: float = B_TESLA):
    return -np.asarray(q, dtype=np.float64) * C_LIGHT * b_tesla / (100.0 * np.asarray(pt, dtype=np.float64))


def _first_crossing(sx, sy, psi, k, r):
    """First forward crossing (arc length s > 0) of each track with each radius.

    Broadcasts track arrays of shape (T, 1) against radii (1, L).  Returns
    (x, y, ok) in fp64.  The circle-circle intersection is solved directly:
    no parameter is recovered from the hit position.
    """
    sx, sy, psi, k, r = np.broadcast_arrays(sx, sy, psi, k, r)
    xo = np.full(sx.shape, np.nan)
    yo = np.full(sx.shape, np.nan)
    ok = np.zeros(sx.shape, dtype=bool)
    eps = 1e-9

    straight = k == 0.0
    if np.any(straight):
        m = straight
        dx, dy = np.cos(psi[m]), np.sin(psi[m])
        b = sx[m] * dx + sy[m] * dy
        c = sx[m] ** 2 + sy[m] ** 2 - r[m] ** 2
        disc = b * b - c
        good = disc >= 0
        sq = np.sqrt(np.where(good, disc, 0.0))
        s1, s2 = -b - sq, -b + sq
        s = np.where(s1 > eps, s1, np.where(s2 > eps, s2, np.nan))
        good &= np.isfinite(s)
        xo[m] = np.where(good, sx[m] + s * dx, np.nan)
        yo[m] = np.where(good, sy[m] + s * dy, np.nan)
        ok[m] = good

    m = ~straight
    if np.any(m):
        kk, ps, rr = k[m], psi[m], r[m]
        rad = 1.0 / np.abs(kk)
        cx = sx[m] - np.sin(ps) / kk
        cy = sy[m] + np.cos(ps) / kk
        dist = np.hypot(cx, cy)
        a = (rr * rr - rad * rad + dist * dist) / (2.0 * dist)
        h2 = rr * rr - a * a
        good = (h2 >= 0) & (dist > 0)
        h = np.sqrt(np.where(good, h2, 0.0))
        ux, uy = cx / dist, cy / dist
        best_s = np.full(kk.shape, np.inf)
        bx = np.full(kk.shape, np.nan)
        by = np.full(kk.shape, np.nan)
        for sign in (1.0, -1.0):
            px = a * ux - sign * h * uy
            py = a * uy + sign * h * ux
            # phase t of the point: (sin t, -cos t) = k * (p - C)
            t = np.arctan2(kk * (px - cx), -kk * (py - cy))
            dphi = np.where(kk > 0, t - ps, ps - t)
            s = np.mod(dphi, TWO_PI) * rad
            s = np.where(s <= eps * rad, s + TWO_PI * rad, s)
            better = good & (s < best_s)
            best_s = np.where(better, s, best_s)
            bx = np.where(better, px, bx)
            by = np.where(better, py, by)
        xo[m], yo[m], ok[m] = bx, by, good & np.isfinite(best_s)
    return xo, yo, ok


def closest_approach(sx, sy, psi, k):
    """(d0, phi0) of the circle through S with direction psi and curvature k."""
    sx, sy, psi, k = (np.asarray(v, dtype=np.float64) for v in (sx, sy, psi, k))
    cx = sx - np.sin(psi) / k
    cy = sy + np.cos(psi) / k
    dist = np.hypot(cx, cy)
    rad = 1.0 / np.abs(k)
    p0x = cx * (1.0 - rad / dist)
    p0y = cy * (1.0 - rad / dist)
    phi0 = np.mod(np.arctan2(k * (p0x - cx), -k * (p0y - cy)), TWO_PI)
    d0 = -p0x * np.sin(phi0) + p0y * np.cos(phi0)
    return d0, phi0


def track_hits(d0, phi0, kappa, radii=LAYERS_CM):
    """Noise-free hits of tracks given by their parameters at closest approach.

    Returns (x, y, ok) fp64 of shape (n_tracks, n_layers); the tracks start at
    P0 and move forward along (cos phi0, sin phi0).
    """
    d0 = np.atleast_1d(np.asarray(d0, dtype=np.float64))[:, None]
    phi0 = np.atleast_1d(np.asarray(phi0, dtype=np.float64))[:, None]
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))[:, None]
    radii = np.asarray(radii, dtype=np.float64)[None, :]
    sx = -d0 * np.sin(phi0)
    sy = d0 * np.cos(phi0)
    return _first_crossing(sx, sy, phi0, kappa, radii)


def _smear(x, y, rng, sigma):
    r = np.hypot(x, y)
    dphi = rng.normal(0.0, sigma, size=x.shape) / r
    c, s = np.cos(dphi), np.sin(dphi)
    return x * c - y * s, x * s + y * c


def _noise(n, rng, radii=LAYERS_CM):
    layer = rng.integers(0, len(radii), size=n)
    phi = rng.uniform(0.0, TWO_PI, size=n)
    r = radii[layer]
    return r * np.cos(phi), r * np.sin(phi)


def sample_pt_lognormal(rng, n, median=0.8, sigma_ln=0.6, lo=0.5, hi=50.0):
    """Lognormal pT truncated to [lo, hi] by resampling (not clamping)."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        v = np.exp(rng.normal(math.log(median), sigma_ln, size=2 * (n - filled) + 16))
        v = v[(v >= lo) & (v <= hi)]
        take = min(len(v), n - filled)
        out[filled:filled + take] = v[:take]
        filled += take
    return out


def sample_track_count(rng, lo=200, hi=8000):
    """Track count lognormal centred on sqrt(lo*hi), sigma ln(hi/lo)/4, resampled into [lo, hi]."""
    mu = 0.5 * (math.log(lo) + math.log(hi))
    sig = math.log(hi / lo) / 4.0
    while True:
        n = int(round(math.exp(rng.normal(mu, sig))))
        if lo <= n <= hi:
            return n


def _assemble(parts_x, parts_y, parts_lab, rng, truth, kind, n_noise=None, noise_to=None):
    x = np.concatenate(parts_x) if parts_x else np.zeros(0)
    y = np.concatenate(parts_y) if parts_y else np.zeros(0)
    lab = np.concatenate(parts_lab) if parts_lab else np.zeros(0, dtype=np.int32)
    if noise_to is not None:
        if x.shape[0] > noise_to:
            keep = np.sort(rng.permutation(x.shape[0])[:noise_to])
            x, y, lab = x[keep], y[keep], lab[keep]
        n_noise = noise_to - x.shape[0]
    if n_noise:
        nx, ny = _noise(n_noise, rng)
        x = np.concatenate([x, nx])
        y = np.concatenate([y, ny])
        lab = np.concatenate([lab, np.full(n_noise, -1, dtype=np.int32)])
    perm = rng.permutation(x.shape[0])
    d0, phi0, kappa = truth
    return Event(x=x[perm].astype(np.float32), y=y[perm].astype(np.float32),
                 label=lab[perm].astype(np.int32), d0=d0, phi0=phi0, kappa=kappa, kind=kind)


def _prompt_hits(rng, n_tracks, pt, smear):
    q = rng.choice([-1.0, 1.0], size=n_tracks)
    phi0 = rng.uniform(0.0, TWO_PI, size=n_tracks)
    kappa = kappa_from_pt(pt, q)
    hx, hy, ok = track_hits(np.zeros(n_tracks), phi0, kappa)
    if smear:
        hx, hy = _smear(hx, hy, rng, SMEAR_RPHI_CM)
    lab = np.broadcast_to(np.arange(n_tracks, dtype=np.int32)[:, None], ok.shape)
    return hx[ok], hy[ok], lab[ok], (np.zeros(n_tracks), phi0, kappa)


def gen_tracks_event(d0, phi0, kappa, *, radii=LAYERS_CM, smear=0.0, rng=None, kind="2d"):
    """An event made of given tracks only (no noise), hits in track order."""
    hx, hy, ok = track_hits(d0, phi0, kappa, radii)
    if smear:
        hx, hy = _smear(hx, hy, rng, smear)
    lab = np.broadcast_to(np.arange(hx.shape[0], dtype=np.int32)[:, None], ok.shape)
    return Event(x=hx[ok].astype(np.float32), y=hy[ok].astype(np.float32),
                 label=lab[ok].astype(np.int32), d0=np.atleast_1d(np.asarray(d0, float)),
                 phi0=np.atleast_1d(np.asarray(phi0, float)),
                 kappa=np.atleast_1d(np.asarray(kappa, float)), kind=kind)


def gen_prompt_event(rng, n_tracks, pt_sampler, noise_frac, smear=True):
    pt = pt_sampler(rng, n_tracks)
    hx, hy, lab, truth = _prompt_hits(rng, n_tracks, pt, smear)
    n_noise = int(round(noise_frac * hx.shape[0]))
    return _assemble([hx], [hy], [lab], rng, truth, "2d", n_noise=n_noise)


def gen_displaced_event(rng, n_prompt=3000, n_vertices=20, tracks_per_vertex=10,
                        lxy_max=30.0, cone=0.3, total_hits=35000):
    """Prompt tracks plus tracks from displaced vertices, padded with noise.

    Vertex tracks start at the vertex, point along its azimuth within +-cone
    and leave hits only on layers outside the vertex radius.
    """
    pt = sample_pt_lognormal(rng, n_prompt)
    px, py, plab, (pd0, pphi, pk) = _prompt_hits(rng, n_prompt, pt, smear=True)
    n_disp = n_vertices * tracks_per_vertex
    lxy = rng.uniform(0.0, lxy_max, size=n_vertices)
    alpha = rng.uniform(0.0, TWO_PI, size=n_vertices)
    vx = np.repeat(lxy * np.cos(alpha), tracks_per_vertex)
    vy = np.repeat(lxy * np.sin(alpha), tracks_per_vertex)
    vr = np.repeat(lxy, tracks_per_vertex)
    psi = np.repeat(alpha, tracks_per_vertex) + rng.uniform(-cone, cone, size=n_disp)
    q = rng.choice([-1.0, 1.0], size=n_disp)
    k = kappa_from_pt(sample_pt_lognormal(rng, n_disp), q)
    hx, hy, ok = _first_crossing(vx[:, None], vy[:, None], psi[:, None], k[:, None],
                                 LAYERS_CM[None, :])
    ok &= LAYERS_CM[None, :] > vr[:, None]
    hx, hy = _smear(np.where(ok, hx, 1.0), np.where(ok, hy, 0.0), rng, SMEAR_RPHI_CM)
    lab = np.broadcast_to(np.arange(n_prompt, n_prompt + n_disp, dtype=np.int32)[:, None], ok.shape)
    dd0, dphi = closest_approach(vx, vy, psi, k)
    truth = (np.concatenate([pd0, dd0]), np.concatenate([pphi, dphi]), np.concatenate([pk, k]))
    return _assemble([px, hx[ok]], [py, hy[ok]], [plab, lab[ok]], rng, truth, "3d",
                     noise_to=total_hits)


def straight_hits(d0, phi0, radii=LAYERS_CM):
    """Noise-free hits of straight lines (the kappa = 0 family) given by d0 and
    phi0 at closest approach: the forward crossing P0 + t (cos phi0, sin phi0),
    t = sqrt(r^2 - d0^2), of every layer with r > |d0|.  (x, y, ok) fp64."""
    d0 = np.asarray(d0, np.float64)[:, None]
    phi0 = np.asarray(phi0, np.float64)[:, None]
    r = np.asarray(radii, np.float64)[None, :]
    ok = r > np.abs(d0)
    t = np.sqrt(np.where(ok, r * r - d0 * d0, 0.0))
    x = -d0 * np.sin(phi0) + t * np.cos(phi0)
    y = d0 * np.cos(phi0) + t * np.sin(phi0)
    ok = np.broadcast_to(ok, x.shape)
    return x, y, ok


def gen_straight_event(rng, n_tracks=2000, d0_max=25.0, noise_frac=0.2, smear=True):
    """Straight displaced tracks (d0 uniform in [-d0_max, d0_max], phi0 uniform)
    with r-phi smearing and a fraction of noise hits."""
    d0 = rng.uniform(-d0_max, d0_max, size=n_tracks)
    phi0 = rng.uniform(0.0, TWO_PI, size=n_tracks)
    hx, hy, ok = straight_hits(d0, phi0)
    if smear:
        hx, hy = _smear(hx, hy, rng, SMEAR_RPHI_CM)
    lab = np.broadcast_to(np.arange(n_tracks, dtype=np.int32)[:, None], ok.shape)
    hx, hy, lab = hx[ok], hy[ok], lab[ok]
    n_noise = int(round(noise_frac * hx.shape[0]))
    return _assemble([hx], [hy], [lab], rng, (d0, phi0, np.zeros(n_tracks)), "straight", n_noise=n_noise)


def _pt_uniform_1_20(rng, n):
    return rng.uniform(1.0, 20.0, size=n)


def gen_config_event(cfg: int, event_index: int = 0, *, seed: int = BASE_SEED):
    """Event ``event_index`` of workload ``cfg`` (1..5), reproducible from the seed.

    1: 40 prompt tracks, pT U[1, 20] GeV, 20 % noise.
    2: 5,000 prompt tracks, lognormal pT, 30 % noise.
    3: 3,000 prompt + 20 vertices x 10 displaced tracks, noise to 35,000 hits.
    4: prompt, track count lognormal in [200, 8000], 30 % noise.
    5: a stream event: 80 % workload-4 style, 20 % workload-3 style.
    6: 2,000 straight tracks, |d0| <= 25 cm, 20 % noise (the kappa = 0 family).
    """
    ss = np.random.SeedSequence(seed + cfg, spawn_key=(event_index,))
    rng = np.random.default_rng(ss)
    if cfg == 1:
        return gen_prompt_event(rng, 40, _pt_uniform_1_20, 0.2)
    if cfg == 2:
        return gen_prompt_event(rng, 5000, sample_pt_lognormal, 0.3)
    if cfg == 3:
        return gen_displaced_event(rng)
    if cfg == 4:
        return gen_prompt_event(rng, sample_track_count(rng), sample_pt_lognormal, 0.3)
    if cfg == 5:
        if rng.uniform() < 0.2:
            return gen_displaced_event(rng)
        return gen_prompt_event(rng, sample_track_count(rng), sample_pt_lognormal, 0.3)
    if cfg == 6:
        return gen_straight_event(rng)
    raise ValueError(f"unknown workload {cfg}")


def pack_events(events) -> Batch:
    off = np.zeros(len(events) + 1, dtype=np.int64)
    off[1:] = np.cumsum([e.n_hits for e in events])
    x = np.concatenate([e.x for e in events]) if events else np.zeros(0, np.float32)
    y = np.concatenate([e.y for e in events]) if events else np.zeros(0, np.float32)
    return Batch(x=x.astype(np.float32), y=y.astype(np.float32), hit_off=off, events=list(events))


def gen_batch(cfg: int = 4, n_events: int = 256, *, seed: int = BASE_SEED, first: int = 0) -> Batch:
    return pack_events([gen_config_event(cfg, first + i, seed=seed) for i in range(n_events)])


def poisson_arrivals(rate_hz: float, n: int, *, seed: int = BASE_SEED + 5, stream: int = 0):
    """Open-loop arrival times (seconds) with exponential gaps."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, stream, int(rate_hz)]))
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
