"""Truth matching of track candidates (a physics report, not part of the method).

The generators label every hit with the track that made it (-1 for noise).
Given the hit association of a candidate list -- (candidate, hit) pairs, as
the library's ``hough_associate`` and the oracle's ``associate`` return them
-- these helpers count, with the labels alone:

* a candidate matches track t when t contributes the most of its hits and
  at least ``min_hits`` of them (noise never matches): the peak was made by
  that track, whatever other hits fall into its window;
* a track is findable when it left at least ``min_hits`` hits;
* efficiency = findable tracks with a matching candidate / findable tracks;
* fake rate  = candidates with hits but no match / candidates with hits;
* duplicates = matching candidates per found track (the full grids count a
  track's mirror peak too, so about 2 there and 1 with the forward option).

Nothing here computes a vote or a bin.
"""

from __future__ import annotations

import numpy as np


def match_candidates(pair_cand, pair_hit, n_cands: int, labels, min_hits: int):
    """Per candidate: the matched track label, or -1; and its number of hits.
    Ties between tracks go to the smaller label."""
    pair_cand = np.asarray(pair_cand, np.int64)
    lab = np.asarray(labels, np.int64)[np.asarray(pair_hit, np.int64)]
    n_hits = np.bincount(pair_cand, minlength=n_cands)[:n_cands]
    match = np.full(n_cands, -1, np.int64)
    if pair_cand.size == 0:
        return match, n_hits
    order = np.lexsort((lab, pair_cand))
    pc, lb = pair_cand[order], lab[order]
    # runs of equal (candidate, label)
    edge = np.ones(pc.size, bool)
    edge[1:] = (pc[1:] != pc[:-1]) | (lb[1:] != lb[:-1])
    start = np.nonzero(edge)[0]
    count = np.diff(np.append(start, pc.size))
    rc, rl = pc[start], lb[start]
    keep = rl >= 0
    rc, rl, count = rc[keep], rl[keep], count[keep]
    # per candidate the largest count, the smaller label on ties
    order = np.lexsort((rl, -count, rc))
    rc, rl, count = rc[order], rl[order], count[order]
    first = np.ones(rc.size, bool)
    first[1:] = rc[1:] != rc[:-1]
    rc, rl, count = rc[first], rl[first], count[first]
    ok = count >= min_hits
    match[rc[ok]] = rl[ok]
    return match, n_hits


def efficiency(match, n_hits_per_cand, labels, min_hits: int) -> dict:
    """Efficiency, fake rate and duplicates of one event's matched candidates."""
    lab = np.asarray(labels, np.int64)
    tracks, hits = np.unique(lab[lab >= 0], return_counts=True)
    findable = set(tracks[hits >= min_hits].tolist())
    match = np.asarray(match, np.int64)
    has_hits = np.asarray(n_hits_per_cand) > 0
    found = findable & set(match[match >= 0].tolist())
    matched_to_found = np.isin(match, list(found)) if found else np.zeros(match.shape, bool)
    return {
        "findable_tracks": len(findable),
        "found_tracks": len(found),
        "efficiency": len(found) / len(findable) if findable else float("nan"),
        "candidates": int(has_hits.sum()),
        "fake_rate": float(((match < 0) & has_hits).sum() / has_hits.sum()) if has_hits.any() else float("nan"),
        "duplicates": float(matched_to_found.sum() / len(found)) if found else float("nan"),
    }
