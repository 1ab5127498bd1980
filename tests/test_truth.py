"""Host logic of the truth report (synth.truth): hand-made pairs and labels."""

import numpy as np

import synth


def test_majority_track_with_enough_hits_matches():
    labels = np.array([0, 0, 0, 1, 1, -1, -1, -1, 2, 2])
    # candidate 0: hits of track 0 (3) and one of track 1 -> track 0
    # candidate 1: two of track 1 and three noise hits -> track 1 (noise never matches)
    # candidate 2: one hit each of tracks 0, 1, 2 -> tie of counts 1 < min_hits 2 -> none
    # candidate 3: no hits
    # candidate 4: two of track 2, two of track 1 -> tie: the smaller label, track 1
    pairs = [(0, 0), (0, 1), (0, 2), (0, 3),
             (1, 3), (1, 4), (1, 5), (1, 6), (1, 7),
             (2, 0), (2, 3), (2, 8),
             (4, 8), (4, 9), (4, 3), (4, 4)]
    pc = np.array([p[0] for p in pairs])
    ph = np.array([p[1] for p in pairs])
    match, n_hits = synth.match_candidates(pc, ph, 5, labels, 2)
    assert match.tolist() == [0, 1, -1, -1, 1]
    assert n_hits.tolist() == [4, 5, 3, 0, 4]
    rep = synth.efficiency(match, n_hits, labels, 2)
    # findable: tracks 0 (3 hits), 1 (2), 2 (2); found: 0 and 1
    assert rep["findable_tracks"] == 3 and rep["found_tracks"] == 2
    assert abs(rep["efficiency"] - 2 / 3) < 1e-12
    # candidates with hits: 0, 1, 2, 4; unmatched among them: 2
    assert rep["candidates"] == 4 and abs(rep["fake_rate"] - 0.25) < 1e-12
    # matched to found tracks: 0, 1, 4 -> 3 over 2 found tracks
    assert abs(rep["duplicates"] - 1.5) < 1e-12


def test_findable_needs_min_hits_and_empty_inputs():
    labels = np.array([0, 1, 1, 1])
    match, n_hits = synth.match_candidates(np.array([0, 0, 0]), np.array([1, 2, 3]), 2, labels, 3)
    assert match.tolist() == [1, -1]
    rep = synth.efficiency(match, n_hits, labels, 3)
    assert rep["findable_tracks"] == 1 and rep["efficiency"] == 1.0 and rep["fake_rate"] == 0.0
    match, n_hits = synth.match_candidates(np.array([], np.int64), np.array([], np.int64), 3, labels, 1)
    assert match.tolist() == [-1, -1, -1] and n_hits.tolist() == [0, 0, 0]
    rep = synth.efficiency(match, n_hits, labels, 1)
    assert rep["found_tracks"] == 0 and rep["efficiency"] == 0.0 and rep["candidates"] == 0
