"""Launch-shape cache of the autotuner: host-only lookups through the C ABI."""

import json

import pytest

import synth
from paper_1311_2769_amd import hough

DEV = "gfx950/256"


def _line(grid, which, hits_log2, rows, threads, split=1, acc="i32", device=DEV, ms=1.0):
    return json.dumps({"device": device, "grid": list(grid.shape), "acc": acc, "which": which,
                       "hits_log2": hits_log2, "rows": rows, "threads": threads, "split": split, "ms": ms}) + "\n"


def test_lookup_picks_nearest_bucket_and_last_line(tmp_path):
    g = synth.GRID_2D
    path = tmp_path / "tune.jsonl"
    path.write_text(
        _line(g, 1, 20, 64, 256) +
        _line(g, 1, 23, 64, 1024) +
        "not json at all\n" +
        '{"device": "gfx950/256", "grid": [1, 1024], "acc": "i32"}\n' +        # malformed: ignored
        _line(g, 1, 23, 32, 512) +                                              # same key, later: wins
        _line(g, 0, 16, 32, 512, split=4) +
        _line(g, 1, 23, 128, 1024, device="gfx942/304") +                      # other device
        _line(synth.GRID_3D, 1, 23, 128, 256, acc="u16"))
    assert hough.tune_lookup(str(path), DEV, g, 1, 1 << 23) == (32, 512, 1)
    assert hough.tune_lookup(str(path), DEV, g, 1, 5_000_000) == (32, 512, 1)    # ceil(log2) = 23
    assert hough.tune_lookup(str(path), DEV, g, 1, 1 << 19) == (64, 256, 1)      # nearest: 20
    assert hough.tune_lookup(str(path), DEV, g, 0, 64_000) == (32, 512, 4)
    assert hough.tune_lookup(str(path), "gfx942/304", g, 1, 1 << 23) == (128, 1024, 1)
    assert hough.tune_lookup(str(path), DEV, synth.GRID_3D, 1, 1 << 10) == (128, 256, 1)
    assert hough.tune_lookup(str(path), DEV, synth.GRID_2D_SMALL, 1, 1 << 23) is None
    assert hough.tune_lookup(str(path), DEV, synth.GRID_3D, 0, 1 << 10) is None


def test_lookup_missing_file_and_env_fallback(tmp_path, monkeypatch):
    g = synth.GRID_2D
    assert hough.tune_lookup(str(tmp_path / "absent.jsonl"), DEV, g, 1, 100) is None
    path = tmp_path / "env.jsonl"
    path.write_text(_line(g, 1, 7, 64, 512))
    monkeypatch.setenv("HOUGH_TUNE_CACHE", str(path))
    assert hough.tune_lookup(None, DEV, g, 1, 100) == (64, 512, 1)
    monkeypatch.delenv("HOUGH_TUNE_CACHE")
    assert hough.tune_lookup(None, DEV, g, 1, 100) is None


def test_lookup_rejects_bad_arguments():
    with pytest.raises(hough.HoughError):
        hough.tune_lookup(None, DEV, synth.GRID_2D, 2, 100)
    with pytest.raises(hough.HoughError):
        hough.tune_lookup(None, DEV, synth.GRID_2D, 1, -1)
