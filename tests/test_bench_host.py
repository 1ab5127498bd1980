"""Host logic of bench.py: the kernel digest that decides whether the
committed counter summary still describes the vote kernel."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _sources():
    out = {}
    for name in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1311_2769_amd", "csrc", name)) as f:
            out[name] = f.read()
    return out


def test_code_text_drops_comments_and_blank_lines():
    src = "int a; // one\n\n/* two\n   lines */ int b;\n  // three\nint c;  \n"
    assert bench.code_text(src) == "int a;\n int b;\nint c;"


def test_digest_ignores_comment_edits_only():
    src = _sources()
    base = bench.kernel_digest(src.__getitem__)
    assert base == bench.kernel_digest()
    commented = dict(src)
    commented["vote.hip"] = "// a note\n" + src["vote.hip"].replace("\n", "  // x\n", 3)
    assert bench.kernel_digest(commented.__getitem__) == base
    changed = dict(src)
    changed["vote_math.h"] = src["vote_math.h"] + "\nstatic const int kProbe = 1;\n"
    assert bench.kernel_digest(changed.__getitem__) != base
    swapped = dict(src)
    swapped["peak_tile.h"], swapped["hough_impl.h"] = src["hough_impl.h"], src["peak_tile.h"]
    assert bench.kernel_digest(swapped.__getitem__) != base


def test_committed_counters_match_the_sources():
    # both launch shapes the tuner may pick carry traffic and VALU counts
    for rows, threads in ((64, 1024), (32, 512)):
        traffic, valu = bench.counter_fields(rows, threads)
        assert traffic is not None and traffic > 0
        assert valu is not None and valu > 0
