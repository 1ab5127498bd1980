"""The device on the votes whose bin depends on the binary32 operation order.

tests/golden/fp32_order.json holds (hit, row) pairs of the workload grids
where a reordered or contracted evaluation of the vote, a division through a
reciprocal or binary64 arithmetic selects another bin than the canonical
sequence (one binary32 rounding per operation, no contraction), with the bin
derived in exact rational arithmetic.  Such pairs sit within a few units in
the last place of a bin edge, exactly where the device's approximate bins must
fall back to the exact quotient.  Each case votes alone, through the single
event path, the batched vote and the fused batch; the fixture's row must hold
its bin, and the whole accumulator must equal the oracle's.
"""

import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1311_2769_amd import hough  # noqa: E402

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "fp32_order.json")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _hx(s):
    return np.float32(float.fromhex(s))


def _doc():
    with open(FIXTURE) as f:
        return json.load(f)


def _curved_grid(case):
    if case["grid"] == "pileup_2d_1024x512":
        return synth.GRID_2D
    if case["l"] is None:     # a d0 off the grid's centres: a one-slice grid holding it
        return dataclasses.replace(synth.GRID_3D, n_d0=1, d0=np.array([_hx(case["d0"])], np.float32))
    return synth.GRID_3D


def _straight_grid(case):
    if case["grid"] == "straight_1024x512":
        return synth.GRID_STRAIGHT
    return synth.make_straight_grid(1024, 512, d0_range=(-30.0, 30.0))


def _groups(cases, grid_of):
    groups = {}
    for i, c in enumerate(cases):
        g = grid_of(c)
        key = (c["grid"], None if g.d0 is None else g.d0.tobytes())
        groups.setdefault(key, (g, []))[1].append(i)
    return groups.values()


def _check_rows(acc, cases, idx, ref_one, what):
    for e, i in enumerate(idx):
        c = cases[i]
        l = c.get("l") or 0
        row = acc[e][l, c["j"]]
        nz = np.flatnonzero(row)
        got = int(nz[0]) if len(nz) else None
        assert len(nz) <= 1 and got == c["bin"], f"{what}: case {i} votes {got}, exact {c['bin']}"
        np.testing.assert_array_equal(acc[e].reshape(-1), ref_one(i).reshape(-1), err_msg=f"{what}: case {i}")


@pytest.mark.parametrize("family", ["curved", "straight"])
def test_order_sensitive_votes_single_and_batched(family):
    doc = _doc()
    cases = doc[family]
    grid_of = _curved_grid if family == "curved" else _straight_grid
    for grid, idx in _groups(cases, grid_of):
        print(f"[fp32-order] {family} {len(idx)} cases on {grid.shape}", flush=True)
        xs = np.array([_hx(cases[i]["x"]) for i in idx], np.float32)
        ys = np.array([_hx(cases[i]["y"]) for i in idx], np.float32)
        vote1 = oracle.vote if family == "curved" else oracle.vote_straight

        def ref_one(i, grid=grid):
            return vote1([_hx(cases[i]["x"])], [_hx(cases[i]["y"])], grid)[0]

        ctx = hough.HoughContext(grid, max_events=len(idx), max_hits=len(idx))
        single = []
        for e in range(len(idx)):
            acc, _ = ctx.vote(_t(xs[e:e + 1]), _t(ys[e:e + 1]))
            single.append(hough.acc_to_numpy(acc, ctx.spec).copy())
        torch.cuda.synchronize()
        _check_rows(single, cases, idx, ref_one, f"{family} single event")

        hit_off = np.arange(len(idx) + 1, dtype=np.int64)
        acc, _ = ctx.vote_batch(hit_off, _t(xs), _t(ys))
        torch.cuda.synchronize()
        accs = [hough.acc_to_numpy(acc[e], ctx.spec) for e in range(len(idx))]
        _check_rows(accs, cases, idx, ref_one, f"{family} batched vote")

        if grid.d0 is None:      # the fused vote + peak batch writes accumulators on request
            acc_b = ctx.new_acc(len(idx))
            ctx.event_batch(hit_off, _t(xs), _t(ys), 1, acc=acc_b)
            torch.cuda.synchronize()
            accs = [hough.acc_to_numpy(acc_b[e], ctx.spec) for e in range(len(idx))]
            _check_rows(accs, cases, idx, ref_one, f"{family} fused batch")


@pytest.mark.parametrize("family", ["curved", "straight"])
def test_order_sensitive_association(family):
    """Candidates one bin below and one above each case's bin: the hit belongs
    to both on the device, as in the oracle."""
    doc = _doc()
    cases = doc[family]
    grid_of = _curved_grid if family == "curved" else _straight_grid
    for i, c in enumerate(cases):
        grid = grid_of(c)
        l = c.get("l") or 0
        base = (l * grid.n_phi + c["j"]) * grid.n_kappa
        cells = np.array([base + c["bin"] - 1, base + c["bin"] + 1], np.int64)
        x, y = np.array([_hx(c["x"])], np.float32), np.array([_hx(c["y"])], np.float32)
        rc, rh = oracle.associate(x, y, grid, [9, 9], cells, 1)
        assert list(rc) == [0, 1] and list(rh) == [0, 0]
        ctx = hough.HoughContext(grid, max_hits=1)
        cands = torch.from_numpy(np.stack([np.full(2, 9, np.int32), cells.astype(np.int32)], 1).copy()).to(_dev())
        ncand = torch.tensor([2], dtype=torch.int32, device=_dev())
        pairs, n_pairs = ctx.associate(_t(x), _t(y), cands, ncand, 1, cap=8)
        torch.cuda.synchronize()
        n = int(n_pairs.item())
        got = sorted(map(tuple, pairs[:n].cpu().numpy().tolist()))
        assert got == [(0, 0), (1, 0)], f"{family} case {i}: pairs {got}"


def test_order_sensitive_vertex_votes():
    """One line per case (a candidate of a track grid whose row 0 holds the
    case's d0, cos and sin) votes into the whole vertex grid; the case's column
    (or row) holds its bin, and the vertex accumulator equals the oracle's."""
    doc = _doc()
    for i, c in enumerate(doc["vertex"]):
        vg = synth.VERTEX_GRID if c["grid"] == "vertex_128x128" else synth.make_vertex_grid(100, 100)
        tgrid = dataclasses.replace(
            synth.GRID_3D, n_d0=1, n_phi=3, n_kappa=2, acc_type="i32",
            cos_phi=np.array([_hx(c["cos"]), 1.0, 0.0], np.float32),
            sin_phi=np.array([_hx(c["sin"]), 0.0, 1.0], np.float32),
            d0=np.array([_hx(c["d0"])], np.float32))
        rv, _ = oracle.vertex_vote([10], [0], 1, tgrid, vg)
        line = rv[c["centre_index"], :] if c["mode"] == "column" else rv[:, c["centre_index"]]
        assert int(np.flatnonzero(line)[0]) == c["bin"]
        ctx = hough.HoughContext(tgrid, max_hits=1)
        cands = torch.tensor([[10, 0]], dtype=torch.int32, device=_dev())
        nf = torch.tensor([1], dtype=torch.int32, device=_dev())
        _, _, _, vacc = ctx.vertices(vg, cands, np.array([0, 1], np.int64), nf, 1, 1, want_acc=True)
        torch.cuda.synchronize()
        got = vacc[0].cpu().numpy()
        np.testing.assert_array_equal(got, rv, err_msg=f"vertex case {i} ({c['mode']})")
