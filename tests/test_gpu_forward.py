"""GPU parity of the forward-hemisphere option (a hit votes only for phi0 with
x cos(phi0) + y sin(phi0) > 0).

With the option the culling keeps each hit's forward arc only and the vote
tests the binary32 condition per row; every accumulator and candidate list
must equal the oracle's run with the same option.
"""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth

hough = pytest.importorskip("paper_1311_2769_amd.hough")

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _fwd(g):
    return dataclasses.replace(g, forward=True)


def _ref(x, y, grid, threshold):
    if grid.family == "straight":
        return oracle.find_straight(x, y, grid, threshold)
    return oracle.find(x, y, grid, threshold)


def _single(ctx, x, y, threshold):
    acc, nv = ctx.vote(_t(x), _t(y))
    out, nf = ctx.peaks(acc, threshold)
    torch.cuda.synchronize()
    v, c, n = hough.cands_to_numpy(out, nf.item())
    return hough.acc_to_numpy(acc, ctx.spec), int(nv.item()), v, c, n


def _assert_same(got, ref, what):
    acc, nv, v, c, n = got
    racc, rnv, rv, rc, rn = ref
    np.testing.assert_array_equal(acc.reshape(racc.shape), racc, err_msg=what)
    assert nv == rnv, what
    assert n == rn, what
    np.testing.assert_array_equal(c, rc, err_msg=what)
    np.testing.assert_array_equal(v, rv, err_msg=what)


@pytest.mark.parametrize("cfg", [1, 2, 3, 6])
def test_forward_event_matches_oracle(cfg):
    wc = synth.CONFIGS[cfg]
    grid = _fwd(wc.grid)
    ev = synth.gen_config_event(cfg, 1)
    ref = _ref(ev.x, ev.y, grid, wc.threshold)
    print(f"[forward] config {cfg}: {ev.n_hits} hits, {ref[1]} votes, {ref[4]} candidates", flush=True)
    ctx = hough.HoughContext(grid, device=_dev(), max_hits=ev.n_hits)
    _assert_same(_single(ctx, ev.x, ev.y, wc.threshold), ref, f"config {cfg}")


@pytest.mark.parametrize("cfg", [4, 6])
def test_forward_batch_matches_oracle_per_event(cfg):
    """The fused batch path (2D int32) with the option, event by event."""
    wc = synth.CONFIGS[cfg]
    grid = _fwd(wc.grid)
    events = [synth.gen_config_event(cfg, i) for i in range(5)]
    b = synth.pack_events(events)
    ctx = hough.HoughContext(grid, device=_dev(), max_events=len(events), max_hits=b.n_hits)
    cands, cand_off, n_found, n_votes = ctx.event_batch(b.hit_off, _t(b.x), _t(b.y), wc.threshold)
    torch.cuda.synchronize()
    cands, n_found, n_votes = cands.cpu().numpy(), n_found.cpu().numpy(), n_votes.cpu().numpy()
    for e, ev in enumerate(events):
        _, rnv, rv, rc, rn = _ref(ev.x, ev.y, grid, wc.threshold)
        print(f"[forward] batch {cfg} event {e}: {rnv} votes, {rn} candidates", flush=True)
        assert int(n_votes[e]) == rnv and int(n_found[e]) == rn
        m = min(rn, int(cand_off[e + 1] - cand_off[e]))
        got = cands[cand_off[e]:cand_off[e] + m]
        np.testing.assert_array_equal(got[:, 0], rv[:m])
        np.testing.assert_array_equal(got[:, 1], rc[:m])


@pytest.mark.parametrize("which", ["2d", "3d", "straight"])
def test_forward_culling_stress(which):
    """Hits at every radius (including those whose sine interval reaches +-1, where the
    forward arc is a half circle), at angles near the row centres and near the
    abreast directions phi0 +- pi/2 of the rows."""
    grid = {"2d": synth.make_grid(512, 64), "3d": synth.make_grid(128, 32, n_d0=8, d0_range=(-6.0, 6.0)),
            "straight": synth.make_straight_grid(512, 64, (-4.0, 4.0))}[which]
    grid = _fwd(grid)
    rng = np.random.default_rng({"2d": 1, "3d": 2, "straight": 3}[which])
    n = 6000
    r = np.concatenate([rng.uniform(0.05, 130.0, n // 2), np.abs(rng.normal(0.0, 2.0, n // 2)) + 1e-3])
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    # a third of the hits sit exactly (in fp64) abreast of a row centre
    j = rng.integers(0, grid.n_phi, n // 3)
    ph[: n // 3] = grid.phi_centre(j) + np.where(rng.uniform(size=n // 3) < 0.5, 0.5, -0.5) * np.pi
    x, y = (r * np.cos(ph)).astype(np.float32), (r * np.sin(ph)).astype(np.float32)
    ref = _ref(x, y, grid, 2)
    ctx = hough.HoughContext(grid, device=_dev(), max_hits=n)
    print(f"[forward] stress {which}: {ref[1]} votes, {ref[4]} candidates", flush=True)
    _assert_same(_single(ctx, x, y, 2), ref, f"stress {which}")


def test_forward_strict_hand_case_without_culling():
    """A table that is not of bin centres (culling off): rows with x c + y s equal to 0,
    1e-30, -1e-30 and 1 for the hit (1, 0); only the positive ones vote."""
    c = np.array([0.0, 1e-30, -1e-30, 1.0], np.float32)
    s = np.array([1.0, 1.0, 1.0, 0.0], np.float32)
    base = synth.make_grid(4, 16, kappa_half_range_inv_cm=0.05)
    g = _fwd(dataclasses.replace(base, cos_phi=c, sin_phi=s))
    ref = oracle.find(np.array([1.0], np.float32), np.array([0.0], np.float32), g, 1)
    assert ref[0][0].sum(axis=1).tolist() == [0, 1, 0, 1]
    ctx = hough.HoughContext(g, device=_dev())
    _assert_same(_single(ctx, np.array([1.0], np.float32), np.array([0.0], np.float32), 1), ref, "strict")



@pytest.mark.parametrize("shape,acc", [((100, 48), "u16"), ((4096, 64), "i32"), ((2048, 40), "u16")])
def test_forward_tile_ranges_and_u16(shape, acc):
    """Forward grids whose slices have more than 63 tiles (culling by tile ranges
    instead of masks), a partial last tile, and uint16 cells."""
    grid = _fwd(synth.make_grid(*shape, acc_type=acc))
    ev = synth.gen_config_event(1, 4)
    ref = _ref(ev.x, ev.y, grid, 3)
    ctx = hough.HoughContext(grid, device=_dev(), max_hits=ev.n_hits)
    print(f"[forward] grid {shape} {acc}: {ref[1]} votes, {ref[4]} candidates", flush=True)
    _assert_same(_single(ctx, ev.x, ev.y, 3), ref, f"grid {shape} {acc}")
