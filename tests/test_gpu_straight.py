"""GPU parity of the straight-line family (the kappa = 0 tracks, phi0 x d0).

The library runs straight grids through the 2D vote path with hit records
that make its quotient the identity, and culls with arcs from the d0 range;
every accumulator and candidate list must equal the oracle's.
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


@pytest.mark.parametrize("index", [0, 1, 2])
def test_straight_event_matches_oracle(index):
    wc = synth.CONFIGS[6]
    ev = synth.gen_config_event(6, index)
    ref = oracle.find_straight(ev.x, ev.y, wc.grid, wc.threshold)
    ctx = hough.HoughContext(wc.grid, device=_dev(), max_hits=ev.n_hits)
    print(f"[straight] event {index}: {ev.n_hits} hits, {ref[1]} votes, {ref[4]} candidates", flush=True)
    _assert_same(_single(ctx, ev.x, ev.y, wc.threshold), ref, f"event {index}")


def test_straight_batch_matches_oracle_per_event():
    wc = synth.CONFIGS[6]
    events = [synth.gen_config_event(6, i) for i in range(6)]
    b = synth.pack_events(events)
    ctx = hough.HoughContext(wc.grid, device=_dev(), max_events=len(events), max_hits=b.n_hits)
    cands, cand_off, n_found, n_votes = ctx.event_batch(b.hit_off, _t(b.x), _t(b.y), wc.threshold)
    torch.cuda.synchronize()
    cands, n_found, n_votes = cands.cpu().numpy(), n_found.cpu().numpy(), n_votes.cpu().numpy()
    for e, ev in enumerate(events):
        _, rnv, rv, rc, rn = oracle.find_straight(ev.x, ev.y, wc.grid, wc.threshold)
        assert int(n_votes[e]) == rnv and int(n_found[e]) == rn
        m = min(rn, int(cand_off[e + 1] - cand_off[e]))
        got = cands[cand_off[e]:cand_off[e] + m]
        np.testing.assert_array_equal(got[:, 0], rv[:m])
        np.testing.assert_array_equal(got[:, 1], rc[:m])


@pytest.mark.parametrize("d0_range", [(-2.0, 2.0), (3.0, 9.0), (-40.0, -0.5), (-0.01, 0.01)])
def test_straight_culling_stress(d0_range):
    """Narrow and one-sided d0 ranges make tight culling arcs; hits at every radius,
    some exactly on the range edges."""
    grid = synth.make_straight_grid(512, 64, d0_range)
    rng = np.random.default_rng(int(1000 * abs(d0_range[0]) + 7))
    n = 20000
    r = np.concatenate([rng.uniform(0.02, 120.0, n // 2), np.abs(rng.normal(0.0, 3.0, n // 2)) + 1e-3])
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    x, y = (r * np.cos(ph)).astype(np.float32), (r * np.sin(ph)).astype(np.float32)
    # hits whose u equals a range edge at the phi0 = 0 direction's neighbourhood
    x[:64], y[:64] = 0.0, np.float32(d0_range[0])
    x[64:128], y[64:128] = 0.0, np.float32(d0_range[1])
    ref = oracle.find_straight(x, y, grid, 3)
    ctx = hough.HoughContext(grid, device=_dev(), max_hits=n)
    _assert_same(_single(ctx, x, y, 3), ref, f"d0 range {d0_range}")


def test_straight_non_centre_table_and_u16():
    """A phi0 table that is not of bin centres turns culling off; uint16 cells."""
    g = synth.make_straight_grid(300, 40, (-10.0, 10.0), acc_type="u16")
    phi = np.linspace(0.1, 6.0, 300)
    g = dataclasses.replace(g, cos_phi=np.cos(phi).astype(np.float32), sin_phi=np.sin(phi).astype(np.float32))
    ev = synth.gen_config_event(6, 4)
    ref = oracle.find_straight(ev.x, ev.y, g, 5)
    ctx = hough.HoughContext(g, device=_dev(), max_hits=ev.n_hits)
    _assert_same(_single(ctx, ev.x, ev.y, 5), ref, "non-centre table, u16")
