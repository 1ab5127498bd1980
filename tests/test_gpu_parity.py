"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integers all the way: accumulators, vote counts and candidate lists must be
bit-exact, at every launch shape, for single events and for batches.
"""

import ctypes
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from synth.grids import Grid, make_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1311_2769_amd import hough  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


_ORACLE_CACHE = {}


def _oracle(key, x, y, grid, thr):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.find(x, y, grid, thr)
    return _ORACLE_CACHE[key]


def _oracle_many(events, grid, thr, workers=8):
    """oracle.find of every event, several at a time (the oracle's C calls release
    the interpreter lock; each call stays single-threaded)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as pool:
        return list(pool.map(lambda ev: oracle.find(ev.x, ev.y, grid, thr), events))


def _gpu_find(ctx, x, y, thr, cap=None):
    acc, nv = ctx.vote(_t(x), _t(y))
    out, nf = ctx.peaks(acc, thr, cap)
    torch.cuda.synchronize()
    a = hough.acc_to_numpy(acc, ctx.spec)
    v, c, n = hough.cands_to_numpy(out, nf.item(), cap)
    return a, int(nv.item()), v, c, n


def _assert_same(gpu, ref, what):
    a, nv, v, c, n = gpu
    ra, rnv, rv, rc, rn = ref
    assert a.shape == ra.reshape(a.shape).shape
    np.testing.assert_array_equal(a.reshape(-1), ra.reshape(-1), err_msg=f"{what}: accumulator")
    assert nv == rnv, f"{what}: vote count"
    assert n == rn, f"{what}: n_found"
    np.testing.assert_array_equal(v, rv[:len(v)], err_msg=f"{what}: votes")
    np.testing.assert_array_equal(c, rc[:len(c)], err_msg=f"{what}: cells")


# --------------------------------------------------------------------------------------
# Single events at the workload sizes
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_workload_event_matches_oracle(cfg):
    print(f"[parity] workload {cfg}", flush=True)
    wc = synth.CONFIGS[cfg]
    ev = synth.gen_config_event(cfg)
    ref = _oracle(("cfg", cfg), ev.x, ev.y, wc.grid, wc.threshold)
    ctx = hough.HoughContext(wc.grid, max_hits=ev.n_hits)
    _assert_same(_gpu_find(ctx, ev.x, ev.y, wc.threshold), ref, f"workload {cfg}")


@pytest.mark.parametrize("shape", [(64, 256, 1), (64, 512, 4), (64, 1024, 2), (64, 512, 16), (64, 256, 64),
                                   (32, 256, 1), (32, 512, 4), (32, 1024, 8)])
def test_vote_launch_shapes_agree_2d(shape):
    print(f"[parity] 2D shape {shape}", flush=True)
    wc = synth.CONFIGS[2]
    ev = synth.gen_config_event(2)
    ref = _oracle(("cfg", 2), ev.x, ev.y, wc.grid, wc.threshold)
    ctx = hough.HoughContext(wc.grid, max_hits=ev.n_hits)
    ctx.set_launch(0, *shape)
    acc, nv = ctx.vote(_t(ev.x), _t(ev.y))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(hough.acc_to_numpy(acc, ctx.spec).reshape(-1), ref[0].reshape(-1))
    assert int(nv.item()) == ref[1]


@pytest.mark.parametrize("shape", [(64, 256, 1), (64, 512, 2), (128, 1024, 1), (128, 256, 3), (32, 512, 1),
                                   (32, 256, 2)])
def test_vote_launch_shapes_agree_3d(shape):
    print(f"[parity] 3D shape {shape}", flush=True)
    wc = synth.CONFIGS[3]
    ev = synth.gen_config_event(3)
    ref = _oracle(("cfg", 3), ev.x, ev.y, wc.grid, wc.threshold)
    ctx = hough.HoughContext(wc.grid, max_hits=ev.n_hits)
    ctx.set_launch(0, *shape)
    acc, nv = ctx.vote(_t(ev.x), _t(ev.y))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(hough.acc_to_numpy(acc, ctx.spec).reshape(-1), ref[0].reshape(-1))
    assert int(nv.item()) == ref[1]


# --------------------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------------------

def test_empty_event():
    ctx = hough.HoughContext(synth.GRID_2D_SMALL)
    x = torch.zeros(0, dtype=torch.float32, device=_dev())
    acc, nv = ctx.vote(x, x)
    out, nf = ctx.peaks(acc, 1)
    torch.cuda.synchronize()
    assert int(acc.abs().sum().item()) == 0 and int(nv.item()) == 0 and int(nf.item()) == 0


def test_nonfinite_origin_and_huge_hits():
    pts = np.array([[np.nan, 1], [1, np.nan], [np.inf, 2], [-np.inf, 0], [0, 0], [np.inf, np.inf],
                    [3e19, 1.0], [1e-30, 2e-30], [-1e-42, 1e-42], [4.0, 0.0], [0.0, -7.0]], np.float32)
    for grid in (synth.GRID_2D_SMALL, synth.GRID_3D):
        ref = oracle.find(pts[:, 0], pts[:, 1], grid, 1)
        ctx = hough.HoughContext(grid)
        _assert_same(_gpu_find(ctx, pts[:, 0], pts[:, 1], 1), ref, f"special hits {grid.shape}")


def test_kappa_min_zero_and_coarse_kappa_scale():
    """kappa_min = +0 (the zero-curvature bin edge: kappa = -0 must still vote
    bin 0) and kappa_scale < 1 (the vote's compare-form range test)."""
    import dataclasses
    ev = synth.gen_config_event(1)
    # hits on the axes give u = +-0 exactly at phi0 = 0 of an exact table: (5, -0) gives u = -0
    extra = np.array([[5.0, 0.0], [5.0, -0.0], [-6.0, 0.0], [-7.0, -0.0], [0.0, 7.0], [0.0, -8.0],
                      [1e-20, 0.0]], np.float32)
    assert np.signbit(extra[1, 1])
    x = np.concatenate([ev.x, extra[:, 0]])
    y = np.concatenate([ev.y, extra[:, 1]])
    half = make_grid(64, 32, kappa_half_range_inv_cm=33.0)
    zero_edge = dataclasses.replace(half, kappa_min=np.float32(0.0))
    exact = make_grid(4, 16, kappa_half_range_inv_cm=33.0, phi_table=np.array([0.0, 0.5, 1.0, 1.5]) * math.pi)
    exact_zero = dataclasses.replace(exact, kappa_min=np.float32(0.0))
    coarse = make_grid(64, 8, kappa_half_range_inv_cm=0.1)        # kappa_scale 0.4
    assert float(coarse.kappa_scale) < 1.0
    for name, grid in (("kappa_min +0", zero_edge), ("exact table, kappa_min +0", exact_zero),
                       ("kappa_scale < 1", coarse)):
        print(f"[parity] {name}", flush=True)
        ref = oracle.find(x, y, grid, 2)
        ctx = hough.HoughContext(grid, max_hits=x.size)
        _assert_same(_gpu_find(ctx, x, y, 2), ref, name)


@pytest.mark.parametrize("dims", [(1, 3, 1), (1, 37, 13), (1, 5, 2), (3, 11, 6), (5, 33, 10), (2, 200, 64)])
def test_odd_small_grids(dims):
    n_d0, n_phi, n_kappa = dims
    print(f"[parity] grid {dims}", flush=True)
    if n_d0 == 1:
        grid = make_grid(n_phi, n_kappa, kappa_half_range_inv_cm=20.0)
    else:
        grid = make_grid(n_phi, n_kappa, n_d0=n_d0, d0_range=(-9.0, 9.0), kappa_half_range_inv_cm=20.0,
                         acc_type="u16")
    ev = synth.gen_config_event(1)
    ref = oracle.find(ev.x, ev.y, grid, 2)
    ctx = hough.HoughContext(grid)
    for rows, threads, split in ((64, 256, 1), (64, 512, 3), (128, 256, 1), (32, 512, 2)):
        try:
            ctx.set_launch(0, rows, threads, split)
        except hough.HoughError:
            assert rows * (ctx.spec.n_kappa + 1) * 4 > 120000
            continue
        _assert_same(_gpu_find(ctx, ev.x, ev.y, 2), ref, f"grid {dims} rows {rows}")


def test_u16_at_the_hit_limit_and_beyond():
    grid = make_grid(16, 8, n_d0=2, d0_range=(-1.0, 1.0), kappa_half_range_inv_cm=0.5, acc_type="u16")
    rng = np.random.default_rng(1)
    # 65535 hits on one spot: every vote lands in the same few cells (max count 65535)
    x = np.full(65535, 50.0, np.float32)
    y = np.full(65535, 0.0, np.float32)
    x[:100] = rng.uniform(-50, 50, 100).astype(np.float32)
    ref = oracle.find(x, y, grid, 1)
    assert ref[0].max() > 65000
    ctx = hough.HoughContext(grid, max_hits=70000)
    _assert_same(_gpu_find(ctx, x, y, 1), ref, "u16 limit")
    big = _t(np.zeros(65536))
    with pytest.raises(hough.HoughError):
        ctx.vote(big, big)


def test_capacity_truncates_to_a_prefix():
    wc = synth.CONFIGS[2]
    ev = synth.gen_config_event(2)
    ref = _oracle(("cfg", 2), ev.x, ev.y, wc.grid, wc.threshold)
    ctx = hough.HoughContext(wc.grid, max_hits=ev.n_hits)
    for cap in (0, 1, 777, ref[4] - 1, ref[4], ref[4] + 5):
        acc, _ = ctx.vote(_t(ev.x), _t(ev.y))
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=_dev())
        out, nf = ctx.peaks(acc, wc.threshold, cap=cap, out=out)
        torch.cuda.synchronize()
        v, c, n = hough.cands_to_numpy(out, nf.item(), cap)
        assert n == ref[4]
        np.testing.assert_array_equal(c, ref[3][:cap])
        np.testing.assert_array_equal(v, ref[2][:cap])


@pytest.mark.parametrize("shape,hi,signed", [((1, 64, 40), 5, True), ((4, 24, 18), 3, False),
                                             ((1, 256, 128), 2000000, True), ((6, 10, 8), 70000, False)])
def test_peaks_on_arbitrary_accumulators(shape, hi, signed):
    """The peak search takes any accumulator: random fields with many ties, negative and
    large values (multi-pass sorts)."""
    n_d0, n_phi, n_kappa = shape
    u16 = n_d0 > 1
    if u16:
        hi = min(hi, 65535)
        grid = make_grid(n_phi, n_kappa, n_d0=n_d0, d0_range=(-1.0, 1.0), acc_type="u16")
    else:
        grid = make_grid(n_phi, n_kappa)
    ctx = hough.HoughContext(grid)
    rng = np.random.default_rng(sum(shape))
    for t in (1, 2, hi // 2):
        lo = -hi if (signed and not u16) else 0
        a = rng.integers(lo, hi + 1, size=shape).astype(np.int64)
        dev = torch.from_numpy(a.astype(np.uint16).view(np.int16) if u16 else a.astype(np.int32)).to(_dev())
        out, nf = ctx.peaks(dev, t)
        torch.cuda.synchronize()
        v, c, n = hough.cands_to_numpy(out, nf.item())
        rv, rc, rn = oracle.peaks(a, t)
        assert n == rn
        np.testing.assert_array_equal(c, rc)
        np.testing.assert_array_equal(v, rv)


@pytest.mark.parametrize("shape,acc_type,offset", [
    ((1, 6, 512), "i32", 0),       # a row is two wavefronts
    ((1, 7, 640), "i32", 0),       # three wavefronts per row: blocks straddle rows
    ((2, 5, 1024), "i32", 0),      # four wavefronts per row
    ((1, 4, 900), "i32", 0),       # a partial fourth wavefront per row
    ((3, 4, 1000), "u16", 0),      # 125 lanes per row
    ((2, 9, 64), "i32", 1),        # accumulator not 16-byte aligned
    ((4, 13, 256), "u16", 2),
    ((3, 7, 6), "u16", 0),         # three dwords per row
    ((11, 6, 16), "u16", 0),       # more d0 slices than one block walks
    ((19, 5, 40), "i32", 0),
])
def test_peak_search_layouts(shape, acc_type, offset):
    """Every lane and block layout of the peak search agrees with the oracle:
    rows spanning several wavefronts, unaligned accumulators, partial lanes
    and long d0 walks."""
    n_d0, n_phi, n_kappa = shape
    u16 = acc_type == "u16"
    if n_d0 > 1:
        grid = make_grid(n_phi, n_kappa, n_d0=n_d0, d0_range=(-1.0, 1.0), acc_type=acc_type)
    else:
        grid = make_grid(n_phi, n_kappa, acc_type=acc_type)
    ctx = hough.HoughContext(grid)
    rng = np.random.default_rng(n_d0 * 1000003 + n_phi * 1009 + n_kappa)
    cells = n_d0 * n_phi * n_kappa
    for hi, t in ((3, 1), (40, 20), (65535 if u16 else 100000, 5)):
        a = rng.integers(0, hi + 1, size=shape).astype(np.int64)
        host = a.astype(np.uint16).view(np.int16) if u16 else a.astype(np.int32)
        buf = torch.zeros(cells + offset, dtype=torch.int16 if u16 else torch.int32, device=_dev())
        buf[offset:] = torch.from_numpy(host.reshape(-1)).to(_dev())
        out, nf = ctx.peaks(buf[offset:], t)
        torch.cuda.synchronize()
        v, c, n = hough.cands_to_numpy(out, nf.item())
        rv, rc, rn = oracle.peaks(a, t)
        print(f"[peaks] {shape} {acc_type} +{offset}: {rn} candidates at threshold {t}", flush=True)
        assert n == rn
        np.testing.assert_array_equal(c, rc)
        np.testing.assert_array_equal(v, rv)


def test_invalid_arguments_raise():
    ctx = hough.HoughContext(synth.GRID_2D_SMALL, max_hits=100)
    x = _t(np.zeros(101))
    with pytest.raises(hough.HoughError):
        ctx.vote(x, x)                                     # more than max_hits
    with pytest.raises(hough.HoughError):
        ctx.set_launch(0, 24, 256, 1)                 # unsupported tile height
    with pytest.raises(hough.HoughError):
        ctx.set_launch(0, 64, 384, 1)                 # unsupported workgroup size
    big = hough.HoughContext(synth.GRID_2D)
    with pytest.raises(hough.HoughError):
        big.set_launch(0, 128, 512, 1)                # 256 KiB of LDS
    with pytest.raises(hough.HoughError):
        ctx.set_launch(1, 64, 256, 2)                 # batch tiles are never split
    with pytest.raises(hough.HoughError):
        ctx.event_batch(np.array([0, 5, 3]), x, x, 7)      # decreasing offsets


# --------------------------------------------------------------------------------------
# Batches
# --------------------------------------------------------------------------------------

def _batch_results(ctx, b, thr, acc=None):
    x, y = _t(b.x), _t(b.y)
    cands, cand_off, nf, nv = ctx.event_batch(b.hit_off, x, y, thr, acc=acc)
    torch.cuda.synchronize()
    out = []
    nf = nf.cpu().numpy()
    nv = nv.cpu().numpy()
    cc = cands.cpu().numpy()
    for e in range(b.n_events):
        s = cc[cand_off[e]:cand_off[e] + min(nf[e], cand_off[e + 1] - cand_off[e])]
        out.append((int(nv[e]), int(nf[e]), s[:, 0].astype(np.int64), s[:, 1].astype(np.int64)))
    return out


def test_batch_matches_oracle_per_event():
    print("[parity] batch of 24 workload-4 events vs oracle", flush=True)
    b = synth.gen_batch(4, 24)
    g = synth.GRID_2D
    ctx = hough.HoughContext(g, max_events=24, max_hits=b.n_hits)
    acc = ctx.new_acc(24)
    res = _batch_results(ctx, b, 7, acc=acc)
    acc_np = hough.acc_to_numpy(acc, ctx.spec)
    for e, ev in enumerate(b.events):
        ra, rnv, rv, rc, rn = oracle.find(ev.x, ev.y, g, 7)
        np.testing.assert_array_equal(acc_np[e].reshape(-1), ra.reshape(-1), err_msg=f"event {e}")
        nv, nf, v, c = res[e]
        assert (nv, nf) == (rnv, rn), e
        np.testing.assert_array_equal(c, rc)
        np.testing.assert_array_equal(v, rv)


def test_batch_3d_matches_single_event_path():
    print("[parity] batch of 3 displaced events", flush=True)
    evs = [synth.gen_config_event(3, i) for i in range(3)]
    b = synth.events.pack_events(evs)
    ctx = hough.HoughContext(synth.GRID_3D, max_events=3, max_hits=b.n_hits)
    res = _batch_results(ctx, b, 5)
    single = hough.HoughContext(synth.GRID_3D, max_hits=40000)
    for e, ev in enumerate(evs):
        a, nv, v, c, n = _gpu_find(single, ev.x, ev.y, 5)
        assert res[e][0] == nv and res[e][1] == n
        np.testing.assert_array_equal(res[e][3], c)
        np.testing.assert_array_equal(res[e][2], v)
    ra, rnv, rv, rc, rn = _oracle(("cfg", 3), evs[0].x, evs[0].y, synth.GRID_3D, 5)
    assert res[0][1] == rn and res[0][0] == rnv
    np.testing.assert_array_equal(res[0][3], rc)


def test_full_batch_equals_single_event_launches_and_is_repeatable():
    """All 256 events of workload 4 in one batch give, bit for bit, what one-event launches
    give; replaying the captured batch ten times changes nothing."""
    print("[parity] full 256-event batch vs single-event launches", flush=True)
    b = synth.gen_batch(4, 256)
    g = synth.GRID_2D
    ctx = hough.HoughContext(g, max_events=256, max_hits=b.n_hits)
    first = _batch_results(ctx, b, 7)
    single = hough.HoughContext(g, max_hits=int(np.diff(b.hit_off).max()))
    for e in range(0, 256, 1):
        ev = b.events[e]
        a, nv, v, c, n = _gpu_find(single, ev.x, ev.y, 7)
        assert first[e][0] == nv and first[e][1] == n, e
        np.testing.assert_array_equal(first[e][3], c)
        np.testing.assert_array_equal(first[e][2], v)
    for rep in range(10):
        again = _batch_results(ctx, b, 7)
        for e in range(256):
            assert again[e][0] == first[e][0] and again[e][1] == first[e][1]
            np.testing.assert_array_equal(again[e][3], first[e][3])
    # every event of the full batch against the oracle
    print("[parity] the 256 batch events against the oracle", flush=True)
    refs = _oracle_many(b.events, g, 7)
    for e, (ra, rnv, rv, rc, rn) in enumerate(refs):
        assert first[e][0] == rnv and first[e][1] == rn, f"event {e}"
        np.testing.assert_array_equal(first[e][2], rv, err_msg=f"event {e}: votes")
        np.testing.assert_array_equal(first[e][3], rc, err_msg=f"event {e}: cells")


def test_packed_batch_lists_are_the_batch_lists_back_to_back():
    """hough_event_batch_packed stores each event's list, as hough_event_batch does, but at
    the running sum of the earlier stored counts: with roomy capacities, and with
    capacities short enough to truncate some events."""
    print("[parity] packed batch lists", flush=True)
    b = synth.gen_batch(4, 40)
    g = synth.GRID_2D
    ctx = hough.HoughContext(g, max_events=40, max_hits=b.n_hits)
    x, y = _t(b.x), _t(b.y)
    ref = _batch_results(ctx, b, 7)
    short = np.array([500 + 1700 * (e % 7) if e % 2 else 131072 for e in range(40)], np.int64)
    for caps in (None, short):
        cand_off = None
        if caps is not None:
            cand_off = np.zeros(41, np.int64)
            cand_off[1:] = np.cumsum(caps)
        cands, start, nf, nv = ctx.event_batch_packed(b.hit_off, x, y, 7, cand_off=cand_off)
        torch.cuda.synchronize()
        start, nf, cc = start.cpu().numpy(), nf.cpu().numpy(), cands.cpu().numpy()
        room = np.full(40, ctx.spec.max_candidates(), np.int64) if caps is None else caps
        stored = np.minimum(nf.astype(np.int64), room)
        assert start[0] == 0 and np.array_equal(np.diff(start), stored)
        for e in range(40):
            nv_e, nf_e, v, c = ref[e]
            assert int(nf[e]) == nf_e
            got = cc[start[e]:start[e + 1]]
            np.testing.assert_array_equal(got[:, 0], v[:stored[e]], err_msg=f"event {e}")
            np.testing.assert_array_equal(got[:, 1], c[:stored[e]], err_msg=f"event {e}")
        if caps is not None:
            assert (nf > caps).any() and (nf <= caps).any()


def test_batch_graph_replay_with_changing_descriptors():
    """The same buffers with different event counts and hit offsets reuse one captured graph;
    every replay must match a fresh single-event computation."""
    g = synth.GRID_2D_SMALL
    evs = [synth.gen_config_event(1, i) for i in range(12)]
    ctx = hough.HoughContext(g, max_events=12, max_hits=20000)
    single = hough.HoughContext(g)
    x = torch.empty(20000, dtype=torch.float32, device=_dev())
    y = torch.empty(20000, dtype=torch.float32, device=_dev())
    cap = 4096
    cands = torch.empty((12 * cap, 2), dtype=torch.int32, device=_dev())
    nf = torch.empty(12, dtype=torch.int32, device=_dev())
    nv = torch.empty(12, dtype=torch.int64, device=_dev())
    for sel in ([0, 1, 2], list(range(12)), [5], [3, 9, 11, 4, 7], [0, 1, 2]):
        b = synth.events.pack_events([evs[i] for i in sel])
        x[:b.n_hits] = _t(b.x)
        y[:b.n_hits] = _t(b.y)
        cand_off = np.arange(len(sel) + 1, dtype=np.int64) * cap
        ctx.event_batch(b.hit_off, x, y, 7, cand_off=cand_off, cands=cands, n_found=nf[:len(sel)],
                        n_votes=nv[:len(sel)])
        torch.cuda.synchronize()
        for k, i in enumerate(sel):
            a, v1, v, c, n = _gpu_find(single, evs[i].x, evs[i].y, 7)
            assert int(nv[k]) == v1 and int(nf[k]) == n
            got = cands[k * cap:k * cap + n].cpu().numpy()
            np.testing.assert_array_equal(got[:, 1], c)


def test_batches_enqueued_back_to_back_without_a_host_sync():
    """Calls A, A, B on one context and stream with no synchronisation between them: the
    second A replays A's graph, whose first node reads the pinned descriptor block, so B
    may rewrite that block only after that replay has read it.  Every result must equal
    the single-event path."""
    print("[parity] batches A, A, B back to back", flush=True)
    g = synth.GRID_2D_SMALL
    evs = [synth.gen_config_event(1, i) for i in range(16)]
    single = hough.HoughContext(g)
    ref = {}
    for i, ev in enumerate(evs):
        _, nv1, v, c, n = _gpu_find(single, ev.x, ev.y, 7)
        ref[i] = (nv1, n, v, c)
    ctx = hough.HoughContext(g, max_events=16, max_hits=20000)
    cap = 4096
    sels = {"A": [0, 1, 2, 3, 4, 5, 6, 7], "B": [8, 9, 10, 11, 12, 13, 14, 15, 1, 2]}
    bufs = {}
    for name, sel in sels.items():
        b = synth.events.pack_events([evs[i] for i in sel])
        bufs[name] = (b, _t(b.x), _t(b.y), torch.empty((len(sel) * cap, 2), dtype=torch.int32, device=_dev()),
                      torch.empty(len(sel), dtype=torch.int32, device=_dev()),
                      torch.empty(len(sel), dtype=torch.int64, device=_dev()))
    torch.cuda.synchronize()
    for rep in range(6):
        for name in ("A", "A", "B"):
            b, x, y, cands, nf, nv = bufs[name]
            cand_off = np.arange(b.n_events + 1, dtype=np.int64) * cap
            ctx.event_batch(b.hit_off, x, y, 7, cand_off=cand_off, cands=cands, n_found=nf, n_votes=nv)
        torch.cuda.synchronize()
        for name, sel in sels.items():
            b, x, y, cands, nf, nv = bufs[name]
            got_nf, got_nv, got = nf.cpu().numpy(), nv.cpu().numpy(), cands.cpu().numpy()
            for k, i in enumerate(sel):
                nv1, n, v, c = ref[i]
                assert (int(got_nv[k]), int(got_nf[k])) == (nv1, n), (rep, name, k)
                np.testing.assert_array_equal(got[k * cap:k * cap + n, 1], c, err_msg=f"{rep} {name} {k}")
                np.testing.assert_array_equal(got[k * cap:k * cap + n, 0], v, err_msg=f"{rep} {name} {k}")


# --------------------------------------------------------------------------------------
# Culling: the tile masks must never drop a vote
# --------------------------------------------------------------------------------------

def test_culling_stress_displaced_hits_near_the_d0_circles():
    """Hits whose radius is close to a d0 bin centre (ill-conditioned chords), tiny and huge
    coordinates, hits on the axes and at bin-edge angles, all against the oracle."""
    rng = np.random.default_rng(77)
    grid = synth.GRID_3D
    d0 = np.abs(grid.d0.astype(np.float64))
    # a band around |r - |d0|| = 0.03 (r + |d0|), the conditioning limit of the arcs, and radii
    # around 2^-8, the lower limit of the 3D hoist-free division
    band = rng.choice(d0, 1000) * (1 + rng.choice([-1.0, 1.0], 1000) * rng.uniform(0.05, 0.15, 1000))
    r = np.concatenate([rng.choice(d0, 3000) + rng.normal(0, 0.05, 3000),
                        rng.uniform(0.01, 120, 3000), rng.choice(d0, 500) * (1 + rng.normal(0, 1e-4, 500)),
                        band, 2.0 ** rng.uniform(-9, -7, 200),
                        10.0 ** rng.uniform(-20, 20, 200)])
    phi = np.concatenate([rng.uniform(0, 2 * math.pi, r.size - 400),
                          (np.arange(400) % 512 + rng.choice([0.0, 0.5], 400)) * 2 * math.pi / 512])
    x = (r * np.cos(phi)).astype(np.float32)
    y = (r * np.sin(phi)).astype(np.float32)
    x[:8] = [0, 0, 5, -5, 1e-39, 3e38, 0, 30]
    y[:8] = [5, -5, 0, 0, 1e-39, 1, 0, 0]
    ref = oracle.find(x, y, grid, 3)
    ctx = hough.HoughContext(grid, max_hits=x.size)
    for shape in ((64, 512, 1), (128, 256, 1), (32, 512, 1)):
        ctx.set_launch(0, *shape)
        _assert_same(_gpu_find(ctx, x, y, 3), ref, f"3D stress {shape}")


def test_culling_stress_prompt_hits():
    rng = np.random.default_rng(78)
    grid = synth.GRID_2D
    r = np.concatenate([rng.uniform(0.001, 200, 20000), 10.0 ** rng.uniform(-30, 30, 500)])
    phi = rng.uniform(-4, 10, r.size)
    x = (r * np.cos(phi)).astype(np.float32)
    y = (r * np.sin(phi)).astype(np.float32)
    ref = oracle.find(x, y, grid, 3)
    ctx = hough.HoughContext(grid, max_hits=x.size)
    _assert_same(_gpu_find(ctx, x, y, 3), ref, "2D stress")
    # the same hits through the fused batch path
    b = synth.events.pack_events([synth.Event(x=x, y=y, label=np.zeros(x.size, np.int32),
                                              d0=np.zeros(0), phi0=np.zeros(0), kappa=np.zeros(0))])
    bctx = hough.HoughContext(grid, max_events=1, max_hits=x.size)
    res = _batch_results(bctx, b, 3)
    assert res[0][0] == ref[1] and res[0][1] == ref[4]
    np.testing.assert_array_equal(res[0][3], ref[3])


def test_non_centre_phi_table_turns_culling_off():
    """A phi0 table that is not the bin centres (here: shifted by a third of a bin) is voted
    without tile masks and still matches the oracle."""
    n_phi, n_kappa = 512, 128
    tab = (np.arange(n_phi) + 0.5 + 1.0 / 3.0) * 2 * math.pi / n_phi
    grid = make_grid(n_phi, n_kappa, phi_table=tab)
    ev = synth.gen_config_event(4, 3)
    ref = oracle.find(ev.x, ev.y, grid, 5)
    ctx = hough.HoughContext(grid, max_hits=ev.n_hits)
    _assert_same(_gpu_find(ctx, ev.x, ev.y, 5), ref, "shifted table")


def test_more_tiles_than_mask_bits():
    """4096 phi0 rows make 64 tiles per slice: the masks (32 bits) are not used."""
    grid = make_grid(4096, 64)
    ev = synth.gen_config_event(1)
    ref = oracle.find(ev.x, ev.y, grid, 4)
    ctx = hough.HoughContext(grid, max_hits=ev.n_hits)
    _assert_same(_gpu_find(ctx, ev.x, ev.y, 4), ref, "64 tiles")
    b = synth.events.pack_events([ev, synth.gen_config_event(1, 1)])
    bctx = hough.HoughContext(grid, max_events=2, max_hits=b.n_hits)
    res = _batch_results(bctx, b, 4)
    assert res[0][1] == ref[4]
    np.testing.assert_array_equal(res[0][3], ref[3])


def test_batch_tile_shapes_agree():
    b = synth.gen_batch(4, 6)
    g = synth.GRID_2D
    base = None
    ctx = hough.HoughContext(g, max_events=6, max_hits=b.n_hits)
    for shape in ((32, 512), (64, 512), (64, 1024), (64, 256), (32, 256), (32, 1024), (128, 512)):
        try:
            ctx.set_launch(1, shape[0], shape[1], 1)
        except hough.HoughError:
            assert shape[0] == 128     # a 128-row int32 tile of 512 kappa bins does not fit in LDS
            continue
        res = _batch_results(ctx, b, 7)
        if base is None:
            base = res
        for e in range(6):
            assert res[e][:2] == base[e][:2]
            np.testing.assert_array_equal(res[e][3], base[e][3])
    ev = b.events[2]
    ra, rnv, rv, rc, rn = oracle.find(ev.x, ev.y, g, 7)
    assert base[2][0] == rnv and base[2][1] == rn
    np.testing.assert_array_equal(base[2][3], rc)


@pytest.mark.parametrize("grid_name,shape", [("2d", (32, 512)), ("2d", (64, 1024)), ("3d", (64, 512))])
def test_batch_events_straddling_hit_chunks(grid_name, shape):
    """Events of 0, 1, 63, 64, 65, 127, 129 ... hits packed back to back: the
    vote stages hits in chunks at multiples of 64 of the record array, so
    most events start and end inside a chunk shared with their neighbours,
    and tile words of other events' hits must not leak into them."""
    print(f"[parity] straddling events {grid_name} {shape}", flush=True)
    d3 = grid_name == "3d"
    src = synth.gen_config_event(3 if d3 else 2)
    rng = np.random.default_rng(64)
    sizes = [0, 1, 65, 129, 500, 63] if d3 else [0, 1, 63, 64, 65, 127, 129, 700, 0, 2000, 31, 3]
    events = []
    for n in sizes:
        pick = rng.choice(src.n_hits, size=n, replace=False)
        events.append((src.x[pick], src.y[pick]))
    hit_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.concatenate([e[0] for e in events]).astype(np.float32)
    y = np.concatenate([e[1] for e in events]).astype(np.float32)
    g = synth.GRID_3D if d3 else synth.GRID_2D
    thr = 5 if d3 else 2
    b = dataclasses.make_dataclass("B", ["x", "y", "hit_off", "n_events"])(x, y, hit_off, len(sizes))
    ctx = hough.HoughContext(g, max_events=len(sizes), max_hits=max(int(hit_off[-1]), 1))
    ctx.set_launch(1, shape[0], shape[1], 1)
    res = _batch_results(ctx, b, thr)
    for e, (ex, ey) in enumerate(events):
        ra, rnv, rv, rc, rn = oracle.find(ex, ey, g, thr)
        nv, nf, v, c = res[e]
        assert (nv, nf) == (rnv, rn), (e, sizes[e])
        np.testing.assert_array_equal(c, rc[:len(c)])
        np.testing.assert_array_equal(v, rv[:len(v)])


def test_timing_mode_gives_the_same_results():
    b = synth.gen_batch(4, 5)
    ctx = hough.HoughContext(synth.GRID_2D, max_events=5, max_hits=b.n_hits)
    base = _batch_results(ctx, b, 7)
    ctx.set_timing(True)
    timed = _batch_results(ctx, b, 7)
    v_ms, t_ms = ctx.get_timing()
    assert 0 < v_ms <= t_ms
    ctx.set_timing(False)
    for e in range(5):
        assert timed[e][:2] == base[e][:2]
        np.testing.assert_array_equal(timed[e][3], base[e][3])


def test_counted_pairs_bound_the_work():
    """Timing mode 2 counts the (hit, row) pairs the vote evaluates: at least one
    per vote cast, at most every row of every tile (halo rows included) for every
    hit, and the culling leaves out a good share; results are unchanged."""
    b = synth.gen_batch(4, 6)
    g = synth.GRID_2D
    ctx = hough.HoughContext(g, max_events=6, max_hits=b.n_hits)
    base = _batch_results(ctx, b, 7)
    with pytest.raises(hough.HoughError):
        ctx.get_work()                      # nothing counted yet
    ctx.set_timing(2)
    counted = _batch_results(ctx, b, 7)
    pairs = ctx.get_work()
    ctx.set_timing(False)
    votes = sum(r[0] for r in counted)
    rows, _, _ = ctx.get_launch(1)
    tiles = -(-g.n_phi // (rows - 2))      # fused tiles of rows - 2 interior rows, each with two halo rows
    assert votes <= pairs <= b.n_hits * tiles * rows
    assert pairs < 0.8 * b.n_hits * g.n_phi
    for e in range(6):
        assert counted[e][:2] == base[e][:2]
        np.testing.assert_array_equal(counted[e][3], base[e][3])


def test_counted_pairs_are_the_culled_tiles():
    """The pairs timing mode 2 counts are the kept (hit, tile) pairs times the
    tile's voted rows, where a hit is kept by the tiles whose rows meet its
    culling arcs -- redone on the CPU (tests/test_culling_cpu.py's binary32
    emulation with correctly rounded angle functions; the device's are within
    1e-6 rad, so a few boundary rows may differ).  Catches staging that keeps
    hits a tile's arcs do not reach, which no result would show."""
    from test_culling_cpu import arc_rows
    b = synth.gen_batch(4, 2)
    g = synth.GRID_2D
    ctx = hough.HoughContext(g, max_events=2, max_hits=b.n_hits)
    ctx.set_timing(2)
    _batch_results(ctx, b, 7)
    pairs = ctx.get_work()
    ctx.set_timing(False)
    rows, _, _ = ctx.get_launch(1)
    S = rows - 2                                 # interior rows of a fused tile
    T = -(-g.n_phi // S)
    voted = []
    for t in range(T):
        s_here = min(S, g.n_phi - t * S)
        voted.append({(t * S - 1 + k) % g.n_phi for k in range(s_here + 2)})
    expect = 0
    for xi, yi in zip(b.x, b.y):
        R = arc_rows(xi, yi, g)[0]
        expect += sum(len(v) for v in voted if not v.isdisjoint(R))
    assert abs(pairs - expect) <= 2e-3 * expect, (pairs, expect)


def test_division_fast_path_equals_the_operator():
    """The hoisted-reciprocal quotient equals fp32 division bit for bit (device self-test)."""
    _dev()
    total = 0
    for seed in (1, 2, 3):
        bad, used = hough.selftest_divide(100_000_000, seed)
        assert bad == 0, f"{bad} mismatches of {used}"
        total += used
    assert total > 100_000_000


def test_culling_angle_functions_stay_within_their_budget():
    """The fp32 angle functions behind the culling arcs err by at most 1e-6 rad,
    so the 1e-4 rad widening of every arc covers them many times over."""
    _dev()
    for seed in (1, 2):
        e_atan, e_asin = hough.selftest_angles(50_000_000, seed)
        print(f"[angles] seed {seed}: atan2f {e_atan:.3g} rad, asinf {e_asin:.3g} rad", flush=True)
        assert 0.0 < e_atan <= 1e-6
        assert 0.0 < e_asin <= 1e-6


def _grid_args(g):
    return float(g.kappa_min), float(g.kappa_scale), g.n_kappa


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("kappa_min,kappa_scale,n_kappa", [
    _grid_args(synth.GRID_3D), _grid_args(synth.GRID_2D), _grid_args(synth.GRID_STRAIGHT),
    (-0.25, 96.0, 48), (-1e-3, 1.0e5, 200), (0.0, 2048.0, 64), (-3.0, 0.75, 5), (-20.0, 500.0, 4096)])
def test_approximate_bins_never_change_a_bin(kappa_min, kappa_scale, n_kappa, form):
    """Device check of the vote's approximate bins (form 0: the 3D one-reciprocal
    quotient, 1: the 2D scaled hit reciprocal): outside the flagged band above
    each integer they always pick the exact bin."""
    _dev()
    bad, redo, used = hough.selftest_near(20_000_000, kappa_min, kappa_scale, n_kappa, form)
    print(f"[near] form {form} kappa_min {kappa_min} scale {kappa_scale} n {n_kappa}: {used} pairs, {redo} redone",
          flush=True)
    assert used > 10_000_000
    assert bad == 0, f"{bad} bins differ"
    assert 0 < redo < used // 4


def test_throughput_probes_report_plausible_rates():
    """The roofline probes run and land within the chip's nominal limits."""
    _dev()
    lds, valu = hough.diag_rates()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # at most 64 dword atomics and 64 lanes per CU per clock at <= 2.6 GHz
    assert 0 < lds <= cus * 64 * 2.6e9
    assert 0 < valu <= cus * 64 * 2.6e9
    print(f"[probe] lds {lds / 1e12:.2f} T/s, valu {valu / 1e12:.2f} T/s on {cus} CUs", flush=True)


def test_autotuner_picks_a_shape_records_it_and_changes_no_result(tmp_path):
    b = synth.gen_batch(4, 6)
    g = synth.GRID_2D
    dev = _dev()
    x, y = _t(b.x), _t(b.y)
    cache = str(tmp_path / "tune.jsonl")
    base = _batch_results(hough.HoughContext(g, max_events=6, max_hits=b.n_hits), b, 7)
    ctx = hough.HoughContext(g, max_events=6, max_hits=b.n_hits)
    rows, threads, split, ms = ctx.autotune(1, b.hit_off, x, y, 7, reps=2, cache=cache)
    assert ms > 0 and split == 1 and (rows, threads) in {(r, t) for r in (32, 64) for t in (256, 512, 1024)}
    tuned = _batch_results(ctx, b, 7)
    for e in range(6):
        assert tuned[e][:2] == base[e][:2]
        np.testing.assert_array_equal(tuned[e][3], base[e][3])
    # single-event vote of event 0
    acc = ctx.new_acc()
    r0, t0, s0, ms0 = ctx.autotune(0, b.hit_off[:2], x, y, acc=acc, reps=2, cache=cache)
    ev = b.events[0]
    ra, rnv, _, _, _ = oracle.find(ev.x, ev.y, g, 7)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(hough.acc_to_numpy(acc, ctx.spec).reshape(-1), ra.reshape(-1))
    lines = open(cache).read().splitlines()
    assert len(lines) == 2
    # a new context created with the cache starts from the tuned shapes
    fresh = hough.HoughContext(g, max_events=6, max_hits=b.n_hits, tune_cache=cache)
    assert fresh.get_launch(1) == (rows, threads, 1)
    assert fresh.get_launch(0) == (r0, t0, s0)


def test_sort_passes_follow_the_largest_event():
    """The sort runs one pass per 8-bit digit that the batch's vote counts can reach
    (bounded by its largest event).  A batch with a 70,000-hit event whose cells pass
    2^16 votes needs the third pass; a small batch on the same context needs one, and
    the two alternate through the context's cached graphs."""
    g = synth.GRID_2D_SMALL
    big = synth.gen_config_event(1)
    # 70,000 copies of one hit: every cell of its curve gets 70,000 votes
    hx = np.concatenate([np.full(70000, big.x[0], np.float32), big.x])
    hy = np.concatenate([np.full(70000, big.y[0], np.float32), big.y])
    ev_big = dataclasses.replace(big, x=hx, y=hy, label=np.zeros(hx.size, np.int32))
    small = [synth.gen_config_event(1, i) for i in (1, 2)]
    b_big = synth.pack_events([ev_big, small[0]])
    b_small = synth.pack_events(small)
    ctx = hough.HoughContext(g, max_events=2, max_hits=b_big.n_hits)
    for b in (b_big, b_small, b_big, b_small):
        res = _batch_results(ctx, b, 7)
        for e, ev in enumerate(b.events):
            _, rnv, rv, rc, rn = oracle.find(ev.x, ev.y, g, 7)
            nv, nf, v, c = res[e]
            print(f"[parity] sort passes: event of {ev.n_hits} hits, {rn} candidates, top {rv[:1]}", flush=True)
            assert (nv, nf) == (rnv, rn)
            np.testing.assert_array_equal(v, rv[:len(v)])
            np.testing.assert_array_equal(c, rc[:len(c)])
    assert oracle.find(ev_big.x, ev_big.y, g, 7)[2][0] > 65535
