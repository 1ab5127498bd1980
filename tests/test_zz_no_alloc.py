"""hough_event_noalloc (the entry point for callers that cannot allocate)
against the context entry points hough_vote + hough_peaks, through the C ABI.

Two calls in a row on one stream, the second with a smaller event, so the
second reads scratch the first has written; both must equal the context path
bit for bit (accumulator, vote count, candidate count and list).
"""

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1311_2769_amd import hough  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _noalloc(dgrid, x, y, thr):
    spec = dgrid.spec
    acc = torch.empty((spec.n_d0, spec.n_phi, spec.n_kappa), dtype=spec.acc_dtype, device=_dev())
    out = torch.empty((spec.max_candidates(), 2), dtype=torch.int32, device=_dev())
    nf = torch.empty(1, dtype=torch.int32, device=_dev())
    nv = torch.empty(1, dtype=torch.int64, device=_dev())
    hough.event_noalloc(dgrid, x, y, thr, acc, out, nf, nv)
    return acc, out, nf, nv


def _context(grid, x, y, thr):
    ctx = hough.HoughContext(grid, max_hits=max(int(x.numel()), 1))
    acc, nv = ctx.vote(x, y)
    out, nf = ctx.peaks(acc, thr)
    return ctx, acc, out, nf, nv


def _same(a, b, spec, what):
    acc_a, out_a, nf_a, nv_a = a
    acc_b, out_b, nf_b, nv_b = b
    np.testing.assert_array_equal(hough.acc_to_numpy(acc_a, spec), hough.acc_to_numpy(acc_b, spec),
                                  err_msg=f"{what}: accumulator")
    assert int(nv_a.item()) == int(nv_b.item()), f"{what}: vote count"
    n = int(nf_a.item())
    assert n == int(nf_b.item()), f"{what}: candidate count"
    np.testing.assert_array_equal(out_a[:n].cpu().numpy(), out_b[:n].cpu().numpy(), err_msg=f"{what}: candidates")


@pytest.mark.parametrize("cfg", [2, 3])
def test_noalloc_matches_the_context_path_twice(cfg):
    print(f"[noalloc] workload {cfg}", flush=True)
    wc = synth.CONFIGS[cfg]
    ev = synth.gen_config_event(cfg)
    small = ev.n_hits // 3 + 7
    dgrid = hough.DeviceGrid(wc.grid, _dev())
    x1, y1 = _t(ev.x), _t(ev.y)
    x2, y2 = _t(ev.x[:small]), _t(ev.y[:small])
    first = _noalloc(dgrid, x1, y1, wc.threshold)
    second = _noalloc(dgrid, x2, y2, wc.threshold)     # same stream, no sync in between
    torch.cuda.synchronize()
    ctx1, *ref1 = _context(wc.grid, x1, y1, wc.threshold)
    ctx2, *ref2 = _context(wc.grid, x2, y2, wc.threshold)
    torch.cuda.synchronize()
    _same(first, (ref1[0], ref1[1], ref1[2], ref1[3]), dgrid.spec, f"workload {cfg}, full event")
    _same(second, (ref2[0], ref2[1], ref2[2], ref2[3]), dgrid.spec, f"workload {cfg}, smaller event")
    if cfg == 2:    # and the oracle on the smaller event
        _, rnv, rv, rc, rn = oracle.find(ev.x[:small], ev.y[:small], wc.grid, wc.threshold)
        assert int(second[3].item()) == rnv and int(second[2].item()) == rn
        got = second[1][:rn].cpu().numpy()
        np.testing.assert_array_equal(got[:, 0], rv)
        np.testing.assert_array_equal(got[:, 1], rc)


def test_noalloc_small_grid_then_empty_event():
    """Workload 1 (480 hits, 256 x 128) and then an empty event on the same grid."""
    wc = synth.CONFIGS[1]
    ev = synth.gen_config_event(1)
    dgrid = hough.DeviceGrid(wc.grid, _dev())
    first = _noalloc(dgrid, _t(ev.x), _t(ev.y), wc.threshold)
    empty = torch.zeros(0, dtype=torch.float32, device=_dev())
    second = _noalloc(dgrid, empty, empty, wc.threshold)
    torch.cuda.synchronize()
    ra, rnv, rv, rc, rn = oracle.find(ev.x, ev.y, wc.grid, wc.threshold)
    np.testing.assert_array_equal(hough.acc_to_numpy(first[0], dgrid.spec).reshape(-1), ra.reshape(-1))
    assert int(first[3].item()) == rnv and int(first[2].item()) == rn
    got = first[1][:rn].cpu().numpy()
    np.testing.assert_array_equal(got[:, 0], rv)
    np.testing.assert_array_equal(got[:, 1], rc)
    assert int(second[0].abs().sum().item()) == 0 and int(second[2].item()) == 0 and int(second[3].item()) == 0


def test_noalloc_rejects_what_does_not_fit():
    """An event whose scratch would exceed the fixed array, and a uint16 event of
    more than 65535 hits, are refused before anything is enqueued."""
    dev = _dev()
    dgrid = hough.DeviceGrid(synth.GRID_2D, dev)
    n = 3_000_000     # 2D: about 24 bytes of scratch per hit, beyond 64 MiB
    x = torch.zeros(n, dtype=torch.float32, device=dev)
    with pytest.raises(hough.HoughError, match="SCRATCH"):
        _noalloc(dgrid, x, x, 7)
    d3 = hough.DeviceGrid(synth.GRID_3D, dev)
    x3 = torch.zeros(70_000, dtype=torch.float32, device=dev)
    with pytest.raises(hough.HoughError, match="65535"):
        _noalloc(d3, x3, x3, 5)
