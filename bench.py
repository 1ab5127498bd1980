#!/usr/bin/env python3
"""Throughput benchmark of the Hough track finder on one MI355X.

One step = one batch of 256 uneven prompt-track events (200-8,000 tracks
each, about 2k-100k hits, 1024 phi0 x 512 kappa int32 accumulators,
threshold 7) through the whole path: vote, peak search and sorted candidate
lists, launched as one captured graph (hough_event_batch) with the launch
shape the autotuner picks.  For `value` the hits are resident in HBM before
the timed region and the candidates stay there.  The line also carries the
same batches with the host transfers (pinned hits in, every stored candidate
back), the per-event-launch rates on the same events, the served stream, the
dominant kernel against its roofline and the CPU oracle timed on a bounded
sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at up to 2.4 GHz, 64 lanes per CU issuing one unpacked
# VALU operation per clock (the 157.3 TFLOP/s fp32 figure counts a packed FMA
# as four flops per lane; packed fp32 is off in this build).
PEAK_VALU_OPS = 256 * 64 * 2.4e9          # 39.3e12 VALU lane-operations / s
# VALU instructions per evaluated (hit, phi0 row) pair in the 2D vote loop of
# the built kernel (approximate bins): u = y c - x s (2 mul, 1 sub), the bin
# estimate (1 fma), its clamp (1 min), the band test (fract, compare), the
# conversion (1 cvt) and the LDS address (1 shift-add).  The exact redo, one
# wave-uniform branch away, runs for a few per cent of pairs.
VALU_PER_PAIR_2D = 9
VERTEX_TRACK_THRESHOLD = 300              # track candidates that vote in the second transform
VERTEX_THRESHOLD = 4                      # vertex candidates: lines meeting in a cell

# HBM bytes of the dominant kernel from rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, each scaled by what the counter reads for a
# plain device copy of known size).  Used only while the kernel's sources are
# the ones the counters were taken from.
COUNTERS = os.path.join(ROOT, "profiles", "vote_fused_batch256_2d_counters.md")
KERNEL_SOURCES = ["vote.hip", "vote_math.h", "peak_tile.h", "hough_impl.h"]


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of each oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency-events", type=int, default=64)
    ap.add_argument("--skip-per-event", action="store_true", help="skip the per-event-launch comparison")
    ap.add_argument("--skip-3d", action="store_true", help="skip the displaced-vertex (3D) batch leg")
    ap.add_argument("--skip-straight", action="store_true", help="skip the straight-line batch leg")
    ap.add_argument("--skip-forward", action="store_true", help="skip the forward-hemisphere batch leg")
    ap.add_argument("--lanes", type=int, default=3,
                    help="batches in flight: contexts on streams of their own, taking the steps in turn "
                         "(a batch's sort and the next ones' hit preparation run between two votes; "
                         "3 lanes measured 1 %% faster than 2, 2 than 1)")
    ap.add_argument("--e2e-lanes", type=int, default=3,
                    help="batches in flight in the leg with host transfers (copies in, compute and "
                         "copies out of different batches overlap)")
    ap.add_argument("--e2e-steps", type=int, default=20, help="timed steps of the leg with host transfers")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--skip-assoc", action="store_true", help="skip the hit-association / truth report leg")
    ap.add_argument("--serve-rates", default="1000,5000,8000,10000,12000,14000,16000,20000",
                    help="offered rates (events/s) of the served stream; empty to skip")
    ap.add_argument("--serve-events", type=int, default=20000, help="measured arrivals per rate")
    ap.add_argument("--serve-lanes", type=int, default=3,
                    help="server lanes per grid (batches in flight; 3 carried 16k events/s of the mix where 2 "
                         "carried 12.6k, 4 measured the same as 3)")
    ap.add_argument("--serve-warmup", type=int, default=1000, help="arrivals per rate before the measured ones")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_text(src):
    """Source text without comments and blank lines: an edit of a comment
    leaves the compiled kernel, and so this text, unchanged.  None of the
    kernel sources holds a string literal with a comment marker in it."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_digest(read=None):
    """SHA-256 of the vote kernel's sources, comments removed (code_text);
    read(name) gives a source's text (default: the file in csrc/)."""
    import hashlib
    if read is None:
        def read(name):
            with open(os.path.join(ROOT, "paper_1311_2769_amd", "csrc", name)) as f:
                return f.read()
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(code_text(read(name)).encode())
    return h.hexdigest()


def counter_fields(rows, threads):
    """Per-dispatch counters of the vote kernel at launch shape rows x threads
    from the committed summary: (HBM bytes per launch, VALU wave-instructions
    per launch), each None when missing, taken at another shape or from other
    kernel sources.  Fields carry the shape as a suffix (`_64x1024`)."""
    try:
        with open(COUNTERS) as f:
            fields = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None, None
    fields = {k.strip().strip("-* `"): v.strip().strip("` ") for k, v in fields.items()}
    if fields.get("kernel_source_sha256") != kernel_digest():
        return None, None
    sfx = f"_{rows}x{threads}"
    traffic = valu = None
    try:
        fetch = float(fields["fetch_kib_per_dispatch" + sfx]) * float(fields["fetch_scale"])
        write = float(fields["write_kib_per_dispatch" + sfx]) * float(fields["write_scale"])
        traffic = 1024.0 * (fetch + write)
    except (KeyError, ValueError):
        pass
    try:
        valu = float(fields["valu_insts_per_dispatch" + sfx])
    except (KeyError, ValueError):
        pass
    return traffic, valu


def _oracle_events(args):
    """Worker of the parallel CPU baseline (a fresh interpreter): run the
    oracle on each (x, y) event, return the count done within the budget."""
    events, grid, threshold, budget_s = args
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    n = 0
    for x, y in events:
        oracle.find(x, y, grid, threshold)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return n, time.perf_counter() - t0


def cpu_baseline(batch, grid, threshold, budget_s, max_workers=16):
    """The oracle as it stands on the host's cores: one thread over the
    batch's events in order, then independent events spread over a pool of
    worker processes (one event per process at a time), one per core the job
    may use: the cores this process may run on, at most max_workers (the
    host share a one-GPU job is given, whatever the machine has)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    evs = [(ev.x, ev.y) for ev in batch.events]
    n1, dt1 = _oracle_events((evs, grid, threshold, budget_s))
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(max_workers, allowed))
    chunks = [evs[i::workers] for i in range(workers)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        res = list(pool.map(_oracle_events, [(c, grid, threshold, budget_s) for c in chunks]))
    rate = sum(n / dt for n, dt in res if dt > 0)
    done = sum(n for n, _ in res)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": rate, "unit": "events/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} of the {batch.n_events} batch events split over {workers} worker processes "
                      f"(about {budget_s:.0f} s each), vote + peaks + sort per event; host CPU {cpu}",
            "host_nproc": os.cpu_count(), "host_cores_allowed": allowed, "cpu_model": cpu,
            "single_thread": {"value": n1 / dt1, "events": n1, "seconds": dt1}}


def per_event(args, hough, torch, dev, batch, grid, thr, cap, x, y, hit_off, shape):
    """One event per call on the same events: resident (hits already in HBM,
    candidates left there) and closed-loop with the host transfers of each
    event (pinned hits in, n_found and exactly the stored candidates out, then
    the next event), each through hough_vote + hough_peaks and through
    hough_event_batch of one event (one graph replay per event)."""
    log("per-event launches")
    n_ev = batch.n_events
    most = int(np.diff(hit_off).max())
    single = hough.HoughContext(grid, device=dev, max_hits=most)
    one = hough.HoughContext(grid, device=dev, max_events=1, max_hits=most)
    if shape:
        one.set_launch(1, shape[0], shape[1])
    acc1 = single.new_acc()
    out1 = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    nf1 = torch.empty(1, dtype=torch.int32, device=dev)
    nv1 = torch.empty(1, dtype=torch.int64, device=dev)
    one_off = np.array([0, cap], np.int64)
    views = [(x[hit_off[e]:hit_off[e + 1]], y[hit_off[e]:hit_off[e + 1]]) for e in range(n_ev)]

    def two_calls(xe, ye):
        single.vote(xe, ye, acc1, nv1)
        single.peaks(acc1, thr, cap, out1, nf1)

    def graph_call(xe, ye):
        n = int(xe.numel())
        one.event_batch(np.array([0, n], np.int64), xe, ye, thr, cand_off=one_off, cands=out1, n_found=nf1,
                        n_votes=nv1)

    out = {}
    for name, call in (("vote_peaks", two_calls), ("graph_of_one", graph_call)):
        for xe, ye in views[:4]:
            call(xe, ye)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for xe, ye in views:
            call(xe, ye)
        torch.cuda.synchronize()
        resident = n_ev / (time.perf_counter() - t0)
        # closed loop with host round trips
        hx = torch.from_numpy(batch.x).pin_memory()
        hy = torch.from_numpy(batch.y).pin_memory()
        host_out = torch.empty((cap, 2), dtype=torch.int32).pin_memory()
        host_nf = torch.empty(1, dtype=torch.int32).pin_memory()
        xd = torch.empty(most, dtype=torch.float32, device=dev)
        yd = torch.empty_like(xd)
        stream = torch.cuda.current_stream()
        lat = []
        t_all = time.perf_counter()
        for e in range(n_ev):
            a, b = int(hit_off[e]), int(hit_off[e + 1])
            ts = time.perf_counter()
            xd[:b - a].copy_(hx[a:b], non_blocking=True)
            yd[:b - a].copy_(hy[a:b], non_blocking=True)
            call(xd[:b - a], yd[:b - a])
            host_nf.copy_(nf1, non_blocking=True)
            stream.synchronize()
            n = min(int(host_nf[0]), cap)
            if n > 0:
                host_out[:n].copy_(out1[:n], non_blocking=True)
                stream.synchronize()
            lat.append(time.perf_counter() - ts)
        closed = n_ev / (time.perf_counter() - t_all)
        lat_ms = 1e3 * np.array(lat)
        out[name] = {"resident_events_per_s": resident, "transfers_events_per_s": closed,
                     "transfers_p50_ms": float(np.percentile(lat_ms, 50)),
                     "transfers_p99_ms": float(np.percentile(lat_ms, 99)), "events": n_ev}
    return out


def end_to_end(args, hough, torch, dev, batch, grid, thr, cap, shape):
    """The batch workload with its host transfers: each step copies the
    batch's hits in from pinned host memory, runs hough_event_batch_packed,
    brings cand_start and n_found back, and then -- the total known -- every
    stored candidate in one copy.  e2e_lanes batches are in flight on streams
    of their own, so one batch's copies overlap another's compute."""
    from collections import deque
    L = max(1, args.e2e_lanes)
    n_ev = batch.n_events
    H = int(batch.n_hits)
    hit_off = batch.hit_off
    cand_off = np.arange(n_ev + 1, dtype=np.int64) * cap
    hx = torch.from_numpy(batch.x).pin_memory()
    hy = torch.from_numpy(batch.y).pin_memory()
    log(f"host transfers: {L} batches in flight")

    class Lane:
        pass

    lanes = []
    for _ in range(L):
        ln = Lane()
        ln.ctx = hough.HoughContext(grid, device=dev, max_events=n_ev, max_hits=H)
        if shape:
            ln.ctx.set_launch(1, shape[0], shape[1])
        ln.stream = torch.cuda.Stream(device=dev)
        ln.x = torch.empty(H, dtype=torch.float32, device=dev)
        ln.y = torch.empty_like(ln.x)
        ln.cands = torch.empty((int(cand_off[-1]), 2), dtype=torch.int32, device=dev)
        ln.start = torch.empty(n_ev + 1, dtype=torch.int64, device=dev)
        ln.nf = torch.empty(n_ev, dtype=torch.int32, device=dev)
        ln.nv = torch.empty(n_ev, dtype=torch.int64, device=dev)
        ln.h_start = torch.empty(n_ev + 1, dtype=torch.int64).pin_memory()
        ln.h_nf = torch.empty(n_ev, dtype=torch.int32).pin_memory()
        ln.h_cands = None
        ln.ev1 = torch.cuda.Event()
        ln.done = torch.cuda.Event()
        ln.used = False
        lanes.append(ln)

    def phase1(ln):
        if ln.used:
            ln.done.synchronize()           # its last candidates have reached the host
        ln.used = True
        with torch.cuda.stream(ln.stream):
            ln.x.copy_(hx, non_blocking=True)
            ln.y.copy_(hy, non_blocking=True)
            ln.ctx.event_batch_packed(hit_off, ln.x, ln.y, thr, cand_off=cand_off, cands=ln.cands,
                                      cand_start=ln.start, n_found=ln.nf, n_votes=ln.nv, stream=ln.stream)
            ln.h_start.copy_(ln.start, non_blocking=True)
            ln.h_nf.copy_(ln.nf, non_blocking=True)
            ln.ev1.record(ln.stream)

    def phase2(ln):
        ln.ev1.synchronize()
        total = int(ln.h_start[-1])
        if ln.h_cands is None or ln.h_cands.shape[0] < total:
            ln.h_cands = torch.empty((max(total, 1), 2), dtype=torch.int32).pin_memory()
        with torch.cuda.stream(ln.stream):
            if total > 0:
                ln.h_cands[:total].copy_(ln.cands[:total], non_blocking=True)
            ln.done.record(ln.stream)
        return total

    def run(steps):
        pending = deque()
        total = 0
        for i in range(steps):
            ln = lanes[i % L]
            phase1(ln)
            pending.append(ln)
            if len(pending) >= L:
                total = phase2(pending.popleft())
        while pending:
            total = phase2(pending.popleft())
        for ln in lanes:
            ln.done.synchronize()
        return total

    run(L)                                  # warm-up: graphs, pinned buffers
    torch.cuda.synchronize()
    steps = max(1, args.e2e_steps)
    t0 = time.perf_counter()
    total = run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nf = lanes[0].h_nf.numpy().astype(np.int64)
    return {"events_per_s": n_ev * steps / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps, "lanes": L,
            "h2d_bytes_per_step": 8 * H, "d2h_bytes_per_step": 8 * int(total) + 12 * n_ev + 8,
            "candidates_per_step": int(total), "n_found_per_step": int(nf.sum()),
            "pcie_gbs": (8 * H + 8 * int(total)) * steps / dt / 1e9}


def displaced_3d(hough, torch, dev, synth, log_fn, n_events=8, reps=10):
    """The displaced-vertex workload (35,000 hits, 64 d0 x 512 phi0 x 256
    kappa uint16, threshold 5) as one batch of n_events through the same
    graph path: ms per event for the whole batch and for its vote kernel."""
    wc = synth.CONFIGS[3]
    b = synth.pack_events([synth.gen_config_event(3, i) for i in range(n_events)])
    x = torch.from_numpy(b.x).to(dev)
    y = torch.from_numpy(b.y).to(dev)
    ctx = hough.HoughContext(wc.grid, device=dev, max_events=n_events, max_hits=b.n_hits)
    cap = ctx.spec.max_candidates()
    cand_off = np.arange(n_events + 1, dtype=np.int64) * cap
    cands = torch.empty((n_events * cap, 2), dtype=torch.int32, device=dev)
    n_found = torch.empty(n_events, dtype=torch.int32, device=dev)
    n_votes = torch.empty(n_events, dtype=torch.int64, device=dev)

    def step():
        ctx.event_batch(b.hit_off, x, y, wc.threshold, cand_off=cand_off, cands=cands, n_found=n_found,
                        n_votes=n_votes)

    log_fn(f"displaced-vertex batch of {n_events}")
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.set_timing(True)
    vote = []
    for _ in range(4):
        step()
        vote.append(ctx.get_timing()[0])
    ctx.set_timing(False)
    evals = int(b.n_hits) * wc.grid.n_d0 * wc.grid.n_phi

    # second transform (Section 5) on the batch's candidates: track candidates
    # with >= 300 votes as lines into 128 x 128 vertex bins of 0.5 cm
    vg = hough.VertexGridSpec(synth.VERTEX_GRID, dev)
    voff = torch.from_numpy(np.arange(n_events + 1, dtype=np.int64) * vg.max_candidates()).to(dev)
    coff = torch.from_numpy(cand_off).to(dev)
    vout = torch.empty((n_events * vg.max_candidates(), 2), dtype=torch.int32, device=dev)
    n_vtx = torch.empty(n_events, dtype=torch.int32, device=dev)

    def vstep():
        ctx.vertices(vg, cands, coff, n_found, VERTEX_TRACK_THRESHOLD, VERTEX_THRESHOLD, vout=vout, vout_off=voff,
                     n_vertices=n_vtx)

    for _ in range(3):
        vstep()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        vstep()
    ev1.record()
    torch.cuda.synchronize()
    v_ms = ev0.elapsed_time(ev1) / reps
    cv = cands[:, 0].cpu().numpy()
    nf = n_found.cpu().numpy()
    lines = sum(int((cv[cand_off[e]:cand_off[e] + min(int(nf[e]), cap)] >= VERTEX_TRACK_THRESHOLD).sum())
                for e in range(n_events))
    vertices = {"track_threshold": VERTEX_TRACK_THRESHOLD, "vertex_threshold": VERTEX_THRESHOLD,
                "grid": [vg.n_x, vg.n_y], "lines_per_event": lines // n_events,
                "ms_per_launch": v_ms, "ms_per_event": v_ms / n_events,
                "vertex_candidates_per_event": int(n_vtx.sum().item()) // n_events}
    return {"workload": "displaced_3d_35k_64x512x256_u16", "events": n_events, "hits": int(b.n_hits),
            "ms_per_event": 1e3 * dt / n_events, "events_per_s": n_events / dt,
            "vote_ms_per_event": float(np.mean(vote[1:])) / n_events,
            "evaluations_per_s": evals / dt, "votes_per_event": int(n_votes.sum().item()) // n_events,
            "candidates_per_event": int(n_found.sum().item()) // n_events, "vertices": vertices}


def straight_2d(hough, torch, dev, synth, log_fn, n_events=256, reps=10):
    """The straight-line family (2,000 lines and 20 % noise per event, 1024 phi0
    x 512 d0 int32, threshold 7) as one graph-replayed batch of n_events."""
    wc = synth.CONFIGS[6]
    log_fn(f"straight-line batch of {n_events}")
    b = synth.pack_events([synth.gen_config_event(6, i) for i in range(n_events)])
    x = torch.from_numpy(b.x).to(dev)
    y = torch.from_numpy(b.y).to(dev)
    ctx = hough.HoughContext(wc.grid, device=dev, max_events=n_events, max_hits=b.n_hits)
    cap = ctx.spec.max_candidates()
    cand_off = np.arange(n_events + 1, dtype=np.int64) * cap
    cands = torch.empty((n_events * cap, 2), dtype=torch.int32, device=dev)
    n_found = torch.empty(n_events, dtype=torch.int32, device=dev)
    n_votes = torch.empty(n_events, dtype=torch.int64, device=dev)

    def step():
        ctx.event_batch(b.hit_off, x, y, wc.threshold, cand_off=cand_off, cands=cands, n_found=n_found,
                        n_votes=n_votes)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.set_timing(True)
    vote = []
    for _ in range(4):
        step()
        vote.append(ctx.get_timing()[0])
    ctx.set_timing(False)
    evals = int(b.n_hits) * wc.grid.n_phi
    return {"workload": "straight_batch256_2000lines_1024x512", "events": n_events, "hits": int(b.n_hits),
            "ms_per_step": 1e3 * dt, "events_per_s": n_events / dt, "vote_ms": float(np.mean(vote[1:])),
            "evaluations_per_s": evals / dt, "votes_per_step": int(n_votes.sum().item()),
            "candidates_per_step": int(n_found.sum().item())}


def forward_2d(hough, torch, dev, synth, batch, x, y, log_fn, reps=10):
    """The batch workload (same events, grid and threshold) with the
    forward-hemisphere option: each hit votes only where it lies ahead of the
    point of closest approach, so the mirror solutions are gone."""
    import dataclasses
    wc = synth.CONFIGS[4]
    grid = dataclasses.replace(wc.grid, forward=True)
    n_events = batch.n_events
    log_fn(f"forward-hemisphere batch of {n_events}")
    ctx = hough.HoughContext(grid, device=dev, max_events=n_events, max_hits=batch.n_hits)
    cap = ctx.spec.max_candidates()
    cand_off = np.arange(n_events + 1, dtype=np.int64) * cap
    cands = torch.empty((n_events * cap, 2), dtype=torch.int32, device=dev)
    n_found = torch.empty(n_events, dtype=torch.int32, device=dev)
    n_votes = torch.empty(n_events, dtype=torch.int64, device=dev)

    def step():
        ctx.event_batch(batch.hit_off, x, y, wc.threshold, cand_off=cand_off, cands=cands, n_found=n_found,
                        n_votes=n_votes)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.set_timing(True)
    vote = []
    for _ in range(6):
        step()
        vote.append(ctx.get_timing()[0])
    ctx.set_timing(False)
    return {"workload": "forward_batch256_uneven2d_1024x512", "events": n_events, "hits": int(batch.n_hits),
            "ms_per_step": 1e3 * dt, "events_per_s": n_events / dt, "vote_ms": float(np.mean(vote[1:])),
            "votes_per_step": int(n_votes.sum().item()), "candidates_per_step": int(n_found.sum().item())}


def association_report(hough, torch, dev, synth, log_fn, reps=5):
    """Hit association of one event per workload on the device (every candidate
    at or above the threshold), timed with HIP events on the stream it runs on,
    and the truth report of its pairs: efficiency, fake rate and duplicates
    (matched candidates per found track) with the threshold as the match
    minimum.  A physics check of the workloads, not a parity figure."""
    import dataclasses
    out = []
    for name, cfg, forward in (("config1_40trk_256x128", 1, False), ("config2_pileup_1024x512", 2, False),
                               ("config2_pileup_1024x512_forward", 2, True), ("config3_displaced_3d", 3, False)):
        wc = synth.CONFIGS[cfg]
        grid = dataclasses.replace(wc.grid, forward=forward)
        ev = synth.gen_config_event(cfg)
        log_fn(f"association: {name}")
        ctx = hough.HoughContext(grid, device=dev, max_hits=ev.n_hits)
        x = torch.from_numpy(ev.x).to(dev)
        y = torch.from_numpy(ev.y).to(dev)
        acc, _ = ctx.vote(x, y)
        cands, nf = ctx.peaks(acc, wc.threshold)
        cap = 1 << 27                    # 1 GiB of pairs: the displaced event has about 108 M
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        n_pairs = torch.empty(1, dtype=torch.int64, device=dev)
        ctx.associate(x, y, cands, nf, wc.threshold, pairs=pairs, n_pairs=n_pairs)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            ctx.associate(x, y, cands, nf, wc.threshold, pairs=pairs, n_pairs=n_pairs)
        t1.record(stream)
        torch.cuda.synchronize()
        n = int(n_pairs.item())
        if n > cap:
            raise RuntimeError(f"association of {name}: {n} pairs exceed the buffer")
        got = pairs[:n].cpu().numpy().astype(np.int64)
        n_cands = int(nf.item())
        match, n_hits = synth.match_candidates(got[:, 0], got[:, 1], n_cands, ev.label, wc.threshold)
        rep = synth.efficiency(match, n_hits, ev.label, wc.threshold)
        out.append({"workload": name, "hits": ev.n_hits, "candidates": n_cands, "pairs": n,
                    "ms": t0.elapsed_time(t1) / reps, **rep})
        del pairs
    return out


def served_stream(args, hough, synth, batch, log_fn):
    """Open-loop served stream: Poisson arrivals of 80 % batch-workload 2D and
    20 % displaced 3D events at each offered rate, through the library's
    server (continuous batching, serve_lanes lanes per grid, 2 ms deadline).  The first
    serve_warmup arrivals of each rate are not measured; a deadline miss is a
    measured event that waited longer than the deadline for its launch."""
    rates = [float(r) for r in args.serve_rates.split(",") if r.strip()]
    if not rates:
        return None
    pool = list(batch.events) + [synth.gen_config_event(3, i) for i in range(32)]
    n2 = batch.n_events
    pool_grid = np.array([0] * n2 + [1] * (len(pool) - n2), np.int32)
    pool_off = np.zeros(len(pool) + 1, np.int64)
    pool_off[1:] = np.cumsum([ev.n_hits for ev in pool])
    pool_x = np.concatenate([ev.x for ev in pool])
    pool_y = np.concatenate([ev.y for ev in pool])
    grids = [synth.CONFIGS[4].grid, synth.CONFIGS[3].grid]
    thr = [synth.CONFIGS[4].threshold, synth.CONFIGS[3].threshold]
    # every event's candidates are copied back to the host before its completion time is taken
    srv = hough.Server(grids, thr, lanes=args.serve_lanes, batch_events=[64, 8], batch_hits=[1 << 22, 1 << 19],
                       deadline_ms=2.0,
                       queue_limit=4096, keep_candidates=True)
    out = []
    deadline_s = 2e-3
    try:
        for rate in rates:
            warm = max(0, args.serve_warmup)
            n = warm + max(1, args.serve_events)
            rng = np.random.default_rng(np.random.SeedSequence([synth.BASE_SEED + 5, int(rate)]))
            kind = (rng.uniform(size=n) < 0.2).astype(np.int32)
            pick = np.where(kind == 1, n2 + rng.integers(0, len(pool) - n2, size=n),
                            rng.integers(0, n2, size=n)).astype(np.int32)
            arrivals = synth.poisson_arrivals(rate, n, stream=1)
            log_fn(f"served stream: {warm} + {n - warm} events at {rate:.0f}/s")
            status = {}
            import threading
            th = threading.Thread(target=lambda: status.update(
                s=srv.replay(arrivals, pick, pool_grid, pool_off, pool_x, pool_y)))
            t_start = srv.clock()
            th.start()
            res = []
            t_wall = time.time()
            limit = 60 + 3 * n / rate
            while th.is_alive() or len(res) < n:
                res += srv.poll(wait_ms=20, cand_cap=1 << 22, with_cands=False)
                if not th.is_alive():
                    accepted = int((status["s"] == 0).sum())
                    if len(res) >= accepted:
                        break
                if time.time() - t_wall > limit:
                    raise RuntimeError(f"served stream at {rate}/s: {len(res)} of {n} events returned in time")
            th.join()
            # statistics over the measured arrivals only (tag = arrival index)
            ok = [r for r in res if r["status"] == 0 and r["tag"] >= warm]
            lat = np.array([r["t_done"] - r["t_submit"] for r in ok]) * 1e3
            wait = np.array([r["t_launch"] - r["t_submit"] for r in ok])
            t_first = t_start + float(arrivals[warm])
            span = max(r["t_done"] for r in ok) - t_first
            refused = int((status["s"][warm:] != 0).sum())
            votes = sum(int(r["n_votes"]) for r in ok)
            stored = sum(int(r["n_stored"]) for r in ok)
            found = sum(min(int(r["n_found"]), 1 << 62) for r in ok)
            out.append({"offered_per_s": rate, "warmup_events": warm, "events": n - warm, "completed": len(ok),
                        "refused": refused, "deadline_misses": int((wait > deadline_s).sum()),
                        "achieved_events_per_s": len(ok) / span, "votes_per_s": votes / span,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "mean_batch_events": float(np.mean([r["batch_events"] for r in ok])),
                        "share_3d": float(kind[warm:].mean()), "candidates_to_host": stored,
                        "candidates_found": found})
    finally:
        srv.close()
    return out


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: events are independent and the path has no cross-GPU step; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1311_2769_amd import hough

    hough.load()                                  # fails loudly if libhough.so is missing
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    wc = synth.CONFIGS[4]
    grid, thr = wc.grid, wc.threshold
    log(f"generating {args.events} events")
    batch = synth.gen_batch(4, args.events)
    n_ev = batch.n_events
    hit_off = batch.hit_off
    x = torch.from_numpy(batch.x).to(dev)
    y = torch.from_numpy(batch.y).to(dev)
    ctx = hough.HoughContext(grid, device=dev, max_events=n_ev, max_hits=batch.n_hits)
    cap = ctx.spec.max_candidates()
    cand_off = np.arange(n_ev + 1, dtype=np.int64) * cap
    cands = torch.empty((n_ev * cap, 2), dtype=torch.int32, device=dev)
    n_found = torch.empty(n_ev, dtype=torch.int32, device=dev)
    n_votes = torch.empty(n_ev, dtype=torch.int64, device=dev)

    def step():
        ctx.event_batch(hit_off, x, y, thr, cand_off=cand_off, cands=cands, n_found=n_found, n_votes=n_votes)

    # Launch shape: the autotuner times every batch shape on these resident
    # events (whole hough_event_batch calls) and keeps the fastest.
    shape = None
    tuned = {"tuned": False}
    if not args.no_tune:
        log("autotuning the batch launch shape")
        rows, threads, _, best_ms = ctx.autotune(1, hit_off, x, y, thr, cand_off=cand_off, cands=cands,
                                                 n_found=n_found, reps=5)
        shape = (rows, threads)
        tuned = {"tuned": True, "tune_best_ms": best_ms}
    rows, threads, _ = ctx.get_launch(1)
    tuned.update({"rows": rows, "threads": threads})

    # Lanes: lane 0 is ctx on the current stream; further lanes are contexts of
    # their own on streams of their own (default priority), so that one batch's
    # sort and hit preparation overlap another's vote, as in the server.
    lanes = [(ctx, torch.cuda.current_stream(), cands, n_found, n_votes)]
    for _ in range(1, max(1, args.lanes)):
        c2 = hough.HoughContext(grid, device=dev, max_events=n_ev, max_hits=batch.n_hits)
        if shape:
            c2.set_launch(1, *shape)
        lanes.append((c2, torch.cuda.Stream(device=dev), torch.empty_like(cands), torch.empty_like(n_found),
                      torch.empty_like(n_votes)))

    def lane_step(i):
        c, s, cc, nf, nv = lanes[i % len(lanes)]
        c.event_batch(hit_off, x, y, thr, cand_off=cand_off, cands=cc, n_found=nf, n_votes=nv, stream=s)

    torch.cuda.synchronize()
    log(f"warmup {args.warmup} (x {len(lanes)} lanes)")
    for i in range(args.warmup * len(lanes)):
        lane_step(i)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        lane_step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    votes = int(n_votes.sum().item())
    evals = int(batch.n_hits) * grid.n_phi * grid.n_d0
    found = int(n_found.sum().item())
    ms_step = 1e3 * dt / args.steps
    events_per_s = n_ev * args.steps / dt

    # Dominant kernel: the batch's vote kernel (fused with the peak search for
    # this grid), timed with HIP events the library records around it on the
    # stream it is launched on (timing mode launches the same kernels without
    # the graph), with the (hit, row) pairs it evaluates counted on the device.
    log("timing the vote kernel")
    k_launch = max(3, args.steps)
    ctx.set_timing(True)
    vote_list, total_list = [], []
    for _ in range(k_launch + 1):
        step()
        v_ms, t_ms = ctx.get_timing()
        vote_list.append(v_ms)
        total_list.append(t_ms)
    # the pairs the vote evaluates, counted on the device in a launch of its own
    # (counting costs an atomic per workgroup; the times above are without it)
    ctx.set_timing(2)
    step()
    pairs = ctx.get_work()
    ctx.set_timing(False)
    vote_ms = float(np.mean(vote_list[1:]))
    assert int(n_votes.sum().item()) == votes
    t_vote = vote_ms * 1e-3
    achieved = pairs * VALU_PER_PAIR_2D / t_vote
    log("throughput probes")
    lds_peak_meas, valu_peak_meas = hough.diag_rates()
    traffic, valu_insts = counter_fields(rows, threads)
    vote_rate = votes / t_vote
    roofline = {"bound": "alu", "kernel": "vote_kernel (batched, persistent, fused peak search)",
                "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12, "unit": "T VALU-ops/s",
                "frac": achieved / PEAK_VALU_OPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "work_per_launch": {"evaluated_pairs": pairs, "valu_per_pair": VALU_PER_PAIR_2D,
                                    "pairs_uncut": evals, "evaluated_share": pairs / evals, "votes": votes,
                                    "hits": int(batch.n_hits)},
                "launch_ms": vote_ms, "batch_ms_timing_mode": float(np.mean(total_list[1:])),
                "peak_measured": valu_peak_meas / 1e12, "frac_of_measured": achieved / valu_peak_meas,
                "lds_atomic": {"achieved": vote_rate / 1e12, "peak_measured": lds_peak_meas / 1e12,
                               "unit": "T atomics/s", "frac_of_measured": vote_rate / lds_peak_meas}}
    if traffic:
        roofline["hbm_gbs"] = traffic / t_vote / 1e9
    if valu_insts:
        # all VALU work of the launch (loop, staging, peak search), from the counters
        roofline["valu_issue_frac"] = valu_insts * 64 / t_vote / PEAK_VALU_OPS

    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    line_extra = {"resident": {"events_per_s": events_per_s, "ms_per_step": ms_step,
                               "note": "hits in HBM before the timed region, candidates left there"}}
    if args.e2e_steps > 0:
        e2e = end_to_end(args, hough, torch, dev, batch, grid, thr, cap, shape)
        e2e["n_found_matches_resident"] = e2e["n_found_per_step"] == found
        line_extra["with_host_transfers"] = e2e
    if not args.skip_3d:
        line_extra["displaced_3d"] = displaced_3d(hough, torch, dev, synth, log)
    if not args.skip_straight:
        line_extra["straight_2d"] = straight_2d(hough, torch, dev, synth, log)
    if not args.skip_forward:
        line_extra["forward_2d"] = forward_2d(hough, torch, dev, synth, batch, x, y, log)
    if not args.skip_assoc:
        line_extra["association"] = association_report(hough, torch, dev, synth, log)
    served = served_stream(args, hough, synth, batch, log)
    if served is not None:
        line_extra["served"] = served
        ok = [r for r in served if r["refused"] == 0 and r["achieved_events_per_s"] >= 0.97 * r["offered_per_s"]]
        if ok:
            best = max(ok, key=lambda r: r["offered_per_s"])
            line_extra["served_sustained"] = {"offered_per_s": best["offered_per_s"],
                                              "achieved_events_per_s": best["achieved_events_per_s"],
                                              "p99_ms": best["p99_ms"]}
    if not args.skip_per_event:
        pe = per_event(args, hough, torch, dev, batch, grid, thr, cap, x, y, hit_off, shape)
        best_res = max(v["resident_events_per_s"] for v in pe.values())
        best_tr = max(v["transfers_events_per_s"] for v in pe.values())
        pe["batched_speedup_resident"] = events_per_s / best_res
        if "with_host_transfers" in line_extra:
            pe["batched_speedup_with_transfers"] = line_extra["with_host_transfers"]["events_per_s"] / best_tr
        line_extra["per_event_launch"] = pe

    line = {
        "metric": "events/s (batched vote + peaks + sorted candidates, one graph per 256-event batch)",
        "value": events_per_s,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wc.name, "events_per_step": n_ev, "hits_per_step": int(batch.n_hits),
                   "grid": [grid.n_d0, grid.n_phi, grid.n_kappa], "acc": grid.acc_type, "threshold": thr,
                   "lanes": len(lanes), "launch": tuned},
        "votes_per_s": votes * args.steps / dt,
        "evals_per_s": evals * args.steps / dt,
        "candidates_per_step": found,
        "roofline": roofline,
    }
    line.update(line_extra)
    if not args.no_cpu:
        log("oracle sample on the host")
        line["cpu_baseline"] = cpu_baseline(batch, grid, thr, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
