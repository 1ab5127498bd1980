"""The served stream's dispatch policy on the CPU (no GPU): the policy header
the server uses, driven by tests/dispatch_sim.cpp with a simulated clock and
a fake executor (a batch keeps its lane busy for a + b * hits seconds).

Checked: an idle grid launches at once; while a lane of the grid is busy a
free lane waits for the deadline, half a pool of hits or full event slots;
batches keep arrival order and respect slots and pool; every admitted event
is launched exactly once; grids do not wait for each other; refusals at
submit; stopping flushes what waits.
"""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1311_2769_amd", "csrc")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("dispatch") / "dispatch_sim")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "dispatch_sim.cpp")], check=True)

    def run(lines):
        res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=60)
        log = []
        for ln in res.stdout.splitlines():
            f = ln.split()
            kind, t = f[0], float(f[1])
            if kind == "launch":
                log.append(("launch", t, int(f[2]), int(f[3]), [int(v) for v in f[4:]]))
            elif kind == "done":
                log.append(("done", t, int(f[2])))
            elif kind == "refuse":
                log.append(("refuse", t, int(f[2]), f[3]))
            else:
                log.append((kind, t))
        assert res.returncode == 0 and log[-1][0] == "end", res.stdout[-500:]
        return log
    return run


def launches(log):
    return [e for e in log if e[0] == "launch"]


def test_idle_grid_launches_at_arrival(sim):
    log = sim(["deadline 0.002", "service 0.001 0", "lane 0 8 1000", "lane 0 8 1000", "event 0.0005 0 10"])
    assert launches(log) == [("launch", 0.0005, 0, 0, [0])]


def test_busy_grid_waits_for_the_deadline(sim):
    # lane 0 is busy with event 0 until 0.010; events 1, 2 arrive and wait for
    # the 2 ms deadline of the oldest (1 at 0.001), then go out together on lane 1
    log = sim(["deadline 0.002", "service 0.010 0", "lane 0 8 1000", "lane 0 8 1000",
               "event 0.0 0 10", "event 0.001 0 10", "event 0.0015 0 10"])
    L = launches(log)
    assert L[0] == ("launch", 0.0, 0, 0, [0])
    assert L[1][2:] == (1, 0, [1, 2]) and L[1][1] == pytest.approx(0.003)


def test_half_a_pool_or_full_slots_launch_before_the_deadline(sim):
    # half a pool: waiting hits reach 500 of 1000 at the third event
    log = sim(["deadline 0.010", "service 0.050 0", "lane 0 8 1000", "lane 0 8 1000",
               "event 0.0 0 10", "event 0.001 0 200", "event 0.002 0 200", "event 0.003 0 100"])
    L = launches(log)
    assert L[1][1] == pytest.approx(0.003) and L[1][4] == [1, 2, 3]
    # full slots: the fourth waiting event fills 4 slots
    log = sim(["deadline 0.010", "service 0.050 0", "lane 0 4 1000", "lane 0 4 1000",
               "event 0.0 0 1"] + [f"event {0.001 * k} 0 1" for k in range(1, 6)])
    L = launches(log)
    assert L[1][1] == pytest.approx(0.004) and L[1][4] == [1, 2, 3, 4]


def test_batches_keep_order_slots_and_pool_and_launch_each_event_once(sim):
    import numpy as np
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.exponential(1 / 4000.0, size=400))
    hits = rng.integers(1, 600, size=400)
    grid = (rng.uniform(size=400) < 0.25).astype(int)
    lines = ["deadline 0.002", "service 0.0002 0.000001", "queue_limit 100000",
             "lane 0 6 1500", "lane 0 6 1500", "lane 1 3 1200", "lane 1 3 1200"]
    lines += [f"event {t[i]:.9f} {grid[i]} {hits[i]}" for i in range(400)]
    log = sim(lines)
    seen = []
    per_grid_order = {0: [], 1: []}
    for _, when, lane, g, ids in launches(log):
        assert ids, "empty batch"
        cap_e, cap_h = (6, 1500) if g == 0 else (3, 1200)
        assert len(ids) <= cap_e and sum(int(hits[i]) for i in ids) <= cap_h
        assert all(grid[i] == g for i in ids)
        assert all(round(float(t[i]), 9) <= when + 1e-9 for i in ids)
        per_grid_order[g] += ids
        seen += ids
    assert sorted(seen) == list(range(400))
    for g, ids in per_grid_order.items():
        assert ids == sorted(ids), f"grid {g} reordered"
    # a lane never runs two batches at once
    busy = {}
    for e in log:
        if e[0] == "launch":
            assert not busy.get(e[2]), "launch on a busy lane"
            busy[e[2]] = True
        elif e[0] == "done":
            busy[e[2]] = False


def test_grids_do_not_wait_for_each_other(sim):
    # grid 0's only lane is busy for a long time; grid 1's event goes out at arrival
    log = sim(["deadline 0.002", "service 0.100 0", "lane 0 4 1000", "lane 1 4 1000",
               "event 0.0 0 10", "event 0.001 0 10", "event 0.0012 1 10"])
    L = launches(log)
    assert ("launch", 0.0012, 1, 1, [2]) in L
    assert L[-1][4] == [1] and L[-1][1] == pytest.approx(0.1)   # grid 0's second event after its lane frees


def test_refusals_at_submit(sim):
    log = sim(["deadline 0.002", "service 0.050 0", "queue_limit 2", "lane 0 1 100",
               "event 0.0 0 101", "event 0.001 0 10", "event 0.002 0 10", "event 0.003 0 10",
               "event 0.004 0 10", "event 0.005 7 10"])
    ref = [(e[2], e[3]) for e in log if e[0] == "refuse"]
    assert (0, "never_fits") in ref and (5, "never_fits") in ref
    # lane busy with event 1 from 0.001: events 2 and 3 wait, 4 finds the queue full
    assert (4, "queue_full") in ref
    assert sorted(i for L in launches(log) for i in L[4]) == [1, 2, 3]


def test_stopping_flushes_what_waits(sim):
    log = sim(["deadline 10.0", "service 0.050 0", "lane 0 8 1000", "lane 0 8 1000", "stop 0.020",
               "event 0.0 0 10", "event 0.001 0 10", "event 0.002 0 10"])
    L = launches(log)
    assert L[1][1] == pytest.approx(0.020) and L[1][4] == [1, 2]
