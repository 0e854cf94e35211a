"""CPU checks of the serving loop's host logic (no device work)."""
import math

from paper_1611_03329_amd.serve import Request, Result, _done, as_requests, summarize


def test_stopping_rule():
    r = Result(0, "a", 10, 0.0)
    assert not _done(r, -1.0, -1, False, 100, 1e-6, 1000)       # no check yet
    assert not _done(r, 2e-6, 100, False, 200, 1e-6, 1000)
    assert r.residual == 2e-6 and r.checked_at == 100 and r.steps == 200
    assert _done(r, 5e-7, 200, False, 300, 1e-6, 1000) and r.converged
    r = Result(1, "b", 10, 0.0)
    assert _done(r, math.nan, 100, True, 200, 1e-6, 1000) and r.unstable and not r.converged
    r = Result(2, "c", 10, 0.0)
    assert _done(r, 1e-3, 900, False, 1000, 1e-6, 1000) and not r.converged and not r.unstable


def test_requests_sorted_by_arrival_and_summary():
    qs = as_requests([(0.3, {"name": "x"}), (0.1, {"name": "y"})])
    assert [q.workload["name"] for q in qs] == ["y", "x"] and [q.rid for q in qs] == [0, 1]
    res = []
    for i in range(100):
        r = Result(i, "", 1000, arrival=0.01 * i, finished=0.01 * i + 1.0 + 0.01 * i, steps=200)
        r.converged = True
        res.append(r)
    s = summarize(res)
    assert s["converged"] == 100 and s["capped"] == 0
    assert abs(s["p50_s"] - (1.0 + 0.01 * 49.5)) < 1e-9
    assert abs(s["makespan_s"] - (0.99 + 1.99)) < 1e-9
    assert abs(s["mlups"] - 100 * 1000 * 200 / (0.99 + 1.99) / 1e6) < 1e-9
    assert isinstance(Request(0, 0.0, {}), Request)


def test_capped_solves_are_not_counted_as_solves():
    """A solve stopped at the step cap (or unstable) counts in `capped`
    (`unstable`), not in solves/s nor in the time-to-converge percentiles; its
    node updates still count in MLUPS."""
    res = []
    for i in range(4):
        r = Result(i, "", 1000, arrival=0.0, finished=1.0 + i, steps=100)
        r.converged = i < 2
        r.unstable = i == 3
        res.append(r)
    s = summarize(res)
    assert (s["converged"], s["capped"], s["unstable"]) == (2, 1, 1)
    assert abs(s["makespan_s"] - 4.0) < 1e-12
    assert abs(s["solves_per_s"] - 2 / 4.0) < 1e-12
    assert abs(s["p99_s"] - (1.0 + 0.99)) < 1e-12          # over the converged latencies 1 and 2
    assert abs(s["mlups"] - 4 * 1000 * 100 / 4.0 / 1e6) < 1e-12


def test_reservations_cover_every_move():
    """A solve reserves, at each ladder level, the largest sum of two
    consecutive precisions it may still hold at once; the reservation never
    grows as it moves on."""
    from paper_1611_03329_amd.serve import reserve_bytes
    b16, b32, b64 = 136, 208, 416
    assert reserve_bytes([b32], 0) == b32
    assert reserve_bytes([b16, b32], 0) == b16 + b32 and reserve_bytes([b16, b32], 1) == b32
    ladder = [b16, b32, b64]
    assert [reserve_bytes(ladder, k) for k in range(3)] == [b32 + b64, b32 + b64, b64]
    assert reserve_bytes([b32, b64], 0) == b32 + b64 and reserve_bytes([b32, b64], 1) == b64


def test_admission_policies():
    """First come first served admits only the head of the queue; smallest
    first takes the fitting request with the fewest nodes; a node cap holds
    requests back unless nothing is resident."""
    from paper_1611_03329_amd.serve import pick_admission
    qs = [Request(0, 0.0, {}), Request(1, 0.1, {}), Request(2, 0.2, {})]
    need = {0: {"admit": 800, "nodes": 8000}, 1: {"admit": 100, "nodes": 1000}, 2: {"admit": 300, "nodes": 3000}}
    # budget 1000, 500 bytes in use: the head (800) does not fit
    assert pick_admission(qs, need, "fcfs", 1, 5000, 500, 1000, 10, None) is None
    assert pick_admission(qs, need, "smallest", 1, 5000, 500, 1000, 10, None).rid == 1
    # nothing in use: fcfs takes the head, smallest the smallest
    assert pick_admission(qs, need, "fcfs", 0, 0, 0, 1000, 10, None).rid == 0
    assert pick_admission(qs, need, "smallest", 0, 0, 0, 1000, 10, None).rid == 1
    # node cap 4500 with 2000 resident: 1 (1000) fits, 2 (3000) does not
    assert pick_admission(qs[2:], need, "smallest", 1, 2000, 0, 10_000, 10, 4500) is None
    assert pick_admission(qs[1:], need, "smallest", 1, 2000, 0, 10_000, 10, 4500).rid == 1
    # an empty GPU takes a request larger than the cap
    assert pick_admission(qs[:1], need, "smallest", 0, 0, 0, 10_000, 10, 4500).rid == 0
    # no free member slot
    assert pick_admission(qs, need, "smallest", 3, 0, 0, 10_000, 3, None) is None
    # ties by arrival
    need2 = {0: {"admit": 1, "nodes": 5}, 1: {"admit": 1, "nodes": 5}}
    assert pick_admission(qs[:2], need2, "smallest", 0, 0, 0, 10, 10, None).rid == 0
