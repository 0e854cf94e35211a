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
