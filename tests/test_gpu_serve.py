"""GPU tests of the serving loop: continuous batching of steady-state solves
with HBM-budget admission and graph-replayed chunks.  Served solves must match
the FP64 oracle stepped the same number of steps (FP32 within 1e-5; FP16
storage with the FP32 finish: Nu within 1e-3); every result must be the same
alone and in the mix (steps to converge, residual and Nusselt numbers bit for
bit), and the same as the sequential baseline in the same precision."""
import sys

import numpy as np
import pytest

import lbm_inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_03329_amd import make_params, required_bytes  # noqa: E402
from paper_1611_03329_amd.serve import Request, Server, solve_sequential, summarize  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests():
    """Six small cavities of uneven sizes and parameters, arriving within 20 ms."""
    draws = [((16, 16, 16), 0.4, 1e-2, 2e3), ((20, 18, 14), 0.7, 1e-3, 5e3), ((12, 12, 12), 0.9, 1e-1, 1e3),
             ((24, 16, 20), 0.5, 1e-4, 1e4), ((14, 22, 18), 0.6, 5e-2, 3e3), ((18, 18, 18), 0.3, 1e-2, 8e3)]
    out = []
    for i, (shape, phi, da, ra) in enumerate(draws):
        wl = lbm_inputs.cavity(shape, porosity=phi, darcy=da, rayleigh=ra, seed=40 + i)
        wl["name"] = f"req{i}"
        out.append(Request(i, 0.004 * i, wl))
    return out


KW = dict(check_interval=100, tol=1e-6, max_steps=30000)


def _field_errors(fl, ref):
    """Max-norm errors of rho, u, T relative to each field's scale; the three
    velocity components share the scale max|u| of the velocity vector."""
    umax = float(np.max(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2 + ref["uz"] ** 2)))
    out = {}
    for k in ("rho", "ux", "uy", "uz", "T"):
        scale = umax if k in ("ux", "uy", "uz") else float(np.max(np.abs(ref[k])))
        out[k] = float(np.max(np.abs(np.asarray(fl[k]) - ref[k])) / (scale if scale > 0 else 1.0))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_served_solves_match_the_oracle(prec):
    """Three cavities (16^3, 12^3, 24x16x20) served together to residual 1e-6,
    each against the FP64 oracle stepped as many steps as the served solve
    took (Nu of Eqs. 53-55 at both isothermal walls, fields element by
    element).  FP32: every field within 1e-5 of its scale and Nu within 1e-5.
    FP16 storage with the FP32 finish (the state moved by lbm_transfer_state):
    Nu within 1e-3, the FP16 target; its fields carry the FP16 phase's
    rounding noise, which the FP32 finish relaxes (bound 1e-3)."""
    reqs = [_requests()[i] for i in (0, 2, 3)]
    _say(f"case served solves vs oracle {prec}: {[q.workload['name'] for q in reqs]}")
    with Server(prec, graph=True, keep_fields=True, **KW) as srv:
        res = srv.run(reqs)
    for q, r in zip(reqs, res):
        assert r.converged, (q.rid, r.residual, r.steps)
        assert (r.promoted_at > 0) == (prec == "fp16"), (q.rid, r.promoted_at)
        with oracle.Oracle(q.workload) as o:
            o.step(r.steps)
            ref, nu_ref = o.fields(), o.nusselt()
        errs = _field_errors(r.fields, ref)
        e_nu = [abs(r.nu[fc] - nu_ref[fc]) / abs(nu_ref[fc]) for fc in (0, 1)]
        _say(f"{prec} {q.workload['name']} steps {r.steps} (fp16 until {r.promoted_at}): fields {errs} Nu {e_nu}")
        bound_f, bound_nu = (1e-5, 1e-5) if prec == "fp32" else (1e-3, 1e-3)
        for k, err in errs.items():
            assert err <= bound_f, (q.rid, k, err)
        assert max(e_nu) <= bound_nu, (q.rid, e_nu)


def test_escalation_to_fp64_below_the_fp32_floor():
    """A tolerance below what FP32 storage can reach (1e-10): with escalation
    the server moves each solve to FP64 once its FP32 residual stalls, and the
    solve converges; its Nu then matches the FP64 oracle stepped as many steps
    (the FP32 phase's rounding relaxed away), and each result is the same
    alone and in the mix."""
    reqs = [_requests()[i] for i in (0, 2)]
    kw = dict(check_interval=100, tol=1e-10, max_steps=80000, escalate=True, plateau_fp32=(0.9, 5))
    _say("case escalation fp32 -> fp64, tol 1e-10")
    with Server("fp32", **kw) as srv:
        mix = srv.run(reqs)
        assert srv.stats["escalated"] == len(reqs)
    for q, m in zip(reqs, mix):
        assert m.converged and m.escalated_at > 0, (q.rid, m.residual, m.steps, m.escalated_at)
        with oracle.Oracle(q.workload) as o:
            o.step(m.steps)
            nu_ref = o.nusselt()
        e_nu = abs(m.nu[0] - nu_ref[0]) / abs(nu_ref[0])
        _say(f"{q.workload['name']}: steps {m.steps}, fp64 from {m.escalated_at}, Nu rel {e_nu:.2e}")
        assert e_nu <= 1e-8, e_nu
        with Server("fp32", **kw) as srv1:
            (a,) = srv1.run([Request(q.rid, 0.0, q.workload)])
        assert ((a.steps, a.checked_at, a.residual, a.nu, a.escalated_at)
                == (m.steps, m.checked_at, m.residual, m.nu, m.escalated_at)), q.rid


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_results_are_the_same_alone_and_in_the_mix(prec):
    reqs = _requests()
    _say(f"case serve mix vs alone {prec}: {len(reqs)} requests")
    with Server(prec, graph=True, **KW) as srv:
        mix = srv.run(reqs)
        assert srv.stats["peak_members"] >= 2
    for q, m in zip(reqs, mix):
        assert m.converged, (q.rid, m.residual, m.steps)
        # FP16 storage stalls above the tolerance: every solve finishes in FP32
        assert (m.promoted_at > 0) == (prec == "fp16"), (q.rid, m.promoted_at)
        with Server(prec, graph=True, **KW) as srv1:
            (a,) = srv1.run([Request(q.rid, 0.0, q.workload)])
        assert ((a.steps, a.checked_at, a.residual, a.nu, a.promoted_at)
                == (m.steps, m.checked_at, m.residual, m.nu, m.promoted_at)), q.rid
    s = summarize(mix)
    _say(f"{prec}: {s}")
    assert s["converged"] == len(reqs)


def test_served_fp32_equals_sequential_fp32():
    """Same precision: the served and the sequential solve take the same number
    of steps and give the same Nusselt numbers (the states are identical; the
    residuals differ at most by summation order)."""
    reqs = _requests()
    _say("case serve vs sequential fp32")
    with Server("fp32", graph=False, **KW) as srv:
        mix = srv.run(reqs)
    seq = solve_sequential(reqs, "fp32", **KW)
    for m, s in zip(mix, seq):
        assert m.converged and s.converged
        assert m.steps == s.steps and m.checked_at == s.checked_at, (m.rid, m.steps, s.steps)
        assert m.nu == s.nu
        assert abs(m.residual - s.residual) <= 1e-9 * s.residual


def test_admission_respects_the_hbm_budget():
    """With room for about two of the requests at a time the server never holds
    more than the budget, and still completes every request."""
    reqs = _requests()
    need = sorted(required_bytes(make_params(q.workload, "fp32", 100)) for q in reqs)
    budget = need[-1] + need[-2]
    _say(f"case admission budget {budget} B")
    with Server("fp32", hbm_budget=budget, **KW) as srv:
        res = srv.run(reqs)
        assert srv.stats["peak_bytes"] <= budget
        assert srv.stats["peak_members"] <= 3
    assert all(r.converged for r in res)
    # first come, first served: admission times follow arrival order
    adm = [r.admitted for r in sorted(res, key=lambda r: r.arrival)]
    assert adm == sorted(adm)


def test_fp16_promotion_respects_the_budget():
    """An FP16 solve is admitted with room for its FP32 copy, so its move never
    waits and the reservations never exceed the budget."""
    reqs = _requests()
    both = sorted(sum(required_bytes(make_params(q.workload, p, 100)) for p in ("fp16", "fp32")) for q in reqs)
    budget = both[-1] + both[-2]
    _say(f"case fp16 promotion budget {budget} B")
    with Server("fp16", hbm_budget=budget, **KW) as srv:
        res = srv.run(reqs)
        assert srv.stats["peak_bytes"] <= budget
        assert srv.stats["promoted"] == len(reqs)
    assert all(r.converged for r in res)


def test_smallest_first_under_a_node_cap():
    """Smallest first with a resident-node cap of two small requests: the
    requests are admitted in order of size, the cap holds, and every result
    is still the one the request gets alone (fp32, bit for bit)."""
    reqs = _requests()
    sizes = sorted(q.workload["nx"] * q.workload["ny"] * q.workload["nz"] for q in reqs)
    cap = sizes[0] + sizes[1]
    _say(f"case smallest first, node cap {cap}")
    with Server("fp32", policy="smallest", max_nodes=cap, **KW) as srv:
        res = srv.run(reqs)
    assert all(r.converged for r in res)
    # every request after the first was admitted when it fitted the cap; the
    # order of admission is the order of size among those waiting
    order = [r.nodes for r in sorted(res, key=lambda r: r.admitted)]
    assert order[1:] == sorted(order[1:]) or order == sorted(order), order
    with Server("fp32", **KW) as srv2:
        ref = srv2.run(reqs)
    for a, b in zip(res, ref):
        assert (a.steps, a.checked_at, a.residual, a.nu) == (b.steps, b.checked_at, b.residual, b.nu), a.rid
