"""Steady-state solve serving on one GPU: continuous batching of lattice
solves behind the batch entry points of the C ABI.

A request is one porous-cavity (or channel) workload to be run until its
residual r (the relative change of u and of theta over one step, checked every
K steps on the GPU) falls below a tolerance.  The server

  * admits arrived requests while their device bytes (lbm_required_bytes) fit
    the HBM budget, a member slot is free and (optionally) the resident nodes
    stay under a cap: first come, first served, or smallest first (the
    request with the fewest nodes that fits, a shortest-job-first proxy that
    lets short solves pass long ones when the GPU is oversubscribed);
  * keeps every admitted state resident in device memory and steps all of
    them together, one batch launch per time step, K steps per host
    round-trip (replayed from a HIP graph when enabled);
  * retires a member as soon as a check finds it converged (or unstable, or
    past the step cap), reads its Nusselt numbers and frees its memory, which
    lets the next waiting request in.

Admission and retirement happen only between chunks of K steps, where the
batch's step counter is a multiple of K; a new lattice (time 0) then joins with
its checks on the same member times as when it runs alone, so every result -
steps to converge, residual, Nusselt numbers, state - is bit for bit the same
alone and in any mix.

``solve_sequential`` is the baseline: the same requests one after another,
each on its own lattice with lbm_step, in plain FP32 by default.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import torch

from .lbm import Batch, Lattice, make_params, required_bytes


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    workload: dict


@dataclasses.dataclass
class Result:
    rid: int
    name: str
    nodes: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0          # time steps the lattice took
    checked_at: int = -1    # member time of the last residual check
    residual: float = -1.0
    converged: bool = False
    unstable: bool = False
    nu: tuple = ()          # face Nusselt numbers at retirement
    promoted_at: int = -1   # steps taken in FP16 storage before the move to FP32
    escalated_at: int = -1  # steps taken before the move from FP32 to FP64 storage
    fields: dict | None = None  # rho, ux, uy, uz, T at retirement (host arrays), if kept

    @property
    def latency(self) -> float:
        """Time to converge: arrival to retirement, queueing included."""
        return self.finished - self.arrival


def as_requests(stream) -> list:
    """(arrival_seconds, workload) pairs -> Request list in arrival order."""
    return [Request(i, float(t), wl) for i, (t, wl) in enumerate(sorted(stream, key=lambda p: p[0]))]


def _done(res: Result, r: float, at: int, unstable: bool, steps: int, tol: float, max_steps: int) -> bool:
    res.steps = steps
    if at >= 0:
        res.checked_at, res.residual = at, r
    if unstable:
        res.unstable = True
        return True
    if at > 0 and r < tol:
        res.converged = True
        return True
    return steps >= max_steps


class Server:
    """Continuous-batching solve server on the current device.

    precision "fp32": every solve in FP32 storage, checked every
    `check_interval` steps with the one-step residual.

    precision "fp16": a solve starts in FP16 storage (132 instead of 208 bytes
    per node and step).  FP16 rounding of the stored populations puts a floor
    under the one-step residual (about 2e-4 to 7e-3 relative on the cavity
    workloads), reached within the first few thousand steps, after the fast
    transient.  When the residual stops falling (no new low by the factor
    plateau[0] within plateau[1] checks) the solve moves to FP32 storage
    (lbm_transfer_state, exact) and finishes there.  Moving early matters: an
    FP16 run kept going drifts towards the FP16 map's own fixed point, whose
    distance from the FP32 one the FP32 finish then has to relax away.  The
    move is decided from the solve's own residuals at a check boundary, and
    the FP32 lattice starts its own check schedule at time 0, so results stay
    independent of the mix.

    escalate=True: a solve whose FP32 residual stops falling just above the
    tolerance (no new low by the factor plateau_fp32[0] within plateau_fp32[1]
    checks while its lowest residual is below plateau_fp32[2] times the
    tolerance: by default 1 % in 100 checks within 10x the tolerance) moves on
    to FP64 storage and finishes there.  The level condition keeps transient
    bumps of the residual, far above the tolerance, from moving solves that
    FP32 finishes by itself.  FP32 rounding puts
    a floor under the one-step residual too, far lower than FP16's but, on
    nearly stagnant flows (strong Darcy drag, low Ra), above 1e-6.  A solve
    reserves at admission the bytes of the largest pair of consecutive
    precisions it may hold at once, so its moves never wait for memory.

    Every batch advances `check_interval` steps per round trip; admission and
    retirement happen between these chunks."""

    def __init__(self, precision: str = "fp32", check_interval: int = 100, tol: float = 1e-6,
                 max_steps: int = 200_000, hbm_budget: int | None = None, max_members: int = 256,
                 graph: bool = True, launch: tuple | None = None, plateau: tuple = (0.9, 5), device=None,
                 policy: str = "fcfs", max_nodes: int | None = None, keep_fields: bool = False,
                 escalate: bool = False, plateau_fp32: tuple = (0.99, 100, 10.0), class_blocks: dict | None = None):
        if check_interval <= 0 or check_interval % 2:
            raise ValueError("check_interval must be a positive even number (chunks keep the parity)")
        if precision not in ("fp32", "fp16"):
            raise ValueError("precision must be fp32 or fp16")
        if policy not in ("fcfs", "smallest"):
            raise ValueError("policy must be fcfs or smallest")
        self.policy = policy
        # keep every retired solve's final fields (host copies) in its Result
        self.keep_fields = bool(keep_fields)
        # cap on the nodes resident at once (None: only the HBM budget limits);
        # a request larger than the cap still runs, alone
        self.max_nodes = None if max_nodes is None else int(max_nodes)
        self.precision = precision
        self.K = int(check_interval)
        self.chunk = self.K
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.plateau = (float(plateau[0]), int(plateau[1]))
        # the precisions a solve goes through, and the plateau rule that moves
        # it on from each but the last
        self.ladder = (["fp16"] if precision == "fp16" else []) + ["fp32"] + (["fp64"] if escalate else [])
        # (factor, checks, level): move on after `checks` checks without a new
        # low by `factor`, once the lowest residual is below level x tol
        self.plateaus = {"fp16": (self.plateau[0], self.plateau[1], math.inf),
                         "fp32": (float(plateau_fp32[0]), int(plateau_fp32[1]),
                                  float(plateau_fp32[2]) if len(plateau_fp32) > 2 else math.inf)}
        self.device = torch.device("cuda") if device is None else torch.device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.hbm_budget = int(hbm_budget)
        self.max_members = int(max_members)
        # one batch per storage precision, each on a stream of its own
        self.batches = {p: Batch(self.K, graph=graph, device=self.device) for p in self.ladder}
        if launch is not None:
            for b in self.batches.values():
                b.set_launch(*launch)
        # threads per tile by member size class, e.g. as the autotuner chose them
        for k, blk in (class_blocks or {}).items():
            for b in self.batches.values():
                b.set_class_block(k, blk)
        self.stats = {"chunks": 0, "lattice_steps": 0, "node_steps": 0, "peak_members": 0, "peak_bytes": 0,
                      "promoted": 0, "escalated": 0}

    def close(self):
        for b in self.batches.values():
            b.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run(self, requests: list, clock=time.perf_counter, progress=None, progress_every: float = 30.0) -> list:
        """Serves `requests` (arrival times relative to the call) to completion;
        returns one Result per request, in request order.  `progress`, if
        given, is called with a one-line status after every retirement and,
        between retirements, at least every `progress_every` seconds."""
        ladder = self.ladder
        first = ladder[0]
        pending = deque(sorted(requests, key=lambda q: q.arrival))
        need = {}

        def reserve(rid, level):
            return reserve_bytes([need[rid][p] for p in ladder], level)

        for q in requests:
            need[q.rid] = {p: required_bytes(make_params(q.workload, p, self.K)) for p in ladder}
            need[q.rid]["admit"] = reserve(q.rid, 0)
            need[q.rid]["nodes"] = q.workload["nx"] * q.workload["ny"] * q.workload["nz"]
            if need[q.rid]["admit"] > self.hbm_budget:
                raise ValueError(f"request {q.rid} needs more than the HBM budget")
        waiting = deque()
        active = {}   # id(lattice) -> entry
        results = {}
        used = 0
        t0 = clock()
        last_note = t0

        def next_admission():
            return pick_admission(list(waiting), need, self.policy, len(active),
                                  sum(e["lat"].nodes for e in active.values()), used,
                                  self.hbm_budget, self.max_members, self.max_nodes)

        def retire(lat, e):
            nonlocal used
            res = e["res"]
            if not res.unstable:
                res.nu = tuple(lat.nusselt())
                if self.keep_fields:
                    res.fields = {k: v.cpu().numpy() for k, v in lat.fields().items()}
            res.finished = clock() - t0
            lat.close()
            del active[id(lat)]
            used -= e["bytes"]
            results[res.rid] = res
            if progress is not None:
                progress(f"{len(results)}/{len(requests)} done at {res.finished:.1f}s: {res.name} "
                         f"steps {res.steps} r {res.residual:.2e} active {len(active)}")

        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission, between chunks
            while True:
                q = next_admission()
                if q is None:
                    break
                waiting.remove(q)
                lat = Lattice(q.workload, first, device=self.device)
                self.batches[first].add(lat)
                res = Result(q.rid, q.workload.get("name", ""), lat.nodes, q.arrival, admitted=clock() - t0)
                active[id(lat)] = {"lat": lat, "res": res, "bytes": need[q.rid]["admit"], "q": q, "prec": first,
                                   "level": 0, "base": 0, "best": math.inf, "since": 0}
                used += need[q.rid]["admit"]
            self.stats["peak_members"] = max(self.stats["peak_members"], len(active))
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            for b in self.batches.values():
                if len(b):
                    b.step(self.chunk)
            self.stats["chunks"] += 1
            if progress is not None and clock() - last_note >= progress_every:
                last_note = clock()
                progress(f"{last_note - t0:.0f}s: {len(active)} active, {len(results)}/{len(requests)} done, "
                         f"longest at step {max(e['base'] + e['lat'].time for e in active.values())}")
            self.stats["lattice_steps"] += self.chunk * len(active)
            self.stats["node_steps"] += self.chunk * sum(e["lat"].nodes for e in active.values())
            promote, done = [], []
            for prec, b in self.batches.items():
                if not len(b):
                    continue
                r, at, un = b.residuals()
                for lat, rr, aa, uu in list(zip(list(b.members), r, at, un)):
                    e = active[id(lat)]
                    res = e["res"]
                    steps = e["base"] + lat.time
                    if _done(res, rr, aa, uu, steps, self.tol, self.max_steps):
                        b.remove(lat)
                        done.append((lat, e))
                    elif e["level"] + 1 < len(ladder) and aa > 0:
                        # the precision's floor: no new low by the factor within the last checks
                        factor, checks, level = self.plateaus[prec]
                        if rr < e["best"] * factor:
                            e["best"], e["since"] = rr, 0
                        else:
                            e["since"] += 1
                        if e["since"] >= checks and e["best"] < level * self.tol:
                            promote.append(lat)
            # the retiring solves' Nusselt reductions start together; the first
            # collection waits for all of them
            for lat, e in done:
                if not e["res"].unstable:
                    lat.nusselt_start()
            for lat, e in done:
                retire(lat, e)
            for lat in promote:
                e = active[id(lat)]
                level = e["level"] + 1
                nxt = ladder[level]
                new = Lattice(e["q"].workload, nxt, device=self.device)
                new.transfer_from(lat)
                self.batches[e["prec"]].remove(lat)
                if e["prec"] == "fp16":
                    e["res"].promoted_at = e["base"] + lat.time
                    self.stats["promoted"] += 1
                else:
                    e["res"].escalated_at = e["base"] + lat.time
                    self.stats["escalated"] += 1
                e["base"] += lat.time
                lat.close()
                del active[id(lat)]
                self.batches[nxt].add(new)
                # the reservation shrinks to what the remaining moves need
                nb = reserve(e["q"].rid, level)
                used -= e["bytes"] - nb
                e.update(lat=new, bytes=nb, prec=nxt, level=level, best=math.inf, since=0)
                active[id(new)] = e
        return [results[q.rid] for q in requests]


def reserve_bytes(sizes: list, level: int) -> int:
    """Device bytes a solve reserves at ladder level `level`, given its
    lattice's bytes at each precision of the ladder: the largest pair of
    consecutive precisions it may still hold at once (a move copies the old
    state into the new lattice before the old one is freed)."""
    return max(sizes[j] + (sizes[j + 1] if j + 1 < len(sizes) else 0) for j in range(level, len(sizes)))


def pick_admission(waiting: list, need: dict, policy: str, n_active: int, resident_nodes: int, used: int,
                   budget: int, max_members: int, max_nodes: int | None):
    """The waiting request (arrival order) to admit next, or None.  need[rid]
    holds its bytes to reserve ("admit") and its nodes.  A request fits while
    a member slot is free, its bytes fit the budget and, with a node cap, the
    resident nodes stay under the cap (a request alone always fits the cap).
    "fcfs" admits the head of the queue only; "smallest" the fitting request
    with the fewest nodes (ties: earliest arrival)."""
    def fits(q) -> bool:
        if n_active >= max_members or used + need[q.rid]["admit"] > budget:
            return False
        return max_nodes is None or n_active == 0 or resident_nodes + need[q.rid]["nodes"] <= max_nodes

    if not waiting:
        return None
    if policy == "fcfs":
        return waiting[0] if fits(waiting[0]) else None
    for q in sorted(waiting, key=lambda q: (need[q.rid]["nodes"], q.arrival)):
        if fits(q):
            return q
    return None


def solve_sequential(requests: list, precision: str = "fp32", check_interval: int = 100, tol: float = 1e-6,
                     max_steps: int = 200_000, clock=time.perf_counter, device=None, progress=None) -> list:
    """The baseline: each request alone on its own lattice (lbm_step), one after
    another in arrival order, with the same check schedule and stopping rule."""
    K = int(check_interval)
    device = torch.device("cuda") if device is None else torch.device(device)
    out = []
    t0 = clock()
    for q in sorted(requests, key=lambda q: q.arrival):
        now = clock() - t0
        if q.arrival > now:
            time.sleep(q.arrival - now)
        lat = Lattice(q.workload, precision, check_interval=K, device=device)
        res = Result(q.rid, q.workload.get("name", ""), lat.nodes, q.arrival, admitted=clock() - t0)
        last_note = clock()
        while True:
            if progress is not None and clock() - last_note >= 30.0:
                last_note = clock()
                progress(f"{last_note - t0:.0f}s: {res.name} at step {lat.time}")
            lat.step(K)
            lat.stream.synchronize()
            try:
                r, at = lat.residual()
                un = False
            except Exception as e:  # the residual check found the lattice unstable
                if getattr(e, "status", None) != 4:
                    raise
                r, at, un = math.nan, lat.time - K, True
            if _done(res, r, at, un, lat.time, tol, max_steps):
                break
        if not res.unstable:
            res.nu = tuple(lat.nusselt())
        res.finished = clock() - t0
        lat.close()
        out.append(res)
        if progress is not None:
            progress(f"{len(out)}/{len(requests)} done at {res.finished:.1f}s: {res.name} steps {res.steps} "
                     f"r {res.residual:.2e}")
    order = {q.rid: i for i, q in enumerate(requests)}
    return sorted(out, key=lambda r: order[r.rid])


def summarize(results: list) -> dict:
    """One run's figures.  Throughput and time to converge count the converged
    solves only (a solve stopped at the step cap or found unstable is no
    solve); their numbers are reported beside.  p50/p99 are taken over the
    converged solves' times from arrival to retirement, solves/s is converged
    solves over the makespan (first arrival to last retirement of any
    request), and MLUPS counts the node updates of every request."""
    import numpy as np
    fin = [r for r in results if not math.isnan(r.finished)]
    conv = [r for r in fin if r.converged]
    lat = np.array([r.latency for r in conv])
    span = max(r.finished for r in fin) - min(r.arrival for r in fin) if fin else math.nan
    node_steps = sum(r.nodes * r.steps for r in fin)
    return {
        "requests": len(results),
        "converged": len(conv),
        "unstable": sum(r.unstable for r in results),
        "capped": sum((not r.converged) and (not r.unstable) for r in results),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
        "makespan_s": span,
        "solves_per_s": len(conv) / span if span > 0 else math.nan,
        "mlups": node_steps / span / 1e6 if span > 0 else math.nan,
        "steps_total": int(sum(r.steps for r in fin)),
    }
