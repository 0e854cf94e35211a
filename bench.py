"""Benchmark of the fused DDF-MRT porous-convection step on one MI355X.

Default workload: the 256^3 porous cavity (D3Q19 flow + D3Q7 temperature, FP32
storage and arithmetic, phi 0.4, Da 1e-4, Ra 1e6, Pr 1, seed 2), residual
checks every 100 steps as part of the step.  A "step" is one lattice
Boltzmann time step of the whole box.  The state is resident in HBM before
the timed region starts.

Prints ONE JSON line: MLUPS (whole job), the roofline of the step kernel
(algorithmic bytes = 2 x 26 populations x 4 B = 208 B per node per step) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
--precision fp16 runs the same cavity with FP16 flow populations (132 B per
node per step).  Like the FP32 step it is bound by HBM; the line adds its VALU
issue rate beside the bytes (wave64 VALU instructions per CU per clock at
2.4 GHz, the instruction count per step taken from the committed counter
profile), which stays at or below the nominal rate of one.

--workload batched | served runs the solve benchmarks instead (one JSON line
each): 64 cavities of uneven sizes and parameters solved to residual 1e-6 in
one batch (all arriving at once), or a Poisson stream of cavity solve requests
served with continuous batching under an HBM budget; both against the same
solves run one after another in plain FP32.  The server runs first come first
served (FP32, then FP16 storage with an FP32 finish) and smallest first under
a resident-node cap (FP32).

--workload channel times the 512x128x128 porous channel (D3Q15 flow + D3Q7
temperature, inflow, open outlet, heated and cooled walls) with FP32 storage
and with FP16 flow storage side by side (FP16 mode with its VALU issue rate,
as above), and (unless --cpu-steps 0) their
errors in u, T and Nu against the FP64 oracle on the 128x32x32 downscale at
t = 1000 and 2000, the oracle's own run timed as the CPU baseline.

--workload parity32 runs the 32^3 FP64 parity cavity whole (2000 steps) on
the GPU and with the oracle on the host cores, and reports both times and the
largest field difference (a cache-resident latency figure, not a roofline).

--workload melting times the enthalpy-based phase-change step (App. B,
conduction melting of Sec. 4.3) on a 1024x128x128 slab in FP32: 7 populations
read and written, 56 B per node per step, against the same HBM roofline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D3Q19+D3Q7) & % HBM roofline; batched-solve p50/p99 latency"
PEAK_HBM_GBPS = 8000.0
# nominal vector instruction issue: one wave64 VALU instruction per CU per
# clock (four SIMDs, four clocks each), 256 CUs at 2.4 GHz
PEAK_VALU_WAVE_INSTR_PER_S = 256 * 2.4e9
# everything the step kernel is compiled from, build flags included
KERNEL_SOURCES = ("paper_1611_03329_amd/csrc/kernels.hpp", "paper_1611_03329_amd/csrc/model.hpp",
                  "paper_1611_03329_amd/csrc/lattice.hpp", "paper_1611_03329_amd/csrc/batch.hpp",
                  "paper_1611_03329_amd/csrc/lbm_capi.hip", "paper_1611_03329_amd/build.py")


def _code_of(rel: str, text: str) -> str:
    """The source without its comments and blank lines: a comment edit leaves
    the compiled kernels, and so the hash, unchanged."""
    if rel.endswith(".py"):
        text = re.sub(r"#[^\n]*", "", text)
    else:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_of(rel, f.read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(nodes: int):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_cavity256_fp32_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash() or rec.get("nodes") != nodes:
        return None
    return rec.get("bytes_per_launch")


def valu_from_profiles(nodes: int, stem: str):
    """Wave-level VALU instructions per step of the whole lattice (mean of the
    two parities' step kernels) from the committed rocprofv3 counter summary
    profiles/<stem>_valu.json, if it was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"{stem}_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash() or rec.get("nodes") != nodes:
        return None
    return rec.get("valu_per_step")


def cpu_baseline(workload: dict, steps: int) -> dict:
    import oracle
    t0 = time.perf_counter()
    with oracle.Oracle(workload) as o:
        t1 = time.perf_counter()
        o.step(steps)
        t2 = time.perf_counter()
        nodes = o.n
    return {
        "value": nodes * steps / (t2 - t1) / 1e6,
        "unit": "MLUPS",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"{workload['nx']}x{workload['ny']}x{workload['nz']} cavity, FP64 oracle, "
                  f"{steps} steps timed after a {t1 - t0:.1f} s initialisation",
    }


def cpu_baseline_one_thread(steps: int):
    """The same oracle on one thread (OMP_NUM_THREADS=1), in a child process
    that starts its own OpenMP runtime; None if it fails."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-only", str(steps)], env=env,
                           capture_output=True, text=True, timeout=900)
        return json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        return None


def _say(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tune_launch(workloads, precision: str, interval: int):
    """Launch shape for a batch of these workloads, chosen by the batch
    autotuner on throw-away copies (the timed solves start fresh): the
    batch-wide shape and the threads per tile of the size classes whose
    choice differs from it."""
    from paper_1611_03329_amd import Batch, Lattice
    b = Batch(interval)
    lats = [Lattice(w, precision) for w in workloads]
    for lat in lats:
        b.add(lat)
    shape = b.autotune()
    classes = b.class_blocks()
    b.close()
    for lat in lats:
        lat.close()
    return shape, classes


def run_solves(reqs, runs, args, budget=None, progress=_say, sequential=True) -> dict:
    """Serves the requests once per entry of `runs` ((name, precision,
    policy, node cap) tuples) and (unless sequential is False) solves them one
    after another in plain FP32 (name "sequential_fp32"), all to residual 1e-6
    with the launch shape the autotuner picks for the first --tune-count
    workloads.  Returns name -> (results, summary) and the launch shape."""
    from paper_1611_03329_amd.serve import Server, solve_sequential, summarize
    shape, classes = tune_launch([q.workload for q in reqs[:args.tune_count]], "fp32", 100)
    progress(f"launch shape (threads, blocks/CU, group bytes, XCD ranges) = {shape}, "
             f"threads per tile by size class {classes}")
    out = {}
    for name, prec, policy, max_nodes in runs:
        with Server(prec, check_interval=100, tol=1e-6, max_steps=args.max_steps, hbm_budget=budget,
                    launch=shape, policy=policy, max_nodes=max_nodes, escalate=args.escalate,
                    class_blocks=classes) as srv:
            res = srv.run(reqs, progress=progress)
            stats = dict(srv.stats)
        out[name] = (res, {**summarize(res), "promoted": stats["promoted"], "escalated": stats["escalated"],
                           "peak_members": stats["peak_members"], "peak_bytes": stats["peak_bytes"]})
        progress(f"served {name}: {out[name][1]}")
    if sequential:
        seq = solve_sequential(reqs, "fp32", check_interval=100, tol=1e-6, max_steps=args.max_steps,
                               progress=progress)
        out["sequential_fp32"] = (seq, summarize(seq))
        progress(f"sequential fp32: {out['sequential_fp32'][1]}")
    return out, (shape, classes)


def nu_rel_diff(res, ref, reqs=None, above=1e-3) -> dict:
    """Largest and median relative difference of the hot-wall Nu between two
    runs of the same requests, over the requests both converged; with the
    requests given, also the ones that differ by more than `above`."""
    pairs = [(a, b, q) for a, b, q in zip(res, ref, reqs or [None] * len(res))
             if a.converged and b.converged and a.nu and b.nu]
    d = sorted(abs(a.nu[0] - b.nu[0]) / abs(b.nu[0]) for a, b, _ in pairs)
    out = {"max": d[-1] if d else None, "median": d[len(d) // 2] if d else None, "count": len(d)}
    if reqs is not None:
        out[f"above_{above:g}"] = [
            {"name": a.name, "nodes": a.nodes, "steps": a.steps, "ref_steps": b.steps, "promoted_at": a.promoted_at,
             "rayleigh": q.workload["rayleigh"], "darcy": q.workload["darcy"], "porosity": q.workload["porosity"],
             "rel_diff": abs(a.nu[0] - b.nu[0]) / abs(b.nu[0])}
            for a, b, q in pairs if abs(a.nu[0] - b.nu[0]) > above * abs(b.nu[0])]
    return out


def batched_object(args) -> dict:
    """The batched-solve half of the headline metric on the default line: the
    64 cavities of uneven sizes and parameters, all submitted at t = 0, served
    with continuous batching in FP32 (smallest first under the resident-node
    cap) against the same 64 solved one after another in plain FP32."""
    import lbm_inputs
    from paper_1611_03329_amd.serve import Request
    reqs = [Request(i, 0.0, w) for i, w in enumerate(lbm_inputs.config_batch(args.count))]
    nodes = sum(q.workload["nx"] * q.workload["ny"] * q.workload["nz"] for q in reqs)
    cap = int(args.smallest_first_mnodes * 1e6)
    _say(f"batched: {len(reqs)} cavities, {nodes} nodes")
    runs, shape = run_solves(reqs, [("served_fp32_smallest_first", "fp32", "smallest", cap)], args,
                             progress=lambda m: None)
    served, seq = runs["served_fp32_smallest_first"][1], runs["sequential_fp32"][1]
    _say(f"batched: served {served['solves_per_s']:.4f} solves/s p50 {served['p50_s']:.1f} s; "
         f"sequential {seq['solves_per_s']:.4f} solves/s p50 {seq['p50_s']:.1f} s")
    return {
        "workload": f"{len(reqs)} porous cavities, edge from {{32,48,64,96,128}}, phi U[0.3,0.9], Da logU[1e-5,1e-1], "
                    "Ra logU[1e3,1e6], Pr 1, FP32, seed 4, all submitted at t=0, each to residual 1e-6",
        "requests": len(reqs), "nodes": nodes, "max_steps": args.max_steps, "launch": list(shape[0]),
        "class_blocks": shape[1],
        "served_fp32_smallest_first": {**served, "max_resident_nodes": cap},
        "sequential_fp32": seq,
        "speedup_solves_per_s": round(served["solves_per_s"] / seq["solves_per_s"], 4),
        "nu_hot_rel_diff_vs_sequential": nu_rel_diff(runs["served_fp32_smallest_first"][0],
                                                     runs["sequential_fp32"][0]),
    }


def bench_solves(args, kind: str) -> int:
    """Solves to residual 1e-6, served with continuous batching (FP32, and FP16
    storage with the FP32 finish) against one-after-another plain FP32 solves."""
    import torch

    import lbm_inputs
    from paper_1611_03329_amd.serve import Request, as_requests

    torch.cuda.set_device(0)
    if kind == "batched":
        reqs = [Request(i, 0.0, w) for i, w in enumerate(lbm_inputs.config_batch(args.count))]
        budget = None
        workload = (f"{len(reqs)} porous cavities, edge from {{32,48,64,96,128}}, phi U[0.3,0.9], Da logU[1e-5,1e-1], "
                    "Ra logU[1e3,1e6], Pr 1, seed 4, all submitted at t=0")
        metric = "batched-solve throughput (solves to residual 1e-6)"
    else:
        reqs = as_requests(lbm_inputs.config_serving(args.count, rate=args.rate))
        budget = int(args.hbm_budget_gib * (1 << 30))
        workload = (f"Poisson stream of {len(reqs)} porous-cavity solve requests at {args.rate} req/s, edge logU[48,192], "
                    f"parameters as the batched config, seed 5, HBM budget {args.hbm_budget_gib} GiB")
        metric = "served-solve throughput and p50/p99 time-to-converge (residual 1e-6)"
    nodes = sum(q.workload["nx"] * q.workload["ny"] * q.workload["nz"] for q in reqs)
    _say(f"{kind}: {len(reqs)} requests, {nodes} nodes in all; tuning the launch shape")
    cap = int(args.smallest_first_mnodes * 1e6)
    table = {"fp32": ("fp32", "fp32", "fcfs", None), "fp16": ("fp16", "fp16", "fcfs", None),
             "fp32_smallest_first": ("fp32_smallest_first", "fp32", "smallest", cap),
             "fp16_smallest_first": ("fp16_smallest_first", "fp16", "smallest", cap)}
    names = [r for r in args.serve_runs.split(",") if r]
    runs, shape = run_solves(reqs, [table[r] for r in names], args, budget=budget, sequential=args.sequential)
    seq_res, q_sum = runs.pop("sequential_fp32", (None, None))
    main = "fp32" if "fp32" in runs else names[0]
    main_sum = runs[main][1]
    line = {
        "metric": metric,
        "value": round(main_sum["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "requests": len(reqs), "nodes": nodes, "check_interval": 100,
                   "max_steps": args.max_steps, "launch": list(shape[0]), "class_blocks": shape[1],
                   "parallelism": "single GPU"},
        "headline_run": main,
        "served_fp32": runs["fp32"][1] if "fp32" in runs else None,
        "served_fp16_then_fp32": runs["fp16"][1] if "fp16" in runs else None,
        "served_fp32_smallest_first": ({**runs["fp32_smallest_first"][1], "max_resident_nodes": cap}
                                       if "fp32_smallest_first" in runs else None),
        "served_fp16_then_fp32_smallest_first": ({**runs["fp16_smallest_first"][1], "max_resident_nodes": cap}
                                                 if "fp16_smallest_first" in runs else None),
        "sequential_fp32": q_sum,
        "speedup_solves_per_s": (None if q_sum is None else
                                 {p: round(runs[p][1]["solves_per_s"] / q_sum["solves_per_s"], 3) for p in runs}),
        "nu_hot_rel_diff_vs_sequential": (None if seq_res is None else
                                          {p: nu_rel_diff(runs[p][0], seq_res, reqs) for p in runs}),
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_nu_steady(args) -> int:
    """How far a solve stopped at residual 1e-6 is from the steady state: for
    the served requests named in --requests, the hot-wall Nu of the plain FP32
    solve, of the FP16-then-FP32 served solve and of an FP64 run continued
    until its residual is below 1e-10 (the steady state), one JSON line."""
    import torch

    import lbm_inputs
    from paper_1611_03329_amd import Lattice
    from paper_1611_03329_amd.serve import Request, Server, solve_sequential

    torch.cuda.set_device(0)
    names = [n for n in args.requests.split(",") if n]
    reqs = [wl for _, wl in lbm_inputs.config_serving(args.count, rate=args.rate) if wl["name"] in names]
    out = {}
    for wl in reqs:
        q = Request(0, 0.0, wl)
        (s32,) = solve_sequential([q], "fp32", check_interval=100, tol=1e-6, max_steps=args.max_steps)
        with Server("fp16", check_interval=100, tol=1e-6, max_steps=args.max_steps) as srv:
            (s16,) = srv.run([q])
        with Lattice(wl, "fp64", check_interval=100) as lat:
            r = 1.0
            while r >= 1e-10 and lat.time < 2_000_000:
                lat.step(5000)
                r, _ = lat.residual()
            nu_inf, t_inf = lat.nusselt()[0], lat.time
        rec = {"nodes": wl["nx"] * wl["ny"] * wl["nz"], "rayleigh": wl["rayleigh"], "darcy": wl["darcy"],
               "porosity": wl["porosity"], "steady_fp64": {"steps": t_inf, "residual": r, "nu": nu_inf}}
        for key, res in (("fp32", s32), ("fp16_then_fp32", s16)):
            rec[key] = {"steps": res.steps, "converged": res.converged, "residual": res.residual, "nu": res.nu[0],
                        "promoted_at": res.promoted_at, "nu_rel_to_steady": abs(res.nu[0] - nu_inf) / abs(nu_inf)}
        out[wl["name"]] = rec
        _say(f"{wl['name']}: FP32 {rec['fp32']['nu_rel_to_steady']:.2e}, FP16 then FP32 "
             f"{rec['fp16_then_fp32']['nu_rel_to_steady']:.2e} from the steady Nu {nu_inf:.6f}")
    line = {"metric": "hot-wall Nu of solves stopped at residual 1e-6, against the steady state",
            "value": max(r["fp32"]["nu_rel_to_steady"] for r in out.values()) if out else None,
            "unit": "relative", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "served porous-cavity requests (seed 5), residual 1e-6; steady state: FP64 "
                                   "to residual 1e-10", "requests": names},
            "requests": out}
    print(json.dumps(line), flush=True)
    return 0


def _time_steps(lat, warmup: int, steps: int) -> float:
    """ms per step over `steps` steps after `warmup`, HIP events on the lattice's stream."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(steps)
    end.record(lat.stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def bench_channel(args) -> int:
    """Porous channel 512x128x128, D3Q15 + D3Q7: FP32 and FP16 flow storage."""
    import numpy as np
    import torch

    import lbm_inputs
    from paper_1611_03329_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    wl = lbm_inputs.config_channel()
    runs = {}
    for prec, bpn in (("fp32", 2 * 22 * 4), ("fp16", 2 * (15 * 2 + 7 * 4))):
        lat = Lattice(wl, prec, check_interval=args.check_interval)
        nodes = lat.nodes
        ms = _time_steps(lat, args.warmup, args.steps)
        lat.close()
        gbps = bpn * nodes / (ms / 1e3) / 1e9
        runs[prec] = {"ms_per_step": round(ms, 5), "mlups": round(nodes / (ms / 1e3) / 1e6, 1),
                      "bytes_per_node": bpn, "achieved_GBps": round(gbps, 1),
                      "frac": round(gbps / PEAK_HBM_GBPS, 4)}
        if prec == "fp16":
            # FP16 mode: its VALU issue rate beside the bytes
            valu = valu_from_profiles(nodes, "step_channel512x128x128_fp16")
            runs[prec]["valu_issue"] = None if valu is None else {
                "wave_instructions_per_step": valu,
                "per_cu_per_clock": round(valu / (ms / 1e3) / PEAK_VALU_WAVE_INSTR_PER_S, 4)}
        _say(f"{wl['name']} {prec}: {ms:.4f} ms/step, {runs[prec]['mlups']} MLUPS, {gbps:.0f} GB/s")

    accuracy, cpu = None, None
    if args.cpu_steps > 0:
        import oracle

        def fields(lat):
            f = lat.fields()
            torch.cuda.synchronize()
            return {k: v.cpu().numpy() for k, v in f.items()}

        def rel(a, b):
            return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b ** 2)))

        small = lbm_inputs.config_channel(True)
        accuracy = {}
        lats = {p: Lattice(small, p) for p in ("fp32", "fp16")}
        oracle_s = 0.0
        with oracle.Oracle(small) as o:
            for t in (1000, 2000):
                t0 = time.perf_counter()
                o.step(t - o.time)
                oracle_s += time.perf_counter() - t0
                ref, nu_ref = o.fields(), o.nusselt()[2]
                u_ref = np.stack([ref["ux"], ref["uy"], ref["uz"]])
                for p, lat in lats.items():
                    lat.step(t - lat.time)
                    f = fields(lat)
                    nu = lat.nusselt()[2]
                    accuracy.setdefault(p, {})[f"t{t}"] = {
                        "E_u": rel(np.stack([f["ux"], f["uy"], f["uz"]]), u_ref),
                        "E_T": rel(f["T"], ref["T"]), "nu_rel": abs(nu - nu_ref) / abs(nu_ref)}
            nodes_small = o.n
        for lat in lats.values():
            lat.close()
        _say(f"accuracy against the oracle on {small['name']}: {accuracy}")
        cpu = {"value": nodes_small * 2000 / oracle_s / 1e6, "unit": "MLUPS", "cores": oracle.threads(),
               "kind": "oracle", "sample": f"{small['name']} downscale, FP64 oracle, 2000 steps"}
    line = {
        "metric": "MLUPS (D3Q15+D3Q7 porous channel) & % HBM roofline",
        "value": runs["fp32"]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs["fp32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "porous channel 512x128x128, D3Q15 MRT flow + D3Q7 MRT temperature, phi 0.7, "
                               "Da 1e-3, Re 10, Ra 1e5, inflow 0.05, open outlet, seed 3, residual check every "
                               f"{args.check_interval} steps", "nodes": 512 * 128 * 128, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": runs["fp32"]["achieved_GBps"], "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": runs["fp32"]["frac"], "traffic": None},
        "fp16_storage": runs["fp16"],
        "accuracy_vs_oracle": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_parity32(args) -> int:
    """The 32^3 FP64 parity cavity run whole (2000 steps from the initial state)
    on the GPU and by the oracle on the host cores, with the largest field
    difference between the two.  Its 6.8 MB state stays in the caches, so the
    GPU figure is a latency, not a roofline measurement."""
    import numpy as np
    import torch

    import lbm_inputs
    import oracle
    from paper_1611_03329_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    wl = lbm_inputs.config_cavity_fp64()
    steps = wl["steps"]
    lat = Lattice(wl, "fp64", check_interval=args.check_interval)
    nodes = lat.nodes
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(steps)
    end.record(lat.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    fl = {k: v.cpu().numpy() for k, v in lat.fields().items()}
    nu = lat.nusselt()[0]
    lat.close()
    _say(f"{wl['name']}: {steps} steps in {ms:.1f} ms on the GPU")
    with oracle.Oracle(wl) as o:
        t0 = time.perf_counter()
        o.step(steps)
        t1 = time.perf_counter()
        ref = o.fields()
        nu_ref = o.nusselt()[0]
    diff = max(float(np.max(np.abs(fl[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in ref)
    _say(f"oracle: {t1 - t0:.2f} s; largest field difference {diff:.2e}")
    line = {
        "metric": "time to run the FP64 parity cavity (2000 steps)",
        "value": round(ms / 1e3, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": round(ms / steps, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "porous cavity 32^3, D3Q19 MRT flow + D3Q7 MRT temperature, FP64, phi 0.6, Da 1e-2, "
                               f"Ra 1e4, Pr 1, seed 1, residual check every {args.check_interval} steps",
                   "nodes": nodes, "parallelism": "single GPU"},
        "mlups": round(nodes * steps / (ms / 1e3) / 1e6, 1),
        "roofline": None,
        "cache_resident": True,
        "nu_hot": nu,
        "max_rel_field_diff_vs_oracle": diff,
        "nu_rel_diff_vs_oracle": abs(nu - nu_ref) / abs(nu_ref),
        "cpu_baseline": {"value": round(t1 - t0, 3), "unit": "s", "cores": oracle.threads(), "kind": "oracle",
                         "sample": "the whole run, 2000 steps of the 32^3 cavity",
                         "mlups": round(nodes * steps / (t1 - t0) / 1e6, 1)},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_melting(args) -> int:
    """Enthalpy phase-change step (FP32) on a 1024x128x128 melting slab."""
    import torch

    import lbm_inputs
    from paper_1611_03329_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    wl = lbm_inputs.melting(1024, 128, 128, alpha_ratio=4.0)
    lat = Lattice(wl, "fp32")
    nodes = lat.nodes
    _say(f"{wl['name']}: {nodes} nodes, warmup {args.warmup}")
    lat.step(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(args.steps)
    end.record(lat.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    mlups = nodes * args.steps / (ms / 1e3) / 1e6
    molten = float(lat.enthalpy_fields()["fl"].sum().item()) / (128 * 128)
    lat.close()
    _say(f"{ms_per_step:.4f} ms/step, {mlups:.1f} MLUPS, molten depth {molten:.2f} nodes")
    achieved = 2 * 7 * 4 * nodes / (ms_per_step / 1e3) / 1e9
    cpu = None
    if args.cpu_steps > 0:
        import oracle
        small = lbm_inputs.melting(1024, 32, 32, alpha_ratio=4.0)
        with oracle.EnthalpyOracle(small) as o:
            t0 = time.perf_counter()
            o.step(args.cpu_steps)
            t1 = time.perf_counter()
        cpu = {"value": 1024 * 32 * 32 * args.cpu_steps / (t1 - t0) / 1e6, "unit": "MLUPS",
               "cores": oracle.threads(), "kind": "oracle",
               "sample": f"1024x32x32 slab of the same melting problem, FP64 oracle, {args.cpu_steps} steps"}
    line = {
        "metric": "MLUPS (D3Q7 enthalpy phase change) & % HBM roofline",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "conduction melting slab 1024x128x128 (Sec. 4.3 setting), enthalpy D3Q7-MRT, "
                               "FP32, alpha_l/alpha_s 4, St 1", "nodes": nodes, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("cavity256", "batched", "served", "channel", "melting", "parity32",
                                           "nu-steady"), default="cavity256")
    ap.add_argument("--requests", default="cavity53_phi0.533_Da6.17e-02_Ra1.33e+04,"
                    "cavity93_phi0.490_Da3.53e-02_Ra3.16e+04,cavity126_phi0.337_Da5.33e-02_Ra2.83e+05,"
                    "cavity48_phi0.309_Da5.32e-02_Ra4.78e+03,cavity103_phi0.781_Da1.19e-05_Ra1.60e+03",
                    help="nu-steady: names of served requests to study")
    ap.add_argument("--count", type=int, default=64, help="solves in the batched / served workloads")
    ap.add_argument("--rate", type=float, default=20.0, help="served: mean arrivals per second")
    ap.add_argument("--hbm-budget-gib", type=float, default=16.0, help="served: HBM budget for admission")
    ap.add_argument("--max-steps", type=int, default=1_000_000,
                    help="solves: step cap per solve (a safety net: the slowest served solve takes about 5e5)")
    ap.add_argument("--serve-runs", default="fp32,fp16,fp32_smallest_first",
                    help="batched / served: the serving runs (fp32, fp16, fp32_smallest_first, fp16_smallest_first)")
    ap.add_argument("--escalate", action=argparse.BooleanOptionalAction, default=True,
                    help="batched / served: a served solve whose FP32 residual stalls above the tolerance "
                         "finishes in FP64 (the sequential baseline stays plain FP32)")
    ap.add_argument("--sequential", action=argparse.BooleanOptionalAction, default=True,
                    help="batched / served: also solve the requests one after another in plain FP32")
    ap.add_argument("--tune-count", type=int, default=16, help="solves: workloads used to tune the launch shape")
    ap.add_argument("--smallest-first-mnodes", type=float, default=4.0,
                    help="solves: resident-node cap (millions) of the smallest-first serving run")
    ap.add_argument("--precision", choices=("fp32", "fp16"), default="fp32",
                    help="cavity256: population storage (FP16 flow populations, FP32 arithmetic)")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--check-interval", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps on the 256^3 sample (0 skips the CPU baseline)")
    ap.add_argument("--cpu-steps-one-thread", type=int, default=1,
                    help="oracle steps on the 256^3 sample on one thread (0 skips them)")
    ap.add_argument("--oracle-only", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--batched", action=argparse.BooleanOptionalAction, default=True,
                    help="cavity256: also run the batched-solve benchmark (64 cavities to residual 1e-6, served "
                         "FP32 against one after another) and report it in the same line")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="size of the plain device-to-device copy timed as the attainable-bandwidth "
                         "reference (0 skips it)")
    args = ap.parse_args(argv)

    if args.oracle_only > 0:
        import lbm_inputs
        print(json.dumps(cpu_baseline(lbm_inputs.config_cavity_fp32(), args.oracle_only)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); there is no "
              "multi-GPU path", file=sys.stderr)
        return 2
    if args.workload == "melting":
        return bench_melting(args)
    if args.workload == "parity32":
        return bench_parity32(args)
    if args.workload == "channel":
        return bench_channel(args)
    if args.workload == "nu-steady":
        return bench_nu_steady(args)
    if args.workload != "cavity256":
        return bench_solves(args, args.workload)

    import torch

    import lbm_inputs
    from paper_1611_03329_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    # the lattice is created (and initialised) first, so that the copy
    # reference keeps the GPU busy right up to the warm-up steps
    wl = lbm_inputs.config_cavity_fp32()
    lat = Lattice(wl, args.precision, check_interval=args.check_interval)
    nodes = lat.nodes
    copy_gbps = None
    if args.copy_bytes > 0:
        # plain copy of a known size: the reference the HBM byte counters are scaled by
        a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(10):
            b.copy_(a)
        c1.record()
        torch.cuda.synchronize()
        copy_gbps = 2 * args.copy_bytes * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
        del a, b
    print(f"[bench] {wl['name']}: {nodes} nodes, warmup {args.warmup}", file=sys.stderr, flush=True)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    stream = lat.stream
    start.record(stream)
    lat.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    mlups = nodes * args.steps / (ms / 1e3) / 1e6
    r, at = lat.residual()
    nu = lat.nusselt()
    lat.close()
    # compare steps (residual checks) that ran inside the timed region: the
    # steps starting at times t = warmup .. warmup + steps - 1 with t % K == 0
    K = args.check_interval
    t0, t1 = args.warmup, args.warmup + args.steps - 1
    checks = 0 if K <= 0 else max(0, t1 // K - max(t0 - 1, K - 1) // K)
    print(f"[bench] {ms_per_step:.4f} ms/step, {mlups:.1f} MLUPS, residual {r:.3e} at {at} "
          f"({checks} checks timed), Nu_hot {nu[0]:.5f}", file=sys.stderr, flush=True)

    fp16 = args.precision == "fp16"
    bytes_per_node = 2 * (19 * 2 + 7 * 4) if fp16 else 2 * (19 + 7) * 4
    achieved = bytes_per_node * nodes / (ms_per_step / 1e3) / 1e9
    traffic = None if fp16 else traffic_from_profiles(nodes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
                "copy_reference_GBps": None if copy_gbps is None else round(copy_gbps, 1)}
    if fp16:
        # FP16 mode: the VALU issue rate beside the bytes (how close the
        # instruction stream comes to the nominal rate; the step is HBM-bound)
        valu = valu_from_profiles(nodes, "step_cavity256_fp16")
        roofline["valu_issue"] = None if valu is None else {
            "wave_instructions_per_step": valu,
            "per_cu_per_clock": round(valu / (ms_per_step / 1e3) / PEAK_VALU_WAVE_INSTR_PER_S, 4)}

    batched = batched_object(args) if args.batched else None

    cpu = None
    if args.cpu_steps > 0:
        print(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_steps)
        if args.cpu_steps_one_thread > 0:
            print(f"[bench] cpu baseline: oracle on one thread, {args.cpu_steps_one_thread} steps", file=sys.stderr,
                  flush=True)
            one = cpu_baseline_one_thread(args.cpu_steps_one_thread)
            cpu["one_thread"] = None if one is None else {k: one[k] for k in ("value", "unit", "cores", "sample")}

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "porous cavity 256^3, D3Q19 MRT flow + D3Q7 MRT temperature, "
                        + ("FP16 flow storage (stochastic rounding), FP32 arithmetic, " if fp16 else "FP32, ")
                        + "phi 0.4, Da 1e-4, Ra 1e6, Pr 1, seed 2"
                        + (f", residual check every {K} steps ({checks} in the timed region)" if checks else
                           ", no residual check in the timed region"),
            "nodes": nodes,
            "check_interval": K,
            "checks_in_timed_region": checks,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
