"""Benchmark of the fused DDF-MRT porous-convection step on one MI355X.

Workload: the 256^3 porous cavity (D3Q19 flow + D3Q7 temperature, FP32
storage and arithmetic, phi 0.4, Da 1e-4, Ra 1e6, Pr 1, seed 2), residual
checks every 100 steps as part of the step.  A "step" is one lattice
Boltzmann time step of the whole box.  The state is resident in HBM before
the timed region starts.

Prints ONE JSON line: MLUPS (whole job), the roofline of the step kernel
(algorithmic bytes = 2 x 26 populations x 4 B = 208 B per node per step) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D3Q19+D3Q7) & % HBM roofline; batched-solve p50/p99 latency"
PEAK_HBM_GBPS = 8000.0
KERNEL_SOURCES = ("paper_1611_03329_amd/csrc/kernels.hpp", "paper_1611_03329_amd/csrc/model.hpp",
                  "paper_1611_03329_amd/csrc/lattice.hpp")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
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


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--check-interval", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps on the 256^3 sample (0 skips the CPU baseline)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="size of the plain device-to-device copy timed as the attainable-bandwidth "
                         "reference (0 skips it)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    import torch

    import lbm_inputs
    from paper_1611_03329_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
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
        torch.cuda.empty_cache()
    wl = lbm_inputs.config_cavity_fp32()
    lat = Lattice(wl, "fp32", check_interval=args.check_interval)
    nodes = lat.nodes
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
    print(f"[bench] {ms_per_step:.4f} ms/step, {mlups:.1f} MLUPS, residual {r:.3e} at {at}, "
          f"Nu_hot {nu[0]:.5f}", file=sys.stderr, flush=True)

    bytes_per_node = 2 * (19 + 7) * 4
    achieved = bytes_per_node * nodes / (ms_per_step / 1e3) / 1e9
    traffic = traffic_from_profiles(nodes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
                "copy_reference_GBps": None if copy_gbps is None else round(copy_gbps, 1)}

    cpu = None
    if args.cpu_steps > 0:
        print(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_steps)

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
            "workload": "porous cavity 256^3, D3Q19 MRT flow + D3Q7 MRT temperature, FP32, "
                        "phi 0.4, Da 1e-4, Ra 1e6, Pr 1, seed 2, residual check every "
                        f"{args.check_interval} steps",
            "nodes": nodes,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
