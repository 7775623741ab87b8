"""Throughput of the per-fragment (T) energy on one MI355X.

python bench.py [--steps K] [--warmup W] [--workload o24v200] [--no-cpu]

A step is one full (T) energy evaluation (W-tilde build, R/D epilogue and the
reductions) of one synthetic fragment whose inputs are already resident in
HBM.  Prints one JSON line.  Metric: algorithmic TFLOP/s,
F = 2 n_o^3 n_v^4 + 2 n_o^4 n_v^3 per fragment, divided by the step time.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6      # MI355X dense FP64 matrix peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="o24v200")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-a", default="120,121",
                    help="outer virtual indices a of the CPU-baseline sample")
    return ap.parse_args()


def cpu_baseline(frag, a_values):
    """Time the CPU oracle on a bounded sample of the same fragment: the
    virtual triples (a, b, c) with a in a_values (all b <= a, c <= b)."""
    import oracle.triples as T
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = 1
    o, v = frag.n_occ, frag.n_vir
    n_tri = sum((a + 1) * (a + 2) // 2 for a in a_values)
    flops = n_tri * 12.0 * o ** 3 * (v + o)       # per virtual triple: 6 terms, K = n_v and n_o
    t0 = time.perf_counter()
    T.energy_literal_vectorized(*frag.arrays(), a_values=list(a_values))
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"oracle.energy_literal_vectorized over the {n_tri} virtual triples "
                      f"with a in {list(a_values)} of the same {o}/{v} fragment ({dt:.1f} s)",
            "seconds": dt}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the (T) path here is single-GPU "
              "(fragments would shard across GPUs as independent work; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2412_18553_amd as sie
    from synth import WORKLOADS, workload_fragment

    w = WORKLOADS[args.workload]
    o, v = w["n_occ"], w["n_vir"]
    t0 = time.perf_counter()
    frag = workload_fragment(args.workload)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    fr = sie.Fragment(frag.eps_occ, frag.eps_vir, cast(frag.t1), cast(frag.t2),
                      cast(frag.ovvv), cast(frag.ooov), cast(frag.ovov), "fp64")
    ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print(f"# workload {args.workload}: generated in {gen_s:.1f} s, workspace "
          f"{ws.numel() / 2**20:.0f} MiB", file=sys.stderr, flush=True)

    for s in range(args.warmup):
        sie.energy(fr, workspace=ws, out=out)
        torch.cuda.synchronize()
        print(f"# warmup {s} done", file=sys.stderr, flush=True)

    sie.profile_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        sie.energy(fr, workspace=ws, out=out)
    stop.record()
    torch.cuda.synchronize()
    prof = sie.profile_collect()
    sie.profile_enable(False)
    ms = start.elapsed_time(stop) / args.steps
    energy = float(out.item())

    F = 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3
    tflops = F / (ms * 1e-3) / 1e12
    n_units = sie.occupied_triples(o)
    work_units = n_units - o                       # i = j = k units are exactly zero
    unit_flops = 12.0 * v ** 4 + 12.0 * o * v ** 3  # 6 K=n_v and 6 K=n_o terms per unit
    b_ms, b_n = prof["w_build"]
    e_ms, e_n = prof["epilogue"]
    build_tflops = work_units * unit_flops * args.steps / (b_ms * 1e-3) / 1e12
    result = {
        "metric": "(T) TFLOP/s",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}",
                   "precision": "fp64", "fragments": 1},
        "fragments_per_s": round(1000.0 / ms, 4),
        "energy": energy,
        "roofline": {
            "bound": "mfma",
            "kernel": "k_build_w_f64",
            "achieved": round(build_tflops, 3),
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(build_tflops / PEAK_FP64_MFMA_TFLOPS, 4),
            "traffic": None,
            "launches": int(b_n),
            "avg_launch_ms": round(b_ms / max(b_n, 1), 4),
            "flops_per_unit": unit_flops,
        },
        "kernel_ms_per_step": {k: round(t / args.steps, 3) for k, (t, _) in prof.items()},
    }
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(frag, [int(a) for a in args.cpu_a.split(",")])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
