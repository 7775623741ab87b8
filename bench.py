"""Throughput of the per-fragment (T) energy on one MI355X.

python bench.py [--steps K] [--warmup W] [--mode fp64|split|batched|backward]
                [--workload NAME] [--no-cpu]

Default (the headline line): a step is one full float64 (T) energy
evaluation (W-tilde build, R/D epilogue and the reductions) of the
24-occupied / 200-virtual synthetic fragment, inputs already resident in
HBM.  Metric: algorithmic TFLOP/s, F = 2 n_o^3 n_v^4 + 2 n_o^4 n_v^3 per
fragment, divided by the step time.  Prints one JSON line.

Other modes (same JSON shape): `split` (float32 inputs, bf16 hi/lo products;
32/320 fragment), `batched` (one evaluation over the 16-fragment batch),
`backward` (energy gradient of the 16/120 fragment).
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
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak

DEFAULT_WORKLOAD = {"fp64": "o24v200", "split": "o32v320", "batched": "batch16",
                    "backward": "o16v120"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="fp64", choices=sorted(DEFAULT_WORKLOAD))
    ap.add_argument("--workload", default=None)
    ap.add_argument("--precision", default=None, choices=["fp64", "split_bf16"],
                    help="batched mode: precision of the evaluation (default fp64)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES device-to-device (a known-size transfer against "
                         "which hardware byte counters are scaled)")
    ap.add_argument("--cpu-a", default="120,121",
                    help="outer virtual indices a of the CPU-baseline sample")
    return ap.parse_args()


def flops(o, v):
    """Algorithmic (T) work of one fragment: F = 2 n_o^3 n_v^4 + 2 n_o^4 n_v^3."""
    return 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3


def build_work(o, v, pair=True, lay3=False):
    """Flops of the W-tilde build actually launched for one fragment: every
    occupied triple that is not i = j = k, 12 terms (6 with K = n_v, 6 with
    K = n_o) in two layouts of six or three layouts of four (`lay3`); a triple
    with exactly two equal indices (n_o (n_o - 1) of them) builds one of two
    layouts or two of three in the energy (`pair`), all of them in the gradient."""
    n_units = o * (o + 1) * (o + 2) // 6
    n_pair = o * (o - 1) if pair else 0
    saved = (1.0 / 3.0 if lay3 else 0.5) * n_pair
    return (n_units - o - saved) * (12.0 * v ** 4 + 12.0 * o * v ** 3)


def lay3_of(v):
    """Whether the float64 energy of a fragment with v virtuals uses the
    three-layout build under the installed tile table."""
    import paper_2412_18553_amd as sie
    return sie.tile_variants()[sie.tile_variant_of(v)][6] >= 3


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
    work = n_tri * 12.0 * o ** 3 * (v + o)       # per virtual triple: 6 terms, K = n_v and n_o
    t0 = time.perf_counter()
    T.energy_literal_vectorized(*frag.arrays(), a_values=list(a_values))
    dt = time.perf_counter() - t0
    return {"value": work / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"oracle.energy_literal_vectorized over the {n_tri} virtual triples "
                      f"with a in {list(a_values)} of the same {o}/{v} fragment ({dt:.1f} s)",
            "seconds": dt}


def sources_sha256():
    """Hash of the kernel sources (csrc/), against which a recorded counter
    measurement is matched: any change to them voids the measurement."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2412_18553_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the FETCH_SIZE /
    WRITE_SIZE counter passes recorded in profiles/*.md (a line
    `<!-- traffic: {json} -->`), or None when none was taken with the current
    kernel sources."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    want = sources_sha256()
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                line = line.strip()
                if not (line.startswith("<!-- traffic:") and line.endswith("-->")):
                    continue
                rec = json.loads(line[len("<!-- traffic:"):-len("-->")])
                if (rec.get("kernel"), rec.get("workload"), rec.get("sources_sha256")) == \
                        (kernel, workload, want):
                    return rec
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def to_device(frag, dtype):
    import numpy as np
    import torch
    import paper_2412_18553_amd as sie
    dev = torch.device("cuda:0")
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev, dtype)  # noqa: E731
    prec = "fp64" if dtype == torch.float64 else "split_bf16"
    return sie.Fragment(frag.eps_occ, frag.eps_vir, cast(frag.t1), cast(frag.t2),
                        cast(frag.ovvv), cast(frag.ooov), cast(frag.ovov), prec)


def timed(step, steps, warmup):
    """Run `step` warmup + steps times; returns (ms per step, profile)."""
    import torch
    import paper_2412_18553_amd as sie
    for s in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"# warmup {s} done")
    sie.profile_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    prof = sie.profile_collect()
    sie.profile_enable(False)
    return start.elapsed_time(stop) / steps, prof


def roofline(prof, cls, kernel, work_per_step, steps, peak, scale=1.0, bound="mfma",
             workload=None):
    ms, n = prof[cls]
    achieved = scale * work_per_step * steps / (ms * 1e-3) / 1e12
    out = {"bound": bound, "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
           "launches": int(n), "avg_launch_ms": round(ms / max(n, 1), 4)}
    rec = recorded_traffic(kernel, workload) if workload else None
    if rec:
        # HBM bytes per launch (counters, copy-calibrated) against the
        # algorithmic bytes per launch
        out.update(traffic=rec["bytes_per_launch"], traffic_unit="bytes/launch",
                   algorithmic_bytes=rec["algorithmic_bytes_per_launch"],
                   traffic_source=rec["profile"])
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the (T) path here is single-GPU "
              "(fragments would shard across GPUs as independent work; not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_18553_amd as sie
    from synth import WORKLOADS, batch_shapes, make_fragment, workload_fragment

    mode = args.mode
    name = args.workload or DEFAULT_WORKLOAD[mode]
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"# calibration copy: {src.numel() * 8} bytes device to device")
        del src, dst
    t0 = time.perf_counter()
    result = {"metric": "(T) TFLOP/s", "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "data": "synthetic"}

    if mode in ("fp64", "split", "backward"):
        w = WORKLOADS[name]
        o, v = w["n_occ"], w["n_vir"]
        frag = workload_fragment(name)
        dtype = torch.float32 if mode == "split" else torch.float64
        fr = to_device(frag, dtype)
        log(f"# workload {name}: generated in {time.perf_counter() - t0:.1f} s")
        out = torch.empty(1, dtype=torch.float64, device=dev)
        F = flops(o, v)
        if mode == "backward":
            ws = torch.empty(sie.backward_workspace_size(fr), dtype=torch.uint8, device=dev)
            grads = [{n: torch.empty_like(getattr(fr, n), dtype=torch.float64)
                      for n in sie.GRAD_NAMES}]
            step = lambda: sie.backward(fr, grads=grads, e_frag=out, workspace=ws)  # noqa: E731
        else:
            ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
            step = lambda: sie.energy(fr, workspace=ws, out=out)  # noqa: E731
        ms, prof = timed(step, args.steps, args.warmup)
        energy = float(out.item())
        bw = build_work(o, v)
        desc = f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}"
        if mode == "fp64":
            result.update(value=round(F / (ms * 1e-3) / 1e12, 3), dtype="f64",
                          config={"workload": desc, "precision": "fp64", "fragments": 1})
            l3 = lay3_of(v)
            lay = sie.tile_variants()[sie.tile_variant_of(v)][6]
            kernel = {2: "k_build_w_f64", 3: "k_build_w3_f64"}[lay]
            result["roofline"] = roofline(prof, "w_build", kernel, build_work(o, v, lay3=l3),
                                          args.steps, PEAK_FP64_MFMA_TFLOPS, workload=name)
            result["roofline"]["tile_variant"] = sie.tile_variant_of(v)
        elif mode == "split":
            result.update(value=round(F / (ms * 1e-3) / 1e12, 3), dtype="bf16x3/f32",
                          config={"workload": desc + " (float32 inputs)",
                                  "precision": "split_bf16", "fragments": 1})
            # three bf16 products (hi*hi + hi*lo + lo*hi) per algorithmic product
            result["roofline"] = roofline(prof, "w_build", "k_build_w_bf16x3", bw, args.steps,
                                          PEAK_BF16_MFMA_TFLOPS, scale=3.0)
        else:
            # the backward recomputes the build (1x) and runs the transposed
            # contractions of every build term (2x): 3x the build's work
            result.update(metric="(T) gradient TFLOP/s (3 x F per step)",
                          value=round(3.0 * F / (ms * 1e-3) / 1e12, 3), dtype="f64",
                          config={"workload": desc, "precision": "fp64", "fragments": 1,
                                  "outputs": "dE/d(t1, t2, ovvv, ooov, ovov)"})
            result["roofline"] = roofline(prof, "grad", "k_adj_contract",
                                          2.0 * build_work(o, v, pair=False), args.steps,
                                          PEAK_FP64_MFMA_TFLOPS)
        result.update(ms_per_step=round(ms, 3), fragments_per_s=round(1000.0 / ms, 4),
                      energy=energy)
        if mode == "fp64" and not args.no_cpu:
            result["cpu_baseline"] = cpu_baseline(frag, [int(a) for a in args.cpu_a.split(",")])
    else:   # batched
        prec = args.precision or "fp64"
        dtype = torch.float64 if prec == "fp64" else torch.float32
        shapes = batch_shapes(name)
        frs = [to_device(make_fragment(o, v, aux, seed), dtype) for (o, v, aux, seed) in shapes]
        log(f"# workload {name}: {len(frs)} fragments in {time.perf_counter() - t0:.1f} s")
        ws = torch.empty(sie.workspace_size(frs), dtype=torch.uint8, device=dev)
        e_frag = torch.empty(len(frs), dtype=torch.float64, device=dev)
        e_tot = torch.empty(1, dtype=torch.float64, device=dev)
        step = lambda: sie.energy_batched(frs, workspace=ws, out=e_frag, total=e_tot)  # noqa: E731
        ms, prof = timed(step, args.steps, args.warmup)
        F = sum(flops(o, v) for (o, v, _, _) in shapes)
        bw = sum(build_work(o, v, lay3=(prec == "fp64" and lay3_of(v))) for (o, v, _, _) in shapes)
        result.update(value=round(F / (ms * 1e-3) / 1e12, 3),
                      dtype="f64" if prec == "fp64" else "bf16x3/f32",
                      config={"workload": f"{name}: {len(frs)} fragments, n_occ "
                                          f"{min(s[0] for s in shapes)}..{max(s[0] for s in shapes)}",
                              "precision": prec, "fragments": len(frs)},
                      ms_per_step=round(ms, 3), fragments_per_s=round(len(frs) * 1000.0 / ms, 4),
                      energy=float(e_tot.item()))
        if prec == "fp64":   # the batch mixes the build shapes its fragment sizes select
            result["roofline"] = roofline(prof, "w_build", "k_build_w_f64 / k_build_w3_f64", bw,
                                          args.steps, PEAK_FP64_MFMA_TFLOPS)
        else:
            result["roofline"] = roofline(prof, "w_build", "k_build_w_bf16x3", bw, args.steps,
                                          PEAK_BF16_MFMA_TFLOPS, scale=3.0)
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof.items()}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
