"""Throughput of the per-fragment (T) energy on one MI355X.

python bench.py [--steps K] [--warmup W]
                [--mode split|fp64|batched|backward|projector|df|mp2|peak]
                [--workload NAME] [--precision fp64|split_bf16] [--no-cpu] [--no-fp64]

Default (the headline line): a step is one full split-precision (T) energy
evaluation (bf16 hi/lo staging, W-tilde build, R/D epilogue, reductions) of
the 32-occupied / 320-virtual synthetic fragment (float32 inputs), inputs
already resident in HBM.  Metric: algorithmic TFLOP/s, F = 2 n_o^3 n_v^4 +
2 n_o^4 n_v^3 per fragment, divided by the step time.  The same run also
times one float64 evaluation of the same fragment (the float32 inputs
widened) for the split-over-float64 speedup, and reports both energies'
errors against the stored CPU-oracle value of that fragment, plus the split
error on its chemically scaled copy (integrals and t2 times 2^-9).  Prints
one JSON line.

Other modes (same JSON shape): `fp64` (24/200 fragment, float64), `batched`
(one evaluation over a named batch, batch16 or batch64, --precision),
`backward` (energy gradient of the 16/120 fragment), `peak` (the matrix-core
microbenchmark alone).
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6      # MI355X dense FP64 matrix peak (published)
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak (published)
CHEM_SCALE = 2.0 ** -9            # integrals and t2 of the chemically scaled copy

DEFAULT_WORKLOAD = {"fp64": "o24v200", "split": "o32v320", "batched": "batch16",
                    "backward": "o16v120", "peak": None, "mp2": "mp2_o64v512",
                    "projector": "o24v200", "df": "o32v320"}
GOLDEN = os.path.join(ROOT, "tests", "golden")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="split", choices=sorted(DEFAULT_WORKLOAD))
    ap.add_argument("--workload", default=None)
    ap.add_argument("--precision", default=None, choices=["fp64", "split_bf16"],
                    help="batched mode: precision of the evaluation (default fp64)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true",
                    help="split mode: skip the float64 evaluation of the same fragment")
    ap.add_argument("--parts", type=int, default=1,
                    help="batched mode: evaluate the batch as this many consecutive groups")
    ap.add_argument("--singles", action="store_true",
                    help="batched mode: also time every fragment alone")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES device-to-device (a known-size transfer against "
                         "which hardware byte counters are scaled)")
    return ap.parse_args()


def flops(o, v):
    """Algorithmic (T) work of one fragment: F = 2 n_o^3 n_v^4 + 2 n_o^4 n_v^3."""
    return 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- peak
def measured_peak(kind):
    """TFLOP/s of the in-repo matrix-core microbenchmark (kind 0: float64
    16x16x4, kind 1: bf16 16x16x32), or None if its library is absent."""
    path = os.path.join(ROOT, "paper_2412_18553_amd", "libsie_mfma_peak.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.sie_mfma_peak.restype = ctypes.c_int
    lib.sie_mfma_peak.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(0.0)
    iters = 40000 if kind == 0 else 80000
    st = lib.sie_mfma_peak(kind, iters, 8192, ctypes.byref(out))
    if st != 0:
        raise RuntimeError(f"sie_mfma_peak failed with {st}")
    return round(out.value, 2)


# ---------------------------------------------------------------- CPU baseline
def cpu_baseline(host_frag, target_s=15.0):
    """Time the CPU oracle on a bounded sample of the same fragment: the
    occupied-outer oracle (oracle.occupied_triple_parts) on occupied triples
    with three distinct indices, taken from a fixed spread until about
    `target_s` seconds have passed; the rate is the sample's flops over its
    time, i.e. an extrapolation of the whole fragment's oracle rate."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = 1
    o, v = host_frag.n_occ, host_frag.n_vir
    spread = [(o - 1, o // 2, 0), (o // 3, o // 4, o // 5), (o - 2, o - 3, o - 4),
              (o // 2, 1, 0), (o - 1, o // 3, o // 6), (2 * o // 3, o // 2, o // 4),
              (o - 3, 2, 1), (o // 2 + 1, o // 2, o // 2 - 1)]
    units = []
    for t in spread:
        if t[0] > t[1] > t[2] >= 0 and t not in units:
            units.append(t)
    done = []
    t0 = time.perf_counter()
    for (i, j, k) in units:
        oracle.occupied_triple_parts(i, j, k, *host_frag.arrays())
        done.append((i, j, k))
        if time.perf_counter() - t0 >= target_s:
            break
    dt = time.perf_counter() - t0
    # flops of one occupied triple with three distinct indices: 12 n_v^4 + 12 n_o n_v^3
    work = len(done) * (12.0 * v ** 4 + 12.0 * o * v ** 3)
    return {"value": round(work / dt / 1e12, 5), "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle", "extrapolated": True,
            "sample": f"oracle.occupied_triple_parts on occupied triples {done} of the same "
                      f"{o}/{v} fragment ({dt:.1f} s); rate = sample flops / sample time, "
                      f"extrapolated to the whole fragment",
            "seconds": round(dt, 2)}


# ---------------------------------------------------------------- helpers
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


def frag_of(df, precision):
    import paper_2412_18553_amd as sie
    return sie.Fragment(df.eps_occ, df.eps_vir, df.t1, df.t2, df.ovvv, df.ooov, df.ovov,
                        precision)


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
    for s in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    prof = sie.profile_collect()
    sie.profile_enable(False)
    log(f"# {steps} timed steps done")
    return start.elapsed_time(stop) / steps, prof


def roofline(prof, cls, kernel, work_per_step, steps, peak, *, issued=1.0, measured=None,
             workload=None):
    """Achieved rate of the dominant kernel class `cls`: algorithmic flops
    (`work_per_step` x `issued` products per algorithmic product) over the
    summed launch durations (HIP events on the launch stream)."""
    ms, n = prof[cls]
    achieved = issued * work_per_step * steps / (ms * 1e-3) / 1e12
    out = {"bound": "mfma", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
           "launches": int(n), "avg_launch_ms": round(ms / max(n, 1), 4),
           "work": "algorithmic F" + (f" x {issued:g} issued products" if issued != 1 else "")}
    if measured:
        out.update(peak_measured=measured, frac_measured=round(achieved / measured, 4))
    rec = recorded_traffic(kernel, workload) if workload else None
    if rec:
        # HBM bytes per launch (counters, copy-calibrated) against the
        # algorithmic bytes per launch
        out.update(traffic=rec["bytes_per_launch"], traffic_unit="bytes/launch",
                   algorithmic_bytes=rec["algorithmic_bytes_per_launch"],
                   traffic_source=rec["profile"])
    return out


def split_kernel_name(nv):
    import paper_2412_18553_amd as sie
    s = sie.split_shape_of(nv)
    shapes = {0: "k_build_w_bf16x3<4, 2>", 1: "k_build_w_bf16x3<5, 5>",
              2: "k_build_w_bf16x3<7, 4>", 3: "k_build_w_bf16x3<4, 4>",
              4: "k_build_w_bf16x3_l<5, 5, 4>", 5: "k_build_w_bf16x3_l<5, 5, 2>"}
    return shapes[s]


def stored_oracle(name):
    p = os.path.join(GOLDEN, name)
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- modes
def run_split(args, result, name):
    import torch
    import paper_2412_18553_amd as sie
    from synth import WORKLOADS
    from synth.device import workload_fragment_device
    w = WORKLOADS[name]
    o, v = w["n_occ"], w["n_vir"]
    F = flops(o, v)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    df = workload_fragment_device(name, device=dev, dtype=torch.float32)
    log(f"# workload {name}: float32 inputs built on the GPU in {time.perf_counter() - t0:.1f} s")
    fr = frag_of(df, "split_bf16")
    out = torch.empty(1, dtype=torch.float64, device=dev)
    ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
    step = lambda: sie.energy(fr, workspace=ws, out=out)  # noqa: E731
    ms, prof = timed(step, args.steps, args.warmup)
    energy = float(out.item())
    peak_bf16 = measured_peak(1)
    desc = f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}, float32 inputs"
    result.update(value=round(F / (ms * 1e-3) / 1e12, 3), dtype="bf16x3/f32",
                  config={"workload": desc, "precision": "split_bf16", "fragments": 1})
    rl = roofline(prof, "w_build", split_kernel_name(v), F, args.steps, PEAK_BF16_MFMA_TFLOPS,
                  issued=3.0, measured=peak_bf16, workload=name)
    eff = F * args.steps / (prof["w_build"][0] * 1e-3) / 1e12
    rl.update(effective_achieved=round(eff, 3), effective_frac=round(eff / PEAK_BF16_MFMA_TFLOPS, 4))
    result["roofline"] = rl
    result.update(ms_per_step=round(ms, 3), fragments_per_s=round(1000.0 / ms, 4), energy=energy)

    g = stored_oracle(f"{name}_f32_all_units.json")
    acc = {}
    if g:
        acc["oracle_energy"] = g["energy"]
        acc["split_error_ueh"] = round((energy - g["energy"]) * 1e6, 3)
        acc["split_error_rel"] = float(f"{(energy - g['energy']) / abs(g['energy']):.3e}")
    # chemically scaled copy: integrals and t2 times 2^-9 (exact in float32)
    with torch.no_grad():
        for x in (df.t2, df.ovvv, df.ooov, df.ovov):
            x.mul_(CHEM_SCALE)
    sie.energy(fr, workspace=ws, out=out)
    e_chem = float(out.item())
    if g:
        ref = math.fsum([x * CHEM_SCALE ** 4 for x in g["e_ww_units"]] +
                        [x * CHEM_SCALE ** 3 for x in g["e_wv_units"]])
        acc.update(chemical_scale_oracle=ref, chemical_scale_split=e_chem,
                   chemical_scale_error_ueh=float(f"{(e_chem - ref) * 1e6:.4e}"))
    with torch.no_grad():
        for x in (df.t2, df.ovvv, df.ooov, df.ovov):
            x.mul_(1.0 / CHEM_SCALE)
    result["accuracy"] = acc
    log("# split accuracy done")

    if not args.no_fp64:
        # one float64 evaluation of the same fragment (the float32 inputs widened)
        del ws
        d64 = type(df)(df.eps_occ, df.eps_vir, *(x.double() for x in df.arrays()[2:]))
        fr64 = frag_of(d64, "fp64")
        ws64 = torch.empty(sie.workspace_size(fr64), dtype=torch.uint8, device=dev)
        out64 = torch.empty(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        sie.profile_enable(True)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        sie.energy(fr64, workspace=ws64, out=out64)
        stop.record()
        torch.cuda.synchronize()
        p64 = sie.profile_collect()
        sie.profile_enable(False)
        ms64 = start.elapsed_time(stop)
        e64 = float(out64.item())
        peak64 = measured_peak(0)
        fp = {"ms": round(ms64, 1), "value": round(F / (ms64 * 1e-3) / 1e12, 3),
              "speedup_split_over_fp64": round(ms64 / ms, 3), "energy": e64,
              "build_achieved": round(F / (p64["w_build"][0] * 1e-3) / 1e12, 3),
              "build_frac": round(F / (p64["w_build"][0] * 1e-3) / 1e12 / PEAK_FP64_MFMA_TFLOPS, 4),
              "peak_measured": peak64}
        if g:
            fp["error_rel"] = float(f"{(e64 - g['energy']) / abs(g['energy']):.3e}")
        result["fp64_same_fragment"] = fp
        log("# float64 evaluation done")
        del ws64, d64, fr64
    if not args.no_cpu:
        host = df.host()
        del df, fr
        torch.cuda.empty_cache()
        result["cpu_baseline"] = cpu_baseline(host)
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof.items()}


def run_single(args, result, name, mode):
    import torch
    import paper_2412_18553_amd as sie
    from synth import WORKLOADS
    from synth.device import workload_fragment_device
    w = WORKLOADS[name]
    o, v = w["n_occ"], w["n_vir"]
    F = flops(o, v)
    dev = torch.device("cuda:0")
    # the gradient in either precision (split: float32 inputs, the bf16 hi/lo
    # rebuild, FP64 contractions); the fp64 line is the float64 energy only
    prec = args.precision or "fp64"
    t0 = time.perf_counter()
    df = workload_fragment_device(
        name, device=dev, dtype=torch.float32 if prec == "split_bf16" else torch.float64)
    log(f"# workload {name}: built on the GPU in {time.perf_counter() - t0:.1f} s")
    fr = frag_of(df, prec)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    desc = f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}"
    if prec == "split_bf16":
        desc += ", float32 inputs"
    if mode == "backward":
        ws = torch.empty(sie.backward_workspace_size(fr), dtype=torch.uint8, device=dev)
        grads = [{n: torch.empty_like(getattr(fr, n), dtype=torch.float64)
                  for n in sie.GRAD_NAMES}]
        grads[0].update({n: torch.empty(len(getattr(fr, n)), dtype=torch.float64, device=dev)
                         for n in sie.EPS_GRAD_NAMES})
        step = lambda: sie.backward(fr, grads=grads, e_frag=out, workspace=ws)  # noqa: E731
    else:
        ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
        step = lambda: sie.energy(fr, workspace=ws, out=out)  # noqa: E731
    ms, prof = timed(step, args.steps, args.warmup)
    energy = float(out.item())
    peak64 = measured_peak(0)
    if mode == "fp64":
        result.update(value=round(F / (ms * 1e-3) / 1e12, 3), dtype="f64",
                      config={"workload": desc, "precision": "fp64", "fragments": 1})
        lay = sie.tile_variants()[sie.tile_variant_of(v)][6]
        kernel = {2: "k_build_w_f64", 3: "k_build_w3_f64"}[lay]
        result["roofline"] = roofline(prof, "w_build", kernel, F, args.steps,
                                      PEAK_FP64_MFMA_TFLOPS, measured=peak64, workload=name)
        result["roofline"]["tile_variant"] = sie.tile_variant_of(v)
        g = stored_oracle(f"{name}.json")
        if g:
            result["accuracy"] = {"oracle_energy": g["energy"],
                                  "error_rel": float(f"{(energy - g['energy']) / abs(g['energy']):.3e}")}
    else:
        # the backward recomputes the build (F) and runs the transposed
        # contractions of every build term (2F): 3F per step
        result.update(metric="(T) gradient TFLOP/s (3 x F per step)",
                      value=round(3.0 * F / (ms * 1e-3) / 1e12, 3),
                      dtype="f64" if prec == "fp64" else "bf16x3/f32 rebuild, f64 contractions",
                      config={"workload": desc, "precision": prec, "fragments": 1,
                              "outputs": "dE/d(t1, t2, ovvv, ooov, ovov, eps_occ, eps_vir)"})
        # (counter traffic is recorded for the float64 gradient only)
        result["roofline"] = roofline(prof, "grad", "k_adj_contract", 2.0 * F, args.steps,
                                      PEAK_FP64_MFMA_TFLOPS, measured=peak64,
                                      workload=name if prec == "fp64" else None)
    result.update(ms_per_step=round(ms, 3), fragments_per_s=round(1000.0 / ms, 4), energy=energy)
    if mode == "fp64" and not args.no_cpu:
        host = df.host()
        del df, fr
        torch.cuda.empty_cache()
        result["cpu_baseline"] = cpu_baseline(host)
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof.items()}


def run_df(args, result, name):
    """The split-precision energy of a fragment given its density-fitting
    factors (sie_triples_energy_df): the library forms (jl|ia), (ia|jb) in
    float32 and (ia|bc) one occupied slice at a time straight into its bf16
    hi/lo copies.  Timed like the split line (factors, t1 and t2 resident in
    HBM); also reports the caller-side input bytes against the integral-block
    form and the energy against the block form's on the same fragment."""
    import torch
    import paper_2412_18553_amd as sie
    from synth import WORKLOADS
    from synth.device import workload_df_factors_device, workload_fragment_device
    w = WORKLOADS[name]
    o, v = w["n_occ"], w["n_vir"]
    F = flops(o, v)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    fb = workload_fragment_device(name, device=dev, dtype=torch.float32)
    b = workload_df_factors_device(name, device=dev)
    log(f"# workload {name}: factors and float32 inputs built in {time.perf_counter() - t0:.1f} s")
    block_bytes = sum(x.numel() * 4 for x in (fb.t1, fb.t2, fb.ovvv, fb.ooov, fb.ovov))
    df_bytes = b.numel() * 8 + (fb.t1.numel() + fb.t2.numel()) * 4
    fr = frag_of(fb, "split_bf16")
    out = torch.empty(1, dtype=torch.float64, device=dev)
    ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
    sie.energy(fr, workspace=ws, out=out)
    e_block = float(out.item())
    t1, t2 = fb.t1, fb.t2
    eo, ev = fb.eps_occ, fb.eps_vir
    del fr, ws, fb
    torch.cuda.empty_cache()
    ws = torch.empty(sie.df_workspace_size(eo, ev, t1, t2, b, "split_bf16"), dtype=torch.uint8,
                     device=dev)
    step = lambda: sie.energy_df(eo, ev, t1, t2, b, "split_bf16", workspace=ws, out=out)  # noqa: E731
    ms, prof = timed(step, args.steps, args.warmup)
    energy = float(out.item())
    peak_bf16 = measured_peak(1)
    desc = (f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}, density-fitting "
            "factors (float64) and float32 amplitudes in")
    result.update(value=round(F / (ms * 1e-3) / 1e12, 3), dtype="bf16x3/f32",
                  config={"workload": desc, "precision": "split_bf16", "fragments": 1},
                  ms_per_step=round(ms, 3), fragments_per_s=round(1000.0 / ms, 4), energy=energy,
                  energy_block_form=e_block,
                  df_vs_block_rel=float(f"{(energy - e_block) / abs(e_block):.3e}"),
                  input_bytes={"density_fitting": df_bytes, "integral_blocks": block_bytes},
                  forming_and_staging_ms=round(prof["split"][0] / args.steps, 3))
    rl = roofline(prof, "w_build", split_kernel_name(v), F, args.steps, PEAK_BF16_MFMA_TFLOPS,
                  issued=3.0, measured=peak_bf16)
    result["roofline"] = rl
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof.items()}


def run_projector(args, result, name):
    """The fragment-projector matrix M of a fragment (E_x(C) = sum C M for any
    C; tr M = E_x), float64, with the unprojected energy of the same
    fragment timed alongside.  Work: the W-tilde build of every ordered
    occupied triple (i', j, k), j >= k, plus the n_o x n_o products over the
    cubes of each pair (j, k)."""
    import torch
    import paper_2412_18553_amd as sie
    from synth import WORKLOADS
    from synth.device import workload_fragment_device
    w = WORKLOADS[name]
    o, v = w["n_occ"], w["n_vir"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    df = workload_fragment_device(name, device=dev)
    log(f"# workload {name}: built on the GPU in {time.perf_counter() - t0:.1f} s")
    fr = frag_of(df, "fp64")
    groups = o * (o + 1) // 2
    build = float(groups * o) * (12.0 * v ** 4 + 12.0 * o * v ** 3)
    contract = float(groups) * 2.0 * o * o * v ** 3
    m = torch.empty((o, o), dtype=torch.float64, device=dev)
    step = lambda: sie.projector_matrix(fr, out=m)  # noqa: E731
    ms, prof = timed(step, args.steps, args.warmup)
    tr = float(torch.trace(m).item())
    out = torch.empty(1, dtype=torch.float64, device=dev)
    ws = torch.empty(sie.workspace_size(fr), dtype=torch.uint8, device=dev)
    e_step = lambda: sie.energy(fr, workspace=ws, out=out)  # noqa: E731
    ms_e, _ = timed(e_step, 1, 1)
    energy = float(out.item())
    peak64 = measured_peak(0)
    result.update(metric="projector matrix TFLOP/s (ordered-triple build + M products)",
                  value=round((build + contract) / (ms * 1e-3) / 1e12, 3), dtype="f64",
                  config={"workload": f"single fragment n_occ={o} n_vir={v} n_aux={w['n_aux']}",
                          "precision": "fp64", "fragments": 1, "outputs": "M [n_occ][n_occ]"},
                  ms_per_step=round(ms, 3), energy_ms=round(ms_e, 3),
                  cost_over_energy=round(ms / ms_e, 3), trace_m=tr, energy=energy,
                  trace_rel_err=float(f"{(tr - energy) / abs(energy):.3e}"))
    # ordered triples are built with a two-layout shape
    result["roofline"] = roofline(prof, "w_build", "k_build_w_f64", build, args.steps,
                                  PEAK_FP64_MFMA_TFLOPS, measured=peak64)
    result["roofline"]["work"] = "ordered-triple build flops"
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof.items()}


def run_batched(args, result, name):
    """One batched evaluation over a named batch (`--parts P`: the batch in P
    consecutive groups of fragments, each group's inputs built, evaluated in
    one batched call and freed, for batches whose inputs exceed the HBM; the
    step time is the sum over the groups).  With --singles every fragment is
    also evaluated alone (same workspace cap) for the batching speedup."""
    import torch
    import paper_2412_18553_amd as sie
    from synth import batch_shapes
    from synth.device import make_fragment_device
    prec = args.precision or "fp64"
    dtype = torch.float64 if prec == "fp64" else torch.float32
    dev = torch.device("cuda:0")
    shapes = batch_shapes(name)
    parts = max(1, min(args.parts, len(shapes)))
    bounds = [len(shapes) * q // parts for q in range(parts + 1)]
    ms_total, singles_ms = 0.0, 0.0
    prof_total = {}
    e_sum = 0.0
    for q in range(parts):
        sub = shapes[bounds[q]:bounds[q + 1]]
        t0 = time.perf_counter()
        frs = []
        for n, (o, v, aux, seed) in enumerate(sub):
            frs.append(frag_of(make_fragment_device(o, v, aux, seed, device=dev, dtype=dtype), prec))
            if n % 8 == 7:
                log(f"# part {q}: {n + 1} fragments built")
        log(f"# workload {name} part {q}: {len(frs)} fragments built on the GPU in "
            f"{time.perf_counter() - t0:.1f} s")
        try:
            ws_bytes = sie.workspace_size(frs)
        except sie.SieError:
            # the group's split copies of its inputs exceed the default cap:
            # give the library most of the free HBM instead
            cap = int(torch.cuda.mem_get_info(dev)[0] * 0.9)
            ws_bytes = sie.workspace_size(frs, max_bytes=cap)
            log(f"# part {q}: workspace cap raised to {cap / 2**30:.1f} GiB")
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        e_frag = torch.empty(len(frs), dtype=torch.float64, device=dev)
        e_tot = torch.empty(1, dtype=torch.float64, device=dev)
        step = lambda: sie.energy_batched(frs, workspace=ws, out=e_frag, total=e_tot)  # noqa: E731
        ms, prof = timed(step, args.steps, args.warmup)
        ms_total += ms
        e_sum += float(e_tot.item())
        for k, (t, c) in prof.items():
            t0_, c0_ = prof_total.get(k, (0.0, 0))
            prof_total[k] = (t0_ + t, c0_ + c)
        if args.singles:
            out = torch.empty(1, dtype=torch.float64, device=dev)
            for fr in frs:
                sie.energy(fr, workspace=ws, out=out)      # warm-up of this size
                torch.cuda.synchronize()
                start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                start.record()
                sie.energy(fr, workspace=ws, out=out)
                stop.record()
                torch.cuda.synchronize()
                singles_ms += start.elapsed_time(stop)
            log(f"# part {q}: singles timed")
        del frs, ws, step
        torch.cuda.empty_cache()
    ms = ms_total
    F = sum(flops(o, v) for (o, v, _, _) in shapes)
    result.update(value=round(F / (ms * 1e-3) / 1e12, 3),
                  dtype="f64" if prec == "fp64" else "bf16x3/f32",
                  config={"workload": f"{name}: {len(shapes)} fragments, n_occ "
                                      f"{min(s[0] for s in shapes)}..{max(s[0] for s in shapes)}, "
                                      f"n_vir {min(s[1] for s in shapes)}..{max(s[1] for s in shapes)}",
                          "precision": prec, "fragments": len(shapes), "batched_calls": parts},
                  ms_per_step=round(ms, 3), fragments_per_s=round(len(shapes) * 1000.0 / ms, 4),
                  energy=e_sum)
    if args.singles:
        result["singles"] = {"ms": round(singles_ms, 3),
                             "batching_speedup": round(singles_ms / ms, 4)}
    if prec == "fp64":   # the batch mixes the build shapes its fragment sizes select
        result["roofline"] = roofline(prof_total, "w_build", "k_build_w_f64 / k_build_w3_f64", F,
                                      args.steps, PEAK_FP64_MFMA_TFLOPS, measured=measured_peak(0))
    else:
        result["roofline"] = roofline(prof_total, "w_build", "k_build_w_bf16x3*", F, args.steps,
                                      PEAK_BF16_MFMA_TFLOPS, issued=3.0, measured=measured_peak(1))
    result["kernel_ms_per_step"] = {k: round(t / args.steps, 3) for k, (t, _) in prof_total.items()}


def run_mp2(args, result, name):
    """MP2 energy and 1-RDM blocks of one cluster from DF factors (the
    embedding workflow's BNO step).  A step is one sie_mp2 call with the
    density (amplitudes kept in the workspace).  The energy-only call, which
    runs the pair kernel alone, is timed separately for its roofline."""
    import torch
    import paper_2412_18553_amd as sie
    from synth import WORKLOADS, mp2_inputs
    from synth.fragments import SEED_ROOT
    w = WORKLOADS[name]
    o, v, na = w["n_occ"], w["n_vir"], w["n_aux"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    eo, ev, l = mp2_inputs(o, v, na, (SEED_ROOT, w["stream"], 0))
    lt = torch.from_numpy(l).to(dev)
    del l
    log(f"# workload {name}: factors built in {time.perf_counter() - t0:.1f} s")
    f_pair = 2.0 * o * o * v * v * na          # (ia|jb) for all ordered pairs
    f_dens = 2.0 * o * o * v ** 3 + 2.0 * o ** 3 * v * v
    for _ in range(args.warmup):
        sie.mp2(eo, ev, lt, want_density=True)
        torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        out = sie.mp2(eo, ev, lt, want_density=True)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    ws = torch.empty(sie._lib.load().sie_mp2_workspace_size(
        ctypes.byref(sie._lib.SieMp2Input(o, v, na, eo.ctypes.data, ev.ctypes.data,
                                          lt.data_ptr())), 0), dtype=torch.uint8, device=dev)
    sie.mp2(eo, ev, lt, workspace=ws)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        sie.mp2(eo, ev, lt, workspace=ws)
    stop.record()
    torch.cuda.synchronize()
    ms_pair = start.elapsed_time(stop) / args.steps
    achieved = f_pair / (ms_pair * 1e-3) / 1e12
    gamma_oo = out["gamma_oo"].cpu().numpy()
    gamma_vv = out["gamma_vv"].cpu().numpy()
    result.update(metric="MP2 energy + 1-RDM TFLOP/s", value=round((f_pair + f_dens) / (ms * 1e-3) / 1e12, 3),
                  dtype="f64",
                  config={"workload": f"cluster MP2 n_occ={o} n_vir={v} n_aux={na}, DF factors",
                          "precision": "fp64", "outputs": "E_MP2, gamma_oo, gamma_vv"},
                  ms_per_step=round(ms, 3), energy=float(out["energy"].item()),
                  electron_count=float(np.trace(gamma_oo) + np.trace(gamma_vv)),
                  roofline={"bound": "mfma", "kernel": "k_mp2_pair", "achieved": round(achieved, 3),
                            "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4), "traffic": None,
                            "avg_launch_ms": round(ms_pair, 4),
                            "work": "algorithmic 2 n_o^2 n_v^2 n_aux (energy-only call)"})


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the (T) path here is single-GPU "
              "(fragments would shard across GPUs as independent work; not built).",
              file=sys.stderr)
        sys.exit(2)
    # modes with one precision refuse another one (batched and backward take
    # either)
    fixed = {"split": "split_bf16", "df": "split_bf16", "fp64": "fp64", "projector": "fp64",
             "mp2": "fp64"}
    if args.precision and args.mode in fixed and args.precision != fixed[args.mode]:
        print(f"--mode {args.mode} runs in {fixed[args.mode]} only; --precision "
              f"{args.precision} applies to --mode batched and --mode backward",
              file=sys.stderr)
        sys.exit(2)

    import torch

    mode = args.mode
    name = args.workload or DEFAULT_WORKLOAD[mode]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"# calibration copy: {src.numel() * 8} bytes device to device")
        del src, dst
    result = {"metric": "(T) TFLOP/s", "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "data": "synthetic"}
    if mode == "peak":
        p64, p16 = measured_peak(0), measured_peak(1)
        result.update(metric="matrix-core peak TFLOP/s", value=p64, dtype="f64",
                      config={"workload": "register-only MFMA chains, 8192 work-groups"},
                      peaks={"fp64_16x16x4": {"measured": p64, "published": PEAK_FP64_MFMA_TFLOPS},
                             "bf16_16x16x32": {"measured": p16, "published": PEAK_BF16_MFMA_TFLOPS}})
    elif mode == "split":
        run_split(args, result, name)
    elif mode in ("fp64", "backward"):
        run_single(args, result, name, mode)
    elif mode == "mp2":
        run_mp2(args, result, name)
    elif mode == "projector":
        run_projector(args, result, name)
    elif mode == "df":
        run_df(args, result, name)
    else:
        run_batched(args, result, name)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
