"""Write oracle energies for the named synthetic workloads to tests/golden/.

Calls only oracle/ and synth/.  Usage (from the repository root):

    python tests/golden/make_golden.py o8v40 [o24v200 ...] [--workers N]
    python tests/golden/make_golden.py --units o32v320 [--workers N]
    python tests/golden/make_golden.py --all-units o32v320 [--f32] [--workers N]

The full-energy mode runs `oracle.energy_literal_vectorized` over a partition
of the outer virtual index a, one process per part, and fsums the parts.  The
--units mode evaluates `oracle.occupied_triple_energy` for a fixed sample of
occupied triples (used where the full oracle would take hours).  The
--all-units mode evaluates `oracle.occupied_triple_parts` (the occupied-outer
form) for every occupied triple i >= j >= k and stores the (E_WW, E_WV) pair
of each, in the per-triple index order u = i(i+1)(i+2)/6 + j(j+1)/2 + k, with
their compensated sums; finished triples are appended to a progress file
(<output>.progress.jsonl) so an interrupted run resumes.  With --f32 the
fragment's amplitudes and integrals are first rounded to float32 (the inputs
of the split-precision form) and the oracle runs on those values.
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import oracle  # noqa: E402
from synth import WORKLOADS, workload_fragment  # noqa: E402

_FRAG = None


def _part(a):
    t0 = time.perf_counter()
    e, ww, wv = oracle.energy_literal_vectorized(*_FRAG.arrays(), a_values=[a],
                                                 return_parts=True)
    return a, e, ww, wv, time.perf_counter() - t0


def _unit(ijk):
    t0 = time.perf_counter()
    e = oracle.occupied_triple_energy(*ijk, *_FRAG.arrays())
    return ijk, e, time.perf_counter() - t0


def _unit_parts(ijk):
    t0 = time.perf_counter()
    ww, wv = oracle.occupied_triple_parts(*ijk, *_FRAG.arrays())
    return ijk, ww, wv, time.perf_counter() - t0


def all_units(name, args, rec):
    """Every occupied triple of a workload with resume; returns the output path."""
    global _FRAG
    if args.f32:
        _FRAG = _FRAG.astype(np.float32).astype(np.float64)
    suffix = "_f32" if args.f32 else ""
    out = os.path.join(HERE, f"{name}{suffix}_all_units.json")
    prog = out + ".progress.jsonl"
    done = {}
    if os.path.exists(prog):
        with open(prog) as fh:
            for line in fh:
                line = line.strip()
                if line:
                    r = json.loads(line)
                    done[tuple(r["ijk"])] = r
    todo = [t for t in oracle.occupied_triples(_FRAG.n_occ) if t not in done]
    print(f"{name}: {len(done)} triples done, {len(todo)} to go", flush=True)
    ctx = mp.get_context("fork")
    with open(prog, "a") as fh, ctx.Pool(args.workers) as pool:
        for n, (t, ww, wv, sec) in enumerate(pool.imap_unordered(_unit_parts, todo, chunksize=1)):
            r = dict(ijk=list(t), e_ww=ww, e_wv=wv, seconds=sec)
            done[tuple(t)] = r
            fh.write(json.dumps(r) + "\n")
            fh.flush()
            if n % 50 == 0:
                print(f"{len(done)} triples done", flush=True)
    units = [done[t] for t in oracle.occupied_triples(_FRAG.n_occ)]
    rec["function"] = "oracle.occupied_triple_parts"
    rec["inputs"] = "float32-rounded amplitudes and integrals" if args.f32 else "float64"
    rec["e_ww_units"] = [u["e_ww"] for u in units]
    rec["e_wv_units"] = [u["e_wv"] for u in units]
    rec["e_ww"] = math.fsum(rec["e_ww_units"])
    rec["e_wv"] = math.fsum(rec["e_wv_units"])
    rec["energy"] = math.fsum(rec["e_ww_units"] + rec["e_wv_units"])
    rec["cpu_seconds"] = sum(u["seconds"] for u in units)
    return out


def unit_sample(n_occ):
    """Fixed sample of occupied triples i >= j >= k: corners, diagonals and a
    spread of interior triples."""
    o = n_occ - 1
    cand = [(o, o - 1, 0), (o, o, o - 1), (o, 0, 0), (1, 0, 0), (2, 1, 0),
            (o, o // 2, o // 3), (o // 2, o // 2, 1), (o - 2, o // 3, o // 4),
            (o, o - 2, o - 5 if o >= 5 else 0), (o // 3, o // 4, o // 5)]
    seen, out = set(), []
    for t in cand:
        if t[0] >= t[1] >= t[2] >= 0 and t not in seen and len(set(t)) > 1:
            seen.add(t)
            out.append(t)
    return out


def main():
    global _FRAG
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--units", action="store_true")
    ap.add_argument("--all-units", action="store_true")
    ap.add_argument("--f32", action="store_true")
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    ctx = mp.get_context("fork")
    for name in args.workloads:
        w = WORKLOADS[name]
        t0 = time.perf_counter()
        _FRAG = workload_fragment(name)
        rec = dict(workload=name, n_occ=w["n_occ"], n_vir=w["n_vir"],
                   n_aux=w["n_aux"], seed=[241218553, w["stream"], 0],
                   generator="synth.workload_fragment",
                   host=platform.node(), workers=args.workers,
                   command="python tests/golden/make_golden.py "
                           + ("--units " if args.units else "")
                           + ("--all-units " if args.all_units else "")
                           + ("--f32 " if args.f32 else "") + name)
        if args.all_units:
            out = all_units(name, args, rec)
        elif args.units:
            sample = unit_sample(w["n_occ"])
            with ctx.Pool(args.workers) as pool:
                res = pool.map(_unit, sample, chunksize=1)
            rec["function"] = "oracle.occupied_triple_energy"
            rec["units"] = [dict(ijk=list(t), energy=e, seconds=s) for t, e, s in res]
            out = os.path.join(HERE, f"{name}_units.json")
        else:
            a_order = sorted(range(w["n_vir"]), reverse=True)   # largest parts first
            with ctx.Pool(args.workers) as pool:
                res = list(pool.imap_unordered(_part, a_order, chunksize=1))
            res.sort()
            rec["function"] = "oracle.energy_literal_vectorized"
            rec["energy"] = math.fsum(r[1] for r in res)
            rec["e_ww"] = math.fsum(r[2] for r in res)
            rec["e_wv"] = math.fsum(r[3] for r in res)
            rec["cpu_seconds"] = sum(r[4] for r in res)
            out = os.path.join(HERE, f"{name}.json")
        rec["wall_seconds"] = time.perf_counter() - t0
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(out, json.dumps({k: rec[k] for k in rec if not k.endswith("units")}), flush=True)


if __name__ == "__main__":
    main()
