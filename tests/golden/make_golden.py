"""Write oracle energies for the named synthetic workloads to tests/golden/.

Calls only oracle/ and synth/.  Usage (from the repository root):

    python tests/golden/make_golden.py o8v40 [o24v200 ...] [--workers N]
    python tests/golden/make_golden.py --units o32v320 [--workers N]

The full-energy mode runs `oracle.energy_literal_vectorized` over a partition
of the outer virtual index a, one process per part, and fsums the parts.  The
--units mode evaluates `oracle.occupied_triple_energy` for a fixed sample of
occupied triples (used where the full oracle would take hours).
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
                           + ("--units " if args.units else "") + name)
        if args.units:
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
        print(out, json.dumps({k: rec[k] for k in rec if k != "units"}), flush=True)


if __name__ == "__main__":
    main()
