"""Autotuner for the tile shape of the float64 W-tilde build.

python -m paper_2412_18553_amd.autotune [--nv 48,64,...] [--n-occ 8] [--write]

For each virtual-orbital count in the list it times every compiled tile
variant (sie_tile_variants: W-tilde build plus epilogue) on one synthetic
fragment of that size (random
inputs of the right shapes; the values do not change the work), keeps the
fastest (the default variant 0 is kept unless another is faster by more than
--margin, so that timing noise does not flip the table), merges neighbouring
sizes with the same winner into ranges and prints the table.  With --write it rewrites csrc/tile_table.inc, the table
compiled into the library (rebuild afterwards with
`python -m paper_2412_18553_amd.build`).  Needs a GPU.
"""

from __future__ import annotations

import argparse
import json
import os

import torch

from . import Fragment, energy, profile_collect, profile_enable, set_tile_table, tile_variants, \
    workspace_size

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "tile_table.inc")


def random_fragment(n_occ: int, n_vir: int, seed: int = 0) -> Fragment:
    g = torch.Generator(device="cuda").manual_seed(seed)
    dev = torch.device("cuda")

    def rnd(*shape):
        return 0.01 * torch.randn(*shape, generator=g, device=dev, dtype=torch.float64)

    eps_occ = [-1.0 - 0.01 * i for i in range(n_occ)]
    eps_vir = [0.5 + 0.01 * a for a in range(n_vir)]
    o, v = n_occ, n_vir
    return Fragment(eps_occ, eps_vir, rnd(o, v), rnd(o, o, v, v), rnd(o, v, v, v), rnd(o, o, o, v),
                    rnd(o, v, o, v))


def time_variant(frag: Fragment, variant: int, reps: int) -> float:
    """Milliseconds of W-tilde build plus epilogue per evaluation with `variant`
    forced (the three-layout shapes leave the epilogue a third cube to read)."""
    set_tile_table([(2048, variant)])
    ws = torch.empty(workspace_size(frag), dtype=torch.uint8, device=frag.device)
    out = torch.empty(1, dtype=torch.float64, device=frag.device)
    energy(frag, workspace=ws, out=out)          # warm-up
    torch.cuda.synchronize()
    profile_enable(True)
    for _ in range(reps):
        energy(frag, workspace=ws, out=out)
    prof = profile_collect()
    profile_enable(False)
    return (prof["w_build"][0] + prof["epilogue"][0]) / reps


def merge(best):
    """[(n_vir, variant)] ascending -> [(upper bound, variant)] ranges."""
    table = []
    for q, (nv, var) in enumerate(best):
        bound = 2048 if q + 1 == len(best) else (nv + best[q + 1][0]) // 2
        if table and table[-1][1] == var:
            table[-1] = (bound, var)
        else:
            table.append((bound, var))
    return table


def write_table(table, results, path=TABLE) -> None:
    lines = ["// Float64 W-tilde build tile table: {n_v upper bound, variant}, ascending.",
             "// Written by paper_2412_18553_amd/autotune.py from W-tilde build plus",
             "// epilogue times (ms) per variant measured on MI355X:"]
    for nv, times in results:
        lines.append(f"//   n_v = {nv}: " + ", ".join(f"v{v} {t:.3f}" for v, t in enumerate(times)))
    lines += [f"{{{b}, {v}}}," for b, v in table]
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nv", default="48,64,80,96,120,160,200,240,320,400")
    ap.add_argument("--n-occ", type=int, default=0,
                    help="occupied orbitals of the timing fragment (0: n_v / 8 within [8, 24], "
                         "about the virtual-to-occupied ratio of the benchmark fragments)")
    ap.add_argument("--margin", type=float, default=0.01)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--table-path", default=TABLE, help="where --write puts the table")
    args = ap.parse_args()
    shapes = tile_variants()
    best, results = [], []
    try:
        for nv in [int(x) for x in args.nv.split(",")]:
            frag = random_fragment(args.n_occ or min(24, max(8, nv // 8)), nv)
            times = []
            for v in range(len(shapes)):
                times.append(time_variant(frag, v, args.reps))
                print(f"# n_vir {nv} variant {v}: {times[-1]:.3f} ms", flush=True)
            win = min(range(len(times)), key=times.__getitem__)
            if times[0] <= (1.0 + args.margin) * times[win]:
                win = 0
            best.append((nv, win))
            results.append((nv, times))
            print(json.dumps({"n_vir": nv, "ms": [round(t, 3) for t in times], "best": win}),
                  flush=True)
            del frag
            torch.cuda.empty_cache()
    finally:
        set_tile_table(None)
    table = merge(best)
    print(json.dumps({"shapes": shapes, "table": table}), flush=True)
    if args.write:
        write_table(table, results, args.table_path)


if __name__ == "__main__":
    main()
