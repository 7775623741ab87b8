"""Autotuner for the tile shapes of the W-tilde build (float64 and split).

python -m paper_2412_18553_amd.autotune [--nv 48,64,...] [--n-occ 8] [--write] [--split]

For each virtual-orbital count in the list it times every compiled tile
variant (sie_tile_variants: W-tilde build plus epilogue) on one synthetic
fragment of that size (random
inputs of the right shapes; the values do not change the work), keeps the
fastest (the default variant 0 is kept unless another is faster by more than
--margin, so that timing noise does not flip the table), merges neighbouring
sizes with the same winner into ranges and prints the table.  With --write it rewrites csrc/tile_table.inc, the table
compiled into the library (rebuild afterwards with
`python -m paper_2412_18553_amd.build`).  With --split it times the
split-precision build shapes (sie_set_split_shape) on float32 fragments
instead, keeping the padded-area choice unless another shape is faster by
more than the margin, and --write rewrites csrc/split_table.inc.  Needs a GPU.
"""

from __future__ import annotations

import argparse
import json
import os

import torch

from . import Fragment, energy, profile_collect, profile_enable, set_split_shape, \
    set_split_table, set_tile_table, split_shape_of, tile_variants, workspace_size

SPLIT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "split_table.inc")
N_SPLIT_SHAPES = 6

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "tile_table.inc")


def random_fragment(n_occ: int, n_vir: int, seed: int = 0, split: bool = False) -> Fragment:
    g = torch.Generator(device="cuda").manual_seed(seed)
    dev = torch.device("cuda")
    dt = torch.float32 if split else torch.float64

    def rnd(*shape):
        return (0.01 * torch.randn(*shape, generator=g, device=dev, dtype=torch.float64)).to(dt)

    eps_occ = [-1.0 - 0.01 * i for i in range(n_occ)]
    eps_vir = [0.5 + 0.01 * a for a in range(n_vir)]
    o, v = n_occ, n_vir
    return Fragment(eps_occ, eps_vir, rnd(o, v), rnd(o, o, v, v), rnd(o, v, v, v), rnd(o, o, o, v),
                    rnd(o, v, o, v), "split_bf16" if split else "fp64")


def time_split_shape(frag: Fragment, shape: int, reps: int) -> float:
    """Milliseconds of split build plus epilogue per evaluation with `shape` forced."""
    set_split_shape(shape)
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


def write_table(table, results, path=TABLE, split=False) -> None:
    if split:
        lines = ["// Split-precision build tile table: {n_v upper bound, shape}, ascending; n_v",
                 "// past the last bound takes the padded-area rule of sie::split_shape_of.",
                 "// Written by paper_2412_18553_amd/autotune.py --split from build plus",
                 "// epilogue times (ms) per shape measured on MI355X:"]
    else:
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
    ap.add_argument("--table-path", default=None, help="where --write puts the table")
    ap.add_argument("--split", action="store_true", help="tune the split-precision shapes")
    args = ap.parse_args()
    shapes = tile_variants()
    best, results = [], []
    try:
        if args.split:
            set_split_table([])          # the area rule is the reference choice
        for nv in [int(x) for x in args.nv.split(",")]:
            frag = random_fragment(args.n_occ or min(24, max(8, nv // 8)), nv, split=args.split)
            times = []
            count = N_SPLIT_SHAPES if args.split else len(shapes)
            ref = split_shape_of(nv) if args.split else 0
            for v in range(count):
                times.append(time_split_shape(frag, v, args.reps) if args.split
                             else time_variant(frag, v, args.reps))
                print(f"# n_vir {nv} {'shape' if args.split else 'variant'} {v}: "
                      f"{times[-1]:.3f} ms", flush=True)
            win = min(range(len(times)), key=times.__getitem__)
            if times[ref] <= (1.0 + args.margin) * times[win]:
                win = ref
            best.append((nv, win))
            results.append((nv, times))
            print(json.dumps({"n_vir": nv, "ms": [round(t, 3) for t in times], "best": win}),
                  flush=True)
            del frag
            torch.cuda.empty_cache()
    finally:
        set_tile_table(None)
        set_split_shape(-1)
        set_split_table(None)
    table = merge(best)
    print(json.dumps({"shapes": shapes, "table": table, "split": args.split}), flush=True)
    if args.write:
        path = args.table_path or (SPLIT_TABLE if args.split else TABLE)
        write_table(table, results, path, split=args.split)


if __name__ == "__main__":
    main()
