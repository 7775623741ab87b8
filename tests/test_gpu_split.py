"""Split-precision (bf16 hi/lo x3, float32 accumulation, float64 epilogue) (T)
on the GPU against the CPU oracle.

References, on the same float32 inputs:
* oracle.energy_literal_vectorized (float64, the method's exact value);
* oracle.split.energy_split_emulated (the split quantization, summed exactly).
The GPU differs from the emulator by float32 accumulation only (tolerance
5e-6 relative) and from the float64 oracle by the split error; the error in
micro-Eh is checked on chemically scaled fragments (DF factors scaled so
that |E| is of the order of 1e-2 Eh).
"""

import numpy as np
import pytest

import oracle.triples as T
from oracle.split import energy_split_emulated
from synth import make_fragment

pytestmark = pytest.mark.gpu


def run_split(f32):
    import torch
    import paper_2412_18553_amd as sie
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")  # noqa: E731
    e, tri = sie.triples_energy(f32.eps_occ, f32.eps_vir, cast(f32.t1), cast(f32.t2),
                                cast(f32.ovvv), cast(f32.ooov), cast(f32.ovov),
                                precision="split_bf16", return_triples=True)
    return float(e.item()), tri.cpu().numpy()


def refs(f32):
    a64 = [np.asarray(x, np.float64) for x in f32.arrays()]
    return T.energy_literal_vectorized(*a64), energy_split_emulated(*f32.arrays())


@pytest.mark.parametrize("o,v,aux,seed", [
    (2, 3, 8, 2), (3, 17, 20, 3), (5, 33, 40, 5), (7, 24, 30, 7), (9, 41, 50, 9),
    (6, 64, 60, 6)])
def test_split_small_vs_emulator(o, v, aux, seed):
    print(f"case o={o} v={v}", flush=True)
    f = make_fragment(o, v, aux, (8, seed)).astype(np.float32)
    e_gpu, tri = run_split(f)
    e64, e_em = refs(f)
    print(f"gpu={e_gpu!r} emulator={e_em!r} fp64={e64!r}", flush=True)
    assert abs(e_gpu - e_em) <= 5e-6 * abs(e_em)
    assert abs(e_gpu - e64) <= 1e-4 * abs(e64)
    assert abs(tri.sum() - e_gpu) <= 1e-12 * abs(e_gpu)


@pytest.mark.parametrize("o,v,aux,seed,scale", [(8, 40, 144, 1, 0.3), (10, 70, 240, 2, 0.25)])
def test_split_micro_hartree_chemical_scale(o, v, aux, seed, scale):
    f = make_fragment(o, v, aux, (8, 100 + seed), b_scale=scale).astype(np.float32)
    e_gpu, _ = run_split(f)
    e64, _ = refs(f)
    err_ueh = abs(e_gpu - e64) * 1e6
    print(f"|E|={abs(e64):.3e} Eh, split error {err_ueh:.4f} micro-Eh", flush=True)
    assert 1e-4 < abs(e64) < 1.0
    assert err_ueh <= 1.0


def test_split_one_occupied_zero():
    f = make_fragment(1, 20, 30, (8, 7)).astype(np.float32)
    e_gpu, tri = run_split(f)
    assert e_gpu == 0.0 and tri.tolist() == [0.0]


def test_split_deterministic():
    f = make_fragment(5, 37, 40, (8, 8)).astype(np.float32)
    e1, t1 = run_split(f)
    e2, t2 = run_split(f)
    assert e1 == e2 and np.array_equal(t1, t2)


_EMULATED = {}


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("o,v,aux,seed", [(4, 33, 40, 11), (3, 97, 60, 12)])
def test_split_every_tile_shape(shape, o, v, aux, seed):
    """Each split build shape, forced, against the emulator on one partial
    tile (v = 33) and on v = 97 (several row tiles for the 64-, 80- and
    112-row shapes, one partial col tile for all)."""
    import paper_2412_18553_amd as sie
    print(f"case shape={shape} o={o} v={v}", flush=True)
    f = make_fragment(o, v, aux, (8, seed)).astype(np.float32)
    sie.set_split_shape(shape)
    try:
        e_gpu, tri = run_split(f)
    finally:
        sie.set_split_shape(-1)
    key = (o, v, aux, seed)
    if key not in _EMULATED:
        _EMULATED[key] = energy_split_emulated(*f.arrays())
    e_em = _EMULATED[key]
    assert abs(e_gpu - e_em) <= 5e-6 * abs(e_em)
    assert abs(tri.sum() - e_gpu) <= 1e-12 * abs(e_gpu)


def test_split_every_tile_shape_multi_tile():
    """337 virtuals: at least two row tiles and two col tiles of every split
    shape (64/80/112/160 rows, 128/160/256/320 cols), each with a ragged
    edge, so every row0 > 0 and col0 > 0 path of both build kernels runs.
    Every output element accumulates its products in the same order whatever
    the tile shape, so the per-triple energies of all shapes are bitwise
    equal; one set is checked against the float64 oracle (stored per
    occupied triple, float32-rounded inputs)."""
    import json
    import os
    import paper_2412_18553_amd as sie
    import torch
    from synth.device import workload_fragment_device
    gpath = os.path.join(os.path.dirname(__file__), "golden", "o3v337_f32_all_units.json")
    with open(gpath) as fh:
        g = json.load(fh)
    ref = np.array(g["e_ww_units"]) + np.array(g["e_wv_units"])
    df = workload_fragment_device("o3v337", device="cuda", dtype=torch.float32)
    frag = sie.Fragment(*df.arrays(), precision="split_bf16")
    first = None
    try:
        for shape in range(6):
            print(f"case shape={shape} o=3 v=337", flush=True)
            sie.set_split_shape(shape)
            tri = torch.empty(frag.n_triples, dtype=torch.float64, device="cuda")
            sie.energy(frag, triples=tri)
            tri = tri.cpu().numpy()
            if first is None:
                first = tri
                err = np.abs(tri - ref).max() / np.abs(ref).max()
                print(f"  worst triple vs oracle: {err:.2e} of the largest", flush=True)
                assert err <= 2e-5
            assert np.array_equal(tri, first), shape
    finally:
        sie.set_split_shape(-1)


def test_split_product_set_on_gpu():
    """Operands x = h (1 + 2^-9) with h a bfloat16 number: the dropped lo*lo
    terms are a coherent 2^-18 of every product, so the three-product sum
    (hi*hi + hi*lo + lo*hi) and the exact value differ by about 2^-17 of
    E_WW.  The GPU must follow the three-product emulator far closer than
    that (float32 accumulation only)."""
    from oracle.split import bf16_rne
    f = make_fragment(4, 24, 30, (8, 77)).astype(np.float32)
    g = lambda x: bf16_rne(x) * np.float32(1.0 + 2.0 ** -9)  # noqa: E731
    f = f.replace(t2=g(f.t2), ovvv=g(f.ovvv), ooov=g(f.ooov))
    e_gpu, _ = run_split(f)
    e64, e_em = refs(f)
    gap = abs(e_em - e64)
    print(f"gpu={e_gpu!r} emulator={e_em!r} exact={e64!r}: |gpu - emulator| = "
          f"{abs(e_gpu - e_em) / abs(e_em):.2e}, lo*lo share {gap / abs(e64):.2e}", flush=True)
    assert gap >= 5e-6 * abs(e64)
    assert abs(e_gpu - e_em) <= 0.1 * gap


def test_split_orbit_table_second_chunk():
    """584 virtuals: 73 orbit blocks, 67525 orbits a unit and 264 for each of
    the unit's 256 epilogue work-groups, so the float32 epilogue decodes its
    orbit table in two chunks of 256.  The split energy is checked against
    the float64 path on the same float32-rounded inputs (whose epilogue does
    not use the table): every occupied triple within 2e-5 of the largest,
    the energy within 2e-6 relative."""
    import torch
    import paper_2412_18553_amd as sie
    from synth.device import make_fragment_device
    print("case o=2 v=584 aux=300", flush=True)
    df = make_fragment_device(2, 584, 300, (8, 584), device="cuda", dtype=torch.float32)

    def run(frag):
        tri = torch.empty(frag.n_triples, dtype=torch.float64, device="cuda")
        e = sie.energy(frag, triples=tri)
        torch.cuda.synchronize()
        return float(e.item()), tri.cpu().numpy()

    e_s, tri_s = run(sie.Fragment(*df.arrays(), precision="split_bf16"))
    d64 = [x.double() for x in df.arrays()[2:]]
    e_d, tri_d = run(sie.Fragment(df.eps_occ, df.eps_vir, *d64, precision="fp64"))
    del d64
    scale = np.abs(tri_d).max()
    err = np.abs(tri_s - tri_d).max() / scale
    print(f"split {e_s!r} float64 {e_d!r}: rel {abs(e_s - e_d) / abs(e_d):.2e}, "
          f"max triple error {err:.2e} of the largest", flush=True)
    assert scale > 0.0
    assert err <= 2e-5
    assert abs(e_s - e_d) <= 2e-6 * abs(e_d)
