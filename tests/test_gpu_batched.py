"""Batched evaluation (many fragments, one work list) on the GPU.

* every fragment's batched E_x equals the single-fragment call bitwise (the
  per-fragment reductions run in the same fixed order) and the CPU oracle;
* the total is the fixed-order sum of the fragment energies;
* a direct sum of two fragments (no cross integrals or amplitudes) has the
  energy of the two fragments (size extensivity);
* a workspace cap that forces many rounds changes nothing;
* a tile table that gives the fragments of one batch different build
  shapes (two- and three-layout) changes nothing either: each round then
  launches the build once per shape over that shape's items, and its
  epilogue reads two- and three-layout cube sets side by side.
"""

import numpy as np
import pytest

import oracle.triples as T
from synth import make_fragment

pytestmark = pytest.mark.gpu

SHAPES = [(3, 17, 20), (6, 50, 60), (2, 9, 12), (8, 40, 50), (5, 28, 40), (1, 12, 10),
          (7, 33, 40)]


def _frag(f, precision="fp64"):
    import torch
    import paper_2412_18553_amd as sie
    dt = np.float64 if precision == "fp64" else np.float32
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(dt))).to("cuda")  # noqa: E731
    return sie.Fragment(f.eps_occ, f.eps_vir, cast(f.t1), cast(f.t2), cast(f.ovvv),
                        cast(f.ooov), cast(f.ovov), precision)


def test_batched_equals_single_and_oracle():
    import paper_2412_18553_amd as sie
    hf = [make_fragment(o, v, a, (9, n)) for n, (o, v, a) in enumerate(SHAPES)]
    frs = [_frag(f) for f in hf]
    e_b, tot = sie.energy_batched(frs)
    e_b = e_b.cpu().numpy()
    singles = np.array([float(sie.energy(fr).item()) for fr in frs])
    assert np.array_equal(e_b, singles)
    for f, e in zip(hf, e_b):
        ref = T.energy_literal_vectorized(*f.arrays())
        assert abs(e - ref) <= 1e-10 * max(abs(ref), 1e-300) or (f.n_occ == 1 and e == 0.0)
    assert abs(float(tot.item()) - e_b.sum()) <= 1e-14 * abs(e_b.sum())


def test_batched_many_rounds():
    import paper_2412_18553_amd as sie
    hf = [make_fragment(o, v, a, (9, 50 + n)) for n, (o, v, a) in enumerate(SHAPES)]
    frs = [_frag(f) for f in hf]
    e_full, _ = sie.energy_batched(frs)
    # a small cap: the cube arena holds only a few occupied triples per round
    minimal = None
    for cap in (1 << 20, 4 << 20, 16 << 20, 64 << 20):
        try:
            minimal = sie.workspace_size(frs, max_bytes=cap)
            break
        except sie.SieError:
            continue
    assert minimal is not None
    e_small, _ = sie.energy_batched(frs, max_workspace_bytes=minimal)
    assert np.array_equal(e_full.cpu().numpy(), e_small.cpu().numpy())


def test_size_extensivity_direct_sum():
    import paper_2412_18553_amd as sie
    from test_oracle_pins import direct_sum
    fa = make_fragment(4, 19, 30, (9, 101))
    fb = make_fragment(3, 14, 24, (9, 102))
    arrs = direct_sum(fa.arrays(), fb.arrays())
    from synth import Fragment
    fab = Fragment(*arrs)
    e_a, e_b, e_ab = (float(sie.energy(_frag(f)).item()) for f in (fa, fb, fab))
    assert abs(e_ab - (e_a + e_b)) <= 1e-12 * abs(e_ab)


def test_batched_split():
    import paper_2412_18553_amd as sie
    hf = [make_fragment(o, v, a, (9, 200 + n)) for n, (o, v, a) in enumerate(SHAPES[:5])]
    frs = [_frag(f, "split_bf16") for f in hf]
    e_b, _ = sie.energy_batched(frs)
    singles = np.array([float(sie.energy(fr).item()) for fr in frs])
    assert np.array_equal(e_b.cpu().numpy(), singles)
    for f, e in zip(hf, e_b.cpu().numpy()):
        f32 = f.astype(np.float32)
        ref = T.energy_literal_vectorized(*[np.asarray(x, np.float64) for x in f32.arrays()])
        assert abs(e - ref) <= 1e-4 * abs(ref)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_batched_workspace_caps_agree(precision):
    """Workspace caps from the minimum to the full size group the units into
    different rounds: the per-fragment energies are bitwise the same, also
    when the same workspace is reused right away."""
    import paper_2412_18553_amd as sie
    hf = [make_fragment(o, v, a, (9, 300 + n)) for n, (o, v, a) in enumerate(SHAPES)]
    frs = [_frag(f, precision) for f in hf]
    e_full, _ = sie.energy_batched(frs)
    full = sie.workspace_size(frs)
    minimal = None
    for cap in (1 << 20, 4 << 20, 16 << 20, 64 << 20):
        try:
            minimal = sie.workspace_size(frs, max_bytes=cap)
            break
        except sie.SieError:
            continue
    assert minimal is not None and minimal < full
    caps = sorted({minimal, 2 * minimal, 3 * minimal, 5 * minimal, (minimal + full) // 2})
    for cap in caps:
        if cap >= full:
            continue
        for _ in range(2):
            e_cap, _ = sie.energy_batched(frs, max_workspace_bytes=sie.workspace_size(frs, max_bytes=cap))
            print(f"cap={cap}", flush=True)
            assert np.array_equal(e_full.cpu().numpy(), e_cap.cpu().numpy())


# n_v of SHAPES -> variant: 9, 12 -> 9 (three layouts), 17, 28 -> 0, 33, 40 -> 11
# (three layouts), 50 -> 6 (wave grid)
MIXED_TABLE = [(12, 9), (30, 0), (45, 11), (2048, 6)]


@pytest.mark.parametrize("cap_rounds", [False, True])
def test_batched_mixed_tile_variants(cap_rounds):
    import paper_2412_18553_amd as sie
    hf = [make_fragment(o, v, a, (9, 400 + n)) for n, (o, v, a) in enumerate(SHAPES)]
    frs = [_frag(f) for f in hf]
    try:
        sie.set_tile_table(MIXED_TABLE)
        variants = {sie.tile_variant_of(f.n_vir) for f in hf}
        layouts = {sie.tile_variants()[v][6] for v in variants}
        assert len(variants) >= 3 and layouts == {2, 3}, (variants, layouts)
        kw = {}
        if cap_rounds:   # a cap that forces several rounds, each mixing shapes
            kw["max_workspace_bytes"] = sie.workspace_size(frs, max_bytes=sie.workspace_size(frs) // 3)
        e_b, tot = sie.energy_batched(frs, **kw)
        e_b = e_b.cpu().numpy()
        singles = np.array([float(sie.energy(fr).item()) for fr in frs])
    finally:
        sie.set_tile_table(None)
    print(f"variants {sorted(variants)}: batched {e_b.tolist()}", flush=True)
    assert np.array_equal(e_b, singles)
    for f, e in zip(hf, e_b):
        ref = T.energy_literal_vectorized(*f.arrays())
        assert abs(e - ref) <= 1e-10 * max(abs(ref), 1e-300) or (f.n_occ == 1 and e == 0.0)
