"""The allocation-free entry point (sie_triples_energy_static) against the
workspace entry point (sie_triples_energy), through the C ABI.

Both run the same kernels in the same reduction order, so the energies and the
per-occupied-triple contributions must be bitwise equal; the energy is also
checked against the CPU oracle at 1e-10 relative.  Two calls in a row share
the GPU's static scratch, the second with a smaller fragment (and, in the
split case, a different precision), so a call that depended on what the
previous one left in the scratch would show here.
"""

import ctypes

import numpy as np
import pytest

import oracle.triples as T
from synth import make_fragment

pytestmark = pytest.mark.gpu


def _frag(f, precision):
    import torch
    import paper_2412_18553_amd as sie
    dt = torch.float64 if precision == "fp64" else torch.float32
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    return sie.Fragment(f.eps_occ, f.eps_vir, cast(f.t1), cast(f.t2), cast(f.ovvv),
                        cast(f.ooov), cast(f.ovov), precision)


def _both(fr):
    """(E, triples) from the static entry point, then from the workspace one."""
    import torch
    import paper_2412_18553_amd as sie
    from paper_2412_18553_amd import _lib
    lib = _lib.load()
    out_s = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    tri_s = torch.full((fr.n_triples,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.sie_triples_energy_static(ctypes.byref(fr.desc), sie.PRECISIONS[fr.precision],
                                       out_s.data_ptr(), tri_s.data_ptr(), stream)
    _lib.check(st)
    torch.cuda.synchronize()
    out_w = torch.empty(1, dtype=torch.float64, device="cuda")
    tri_w = torch.empty(fr.n_triples, dtype=torch.float64, device="cuda")
    sie.energy(fr, out=out_w, triples=tri_w)
    torch.cuda.synchronize()
    return (float(out_s.item()), tri_s.cpu().numpy()), (float(out_w.item()), tri_w.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_static_matches_workspace_entry_point_two_calls(precision):
    # first call: 6 occupied / 50 virtuals; second: smaller, 4 / 23 (ragged)
    for (o, v, aux, seed) in [(6, 50, 60, 31), (4, 23, 30, 32)]:
        print(f"case static {precision} o={o} v={v} seed={seed}", flush=True)
        f = make_fragment(o, v, aux, (11, seed))
        fr = _frag(f, precision)
        (e_s, t_s), (e_w, t_w) = _both(fr)
        assert e_s == e_w, (e_s, e_w)
        assert np.array_equal(t_s, t_w)
        if precision == "fp64":
            e_ref = T.energy_literal_vectorized(*f.arrays())
            assert abs(e_s - e_ref) <= 1e-10 * abs(e_ref), (e_s, e_ref)


def test_static_many_rounds_and_mixed_precisions():
    """A fragment whose cubes fill most of the scratch (so the call runs in
    many rounds), then a split call, then a small float64 call again."""
    cases = [("fp64", (5, 160, 60, 33)), ("split_bf16", (5, 64, 60, 34)),
             ("fp64", (3, 17, 20, 35))]
    for precision, (o, v, aux, seed) in cases:
        print(f"case static {precision} o={o} v={v} seed={seed}", flush=True)
        f = make_fragment(o, v, aux, (12, seed))
        fr = _frag(f, precision)
        (e_s, t_s), (e_w, t_w) = _both(fr)
        assert e_s == e_w, (precision, e_s, e_w)
        assert np.array_equal(t_s, t_w)


def test_static_rejects_oversized_fragment():
    import torch
    import paper_2412_18553_amd as sie
    from paper_2412_18553_amd import _lib
    o, v = 2, 400   # one unit's float64 cubes: 3 x 512 MB > 256 MiB
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")  # noqa: E731
    fr = sie.Fragment(np.linspace(-1.0, -0.5, o), np.linspace(0.2, 3.0, v), z(o, v),
                      z(o, o, v, v), z(o, v, v, v), z(o, o, o, v), z(o, v, o, v), "fp64")
    with pytest.raises(sie.SieError) as ex:
        sie.energy_static(fr)
    assert ex.value.status == _lib.SIE_ERR_WORKSPACE
