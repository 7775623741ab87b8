"""(T) energy from density-fitting factors (sie_triples_energy_df): the
library forms (ia|bc), (jl|ia) and (ia|jb) from the factors itself; for the
split form (ia|bc) never exists as a float32 array (one occupied slice at a
time goes straight into the bf16 hi/lo copies).

* float64 from factors against the oracle energy of the same fragment (the
  host generator's integral blocks are the same factor products), 1e-10
  relative, on ragged sizes; per-triple output against the oracle's triples;
* float64 from factors against sie_triples_energy on the host-built blocks,
  1e-12 relative; many small rounds give the same energy bitwise;
* split from factors against the split energy on the float32-rounded
  host-built blocks (1e-7 relative: the formed blocks round to float32 in
  the same place except where a float64 sum lies on a rounding boundary),
  and against the float64 oracle within the split bound (1e-5);
* a NaN in the factors is reported with the finite check on.
"""

import numpy as np
import pytest

import oracle
from synth import make_fragment
from synth.fragments import df_factors

pytestmark = pytest.mark.gpu

CASES = [(2, 3, 8, 1), (3, 9, 24, 2), (4, 12, 30, 3), (5, 20, 60, 4), (3, 33, 40, 5),
         (6, 41, 60, 6), (7, 50, 90, 7)]


def _dev(x, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)


def _df_energy(f, b, precision="fp64", **kw):
    import torch
    import paper_2412_18553_amd as sie
    dt = torch.float64 if precision == "fp64" else torch.float32
    e = sie.energy_df(f.eps_occ, f.eps_vir, _dev(f.t1, dt), _dev(f.t2, dt),
                      _dev(b, torch.float64), precision, **kw)
    torch.cuda.synchronize()
    return float(e.item())


def _block_energy(f, precision="fp64"):
    import torch
    import paper_2412_18553_amd as sie
    dt = torch.float64 if precision == "fp64" else torch.float32
    fr = sie.Fragment(f.eps_occ, f.eps_vir, _dev(f.t1, dt), _dev(f.t2, dt), _dev(f.ovvv, dt),
                      _dev(f.ooov, dt), _dev(f.ovov, dt), precision)
    e = sie.energy(fr)
    torch.cuda.synchronize()
    return float(e.item())


@pytest.mark.parametrize("o,v,aux,seed", CASES)
def test_df_fp64_vs_oracle_and_blocks(o, v, aux, seed):
    print(f"case df fp64 o={o} v={v} aux={aux}", flush=True)
    f = make_fragment(o, v, aux, (seed, 11))
    b = df_factors(o, v, aux, (seed, 11))
    e_df = _df_energy(f, b)
    e_ref = oracle.energy_by_occupied_triples(*f.arrays())
    e_blk = _block_energy(f)
    print(f"  df {e_df!r} oracle {e_ref!r} blocks {e_blk!r}", flush=True)
    assert abs(e_df - e_ref) <= 1e-10 * abs(e_ref)
    assert abs(e_df - e_blk) <= 1e-12 * abs(e_blk)


def test_df_triples_and_rounds():
    import torch
    import paper_2412_18553_amd as sie
    o, v, aux = 6, 41, 60
    f = make_fragment(o, v, aux, (21, 11))
    b = df_factors(o, v, aux, (21, 11))
    tri = torch.empty(sie.occupied_triples(o), dtype=torch.float64, device="cuda")
    e_all = _df_energy(f, b, triples=tri)
    got = tri.cpu().numpy()
    ref = np.array([oracle.occupied_triple_energy(i, j, k, *f.arrays())
                    for (i, j, k) in oracle.occupied_triples(o)])
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    assert abs(got.sum() - e_all) <= 1e-12 * abs(e_all)
    # smallest workspace: one unit of cubes per round
    from paper_2412_18553_amd import _lib
    import ctypes
    eo, ev = np.ascontiguousarray(f.eps_occ), np.ascontiguousarray(f.eps_vir)
    t1, t2, bd = _dev(f.t1, torch.float64), _dev(f.t2, torch.float64), _dev(b, torch.float64)
    desc = _lib.SieFragmentDf(o, v, aux, eo.ctypes.data, ev.ctypes.data, t1.data_ptr(),
                              t2.data_ptr(), bd.data_ptr())
    lib = _lib.load()
    full = lib.sie_triples_df_workspace_size(ctypes.byref(desc), 0, 0)
    lo, hi = 1, full
    while lo < hi:
        mid = (lo + hi) // 2
        if lib.sie_triples_df_workspace_size(ctypes.byref(desc), 0, mid):
            hi = mid
        else:
            lo = mid + 1
    assert lo < full
    e_small = _df_energy(f, b, max_workspace_bytes=lo)
    assert e_small == e_all


@pytest.mark.parametrize("o,v,aux,seed", [(3, 9, 24, 2), (5, 20, 60, 4), (6, 41, 60, 6),
                                          (4, 97, 80, 8)])
def test_df_split(o, v, aux, seed):
    print(f"case df split o={o} v={v} aux={aux}", flush=True)
    f = make_fragment(o, v, aux, (seed, 11))
    b = df_factors(o, v, aux, (seed, 11))
    e_df = _df_energy(f, b, "split_bf16")
    e_blk = _block_energy(f, "split_bf16")
    e_ref = oracle.energy_by_occupied_triples(*f.arrays())
    print(f"  df split {e_df!r} blocks split {e_blk!r} oracle {e_ref!r}", flush=True)
    assert abs(e_df - e_blk) <= 1e-7 * abs(e_blk)
    assert abs(e_df - e_ref) <= 1e-5 * abs(e_ref)


def test_df_nonfinite_factors():
    import paper_2412_18553_amd as sie
    f = make_fragment(3, 9, 24, (2, 11))
    b = df_factors(3, 9, 24, (2, 11))
    b[5, 1, 7] = np.nan
    sie.set_check_finite(True)
    try:
        with pytest.raises(sie.SieError, match="NONFINITE"):
            _df_energy(f, b)
    finally:
        sie.set_check_finite(False)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_df_single_occupied_is_zero(precision):
    """One occupied orbital: the only occupied triple has i = j = k, whose
    contribution vanishes identically, so E_x = 0 exactly (the formed blocks
    and the staging still run)."""
    f = make_fragment(1, 20, 30, (7, 11))
    b = df_factors(1, 20, 30, (7, 11))
    assert _df_energy(f, b, precision) == 0.0
