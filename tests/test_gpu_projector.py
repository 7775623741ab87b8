"""Fragment projector C^f of the in-situ (T) energy on the GPU
(sie_triples_projector_matrix, and sie_triples_energy with frag_proj set).

* small ragged fragments, float64: every entry of M against the oracle's
  dense M (oracle.projector_matrix, pinned by the projected energy of the
  unrestricted reading, its trace and a projector partition), within 1e-10 of
  the largest entry; E_x(C) for a random C against the oracle's projected
  energy (C applied to W-tilde first), 1e-10 relative;
* tr M equals the unprojected energy of the energy entry point (1e-12
  relative), also at 16 occupied / 120 virtuals, where the oracle's dense M
  is out of reach; a complete orthogonal set of fragment projectors sums to
  the unprojected energy there too;
* a workspace of one group per round gives the same M bit for bit (the
  groups are added into M in one fixed order);
* split precision against the float64 oracle (bound 1e-4 of the largest
  entry, reported);
* a non-finite frag_proj is rejected with SIE_ERR_NONFINITE.
"""

import numpy as np
import pytest

import oracle
from synth import make_fragment

pytestmark = pytest.mark.gpu


def _frag(f, precision="fp64", frag_proj=None):
    import torch
    import paper_2412_18553_amd as sie
    dt = torch.float64 if precision == "fp64" else torch.float32
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    return sie.Fragment(f.eps_occ, f.eps_vir, cast(f.t1), cast(f.t2), cast(f.ovvv),
                        cast(f.ooov), cast(f.ovov), precision, frag_proj=frag_proj)


def _m(fr, **kw):
    import torch
    import paper_2412_18553_amd as sie
    m = sie.projector_matrix(fr, **kw)
    torch.cuda.synchronize()
    return m.cpu().numpy()


def _e(fr):
    import torch
    import paper_2412_18553_amd as sie
    e = sie.energy(fr)
    torch.cuda.synchronize()
    return float(e.item())


def _rand_proj(o, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(o, o))


def _partition(o, seed):
    """Two orthogonal projectors onto complementary subspaces (sum = I)."""
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.normal(size=(o, o)))
    h = max(1, o // 3)
    return u[:, :h] @ u[:, :h].T, u[:, h:] @ u[:, h:].T


@pytest.mark.parametrize("o,v,aux,seed", [
    (2, 3, 8, 1), (3, 9, 24, 2), (4, 12, 30, 3), (5, 20, 60, 4),
    (3, 33, 40, 5), (6, 41, 60, 6)])
def test_projector_matrix_vs_oracle(o, v, aux, seed):
    f = make_fragment(o, v, aux, (seed, 7))
    args = f.arrays()
    m_ref = oracle.projector_matrix(*args)
    m = _m(_frag(f))
    scale = np.abs(m_ref).max()
    err = np.abs(m - m_ref).max() / scale
    print(f"o={o} v={v}: max|dM|/max|M| = {err:.2e}", flush=True)
    assert err <= 1e-10
    c = _rand_proj(o, seed)
    e_ref = oracle.energy_dense(*args, frag_proj=c, form="unrestricted")
    e_c = _e(_frag(f, frag_proj=c))
    assert abs(e_c - e_ref) <= 1e-10 * float(np.sum(np.abs(c * m_ref)))
    e_full = _e(_frag(f))
    assert abs(np.trace(m) - e_full) <= 1e-12 * abs(e_full)


def test_projector_identity_and_partition_mid():
    f = make_fragment(16, 120, 300, (42, 7))
    m = _m(_frag(f))
    e_full = _e(_frag(f))
    print(f"tr M = {np.trace(m):.15e}, E = {e_full:.15e}", flush=True)
    assert abs(np.trace(m) - e_full) <= 1e-12 * abs(e_full)
    e_id = _e(_frag(f, frag_proj=np.eye(16)))
    assert abs(e_id - e_full) <= 1e-12 * abs(e_full)
    p1, p2 = _partition(16, 42)
    e1, e2 = _e(_frag(f, frag_proj=p1)), _e(_frag(f, frag_proj=p2))
    assert abs(e1 + e2 - e_full) <= 1e-11 * abs(e_full)
    assert abs(e1 - float(np.sum(p1 * m))) <= 1e-12 * abs(e_full)


def test_projector_rounds_bitwise():
    import paper_2412_18553_amd as sie
    from paper_2412_18553_amd import _lib
    import ctypes
    f = make_fragment(5, 40, 60, (9, 7))
    fr = _frag(f)
    m_all = _m(fr)
    lib = _lib.load()
    one = lib.sie_triples_projector_workspace_size(ctypes.byref(fr.desc),
                                                   sie.PRECISIONS["fp64"], 1)
    assert one == 0      # a cap of one byte is below one group
    full = lib.sie_triples_projector_workspace_size(ctypes.byref(fr.desc),
                                                    sie.PRECISIONS["fp64"], 0)
    # smallest workspace: fixed part plus one group of 2 n_o cubes
    lo, hi = 1, full
    while lo < hi:
        mid = (lo + hi) // 2
        if lib.sie_triples_projector_workspace_size(ctypes.byref(fr.desc),
                                                    sie.PRECISIONS["fp64"], mid):
            hi = mid
        else:
            lo = mid + 1
    m_one = _m(fr, max_workspace_bytes=lo)
    assert lo < full
    assert np.array_equal(m_one, m_all)


@pytest.mark.parametrize("o,v,aux,seed", [(3, 9, 24, 2), (5, 20, 60, 4), (6, 41, 60, 6)])
def test_projector_split(o, v, aux, seed):
    f = make_fragment(o, v, aux, (seed, 7))
    m_ref = oracle.projector_matrix(*f.arrays())
    m = _m(_frag(f, "split_bf16"))
    err = np.abs(m - m_ref).max() / np.abs(m_ref).max()
    print(f"split o={o} v={v}: max|dM|/max|M| = {err:.2e}", flush=True)
    assert err <= 1e-4


def test_projector_nonfinite_rejected():
    import paper_2412_18553_amd as sie
    f = make_fragment(3, 9, 24, (2, 7))
    c = np.eye(3)
    c[1, 2] = np.nan
    with pytest.raises(sie.SieError, match="non-finite"):
        _e(_frag(f, frag_proj=c))


def test_projector_single_occupied():
    """One occupied orbital: M is 1 x 1 (the i = j = k triple, whose
    contribution vanishes but for rounding: W-tilde and Z are symmetric in
    abc, which R' annihilates), and E(C) = C M exactly."""
    f = make_fragment(1, 20, 30, (7, 1))
    m = _m(_frag(f))
    assert m.shape == (1, 1) and np.isfinite(m).all()
    e_ref = oracle.energy_dense(*f.arrays())
    assert e_ref == 0.0 or abs(e_ref) < 1e-12
    assert _e(_frag(f, frag_proj=np.array([[0.7]]))) == 0.7 * float(m[0, 0])
