"""MP2 energy, amplitudes and 1-RDM blocks on the GPU (sie_mp2) against the
CPU oracle (oracle/mp2.py, pinned by the spin-orbital formulas and the
electron-count identity).

* small and ragged sizes (virtual counts off the 64- and 32-wide tiles, odd
  auxiliary counts): energy within 1e-12 relative, every amplitude and
  density entry within 1e-12 of the block's largest;
* the energy alone (no amplitudes stored) equals the energy of the full call
  bitwise;
* a mid-size cluster: electron count tr gamma_oo + tr gamma_vv = 2 n_occ and
  symmetric blocks, energy against the oracle.
"""

import numpy as np
import pytest

from oracle.mp2 import amplitudes, mp2_density, mp2_energy, ovov_from_factors
from synth import mp2_inputs

pytestmark = pytest.mark.gpu


def run(eo, ev, l, **kw):
    import torch
    import paper_2412_18553_amd as sie
    lt = torch.from_numpy(np.ascontiguousarray(l)).to("cuda")
    out = sie.mp2(eo, ev, lt, **kw)
    torch.cuda.synchronize()
    return {k: (float(x.item()) if k == "energy" else x.cpu().numpy()) for k, x in out.items()}


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("o,v,naux,seed", [
    (1, 3, 2, 1), (2, 5, 7, 2), (3, 17, 21, 3), (4, 64, 40, 4), (5, 70, 33, 5), (6, 131, 60, 6)])
def test_mp2_vs_oracle(o, v, naux, seed):
    print(f"case mp2 o={o} v={v} naux={naux}", flush=True)
    eo, ev, l = mp2_inputs(o, v, naux, (41, seed))
    g = ovov_from_factors(l)
    got = run(eo, ev, l, want_t2=True, want_density=True)
    e = mp2_energy(eo, ev, g)
    print(f"  E gpu {got['energy']!r} oracle {e!r}", flush=True)
    assert abs(got["energy"] - e) <= 1e-12 * abs(e)
    assert rel(got["t2"], amplitudes(eo, ev, g)) <= 1e-12
    goo, gvv = mp2_density(eo, ev, g)
    assert rel(got["gamma_oo"] - 2 * np.eye(o), goo - 2 * np.eye(o)) <= 1e-12
    assert rel(got["gamma_vv"], gvv) <= 1e-12


def test_mp2_energy_only_matches_full_call():
    eo, ev, l = mp2_inputs(5, 70, 33, (41, 7))
    full = run(eo, ev, l, want_t2=True, want_density=True)
    only = run(eo, ev, l)
    assert only["energy"] == full["energy"]
    assert set(only) == {"energy"}


def test_mp2_mid_size_identities():
    eo, ev, l = mp2_inputs(24, 200, 672, (41, 8))
    print("case mp2 o=24 v=200 naux=672", flush=True)
    got = run(eo, ev, l, want_density=True)
    goo, gvv = got["gamma_oo"], got["gamma_vv"]
    tr = np.trace(goo) + np.trace(gvv)
    print(f"  tr gamma = {tr!r}", flush=True)
    assert abs(tr - 2 * 24) <= 1e-12 * 48
    assert rel(goo, goo.T) <= 1e-13 and rel(gvv, gvv.T) <= 1e-13
    e = mp2_energy(eo, ev, ovov_from_factors(l))
    assert abs(got["energy"] - e) <= 1e-12 * abs(e)
