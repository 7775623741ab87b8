"""Pins of the MP2 oracle (oracle/mp2.py) against facts that do not come from
its own closed-shell code.

M1  spin-orbital brute force: energy and both density blocks from the
    textbook spin-orbital formulas on explicit spin orbitals (tiny inputs)
M2  electron count: tr gamma_oo + tr gamma_vv = 2 n_occ exactly (the
    correlation parts of the two blocks are the same sum with opposite signs)
M3  symmetry and sign: both blocks symmetric; gamma_vv positive semidefinite
    and the occupied natural occupations at most 2; E_MP2 < 0
M4  scaling: the amplitudes are linear and the energy and the density
    corrections quadratic in the integrals (factors L scaled by s: s^2 and s^4)
M5  factor route: (ia|jb) from L L^T equals the (T) workload's integrals
M   planted mistakes (exchange sign, a dropped factor 2) fail M1
"""

import numpy as np
import pytest

from oracle.mp2 import (amplitudes, mp2_density, mp2_energy, ovov_from_factors,
                        spin_orbital_mp2)


def inputs(o, v, naux, seed):
    rng = np.random.default_rng(seed)
    eo = np.sort(rng.uniform(-1.5, -0.3, o))
    ev = np.sort(rng.uniform(0.1, 3.0, v))
    l = rng.normal(0.0, 0.3, (o, v, naux))
    return eo, ev, l


@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 4, 1), (3, 4, 6, 2), (2, 5, 5, 3)])
def test_m1_spin_orbital_brute_force(o, v, naux, seed):
    eo, ev, l = inputs(o, v, naux, seed)
    g = ovov_from_factors(l)
    e = mp2_energy(eo, ev, g)
    goo, gvv = mp2_density(eo, ev, g)
    e_so, goo_so, gvv_so = spin_orbital_mp2(eo, ev, g)
    assert abs(e - e_so) <= 1e-13 * abs(e)
    assert np.abs(goo - goo_so).max() <= 1e-13
    assert np.abs(gvv - gvv_so).max() <= 1e-13 * max(np.abs(gvv).max(), 1e-300)


@pytest.mark.parametrize("o,v,naux,seed", [(4, 12, 20, 4), (6, 17, 30, 5)])
def test_m2_m3_trace_symmetry_sign(o, v, naux, seed):
    eo, ev, l = inputs(o, v, naux, seed)
    g = ovov_from_factors(l)
    goo, gvv = mp2_density(eo, ev, g)
    assert abs(np.trace(goo) + np.trace(gvv) - 2 * o) <= 1e-12 * 2 * o
    assert np.abs(goo - goo.T).max() <= 1e-14 * np.abs(goo).max()
    assert np.abs(gvv - gvv.T).max() <= 1e-14 * np.abs(gvv).max()
    assert np.linalg.eigvalsh(gvv).min() >= -1e-13 * np.abs(gvv).max()
    assert np.linalg.eigvalsh(goo).max() <= 2.0 + 1e-13
    assert mp2_energy(eo, ev, g) < 0.0


def test_m4_scaling():
    eo, ev, l = inputs(3, 7, 10, 6)
    s = 0.5
    g1, g2 = ovov_from_factors(l), ovov_from_factors(s * l)
    assert np.allclose(amplitudes(eo, ev, g2), s ** 2 * amplitudes(eo, ev, g1), rtol=1e-14,
                       atol=0)
    assert abs(mp2_energy(eo, ev, g2) - s ** 4 * mp2_energy(eo, ev, g1)) <= \
        1e-14 * abs(mp2_energy(eo, ev, g1))
    o1, v1 = mp2_density(eo, ev, g1)
    o2, v2 = mp2_density(eo, ev, g2)
    assert np.allclose(v2, s ** 4 * v1, rtol=1e-13, atol=0)
    assert np.allclose(o2 - 2 * np.eye(3), s ** 4 * (o1 - 2 * np.eye(3)), rtol=1e-13, atol=0)


def test_m5_factor_route_matches_workload_integrals():
    from synth import make_fragment
    from synth.fragments import ov_factors
    f = make_fragment(3, 9, 20, (31, 1))
    l = ov_factors(3, 9, 20, (31, 1))
    assert np.abs(ovov_from_factors(l) - f.ovov).max() <= 1e-14 * np.abs(f.ovov).max()


@pytest.mark.parametrize("mistake", ["exchange_sign", "factor_two"])
def test_planted_mistakes_fail_m1(mistake):
    eo, ev, l = inputs(2, 4, 5, 7)
    g = ovov_from_factors(l)
    t = amplitudes(eo, ev, g)
    k = g.transpose(0, 2, 1, 3)
    if mistake == "exchange_sign":
        e_bad = float(np.sum(t * (2 * k + k.transpose(0, 1, 3, 2))))
    else:
        e_bad = float(np.sum(t * (k - k.transpose(0, 1, 3, 2))))
    e_so, _, _ = spin_orbital_mp2(eo, ev, g)
    assert abs(e_bad - e_so) > 1e-6 * abs(e_so)
