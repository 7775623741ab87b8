"""Algebra behind the float32 epilogue's triple orbits, checked on the CPU.

The kernel (k_fp64.hpp, epi_triple_orbits) sums W-tilde R'[Z] / D of the
in-situ (T) energy (eq. E_corr_CCSD_T with R' of the closed-shell (T) form)
per virtual triple (a, b, c) together with its five other orderings, which
share D.  Two facts make that correct, and both are pinned here without the
GPU:

* the class-sum identity: with the cyclic orderings (abc, bca, cab) as even
  and the others as odd, sum over the six orderings of W R'[Z] equals
  3 sum W Z + (S_e - 2 S_o) W_e + (S_o - 2 S_e) W_o, where S and W with a
  class index are sums of Z and W over that class (checked against R' written
  out per ordering, as oracle/triples.py defines it);
* the counting rule for orbits of 8^3 blocks with repeated block indices:
  the threads' triples, taken with their six orderings and the kernel's
  weights (1, 1/2, 0), cover every virtual triple below n_v exactly once,
  except a = b = c, which R' annihilates and which is not counted.
"""

import itertools

import numpy as np
import pytest

ORDERINGS = {            # name: permutation of (a, b, c)
    "abc": (0, 1, 2), "bca": (1, 2, 0), "cab": (2, 0, 1),    # even
    "acb": (0, 2, 1), "bac": (1, 0, 2), "cba": (2, 1, 0),    # odd
}
EVEN = ("abc", "bca", "cab")
ODD = ("acb", "bac", "cba")


def _rprime_at(z, p):
    """R'[Z] at the ordered triple p = (p, q, r) of a virtual index set, with
    z a dict from index tuples to values: 4 Z_pqr + Z_rpq + Z_qrp
    - 2 (Z_rqp + Z_prq + Z_qpr)."""
    a, b, c = p
    return (4.0 * z[(a, b, c)] + z[(c, a, b)] + z[(b, c, a)]
            - 2.0 * (z[(c, b, a)] + z[(a, c, b)] + z[(b, a, c)]))


@pytest.mark.parametrize("seed", range(6))
def test_class_sum_identity(seed):
    rng = np.random.default_rng(seed)
    idx = (0, 1, 2)
    w = {}
    z = {}
    for name, perm in ORDERINGS.items():
        t = tuple(idx[k] for k in perm)
        w[t] = rng.normal()
        z[t] = rng.normal()
    direct = sum(w[t] * _rprime_at(z, t) for t in w)
    tup = {name: tuple(idx[k] for k in perm) for name, perm in ORDERINGS.items()}
    se = sum(z[tup[n]] for n in EVEN)
    so = sum(z[tup[n]] for n in ODD)
    we = sum(w[tup[n]] for n in EVEN)
    wo = sum(w[tup[n]] for n in ODD)
    swz = sum(w[t] * z[t] for t in w)
    classes = 3.0 * swz + (se - 2.0 * so) * we + (so - 2.0 * se) * wo
    assert abs(classes - direct) <= 1e-12 * (1.0 + abs(direct))


def test_class_sum_identity_planted_sign_fails():
    """A sign slip in the odd class (S_o + 2 S_e) breaks the identity."""
    rng = np.random.default_rng(11)
    idx = (0, 1, 2)
    w, z = {}, {}
    for perm in ORDERINGS.values():
        t = tuple(idx[k] for k in perm)
        w[t], z[t] = rng.normal(), rng.normal()
    direct = sum(w[t] * _rprime_at(z, t) for t in w)
    tup = {name: tuple(idx[k] for k in perm) for name, perm in ORDERINGS.items()}
    se = sum(z[tup[n]] for n in EVEN)
    so = sum(z[tup[n]] for n in ODD)
    we = sum(w[tup[n]] for n in EVEN)
    wo = sum(w[tup[n]] for n in ODD)
    swz = sum(w[t] * z[t] for t in w)
    wrong = 3.0 * swz + (se - 2.0 * so) * we + (so + 2.0 * se) * wo
    assert abs(wrong - direct) > 1e-6


def _weight(t0, t1b, t2b, x, y, zz):
    """The kernel's weight of the triple set with first-slot block triple
    (t0, t1b, t2b) (t0 >= t1b >= t2b) and in-block offsets (x, y, zz)."""
    e01, e12 = t0 == t1b, t1b == t2b
    if e01 and e12:
        if x > y > zz:
            return 1.0
        if x >= y >= zz and not (x == y == zz):
            return 0.5
        return 0.0
    if e01:
        return 1.0 if x > y else (0.5 if x == y else 0.0)
    if e12:
        return 1.0 if y > zz else (0.5 if y == zz else 0.0)
    return 1.0


@pytest.mark.parametrize("nv", [1, 7, 8, 13, 16, 21, 24])
def test_orbit_counting_covers_each_triple_once(nv):
    kb = 8
    nb = (nv + kb - 1) // kb
    count = {}
    for t0 in range(nb):
        for t1b in range(t0 + 1):
            for t2b in range(t1b + 1):
                for x, y, zz in itertools.product(range(kb), repeat=3):
                    a, b, c = kb * t0 + x, kb * t1b + y, kb * t2b + zz
                    if a >= nv or b >= nv or c >= nv:
                        continue
                    wgt = _weight(t0, t1b, t2b, x, y, zz)
                    if wgt == 0.0:
                        continue
                    for perm in ORDERINGS.values():
                        t = tuple((a, b, c)[k] for k in perm)
                        count[t] = count.get(t, 0.0) + wgt
    for t in itertools.product(range(nv), repeat=3):
        want = 0.0 if t[0] == t[1] == t[2] else 1.0
        assert count.get(t, 0.0) == want, (t, count.get(t, 0.0))
    assert set(count) <= set(itertools.product(range(nv), repeat=3))
