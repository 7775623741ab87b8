"""Pins of the CPU oracle against facts that do not come from the oracle itself.

P1  closed-shell formula == textbook spin-orbital (T) (oracle/spinorb.py), on
    random inputs with only the twin symmetries the formula assumes
P2  MP2 amplitudes, t1 = 0  ==  MP4 triples over strictly ordered spin orbitals
P3  exact zeros: t2 = 0, one occupied, one virtual, i = j = k, C = 0
P4  sign: t1 = 0  =>  E <= 0
P5  polynomial structure in t1, t2 and the (ov|vv), (oo|ov) blocks
P6  invariance under relabelling occupied or virtual orbitals
P7  twin invariance: reading the other twin of each symmetric block
P8  size extensivity for a direct sum of two fragments
P9  fragment projector: linear, and a complete set sums to C = I
P10 literal, vectorized, dense, unrestricted, per-occupied-triple and
    occupied-outer (R on the virtual indices) forms agree, part by part
M   planted mistakes in the oracle fail P1 (the pins have teeth)
"""

import json
import os

import numpy as np
import pytest

import oracle
import oracle.triples as T
from oracle.spinorb import mp4_triples_ordered, spin_orbital_triples
from synth import make_fragment, workload_fragment

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_symmetric_inputs(o, v, seed, t1_scale=0.1):
    """Random inputs with exactly the twin symmetries the (T) formula assumes,
    and nothing else (not density-fitted, amplitudes not MP2)."""
    rng = np.random.default_rng(seed)
    eps_occ = np.sort(rng.uniform(-2.0, -0.5, o))
    eps_vir = np.sort(rng.uniform(0.2, 2.0, v))
    t1 = t1_scale * rng.normal(size=(o, v))
    t2 = rng.normal(size=(o, o, v, v))
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    ovvv = rng.normal(size=(o, v, v, v))
    ovvv = 0.5 * (ovvv + ovvv.transpose(0, 1, 3, 2))
    ooov = rng.normal(size=(o, o, o, v))
    ooov = 0.5 * (ooov + ooov.transpose(1, 0, 2, 3))
    ovov = rng.normal(size=(o, v, o, v))
    ovov = 0.5 * (ovov + ovov.transpose(2, 3, 0, 1))
    return eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- P1, P2
@pytest.mark.parametrize("o,v,seed", [(2, 2, 1), (2, 3, 2), (3, 3, 3),
                                      (3, 4, 4), (3, 5, 5), (2, 5, 6)])
def test_p1_spin_orbital_random(o, v, seed):
    args = random_symmetric_inputs(o, v, seed)
    e_cs = oracle.energy_literal(*args)
    e_so = spin_orbital_triples(*args)
    assert abs(e_cs) > 1e-6
    assert rel(e_cs, e_so) < 1e-12


@pytest.mark.parametrize("o,v,aux,seed", [(3, 4, 12, 11), (3, 5, 16, 12)])
def test_p1_spin_orbital_df(o, v, aux, seed):
    f = make_fragment(o, v, aux, (seed,))
    assert rel(oracle.energy_literal(*f.arrays()),
               spin_orbital_triples(*f.arrays())) < 1e-12


@pytest.mark.parametrize("o,v,aux,seed", [(2, 4, 10, 21), (3, 4, 14, 22)])
def test_p2_mp4_limit(o, v, aux, seed):
    f = make_fragment(o, v, aux, (seed,), zero_t1=True)
    e = oracle.energy_literal(*f.arrays())
    e4 = mp4_triples_ordered(f.eps_occ, f.eps_vir, f.t2, f.ovvv, f.ooov)
    assert e < 0
    assert rel(e, e4) < 1e-12


# ---------------------------------------------------------------- P3, P4
def test_p3_zeros():
    args = list(random_symmetric_inputs(3, 4, 31))
    z = list(args)
    z[3] = np.zeros_like(args[3])                     # t2 = 0
    assert oracle.energy_literal(*z) == 0.0
    e = oracle.energy_literal(*args)
    # zero up to rounding: compare with the magnitude of a same-sized case
    one_occ = random_symmetric_inputs(1, 5, 32)
    assert abs(oracle.energy_literal(*one_occ)) < 1e-12 * abs(e)
    one_vir = random_symmetric_inputs(4, 1, 33)
    assert abs(oracle.energy_literal(*one_vir)) < 1e-12 * abs(e)
    for i in range(3):
        assert abs(oracle.occupied_triple_energy(i, i, i, *args)) < 1e-12 * abs(e)
    assert oracle.energy_literal(*args, frag_proj=np.zeros((3, 3))) == 0.0


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_p4_sign(seed):
    args = list(random_symmetric_inputs(3, 4, seed))
    args[2] = np.zeros_like(args[2])
    assert oracle.energy_literal(*args) < 0.0


# ---------------------------------------------------------------- P5
def test_p5_polynomial():
    args = list(random_symmetric_inputs(3, 4, 51))
    e, e_ww, e_wv = oracle.energy_literal(*args, return_parts=True)
    assert rel(e, e_ww + e_wv) < 1e-14
    neg = list(args)
    neg[2] = -args[2]
    zero = list(args)
    zero[2] = np.zeros_like(args[2])
    e0 = oracle.energy_literal(*zero)
    assert rel(oracle.energy_literal(*neg) + e, 2 * e0) < 1e-12
    assert rel(e0, e_ww) < 1e-12
    s = 1.7
    sc = list(args)
    sc[2] = s * args[2]
    assert rel(oracle.energy_literal(*sc), e_ww + s * e_wv) < 1e-12
    st2 = list(zero)
    st2[3] = s * zero[3]
    assert rel(oracle.energy_literal(*st2), s * s * e0) < 1e-12
    si = list(args)
    si[4] = s * args[4]
    si[5] = s * args[5]
    assert rel(oracle.energy_literal(*si), s * s * e_ww + s * e_wv) < 1e-12


# ---------------------------------------------------------------- P6
def test_p6_relabelling():
    eo, ev, t1, t2, ovvv, ooov, ovov = random_symmetric_inputs(3, 5, 61)
    e = oracle.energy_literal(eo, ev, t1, t2, ovvv, ooov, ovov)
    po = np.array([2, 0, 1])
    pv = np.array([3, 1, 4, 0, 2])
    e_o = oracle.energy_literal(
        eo[po], ev, t1[po], t2[np.ix_(po, po, range(5), range(5))],
        ovvv[po], ooov[np.ix_(po, po, po, range(5))],
        ovov[np.ix_(po, range(5), po, range(5))])
    e_v = oracle.energy_literal(
        eo, ev[pv], t1[:, pv], t2[:, :, pv][:, :, :, pv],
        ovvv[:, pv][:, :, pv][:, :, :, pv], ooov[..., pv],
        ovov[:, pv][:, :, :, pv])
    assert rel(e_o, e) < 1e-13
    assert rel(e_v, e) < 1e-13


# ---------------------------------------------------------------- P7
def _twins(args):
    """The same inputs read through the other twin of every symmetric block."""
    eo, ev, t1, t2, ovvv, ooov, ovov = args
    return (eo, ev, t1, t2.transpose(1, 0, 3, 2), ovvv.transpose(0, 1, 3, 2),
            ooov.transpose(1, 0, 2, 3), ovov.transpose(2, 3, 0, 1))


def test_p7_twin_invariance():
    """Inputs with the twin symmetries give the same energy through either
    twin; inputs without them do not (the oracle reads one particular twin,
    so the invariance is a property of the symmetric inputs, not of the
    code)."""
    args = random_symmetric_inputs(3, 5, 71)
    e = oracle.energy_literal(*args)
    assert oracle.energy_literal(*_twins(args)) == e
    rng = np.random.default_rng(72)
    for pos in (3, 4, 5, 6):      # break one block's symmetry
        broken = list(args)
        broken[pos] = args[pos] + 0.3 * rng.normal(size=args[pos].shape)
        e1 = oracle.energy_literal(*broken)
        e2 = oracle.energy_literal(*_twins(broken))
        if pos == 6:
            assert rel(e1, e2) < 1e-13
        else:
            assert rel(e1, e2) > 1e-8, pos


# ---------------------------------------------------------------- P5 (power-of-two scale)
def test_p5_power_of_two_integral_scale_is_exact():
    """Integrals and t2 scaled by 2^-9 (a chemically scaled copy): Wt scales by
    2^-18 and Vt by 2^-9, so E = 2^-36 E_WW + 2^-27 E_WV, with every
    floating-point step scaled exactly; the parts reproduce bitwise."""
    args = list(random_symmetric_inputs(3, 5, 73))
    s = 2.0 ** -9
    sc = list(args)
    for pos in (3, 4, 5, 6):
        sc[pos] = args[pos] * s
    _, ww, wv = oracle.energy_literal(*args, return_parts=True)
    _, ww_s, wv_s = oracle.energy_literal(*sc, return_parts=True)
    assert ww_s == ww * s ** 4
    assert wv_s == wv * s ** 3


# ---------------------------------------------------------------- P8
def direct_sum(fa, fb):
    oa, va = fa[2].shape
    ob, vb = fb[2].shape
    o, v = oa + ob, va + vb
    so, sv = slice(0, oa), slice(0, va)
    to, tv = slice(oa, o), slice(va, v)
    eo = np.concatenate([fa[0], fb[0]])
    ev = np.concatenate([fa[1], fb[1]])
    t1 = np.zeros((o, v)); t1[so, sv] = fa[2]; t1[to, tv] = fb[2]
    t2 = np.zeros((o, o, v, v)); t2[so, so, sv, sv] = fa[3]; t2[to, to, tv, tv] = fb[3]
    ovvv = np.zeros((o, v, v, v)); ovvv[so, sv, sv, sv] = fa[4]; ovvv[to, tv, tv, tv] = fb[4]
    ooov = np.zeros((o, o, o, v)); ooov[so, so, so, sv] = fa[5]; ooov[to, to, to, tv] = fb[5]
    ovov = np.zeros((o, v, o, v)); ovov[so, sv, so, sv] = fa[6]; ovov[to, tv, to, tv] = fb[6]
    return eo, ev, t1, t2, ovvv, ooov, ovov


def test_p8_size_extensivity():
    fa = make_fragment(2, 4, 12, (81,)).arrays()
    fb = make_fragment(3, 3, 12, (82,)).arrays()
    ea, eb = oracle.energy_literal(*fa), oracle.energy_literal(*fb)
    eab = oracle.energy_literal(*direct_sum(fa, fb))
    assert rel(eab, ea + eb) < 1e-12


# ---------------------------------------------------------------- P9
def test_p9_projector():
    args = random_symmetric_inputs(3, 4, 91)
    o = 3
    e_i = oracle.energy_literal(*args)
    assert rel(oracle.energy_literal(*args, frag_proj=np.eye(o)), e_i) < 1e-14
    rng = np.random.default_rng(92)
    q, _ = np.linalg.qr(rng.normal(size=(o, o)))
    parts = [q[:, :1] @ q[:, :1].T, q[:, 1:] @ q[:, 1:].T]   # fragments {0}, {1, 2}
    for form in ("literal", "unrestricted"):
        ef = [oracle.energy_dense(*args, frag_proj=c, form=form) for c in parts]
        assert rel(sum(ef), e_i) < 1e-12
    lit = [oracle.energy_literal(*args, frag_proj=c) for c in parts]
    assert rel(sum(lit), e_i) < 1e-12
    for c in parts:
        assert rel(oracle.energy_literal(*args, frag_proj=c),
                   oracle.energy_dense(*args, frag_proj=c, form="literal")) < 1e-12
    # linear in C
    c2 = 2.5 * parts[0] - 0.5 * parts[1]
    assert rel(oracle.energy_literal(*args, frag_proj=c2),
               2.5 * lit[0] - 0.5 * lit[1]) < 1e-12


# ---------------------------------------------------------------- P10
@pytest.mark.parametrize("o,v,seed", [(3, 4, 101), (4, 6, 102)])
def test_p10_forms_agree(o, v, seed):
    args = random_symmetric_inputs(o, v, seed)
    e = oracle.energy_literal(*args)
    assert rel(T.energy_literal_vectorized(*args), e) < 1e-13
    assert rel(oracle.energy_dense(*args), e) < 1e-13
    assert rel(oracle.energy_dense(*args, form="unrestricted"), e) < 1e-13
    units = [oracle.occupied_triple_energy(i, j, k, *args)
             for (i, j, k) in oracle.occupied_triples(o)]
    assert rel(sum(units), e) < 1e-13
    _, ww, wv = oracle.energy_literal(*args, return_parts=True)
    e_o, ww_o, wv_o = oracle.energy_by_occupied_triples(*args, return_parts=True)
    assert rel(e_o, e) < 1e-13 and rel(ww_o, ww) < 1e-13 and rel(wv_o, wv) < 1e-13
    for u, (i, j, k) in enumerate(oracle.occupied_triples(o)):
        a, b = oracle.occupied_triple_parts(i, j, k, *args)
        assert abs(a + b - units[u]) <= 1e-13 * abs(e)


def test_p10_occupied_outer_fragment():
    """The occupied-outer form on a density-fitted fragment with ragged sizes,
    part by part against the literal loop."""
    f = make_fragment(5, 11, 24, (103,))
    e, ww, wv = T.energy_literal_vectorized(*f.arrays(), return_parts=True)
    e_o, ww_o, wv_o = oracle.energy_by_occupied_triples(*f.arrays(), return_parts=True)
    assert rel(e_o, e) < 1e-13 and rel(ww_o, ww) < 1e-13 and rel(wv_o, wv) < 1e-12


def test_golden_small_workload():
    """The stored value for the 8/40 workload is reproduced by the oracle."""
    with open(os.path.join(GOLDEN, "o8v40.json")) as fh:
        g = json.load(fh)
    f = workload_fragment("o8v40")
    e, ww, wv = T.energy_literal_vectorized(*f.arrays(), return_parts=True)
    assert rel(e, g["energy"]) < 1e-13
    assert rel(ww, g["e_ww"]) < 1e-13


def test_flop_count():
    assert oracle.flops_per_fragment(24, 200) == pytest.approx(4.953e13, rel=1e-3)
    assert len(oracle.occupied_triples(24)) == 2600


# ---------------------------------------------------------------- M
def _r_wrong_cyclic(y):     # the printed X_klj term read as a transposition
    return (4.0 * y + np.einsum("jki->ijk", y) + np.einsum("kji->ijk", y)
            - 2.0 * np.einsum("kji->ijk", y) - 2.0 * np.einsum("ikj->ijk", y)
            - 2.0 * np.einsum("jik->ijk", y))


def _r_wrong_sign(y):
    return (4.0 * y + np.einsum("jki->ijk", y) + np.einsum("kij->ijk", y)
            - 2.0 * np.einsum("kji->ijk", y) - 2.0 * np.einsum("ikj->ijk", y)
            + 2.0 * np.einsum("jik->ijk", y))


def _p_dropped_term(block, a, b, c):
    return (block(a, b, c)
            + np.einsum("jki->ijk", block(b, c, a))
            + np.einsum("kij->ijk", block(c, a, b))
            + np.einsum("ikj->ijk", block(a, c, b))
            + np.einsum("kji->ijk", block(c, b, a)))


def _p_wrong_index(block, a, b, c):
    return (block(a, b, c)
            + np.einsum("jki->ijk", block(b, c, a))
            + np.einsum("kij->ijk", block(c, a, b))
            + np.einsum("ikj->ijk", block(a, c, b))
            + np.einsum("kji->ijk", block(c, b, a))
            + np.einsum("jki->ijk", block(b, a, c)))


@pytest.mark.parametrize("name,patch", [
    ("_R_occ", _r_wrong_cyclic), ("_R_occ", _r_wrong_sign),
    ("_P_abc", _p_dropped_term), ("_P_abc", _p_wrong_index)])
def test_planted_mistakes_fail_p1(monkeypatch, name, patch):
    args = random_symmetric_inputs(3, 4, 111)
    e_so = spin_orbital_triples(*args)
    monkeypatch.setattr(T, name, patch)
    assert rel(T.energy_literal(*args), e_so) > 1e-6


def test_planted_layout_mistakes_fail_p1():
    eo, ev, t1, t2, ovvv, ooov, ovov = random_symmetric_inputs(3, 4, 112)
    e_so = spin_orbital_triples(eo, ev, t1, t2, ovvv, ooov, ovov)
    # (oo|ov) stored as [i, l, j, a] instead of [j, l, i, a]
    bad = oracle.energy_literal(eo, ev, t1, t2, ovvv, ooov.transpose(2, 1, 0, 3), ovov)
    assert rel(bad, e_so) > 1e-6
    # t2 with its virtual pair swapped (t_ij^ba for t_ij^ab)
    bad = oracle.energy_literal(eo, ev, t1, t2.transpose(0, 1, 3, 2), ovvv, ooov, ovov)
    assert rel(bad, e_so) > 1e-6
    # t1 term with the wrong sign
    bad = oracle.energy_literal(eo, ev, -t1, t2, ovvv, ooov, ovov)
    assert rel(bad, e_so) > 1e-6


# ---------------------------------------------------------------- P9b
def test_p9b_projector_matrix():
    """The projector matrix reproduces the projected energy of the
    unrestricted reading for arbitrary C (computed there with C applied to
    W-tilde first), its trace is the unprojected energy, and a complete
    orthogonal set of projectors sums to it."""
    args = random_symmetric_inputs(3, 4, 61)
    m = oracle.projector_matrix(*args)
    e = oracle.energy_literal(*args)
    assert abs(np.trace(m) - e) <= 1e-12 * abs(e)
    rng = np.random.default_rng(61)
    c = rng.normal(size=(3, 3))
    e_c = oracle.energy_dense(*args, frag_proj=c, form="unrestricted")
    assert abs(float(np.sum(c * m)) - e_c) <= 1e-12 * abs(e_c)
    u, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    parts = [u[:, :1] @ u[:, :1].T, u[:, 1:] @ u[:, 1:].T]
    assert abs(sum(float(np.sum(p * m)) for p in parts) - e) <= 1e-12 * abs(e)
