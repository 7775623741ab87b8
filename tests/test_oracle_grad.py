"""Pins of the oracle gradient (oracle/grad.py) against facts that do not come
from the gradient code itself.

G1  directional central differences of the textbook spin-orbital energy
    (oracle/spinorb.py) along random symmetric directions, per input block.
    E is at most quadratic in each block separately, so a central difference
    is exact up to rounding at any step size.
G2  the same with the literal a >= b >= c energy on synthetic fragments
    spanning the sizes the GPU tests use
G3  Euler identities of the polynomial structure: sum t1 dE/dt1 = E_WV =
    sum ovov dE/dovov; sum t2 dE/dt2 = 2 E_WW + E_WV = sum ovvv dE/dovvv +
    sum ooov dE/dooov (E_WW, E_WV from the literal energy)
G4  torch float64 automatic differentiation of the plain definition
G5  single-orbit differences: perturbing one symmetry orbit of an entry moves
    E by |orbit| * (symmetrized gradient entry)
G6  the orbital-energy gradient: Richardson-extrapolated central differences
    of the spin-orbital energy along random directions of eps_occ and eps_vir;
    homogeneity (E is of degree -1 in the orbital energies, so
    sum_p eps_p dE/deps_p = -E); invariance under a common shift of all
    orbital energies (sum_p dE/deps_p = 0); torch autograd (G4)
M   planted mistakes (a flipped sign, a wrong factor) fail G1 or G6
"""

import numpy as np
import pytest

import oracle
from oracle.grad import energy_gradient, symmetrize_direction
from oracle.spinorb import spin_orbital_triples
from synth import make_fragment

from test_oracle_pins import random_symmetric_inputs

NAMES = ("t1", "t2", "ovvv", "ooov", "ovov")
IDX = {n: 2 + i for i, n in enumerate(NAMES)}    # position in the argument tuple


def directional_fd(energy, args, name, v, h):
    """(E(x + h v) - E(x - h v)) / 2h for input `name`."""
    plus, minus = list(args), list(args)
    plus[IDX[name]] = args[IDX[name]] + h * v
    minus[IDX[name]] = args[IDX[name]] - h * v
    return (energy(*plus) - energy(*minus)) / (2.0 * h)


def random_direction(args, name, rng):
    x = args[IDX[name]]
    v = rng.normal(size=x.shape) * (np.abs(x).mean() + 1e-300)
    return symmetrize_direction(name, v)


def check_fd(energy, args, grads, seed, tol, h=1e-2):
    rng = np.random.default_rng(seed)
    worst = {}
    for name in NAMES:
        v = random_direction(args, name, rng)
        fd = directional_fd(energy, args, name, v, h)
        an = float(np.sum(grads[name] * v))
        worst[name] = abs(an - fd) / max(abs(fd), 1e-300)
    return all(w < tol for w in worst.values()), worst


# ---------------------------------------------------------------- G1
@pytest.mark.parametrize("o,v,seed", [(2, 3, 11), (3, 3, 12), (3, 4, 13), (2, 5, 14)])
def test_g1_fd_of_spin_orbital_energy(o, v, seed):
    args = random_symmetric_inputs(o, v, seed)
    e, _, _, g = energy_gradient(*args)
    assert abs(e - spin_orbital_triples(*args)) < 1e-12 * abs(e)
    ok, worst = check_fd(spin_orbital_triples, args, g, seed, 1e-9)
    assert ok, worst


# ---------------------------------------------------------------- G2
@pytest.mark.parametrize("o,v,naux,seed", [(3, 9, 24, (9, 1)), (4, 12, 30, (9, 2)),
                                           (5, 20, 60, (9, 3))])
def test_g2_fd_of_literal_energy(o, v, naux, seed):
    f = make_fragment(o, v, naux, seed)
    args = f.arrays()
    e, _, _, g = energy_gradient(*args)
    ok, worst = check_fd(oracle.energy_literal_vectorized, args, g, 5, 1e-9)
    assert ok, worst


# ---------------------------------------------------------------- G3
@pytest.mark.parametrize("o,v,naux,seed", [(4, 12, 30, (9, 4)), (6, 17, 40, (9, 5))])
def test_g3_euler_identities(o, v, naux, seed):
    f = make_fragment(o, v, naux, seed)
    args = f.arrays()
    _, ww, wv, g = energy_gradient(*args)
    e, e_ww, e_wv = oracle.energy_literal_vectorized(*args, return_parts=True)
    dot = {n: float(np.sum(args[IDX[n]] * g[n])) for n in NAMES}
    assert abs(dot["t1"] - e_wv) < 1e-11 * abs(e)
    assert abs(dot["ovov"] - e_wv) < 1e-11 * abs(e)
    assert abs(dot["t2"] - (2 * e_ww + e_wv)) < 1e-11 * abs(e)
    assert abs(dot["ovvv"] + dot["ooov"] - (2 * e_ww + e_wv)) < 1e-11 * abs(e)
    assert abs(ww - e_ww) < 1e-12 * abs(e) and abs(wv - e_wv) < 1e-12 * abs(e)


# ---------------------------------------------------------------- G4
def test_g4_torch_autograd():
    torch = pytest.importorskip("torch")
    args = random_symmetric_inputs(3, 5, 21)
    _, _, _, g = energy_gradient(*args)
    eo, ev = (torch.tensor(a) for a in args[:2])
    leaves = [torch.tensor(a, requires_grad=True) for a in args[2:]]
    t1, t2, ovvv, ooov, ovov = leaves
    x = (torch.einsum("iabd,kjcd->ijkabc", ovvv, t2)
         - torch.einsum("jlia,lkbc->ijkabc", ooov, t2))
    u = torch.einsum("iajb,kc->ijkabc", ovov, t1)

    def perm_sum(y):   # the six simultaneous (occupied, virtual) permutations
        return (y + y.permute(2, 0, 1, 5, 3, 4) + y.permute(1, 2, 0, 4, 5, 3)
                + y.permute(0, 2, 1, 3, 5, 4) + y.permute(2, 1, 0, 5, 4, 3)
                + y.permute(1, 0, 2, 4, 3, 5))

    eo.requires_grad_(True)
    ev.requires_grad_(True)
    wt, vt = perm_sum(x), 0.5 * perm_sum(u)
    d = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    z = (wt + vt) / d
    # R on the occupied axes: 4 z_ijk + z_jki + z_kij - 2 (z_kji + z_ikj + z_jik)
    rz = (4 * z + z.permute(1, 2, 0, 3, 4, 5) + z.permute(2, 0, 1, 3, 4, 5)
          - 2 * (z.permute(2, 1, 0, 3, 4, 5) + z.permute(0, 2, 1, 3, 4, 5)
                 + z.permute(1, 0, 2, 3, 4, 5)))
    e = (rz * wt).sum() / 3.0
    e.backward()
    for name, leaf in zip(NAMES, leaves):
        ref = symmetrize_direction(name, leaf.grad.numpy())
        err = np.abs(ref - g[name]).max() / np.abs(ref).max()
        assert err < 1e-12, (name, err)
    for name, leaf in (("eps_occ", eo), ("eps_vir", ev)):
        ref = leaf.grad.numpy()
        err = np.abs(ref - g[name]).max() / np.abs(ref).max()
        assert err < 1e-12, (name, err)


# ---------------------------------------------------------------- G5
def test_g5_single_orbit_differences():
    f = make_fragment(4, 10, 30, (9, 6))
    args = f.arrays()
    _, _, _, g = energy_gradient(*args)
    for name in NAMES:
        gn = g[name]
        for flat in np.argsort(np.abs(gn).ravel())[-3:]:
            idx = np.unravel_index(flat, gn.shape)
            e = np.zeros_like(gn)
            e[idx] = 1.0
            orbit = symmetrize_direction(name, e)
            orbit = (orbit > 0).astype(np.float64)        # indicator of the orbit
            h = 1e-3 * (np.abs(args[IDX[name]]).mean())
            fd = directional_fd(oracle.energy_literal_vectorized, args, name, orbit, h)
            want = orbit.sum() * gn[idx]
            assert abs(fd - want) < 1e-7 * abs(want), (name, idx, fd, want)


# ---------------------------------------------------------------- M
@pytest.mark.parametrize("mistake", ["ooov_sign", "t1_factor", "t2_oo_dropped"])
def test_planted_mistakes_fail_g1(mistake):
    args = random_symmetric_inputs(3, 4, 31)
    _, _, _, g = energy_gradient(*args)
    bad = dict(g)
    if mistake == "ooov_sign":
        bad["ooov"] = -g["ooov"]
    elif mistake == "t1_factor":
        bad["t1"] = 2.0 * g["t1"]
    else:
        # the t2 gradient without the contribution of the (oo|ov) sum: zero
        # ooov and recompute, which keeps only the (ov|vv) product's part
        args0 = list(args)
        args0[IDX["ooov"]] = np.zeros_like(args[IDX["ooov"]])
        _, _, _, g0 = energy_gradient(*args0)
        bad["t2"] = g0["t2"]
    ok, worst = check_fd(spin_orbital_triples, args, bad, 31, 1e-9)
    assert not ok, worst


# ---------------------------------------------------------------- G6
def eps_fd(energy, args, which, v, h):
    """Richardson-extrapolated central difference of E along v in eps_occ
    (which = 0) or eps_vir (which = 1): (4 C(h/2) - C(h)) / 3, error O(h^4)."""
    def central(step):
        plus, minus = list(args), list(args)
        plus[which] = args[which] + step * v
        minus[which] = args[which] - step * v
        return (energy(*plus) - energy(*minus)) / (2.0 * step)
    return (4.0 * central(h / 2) - central(h)) / 3.0


@pytest.mark.parametrize("o,v,seed", [(2, 3, 41), (3, 4, 42), (2, 5, 43)])
def test_g6_eps_fd_of_spin_orbital_energy(o, v, seed):
    args = random_symmetric_inputs(o, v, seed)
    _, _, _, g = energy_gradient(*args)
    rng = np.random.default_rng(seed)
    for which, name in ((0, "eps_occ"), (1, "eps_vir")):
        d = rng.normal(size=args[which].shape)
        fd = eps_fd(spin_orbital_triples, args, which, d, 1e-3)
        an = float(np.sum(g[name] * d))
        assert abs(an - fd) < 1e-9 * abs(fd), (name, an, fd)


@pytest.mark.parametrize("o,v,naux,seed", [(4, 12, 30, (9, 7)), (5, 20, 60, (9, 8))])
def test_g6_eps_homogeneity_and_shift(o, v, naux, seed):
    f = make_fragment(o, v, naux, seed)
    args = f.arrays()
    e, _, _, g = energy_gradient(*args)
    euler = float(np.dot(args[0], g["eps_occ"]) + np.dot(args[1], g["eps_vir"]))
    assert abs(euler + e) < 1e-12 * abs(e), (euler, e)
    total = float(g["eps_occ"].sum() + g["eps_vir"].sum())
    scale = float(np.abs(g["eps_occ"]).sum() + np.abs(g["eps_vir"]).sum())
    assert abs(total) < 1e-13 * scale, (total, scale)
    # and against central differences of the literal energy
    rng = np.random.default_rng(3)
    d = rng.normal(size=args[1].shape)
    fd = eps_fd(oracle.energy_literal_vectorized, args, 1, d, 1e-3)
    assert abs(float(np.sum(g["eps_vir"] * d)) - fd) < 1e-9 * abs(fd)


@pytest.mark.parametrize("mistake", ["vir_sign", "occ_count"])
def test_planted_eps_mistakes_fail_g6(mistake):
    args = random_symmetric_inputs(3, 4, 44)
    _, _, _, g = energy_gradient(*args)
    rng = np.random.default_rng(44)
    which = 1 if mistake == "vir_sign" else 0
    name = ("eps_occ", "eps_vir")[which]
    bad = -g[name] if mistake == "vir_sign" else g[name] / 3.0   # one index of three
    d = rng.normal(size=args[which].shape)
    fd = eps_fd(spin_orbital_triples, args, which, d, 1e-3)
    assert abs(float(np.sum(bad * d)) - fd) > 1e-6 * abs(fd)
