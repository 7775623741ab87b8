"""MP2 energy, amplitudes and one-particle density matrix of a cluster (or of
a subspace), closed shell, in plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written from the paper's SI section "Systematically Improvable Quantum
Embedding Workflow" (the bath-natural-orbital construction), which gives

  t_ij^ab = -(ia|jb) / D_ij^ab,        D_ij^ab = e_a + e_b - e_i - e_j,
  gamma_ab = 2 sum_ij sum_c t_ij^ac (2 t_ij^bc - t_ij^cb),
  gamma_ij = 2 delta_ij - 2 sum_k sum_ab t_ik^ab (2 t_jk^ab - t_jk^ba),

with the occupied-virtual block of the MP2 1-RDM zero.  The correlation
energy of these amplitudes (the E_MP2 the paper's bath-truncation correction
uses) is the standard closed-shell expression

  E_MP2 = sum_ijab t_ij^ab [2 (ia|jb) - (ib|ja)].

The integrals come from density-fitting factors, (ia|jb) = sum_P L_ia^P
L_jb^P, as in the (T) workloads.  `spin_orbital_mp2` evaluates the textbook
spin-orbital formulas on explicit spin orbitals for tiny inputs, sharing no
code with the closed-shell functions (a pin).
"""

from __future__ import annotations

import numpy as np


def ovov_from_factors(l_ovp):
    """(ia|jb) [i, a, j, b] from factors L[i, a, P]."""
    l_ovp = np.asarray(l_ovp, np.float64)
    o, v, p = l_ovp.shape
    m = l_ovp.reshape(o * v, p)
    return (m @ m.T).reshape(o, v, o, v)


def amplitudes(eps_occ, eps_vir, ovov):
    """t[i, j, a, b] = t_ij^ab = -(ia|jb) / (e_a + e_b - e_i - e_j)."""
    eo = np.asarray(eps_occ, np.float64)
    ev = np.asarray(eps_vir, np.float64)
    d = (ev[None, None, :, None] + ev[None, None, None, :]
         - eo[:, None, None, None] - eo[None, :, None, None])
    return -np.asarray(ovov, np.float64).transpose(0, 2, 1, 3) / d


def mp2_energy(eps_occ, eps_vir, ovov):
    """E_MP2 = sum_ijab t_ij^ab [2 (ia|jb) - (ib|ja)] (float, compensated sum)."""
    t = amplitudes(eps_occ, eps_vir, ovov)
    k = np.asarray(ovov, np.float64).transpose(0, 2, 1, 3)     # k[i, j, a, b] = (ia|jb)
    terms = t * (2.0 * k - k.transpose(0, 1, 3, 2))            # (ib|ja) = k[i, j, b, a]
    return float(np.sum(np.sort(terms.ravel())))


def mp2_density(eps_occ, eps_vir, ovov):
    """(gamma_oo [o, o], gamma_vv [v, v]) of the MP2 amplitudes, as printed."""
    t = amplitudes(eps_occ, eps_vir, ovov)
    o = t.shape[0]
    gvv = 2.0 * np.einsum("ijac,ijbc->ab", t, 2.0 * t - t.transpose(0, 1, 3, 2))
    goo = 2.0 * np.eye(o) - 2.0 * np.einsum("ikab,jkab->ij", t, 2.0 * t - t.transpose(0, 1, 3, 2))
    return goo, gvv


def spin_orbital_mp2(eps_occ, eps_vir, ovov):
    """(E, gamma_oo, gamma_vv) from the spin-orbital formulas on explicit spin
    orbitals, the spin-orbital densities summed over the two spins of each
    spatial orbital:
      <ij||ab> = (ia|jb) d(s_i,s_a) d(s_j,s_b) - (ib|ja) d(s_i,s_b) d(s_j,s_a),
      T_ij^ab = <ij||ab> / (e_i + e_j - e_a - e_b),
      E = (1/4) sum |<ij||ab>|^2 / (e_i + e_j - e_a - e_b),
      gamma_ab = (1/2) sum_ijc T_ij^ac T_ij^bc,
      gamma_ij = delta_ij - (1/2) sum_kab T_ik^ab T_jk^ab.
    Tiny inputs only."""
    eo = np.asarray(eps_occ, np.float64)
    ev = np.asarray(eps_vir, np.float64)
    g = np.asarray(ovov, np.float64)
    o, v = eo.shape[0], ev.shape[0]
    po, so = np.repeat(np.arange(o), 2), np.tile([0, 1], o)
    pv, sv = np.repeat(np.arange(v), 2), np.tile([0, 1], v)
    no, nv = 2 * o, 2 * v
    anti = np.zeros((no, no, nv, nv))
    for i in range(no):
        for j in range(no):
            for a in range(nv):
                for b in range(nv):
                    x = 0.0
                    if so[i] == sv[a] and so[j] == sv[b]:
                        x += g[po[i], pv[a], po[j], pv[b]]
                    if so[i] == sv[b] and so[j] == sv[a]:
                        x -= g[po[i], pv[b], po[j], pv[a]]
                    anti[i, j, a, b] = x
    d = (eo[po][:, None, None, None] + eo[po][None, :, None, None]
         - ev[pv][None, None, :, None] - ev[pv][None, None, None, :])
    tt = anti / d
    e = 0.25 * float(np.sum(anti * anti / d))
    gv_so = 0.5 * np.einsum("ijac,ijbc->ab", tt, tt)
    go_so = np.eye(no) - 0.5 * np.einsum("ikab,jkab->ij", tt, tt)
    gvv = np.zeros((v, v))
    goo = np.zeros((o, o))
    for a in range(nv):
        for b in range(nv):
            if sv[a] == sv[b]:
                gvv[pv[a], pv[b]] += gv_so[a, b]
    for i in range(no):
        for j in range(no):
            if so[i] == so[j]:
                goo[po[i], po[j]] += go_so[i, j]
    return e, goo, gvv
