"""Gradient of the closed-shell in-situ (T) energy (C = I) in plain float64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper gives the energy (section "The In-situ Form of Perturbative (T) in
SIE", equation E_corr_CCSD_T with the definitions of W, V, Z, D, P, R) and
asks for nothing beyond it; the gradient here is the exact adjoint of that
energy, derived by hand and written out on whole six-index tensors (tiny
inputs only):

  E   = (1/3) sum_{ijk abc} Wt R[Wt + Vt] / D              (C = I)
      = B(Wt, Wt) + B(Wt, Vt),   B(X, Y) = (1/3) sum X R[Y] / D

R over occupied indices is symmetric as a linear map (its transpose maps each
cyclic permutation to the other and each transposition to itself) and D is
symmetric in ijk, so B is a symmetric bilinear form and

  dE  = sum Wh dWt + sum Vh dVt,
  Wh  = (1/3) R[2 Wt + Vt] / D,     Vh = (1/3) R[Wt] / D.

Wh and Vh inherit the pair symmetry of Wt (invariance under simultaneous
permutation of (i, a), (j, b), (k, c)).  Wt = P[X] is a sum of six such
permutations of X, so sum Wh dWt = 6 sum Wh dX; Vt = (1/2) P[U] with
U^{abc}_{ijk} = (ia|jb) t_k^c, so sum Vh dVt = 3 sum Vh dU.  X and U are
bilinear in the input arrays, which gives, for the arrays as stored
(t2[i,j,a,b] = t_ij^ab, ovvv[i,a,b,d] = (ia|bd), ooov[j,l,i,a] = (jl|ia) =
(ia|jl), ovov[i,a,j,b] = (ia|jb), t1[k,c] = t_k^c):

  dE/d ovvv[i,a,b,d] =  6 sum_{jkc} Wh^{abc}_{ijk} t2[k,j,c,d]
  dE/d t2[k,j,c,d]  +=  6 sum_{iab} Wh^{abc}_{ijk} ovvv[i,a,b,d]
  dE/d ooov[j,l,i,a] = -6 sum_{kbc} Wh^{abc}_{ijk} t2[l,k,b,c]
  dE/d t2[l,k,b,c]  += -6 sum_{ija} Wh^{abc}_{ijk} ooov[j,l,i,a]
  dE/d ovov[i,a,j,b] =  3 sum_{kc}  Vh^{abc}_{ijk} t1[k,c]
  dE/d t1[k,c]       =  3 sum_{ijab} Vh^{abc}_{ijk} ovov[i,a,j,b]

The inputs carry index symmetries (t_ij^ab = t_ji^ba, (ia|bd) = (ia|db),
(jl|ia) = (lj|ia), (ia|jb) = (jb|ia)), so the derivative with respect to one
stored entry depends on which twin an implementation happens to read.  The
gradients returned here are symmetrized: each entry is the mean over its
symmetry orbit of the array-entry derivatives above.  For a perturbation that
keeps the symmetry, sum(grad * dx) is the first-order change of E.
"""

from __future__ import annotations

import numpy as np

from .triples import _check, _P6, _R6


_TWIN_AXES = {"t2": (1, 0, 3, 2), "ovvv": (0, 1, 3, 2), "ooov": (1, 0, 2, 3),
              "ovov": (2, 3, 0, 1)}


def _orbit_mean(name, x):
    """Mean of x over the index-symmetry orbit of input `name` (t1 and the
    orbital energies have none)."""
    if name not in _TWIN_AXES:
        return x
    return 0.5 * (x + x.transpose(_TWIN_AXES[name]))


def _symmetrize(g):
    return {name: _orbit_mean(name, x) for name, x in g.items()}


def energy_gradient(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, symmetrize=True):
    """(E, E_WW, E_WV, grads) with grads = {"t1", "t2", "ovvv", "ooov", "ovov",
    "eps_occ", "eps_vir"} of dE/d(input) for C = I.  The orbital energies enter
    through the denominators only (the diagonal Fock elements of the canonical
    cluster orbitals), so dE/d(eps) is the contraction of dE/dD with the index
    counts of D.  Memory is O(n_o^3 n_v^3)."""
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    # forward quantities (same definitions as the energy)
    x6 = (np.einsum("iabd,kjcd->ijkabc", ovvv, t2, optimize=True)
          - np.einsum("jlia,lkbc->ijkabc", ooov, t2, optimize=True))
    wt = _P6(x6)
    del x6
    vt = 0.5 * _P6(np.einsum("iajb,kc->ijkabc", ovov, t1))
    eo, ev = eps_occ, eps_vir
    d = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    r_w = _R6(wt)
    r_v = _R6(vt)
    e_ww = float(np.sum(wt * r_w / d)) / 3.0
    e_wv = float(np.sum(wt * r_v / d)) / 3.0
    # orbital energies enter through D only: dE/dD = -(1/3) Wt R[Wt + Vt] / D^2
    # elementwise, and D = e_i + e_j + e_k - e_a - e_b - e_c
    e_d = -(wt * (r_w + r_v)) / (3.0 * d * d)
    g_eo = (np.einsum("ijkabc->i", e_d) + np.einsum("ijkabc->j", e_d)
            + np.einsum("ijkabc->k", e_d))
    g_ev = -(np.einsum("ijkabc->a", e_d) + np.einsum("ijkabc->b", e_d)
             + np.einsum("ijkabc->c", e_d))
    del e_d
    # adjoint cubes
    w_hat = (2.0 * r_w + r_v) / (3.0 * d)
    v_hat = r_w / (3.0 * d)
    del r_w, r_v, wt, vt, d
    g = {
        "ovvv": 6.0 * np.einsum("ijkabc,kjcd->iabd", w_hat, t2, optimize=True),
        "t2": (6.0 * np.einsum("ijkabc,iabd->kjcd", w_hat, ovvv, optimize=True)
               - 6.0 * np.einsum("ijkabc,jlia->lkbc", w_hat, ooov, optimize=True)),
        "ooov": -6.0 * np.einsum("ijkabc,lkbc->jlia", w_hat, t2, optimize=True),
        "ovov": 3.0 * np.einsum("ijkabc,kc->iajb", v_hat, t1, optimize=True),
        "t1": 3.0 * np.einsum("ijkabc,iajb->kc", v_hat, ovov, optimize=True),
        "eps_occ": g_eo,
        "eps_vir": g_ev,
    }
    if symmetrize:
        g = _symmetrize(g)
    return e_ww + e_wv, e_ww, e_wv, g


def symmetrize_direction(name, v):
    """Project a perturbation of input `name` onto arrays with that input's
    index symmetry (the mean over each symmetry orbit)."""
    return _orbit_mean(name, np.asarray(v, np.float64))
