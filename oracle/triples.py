"""Closed-shell in-situ (T) energy of one SIE cluster in plain float64 (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Source: the paper's section "The In-situ Form of Perturbative (T) in SIE",
equation E_corr_CCSD_T and the definitions printed after it:

  E_x = 2 sum_{a>=b>=c} A_abc sum_{ijk} sum_{i'} R[Z^{abc}]_{ijk} Wt^{abc}_{i'jk} C^f_{ii'}

  A_abc = 1/6 if a = b = c, 1/2 if a = b or b = c, 1 otherwise
  Z     = W + V,        Wt = W D
  W     = P[X] / D,     X^{abc}_{ijk} = sum_d (ia|bd) t_kj^{cd} - sum_l (ia|jl) t_lk^{bc}
  V     = 1/2 P[U] / D, U^{abc}_{ijk} = (ia|jb) t_k^c
  D     = e_i + e_j + e_k - e_a - e_b - e_c
  P[X]  = X^{abc}_{ijk} + X^{bca}_{jki} + X^{cab}_{kij} + X^{acb}_{ikj} + X^{cba}_{kji} + X^{bac}_{jik}
  R[Y]_{ijk} = 4 Y_{ijk} + Y_{jki} + Y_{kij} - 2 Y_{kji} - 2 Y_{ikj} - 2 Y_{jik}   (abc fixed)
  C^f_{ii'} = sum_f C_if C_i'f   (identity when no projector is given)

Readings of the printed equations, each pinned by tests/test_oracle_pins.py:
  * W: the printed bracket has the two dummy indices swapped (an occupied l in
    a virtual slot, a virtual d in an occupied slot); the type-consistent
    reading is X = sum_d (ia|bd) t_kj^{cd} - sum_l (ia|jl) t_lk^{bc}.
  * R: the printed second term X_{klj} contains l, which is not one of i, j,
    k; it is read as the second cyclic permutation X_{kij}.
  * the summation domain printed as (ia >= jb >= kc) is read as a >= b >= c
    over virtual triples with i, j, k unrestricted (A depends on abc only).
  * V has no f_ov t2 term: the cluster orbitals are canonical.
  * with a projector, the literal form above applies C^f to the occupied
    index paired with the first virtual of each a >= b >= c triple
    (`energy_literal`); `energy_dense(form="unrestricted")` gives the
    virtual-order-independent variant (1/3) sum_all (C Wt) R[Z].  Both are
    linear in C and both reduce to the same value for C = I.

Array layouts: see synth/fragments.py (t2[i,j,a,b], ovvv[i,a,b,c],
ooov[j,l,i,a] = (jl|ia), ovov[i,a,j,b]).
"""

from __future__ import annotations

import math

import numpy as np


def _f64(*xs):
    return tuple(np.asarray(x, dtype=np.float64) for x in xs)


def _check(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _f64(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    o, v = eps_occ.shape[0], eps_vir.shape[0]
    want = {"t1": (o, v), "t2": (o, o, v, v), "ovvv": (o, v, v, v),
            "ooov": (o, o, o, v), "ovov": (o, v, o, v)}
    for name, arr in zip(want, (t1, t2, ovvv, ooov, ovov)):
        if arr.shape != want[name]:
            raise ValueError(f"{name}: shape {arr.shape}, expected {want[name]}")
    return eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov


def triple_weight(p: int, q: int, r: int) -> float:
    """A of eq. E_corr_CCSD_T for a sorted index triple p >= q >= r."""
    if p == q and q == r:
        return 1.0 / 6.0
    if p == q or q == r:
        return 0.5
    return 1.0


def occupied_triples(n_occ: int):
    """All (i, j, k) with i >= j >= k, in lexicographic order of (i, j, k)."""
    return [(i, j, k) for i in range(n_occ) for j in range(i + 1)
            for k in range(j + 1)]


def flops_per_fragment(n_occ: int, n_vir: int) -> float:
    """Algorithmic work of one fragment: the two dense contractions that build
    Wt (eq. W_in_CCSD_T), counted once per i >= j >= k triple and 6 terms each,
    2 flops per multiply-add: 2 n_o^3 n_v^4 + 2 n_o^4 n_v^3."""
    o, v = float(n_occ), float(n_vir)
    return 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3


# ---------------------------------------------------------------------------
# literal form: one virtual triple a >= b >= c at a time, all i, j, k
# ---------------------------------------------------------------------------

def _R_occ(y):
    """R[Y]_{ijk} over the three occupied axes of y[i, j, k] (abc fixed)."""
    return (4.0 * y
            + np.einsum("jki->ijk", y) + np.einsum("kij->ijk", y)
            - 2.0 * np.einsum("kji->ijk", y)
            - 2.0 * np.einsum("ikj->ijk", y)
            - 2.0 * np.einsum("jik->ijk", y))


def _P_abc(block, a, b, c):
    """P[X]^{abc}_{ijk} for all i, j, k, given block(a, b, c)[i, j, k] = X^{abc}_{ijk}."""
    return (block(a, b, c)
            + np.einsum("jki->ijk", block(b, c, a))    # X^{bca}_{jki}
            + np.einsum("kij->ijk", block(c, a, b))    # X^{cab}_{kij}
            + np.einsum("ikj->ijk", block(a, c, b))    # X^{acb}_{ikj}
            + np.einsum("kji->ijk", block(c, b, a))    # X^{cba}_{kji}
            + np.einsum("jik->ijk", block(b, a, c)))   # X^{bac}_{jik}


def energy_literal(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov,
                   frag_proj=None, return_parts=False):
    """E_x of eq. E_corr_CCSD_T, looping a >= b >= c exactly as printed.

    Returns the energy (float); with return_parts=True returns
    (E, E_WW, E_WV) where E_WW keeps only W in Z and E_WV only V.
    Per-triple partials are accumulated with math.fsum.
    Cost: O(n_o^3 n_v^4) with one small contraction per term: use for
    n_v up to a few tens.
    """
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    o, v = eps_occ.shape[0], eps_vir.shape[0]
    cf = np.eye(o) if frag_proj is None else np.asarray(frag_proj, np.float64)
    e3 = (eps_occ[:, None, None] + eps_occ[None, :, None]
          + eps_occ[None, None, :])

    def x_block(a, b, c):
        # sum_d (ia|bd) t_kj^{cd}
        vv = np.einsum("id,kjd->ijk", ovvv[:, a, b, :], t2[:, :, c, :],
                       optimize=True)
        # sum_l (ia|jl) t_lk^{bc}, with (ia|jl) = (jl|ia) = ooov[j, l, i, a]
        oo = np.einsum("jli,lk->ijk", ooov[:, :, :, a], t2[:, :, b, c],
                       optimize=True)
        return vv - oo

    def u_block(a, b, c):
        # (ia|jb) t_k^c
        return np.einsum("ij,k->ijk", ovov[:, a, :, b], t1[:, c])

    ww, wv = [], []
    for a in range(v):
        for b in range(a + 1):
            for c in range(b + 1):
                wt = _P_abc(x_block, a, b, c)            # Wt = W D
                vt = 0.5 * _P_abc(u_block, a, b, c)      # V D
                d = e3 - eps_vir[a] - eps_vir[b] - eps_vir[c]
                cw = np.einsum("ip,pjk->ijk", cf, wt)    # sum_i' C_ii' Wt_i'jk
                s = 2.0 * triple_weight(a, b, c)
                ww.append(s * float(np.sum(_R_occ(wt / d) * cw)))
                wv.append(s * float(np.sum(_R_occ(vt / d) * cw)))
    e_ww, e_wv = math.fsum(ww), math.fsum(wv)
    e = math.fsum(ww + wv)
    return (e, e_ww, e_wv) if return_parts else e


def energy_literal_vectorized(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov,
                              a_values=None, return_parts=False, x_terms=None):
    """Same sum as `energy_literal` (C = I), with the innermost c loop done as
    one batched contraction per (a, b) pair.

    a_values restricts the outer loop (for splitting the work over processes;
    the full energy is the fsum of the parts over a partition of range(n_v)).
    Returns the partial sum over the given a values.

    x_terms, if given, is a list of (ovvv', ooov', t2') triples: X is then the
    sum of the brackets of eq. W_in_CCSD_T evaluated with each triple (X is
    bilinear in the integrals and t2, so this expresses products of split
    operands).  t2, ovvv and ooov are then used only for their shapes.
    """
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    terms = [(ovvv, ooov, t2)] if x_terms is None else [
        tuple(np.asarray(x, np.float64) for x in tr) for tr in x_terms]
    o, v = eps_occ.shape[0], eps_vir.shape[0]
    e3 = (eps_occ[:, None, None] + eps_occ[None, :, None]
          + eps_occ[None, None, :])
    a_values = range(v) if a_values is None else a_values

    def x_gen(A, B, C):
        """X^{abc}_{ijk} for a in A, b in B, c in C (slices): array [a, b, c, i, j, k]."""
        out = 0.0
        for (vvvi, oooi, tt) in terms:
            vv = np.einsum("iabd,kjcd->abcijk", vvvi[:, A, B, :], tt[:, :, C, :],
                           optimize=True)
            oo = np.einsum("jlia,lkbc->abcijk", oooi[:, :, :, A], tt[:, :, B, C],
                           optimize=True)
            out = out + (vv - oo)
        return out

    def u_gen(A, B, C):
        """U^{abc}_{ijk} = (ia|jb) t_k^c for slices A, B, C: array [a, b, c, i, j, k]."""
        return np.einsum("iajb,kc->abcijk", ovov[:, A, :, B], t1[:, C])

    def p_over_c(gen, a, b, nc):
        """P[X]^{abc}_{ijk} for fixed a, b and c < nc: array [c, i, j, k]."""
        A, B, cs = slice(a, a + 1), slice(b, b + 1), slice(0, nc)
        return (gen(A, B, cs)[0, 0]
                + np.einsum("cjki->cijk", gen(B, cs, A)[0, :, 0])   # X^{bca}_{jki}
                + np.einsum("ckij->cijk", gen(cs, A, B)[:, 0, 0])   # X^{cab}_{kij}
                + np.einsum("cikj->cijk", gen(A, cs, B)[0, :, 0])   # X^{acb}_{ikj}
                + np.einsum("ckji->cijk", gen(cs, B, A)[:, 0, 0])   # X^{cba}_{kji}
                + np.einsum("cjik->cijk", gen(B, A, cs)[0, 0]))     # X^{bac}_{jik}

    def r_over_c(y):
        return (4.0 * y
                + np.einsum("cjki->cijk", y) + np.einsum("ckij->cijk", y)
                - 2.0 * np.einsum("ckji->cijk", y)
                - 2.0 * np.einsum("cikj->cijk", y)
                - 2.0 * np.einsum("cjik->cijk", y))

    ww, wv = [], []
    for a in a_values:
        for b in range(a + 1):
            cs = np.arange(b + 1)
            wt = p_over_c(x_gen, a, b, b + 1)
            vt = 0.5 * p_over_c(u_gen, a, b, b + 1)
            d = (e3[None] - eps_vir[a] - eps_vir[b]
                 - eps_vir[cs][:, None, None, None])
            wgt = np.array([2.0 * triple_weight(a, b, c) for c in cs])
            ww.extend((wgt * np.sum(r_over_c(wt / d) * wt, axis=(1, 2, 3))).tolist())
            wv.extend((wgt * np.sum(r_over_c(vt / d) * wt, axis=(1, 2, 3))).tolist())
    e_ww, e_wv = math.fsum(ww), math.fsum(wv)
    e = math.fsum(ww + wv)
    return (e, e_ww, e_wv) if return_parts else e


# ---------------------------------------------------------------------------
# dense form: whole six-index tensors (tiny inputs only)
# ---------------------------------------------------------------------------

def _P6(x):
    """P over six-index arrays x[i, j, k, a, b, c]."""
    return (x
            + np.einsum("jkibca->ijkabc", x)
            + np.einsum("kijcab->ijkabc", x)
            + np.einsum("ikjacb->ijkabc", x)
            + np.einsum("kjicba->ijkabc", x)
            + np.einsum("jikbac->ijkabc", x))


def _R6(y):
    """R over the occupied axes of y[i, j, k, a, b, c]."""
    return (4.0 * y
            + np.einsum("jkiabc->ijkabc", y) + np.einsum("kijabc->ijkabc", y)
            - 2.0 * np.einsum("kjiabc->ijkabc", y)
            - 2.0 * np.einsum("ikjabc->ijkabc", y)
            - 2.0 * np.einsum("jikabc->ijkabc", y))


def energy_dense(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov,
                 frag_proj=None, form="literal"):
    """The same definitions with every six-index tensor formed explicitly.

    form="literal":      2 sum_{a>=b>=c} A_abc sum_{ijk} R[Z]_{ijk} (C Wt)_{ijk}
    form="unrestricted": (1/3) sum_{all ijk abc} R[Z]_{ijk} (C Wt)_{ijk}
    For C = I the two coincide (the summand summed over ijk is symmetric
    under permutations of abc).  Memory is O(n_o^3 n_v^3).
    """
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    o, v = eps_occ.shape[0], eps_vir.shape[0]
    cf = np.eye(o) if frag_proj is None else np.asarray(frag_proj, np.float64)
    x6 = (np.einsum("iabd,kjcd->ijkabc", ovvv, t2, optimize=True)
          - np.einsum("jlia,lkbc->ijkabc", ooov, t2, optimize=True))
    wt = _P6(x6)
    vt = 0.5 * _P6(np.einsum("iajb,kc->ijkabc", ovov, t1))
    eo = eps_occ
    ev = eps_vir
    d = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    cw = np.einsum("ip,pjkabc->ijkabc", cf, wt)
    summand = _R6((wt + vt) / d) * cw
    if form == "unrestricted":
        return float(np.sum(summand)) / 3.0
    if form != "literal":
        raise ValueError(form)
    a_idx = np.arange(v)
    weight = np.zeros((v, v, v))
    for a in a_idx:
        for b in range(a + 1):
            for c in range(b + 1):
                weight[a, b, c] = 2.0 * triple_weight(a, b, c)
    return float(np.einsum("ijkabc,abc->", summand, weight))


# ---------------------------------------------------------------------------
# contribution of one unordered occupied triple (sampled checks at full size)
# ---------------------------------------------------------------------------

def occupied_triple_energy(i, j, k, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    """Contribution of the occupied triple {i, j, k} (i >= j >= k) to E_x, C = I.

    With g(ijk) = sum_{all abc} R[Z^{abc}]_{ijk} Wt^{abc}_{ijk}, the energy of
    eq. E_corr_CCSD_T equals (1/3) sum_{all ordered ijk} g(ijk); g takes the
    same value on every ordering of {i, j, k} (a simultaneous relabelling of
    occupied and virtual indices leaves Wt, Z and R unchanged), so the
    contribution of the unordered triple is 2 A_ijk g(ijk), with A_ijk the
    equal-index weight of the same equation applied to occupied indices.
    Summing this over all i >= j >= k gives E_x.  Here g is evaluated from
    the definitions at all six orderings of (i, j, k), over all abc.
    Cost: six contractions of 2 n_v^4 flops.
    """
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    if not (i >= j >= k):
        raise ValueError("need i >= j >= k")
    v = eps_vir.shape[0]

    x_cache = {}

    def xo(p, q, r):
        """X^{abc}_{pqr} over all a, b, c: array [a, b, c]."""
        key = (p, q, r)
        if key not in x_cache:
            # sum_d (pa|bd) t_rq^{cd}
            vv = (ovvv[p].reshape(v * v, v) @ t2[r, q].T).reshape(v, v, v)
            # sum_l (pa|ql) t_lr^{bc}, with (pa|ql) = ooov[q, l, p, a]
            oo = np.einsum("la,lbc->abc", ooov[q, :, p, :], t2[:, r],
                           optimize=True)
            x_cache[key] = vv - oo
        return x_cache[key]

    def uo(p, q, r):
        """U^{abc}_{pqr} = (pa|qb) t_r^c: array [a, b, c]."""
        return np.einsum("ab,c->abc", ovov[p, :, q, :], t1[r])

    def p_occ(block, p, q, r):
        """P[X]^{abc}_{pqr} over all a, b, c."""
        return (block(p, q, r)
                + np.einsum("bca->abc", block(q, r, p))   # X^{bca}_{qrp}
                + np.einsum("cab->abc", block(r, p, q))   # X^{cab}_{rpq}
                + np.einsum("acb->abc", block(p, r, q))   # X^{acb}_{prq}
                + np.einsum("cba->abc", block(r, q, p))   # X^{cba}_{rqp}
                + np.einsum("bac->abc", block(q, p, r)))  # X^{bac}_{qpr}

    d = (eps_occ[i] + eps_occ[j] + eps_occ[k] - eps_vir[:, None, None]
         - eps_vir[None, :, None] - eps_vir[None, None, :])

    def z(p, q, r):
        return (p_occ(xo, p, q, r) + 0.5 * p_occ(uo, p, q, r)) / d

    r_z = (4.0 * z(i, j, k) + z(j, k, i) + z(k, i, j)
           - 2.0 * z(k, j, i) - 2.0 * z(i, k, j) - 2.0 * z(j, i, k))
    g = float(np.sum(r_z * p_occ(xo, i, j, k)))
    return 2.0 * triple_weight(i, j, k) * g


# ---------------------------------------------------------------------------
# occupied-outer form: one unordered occupied triple at a time, R moved onto
# the virtual indices (full-size reference values)
# ---------------------------------------------------------------------------

def _r_vir(y):
    """R moved from the occupied to the virtual indices of one occupied
    triple's cube y[a, b, c]:
        R'[Y]^{abc} = 4 Y^{abc} + Y^{cab} + Y^{bca} - 2 Y^{cba} - 2 Y^{acb} - 2 Y^{bac}.
    With Y = Wt or Vt (both unchanged by a simultaneous permutation of the
    occupied and the virtual indices), Y_{jki}^{abc} = Y_{ijk}^{cab},
    Y_{kij}^{abc} = Y_{ijk}^{bca}, Y_{kji}^{abc} = Y_{ijk}^{cba},
    Y_{ikj}^{abc} = Y_{ijk}^{acb} and Y_{jik}^{abc} = Y_{ijk}^{bac}, so
    R'[Y_{ijk}] equals R[Y]_{ijk} of eq. E_corr_CCSD_T."""
    return (4.0 * y
            + np.einsum("cab->abc", y) + np.einsum("bca->abc", y)
            - 2.0 * np.einsum("cba->abc", y)
            - 2.0 * np.einsum("acb->abc", y)
            - 2.0 * np.einsum("bac->abc", y))


def occupied_triple_parts(i, j, k, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    """(E_WW, E_WV) contributions of the occupied triple {i, j, k} (i >= j >= k)
    to E_x, C = I, in the occupied-outer form:

        E_unit = 2 A_ijk sum_{abc} Wt^{abc}_{ijk} R'[Wt + Vt]^{abc}_{ijk} / D^{abc}_{ijk},

    with Wt = P[X] and Vt = (1/2) P[U] at the fixed occupied triple (each of
    the six P-images is the X (or U) of a reordered occupied triple with its
    virtual axes reordered the same way) and R' the virtual-index form of R
    (see `_r_vir`).  E_WW keeps Wt in the bracket, E_WV keeps Vt; their sum is
    what `occupied_triple_energy` gives, which evaluates R over six occupied
    orderings instead.  Cost: six contractions of 2 n_v^4 flops and a few
    dozen passes over n_v^3 cubes.
    """
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    if not (i >= j >= k):
        raise ValueError("need i >= j >= k")
    v = eps_vir.shape[0]

    def x(p, q, r):
        """X^{abc}_{pqr} over all a, b, c: array [a, b, c]."""
        # sum_d (pa|bd) t_rq^{cd}
        vv = (ovvv[p].reshape(v * v, v) @ t2[r, q].T).reshape(v, v, v)
        # sum_l (pa|ql) t_lr^{bc}, with (pa|ql) = ooov[q, l, p, a]
        vv -= np.einsum("la,lbc->abc", ooov[q, :, p, :], t2[:, r], optimize=True)
        return vv

    # Wt^{abc}_{ijk} = X^{abc}_{ijk} + X^{bca}_{jki} + X^{cab}_{kij}
    #                + X^{acb}_{ikj} + X^{cba}_{kji} + X^{bac}_{jik}
    wt = x(i, j, k)
    wt += np.einsum("bca->abc", x(j, k, i))
    wt += np.einsum("cab->abc", x(k, i, j))
    wt += np.einsum("acb->abc", x(i, k, j))
    wt += np.einsum("cba->abc", x(k, j, i))
    wt += np.einsum("bac->abc", x(j, i, k))
    # Vt = (1/2) P[U], U^{abc}_{pqr} = (pa|qb) t_r^c: the six images pair up
    # into (ia|jb) t_k^c + (ia|kc) t_j^b + (jb|kc) t_i^a
    vt = (np.einsum("ab,c->abc", ovov[i, :, j, :], t1[k])
          + np.einsum("ac,b->abc", ovov[i, :, k, :], t1[j])
          + np.einsum("bc,a->abc", ovov[j, :, k, :], t1[i]))
    d = (eps_occ[i] + eps_occ[j] + eps_occ[k] - eps_vir[:, None, None]
         - eps_vir[None, :, None] - eps_vir[None, None, :])
    w = 2.0 * triple_weight(i, j, k)
    wd = wt / d
    e_ww = w * float(np.sum(_r_vir(wt) * wd))
    e_wv = w * float(np.sum(_r_vir(vt) * wd))
    return e_ww, e_wv


def projector_matrix(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    """M[i, i'] = (1/3) sum_{jk abc} Wt^{abc}_{i'jk} (R[Wt + Vt] / D)^{abc}_{ijk}
    (plain six-index tensors, tiny inputs), so that the projected energy of
    the unrestricted reading, (1/3) sum (C Wt) R[Wt + Vt] / D, equals
    sum_{i i'} C[i, i'] M[i, i'] for every C, and tr M is E_x."""
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = _check(
        eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    x6 = (np.einsum("iabd,kjcd->ijkabc", ovvv, t2, optimize=True)
          - np.einsum("jlia,lkbc->ijkabc", ooov, t2, optimize=True))
    wt = _P6(x6)
    vt = 0.5 * _P6(np.einsum("iajb,kc->ijkabc", ovov, t1))
    eo, ev = eps_occ, eps_vir
    d = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    q = _R6((wt + vt) / d)
    return np.einsum("pjkabc,ijkabc->ip", wt, q, optimize=True) / 3.0


def energy_by_occupied_triples(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov,
                               return_parts=False):
    """E_x (C = I) as the compensated sum of `occupied_triple_parts` over all
    i >= j >= k; with return_parts=True returns (E, E_WW, E_WV)."""
    o = np.asarray(eps_occ).shape[0]
    ww, wv = [], []
    for (i, j, k) in occupied_triples(o):
        a, b = occupied_triple_parts(i, j, k, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
        ww.append(a)
        wv.append(b)
    e_ww, e_wv = math.fsum(ww), math.fsum(wv)
    e = math.fsum(ww + wv)
    return (e, e_ww, e_wv) if return_parts else e
