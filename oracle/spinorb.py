"""Spin-orbital (T) energy by brute force: an independent pin for the
closed-shell formula of the paper's in-situ (T) section.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This is the standard spin-orbital form of the (T) correction of Raghavachari
et al. (1989, the (T) reference the paper cites), in the presentation of
Crawford and Schaefer (Rev. Comp. Chem. 14, 2000):

  D t_c = P(i/jk) P(a/bc) [ sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk> ]
  D t_d = P(i/jk) P(a/bc) t_i^a <jk||bc>
  E     = (1/36) sum_{ijkabc} t_c D (t_c + t_d)

with P(i/jk) f(ijk) = f(ijk) - f(jik) - f(kji) (same for a/bc),
D = e_i + e_j + e_k - e_a - e_b - e_c and <pq||rs> = <pq|rs> - <pq|sr>,
<pq|rs> = (pr|qs) delta(s_p, s_r) delta(s_q, s_s).

Closed-shell amplitudes map to spin orbitals as
  t_i^a   = t_I^A delta(s_i, s_a)
  t_ij^ab = t_IJ^AB delta(s_i,s_a) delta(s_j,s_b) - t_IJ^BA delta(s_i,s_b) delta(s_j,s_a).

Nothing here shares code with oracle/triples.py: different formula, different
index structure, explicit spin.  Tiny inputs only (arrays are (2n)^3 (2m)^3).
"""

from __future__ import annotations

import numpy as np


def _spin_maps(n):
    spatial = np.repeat(np.arange(n), 2)       # spin orbital p -> spatial P
    spin = np.tile(np.array([0, 1]), n)        # 0 = alpha, 1 = beta
    return spatial, spin


def _antisym_permute(x):
    """P(i/jk) P(a/bc) over x[i, j, k, a, b, c]."""
    y = x - x.transpose(1, 0, 2, 3, 4, 5) - x.transpose(2, 1, 0, 3, 4, 5)
    return y - y.transpose(0, 1, 2, 4, 3, 5) - y.transpose(0, 1, 2, 5, 4, 3)


def _spin_blocks(t1, t2, ovvv, ooov, ovov):
    o, v = t1.shape
    po, so = _spin_maps(o)
    pv, sv = _spin_maps(v)
    eq = lambda s, t: (s[:, None] == t[None, :]).astype(np.float64)  # noqa: E731
    d_ov = eq(so, sv)                       # [i, a]
    d_vv = eq(sv, sv)                       # [a, b]
    d_oo = eq(so, so)                       # [i, j]

    t1s = t1[po][:, pv] * d_ov
    t2_ab = t2[np.ix_(po, po, pv, pv)]      # t_IJ^AB at spin-orbital indices
    t2s = (t2_ab * d_ov[:, None, :, None] * d_ov[None, :, None, :]
           - t2_ab.transpose(0, 1, 3, 2) * d_ov[:, None, None, :] * d_ov[None, :, :, None])

    # <ei||bc>  (e, b, c virtual, i occupied): <ei|bc> = (eb|ic) = (ic|eb)
    g1 = ovvv[np.ix_(po, pv, pv, pv)]       # g1[i, c, e, b] = (ic|eb)
    ei_bc = np.einsum("iceb->eibc", g1) * d_vv[:, None, :, None] * d_ov[None, :, None, :]
    ei_cb = np.einsum("ibec->eibc", g1) * d_vv[:, None, None, :] * d_ov[None, :, :, None]
    g_vovv = ei_bc - ei_cb                   # [e, i, b, c]

    # <ma||jk>  (m, j, k occupied, a virtual): <ma|jk> = (mj|ak) = (mj|ka)
    g2 = ooov[np.ix_(po, po, po, pv)]       # g2[m, j, k, a] = (mj|ka)
    ma_jk = (np.einsum("mjka->majk", g2)
             * d_oo[:, None, :, None]                 # s_m == s_j
             * d_ov.T[None, :, None, :])              # s_a == s_k
    ma_kj = (np.einsum("mkja->majk", g2)
             * d_oo[:, None, None, :]                 # s_m == s_k
             * d_ov.T[None, :, :, None])              # s_a == s_j
    g_ovoo = ma_jk - ma_kj                   # [m, a, j, k]

    # <jk||bc>: <jk|bc> = (jb|kc)
    g3 = ovov[np.ix_(po, pv, po, pv)]       # g3[j, b, k, c] = (jb|kc)
    jk_bc = np.einsum("jbkc->jkbc", g3) * d_ov[:, None, :, None] * d_ov[None, :, None, :]
    jk_cb = np.einsum("jckb->jkbc", g3) * d_ov[:, None, None, :] * d_ov[None, :, :, None]
    g_oovv = jk_bc - jk_cb                   # [j, k, b, c]
    return po, pv, t1s, t2s, g_vovv, g_ovoo, g_oovv


def _numerators(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov = (
        np.asarray(x, np.float64) for x in (eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov))
    po, pv, t1s, t2s, g_vovv, g_ovoo, g_oovv = _spin_blocks(t1, t2, ovvv, ooov, ovov)
    eo, ev = eps_occ[po], eps_vir[pv]
    d = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    # sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk>, at [i, j, k, a, b, c]
    raw_c = (np.einsum("jkae,eibc->ijkabc", t2s, g_vovv, optimize=True)
             - np.einsum("imbc,majk->ijkabc", t2s, g_ovoo, optimize=True))
    raw_d = np.einsum("ia,jkbc->ijkabc", t1s, g_oovv)
    return _antisym_permute(raw_c), _antisym_permute(raw_d), d


def spin_orbital_triples(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov):
    """(T) energy from the spin-orbital formula (1/36) sum t_c D (t_c + t_d)."""
    nc, nd, d = _numerators(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    return float(np.sum(nc * (nc + nd) / d)) / 36.0


def mp4_triples_ordered(eps_occ, eps_vir, t2, ovvv, ooov):
    """Fourth-order triples energy sum_{i<j<k, a<b<c} (D t_c)^2 / D.

    With t2 = first-order (MP2) amplitudes this is the MP4 triples energy,
    which the (T) correction reproduces at t1 = 0.  The strictly ordered sum
    uses the antisymmetry of t_c instead of the 1/36 prefactor.
    """
    o, v = len(eps_occ), len(eps_vir)
    t1 = np.zeros((o, v))
    ovov = np.zeros((o, v, o, v))
    nc, _, d = _numerators(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)
    so, sv = 2 * o, 2 * v
    total = 0.0
    for i in range(so):
        for j in range(i + 1, so):
            for k in range(j + 1, so):
                for a in range(sv):
                    for b in range(a + 1, sv):
                        for c in range(b + 1, sv):
                            total += nc[i, j, k, a, b, c] ** 2 / d[i, j, k, a, b, c]
    return total
