"""Seeded synthetic embedded-cluster inputs for the (T) energy.

The paper's clusters (hundreds of orbitals, dense canonical integrals, see its
sections on the SIE workflow and on the choice of BNO threshold) are not
available here, so dense synthetic stand-ins of the same shapes are generated:

* orbital energies  eps_occ ~ U[-1.5, -0.3] Eh (sorted), eps_vir ~ U[0.1, 3.0] Eh
  (sorted), so every triples denominator is <= -1.2 Eh;
* density-fitting factors B^P_pq with i.i.d. N(0, b_std^2) entries on p <= q,
  mirrored to make each B^P symmetric; orbital order is occupied then virtual;
* integrals (pq|rs) = sum_P B^P_pq B^P_rs in float64, sliced into the three
  blocks the (T) energy reads;
* t2 = MP2 amplitudes t_ij^ab = (ia|jb) / (e_i + e_j - e_a - e_b), the
  subspace-MP2 amplitude formula of the paper's embedding workflow section;
* t1 ~ N(0, t1_std^2).

Array layouts (row-major, float64):
    eps_occ[i], eps_vir[a]
    t1[i, a]          = t_i^a
    t2[i, j, a, b]    = t_ij^ab,  exactly equal to t2[j, i, b, a]
    ovvv[i, a, b, c]  = (ia|bc),  exactly symmetric in b <-> c
    ooov[j, l, i, a]  = (jl|ia),  exactly symmetric in j <-> l
    ovov[i, a, j, b]  = (ia|jb),  exactly symmetric in (ia) <-> (jb)

The twin symmetries are made exact (bitwise) by averaging each block with its
twin, so that any implementation may read either twin.

Seeds: numpy default_rng(SeedSequence(seed)) with draw order eps_occ, eps_vir,
B, t1.  No (T) arithmetic is done here.
"""

from __future__ import annotations

import dataclasses

import numpy as np

SEED_ROOT = 241218553


@dataclasses.dataclass
class Fragment:
    eps_occ: np.ndarray
    eps_vir: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    ovvv: np.ndarray
    ooov: np.ndarray
    ovov: np.ndarray

    @property
    def n_occ(self) -> int:
        return int(self.eps_occ.shape[0])

    @property
    def n_vir(self) -> int:
        return int(self.eps_vir.shape[0])

    def arrays(self):
        """The seven inputs in the order (eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov)."""
        return (self.eps_occ, self.eps_vir, self.t1, self.t2,
                self.ovvv, self.ooov, self.ovov)

    def astype(self, dtype) -> "Fragment":
        """Amplitudes and integrals cast to `dtype`; orbital energies stay float64."""
        c = lambda x: np.ascontiguousarray(x.astype(dtype))  # noqa: E731
        return Fragment(self.eps_occ, self.eps_vir, c(self.t1), c(self.t2),
                        c(self.ovvv), c(self.ooov), c(self.ovov))

    def replace(self, **kw) -> "Fragment":
        return dataclasses.replace(self, **kw)


def make_fragment(n_occ: int, n_vir: int, n_aux: int, seed, *,
                  b_std: float = 0.05, t1_std: float = 1e-2,
                  b_scale: float = 1.0, zero_t1: bool = False) -> Fragment:
    """Build one seeded synthetic fragment.

    `seed` is a sequence of non-negative ints fed to numpy's SeedSequence.
    `b_scale` multiplies the DF factors after drawing them (same random
    stream), which gives a chemically scaled copy of the same fragment.
    """
    if n_occ < 1 or n_vir < 1 or n_aux < 1:
        raise ValueError("n_occ, n_vir and n_aux must be >= 1")
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    eps_vir = np.sort(rng.uniform(0.1, 3.0, n_vir))
    n = n_occ + n_vir
    g = rng.normal(0.0, b_std, size=(n_aux, n, n))
    bfac = np.triu(g) + np.triu(g, 1).transpose(0, 2, 1)
    del g
    if b_scale != 1.0:
        bfac *= b_scale
    t1 = rng.normal(0.0, t1_std, size=(n_occ, n_vir))
    if zero_t1:
        t1[...] = 0.0
    o, v = n_occ, n_vir
    b_oo = np.ascontiguousarray(bfac[:, :o, :o]).reshape(n_aux, o * o)
    b_ov = np.ascontiguousarray(bfac[:, :o, o:]).reshape(n_aux, o * v)
    b_vv = np.ascontiguousarray(bfac[:, o:, o:]).reshape(n_aux, v * v)
    del bfac

    ovvv = (b_ov.T @ b_vv).reshape(o, v, v, v)
    for i in range(o):  # exact b <-> c symmetry, one occupied slice at a time
        s = ovvv[i]
        s += s.transpose(0, 2, 1).copy()
        s *= 0.5
    ooov = (b_oo.T @ b_ov).reshape(o, o, o, v)
    ooov = 0.5 * (ooov + ooov.transpose(1, 0, 2, 3))
    ovov = (b_ov.T @ b_ov).reshape(o, v, o, v)
    ovov = 0.5 * (ovov + ovov.transpose(2, 3, 0, 1))

    e_oo = eps_occ[:, None] + eps_occ[None, :]
    e_vv = eps_vir[:, None] + eps_vir[None, :]
    d2 = e_oo[:, :, None, None] - e_vv[None, None, :, :]
    t2 = np.ascontiguousarray(ovov.transpose(0, 2, 1, 3)) / d2
    return Fragment(eps_occ, eps_vir, t1, np.ascontiguousarray(t2),
                    np.ascontiguousarray(ovvv), np.ascontiguousarray(ooov),
                    np.ascontiguousarray(ovov))


def df_factors(n_occ: int, n_vir: int, n_aux: int, seed, *, b_std: float = 0.05,
               b_scale: float = 1.0) -> np.ndarray:
    """The symmetric density-fitting factors B[P, p, q] (occupied orbitals
    first) that `make_fragment` draws for the same arguments (same random
    stream): its integral blocks are sum_P B[P, p, q] B[P, r, s]."""
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    rng.uniform(-1.5, -0.3, n_occ)
    rng.uniform(0.1, 3.0, n_vir)
    n = n_occ + n_vir
    g = rng.normal(0.0, b_std, size=(n_aux, n, n))
    bfac = np.triu(g) + np.triu(g, 1).transpose(0, 2, 1)
    if b_scale != 1.0:
        bfac *= b_scale
    return np.ascontiguousarray(bfac)


def ov_factors(n_occ: int, n_vir: int, n_aux: int, seed, *, b_std: float = 0.05,
               b_scale: float = 1.0) -> np.ndarray:
    """The occupied-virtual density-fitting factors L[i, a, P] = B^P_{i, a}
    that `make_fragment` draws for the same arguments (same random stream),
    so that (ia|jb) = sum_P L[i, a, P] L[j, b, P] is its ovov block up to the
    rounding of the contraction."""
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    rng.uniform(-1.5, -0.3, n_occ)
    rng.uniform(0.1, 3.0, n_vir)
    n = n_occ + n_vir
    g = rng.normal(0.0, b_std, size=(n_aux, n, n))
    # the occupied-virtual block lies in the drawn upper triangle (i < n_occ <= p)
    out = np.ascontiguousarray(g[:, :n_occ, n_occ:].transpose(1, 2, 0))
    del g
    if b_scale != 1.0:
        out *= b_scale
    return out


def mp2_inputs(n_occ: int, n_vir: int, n_aux: int, seed):
    """(eps_occ, eps_vir, L[i, a, P]) of one seeded synthetic cluster for the
    MP2 energy and density: the orbital energies and factors `make_fragment`
    draws, without the (T) blocks."""
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    eps_vir = np.sort(rng.uniform(0.1, 3.0, n_vir))
    return eps_occ, eps_vir, ov_factors(n_occ, n_vir, n_aux, seed)


# Named single-fragment workloads: occupied / virtual / auxiliary sizes and the
# seed stream they draw from.
WORKLOADS = {
    "o8v40":   dict(n_occ=8,  n_vir=40,  n_aux=144,  stream=0),
    "o24v200": dict(n_occ=24, n_vir=200, n_aux=672,  stream=1),
    "o32v320": dict(n_occ=32, n_vir=320, n_aux=1056, stream=2),
    "o16v120": dict(n_occ=16, n_vir=120, n_aux=408,  stream=4),
    # parity case: 337 virtuals span at least two row and two col tiles of
    # every split build shape, with a ragged edge
    "o3v337":  dict(n_occ=3,  n_vir=337, n_aux=1020, stream=5),
    # MP2 energy and density of a cluster (factors and orbital energies only)
    "mp2_o64v512": dict(n_occ=64, n_vir=512, n_aux=1728, stream=6),
}


def workload_fragment(name: str, **kw) -> Fragment:
    w = WORKLOADS[name]
    return make_fragment(w["n_occ"], w["n_vir"], w["n_aux"],
                         (SEED_ROOT, w["stream"], 0), **kw)


def batch_shapes(name: str):
    """(n_occ, n_vir, n_aux, seed) for each fragment of a named batch.

    batch64: 64 fragments, n_occ ~ U{8..40}, n_vir = rint(n_occ * U[6, 10]).
    batch16: 16 fragments, n_occ ~ U{8..24}, n_vir = rint(n_occ * U[6, 8]).
    Both use n_aux = 3 (n_occ + n_vir).
    """
    if name == "batch64":
        stream, count, lo, hi, rlo, rhi = 3, 64, 8, 40, 6.0, 10.0
    elif name == "batch16":
        stream, count, lo, hi, rlo, rhi = 4, 16, 8, 24, 6.0, 8.0
    else:
        raise KeyError(name)
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, stream, 999]))
    n_occ = rng.integers(lo, hi + 1, size=count)
    ratio = rng.uniform(rlo, rhi, size=count)
    n_vir = np.rint(n_occ * ratio).astype(int)
    out = []
    for f in range(count):
        o, v = int(n_occ[f]), int(n_vir[f])
        out.append((o, v, 3 * (o + v), (SEED_ROOT, stream, 1000 + f)))
    return out
