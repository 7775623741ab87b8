"""The seeded synthetic fragments of synth/fragments.py, built on a torch
device.

The random draws (orbital energies, DF factors, t1) are the same numpy draws
in the same order as `make_fragment`; the DF contractions, the twin
averaging and the MP2 amplitudes run with torch on `device`, so a fragment
with tens of GB of integrals is built in seconds on a GPU instead of minutes
with host BLAS.  The values equal the host generator's up to the rounding of
the contractions (about 1e-16 relative); the twin symmetries are exact.
No (T) arithmetic is done here.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class DeviceFragment:
    eps_occ: np.ndarray          # host float64
    eps_vir: np.ndarray          # host float64
    t1: "object"                 # torch tensors on the device, dtype as requested
    t2: "object"
    ovvv: "object"
    ooov: "object"
    ovov: "object"

    @property
    def n_occ(self) -> int:
        return int(self.eps_occ.shape[0])

    @property
    def n_vir(self) -> int:
        return int(self.eps_vir.shape[0])

    def arrays(self):
        return (self.eps_occ, self.eps_vir, self.t1, self.t2, self.ovvv, self.ooov, self.ovov)

    def host(self):
        """The same fragment as host float64 numpy arrays (synth.Fragment)."""
        from .fragments import Fragment
        h = lambda x: x.detach().to("cpu").double().numpy()  # noqa: E731
        return Fragment(self.eps_occ, self.eps_vir, h(self.t1), h(self.t2), h(self.ovvv),
                        h(self.ooov), h(self.ovov))


def make_fragment_device(n_occ: int, n_vir: int, n_aux: int, seed, *, device,
                         dtype=None, b_std: float = 0.05, t1_std: float = 1e-2,
                         b_scale: float = 1.0, zero_t1: bool = False,
                         int_scale: float = 1.0) -> DeviceFragment:
    """`make_fragment` with the contractions on `device`.

    dtype: torch dtype of the returned amplitudes and integrals (float64 by
    default; float32 rounds the float64 values to nearest).  `int_scale`
    multiplies the integrals and t2 after they are built (a power of two
    scales them exactly, also after rounding to float32)."""
    import torch

    dtype = torch.float64 if dtype is None else dtype
    if n_occ < 1 or n_vir < 1 or n_aux < 1:
        raise ValueError("n_occ, n_vir and n_aux must be >= 1")
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    eps_vir = np.sort(rng.uniform(0.1, 3.0, n_vir))
    n = n_occ + n_vir
    g = torch.from_numpy(rng.normal(0.0, b_std, size=(n_aux, n, n))).to(device)
    bfac = torch.triu(g) + torch.triu(g, 1).transpose(1, 2)
    del g
    if b_scale != 1.0:
        bfac *= b_scale
    t1 = rng.normal(0.0, t1_std, size=(n_occ, n_vir))
    if zero_t1:
        t1[...] = 0.0
    o, v = n_occ, n_vir
    b_oo = bfac[:, :o, :o].reshape(n_aux, o * o)
    b_ov = bfac[:, :o, o:].reshape(n_aux, o * v)
    b_vv = bfac[:, o:, o:].reshape(n_aux, v * v)

    ovvv = torch.empty((o, v, v, v), dtype=dtype, device=device)
    for i in range(o):   # one occupied slice at a time: exact b <-> c symmetry
        s = (b_ov[:, i * v:(i + 1) * v].T @ b_vv).reshape(v, v, v)
        s = 0.5 * (s + s.transpose(1, 2))
        if int_scale != 1.0:
            s *= int_scale
        ovvv[i] = s.to(dtype)
        del s
    ooov = (b_oo.T @ b_ov).reshape(o, o, o, v)
    ooov = 0.5 * (ooov + ooov.transpose(0, 1))
    ovov = (b_ov.T @ b_ov).reshape(o, v, o, v)
    ovov = 0.5 * (ovov + ovov.permute(2, 3, 0, 1))
    del bfac, b_oo, b_ov, b_vv

    eo = torch.from_numpy(eps_occ).to(device)
    ev = torch.from_numpy(eps_vir).to(device)
    e_oo = eo[:, None] + eo[None, :]
    e_vv = ev[:, None] + ev[None, :]
    d2 = e_oo[:, :, None, None] - e_vv[None, None, :, :]
    t2 = ovov.permute(0, 2, 1, 3).contiguous() / d2
    if int_scale != 1.0:
        ooov *= int_scale
        ovov *= int_scale
        t2 *= int_scale
    cast = lambda x: x.to(dtype).contiguous()  # noqa: E731
    return DeviceFragment(eps_occ, eps_vir, cast(torch.from_numpy(t1).to(device)), cast(t2),
                          ovvv, cast(ooov), cast(ovov))


def df_factors_device(n_occ: int, n_vir: int, n_aux: int, seed, *, device,
                      b_std: float = 0.05):
    """The symmetric factors B[P, p, q] (float64, on `device`) that
    `make_fragment_device` draws for the same arguments."""
    import torch
    rng = np.random.default_rng(np.random.SeedSequence([int(s) for s in seed]))
    rng.uniform(-1.5, -0.3, n_occ)
    rng.uniform(0.1, 3.0, n_vir)
    n = n_occ + n_vir
    g = torch.from_numpy(rng.normal(0.0, b_std, size=(n_aux, n, n))).to(device)
    return (torch.triu(g) + torch.triu(g, 1).transpose(1, 2)).contiguous()


def workload_df_factors_device(name: str, **kw):
    from .fragments import SEED_ROOT, WORKLOADS
    w = WORKLOADS[name]
    return df_factors_device(w["n_occ"], w["n_vir"], w["n_aux"], (SEED_ROOT, w["stream"], 0),
                             **kw)


def workload_fragment_device(name: str, **kw) -> DeviceFragment:
    from .fragments import SEED_ROOT, WORKLOADS
    w = WORKLOADS[name]
    return make_fragment_device(w["n_occ"], w["n_vir"], w["n_aux"],
                                (SEED_ROOT, w["stream"], 0), **kw)
