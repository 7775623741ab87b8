"""Orbital-energy gradient of the (T) energy on the GPU (the eps_occ and
eps_vir outputs of sie_triples_backward).

* small ragged fragments: every entry against the oracle (oracle/grad.py,
  pinned by Richardson differences of the spin-orbital energy), within 1e-10
  of the largest entry;
* 16 occupied / 120 virtuals: homogeneity (E is of degree -1 in the orbital
  energies: sum_p e_p dE/de_p = -E), invariance under a common shift
  (sum_p dE/de_p = 0) and Richardson central differences of the GPU energy
  along a seeded direction;
* batched gradients equal single-fragment ones bitwise; many small rounds
  agree with one round to rounding; the upstream scale enters linearly;
* split precision against the float64 oracle (reported, bound 1e-4 of the
  largest entry);
* torch autograd through SieTriples with orbital energies as tensors.
"""

import numpy as np
import pytest

from oracle.grad import energy_gradient
from synth import make_fragment, workload_fragment

pytestmark = pytest.mark.gpu

EPS = ("eps_occ", "eps_vir")
RTOL = 1e-10


def _frag(f, precision="fp64"):
    import torch
    import paper_2412_18553_amd as sie
    dt = torch.float64 if precision == "fp64" else torch.float32
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    return sie.Fragment(f.eps_occ, f.eps_vir, cast(f.t1), cast(f.t2), cast(f.ovvv),
                        cast(f.ooov), cast(f.ovov), precision)


def eps_grad(frags, grad_e=None, max_workspace_bytes=0):
    import torch
    import paper_2412_18553_amd as sie
    ge = None if grad_e is None else torch.tensor(grad_e, dtype=torch.float64, device="cuda")
    g = sie.backward(frags, grad_e=ge, want=EPS, max_workspace_bytes=max_workspace_bytes)
    torch.cuda.synchronize()
    if isinstance(g, dict):
        return {n: g[n].cpu().numpy() for n in EPS}
    return [{n: gx[n].cpu().numpy() for n in EPS} for gx in g]


def _check(got, ref, tol):
    for n in EPS:
        scale = max(np.abs(ref[n]).max(), 1e-300)
        err = np.abs(got[n] - ref[n]).max() / scale
        print(f"  {n}: max|err|/max|g| = {err:.2e}", flush=True)
        assert err <= tol, (n, err)


@pytest.mark.parametrize("o,v,aux,seed", [
    (2, 3, 8, 1), (3, 9, 24, 2), (4, 12, 30, 3), (5, 20, 60, 4), (3, 33, 40, 5),
    (4, 41, 60, 6)])
def test_eps_gradient_vs_oracle(o, v, aux, seed):
    """Virtual counts off the 8-wide orbit blocks (ragged last blocks) and
    equal-block orbits of every kind."""
    print(f"case eps o={o} v={v} seed={seed}", flush=True)
    f = make_fragment(o, v, aux, (21, seed))
    _, _, _, ref = energy_gradient(*f.arrays())
    _check(eps_grad(_frag(f)), ref, RTOL)


def test_eps_gradient_with_other_gradients_and_one_occupied():
    """Requested together with the amplitude and integral gradients it is
    unchanged; with one occupied orbital the energy and gradient are zero."""
    import torch
    import paper_2412_18553_amd as sie
    f = make_fragment(4, 20, 30, (21, 7))
    fr = _frag(f)
    g_all = sie.backward(fr, want=sie.ALL_GRAD_NAMES)
    torch.cuda.synchronize()
    g_eps = eps_grad(fr)
    for n in EPS:
        assert np.array_equal(g_all[n].cpu().numpy(), g_eps[n]), n
    g1 = eps_grad(_frag(make_fragment(1, 12, 20, (21, 8))))
    for n in EPS:
        assert np.all(g1[n] == 0.0), n


def test_eps_gradient_o16v120_identities():
    import paper_2412_18553_amd as sie
    f = workload_fragment("o16v120")
    fr = _frag(f)
    print("case eps o16v120", flush=True)
    g = eps_grad(fr)
    e = float(sie.energy(fr).item())
    euler = float(np.dot(f.eps_occ, g["eps_occ"]) + np.dot(f.eps_vir, g["eps_vir"]))
    print(f"  E = {e!r}, sum e dE/de = {euler!r}", flush=True)
    assert abs(euler + e) <= 1e-10 * abs(e)
    total = float(g["eps_occ"].sum() + g["eps_vir"].sum())
    scale = float(np.abs(g["eps_occ"]).sum() + np.abs(g["eps_vir"]).sum())
    assert abs(total) <= 1e-12 * scale, (total, scale)
    # Richardson central differences of the GPU energy along a seeded direction
    rng = np.random.default_rng(16)
    for which, name in ((0, "eps_occ"), (1, "eps_vir")):
        d = rng.normal(size=(f.n_occ,) if which == 0 else (f.n_vir,))

        def energy_at(step):
            eo, ev = f.eps_occ.copy(), f.eps_vir.copy()
            (eo if which == 0 else ev)[:] += step * d
            frs = sie.Fragment(eo, ev, fr.t1, fr.t2, fr.ovvv, fr.ooov, fr.ovov, "fp64")
            return float(sie.energy(frs).item())

        def central(h):
            return (energy_at(h) - energy_at(-h)) / (2 * h)

        h = 1e-3
        fd = (4 * central(h / 2) - central(h)) / 3
        an = float(np.dot(g[name], d))
        print(f"  {name}: analytic {an!r} differences {fd!r}", flush=True)
        assert abs(an - fd) <= 1e-8 * abs(fd)


def test_eps_gradient_batched_rounds_and_scale():
    import paper_2412_18553_amd as sie
    shapes = [(3, 17, 30, 1), (5, 24, 40, 2), (4, 9, 20, 3)]
    fs = [make_fragment(o, v, a, (22, s)) for o, v, a, s in shapes]
    frs = [_frag(f) for f in fs]
    batched = eps_grad(frs)
    for fr, gb in zip(frs, batched):
        gs = eps_grad(fr)
        for n in EPS:
            assert np.array_equal(gs[n], gb[n]), n
    # many small rounds (one occupied triple per round) against one round
    f = make_fragment(5, 20, 60, (22, 4))
    fr = _frag(f)
    full = sie.backward_workspace_size(fr)
    cube3 = 3 * 20 ** 3 * 8                    # G, H and G transposed of one triple
    g_small = eps_grad(fr, max_workspace_bytes=full - 29 * cube3)
    g_full = eps_grad(fr)
    for n in EPS:
        assert np.abs(g_small[n] - g_full[n]).max() <= 1e-13 * np.abs(g_full[n]).max(), n
    g25 = eps_grad(fr, grad_e=[2.5])
    for n in EPS:
        assert np.abs(g25[n] - 2.5 * g_full[n]).max() <= 1e-13 * np.abs(2.5 * g_full[n]).max()


def test_eps_gradient_split_vs_fp64_oracle():
    f = make_fragment(4, 33, 60, (23, 1))
    _, _, _, ref = energy_gradient(*f.arrays())
    got = eps_grad(_frag(f.astype(np.float32).astype(np.float64), "split_bf16"))
    _check(got, ref, 1e-4)


def test_autograd_orbital_energies():
    import torch
    import paper_2412_18553_amd as sie
    f = make_fragment(4, 15, 30, (23, 2))
    _, _, _, ref = energy_gradient(*f.arrays())
    eo = torch.tensor(f.eps_occ, requires_grad=True)
    ev = torch.tensor(f.eps_vir, requires_grad=True)
    fr = _frag(f)
    e = sie.SieTriples.apply(eo, ev, fr.t1, fr.t2, fr.ovvv, fr.ooov, fr.ovov)
    (3.0 * e).backward()
    for name, leaf in (("eps_occ", eo), ("eps_vir", ev)):
        err = np.abs(leaf.grad.numpy() - 3.0 * ref[name]).max() / np.abs(3.0 * ref[name]).max()
        assert err <= RTOL, (name, err)
