"""float64 gradient of the (T) energy on the GPU (sie_triples_backward).

Small fragments: every entry of every gradient block against the oracle
gradient (oracle/grad.py, itself pinned by finite differences of the
textbook spin-orbital energy), within 1e-10 of the block's largest entry.

The 16-occupied / 120-virtual fragment (too large for the dense oracle):
properties that hold at any size, evaluated with the GPU energy path
  * central differences along seeded symmetric directions, per block (the
    energy is at most quadratic in each block, so the difference is exact
    up to rounding), within 1e-8 relative;
  * the Euler identities of the W/V split: sum t1 g_t1 = E_WV = sum ovov
    g_ovov, sum t2 g_t2 = 2 E_WW + E_WV = sum ovvv g_ovvv + sum ooov g_ooov,
    with E_WV = E - E(t1 = 0) and E_WW = E(t1 = 0) from the energy path.
"""

import numpy as np
import pytest

from oracle.grad import energy_gradient, symmetrize_direction
from synth import make_fragment, workload_fragment

pytestmark = pytest.mark.gpu

NAMES = ("t1", "t2", "ovvv", "ooov", "ovov")
RTOL = 1e-10


def _dev(f):
    import torch
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)  # noqa: E731
    return [f.eps_occ, f.eps_vir] + [cast(getattr(f, n)) for n in NAMES]


def gpu_grad(f, grad_e=None, e_frag=None, max_workspace_bytes=0):
    import torch
    import paper_2412_18553_amd as sie
    frag = sie.Fragment(*_dev(f))
    ge = None if grad_e is None else torch.tensor([grad_e], dtype=torch.float64, device="cuda")
    g = sie.backward(frag, grad_e=ge, e_frag=e_frag, max_workspace_bytes=max_workspace_bytes)
    torch.cuda.synchronize()
    return {n: g[n].cpu().numpy() for n in NAMES}


def gpu_energy(args):
    import paper_2412_18553_amd as sie
    return float(sie.triples_energy(*args).item())


@pytest.mark.parametrize("o,v,aux,seed", [
    (2, 3, 8, 1), (3, 9, 24, 2), (4, 12, 30, 3), (5, 20, 60, 4), (3, 33, 40, 5),
    (4, 70, 90, 6)])
def test_gradient_vs_oracle(o, v, aux, seed):
    """Ragged sizes: virtual counts off the 8-, 32- and 64-wide tiles, and
    70 virtuals spanning two 64-row tiles and three 32-col tiles."""
    print(f"case o={o} v={v} seed={seed}", flush=True)
    f = make_fragment(o, v, aux, (11, seed))
    _, _, _, ref = energy_gradient(*f.arrays())
    got = gpu_grad(f)
    for n in NAMES:
        scale = max(np.abs(ref[n]).max(), 1e-300)
        err = np.abs(got[n] - ref[n]).max() / scale
        print(f"  {n}: max|err|/max|g| = {err:.2e}", flush=True)
        assert err <= RTOL, (n, err)


def test_gradient_with_three_layout_table():
    """A tile table that selects a three-layout build shape for the energy:
    the gradient rebuilds W-tilde with a two-layout shape and is unchanged."""
    import paper_2412_18553_amd as sie
    three = [v for v, s in enumerate(sie.tile_variants()) if s[6] >= 3]
    assert three
    f = make_fragment(4, 20, 30, (11, 12))
    _, _, _, ref = energy_gradient(*f.arrays())
    try:
        sie.set_tile_table([(2048, three[0])])
        got = gpu_grad(f)
    finally:
        sie.set_tile_table(None)
    for n in NAMES:
        scale = max(np.abs(ref[n]).max(), 1e-300)
        assert np.abs(got[n] - ref[n]).max() <= RTOL * scale, n


def test_one_occupied_gradient_is_zero():
    f = make_fragment(1, 12, 20, (11, 9))
    got = gpu_grad(f)
    for n in NAMES:
        assert np.all(got[n] == 0.0), n


def test_energy_output_matches_forward_and_scaling():
    import torch
    import paper_2412_18553_amd as sie
    f = make_fragment(4, 20, 40, (11, 10))
    e_fwd = gpu_energy(_dev(f))
    e_frag = torch.empty(1, dtype=torch.float64, device="cuda")
    g1 = gpu_grad(f, e_frag=e_frag)
    assert float(e_frag.item()) == e_fwd                   # same kernels, same order
    g25 = gpu_grad(f, grad_e=2.5)
    for n in NAMES:      # the scale enters before the contractions: rounding differs
        assert np.abs(g25[n] - 2.5 * g1[n]).max() <= 1e-13 * np.abs(2.5 * g1[n]).max(), n
    g1b = gpu_grad(f)
    for n in NAMES:
        assert np.array_equal(g1b[n], g1[n]), n            # deterministic
    del sie


def test_small_workspace_many_rounds():
    """A workspace cap that admits one occupied triple per round."""
    import paper_2412_18553_amd as sie
    f = make_fragment(5, 20, 60, (11, 4))
    frag = sie.Fragment(*_dev(f))
    full = sie.backward_workspace_size(frag)
    pair = 2 * 20 ** 3 * 8                      # two float64 cubes of one triple
    small = sie.backward_workspace_size(frag, max_bytes=full - 29 * pair)
    assert small == full - 29 * pair
    g_small = gpu_grad(f, max_workspace_bytes=small)
    g_full = gpu_grad(f)
    for n in NAMES:
        scale = np.abs(g_full[n]).max()
        assert np.abs(g_small[n] - g_full[n]).max() <= 1e-13 * scale, n


def test_batched_backward_matches_single():
    import torch
    import paper_2412_18553_amd as sie
    fs = [make_fragment(4, 20, 40, (11, 20)), make_fragment(3, 13, 30, (11, 21)),
          make_fragment(5, 9, 20, (11, 22))]
    frags = [sie.Fragment(*_dev(f)) for f in fs]
    ge = torch.tensor([1.0, -0.5, 3.0], dtype=torch.float64, device="cuda")
    e_frag = torch.empty(3, dtype=torch.float64, device="cuda")
    gs = sie.backward(frags, grad_e=ge, e_frag=e_frag)
    torch.cuda.synchronize()
    for x, f in enumerate(fs):
        single = gpu_grad(f, grad_e=float(ge[x].item()))
        for n in NAMES:
            got = gs[x][n].cpu().numpy()
            scale = np.abs(single[n]).max()
            assert np.abs(got - single[n]).max() <= 1e-13 * scale, (x, n)
        assert float(e_frag[x].item()) == gpu_energy(_dev(f))


def test_autograd_function():
    import torch
    import paper_2412_18553_amd as sie
    f = make_fragment(3, 17, 30, (11, 30))
    args = _dev(f)
    leaves = [a.clone().requires_grad_(True) for a in args[2:]]
    e = sie.SieTriples.apply(args[0], args[1], *leaves)
    (3.0 * e).backward()
    ref = gpu_grad(f, grad_e=3.0)
    for n, leaf in zip(NAMES, leaves):
        assert np.array_equal(leaf.grad.cpu().numpy(), ref[n]), n
    _, _, _, oref = energy_gradient(*f.arrays())
    for n, leaf in zip(NAMES, leaves):
        g = leaf.grad.cpu().numpy()
        assert np.abs(g - 3.0 * oref[n]).max() <= RTOL * 3.0 * np.abs(oref[n]).max(), n


@pytest.mark.parametrize("o,v,aux,seed,b_scale", [(4, 20, 40, 40, 1.0), (4, 33, 60, 41, 0.3)])
def test_split_backward_vs_fp64_oracle(o, v, aux, seed, b_scale):
    """Split precision (float32 inputs, bf16 hi/lo products, float32 G and H,
    float64 contractions and sums) against the float64 oracle gradient; the
    relative error per block is printed and bounded by 1e-5 of the block's
    largest entry."""
    import torch
    import paper_2412_18553_amd as sie
    f = make_fragment(o, v, aux, (11, seed), b_scale=b_scale)
    _, _, _, ref = energy_gradient(*f.arrays())
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32)  # noqa: E731
    frag = sie.Fragment(f.eps_occ, f.eps_vir, *[cast(getattr(f, n)) for n in NAMES],
                        precision="split_bf16")
    g = sie.backward(frag)
    torch.cuda.synchronize()
    for n in NAMES:
        got = g[n].cpu().numpy()
        err = np.abs(got - ref[n]).max() / np.abs(ref[n]).max()
        print(f"  split {n}: max|err|/max|g| = {err:.2e}", flush=True)
        assert err <= 1e-5, (n, err)


def test_split_batched_backward_matches_single_and_oracle():
    """Split precision over a batch of ragged fragments: each fragment's
    gradient equals its single-fragment split gradient up to the order of
    the float64 sums, and the float64 oracle gradient within 1e-5 of each
    block's largest entry."""
    import torch
    import paper_2412_18553_amd as sie
    fs = [make_fragment(4, 20, 40, (11, 50)), make_fragment(3, 13, 30, (11, 51)),
          make_fragment(5, 9, 20, (11, 52)), make_fragment(3, 33, 40, (11, 53))]
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32)  # noqa: E731
    frags = [sie.Fragment(f.eps_occ, f.eps_vir, *[cast(getattr(f, n)) for n in NAMES],
                          precision="split_bf16") for f in fs]
    ge = torch.tensor([1.0, -0.5, 3.0, 2.0], dtype=torch.float64, device="cuda")
    gs = sie.backward(frags, grad_e=ge)
    torch.cuda.synchronize()
    for x, (f, fr) in enumerate(zip(fs, frags)):
        single = sie.backward(fr, grad_e=ge[x:x + 1].contiguous())
        f32 = f.astype(np.float32)
        _, _, _, ref = energy_gradient(*[np.asarray(a, np.float64) for a in f32.arrays()])
        for n in NAMES:
            got = gs[x][n].cpu().numpy()
            one = single[n].cpu().numpy()
            scale = np.abs(one).max()
            assert np.abs(got - one).max() <= 1e-12 * scale, (x, n)
            gx = float(ge[x].item())
            err = np.abs(got - gx * ref[n]).max() / np.abs(gx * ref[n]).max()
            print(f"  fragment {x} {n}: split vs oracle {err:.2e}", flush=True)
            assert err <= 1e-5, (x, n, err)


def test_batch16_split_gradient_vs_fp64():
    """The 16-fragment adjoint batch (n_occ 8..24, n_vir 6-8 n_occ) in split
    precision against the float64 GPU gradient of the same float32-rounded
    inputs (itself pinned to the oracle gradient on the small cases above and
    by differences and Euler identities at 16/120): per block within 1e-5 of
    the largest entry; the float64 gradient satisfies the Euler identity
    sum t1 dE/dt1 = sum ovov dE/dovov (both equal E_WV)."""
    import torch
    import paper_2412_18553_amd as sie
    from synth import batch_shapes
    from synth.device import make_fragment_device
    shapes = batch_shapes("batch16")
    dfs = [make_fragment_device(o, v, a, seed, device="cuda", dtype=torch.float32)
           for (o, v, a, seed) in shapes]
    f32 = [sie.Fragment(*d.arrays(), precision="split_bf16") for d in dfs]
    f64 = [sie.Fragment(d.eps_occ, d.eps_vir, *(x.double() for x in d.arrays()[2:]))
           for d in dfs]
    print(f"case batch16: {[(o, v) for (o, v, _, _) in shapes]}", flush=True)
    g32 = sie.backward(f32)
    g64 = sie.backward(f64)
    torch.cuda.synchronize()
    worst = {n: 0.0 for n in NAMES}
    for x in range(len(shapes)):
        for n in NAMES:
            a, b = g32[x][n], g64[x][n]
            err = float((a - b).abs().max() / b.abs().max())
            worst[n] = max(worst[n], err)
        e1 = float((f64[x].t1 * g64[x]["t1"]).sum())
        e2 = float((f64[x].ovov * g64[x]["ovov"]).sum())
        assert abs(e1 - e2) <= 1e-10 * max(abs(e1), abs(e2)), x
    print("  worst split error per block: " + ", ".join(f"{n} {worst[n]:.2e}" for n in NAMES),
          flush=True)
    for n in NAMES:
        assert worst[n] <= 1e-5, n


# ------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def o16v120():
    f = workload_fragment("o16v120")
    return f, _dev(f), gpu_grad(f)


def test_o16v120_directional_differences(o16v120):
    f, args, g = o16v120
    rng = np.random.default_rng(16120)
    for pos, n in enumerate(NAMES):
        x = getattr(f, n)
        v = symmetrize_direction(n, rng.normal(size=x.shape) * np.abs(x).mean())
        h = 0.5        # exact for any step: E is at most quadratic in each block
        plus, minus = list(args), list(args)
        import torch
        vd = torch.from_numpy(v).to("cuda", torch.float64)
        plus[2 + pos] = args[2 + pos] + h * vd
        minus[2 + pos] = args[2 + pos] - h * vd
        fd = (gpu_energy(plus) - gpu_energy(minus)) / (2 * h)
        an = float(np.sum(g[n] * v))
        print(f"  {n}: analytic {an:.12e} differences {fd:.12e}", flush=True)
        assert abs(an - fd) <= 1e-8 * abs(fd), (n, an, fd)


def test_o16v120_euler_identities(o16v120):
    import torch
    f, args, g = o16v120
    e = gpu_energy(args)
    zero_t1 = list(args)
    zero_t1[2] = torch.zeros_like(args[2])
    e_ww = gpu_energy(zero_t1)
    e_wv = e - e_ww
    dot = {n: float(np.sum(getattr(f, n) * g[n])) for n in NAMES}
    tol = 1e-10 * abs(e)
    assert abs(dot["t1"] - e_wv) <= tol
    assert abs(dot["ovov"] - e_wv) <= tol
    assert abs(dot["t2"] - (2 * e_ww + e_wv)) <= tol
    assert abs(dot["ovvv"] + dot["ooov"] - (2 * e_ww + e_wv)) <= tol
