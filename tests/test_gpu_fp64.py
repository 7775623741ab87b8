"""float64 (T) on the GPU against the CPU oracle, element by element.

Tolerance: 1e-10 relative for the fragment energy; each per-occupied-triple
contribution within 1e-10 of the largest contribution's magnitude.
"""

import json
import os

import numpy as np
import pytest

import oracle
import oracle.triples as T
from synth import make_fragment, workload_fragment

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RTOL = 1e-10


def _dev(f):
    import torch
    cast = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)  # noqa: E731
    return (f.eps_occ, f.eps_vir, cast(f.t1), cast(f.t2), cast(f.ovvv), cast(f.ooov),
            cast(f.ovov))


def run_gpu(f):
    import paper_2412_18553_amd as sie
    e, tri = sie.triples_energy(*_dev(f), return_triples=True)
    return float(e.item()), tri.cpu().numpy()


def check_triples(tri, f, sample=None):
    trip = oracle.occupied_triples(f.n_occ)
    idx = range(len(trip)) if sample is None else sample
    ref = np.array([oracle.occupied_triple_energy(*trip[u], *f.arrays()) for u in idx])
    got = tri[list(idx)]
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert np.max(np.abs(got - ref)) <= RTOL * scale, (got, ref)


@pytest.mark.parametrize("o,v,aux,seed", [
    (2, 3, 8, 2), (3, 17, 20, 3), (4, 16, 24, 4), (5, 33, 40, 5),
    (7, 24, 30, 7), (6, 50, 60, 6), (9, 41, 50, 9)])
def test_small_ragged_vs_oracle(o, v, aux, seed):
    """Sizes that are not multiples of the 16- and 8-wide tiles or of the
    4-deep occupied k-steps, so every ragged edge is exercised."""
    print(f"case o={o} v={v} seed={seed}", flush=True)
    f = make_fragment(o, v, aux, (7, seed))
    e_gpu, tri = run_gpu(f)
    e_ref = T.energy_literal_vectorized(*f.arrays())
    assert abs(e_gpu - e_ref) <= RTOL * abs(e_ref), (e_gpu, e_ref)
    check_triples(tri, f)
    assert abs(tri.sum() - e_gpu) <= 1e-13 * abs(e_gpu)


def test_one_occupied_is_zero():
    f = make_fragment(1, 20, 30, (7, 1))
    e_gpu, tri = run_gpu(f)
    assert e_gpu == 0.0 and tri.tolist() == [0.0]


def test_zero_t2_is_zero():
    f = make_fragment(4, 20, 30, (7, 11))
    f = f.replace(t2=np.zeros_like(f.t2))
    e_gpu, _ = run_gpu(f)
    assert e_gpu == 0.0


def test_small_workload_golden_and_all_triples():
    with open(os.path.join(GOLDEN, "o8v40.json")) as fh:
        g = json.load(fh)
    f = workload_fragment("o8v40")
    e_gpu, tri = run_gpu(f)
    assert abs(e_gpu - g["energy"]) <= RTOL * abs(g["energy"])
    check_triples(tri, f)


def test_deterministic():
    f = make_fragment(6, 37, 40, (7, 21))
    e1, t1 = run_gpu(f)
    e2, t2 = run_gpu(f)
    assert e1 == e2
    assert np.array_equal(t1, t2)


def _golden(name):
    p = os.path.join(GOLDEN, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not generated")
    with open(p) as fh:
        return json.load(fh)


def test_o24v200_full_size():
    """Full 24/200 fragment in the benchmark's launch configuration: the
    energy against the stored oracle value and sampled occupied triples
    against the oracle."""
    g = _golden("o24v200.json")
    f = workload_fragment("o24v200")
    e_gpu, tri = run_gpu(f)
    print(f"o24v200 gpu={e_gpu!r} oracle={g['energy']!r}", flush=True)
    assert abs(e_gpu - g["energy"]) <= RTOL * abs(g["energy"])
    gu = _golden("o24v200_units.json")
    trip = oracle.occupied_triples(f.n_occ)
    pos = {t: u for u, t in enumerate(trip)}
    for rec in gu["units"]:
        u = pos[tuple(rec["ijk"])]
        assert abs(tri[u] - rec["energy"]) <= RTOL * abs(rec["energy"]), rec


@pytest.mark.parametrize("o,v,aux,seed", [(5, 45, 40, 21), (4, 70, 60, 22), (3, 130, 60, 23)])
def test_every_tile_variant(o, v, aux, seed):
    """Each compiled tile shape of the build, forced through the tile table,
    against the oracle (ragged: 45, 70 and 130 are off every tile edge)."""
    import paper_2412_18553_amd as sie
    f = make_fragment(o, v, aux, (7, seed))
    e_ref = T.energy_literal_vectorized(*f.arrays())
    tri0 = None
    try:
        for variant in range(len(sie.tile_variants())):
            print(f"case o={o} v={v} variant={variant}", flush=True)
            sie.set_tile_table([(2048, variant)])
            e_gpu, tri = run_gpu(f)
            assert abs(e_gpu - e_ref) <= RTOL * abs(e_ref), (variant, e_gpu, e_ref)
            # per-unit energies agree between shapes (an error in one layout's
            # terms could cancel in the total only by accident)
            tri0 = tri if tri0 is None else tri0
            scale = np.max(np.abs(tri0))
            assert np.max(np.abs(tri - tri0)) <= RTOL * scale, variant
    finally:
        sie.set_tile_table(None)


def test_finite_check():
    """With the finite check on, a NaN in t2 is reported as
    SIE_ERR_NONFINITE before any (T) kernel runs; with it off the call
    computes (a non-finite energy, no fault); clean inputs pass the scan
    and give the same energy as without it."""
    import torch
    import paper_2412_18553_amd as sie
    from paper_2412_18553_amd import _lib
    f = make_fragment(4, 20, 30, (7, 31))
    args = _dev(f)
    e_ref = float(sie.triples_energy(*args).item())
    bad = list(args)
    bad[3] = args[3].clone()
    bad[3][1, 2, 3, 4] = float("nan")
    try:
        sie.set_check_finite(True)
        assert float(sie.triples_energy(*args).item()) == e_ref
        with pytest.raises(sie.SieError) as err:
            sie.triples_energy(*bad)
        assert err.value.status == _lib.SIE_ERR_NONFINITE and "t2" in str(err.value)
    finally:
        sie.set_check_finite(False)
    assert not np.isfinite(float(sie.triples_energy(*bad).item()))
    torch.cuda.synchronize()


def test_call_returns_before_the_device_finishes():
    """The energy call enqueues its table uploads and kernels without waiting
    for work already on the stream: queued behind a long spin kernel, it
    returns long before the spin ends, and the result is then correct."""
    import time
    import torch
    import paper_2412_18553_amd as sie
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("no spin kernel in this torch build")
    f = make_fragment(5, 24, 30, (7, 32))
    frag = sie.Fragment(*_dev(f))
    ws = torch.empty(sie.workspace_size(frag), dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    e_ref = float(sie.energy(frag, workspace=ws, out=out).item())
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    torch.cuda._sleep(1 << 29)
    stop.record()
    t0 = time.perf_counter()
    sie.energy(frag, workspace=ws, out=out)
    host_ms = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()
    spin_ms = start.elapsed_time(stop)
    print(f"spin {spin_ms:.1f} ms, energy call returned after {host_ms:.2f} ms", flush=True)
    if spin_ms < 20.0:
        pytest.skip("spin kernel too short to tell")
    assert host_ms < 0.5 * spin_ms
    assert float(out.item()) == e_ref
