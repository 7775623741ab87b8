"""The 32-occupied / 320-virtual fragment at full size, in the launch
configuration the benchmark times, against the CPU oracle.

Stored oracle values (tests/golden/, written by make_golden.py from oracle/
and synth/ only):
* o32v320_units.json: ten occupied triples of the float64 fragment;
* o32v320_f32_all_units.json: every occupied triple's (E_WW, E_WV) of the
  fragment with its amplitudes and integrals rounded to float32 (the inputs of
  the split form), and their compensated sums.

Checks:
* float64 path, float64 inputs: the ten stored triples within 1e-10;
* float64 path on the float32-rounded inputs (as float64): every triple within
  1e-10 of the largest and the energy within 1e-10 relative;
* split path on the float32 inputs: error of the energy in micro-Eh and
  relative (bound 2e-6 relative), every triple within 2e-5 of the largest;
* chemically scaled copy (integrals and t2 times 2^-9, exact in float32): the
  oracle value is 2^-36 E_WW + 2^-27 E_WV of the stored parts (every step
  scales exactly by a power of two); the split energy is within 1 micro-Eh
  and the float64 energy within 1e-10 relative.

The inputs are built on the GPU (synth.device): the same draws as the host
generator, values equal up to the rounding of the contractions.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from synth.device import workload_fragment_device

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCALE = 2.0 ** -9


def _golden(name):
    p = os.path.join(GOLDEN, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not generated")
    with open(p) as fh:
        return json.load(fh)


def _run(df, precision):
    import torch
    import paper_2412_18553_amd as sie
    frag = sie.Fragment(df.eps_occ, df.eps_vir, df.t1, df.t2, df.ovvv, df.ooov, df.ovov,
                        precision)
    tri = torch.empty(frag.n_triples, dtype=torch.float64, device="cuda")
    e = sie.energy(frag, triples=tri)
    torch.cuda.synchronize()
    return float(e.item()), tri.cpu().numpy()


def test_o32v320_fp64_stored_triples():
    import torch
    g = _golden("o32v320_units.json")
    print("case o32v320 fp64", flush=True)
    df = workload_fragment_device("o32v320", device="cuda")
    e, tri = _run(df, "fp64")
    del df
    torch.cuda.empty_cache()
    pos = {t: u for u, t in enumerate(oracle.occupied_triples(32))}
    for rec in g["units"]:
        u = pos[tuple(rec["ijk"])]
        print(f"  {rec['ijk']}: gpu {tri[u]!r} oracle {rec['energy']!r}", flush=True)
        assert abs(tri[u] - rec["energy"]) <= 1e-10 * abs(rec["energy"]), rec
    assert abs(tri.sum() - e) <= 1e-12 * abs(e)


@pytest.fixture(scope="module")
def f32_oracle():
    g = _golden("o32v320_f32_all_units.json")
    ww = np.array(g["e_ww_units"])
    wv = np.array(g["e_wv_units"])
    assert ww.shape == (oracle.occupied_triples(32).__len__(),)
    return g, ww, wv


def test_o32v320_fp64_on_float32_inputs_every_triple(f32_oracle):
    import torch
    g, ww, wv = f32_oracle
    print("case o32v320 fp64 on float32-rounded inputs", flush=True)
    df = workload_fragment_device("o32v320", device="cuda", dtype=torch.float32)
    df64 = type(df)(df.eps_occ, df.eps_vir, *(x.double() for x in df.arrays()[2:]))
    del df
    e, tri = _run(df64, "fp64")
    ref = ww + wv
    err = np.abs(tri - ref).max() / np.abs(ref).max()
    print(f"  E gpu {e!r} oracle {g['energy']!r} rel {abs(e - g['energy']) / abs(g['energy']):.2e}"
          f"; worst triple {err:.2e} of the largest", flush=True)
    assert abs(e - g["energy"]) <= 1e-10 * abs(g["energy"])
    assert err <= 1e-10


def test_o32v320_split_vs_oracle(f32_oracle):
    import torch
    g, ww, wv = f32_oracle
    print("case o32v320 split", flush=True)
    df = workload_fragment_device("o32v320", device="cuda", dtype=torch.float32)
    e, tri = _run(df, "split_bf16")
    ref = ww + wv
    err_e = abs(e - g["energy"])
    err_t = np.abs(tri - ref).max() / np.abs(ref).max()
    print(f"  E split {e!r} oracle {g['energy']!r}: error {err_e * 1e6:.4e} micro-Eh, "
          f"{err_e / abs(g['energy']):.2e} relative; worst triple {err_t:.2e} of the largest",
          flush=True)
    assert err_e <= 2e-6 * abs(g["energy"])
    assert err_t <= 2e-5


def test_o32v320_chemical_scale_micro_hartree(f32_oracle):
    import torch
    g, ww, wv = f32_oracle
    # exact: every step of the oracle scales by a power of two
    e_ref = math.fsum(list(ww * SCALE ** 4) + list(wv * SCALE ** 3))
    print(f"case o32v320 chemical scale: oracle {e_ref!r} Eh", flush=True)
    assert 1e-3 < abs(e_ref) < 1e-1
    df = workload_fragment_device("o32v320", device="cuda", dtype=torch.float32,
                                  int_scale=SCALE)
    e_split, _ = _run(df, "split_bf16")
    err = abs(e_split - e_ref)
    print(f"  split {e_split!r}: error {err * 1e6:.4e} micro-Eh ({err / abs(e_ref):.2e} relative)",
          flush=True)
    assert err <= 1e-6
    df64 = type(df)(df.eps_occ, df.eps_vir, *(x.double() for x in df.arrays()[2:]))
    del df
    e64, _ = _run(df64, "fp64")
    print(f"  fp64 {e64!r}: relative error {abs(e64 - e_ref) / abs(e_ref):.2e}", flush=True)
    assert abs(e64 - e_ref) <= 1e-10 * abs(e_ref)
