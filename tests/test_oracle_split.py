"""Pins of the split-precision quantization emulator (oracle/split.py).

* bf16 rounding equals torch's float32 -> bfloat16 conversion (round to
  nearest even), an independent library routine;
* hi + lo represents x to 16 significant bits, and lo is exactly zero when x
  is already a bfloat16 number;
* with operands that are bfloat16 numbers the emulator is the float64 oracle;
* the split error is small and bounded as the representation predicts;
* the product set is hi*hi + hi*lo + lo*hi: on operands x = h (1 + 2^-9)
  (h a bfloat16 number, so hi = h and lo = h 2^-9 exactly) every dropped
  lo*lo term is the same fraction c = 2^-18 / (1 + 2^-9)^2 of its product,
  Wt scales by (1 - c) exactly and E_split = (1 - c)^2 E_WW + (1 - c) E_WV
  in closed form; keeping lo*lo (4 products) or dropping hi*lo or lo*hi
  (2 products) gives a different value.
"""

import numpy as np
import pytest

import oracle.triples as T
from oracle.split import bf16_rne, energy_split_emulated, split_bf16
from synth import make_fragment


def test_bf16_rne_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.normal(size=200000) * 10.0 ** rng.uniform(-6, 6, 200000)).astype(np.float32)
    # ties: values exactly halfway between two bf16 numbers
    base = bf16_rne(x[:1000])
    ties = (base.view(np.uint32) | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16_rne(x), ref)


def test_split_representation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=100000).astype(np.float32)
    hi, lo = split_bf16(x)
    rel = np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    exact = bf16_rne(x)
    h2, l2 = split_bf16(exact)
    assert np.array_equal(h2, exact) and not np.any(l2)


def test_emulator_exact_for_bf16_operands():
    f = make_fragment(3, 9, 16, (31,)).astype(np.float32)
    q = f.replace(t2=bf16_rne(f.t2), ovvv=bf16_rne(f.ovvv), ooov=bf16_rne(f.ooov))
    a64 = [np.asarray(x, np.float64) for x in q.arrays()]
    e64 = T.energy_literal_vectorized(*a64)
    assert abs(energy_split_emulated(*q.arrays()) - e64) <= 1e-13 * abs(e64)


def test_emulator_error_small():
    f = make_fragment(4, 12, 20, (32,)).astype(np.float32)
    a64 = [np.asarray(x, np.float64) for x in f.arrays()]
    e64 = T.energy_literal_vectorized(*a64)
    es = energy_split_emulated(*f.arrays())
    assert 0 < abs(es - e64) <= 1e-5 * abs(e64)


def _coherent_operands(f):
    """Every t2, ovvv and ooov entry replaced by h (1 + 2^-9) with h its
    bfloat16 rounding (exact in float32; hi = h, lo = h 2^-9)."""
    g = lambda x: bf16_rne(x) * np.float32(1.0 + 2.0 ** -9)  # noqa: E731
    return f.replace(t2=g(f.t2), ovvv=g(f.ovvv), ooov=g(f.ooov))


def test_emulator_product_set_closed_form():
    f = _coherent_operands(make_fragment(3, 10, 16, (33,)).astype(np.float32))
    hi, lo = split_bf16(f.ovvv)
    assert np.array_equal(hi * np.float32(2.0 ** -9), lo)
    a64 = [np.asarray(x, np.float64) for x in f.arrays()]
    _, ww, wv = T.energy_literal_vectorized(*a64, return_parts=True)
    c = 2.0 ** -18 / (1.0 + 2.0 ** -9) ** 2
    predicted = (1 - c) ** 2 * ww + (1 - c) * wv
    e3 = energy_split_emulated(*f.arrays())
    assert abs(e3 - predicted) <= 1e-13 * abs(predicted)
    # the exact value (four products) and the two-product sums are far off
    e4 = ww + wv
    assert abs(e3 - e4) >= 0.5 * 2 * c * abs(ww)
    t2h, t2l = split_bf16(f.t2)
    vh, vl = split_bf16(f.ovvv)
    oh, ol = split_bf16(f.ooov)
    two = T.energy_literal_vectorized(*a64, x_terms=[(vh, oh, t2h), (vh, oh, t2l)])
    assert abs(two - e3) >= 100 * abs(e3 - predicted) + 1e-3 * abs(e3)
