"""The device-side fragment builder (synth/device.py) run on the CPU against
the host generator: same draws, same values up to the rounding of the
contractions, exact twin symmetries, exact power-of-two integral scaling."""

import numpy as np
import pytest

from synth import make_fragment
from synth.device import make_fragment_device

torch = pytest.importorskip("torch")
NAMES = ("t1", "t2", "ovvv", "ooov", "ovov")


@pytest.mark.parametrize("o,v,aux,seed", [(3, 17, 20, (1, 2)), (5, 28, 40, (3,)), (1, 4, 5, (4,))])
def test_device_builder_matches_host(o, v, aux, seed):
    h = make_fragment(o, v, aux, seed)
    d = make_fragment_device(o, v, aux, seed, device="cpu")
    assert np.array_equal(h.eps_occ, d.eps_occ) and np.array_equal(h.eps_vir, d.eps_vir)
    for n in NAMES:
        x, y = getattr(h, n), getattr(d, n).numpy()
        assert np.abs(x - y).max() <= 1e-15 * np.abs(x).max(), n
    t2, ovvv = d.t2.numpy(), d.ovvv.numpy()
    assert np.array_equal(t2, t2.transpose(1, 0, 3, 2))
    assert np.array_equal(ovvv, ovvv.transpose(0, 1, 3, 2))
    ooov, ovov = d.ooov.numpy(), d.ovov.numpy()
    assert np.array_equal(ooov, ooov.transpose(1, 0, 2, 3))
    assert np.array_equal(ovov, ovov.transpose(2, 3, 0, 1))


def test_float32_and_power_of_two_scale():
    base = make_fragment_device(4, 21, 30, (5,), device="cpu", dtype=torch.float32)
    sc = make_fragment_device(4, 21, 30, (5,), device="cpu", dtype=torch.float32,
                              int_scale=2.0 ** -9)
    assert torch.equal(base.t1, sc.t1)
    for n in ("t2", "ovvv", "ooov", "ovov"):
        assert torch.equal(getattr(base, n) * 2.0 ** -9, getattr(sc, n)), n
    h = make_fragment(4, 21, 30, (5,)).astype(np.float32)
    for n in NAMES:   # float32 rounding of values equal to ~1e-16: equal or one ulp apart
        x, y = getattr(h, n), getattr(base, n).numpy()
        assert np.abs(x - y).max() <= 2.0 ** -23 * np.abs(x).max(), n
