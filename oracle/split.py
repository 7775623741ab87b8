"""Quantization emulator for the split-precision (T) form.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The split form stores every float32 amplitude and integral x that enters the
W-tilde contractions (eq. W_in_CCSD_T) as two bfloat16 numbers
    hi = bf16_rne(x),   lo = bf16_rne(x - hi)
(x - hi is exact in float32), and forms each product as hi*hi + hi*lo + lo*hi,
dropping lo*lo.  This module evaluates exactly that arithmetic in float64 (no
float32 accumulation), with D, V, R and the energy sum in float64 as in the
plain oracle, so that the GPU split result can be compared with the pure
quantization effect.  bf16_rne is round-to-nearest-even on the float32 bit
pattern (finite inputs).
"""

from __future__ import annotations

import numpy as np

from .triples import energy_literal_vectorized


def bf16_rne(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returned
    as float32 values that bfloat16 represents exactly."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).reshape(x.shape)


def split_bf16(x):
    """(hi, lo) with hi = bf16_rne(x), lo = bf16_rne(x - hi), both float32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne(x - hi)
    return hi, lo


def energy_split_emulated(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, return_parts=False):
    """E_x with the contractions of eq. W_in_CCSD_T evaluated as
    hi*hi + hi*lo + lo*hi products of split float32 operands, summed exactly;
    everything else as in `energy_literal_vectorized`.  t1 and ovov enter only
    V (float64 epilogue) and are taken at their float32 values."""
    f32 = lambda a: np.asarray(a, dtype=np.float32)  # noqa: E731
    t2h, t2l = split_bf16(f32(t2))
    vh, vl = split_bf16(f32(ovvv))
    oh, ol = split_bf16(f32(ooov))
    terms = [(vh, oh, t2h), (vh, oh, t2l), (vl, ol, t2h)]
    return energy_literal_vectorized(
        eps_occ, eps_vir, f32(t1).astype(np.float64), f32(t2).astype(np.float64),
        f32(ovvv).astype(np.float64), f32(ooov).astype(np.float64),
        f32(ovov).astype(np.float64), return_parts=return_parts, x_terms=terms)
