"""MI355X (gfx950) per-fragment (T) energy: Python binding of the C ABI.

Argument marshalling only: every arithmetic step runs in the HIP kernels of
libsie_triples.so (see include/sie_triples.h).  PyTorch supplies device
memory and the current stream.  The library must be built
(`python -m paper_2412_18553_amd.build`); there is no fallback.

Inputs (row-major, contiguous):
  eps_occ [n_occ], eps_vir [n_vir]                     host or device, float64
  t1 [o][v], t2 [o][o][v][v], ovvv [o][v][v][v],
  ooov [o][o][o][v] = (jl|ia), ovov [o][v][o][v]       CUDA tensors
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SieError, SieFragment  # noqa: F401

PRECISIONS = {"fp64": _lib.SIE_FP64, "split_bf16": _lib.SIE_SPLIT_BF16}
INPUT_DTYPE = {"fp64": torch.float64, "split_bf16": torch.float32}


def occupied_triples(n_occ: int) -> int:
    return n_occ * (n_occ + 1) * (n_occ + 2) // 6


def _host_f64(x, name):
    if isinstance(x, torch.Tensor):
        x = x.detach().to("cpu")
        x = x.numpy()
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if arr.ndim != 1:
        raise ValueError(f"{name} must be 1-d")
    return arr


def _device_input(x, name, shape, dtype):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name}: dtype {x.dtype}, expected {dtype}")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(x.shape)}, expected {tuple(shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


class Fragment:
    """Validated inputs of one fragment plus the C descriptor pointing at them.

    Keeps references to every buffer the descriptor points at."""

    def __init__(self, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision="fp64"):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        self.precision = precision
        self.eps_occ = _host_f64(eps_occ, "eps_occ")
        self.eps_vir = _host_f64(eps_vir, "eps_vir")
        o, v = self.eps_occ.shape[0], self.eps_vir.shape[0]
        dt = INPUT_DTYPE[precision]
        self.t1 = _device_input(t1, "t1", (o, v), dt)
        self.device = self.t1.device
        self.t2 = _device_input(t2, "t2", (o, o, v, v), dt)
        self.ovvv = _device_input(ovvv, "ovvv", (o, v, v, v), dt)
        self.ooov = _device_input(ooov, "ooov", (o, o, o, v), dt)
        self.ovov = _device_input(ovov, "ovov", (o, v, o, v), dt)
        for name in ("t2", "ovvv", "ooov", "ovov"):
            if getattr(self, name).device != self.device:
                raise ValueError("all device inputs must be on the same GPU")
        self.n_occ, self.n_vir = o, v
        self.desc = SieFragment(
            o, v, self.eps_occ.ctypes.data, self.eps_vir.ctypes.data,
            self.t1.data_ptr(), self.t2.data_ptr(), self.ovvv.data_ptr(),
            self.ooov.data_ptr(), self.ovov.data_ptr(), None)

    @property
    def n_triples(self) -> int:
        return occupied_triples(self.n_occ)


def workspace_size(frag: Fragment, max_bytes: int = 0) -> int:
    lib = _lib.load()
    n = lib.sie_triples_workspace_size(ctypes.byref(frag.desc), 1,
                                       PRECISIONS[frag.precision], max_bytes)
    if n == 0:
        raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
    return int(n)


def energy(frag: Fragment, *, workspace: torch.Tensor | None = None,
           out: torch.Tensor | None = None, triples: torch.Tensor | None = None,
           max_workspace_bytes: int = 0) -> torch.Tensor:
    """Enqueue E_x for `frag` on the current stream; returns a 1-element
    float64 device tensor (no synchronisation).  `triples`, if given, receives
    the per-occupied-triple contributions (float64 [n_triples])."""
    lib = _lib.load()
    if workspace is None:
        workspace = torch.empty(workspace_size(frag, max_workspace_bytes),
                                dtype=torch.uint8, device=frag.device)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=frag.device)
    if triples is not None and (triples.dtype != torch.float64 or
                                triples.numel() != frag.n_triples or
                                not triples.is_contiguous() or not triples.is_cuda):
        raise ValueError("triples must be a contiguous float64 CUDA tensor of n_triples entries")
    stream = torch.cuda.current_stream(frag.device).cuda_stream
    st = lib.sie_triples_energy(ctypes.byref(frag.desc), PRECISIONS[frag.precision],
                                out.data_ptr(),
                                None if triples is None else triples.data_ptr(),
                                workspace.data_ptr(), workspace.numel(), stream)
    _lib.check(st)
    return out


def triples_energy(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, *, precision="fp64",
                   return_triples=False):
    """E_x of one fragment as a 0-d float64 device tensor (and, with
    return_triples, the per-occupied-triple contributions)."""
    frag = Fragment(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision)
    tri = (torch.empty(frag.n_triples, dtype=torch.float64, device=frag.device)
           if return_triples else None)
    e = energy(frag, triples=tri)
    return (e[0], tri) if return_triples else e[0]


def profile_enable(on: bool = True) -> None:
    """Time every library kernel launch on this thread with HIP events."""
    _lib.load().sie_profile_enable(1 if on else 0)


def profile_collect() -> dict:
    """Wait for the recorded launches; return {class: (total_ms, launches)}."""
    lib = _lib.load()
    n = len(_lib.PROF_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _lib.check(lib.sie_profile_collect(ms, cnt))
    return {name: (ms[c], cnt[c]) for c, name in enumerate(_lib.PROF_CLASSES)}
