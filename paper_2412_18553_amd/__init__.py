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
from ._lib import SieError, SieFragment, SieFragmentGrad  # noqa: F401

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

    def __init__(self, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision="fp64",
                 frag_proj=None):
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
        self.frag_proj = None
        if frag_proj is not None:   # host float64 [n_occ][n_occ], C^f of the fragment
            c = frag_proj.detach().to("cpu").numpy() if isinstance(frag_proj, torch.Tensor) \
                else frag_proj
            self.frag_proj = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
            if self.frag_proj.shape != (o, o):
                raise ValueError(f"frag_proj must be [{o}][{o}]")
        self.desc = SieFragment(
            o, v, self.eps_occ.ctypes.data, self.eps_vir.ctypes.data,
            self.t1.data_ptr(), self.t2.data_ptr(), self.ovvv.data_ptr(),
            self.ooov.data_ptr(), self.ovov.data_ptr(),
            None if self.frag_proj is None else self.frag_proj.ctypes.data)

    @property
    def n_triples(self) -> int:
        return occupied_triples(self.n_occ)


def _desc_array(frags):
    frags = [frags] if isinstance(frags, Fragment) else list(frags)
    if not frags:
        raise ValueError("need at least one fragment")
    prec = {f.precision for f in frags}
    if len(prec) != 1:
        raise ValueError("all fragments of one evaluation must share the precision")
    dev = {f.device for f in frags}
    if len(dev) != 1:
        raise ValueError("all fragments of one evaluation must be on one GPU")
    arr = (SieFragment * len(frags))(*[f.desc for f in frags])
    return frags, arr, PRECISIONS[frags[0].precision]


def workspace_size(frags, max_bytes: int = 0) -> int:
    """Workspace bytes for one fragment or a list of fragments (see the C header)."""
    lib = _lib.load()
    frags, arr, prec = _desc_array(frags)
    n = lib.sie_triples_workspace_size(arr, len(frags), prec, max_bytes)
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


def projector_matrix(frag: Fragment, *, out: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None,
                     max_workspace_bytes: int = 0) -> torch.Tensor:
    """M [n_occ][n_occ] (float64, device) with E_x(C) = sum_{ii'} C_ii' M_ii' for
    any fragment projector C (see sie_triples_projector_matrix; tr M = E_x).
    Enqueued on the current stream."""
    lib = _lib.load()
    prec = PRECISIONS[frag.precision]
    if workspace is None:
        n = lib.sie_triples_projector_workspace_size(ctypes.byref(frag.desc), prec,
                                                     max_workspace_bytes)
        if n == 0:
            raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
        workspace = torch.empty(n, dtype=torch.uint8, device=frag.device)
    if out is None:
        out = torch.empty((frag.n_occ, frag.n_occ), dtype=torch.float64, device=frag.device)
    if out.dtype != torch.float64 or out.numel() != frag.n_occ ** 2 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of n_occ^2 entries")
    stream = torch.cuda.current_stream(frag.device).cuda_stream
    st = lib.sie_triples_projector_matrix(ctypes.byref(frag.desc), prec, out.data_ptr(),
                                          workspace.data_ptr(), workspace.numel(), stream)
    _lib.check(st)
    return out


def energy_static(frag: Fragment, *, out: torch.Tensor | None = None,
                  triples: torch.Tensor | None = None) -> torch.Tensor:
    """E_x like `energy`, through the entry point that allocates nothing: the
    library's static device scratch (SIE_STATIC_SCRATCH_BYTES per GPU) serves
    as the workspace.  `out` and `triples`, when given, are written in place,
    so a caller that passes both allocates nothing here either."""
    lib = _lib.load()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=frag.device)
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1:
        raise ValueError("out must be a float64 CUDA tensor")
    if triples is not None and (triples.dtype != torch.float64 or
                                triples.numel() != frag.n_triples or
                                not triples.is_contiguous() or not triples.is_cuda):
        raise ValueError("triples must be a contiguous float64 CUDA tensor of n_triples entries")
    stream = torch.cuda.current_stream(frag.device).cuda_stream
    st = lib.sie_triples_energy_static(ctypes.byref(frag.desc), PRECISIONS[frag.precision],
                                       out.data_ptr(),
                                       None if triples is None else triples.data_ptr(), stream)
    _lib.check(st)
    return out


def energy_batched(frags, *, workspace: torch.Tensor | None = None,
                   out: torch.Tensor | None = None, total: torch.Tensor | None = None,
                   max_workspace_bytes: int = 0):
    """Enqueue E_x for every fragment of `frags` (one evaluation, one work
    list) on the current stream; returns (e_frag [n], e_total [1]) float64
    device tensors."""
    lib = _lib.load()
    frags, arr, prec = _desc_array(frags)
    device = frags[0].device
    if workspace is None:
        workspace = torch.empty(workspace_size(frags, max_workspace_bytes), dtype=torch.uint8,
                                device=device)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty(len(frags), dtype=torch.float64, device=device)
    if total is None:
        total = torch.empty(1, dtype=torch.float64, device=device)
    if out.numel() != len(frags) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor with one entry per fragment")
    stream = torch.cuda.current_stream(device).cuda_stream
    st = lib.sie_triples_energy_batched(arr, len(frags), prec, out.data_ptr(), total.data_ptr(),
                                        workspace.data_ptr(), workspace.numel(), stream)
    _lib.check(st)
    return out, total


GRAD_NAMES = ("t1", "t2", "ovvv", "ooov", "ovov")
# gradients with respect to the orbital energies (device float64 [n_occ], [n_vir])
EPS_GRAD_NAMES = ("eps_occ", "eps_vir")
ALL_GRAD_NAMES = GRAD_NAMES + EPS_GRAD_NAMES


def _grad_shape(f, name):
    if name == "eps_occ":
        return (f.n_occ,)
    if name == "eps_vir":
        return (f.n_vir,)
    return tuple(getattr(f, name).shape)


def backward_workspace_size(frags, max_bytes: int = 0) -> int:
    """Workspace bytes of `backward` for one fragment or a list (see the C header)."""
    lib = _lib.load()
    frags, arr, prec = _desc_array(frags)
    n = lib.sie_triples_backward_workspace_size(arr, len(frags), prec, max_bytes)
    if n == 0:
        raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
    return int(n)


def backward(frags, *, grad_e: torch.Tensor | None = None, grads=None,
             e_frag: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
             max_workspace_bytes: int = 0, want=GRAD_NAMES):
    """Enqueue the gradient of E_x for each fragment on the current stream.

    Returns a list (one dict per fragment) of float64 device tensors
    {name: grad_e[x] * dE_x/d name} for the names in `want` (any of
    ALL_GRAD_NAMES), symmetrized over each input's index-symmetry orbit.
    `grads`, if given, is such a list of preallocated tensors to overwrite.
    `grad_e`: float64 device tensor [n] or None (ones).  `e_frag`: optional
    float64 [n] receiving E_x."""
    lib = _lib.load()
    single = isinstance(frags, Fragment)
    frags, arr, prec = _desc_array(frags)
    device = frags[0].device
    for name in want:
        if name not in ALL_GRAD_NAMES:
            raise ValueError(f"unknown gradient {name!r}")
    if grads is None:
        grads = [{name: torch.empty(_grad_shape(f, name), dtype=torch.float64, device=device)
                  for name in want} for f in frags]
    if len(grads) != len(frags):
        raise ValueError("grads needs one dict per fragment")
    garr = (SieFragmentGrad * len(frags))()
    for x, (f, g) in enumerate(zip(frags, grads)):
        for name in ALL_GRAD_NAMES:
            t = g.get(name)
            if t is None:
                continue
            shape = _grad_shape(f, name)
            if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or
                    tuple(t.shape) != shape or not t.is_contiguous() or t.device != device):
                raise ValueError(f"grads[{x}][{name!r}] must be a contiguous float64 tensor "
                                 f"of shape {shape} on {device}")
            setattr(garr[x], name, t.data_ptr())
    if grad_e is not None:
        if (grad_e.dtype != torch.float64 or grad_e.numel() != len(frags) or
                not grad_e.is_contiguous() or grad_e.device != device):
            raise ValueError("grad_e must be a contiguous float64 tensor with one entry per fragment")
    if e_frag is not None:
        if (e_frag.dtype != torch.float64 or e_frag.numel() != len(frags) or
                not e_frag.is_contiguous() or e_frag.device != device):
            raise ValueError("e_frag must be a contiguous float64 tensor with one entry per fragment")
    if workspace is None:
        workspace = torch.empty(backward_workspace_size(frags, max_workspace_bytes),
                                dtype=torch.uint8, device=device)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    stream = torch.cuda.current_stream(device).cuda_stream
    st = lib.sie_triples_backward(arr, len(frags), prec,
                                  None if grad_e is None else grad_e.data_ptr(), garr,
                                  None if e_frag is None else e_frag.data_ptr(),
                                  workspace.data_ptr(), workspace.numel(), stream)
    _lib.check(st)
    return grads[0] if single else grads


class SieTriples(torch.autograd.Function):
    """E_x as a differentiable function of (eps_occ, eps_vir, t1, t2, ovvv,
    ooov, ovov).

    SieTriples.apply(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov[, precision])
    returns a 0-d float64 tensor; backward calls the library's adjoint and
    returns the symmetrized gradients cast to each input's dtype (and, for
    orbital energies given as tensors, on their device).  precision is "fp64"
    (float64 inputs) or "split_bf16" (float32 inputs)."""

    @staticmethod
    def forward(ctx, eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision="fp64"):
        frag = Fragment(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision)
        ctx.frag = frag
        ctx.eps_like = [x if isinstance(x, torch.Tensor) else None for x in (eps_occ, eps_vir)]
        return energy(frag)[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        frag = ctx.frag
        want = [name for name, need in zip(ALL_GRAD_NAMES,
                                           tuple(ctx.needs_input_grad[2:7]) +
                                           tuple(ctx.needs_input_grad[0:2])) if need]
        if not want:
            return (None,) * 8
        ge = grad_out.detach().reshape(1).to(device=frag.device, dtype=torch.float64).contiguous()
        g = backward(frag, grad_e=ge, want=want)
        eps = tuple(g[name].to(device=like.device, dtype=like.dtype) if name in g else None
                    for name, like in zip(EPS_GRAD_NAMES, ctx.eps_like))
        return eps + tuple(
            g[name].to(getattr(frag, name).dtype) if name in g else None
            for name in GRAD_NAMES) + (None,)


def triples_energy(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, *, precision="fp64",
                   return_triples=False):
    """E_x of one fragment as a 0-d float64 device tensor (and, with
    return_triples, the per-occupied-triple contributions)."""
    frag = Fragment(eps_occ, eps_vir, t1, t2, ovvv, ooov, ovov, precision)
    tri = (torch.empty(frag.n_triples, dtype=torch.float64, device=frag.device)
           if return_triples else None)
    e = energy(frag, triples=tri)
    return (e[0], tri) if return_triples else e[0]


def mp2(eps_occ, eps_vir, l_ov: torch.Tensor, *, want_t2: bool = False,
        want_density: bool = False, workspace: torch.Tensor | None = None):
    """MP2 energy of one cluster from density-fitting factors l_ov [n_occ][n_vir]
    [n_aux] (float64 CUDA tensor), enqueued on the current stream.  Returns
    {"energy": float64 [1]} plus "t2" [o][o][v][v] with want_t2 and
    "gamma_oo" [o][o], "gamma_vv" [v][v] with want_density (device
    tensors, no synchronisation); see sie_mp2 in the C header."""
    lib = _lib.load()
    eo, ev = _host_f64(eps_occ, "eps_occ"), _host_f64(eps_vir, "eps_vir")
    o, v = eo.shape[0], ev.shape[0]
    if (not isinstance(l_ov, torch.Tensor) or not l_ov.is_cuda or l_ov.dtype != torch.float64
            or l_ov.dim() != 3 or tuple(l_ov.shape[:2]) != (o, v) or not l_ov.is_contiguous()):
        raise ValueError("l_ov must be a contiguous float64 CUDA tensor [n_occ][n_vir][n_aux]")
    dev = l_ov.device
    desc = _lib.SieMp2Input(o, v, int(l_ov.shape[2]), eo.ctypes.data, ev.ctypes.data,
                            l_ov.data_ptr())
    out = {"energy": torch.empty(1, dtype=torch.float64, device=dev)}
    if want_t2:
        out["t2"] = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    if want_density:
        out["gamma_oo"] = torch.empty((o, o), dtype=torch.float64, device=dev)
        out["gamma_vv"] = torch.empty((v, v), dtype=torch.float64, device=dev)
    if workspace is None:
        n = lib.sie_mp2_workspace_size(ctypes.byref(desc), 1 if want_density else 0)
        if n == 0:
            raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
        workspace = torch.empty(n, dtype=torch.uint8, device=dev)
    ptr = lambda k: out[k].data_ptr() if k in out else None  # noqa: E731
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = lib.sie_mp2(ctypes.byref(desc), ptr("energy"), ptr("t2"), ptr("gamma_oo"),
                     ptr("gamma_vv"), workspace.data_ptr(), workspace.numel(), stream)
    _lib.check(st)
    return out


def _df_desc(eps_occ, eps_vir, t1, t2, b, precision):
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}")
    eo, ev = _host_f64(eps_occ, "eps_occ"), _host_f64(eps_vir, "eps_vir")
    o, v = eo.shape[0], ev.shape[0]
    dt = torch.float64 if precision == "fp64" else torch.float32
    for name, x, shape in (("t1", t1, (o, v)), ("t2", t2, (o, o, v, v))):
        if (not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != dt
                or tuple(x.shape) != shape or not x.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of shape {shape}")
    n = o + v
    if (not isinstance(b, torch.Tensor) or not b.is_cuda or b.dtype != torch.float64
            or b.dim() != 3 or tuple(b.shape[1:]) != (n, n) or not b.is_contiguous()):
        raise ValueError("b must be a contiguous float64 CUDA tensor [n_aux][n][n]")
    desc = _lib.SieFragmentDf(o, v, int(b.shape[0]), eo.ctypes.data, ev.ctypes.data,
                              t1.data_ptr(), t2.data_ptr(), b.data_ptr())
    return desc, (eo, ev), PRECISIONS[precision]


def df_workspace_size(eps_occ, eps_vir, t1, t2, b, precision: str = "fp64",
                      max_bytes: int = 0) -> int:
    """Workspace bytes of `energy_df` (see sie_triples_df_workspace_size)."""
    lib = _lib.load()
    desc, keep, prec = _df_desc(eps_occ, eps_vir, t1, t2, b, precision)
    n = lib.sie_triples_df_workspace_size(ctypes.byref(desc), prec, max_bytes)
    del keep
    if n == 0:
        raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
    return n


def energy_df(eps_occ, eps_vir, t1: torch.Tensor, t2: torch.Tensor, b: torch.Tensor,
              precision: str = "fp64", *, workspace: torch.Tensor | None = None,
              out: torch.Tensor | None = None, triples: torch.Tensor | None = None,
              max_workspace_bytes: int = 0) -> torch.Tensor:
    """E_x of one fragment from its density-fitting factors b [n_aux][n][n]
    (float64 CUDA tensor, n = n_occ + n_vir, occupied first, symmetric in the
    last two indices) and amplitudes t1, t2 (float64 for "fp64", float32 for
    "split_bf16"); the library forms the integral blocks itself (see
    sie_triples_energy_df).  Enqueued on the current stream; returns a
    1-element float64 device tensor."""
    lib = _lib.load()
    desc, keep, prec = _df_desc(eps_occ, eps_vir, t1, t2, b, precision)
    dev = b.device
    o = desc.n_occ
    if workspace is None:
        nbytes = lib.sie_triples_df_workspace_size(ctypes.byref(desc), prec, max_workspace_bytes)
        if nbytes == 0:
            raise SieError(_lib.SIE_ERR_INVALID_ARG, _lib.last_error())
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=dev)
    if triples is not None and (triples.dtype != torch.float64 or
                                triples.numel() != occupied_triples(o) or
                                not triples.is_contiguous() or not triples.is_cuda):
        raise ValueError("triples must be a contiguous float64 CUDA tensor of n_triples entries")
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = lib.sie_triples_energy_df(ctypes.byref(desc), prec, out.data_ptr(),
                                   None if triples is None else triples.data_ptr(),
                                   workspace.data_ptr(), workspace.numel(), stream)
    del keep
    _lib.check(st)
    return out


def tile_variants():
    """Tile shapes of the float64 build: [(blocks/wave, row tiles, col tiles, WGs/CU,
    wave rows, wave cols, layouts, k-steps per chunk)] (see sie_tile_variant_shape)."""
    lib = _lib.load()
    out = []
    for v in range(lib.sie_tile_variants()):
        shape = (ctypes.c_int32 * 8)()
        _lib.check(lib.sie_tile_variant_shape(v, shape))
        out.append(tuple(shape))
    return out


def tile_variant_of(n_vir: int) -> int:
    """The tile variant the float64 energy of a fragment with n_vir virtuals
    builds with under the installed table."""
    return int(_lib.load().sie_tile_variant_of(int(n_vir)))


def split_shape_of(n_vir: int) -> int:
    """The tile shape the split-precision build of a fragment with n_vir
    virtuals uses (see sie_split_shape_of)."""
    return int(_lib.load().sie_split_shape_of(int(n_vir)))


def set_split_shape(shape: int = -1) -> None:
    """Force split build shape `shape` for all fragments, or restore the
    automatic choice with -1."""
    _lib.check(_lib.load().sie_set_split_shape(int(shape)))


def set_tile_table(table=None) -> None:
    """Install [(n_vir upper bound, variant), ...] (ascending) for the float64
    build, or the built-in tuned table with None."""
    lib = _lib.load()
    table = list(table or [])
    n = len(table)
    nv = (ctypes.c_int32 * max(n, 1))(*[int(b) for b, _ in table])
    var = (ctypes.c_int32 * max(n, 1))(*[int(v) for _, v in table])
    _lib.check(lib.sie_set_tile_table(n, nv, var))


def set_split_table(table=None) -> None:
    """Install [(n_vir upper bound, split shape), ...] (ascending) for the
    split-precision build, or the built-in tuned table with None."""
    lib = _lib.load()
    table = list(table or [])
    n = len(table)
    nv = (ctypes.c_int32 * max(n, 1))(*[int(b) for b, _ in table])
    sh = (ctypes.c_int32 * max(n, 1))(*[int(v) for _, v in table])
    _lib.check(lib.sie_set_split_table(n, nv, sh))


def set_check_finite(on: bool = True) -> None:
    """Scan the device inputs for NaN / infinity before each evaluation
    (SieError SIE_ERR_NONFINITE if found; the call then waits for the scan)."""
    _lib.load().sie_set_check_finite(1 if on else 0)


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
