"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and every argument error is reported by the host checks
(no HIP call is made on these paths, so fake device pointers are never read).
"""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2412_18553_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sie_triples.h")

FAKE = 0x100000          # 1 MiB: non-NULL, aligned, never dereferenced


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sie_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def frag(o=4, v=10, eps_occ=None, eps_vir=None, keep=None, **ptrs):
    eo = np.linspace(-1.0, -0.5, o) if eps_occ is None else np.asarray(eps_occ, np.float64)
    ev = np.linspace(0.2, 1.0, v) if eps_vir is None else np.asarray(eps_vir, np.float64)
    if keep is not None:
        keep.extend([eo, ev])
    p = dict(t1=FAKE, t2=FAKE, ovvv=FAKE, ooov=FAKE, ovov=FAKE, frag_proj=None)
    p.update(ptrs)
    return _lib.SieFragment(o, v, eo.ctypes.data, ev.ctypes.data, p["t1"], p["t2"],
                            p["ovvv"], p["ooov"], p["ovov"], p["frag_proj"])


def test_every_declared_symbol_exported(lib):
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_counts(lib):
    assert lib.sie_abi_version() == 2
    assert lib.sie_occupied_triples(24) == 2600
    assert lib.sie_occupied_triples(1) == 1


def energy(lib, f, prec=_lib.SIE_FP64, e_out=FAKE, e_tri=None, ws=FAKE, ws_bytes=1 << 30):
    return lib.sie_triples_energy(ctypes.byref(f) if f is not None else None, prec, e_out,
                                  e_tri, ws, ws_bytes, None)


def test_valid_workspace_query(lib):
    keep = []
    f = frag(keep=keep)
    n = lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0)
    assert n >= 10 ** 3 * 8
    # a cap forces fewer units per launch but never below one unit's cubes
    # (8^3-blocked: a 10-virtual cube pads to 16^3 elements, 32 KiB in float64)
    small = lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 200000)
    assert 0 < small <= 200000
    assert small < n
    assert lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 100) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(o=0), _lib.SIE_ERR_INVALID_ARG),
    (dict(v=0), _lib.SIE_ERR_INVALID_ARG),
    (dict(o=300), _lib.SIE_ERR_INVALID_ARG),
    (dict(t2=None), _lib.SIE_ERR_INVALID_ARG),
    (dict(ovvv=FAKE + 4), _lib.SIE_ERR_INVALID_ARG),            # misaligned float64
    (dict(eps_occ=[-1.0, 0.5], eps_vir=[0.4, 1.0], o=2, v=2), _lib.SIE_ERR_INVALID_ARG),
    (dict(eps_occ=[-1.0, float("nan")], o=2), _lib.SIE_ERR_NONFINITE),
    (dict(eps_vir=[0.4, float("inf")], v=2), _lib.SIE_ERR_NONFINITE),
    (dict(o=100, v=700), _lib.SIE_ERR_UNSUPPORTED),             # float64 extent > 2^32 bytes
])
def test_argument_errors(lib, kw, code):
    keep = []
    o = kw.pop("o", 4)
    v = kw.pop("v", 10)
    eo = kw.pop("eps_occ", None)
    ev = kw.pop("eps_vir", None)
    f = frag(max(o, 1) if o > 0 else o, v, eps_occ=eo if eo is not None else
             (np.linspace(-1.0, -0.5, max(o, 1)) if o <= 256 else np.linspace(-1, -0.5, o)),
             eps_vir=ev, keep=keep, **kw)
    assert energy(lib, f) == code
    assert len(_lib.last_error()) > 0


def test_null_descriptor_and_outputs(lib):
    assert energy(lib, None) == _lib.SIE_ERR_INVALID_ARG
    keep = []
    f = frag(keep=keep)
    assert energy(lib, f, e_out=None) == _lib.SIE_ERR_INVALID_ARG
    assert energy(lib, f, e_out=FAKE + 4) == _lib.SIE_ERR_INVALID_ARG
    assert energy(lib, f, prec=7) == _lib.SIE_ERR_INVALID_ARG


def test_workspace_errors(lib):
    keep = []
    f = frag(keep=keep)
    assert energy(lib, f, ws=None) == _lib.SIE_ERR_WORKSPACE
    assert energy(lib, f, ws=FAKE + 8) == _lib.SIE_ERR_WORKSPACE
    assert energy(lib, f, ws_bytes=64) == _lib.SIE_ERR_WORKSPACE


def test_split_precision_checks(lib):
    keep = []
    f = frag(keep=keep, ovvv=FAKE + 4)            # float32 needs 4-byte alignment only
    assert lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_SPLIT_BF16, 0) > 0
    f = frag(keep=keep, ovvv=FAKE + 2)
    assert energy(lib, f, prec=_lib.SIE_SPLIT_BF16) == _lib.SIE_ERR_INVALID_ARG


def test_profile_collect_empty(lib):
    header = open(HEADER).read()
    n = int(re.search(r"#define SIE_PROF_CLASSES (\d+)", header).group(1))
    assert n == len(_lib.PROF_CLASSES)
    lib.sie_profile_enable(1)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    assert lib.sie_profile_collect(ms, cnt) == _lib.SIE_OK
    assert list(cnt) == [0] * n
    lib.sie_profile_enable(0)
    assert lib.sie_profile_collect(None, None) == _lib.SIE_ERR_INVALID_ARG


def test_python_binding_rejects_bad_shapes():
    torch = pytest.importorskip("torch")
    import paper_2412_18553_amd as sie
    with pytest.raises(TypeError):
        sie.Fragment(np.zeros(2), np.ones(3), torch.zeros(2, 3, dtype=torch.float64),
                     None, None, None, None)


def backward(lib, f, grads, prec=_lib.SIE_FP64, ws=FAKE, ws_bytes=1 << 30, grad_e=None):
    return lib.sie_triples_backward(ctypes.byref(f), 1, prec, grad_e, grads, None, ws, ws_bytes,
                                    None)


def test_backward_workspace_and_errors(lib):
    keep = []
    f = frag(keep=keep)
    fwd = lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0)
    bwd = lib.sie_triples_backward_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0)
    assert bwd > fwd > 0
    g = _lib.SieFragmentGrad(FAKE, FAKE, FAKE, FAKE, FAKE)
    assert lib.sie_triples_backward(ctypes.byref(f), 1, _lib.SIE_FP64, None, None, None, FAKE,
                                    1 << 30, None) == _lib.SIE_ERR_INVALID_ARG
    assert backward(lib, f, ctypes.byref(_lib.SieFragmentGrad(FAKE, FAKE + 4, None, None, None))
                    ) == _lib.SIE_ERR_INVALID_ARG
    assert backward(lib, f, ctypes.byref(g), grad_e=FAKE + 4) == _lib.SIE_ERR_INVALID_ARG
    assert backward(lib, f, ctypes.byref(g), ws=None) == _lib.SIE_ERR_WORKSPACE
    assert backward(lib, f, ctypes.byref(g), ws_bytes=4096) == _lib.SIE_ERR_WORKSPACE
    fp = frag(keep=keep, frag_proj=FAKE)
    assert backward(lib, fp, ctypes.byref(g)) == _lib.SIE_ERR_UNSUPPORTED
    assert len(_lib.last_error()) > 0


def test_tile_table(lib):
    n = lib.sie_tile_variants()
    assert n >= 2
    shape = (ctypes.c_int32 * 8)()
    for v in range(n):
        assert lib.sie_tile_variant_shape(v, shape) == _lib.SIE_OK
        assert all(x >= 1 for x in shape)
        assert shape[6] in (2, 3) and shape[7] in (2, 4)
    assert lib.sie_tile_variant_shape(n, shape) == _lib.SIE_ERR_INVALID_ARG
    arr = lambda *x: (ctypes.c_int32 * len(x))(*x)  # noqa: E731
    assert lib.sie_set_tile_table(2, arr(100, 400), arr(1, 0)) == _lib.SIE_OK
    assert lib.sie_set_tile_table(2, arr(400, 100), arr(1, 0)) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_set_tile_table(1, arr(100), arr(n)) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_set_tile_table(1, None, None) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_set_tile_table(0, None, None) == _lib.SIE_OK
    assert lib.sie_tile_variant_of(0) == -1
    assert lib.sie_set_tile_table(2, arr(100, 400), arr(1, 2)) == _lib.SIE_OK
    assert [lib.sie_tile_variant_of(v) for v in (1, 100, 101, 400, 401)] == [1, 1, 2, 2, 0]
    assert lib.sie_set_tile_table(0, None, None) == _lib.SIE_OK
    # split build shapes: automatic choice, forcing and range checks
    m = int(re.search(r"#define SIE_SPLIT_SHAPES (\d+)", open(HEADER).read()).group(1))
    assert lib.sie_split_shape_of(0) == -1
    assert lib.sie_split_shape_of(320) == 5            # 160 x 160 tiles cover 320 exactly
    assert lib.sie_split_shape_of(160) == 5
    assert lib.sie_split_shape_of(200) == 2            # 112 x 256: least padding at 200
    assert lib.sie_split_shape_of(64) == 0
    assert lib.sie_set_split_shape(m) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_set_split_shape(-2) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_set_split_shape(3) == _lib.SIE_OK
    assert lib.sie_split_shape_of(320) == 3
    assert lib.sie_set_split_shape(-1) == _lib.SIE_OK
    assert lib.sie_split_shape_of(320) == 5
    # the work-group count of a fragment depends on its variant only through sizing
    keep = []
    f = frag(keep=keep)
    assert lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0) > 0


def test_static_entry_point_rejects_before_any_hip_call(lib):
    """The allocation-free entry point checks its arguments and the fit of the
    fragment's minimum workspace in the static scratch on the host, before it
    looks up the scratch on a device."""
    keep = []
    f = frag(keep=keep)
    static = lambda fr, prec=_lib.SIE_FP64, e_out=FAKE: lib.sie_triples_energy_static(  # noqa: E731
        ctypes.byref(fr) if fr is not None else None, prec, e_out, None, None)
    assert static(None) == _lib.SIE_ERR_INVALID_ARG
    assert static(f, e_out=None) == _lib.SIE_ERR_INVALID_ARG
    assert static(f, e_out=FAKE + 4) == _lib.SIE_ERR_INVALID_ARG
    assert static(frag(keep=keep, frag_proj=FAKE)) == _lib.SIE_ERR_UNSUPPORTED
    # 32 / 320 split needs its bf16 copies (~0.4 GB) in the workspace: too big
    big = frag(o=32, v=320, keep=keep)
    assert static(big, prec=_lib.SIE_SPLIT_BF16) == _lib.SIE_ERR_WORKSPACE
    assert "static scratch" in _lib.last_error()
    # 24 / 400 float64: one unit's three cubes alone exceed 256 MiB
    assert static(frag(o=24, v=400, keep=keep)) == _lib.SIE_ERR_WORKSPACE
    assert _lib.SIE_STATIC_SCRATCH_BYTES == 256 * 1024 * 1024


def test_mp2_argument_errors(lib):
    """sie_mp2 checks everything on the host before any HIP call."""
    eo = np.linspace(-1.0, -0.5, 3)
    ev = np.linspace(0.2, 1.0, 5)
    keep = [eo, ev]

    def desc(o=3, v=5, naux=4, e_o=eo, e_v=ev, l=FAKE):
        keep.extend([e_o, e_v])
        return _lib.SieMp2Input(o, v, naux, e_o.ctypes.data if e_o is not None else None,
                                e_v.ctypes.data if e_v is not None else None, l)

    call = lambda d, e_out=FAKE, ws=FAKE, ws_bytes=1 << 30: lib.sie_mp2(  # noqa: E731
        ctypes.byref(d) if d is not None else None, e_out, None, None, None, ws, ws_bytes, None)
    assert call(None) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(o=0)) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(naux=0)) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(l=None)) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(l=FAKE + 4)) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(e_o=np.array([-1.0, 0.5, 0.1]), e_v=ev)) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(e_o=np.array([-1.0, np.nan, -0.5]))) == _lib.SIE_ERR_NONFINITE
    assert call(desc(), e_out=None) == _lib.SIE_ERR_INVALID_ARG
    assert call(desc(), ws=None) == _lib.SIE_ERR_WORKSPACE
    assert call(desc(), ws_bytes=16) == _lib.SIE_ERR_WORKSPACE
    assert lib.sie_mp2_workspace_size(ctypes.byref(desc()), 0) > 0
    assert lib.sie_mp2_workspace_size(ctypes.byref(desc()), 1) > \
        lib.sie_mp2_workspace_size(ctypes.byref(desc()), 0)
    assert lib.sie_mp2_workspace_size(ctypes.byref(desc(o=0)), 0) == 0


def test_projector_argument_checks(lib):
    """frag_proj is a host array the energy entry point reads on the host:
    non-finite entries and a per-triple output request are rejected before
    any HIP call; the batched entry point rejects a projector outright."""
    keep = []
    c = np.eye(4)
    f = frag(keep=keep, frag_proj=c.ctypes.data)
    assert energy(lib, f, e_tri=FAKE) == _lib.SIE_ERR_UNSUPPORTED
    bad = np.eye(4)
    bad[1, 2] = np.nan
    fb = frag(keep=keep, frag_proj=bad.ctypes.data)
    assert energy(lib, fb) == _lib.SIE_ERR_NONFINITE
    assert lib.sie_triples_energy_batched(ctypes.byref(f), 1, _lib.SIE_FP64, FAKE, None, FAKE,
                                          1 << 30, None) == _lib.SIE_ERR_UNSUPPORTED
    n = lib.sie_triples_projector_workspace_size(ctypes.byref(f), _lib.SIE_FP64, 0)
    assert n > 0
    assert lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0) == n
    assert lib.sie_triples_projector_matrix(ctypes.byref(f), _lib.SIE_FP64, None, FAKE, n,
                                            None) == _lib.SIE_ERR_INVALID_ARG
    assert lib.sie_triples_projector_matrix(ctypes.byref(f), _lib.SIE_FP64, FAKE, FAKE, 64,
                                            None) == _lib.SIE_ERR_WORKSPACE
    keep.extend([c, bad])


def test_df_argument_checks(lib):
    """The density-fitting entry point checks its descriptor, the formed
    fragment (orbital energies, amplitude pointers) and the workspace on the
    host before any HIP call; its workspace is the formed blocks plus the
    energy's workspace for them."""
    o, v, naux = 4, 10, 12
    eo = np.linspace(-1.0, -0.5, o)
    ev = np.linspace(0.2, 1.0, v)

    def df(**kw):
        p = dict(n_occ=o, n_vir=v, n_aux=naux, t1=FAKE, t2=FAKE, b=FAKE, eo=eo, ev=ev)
        p.update(kw)
        return _lib.SieFragmentDf(p["n_occ"], p["n_vir"], p["n_aux"], p["eo"].ctypes.data,
                                  p["ev"].ctypes.data, p["t1"], p["t2"], p["b"])

    def size(d, prec=_lib.SIE_FP64, cap=0):
        return lib.sie_triples_df_workspace_size(ctypes.byref(d) if d is not None else None,
                                                 prec, cap)

    def run(d, prec=_lib.SIE_FP64, e_out=FAKE, ws=FAKE, ws_bytes=1 << 30):
        return lib.sie_triples_energy_df(ctypes.byref(d) if d is not None else None, prec,
                                         e_out, None, ws, ws_bytes, None)

    good = df()
    n64, n32 = size(good), size(good, _lib.SIE_SPLIT_BF16)
    # float64: formed ovvv, ooov, ovov (8 bytes) ahead of the energy workspace
    f = frag(o, v, keep=[])
    e64 = lib.sie_triples_workspace_size(ctypes.byref(f), 1, _lib.SIE_FP64, 0)
    formed = sum((8 * x + 255) // 256 * 256 for x in (o * v ** 3, o ** 3 * v, o * o * v * v))
    assert n64 == formed + e64
    assert 0 < n32 < n64 + 8 * o * v ** 3
    assert size(None) == 0
    assert size(df(n_aux=0)) == 0
    assert size(df(b=0)) == 0
    assert size(df(b=FAKE + 4)) == 0
    assert size(df(t2=0)) == 0
    assert size(good, cap=1024) == 0
    assert run(None) == _lib.SIE_ERR_INVALID_ARG
    assert run(df(n_aux=0)) == _lib.SIE_ERR_INVALID_ARG
    assert run(df(b=0)) == _lib.SIE_ERR_INVALID_ARG
    assert run(good, e_out=None) == _lib.SIE_ERR_INVALID_ARG
    assert run(good, ws=FAKE + 8) == _lib.SIE_ERR_WORKSPACE
    assert run(good, ws_bytes=4096) == _lib.SIE_ERR_WORKSPACE
    assert run(good, 7) == _lib.SIE_ERR_INVALID_ARG
    bad_eo = np.array([-1.0, -0.5, 0.5, -0.2])
    assert run(df(eo=bad_eo)) == _lib.SIE_ERR_INVALID_ARG
    nan_ev = ev.copy()
    nan_ev[3] = np.nan
    assert run(df(ev=nan_ev)) == _lib.SIE_ERR_NONFINITE
