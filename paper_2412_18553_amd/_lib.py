"""ctypes view of the C ABI in include/sie_triples.h.

Loads the in-tree libsie_triples.so; raises if it has not been built (there is
no fallback path).
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsie_triples.so")

SIE_OK = 0
SIE_ERR_INVALID_ARG = 1
SIE_ERR_UNSUPPORTED = 2
SIE_ERR_WORKSPACE = 3
SIE_ERR_NONFINITE = 4
SIE_ERR_HIP = 5

SIE_FP64 = 0
SIE_SPLIT_BF16 = 1

SIE_STATIC_SCRATCH_BYTES = 256 * 1024 * 1024

STATUS_NAMES = {0: "SIE_OK", 1: "SIE_ERR_INVALID_ARG", 2: "SIE_ERR_UNSUPPORTED",
                3: "SIE_ERR_WORKSPACE", 4: "SIE_ERR_NONFINITE", 5: "SIE_ERR_HIP"}

# every symbol include/sie_triples.h declares
EXPORTED = ["sie_abi_version", "sie_last_error", "sie_occupied_triples",
            "sie_triples_workspace_size", "sie_triples_energy", "sie_triples_energy_batched",
            "sie_triples_energy_static",
            "sie_triples_backward_workspace_size", "sie_triples_backward",
            "sie_tile_variants", "sie_tile_variant_shape", "sie_tile_variant_of",
            "sie_set_tile_table", "sie_split_shape_of", "sie_set_split_shape",
            "sie_set_split_table",
            "sie_profile_enable", "sie_profile_collect", "sie_set_check_finite",
            "sie_mp2_workspace_size", "sie_mp2",
            "sie_triples_projector_workspace_size", "sie_triples_projector_matrix",
            "sie_triples_df_workspace_size", "sie_triples_energy_df"]
PROF_CLASSES = ("w_build", "epilogue", "reduce", "split", "grad")


class SieFragment(ctypes.Structure):
    _fields_ = [
        ("n_occ", ctypes.c_int32),
        ("n_vir", ctypes.c_int32),
        ("eps_occ", ctypes.c_void_p),
        ("eps_vir", ctypes.c_void_p),
        ("t1", ctypes.c_void_p),
        ("t2", ctypes.c_void_p),
        ("ovvv", ctypes.c_void_p),
        ("ooov", ctypes.c_void_p),
        ("ovov", ctypes.c_void_p),
        ("frag_proj", ctypes.c_void_p),
    ]


class SieFragmentGrad(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p)
                for name in ("t1", "t2", "ovvv", "ooov", "ovov", "eps_occ", "eps_vir")]


class SieMp2Input(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int32), ("n_vir", ctypes.c_int32), ("n_aux", ctypes.c_int32),
                ("eps_occ", ctypes.c_void_p), ("eps_vir", ctypes.c_void_p),
                ("l_ov", ctypes.c_void_p)]


class SieFragmentDf(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int32), ("n_vir", ctypes.c_int32), ("n_aux", ctypes.c_int32),
                ("eps_occ", ctypes.c_void_p), ("eps_vir", ctypes.c_void_p),
                ("t1", ctypes.c_void_p), ("t2", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class SieError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2412_18553_amd.build` "
            "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.sie_abi_version.restype = ctypes.c_int
    lib.sie_abi_version.argtypes = []
    lib.sie_last_error.restype = ctypes.c_char_p
    lib.sie_last_error.argtypes = []
    lib.sie_occupied_triples.restype = ctypes.c_int64
    lib.sie_occupied_triples.argtypes = [ctypes.c_int32]
    lib.sie_triples_workspace_size.restype = ctypes.c_size_t
    lib.sie_triples_workspace_size.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int32,
                                               ctypes.c_int, ctypes.c_size_t]
    lib.sie_triples_energy.restype = ctypes.c_int
    lib.sie_triples_energy.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]
    lib.sie_triples_energy_static.restype = ctypes.c_int
    lib.sie_triples_energy_static.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.sie_triples_energy_batched.restype = ctypes.c_int
    lib.sie_triples_energy_batched.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int32,
                                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.sie_triples_backward_workspace_size.restype = ctypes.c_size_t
    lib.sie_triples_backward_workspace_size.argtypes = [ctypes.POINTER(SieFragment),
                                                        ctypes.c_int32, ctypes.c_int,
                                                        ctypes.c_size_t]
    lib.sie_triples_backward.restype = ctypes.c_int
    lib.sie_triples_backward.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int32,
                                         ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(SieFragmentGrad), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.sie_tile_variants.restype = ctypes.c_int32
    lib.sie_tile_variants.argtypes = []
    lib.sie_tile_variant_shape.restype = ctypes.c_int
    lib.sie_tile_variant_shape.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.sie_tile_variant_of.restype = ctypes.c_int32
    lib.sie_tile_variant_of.argtypes = [ctypes.c_int32]
    lib.sie_set_tile_table.restype = ctypes.c_int
    lib.sie_set_tile_table.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.sie_split_shape_of.restype = ctypes.c_int32
    lib.sie_split_shape_of.argtypes = [ctypes.c_int32]
    lib.sie_set_split_shape.restype = ctypes.c_int
    lib.sie_set_split_shape.argtypes = [ctypes.c_int32]
    lib.sie_set_split_table.restype = ctypes.c_int
    lib.sie_set_split_table.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.sie_profile_enable.restype = None
    lib.sie_profile_enable.argtypes = [ctypes.c_int]
    lib.sie_set_check_finite.restype = None
    lib.sie_set_check_finite.argtypes = [ctypes.c_int]
    lib.sie_profile_collect.restype = ctypes.c_int
    lib.sie_profile_collect.argtypes = [ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.sie_triples_projector_workspace_size.restype = ctypes.c_size_t
    lib.sie_triples_projector_workspace_size.argtypes = [ctypes.POINTER(SieFragment),
                                                         ctypes.c_int, ctypes.c_size_t]
    lib.sie_triples_projector_matrix.restype = ctypes.c_int
    lib.sie_triples_projector_matrix.argtypes = [ctypes.POINTER(SieFragment), ctypes.c_int,
                                                 ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]
    lib.sie_triples_df_workspace_size.restype = ctypes.c_size_t
    lib.sie_triples_df_workspace_size.argtypes = [ctypes.POINTER(SieFragmentDf), ctypes.c_int,
                                                  ctypes.c_size_t]
    lib.sie_triples_energy_df.restype = ctypes.c_int
    lib.sie_triples_energy_df.argtypes = [ctypes.POINTER(SieFragmentDf), ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]
    lib.sie_mp2_workspace_size.restype = ctypes.c_size_t
    lib.sie_mp2_workspace_size.argtypes = [ctypes.POINTER(SieMp2Input), ctypes.c_int32]
    lib.sie_mp2.restype = ctypes.c_int
    lib.sie_mp2.argtypes = [ctypes.POINTER(SieMp2Input), ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.c_void_p]
    _lib = lib
    return lib


def last_error() -> str:
    return load().sie_last_error().decode()


def check(status: int) -> None:
    if status != SIE_OK:
        raise SieError(status, last_error())
