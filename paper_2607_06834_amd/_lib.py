"""ctypes declarations of the libptafs C ABI (include/ptafs.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (load torch's HIP runtime before libptafs shares it)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptafs.so")

c_double_p = C.POINTER(C.c_double)
c_int64_p = C.POINTER(C.c_int64)
c_int32_p = C.POINTER(C.c_int32)

PTAFS_ST = {0: "ok", 1: "outside prior", 2: "phi not positive definite",
            3: "CW coalescence", 4: "non-finite"}
MAX_PSR = 128
MAX_HARM = 30


class DatasetDesc(C.Structure):
    _fields_ = [
        ("n_psr", C.c_int32),
        ("toa_offsets", c_int64_p),
        ("t", c_double_p),
        ("dt", c_double_p),
        ("sigma", c_double_p),
        ("nu", c_double_p),
        ("backend", c_int32_p),
        ("n_backend", C.c_int32),
        ("efac", c_double_p),
        ("equad", c_double_p),
        ("psr_pos", c_double_p),
        ("tspan", C.c_double),
        ("nf_rn", C.c_int32),
        ("nf_gw", C.c_int32),
        ("nf_dm", C.c_int32),
        ("dm_scale", C.c_double),
        ("sigma_b", C.c_double),
        ("has_cw", C.c_int32),
        ("prior_lo", c_double_p),
        ("prior_hi", c_double_p),
    ]


class StdDesc(C.Structure):
    _fields_ = [
        ("n_psr", C.c_int32),
        ("toa_offsets", c_int64_p),
        ("t", c_double_p),
        ("dt", c_double_p),
        ("sigma", c_double_p),
        ("nu", c_double_p),
        ("backend", c_int32_p),
        ("n_backend", C.c_int32),
        ("efac", c_double_p),
        ("equad", c_double_p),
        ("psr_pos", c_double_p),
        ("tspan", C.c_double),
        ("nf_rn", C.c_int32),
        ("nf_gw", C.c_int32),
        ("nf_dm", C.c_int32),
        ("dm_scale", C.c_double),
        ("n_tm", C.c_int32),
        ("tm", c_double_p),
        ("spectrum", C.c_int32),
        ("prior_lo", c_double_p),
        ("prior_hi", c_double_p),
        ("has_cw", C.c_int32),
        ("cw_nf", C.c_int32),
        ("cw_tspan", C.c_double),
        ("split", C.c_int32),
    ]


class StdLayoutInfo(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "d", "n_theta", "off_gw", "off_rn", "off_dm", "off_z", "n_psr", "n_toa", "k_coef", "k_dm", "p")] + [
        ("dataset_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t), ("hmc_bytes", C.c_size_t),
        ("off_cw", C.c_int64),
        ("pz", C.c_int64)]


class LayoutInfo(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "d", "n_theta", "off_gw", "off_rn", "off_dm", "off_cw", "off_u", "off_z", "off_zdm",
        "n_psr", "n_toa", "k_coef", "k_dm")] + [
        ("dataset_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
        ("hmc_bytes", C.c_size_t)]


EXPORTS = (
    "ptafs_dataset_create", "ptafs_dataset_destroy", "ptafs_layout", "ptafs_estimate",
    "ptafs_reserve",
    "ptafs_logp_grad", "ptafs_logp_grad_plain", "ptafs_logp_grad_noalloc",
    "ptafs_set_tuning", "ptafs_get_tuning",
    "ptafs_hmc_run", "ptafs_profile_stages", "ptafs_strerror",
    "ptafs_std_create", "ptafs_std_destroy", "ptafs_std_layout", "ptafs_std_logp_grad",
    "ptafs_std_coefficients", "ptafs_std_hmc_run", "ptafs_std_precompute", "ptafs_std_precompute_cw",
    "ptafs_std_profile_stages",
)

_lib = None


def load():
    """Load libptafs.so (built by ``paper_2607_06834_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libptafs.so not built: {LIB_PATH} missing "
                           "(run __graft_entry__.build() or paper_2607_06834_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.ptafs_dataset_create.argtypes = [C.POINTER(DatasetDesc), vp, C.POINTER(vp)]
    lib.ptafs_dataset_create.restype = C.c_int
    lib.ptafs_dataset_destroy.argtypes = [vp]
    lib.ptafs_dataset_destroy.restype = None
    lib.ptafs_layout.argtypes = [vp, C.c_int32, C.POINTER(LayoutInfo)]
    lib.ptafs_layout.restype = C.c_int
    lib.ptafs_estimate.argtypes = [C.POINTER(DatasetDesc), C.c_int32, C.POINTER(LayoutInfo)]
    lib.ptafs_estimate.restype = C.c_int
    lib.ptafs_reserve.argtypes = [vp, C.c_int32]
    lib.ptafs_reserve.restype = C.c_int
    for name in ("ptafs_logp_grad", "ptafs_logp_grad_plain", "ptafs_logp_grad_noalloc"):
        f = getattr(lib, name)
        f.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
        f.restype = C.c_int
    lib.ptafs_set_tuning.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    lib.ptafs_set_tuning.restype = C.c_int
    lib.ptafs_get_tuning.argtypes = [vp, c_int32_p, c_int32_p, c_int32_p]
    lib.ptafs_get_tuning.restype = C.c_int
    lib.ptafs_hmc_run.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, vp,
                                  C.c_uint64, C.c_uint64, vp, vp, vp, vp, vp, vp, C.c_int32, vp]
    lib.ptafs_hmc_run.restype = C.c_int
    lib.ptafs_profile_stages.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.c_int32, C.c_int32,
                                         c_double_p, vp]
    lib.ptafs_profile_stages.restype = C.c_int
    lib.ptafs_std_create.argtypes = [C.POINTER(StdDesc), vp, C.POINTER(vp)]
    lib.ptafs_std_create.restype = C.c_int
    lib.ptafs_std_destroy.argtypes = [vp]
    lib.ptafs_std_destroy.restype = None
    lib.ptafs_std_precompute.argtypes = [C.POINTER(StdDesc), C.c_int32, c_double_p, c_double_p, c_double_p]
    lib.ptafs_std_precompute.restype = C.c_int
    lib.ptafs_std_precompute_cw.argtypes = [C.POINTER(StdDesc), C.c_int32, c_double_p, c_double_p, c_double_p]
    lib.ptafs_std_precompute_cw.restype = C.c_int
    lib.ptafs_std_layout.argtypes = [vp, C.c_int32, C.POINTER(StdLayoutInfo)]
    lib.ptafs_std_layout.restype = C.c_int
    lib.ptafs_std_logp_grad.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp]
    lib.ptafs_std_logp_grad.restype = C.c_int
    lib.ptafs_std_profile_stages.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, C.c_int32, c_double_p, vp]
    lib.ptafs_std_profile_stages.restype = C.c_int
    lib.ptafs_std_coefficients.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    lib.ptafs_std_coefficients.restype = C.c_int
    lib.ptafs_std_hmc_run.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, vp, C.c_uint64,
                                      C.c_uint64, vp, vp, vp, vp, vp, vp, vp, C.c_int32, vp]
    lib.ptafs_std_hmc_run.restype = C.c_int
    lib.ptafs_strerror.argtypes = [C.c_int]
    lib.ptafs_strerror.restype = C.c_char_p
    _lib = lib
    return lib


def check(rc, what):
    if rc != 0:
        msg = load().ptafs_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} ({rc})")
