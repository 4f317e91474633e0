"""ctypes binding of libtn.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module converts
NumPy/torch arguments to pointers and status codes to exceptions.  Loading
fails loudly when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtn.so")

TN_OK, TN_EINVAL, TN_ENOMEM, TN_EHIP, TN_ENUMERIC, TN_ESTATE = 0, -1, -2, -3, -4, -5
TN_FP64, TN_FP32, TN_BF16X3 = 0, 1, 2
_NAMES = {TN_EINVAL: "TN_EINVAL", TN_ENOMEM: "TN_ENOMEM", TN_EHIP: "TN_EHIP",
          TN_ENUMERIC: "TN_ENUMERIC", TN_ESTATE: "TN_ESTATE"}


class TnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class tn_allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("user", C.c_void_p)]


class tn_problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("D_raw", C.c_int32), ("d", C.c_int32),
                ("r", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("iso", C.POINTER(C.c_double)), ("kappa", C.c_double)]


class tn_sweep_opts(C.Structure):
    _fields_ = [("chi_max", C.c_int32), ("sigma_cut", C.c_double), ("tol", C.c_double),
                ("krylov_max", C.c_int32), ("max_matvecs", C.c_int32), ("precision", C.c_int32),
                ("lbo", C.c_int32), ("compute_energy", C.c_int32), ("lbo_matvecs", C.c_int32)]


class tn_sweep_stats(C.Structure):
    _fields_ = [("energy", C.c_double), ("last_eigenvalue", C.c_double),
                ("max_discarded", C.c_double), ("sum_discarded", C.c_double),
                ("lbo_discarded", C.c_double), ("matvecs", C.c_int64),
                ("unconverged_steps", C.c_int32), ("pad_", C.c_int32),
                ("heff_flops", C.c_double), ("env_flops", C.c_double),
                ("t_heff", C.c_double), ("t_lanczos", C.c_double), ("t_svd", C.c_double),
                ("t_env", C.c_double), ("t_lbo", C.c_double), ("t_energy", C.c_double),
                ("t_total", C.c_double), ("svd_flops", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class tn_solve_opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("bulk_precision", C.c_int32), ("max_refine", C.c_int32),
                ("lbo_bulk", C.c_int32), ("lbo_refine", C.c_int32), ("pad_", C.c_int32),
                ("target", C.c_double), ("switch_tol", C.c_double), ("conv_tol", C.c_double),
                ("bulk_tol", C.c_double), ("refine_tol", C.c_double), ("sweep", tn_sweep_opts)]


class tn_plbo_opts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("matvecs", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("mask", C.c_uint32), ("optimizer", C.c_int32)]


class tn_solve_result(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("refine_sweeps", C.c_int32), ("reached", C.c_int32), ("pad_", C.c_int32),
                ("energy", C.c_double), ("seconds", C.c_double), ("t_target", C.c_double),
                ("heff_flops", C.c_double), ("t_heff", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


_lib = None


def lib():
    """Load libtn.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2410_18740_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, szt = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "tn_version": (C.c_char_p, []),
        "tn_ctx_create": (i32, [C.c_int, vp, P(tn_allocator), P(vp)]),
        "tn_ctx_destroy": (None, [vp]),
        "tn_last_error": (C.c_char_p, [vp]),
        "tn_mpo_build": (i32, [vp, P(tn_problem), P(vp)]),
        "tn_mpo_structure": (i32, [vp, P(i32), P(C.c_int8)]),
        "tn_mpo_coefficients": (i32, [vp, P(dbl), P(dbl), P(dbl)]),
        "tn_mpo_isometries": (i32, [vp, P(dbl)]),
        "tn_mpo_site_ops": (i32, [vp, i32, P(dbl)]),
        "tn_mpo_destroy": (None, [vp]),
        "tn_mps_create": (i32, [vp, i32, i32, P(i32), P(dbl), P(vp)]),
        "tn_mps_bond_dims": (i32, [vp, P(i32)]),
        "tn_mps_export": (i32, [vp, vp, P(dbl), szt, P(szt)]),
        "tn_mps_canonicalize": (i32, [vp, vp]),
        "tn_mps_checkpoint": (i32, [vp, vp, vp, P(dbl), szt, P(szt)]),
        "tn_mps_import": (i32, [vp, P(dbl), szt, P(vp), P(dbl), P(i32)]),
        "tn_mps_sweeps": (i32, [vp, P(i64)]),
        "tn_mps_destroy": (None, [vp]),
        "tn_dmrg_sweep": (i32, [vp, vp, vp, P(tn_sweep_opts), P(tn_sweep_stats)]),
        "tn_energy": (i32, [vp, vp, vp, P(dbl), P(dbl)]),
        "tn_energy_variance": (i32, [vp, vp, vp, P(dbl), P(dbl), P(dbl)]),
        "tn_dmrg_solve": (i32, [vp, vp, vp, P(tn_solve_opts), P(tn_solve_result), P(dbl), P(dbl)]),
        "tn_lbo_step": (i32, [vp, vp, vp, i32, P(tn_sweep_opts), P(dbl)]),
        "tn_marginals": (i32, [vp, vp, vp, i32, P(dbl)]),
        "tn_sample": (i32, [vp, vp, vp, i64, C.c_uint64, vp]),
        "tn_sample_noalloc": (i32, [vp, vp, vp, i64, C.c_uint64, vp]),
        "tn_heff_apply": (i32, [vp, vp, i32, i32, i32, vp, vp, vp, vp, i32]),
        "tn_env_update": (i32, [vp, vp, i32, i32, i32, i32, vp, vp, vp, i32]),
        "tn_truncate": (i32, [vp, i32, i32, vp, i32, dbl, i32, vp, vp, P(i32), P(dbl), P(dbl)]),
        "tn_profile": (i32, [vp, i32, P(dbl)]),
        "tn_cgemm": (i32, [vp, i32, i32, i32, i32, i32, i32, vp, i64, vp, i64, vp, i64]),
        "tn_philox4x32_10": (i32, [vp, P(C.c_uint32), P(C.c_uint32), P(C.c_uint32), i32]),
        "tn_matvec_flops": (dbl, [vp, i32, i32, i32]),
        "tn_env_flops": (dbl, [vp, i32, i32, i32]),
        "tn_rdm": (i32, [vp, vp, vp, i32, P(dbl)]),
        "tn_mlp_create": (i32, [vp, i32, i32, i32, C.c_uint64, P(vp)]),
        "tn_mlp_destroy": (None, [vp]),
        "tn_mlp_num_params": (i64, [vp]),
        "tn_mlp_params": (i32, [vp, vp, P(C.c_float), P(C.c_float)]),
        "tn_mlp_forward": (i32, [vp, vp, vp, i32, vp]),
        "tn_mlp_grad": (i32, [vp, vp, vp, vp, i32, P(C.c_float), P(C.c_float)]),
        "tn_mlp_train_step": (i32, [vp, vp, vp, vp, i32, C.c_float, P(C.c_float)]),
        "tn_squeezed_basis": (i32, [dbl, dbl, i32, i32, i32, P(dbl)]),
        "tn_ws_features": (i32, [i32, P(dbl), P(dbl), P(C.c_float)]),
        "tn_ws_targets": (i32, [i32, i32, P(dbl), P(C.c_float)]),
        "tn_ws_gaussian_params": (i32, [i32, P(dbl), P(dbl), P(C.c_float)]),
        "tn_cutoff_report": (i32, [i32, P(dbl), P(dbl), i32, i32, dbl, P(dbl), P(i32), P(dbl)]),
        "tn_ws_initial_state": (i32, [i32, i32, i32, i32, P(C.c_float), C.c_uint64, dbl, P(dbl), P(i32), P(dbl),
                                      szt, P(szt)]),
        "tn_noise_uniform_loss": (i32, [i32, P(dbl), P(dbl), dbl, P(dbl), P(dbl)]),
        "tn_sample_displaced": (i32, [vp, vp, vp, i64, C.c_uint64, i32, vp, P(dbl), vp]),
        "tn_noise_williamson": (i32, [i32, P(dbl), P(dbl), P(dbl), P(dbl), P(i32)]),
        "tn_plbo_ops": (i32, [i32, P(dbl), dbl, dbl, dbl, P(dbl), P(dbl)]),
        "tn_plbo_fock_isometry": (i32, [i32, i32, P(dbl), i32, P(dbl)]),
        "tn_plbo_effective_cutoff": (i32, [i32, P(dbl), i32, dbl, P(i32)]),
        "tn_plbo_enable": (i32, [vp, P(dbl)]),
        "tn_plbo_minimize": (i32, [i32, P(dbl), dbl, dbl, dbl, P(tn_plbo_opts), P(dbl), P(dbl)]),
        "tn_plbo_params": (i32, [vp, P(dbl)]),
        "tn_plbo_linear": (i32, [vp]),
        "tn_plbo_linear_isometries": (i32, [vp, P(dbl)]),
        "tn_plbo_site_gradient": (i32, [vp, vp, vp, i32, i32, P(dbl), P(dbl), P(dbl)]),
        "tn_plbo_sweep": (i32, [vp, vp, vp, P(tn_sweep_opts), P(tn_plbo_opts), P(tn_sweep_stats), P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def dptr(a: np.ndarray, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))
