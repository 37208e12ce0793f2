"""ctypes view of ``libpwf.so`` (declarations mirror ``include/pwf.h``)."""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpwf.so")

PWF_OK = 0
PWF_ERR_ARG = -1
PWF_ERR_SIZE = -2
PWF_ERR_EVANESCENT = -3
PWF_ERR_WORKSPACE = -4
PWF_ERR_HIP = -5
PWF_ERR_NONFINITE = -6
PWF_ERR_SCRATCH = -7


class pwf_geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pixel_m", ctypes.c_double),
                ("wavelength_m", ctypes.c_double), ("z1_m", ctypes.c_double), ("z2_m", ctypes.c_double)]


PWF_SRC_GAUSS = 0
PWF_SRC_COHERENCE = 1
PWF_SRC_IOTF = 2


class pwf_source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("sigma_x_px", ctypes.c_double), ("sigma_y_px", ctypes.c_double),
                ("x_coh_m", ctypes.c_double), ("y_coh_m", ctypes.c_double),
                ("iotf_x", ctypes.c_void_p), ("iotf_y", ctypes.c_void_p)]


class pwf_params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("alpha_re", ctypes.c_double), ("alpha_im", ctypes.c_double),
                ("gamma", ctypes.c_double), ("precond_scale", ctypes.c_double), ("precondition", ctypes.c_int32)]


class pwf_problem(ctypes.Structure):
    _fields_ = [("geom", pwf_geometry), ("source", pwf_source), ("params", pwf_params),
                ("diffuser", ctypes.c_void_p)]


class pwf_state(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("psi_hat", ctypes.c_void_p), ("z_hat", ctypes.c_void_p),
                ("y_hat", ctypes.c_void_p), ("k", ctypes.c_int32)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32

# name -> (restype, argtypes)
SIGNATURES = {
    "pwf_status_string": (ctypes.c_char_p, [_i32]),
    "pwf_version": (_i32, []),
    "pwf_workspace_size": (ctypes.c_size_t, [_P(pwf_problem), _i32]),
    "pwf_forward": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _vp, ctypes.c_size_t, _vp]),
    "pwf_gradient": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _P(_vp), _P(_vp), _vp, _vp,
                            ctypes.c_size_t, _vp]),
    "pwf_loss_grad": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _P(_vp), _vp, _vp, ctypes.c_size_t, _vp]),
    "pwf_loss_grad_noalloc": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _P(_vp), _vp, _vp]),
    "pwf_loss_grad_noalloc_limit": (ctypes.c_size_t, []),
    "pwf_state_init": (_i32, [_P(pwf_problem), _i32, _P(pwf_state), _P(_vp), _P(_vp), _vp, ctypes.c_size_t, _vp]),
    "pwf_step": (_i32, [_P(pwf_problem), _i32, _P(pwf_state), _vp, _vp, ctypes.c_size_t, _vp]),
    "pwf_solve": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _i32, ctypes.c_double, _vp, _P(_i32), _vp,
                         ctypes.c_size_t, _vp]),
    "pwf_joint_workspace_size": (ctypes.c_size_t, [_P(pwf_problem), _i32]),
    "pwf_solve_joint": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _i32, ctypes.c_double, _vp, _vp,
                               ctypes.c_size_t, _vp]),
    "pwf_solve_plain": (_i32, [_P(pwf_problem), _vp, _vp, _i32, _vp, _vp, ctypes.c_size_t, _vp]),
    "pwf_bench_sweep": (_i32, [_P(pwf_problem), _i32, _i32, _i32, _vp, ctypes.c_size_t, _vp]),
    "pwf_set_column_tile": (_i32, [_i32, _i32, _i32]),
    "pwf_column_tile": (_i32, [_i32, _i32]),
    "pwf_set_row_plan": (_i32, [_i32, _i32, _i32]),
    "pwf_row_plan": (_i32, [_i32, _i32]),
    "pwf_autotune": (_i32, [_P(pwf_problem), _i32, _i32, _vp, ctypes.c_size_t, _vp]),
    "pwf_autotune_cached": (_i32, [_P(pwf_problem), _i32, _i32, ctypes.c_char_p, _i32, _P(_i32), _vp,
                                   ctypes.c_size_t, _vp]),
    "pwf_set_graph_mode": (None, [_i32]),
    "pwf_set_merged_launch": (None, [_i32]),
    "pwf_sync_status": (_i32, [_vp, _vp]),
    "pwf_speckle_workspace_size": (ctypes.c_size_t, []),
    "pwf_speckle_g2": (_i32, [_vp, _i32, _i32, _i32, _P(ctypes.c_double), _P(ctypes.c_double), _vp, ctypes.c_size_t,
                              _vp]),
    "pwf_fit_coherence": (_i32, [_P(ctypes.c_double), _i32, ctypes.c_double, _P(ctypes.c_double),
                                 _P(ctypes.c_double)]),
    "pwf_rmse_image": (_i32, [_P(pwf_problem), _i32, _P(_vp), _P(_vp), _P(ctypes.c_double), _P(_vp), _vp,
                              ctypes.c_size_t, _vp]),
    "pwf_shell_correlation_workspace_size": (ctypes.c_size_t, [_i32, _i32]),
    "pwf_shell_correlation": (_i32, [_vp, _vp, _i32, _i32, _i32, _P(ctypes.c_double), _vp, ctypes.c_size_t, _vp]),
    "pwf_background_workspace_size": (ctypes.c_size_t, [_i32, _i32]),
    "pwf_background_quadratic": (_i32, [_vp, _i32, _i32, ctypes.c_double, _P(ctypes.c_double), _vp, ctypes.c_size_t,
                                        _vp]),
    "pwf_fbp_workspace_size": (ctypes.c_size_t, [_i32, _i32, _i32]),
    "pwf_fbp": (_i32, [_P(_vp), _i32, _i32, _i32, _P(ctypes.c_double), _i32, ctypes.c_double, _vp, _vp,
                       ctypes.c_size_t, _vp]),
    "pwf_diffuser_from_reference": (_i32, [_P(pwf_problem), _vp, ctypes.c_double, _vp, _vp, ctypes.c_size_t, _vp]),
    "pwf_finalize": (None, []),
}

_lib = None


class PwfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpwf.so not found at {LIB_PATH}; build it with "
                              "`python -m paper_2503_20146_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().pwf_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != PWF_OK:
        raise PwfError(status, where)
