"""ctypes loader for libfmmbem.so (argument marshalling only).

The shared library is built in-tree by ``paper_2103_01048_amd.build``.  There
is no fallback: if the library is missing, loading raises."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmmbem.so")

FMM_LAPLACE, FMM_YUKAWA = 0, 1
FMM_FP64, FMM_FP32, FMM_FP32_BF16X3 = 0, 1, 2
FMM_BEM_DIRECT, FMM_BEM_DERIVATIVE, FMM_BEM_EXTERIOR, FMM_BEM_EXTERIOR_P1 = 0, 1, 2, 3
FMM_BEM_PRECOND_BLOCK, FMM_BEM_PRECOND_MASS = 0, 1
FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EHIP, FMM_ENOTCONV, FMM_EBREAKDOWN = 0, -1, -2, -3, -4, -5
BEM_RHS_SCRATCH_DOUBLES = 1 << 23
FMM_PROFILE_SERIAL = 0x10000

PHASES = ["permute", "p2m", "uc2e", "m2m", "p2l", "m2l", "m2l_sum", "l2l", "dc2e", "leaf", "near", "far",
          "near_early"]

STATUS_NAMES = {0: "FMM_OK", -1: "FMM_EINVAL", -2: "FMM_ENOMEM", -3: "FMM_EHIP", -4: "FMM_ENOTCONV",
                -5: "FMM_EBREAKDOWN"}


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class FmmInfo(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
        ("max_level", ctypes.c_int32), ("n_surf", ctypes.c_int32), ("n_u_pairs", ctypes.c_int64),
        ("n_v_pairs", ctypes.c_int64), ("n_w_pairs", ctypes.c_int64), ("n_x_pairs", ctypes.c_int64),
        ("n_p2p_interactions", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
        ("n_far_interactions", ctypes.c_int64), ("rank_up", ctypes.c_int32), ("rank_down", ctypes.c_int32),
        ("setup_sort_ms", ctypes.c_double), ("setup_tree_ms", ctypes.c_double), ("setup_lists_ms", ctypes.c_double),
        ("setup_items_ms", ctypes.c_double), ("setup_ops_ms", ctypes.c_double), ("tree_on_device", ctypes.c_int32),
        ("tree_shared", ctypes.c_int32), ("chain_timeouts", ctypes.c_int32), ("n_p2p_early", ctypes.c_int64),
        ("n_items", ctypes.c_int32), ("n_items_early", ctypes.c_int32),
    ]


class FmmTuning(ctypes.Structure):
    _fields_ = [
        ("tile_split2", ctypes.c_int32), ("tile_split4", ctypes.c_int32), ("work_cap_min", ctypes.c_int32),
        ("work_cap_div", ctypes.c_int32), ("far_weight", ctypes.c_double), ("gemm_rbw", ctypes.c_int32),
        ("m2l_factored", ctypes.c_int32), ("pair_order", ctypes.c_int32),
        ("near_lds", ctypes.c_int32), ("gemm_lat", ctypes.c_int32),
        ("gemm_chain", ctypes.c_int32), ("m2l_cols", ctypes.c_int32),
        ("gemm_narrow", ctypes.c_int32), ("near_early", ctypes.c_int32), ("near_early_grid", ctypes.c_int32),
        ("m2l_early", ctypes.c_int32), ("near_early_start", ctypes.c_int32),
    ]


_LIB = None

vp = ctypes.c_void_p
i64 = ctypes.c_int64
i32 = ctypes.c_int
dbl = ctypes.c_double
P = ctypes.POINTER

SIGNATURES = {
    "fmm_setup": (i32, [vp, i64, i32, dbl, i32, i32, i32, vp, P(vp)]),
    "fmm_eval": (i32, [vp, vp, i32, vp, vp, vp]),
    "fmm_eval_pair": (i32, [vp, vp, vp, i32, vp, vp, vp, vp, vp]),
    "fmm_eval_pair_md": (i32, [vp, vp, vp, vp, dbl, dbl, vp, vp, vp, vp, vp]),
    "fmm_setup_batch": (i32, [vp, vp, i32, i32, dbl, i32, i32, i32, vp, P(vp)]),
    "fmm_info": (i32, [vp, P(FmmInfo)]),
    "fmm_get_tree": (i32, [vp] + [vp] * 11),
    "fmm_get_root": (i32, [vp, vp, vp]),
    "fmm_free": (None, [vp]),
    "fmm_last_error": (ctypes.c_char_p, []),
    "fmm_set_profiling": (i32, [vp, i32]),
    "fmm_adjoint": (i32, [vp, vp, vp, vp, i32, vp, vp, vp]),
    "bem_setup": (i32, [vp, i64, vp, i64, i32, dbl, dbl, dbl, i32, i32, i32, i32, vp, P(vp)]),
    "bem_matvec": (i32, [vp, vp, vp, vp]),
    "bem_rhs": (i32, [vp, vp, vp, i64, vp, vp]),
    "bem_rhs_noalloc": (i32, [vp, vp, vp, i64, vp, vp]),
    "bem_energy": (i32, [vp, vp, vp, vp, i64, P(dbl), vp]),
    "bem_precondition": (i32, [vp, vp, vp, vp]),
    "bem_set_preconditioner": (i32, [vp, i32, vp]),
    "gmres_solve": (i32, [vp, vp, vp, vp, dbl, dbl, i32, i32, P(i32), vp, vp]),
    "bem_info": (i32, [vp, vp]),
    "bem_fmm_plan": (vp, [vp, i32]),
    "bem_free": (None, [vp]),
    "fmm_get_phase_times": (i32, [vp, vp, vp, i32]),
    "fmm_set_tuning": (i32, [P(FmmTuning)]),
    "fmm_get_tuning": (i32, [P(FmmTuning)]),
}


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_01048_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _LIB = L
    return _LIB


def check(code, what=""):
    if code != FMM_OK:
        msg = lib().fmm_last_error().decode(errors="replace")
        raise FmmError(code, f"{what}: {msg}" if what else msg)
    return code
