"""ctypes declarations of the C ABI in include/rbf_fmm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librbffmm.so")

RBF_OK, RBF_ENOCONV, RBF_EINVAL, RBF_EUNSUPPORTED, RBF_ENOMEM, RBF_EHIP, RBF_ESTATE = 0, 1, -1, -2, -3, -4, -5
RBF_F32, RBF_F64 = 0, 1
(RBF_GAUSSIAN, RBF_MULTIQUADRIC, RBF_INVERSE_MULTIQUADRIC, RBF_WENDLAND, RBF_THIN_PLATE, RBF_R5,
 RBF_GAUSSIAN_BANDLIMITED) = 0, 1, 2, 3, 4, 5, 6
RBF_PC_NONE, RBF_PC_BLOCK_JACOBI, RBF_PC_LEARNED = 0, 1, 2
RBF_NPHASES = 7
RBF_PC_BLOCK, RBF_MLP_IN, RBF_MLP_HIDDEN, RBF_MLP_NPARAMS = 64, 64, 256, 164672
RBF_MLP_BF16, RBF_MLP_F32 = 0, 1
RBF_MLP_STATIC_MAX_ROWS = 4096
PHASES = ["permute", "p2p", "p2m", "m2m", "m2l_coarse", "m2l_leaf", "l2p"]


class RbfOpts(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int), ("max_level", ctypes.c_int), ("min_level", ctypes.c_int),
                ("coarse_level", ctypes.c_int), ("coarse_radius", ctypes.c_int), ("nodes", ctypes.c_int),
                ("band", ctypes.c_double), ("m2l_schedule", ctypes.c_int), ("exact", ctypes.c_int),
                ("band_transfer", ctypes.c_int), ("reserved", ctypes.c_int * 5)]


class RbfSolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iters", ctypes.c_int), ("precond", ctypes.c_int),
                ("zero_init", ctypes.c_int), ("fallback", ctypes.c_int), ("time_limit_s", ctypes.c_double),
                ("reserved", ctypes.c_int * 8)]


class RbfSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("fallback_used", ctypes.c_int), ("true_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.c_double * 256), ("nhistory", ctypes.c_int),
                ("history_s", ctypes.c_double * 256)]


class RbfPlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int), ("dtype", ctypes.c_int), ("kernel", ctypes.c_int),
                ("nleaves", ctypes.c_int), ("nlevels", ctypes.c_int), ("coarse_level", ctypes.c_int),
                ("coarse_radius", ctypes.c_int), ("nodes", ctypes.c_int), ("bits", ctypes.c_int),
                ("half_nodes", ctypes.c_int64), ("ncells", ctypes.c_int64), ("nnear", ctypes.c_int64),
                ("near_pairs", ctypes.c_int64), ("shape", ctypes.c_double), ("tol", ctypes.c_double),
                ("band", ctypes.c_double), ("period", ctypes.c_double), ("rcut", ctypes.c_double),
                ("rfar", ctypes.c_double), ("ext", ctypes.c_double), ("lo", ctypes.c_double * 5),
                ("device_bytes", ctypes.c_int64), ("far_field", ctypes.c_int), ("nbands", ctypes.c_int),
                ("residual_width", ctypes.c_double), ("residual_in_q", ctypes.c_int),
                ("reserved_info", ctypes.c_int)]


class RbfBandInfo(ctypes.Structure):
    _fields_ = [("top", ctypes.c_int), ("coarse_level", ctypes.c_int), ("coarse_radius", ctypes.c_int),
                ("nodes", ctypes.c_int), ("half_nodes", ctypes.c_int64), ("nunits", ctypes.c_int),
                ("nchunks", ctypes.c_int), ("width_lo", ctypes.c_double), ("width_hi", ctypes.c_double),
                ("tol", ctypes.c_double), ("band", ctypes.c_double), ("period", ctypes.c_double),
                ("reach", ctypes.c_double), ("rfar", ctypes.c_double), ("scale", ctypes.c_double),
                ("transfer", ctypes.c_int), ("transfer_order", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class RbfBatchInfo(ctypes.Structure):
    _fields_ = [("nprob", ctypes.c_int), ("ngroups", ctypes.c_int), ("nfar", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("total_n", ctypes.c_int64), ("total_leaves", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("plan_seconds", ctypes.c_double)]


class RbfTrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("patience", ctypes.c_int),
                ("reserved0", ctypes.c_int), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("val_frac", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("reserved", ctypes.c_int * 8)]


class RbfTrainInfo(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int), ("best_epoch", ctypes.c_int), ("nhist", ctypes.c_int),
                ("reserved0", ctypes.c_int), ("init_val_loss", ctypes.c_double), ("best_val_loss", ctypes.c_double),
                ("final_train_loss", ctypes.c_double), ("seconds", ctypes.c_double),
                ("train_loss", ctypes.c_double * 256), ("val_loss", ctypes.c_double * 256)]


_P = ctypes.c_void_p
# name -> (restype, argtypes)
SIGNATURES = {
    "rbf_fmm_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.POINTER(RbfOpts), ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_fmm_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_direct_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_fmm_plan_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(RbfOpts), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_fmm_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_direct_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_interp_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.POINTER(RbfSolveOpts), ctypes.POINTER(RbfSolveInfo)]),
    "rbf_interp_solve_poly": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_double, ctypes.POINTER(RbfSolveOpts),
                                             ctypes.POINTER(RbfSolveInfo)]),
    "rbf_poly_terms": (ctypes.c_int, [ctypes.c_void_p]),
    "rbf_fmm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rbf_last_error": (ctypes.c_char_p, []),
    "rbf_fmm_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RbfPlanInfo)]),
    "rbf_fmm_band_info": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(RbfBandInfo)]),
    "rbf_fmm_tree_export": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 6),
    "rbf_fmm_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "rbf_fmm_phase_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "rbf_fmm_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, ctypes.POINTER(RbfOpts), ctypes.c_int,
                                        ctypes.c_void_p, ctypes.POINTER(RbfOpts), ctypes.POINTER(ctypes.c_double)]),
    "rbf_fmm_plan_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(RbfOpts),
                                          ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rbf_fmm_matvec_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbf_fmm_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "rbf_fmm_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RbfBatchInfo), ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "rbf_fmm_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rbf_interp_solve_batch": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(RbfSolveOpts), _P]),
    "rbf_pc_block_jacobi": (ctypes.c_int, [_P, ctypes.c_double]),
    "rbf_pc_learned_features": (ctypes.c_int, [_P, ctypes.c_double]),
    "rbf_pc_apply": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "rbf_mlp_create": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "rbf_mlp_destroy": (ctypes.c_int, [_P]),
    "rbf_mlp_get_params": (ctypes.c_int, [_P, _P]),
    "rbf_mlp_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "rbf_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "rbf_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int, _P]),
    "rbf_mlp_forward_static": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "rbf_mlp_loss_grad": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), _P, _P]),
    "rbf_mlp_train": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(RbfTrainOpts), _P,
                                     ctypes.POINTER(RbfTrainInfo)]),
    "rbf_pc_set_learned": (ctypes.c_int, [_P, _P]),
    "rbf_pc_pairs": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "rbf_pc_harvest": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P, _P,
                                      _P]),
    "rbf_pc_train": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int, _P, ctypes.c_int,
                                    ctypes.c_uint64, ctypes.POINTER(RbfTrainOpts), ctypes.c_char_p,
                                    ctypes.POINTER(RbfTrainInfo)]),
    "rbf_pc_load": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(_P)]),
}

_lib = None


class RbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def load():
    """Load the in-tree library; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_1606_07652_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int, allow=(RBF_OK,)) -> int:
    if code not in allow:
        raise RbfError(code, load().rbf_last_error().decode(errors="replace"))
    return code


def check_count(code: int) -> int:
    """A count (>= 0) or a negative error code."""
    if code < 0:
        raise RbfError(code, load().rbf_last_error().decode(errors="replace"))
    return code
