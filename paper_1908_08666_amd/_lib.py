"""ctypes declarations of the C ABI in include/hhg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhhg.so")

HHG_OK, HHG_EINVAL, HHG_EHIP, HHG_ENOCONV, HHG_EBREAKDOWN, HHG_ENOMEM = 0, -1, -2, -3, -4, -5
HHG_F64, HHG_F32 = 0, 1
HHG_CONFORMING, HHG_INDEPENDENT = 0, 1
HHG_DIRICHLET_OUTER, HHG_DIRICHLET_NONE = 0, 1
HHG_CORR_PHYSICAL, HHG_CORR_NONE = 0, 1
HHG_KHAT_PATCH, HHG_KHAT_EDGE = 0, 1
HHG_IFACE_SYMMETRIC, HHG_IFACE_ROWWISE, HHG_IFACE_ZEROSUM = 0, 1, 2
HHG_STRAIN_LSQ, HHG_STRAIN_AVERAGE = 0, 1
HHG_METHOD_SCALED, HHG_METHOD_ONTHEFLY = 0, 1
HHG_K_INTERIOR_SCALED, HHG_K_INTERIOR_ONTHEFLY, HHG_K_BOUNDARY_ROWS, HHG_K_GROUP_SUM = 0, 1, 2, 3
KERNEL_NAMES = {0: "interior_scaled", 1: "interior_onthefly", 2: "boundary_rows", 3: "group_sum",
                4: "solver_vector", 5: "learned"}

STATUS_NAMES = {0: "HHG_OK", -1: "HHG_EINVAL", -2: "HHG_EHIP", -3: "HHG_ENOCONV",
                -4: "HHG_EBREAKDOWN", -5: "HHG_ENOMEM"}


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int32), ("verts", ctypes.POINTER(ctypes.c_double)),
                ("level", ctypes.POINTER(ctypes.c_int32)), ("coupling", ctypes.c_int32),
                ("dirichlet", ctypes.c_int32)]


class OpDesc(ctypes.Structure):
    _fields_ = [("mu0", ctypes.c_double), ("lam0", ctypes.c_double), ("mu1", ctypes.c_double),
                ("lam1", ctypes.c_double), ("corr", ctypes.c_int32), ("khat", ctypes.c_int32),
                ("iface", ctypes.c_int32)]


class MeshDesc2D(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int32), ("verts", ctypes.POINTER(ctypes.c_double)),
                ("level", ctypes.c_int32), ("dirichlet", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precond", ctypes.c_int32), ("method", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer_iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("iterations_run", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


HHG_CG_F64, HHG_IR_F32, HHG_FCG_F64 = 0, 1, 2
HHG_PRECOND_NONE, HHG_PRECOND_BLOCK_JACOBI, HHG_PRECOND_LEARNED = 0, 1, 2
HHG_MLP_IN, HHG_MLP_HIDDEN, HHG_MLP_OUT = 16, 64, 9
HHG_MLP_NPARAM = 16 * 64 + 64 + 64 * 9 + 9
HHG_SAMPLE_BYTES = 128


class MgOpts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("omega", ctypes.c_double),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int32), ("method", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("nu_inc", ctypes.c_int32)]


HHG_MG_CG, HHG_MG_CYCLE = 0, 1


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class Carreau(ctypes.Structure):
    _fields_ = [("eta0", ctypes.c_double), ("eta_inf", ctypes.c_double), ("kappa", ctypes.c_double),
                ("r", ctypes.c_double), ("boundary", ctypes.c_int32), ("pad", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("persist_blocks", ctypes.c_int32),
                ("level", ctypes.c_int32 * 8), ("slab", ctypes.c_int32 * 8),
                ("macros", ctypes.c_int32 * 8), ("rows", ctypes.c_int64 * 8),
                ("ms", ctypes.c_double * 8), ("ms_total", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("pad", ctypes.c_int32)]


HHG_STOKES_DIV, HHG_STOKES_GRAD, HHG_STOKES_STAB, HHG_STOKES_MASS = 0, 1, 2, 3


class StokesOpts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("omega", ctypes.c_double),
                ("omega_p", ctypes.c_double), ("h", ctypes.c_double), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("nu_inc", ctypes.c_int32)]


class PicardInfo(ctypes.Structure):
    _fields_ = [("picard", ctypes.c_int32), ("final_iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("rel_change", ctypes.c_double),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class HHGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_I64P = ctypes.POINTER(ctypes.c_int64)

SIGNATURES = {
    "hhg_setup_macro": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(OpDesc), ctypes.POINTER(_VP)], ctypes.c_int),
    "hhg_destroy": ([_VP], ctypes.c_int),
    "hhg_layout": ([_VP, _I64P, _I64P, _I64P], ctypes.c_int),
    "hhg_node_coords": ([_VP, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hhg_node_flags": ([_VP, ctypes.POINTER(ctypes.c_uint8)], ctypes.c_int),
    "hhg_apply_scaled": ([_VP, _I32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_apply_onthefly": ([_VP, _I32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_residual": ([_VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_workspace_bytes": ([_VP, ctypes.POINTER(SolveOpts), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hhg_cg_solve": ([_VP, ctypes.POINTER(SolveOpts), _VP, _VP, _VP, _VP, ctypes.POINTER(SolveInfo), _VP],
                     ctypes.c_int),
    "hhg_viscosity_workspace_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hhg_nodal_viscosity": ([_VP, _VP, ctypes.POINTER(Carreau), _VP, _VP, _VP], ctypes.c_int),
    "hhg_autotune": ([_VP, _I32, _I32, _VP, _VP, _VP, _I32, ctypes.POINTER(TuneReport), _VP], ctypes.c_int),
    "hhg_set_tuning": ([_VP, ctypes.POINTER(TuneReport)], ctypes.c_int),
    "hhg_graph_create": ([_VP, _I32, _I32, _VP, _VP, _VP, _I32, ctypes.POINTER(_I32)], ctypes.c_int),
    "hhg_graph_launch": ([_VP, _I32, _VP], ctypes.c_int),
    "hhg_graph_destroy": ([_VP, _I32], ctypes.c_int),
    "hhg_mlp_create": ([ctypes.POINTER(_VP)], ctypes.c_int),
    "hhg_mlp_destroy": ([_VP], ctypes.c_int),
    "hhg_mlp_set_weights": ([_VP, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "hhg_mlp_get_weights": ([_VP, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "hhg_learn_features": ([_VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mlp_forward": ([_VP, _VP, _I64, _I64, _VP, _VP], ctypes.c_int),
    "hhg_learn_collect": ([_VP, _I32, _VP, _VP, _VP, _VP, _I64, _VP, _VP], ctypes.c_int),
    "hhg_mlp_loss_grad": ([_VP, _VP, _I64, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_float), _VP], ctypes.c_int),
    "hhg_mlp_train": ([_VP, _VP, _I64, ctypes.POINTER(TrainOpts), ctypes.POINTER(ctypes.c_float), _VP],
                      ctypes.c_int),
    "hhg_set_learned_model": ([_VP, _VP], ctypes.c_int),
    "hhg_preconditioner": ([_VP, _I32, _I32, _VP, _VP, _VP], ctypes.c_int),
    "hhg_preconditioner_noalloc": ([_VP, _I32, _I32, _VP, _VP, _VP], ctypes.c_int),
    "hhg2d_setup": ([ctypes.POINTER(MeshDesc2D), ctypes.POINTER(OpDesc), ctypes.POINTER(_VP)], ctypes.c_int),
    "hhg2d_destroy": ([_VP], ctypes.c_int),
    "hhg2d_layout": ([_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "hhg2d_node_coords": ([_VP, _VP], ctypes.c_int),
    "hhg2d_node_flags": ([_VP, _VP], ctypes.c_int),
    "hhg2d_apply": ([_VP, _I32, _I32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_create": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(OpDesc), _I32, ctypes.POINTER(_VP)],
                      ctypes.c_int),
    "hhg_mg_destroy": ([_VP], ctypes.c_int),
    "hhg_mg_set_smoother": ([_VP, _I32], ctypes.c_int),
    "hhg_mg_level": ([_VP, _I32, ctypes.POINTER(_VP)], ctypes.c_int),
    "hhg_mg_workspace_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hhg_mg_prolong": ([_VP, _I32, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_restrict": ([_VP, _I32, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_setup_coefficient": ([_VP, _I32, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_vcycle": ([_VP, ctypes.POINTER(MgOpts), _VP, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_solve": ([_VP, ctypes.POINTER(MgOpts), _VP, _VP, _VP, ctypes.POINTER(SolveInfo), _VP],
                     ctypes.c_int),
    "hhg_stokes_rows": ([_VP, _I32, ctypes.c_double, _VP, _VP, _VP], ctypes.c_int),
    "hhg_mg_stokes_workspace_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hhg_mg_stokes_solve": ([_VP, ctypes.POINTER(StokesOpts), _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                             ctypes.POINTER(SolveInfo), _VP], ctypes.c_int),
    "hhg_mg_stokes_picard": ([_VP, ctypes.POINTER(StokesOpts), ctypes.POINTER(Carreau), _I32, _I32, _VP,
                              _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(PicardInfo), _VP], ctypes.c_int),
    "hhg_profile_enable": ([_VP, _I32], ctypes.c_int),
    "hhg_profile_read": ([_VP, _I32, _I64P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hhg_last_error": ([], ctypes.c_char_p),
}


def lib():
    """Load libhhg.so from the package directory; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    # torch's HIP runtime is brought up first: when libhhg.so was loaded
    # before it, the library's first HIP call found no device
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(code: int):
    if code != HHG_OK:
        msg = lib().hhg_last_error()
        raise HHGError(code, msg.decode() if msg else "")
    return code
