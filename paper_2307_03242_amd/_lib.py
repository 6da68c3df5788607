"""ctypes loader of libelh.so and the C structures of include/elh.h."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelh.so")

ELH_OK, ELH_NOT_CONVERGED = 0, 1
ELH_ERR_ARG, ELH_ERR_HIP, ELH_ERR_NUMERIC, ELH_ERR_OOM, ELH_ERR_STATE = -1, -2, -3, -4, -5
ELH_C64, ELH_C128 = 1, 2
ELH_SHIFTED, ELH_ADJOINT = 1, 2
ELH_COARSE_KRYLOV, ELH_COARSE_DENSE, ELH_COARSE_RELAX, ELH_COARSE_KACZMARZ = 0, 1, 2, 3

EXPORTED = [
    "elh_create", "elh_set_media", "elh_destroy", "elh_apply", "elh_residual",
    "elh_restrict_residual", "elh_prolong_add", "elh_relax", "elh_relax_noalloc", "elh_coarse_solve", "elh_kaczmarz", "elh_apply_f32in",
    "elh_vcycle", "elh_solve", "elh_solve_adjoint", "elh_solve_batch", "elh_gradient",
    "elh_level_info", "elh_stencil_choice", "elh_status_string", "elh_last_error",
    "elh_batch_create", "elh_batch_size", "elh_batch_handle", "elh_batch_solve", "elh_batch_destroy",
    "elh_receivers", "elh_inject",
]


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double), ("omega", ctypes.c_double), ("gamma", ctypes.c_double),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("abl_width", ctypes.c_double), ("abl_amp", ctypes.c_double),
        ("levels", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
        ("cycle_calls", ctypes.c_int),
        ("damping", ctypes.c_double * 8),
        ("coarse_mode", ctypes.c_int), ("coarse_sweeps", ctypes.c_int),
        ("coarse_restart", ctypes.c_int), ("coarse_maxit", ctypes.c_int),
        ("coarse_rtol", ctypes.c_double), ("coarse_damping", ctypes.c_double),
        ("precond_dtype", ctypes.c_int),
        ("kacz_box", ctypes.c_int),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("rtol", ctypes.c_double),
                ("zero_x0", ctypes.c_int), ("store_z_fp32", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("status", ctypes.c_int),
                ("relres", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_cap", ctypes.c_int), ("history_len", ctypes.c_int),
                ("t_total_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double),
                ("t_apply_ms", ctypes.c_double), ("t_orth_ms", ctypes.c_double),
                ("kernels", ctypes.c_ulonglong)]


_lib = None


def load():
    """Load libelh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libelh.so not found at %s: build it with "
                          "`python -m paper_2307_03242_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    H = ctypes.c_void_p
    sig = {
        "elh_create": [ctypes.POINTER(Desc), vp, vp, vp, vp, ctypes.POINTER(ctypes.c_void_p)],
        "elh_set_media": [H, vp, vp, vp],
        "elh_destroy": [H],
        "elh_apply": [H, ip, ip, ip, ip, vp, vp],
        "elh_residual": [H, ip, ip, ip, ip, vp, vp, vp],
        "elh_restrict_residual": [H, ip, ip, ip, ip, vp, vp, vp],
        "elh_prolong_add": [H, ip, ip, ip, vp, vp],
        "elh_relax": [H, ip, ip, ip, ip, ip, vp, vp],
        "elh_relax_noalloc": [H, ip, ip, ip, ip, ip, vp, vp],
        "elh_coarse_solve": [H, ip, ip, ip, vp, vp],
        "elh_kaczmarz": [H, ip, ip, ip, ip, vp, vp],
        "elh_apply_f32in": [H, ip, ip, vp, vp],
        "elh_vcycle": [H, ip, ip, ip, vp, vp],
        "elh_solve": [H, ip, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)],
        "elh_solve_adjoint": [H, ip, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)],
        "elh_solve_batch": [ip, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                            ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)],
        "elh_gradient": [H, ip, vp, vp, vp, vp, vp],
        "elh_level_info": [H, ip, ctypes.POINTER(ctypes.c_int), dp],
        "elh_stencil_choice": [H, ip, ip, ip, ip, ip, ctypes.POINTER(ctypes.c_int)],
        "elh_batch_create": [ip, ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_void_p), vp, ctypes.POINTER(ctypes.c_void_p)],
        "elh_batch_size": [vp],
        "elh_batch_handle": [vp, ip, ctypes.POINTER(ctypes.c_void_p)],
        "elh_batch_solve": [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p),
                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)],
        "elh_batch_destroy": [vp],
        "elh_receivers": [H, ip, vp, ip, vp, vp, vp, vp],
        "elh_inject": [H, ip, ip, vp, vp, ctypes.c_double, vp],
        "elh_status_string": [ip],
        "elh_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("elh_status_string", "elh_last_error") else ctypes.c_int
    _lib = lib
    return lib


class ElhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (load().elh_status_string(code).decode(), code, msg))
        self.code = code


def check(code):
    if code < 0:
        raise ElhError(code, load().elh_last_error().decode())
    return code
