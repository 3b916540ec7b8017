"""ctypes view of librte's C ABI (include/rte.h).  Argument marshalling only."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librte.so")

RTE_OK, RTE_EINVAL, RTE_ENOMEM, RTE_EDEVICE, RTE_ENOCONV = 0, -1, -2, -3, -4
RTE_EBREAKDOWN, RTE_EAGAIN, RTE_EFORMAT, RTE_ENOTFOUND = -5, -6, -7, -8
STATUS_NAMES = {0: "RTE_OK", -1: "RTE_EINVAL", -2: "RTE_ENOMEM", -3: "RTE_EDEVICE", -4: "RTE_ENOCONV",
                -5: "RTE_EBREAKDOWN", -6: "RTE_EAGAIN", -7: "RTE_EFORMAT", -8: "RTE_ENOTFOUND"}
HG_AUTO, HG_FLATLAND, HG_SPHERE = 0, 1, 2
SCHEME_UPWIND, SCHEME_TFPS = 0, 1
FP32, FP64 = 0, 1
PC_NONE, PC_MGNET_BF16, PC_MGNET_FP32, PC_BLOCK_JACOBI = 0, 1, 2, 3
BJ_MAX_DIRS = 112
ARR_RHS, ARR_SCATTER, ARR_SIGMA, ARR_FIELD_A, ARR_FIELD_AINV = 0, 1, 2, 3, 4
K_APPLY, K_RESIDUAL, K_CONV, K_ORTH, K_PRECOND = 0, 1, 2, 3, 4
W_A, W_BPRE, W_BPOST, W_BCOARSE, W_R, W_PR = 0, 1, 2, 3, 4, 5
EPI_STORE, EPI_ACCUM, EPI_STORE_T, EPI_RESID_R, EPI_RESID_T = 0, 1, 2, 3, 4


class RteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("ndir", C.c_int),
                ("dirs", C.POINTER(C.c_double)), ("weights", C.POINTER(C.c_double)),
                ("g", C.c_double), ("kernel", C.c_int), ("scheme", C.c_int)]


class Medium(C.Structure):
    _fields_ = [("sigma_t", C.POINTER(C.c_double)), ("sigma_a", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
                ("eps_scalar", C.c_double), ("inflow", C.POINTER(C.c_double)),
                ("inflow_face_stride", C.c_size_t)]


class OperatorInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("ndir", C.c_int), ("kernel", C.c_int), ("cells", C.c_int64), ("n", C.c_int64),
                ("h", C.c_double), ("g", C.c_double), ("has_fields", C.c_int), ("scheme", C.c_int),
                ("nbasis", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("rtol", C.c_double), ("max_iters", C.c_int),
                ("precond", C.c_int), ("x0", C.c_void_p), ("b", C.c_void_p)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("rel_residual", C.c_double), ("ms_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("active", C.c_int64),
                ("queued", C.c_int64), ("arena_bytes", C.c_size_t), ("arena_in_use", C.c_size_t),
                ("arena_peak", C.c_size_t)]


_P = C.c_void_p
_SIGS = {
    "rte_build_operator": [C.POINTER(Geometry), C.POINTER(Medium), _P, _P, C.POINTER(_P)],
    "rte_operator_free": [_P],
    "rte_operator_get_info": [_P, C.POINTER(OperatorInfo)],
    "rte_operator_copy_array": [_P, C.c_int, C.c_int, _P, C.c_size_t, _P],
    "mgnet_load": [_P, C.c_size_t, C.POINTER(_P)],
    "mgnet_free": [_P],
    "mgnet_describe": [_P, C.POINTER(C.c_int)],
    "rte_apply": [_P, _P, _P, C.c_int, _P],
    "rte_residual": [_P, _P, _P, _P],
    "rte_cell_values": [_P, _P, _P, _P],
    "rte_atfps_build": [_P, C.c_double, C.POINTER(_P)],
    "rte_atfps_free": [_P],
    "rte_atfps_get_info": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "rte_atfps_residual": [_P, _P, _P, _P],
    "rte_atfps_reconstruct": [_P, _P, _P, _P],
    "rte_atfps_filtered_loss": [_P, _P, _P, _P, _P],
    "rte_precond_workspace_bytes": [_P, _P, C.POINTER(C.c_size_t)],
    "rte_precond_apply": [_P, _P, C.c_int, _P, _P, _P, C.c_size_t, _P],
    "rte_precond_apply_noalloc": [_P, _P, C.c_int, _P, _P, _P],
    "mgnet_conv_apply": [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int,
                         C.c_size_t, _P, _P, _P, _P, _P, _P, _P, _P],
    "rte_workspace_bytes": [_P, _P, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)],
    "rte_solve": [_P, _P, C.POINTER(SolveOpts), _P, C.c_size_t, _P, C.POINTER(SolveStats), _P],
    "rte_server_create": [_P, C.c_size_t, C.c_int, C.POINTER(_P)],
    "rte_submit": [_P, _P, _P, C.POINTER(SolveOpts), _P, C.POINTER(C.c_uint64)],
    "rte_submit_many": [_P, C.c_int, C.POINTER(_P), C.POINTER(_P), C.POINTER(SolveOpts), C.POINTER(_P),
                        C.POINTER(C.c_uint64)],
    "rte_poll": [_P, C.c_uint64, C.POINTER(SolveStats)],
    "rte_server_query": [_P, C.POINTER(ServerStats)],
    "rte_server_destroy": [_P],
    "rte_prof_enable": [C.c_int, C.c_int],
    "rte_prof_query": [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                       C.POINTER(C.c_double)],
    "rte_prof_query_key": [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                           C.POINTER(C.c_double)],
    "rte_prof_reset": [],
}

_lib = None


def lib():
    """Load librte.so (built in-tree); raise if it is missing -- there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librte.so is not built (run paper_2604_23265_amd.build.build())")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.rte_last_error.argtypes = []
        L.rte_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(code, allow=()):
    if code != RTE_OK and code not in allow:
        msg = lib().rte_last_error().decode(errors="replace")
        raise RteError(code, msg)
    return code


def exported_symbols():
    return list(_SIGS) + ["rte_last_error"]
