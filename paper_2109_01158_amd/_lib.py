"""ctypes view of libp1e.so (declarations in include/p1e.h).

torch is imported first so that the process has exactly one HIP runtime: libp1e.so links
against libamdhip64.so.7, which then resolves to the runtime torch already loaded.
The product has no fallback: if the library is missing, importing this module fails.
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libp1e.so binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp1e.so")

P1E_OK = 0
P1E_EINVAL = -1
P1E_EDEGEN = -2
P1E_ENOMEM = -3
P1E_EHIP = -4
P1E_EDOMAIN = -5
P1E_EBUSY = -6
P1E_ESTATE = -7

P1E_PLAPLACE = 1
P1E_NEOHOOKE = 2
P1E_SVK = 3
P1E_GINZBURG_LANDAU = 4
P1E_PLAPLACE_ORTHO = 5

P1E_FP64 = 1
P1E_MIXED = 2
P1E_FD = 4

P1E_INPUT_ORDER = 1
P1E_FULL_GEOMETRY = 4

P1E_STATIC_SCRATCH_BYTES = 64 << 20

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EDEGEN", -3: "ENOMEM", -4: "EHIP", -5: "EDOMAIN",
                -6: "EBUSY", -7: "ESTATE"}


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("kind", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("nn", ctypes.c_int64), ("ne", ctypes.c_int64),
        ("conn", ctypes.c_void_p), ("coords", ctypes.c_void_p), ("dirichlet", ctypes.c_void_p),
        ("dirichlet_values", ctypes.c_void_p), ("load", ctypes.c_void_p),
        ("p", ctypes.c_double), ("C1", ctypes.c_double), ("D1", ctypes.c_double),
    ]


class MeshInfo(ctypes.Structure):
    _fields_ = [
        ("nn", ctypes.c_int64), ("ne", ctypes.c_int64), ("n_free_nodes", ctypes.c_int64),
        ("n_free_dofs", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("dim", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("kind", ctypes.c_int32),
        ("max_valence", ctypes.c_int32),
        ("total_volume", ctypes.c_double), ("min_volume", ctypes.c_double),
        ("max_volume", ctypes.c_double), ("dirichlet_bv", ctypes.c_double),
        ("alignment", ctypes.c_uint64), ("geometry_classes", ctypes.c_int32),
        ("geometry_mode", ctypes.c_int32), ("n_tiles", ctypes.c_int64),
        ("n_tile_nodes", ctypes.c_int64), ("n_halo_rows", ctypes.c_int64),
        ("n_halo_slots", ctypes.c_int64), ("geometry_class_deviation", ctypes.c_double),
    ]


class LbfgsOpts(ctypes.Structure):
    _fields_ = [("history", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MinReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("evaluations", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("J", ctypes.c_double), ("J_grad", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("history", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("setup_threads", ctypes.c_int32),
                ("pool_bytes", ctypes.c_uint64), ("pool", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("evaluations", ctypes.c_int32),
                ("n_free_dofs", ctypes.c_int32), ("J", ctypes.c_double),
                ("J_grad", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64)]


P1E_MIN_OK, P1E_MIN_STALLED, P1E_MIN_CONVERGED, P1E_MIN_BAD_START = 0, 1, 2, -5


class P1EError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"p1e status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libp1e.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2109_01158_amd.build` (there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    sig = {
        "p1e_mesh_create": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)], ctypes.c_int),
        "p1e_mesh_destroy": ([vp], None),
        "p1e_material_constants": ([ctypes.c_int, dbl, dbl, ctypes.POINTER(dbl),
                                    ctypes.POINTER(dbl)], ctypes.c_int),
        "p1e_mesh_get_info": ([vp, ctypes.POINTER(MeshInfo)], ctypes.c_int),
        "p1e_workspace_bytes": ([vp, ctypes.c_int], u64),
        "p1e_mesh_bind": ([vp, vp, u64, ctypes.c_int, vp], ctypes.c_int),
        "p1e_energy": ([vp, vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "p1e_grad_exact": ([vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "p1e_grad_exact_static": ([vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "p1e_grad_patch_fd": ([vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "p1e_grad_patch_fd4": ([vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "p1e_energy_forces": ([vp, vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "p1e_grad_gather": ([vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "p1e_grad_scale": ([vp, vp, vp, vp], ctypes.c_int),
        "p1e_last_error": ([], ctypes.c_char_p),
        "p1e_minimize_workspace_bytes": ([vp, ctypes.POINTER(LbfgsOpts)], u64),
        "p1e_minimize": ([vp, vp, ctypes.POINTER(LbfgsOpts), vp, u64, ctypes.POINTER(MinReport),
                          vp], ctypes.c_int),
        "p1e_server_table_bytes": ([i32, u64], u64),
        "p1e_server_create": ([ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)], ctypes.c_int),
        "p1e_server_destroy": ([vp], None),
        "p1e_server_clock": ([vp], dbl),
        "p1e_server_submit": ([vp, ctypes.POINTER(MeshDesc), vp, i64, ctypes.POINTER(i64)],
                              ctypes.c_int),
        "p1e_server_step": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "p1e_server_submit_at": ([vp, ctypes.POINTER(MeshDesc), vp, i64, dbl,
                                  ctypes.POINTER(i64)], ctypes.c_int),
        "p1e_server_run": ([vp, i64, dbl, ctypes.POINTER(i32), ctypes.POINTER(i32)],
                           ctypes.c_int),
        "p1e_server_poll": ([vp, ctypes.POINTER(RequestInfo), i32, ctypes.POINTER(i32)],
                            ctypes.c_int),
        "p1e_server_result_vhat": ([vp, i64, vp, i64], ctypes.c_int),
        "p1e_server_release": ([vp, i64], ctypes.c_int),
        "p1e_prof_enable": ([ctypes.c_int], ctypes.c_int),
        "p1e_prof_reset": ([], ctypes.c_int),
        "p1e_prof_collect": ([vp, i64, vp, vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status):
    """Raise P1EError for a negative status, with the library's thread-local message."""
    if status != P1E_OK:
        raise P1EError(status, lib().p1e_last_error().decode(errors="replace"))
    return status
