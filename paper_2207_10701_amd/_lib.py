"""ctypes declarations of librecip's C ABI (include/recip.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of librecip.so.  Importing this module fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "librecip.so"

RCP_OK, RCP_EINVAL, RCP_ENOMEM, RCP_ESINGULAR, RCP_ENOCONV, RCP_EHIP = 0, -1, -2, -3, -4, -5
RCP_FP64, RCP_FP32_REFINED = 0, 1
RCP_CONCENTRATOR, RCP_COLLIMATOR = 0, 1
RCP_CONE, RCP_ANNULUS, RCP_SYMBOL_TABLE = 0, 1, 2

ERROR_NAMES = {RCP_EINVAL: "RCP_EINVAL", RCP_ENOMEM: "RCP_ENOMEM", RCP_ESINGULAR: "RCP_ESINGULAR",
               RCP_ENOCONV: "RCP_ENOCONV", RCP_EHIP: "RCP_EHIP"}


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("npml", C.c_int32),
                ("h", C.c_double), ("k0", C.c_double), ("pml_R", C.c_double),
                ("pml_m", C.c_int32), ("eps_dev", C.c_void_p)]


class Pillars(C.Structure):
    _fields_ = [("n", C.c_int32), ("centers_dev", C.c_void_p), ("widths_dev", C.c_void_p),
                ("eps_bg", C.c_double), ("eps_sub", C.c_double), ("eps_pillar", C.c_double),
                ("sub_rows", C.c_int32), ("row0", C.c_int32), ("rows", C.c_int32)]


class Objective(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i_f", C.c_int32), ("j_f", C.c_int32),
                ("j_m", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32),
                ("phi", C.c_double), ("n_m", C.c_double)]


class Light(C.Structure):
    _fields_ = [("j_s", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32),
                ("n_s", C.c_double), ("kind", C.c_int32), ("c", C.c_double),
                ("th1", C.c_double), ("th2", C.c_double), ("symbol_dev", C.c_void_p)]


class Grid3D(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("npml", C.c_int32),
                ("h", C.c_double), ("k0", C.c_double), ("pml_R", C.c_double),
                ("pml_m", C.c_int32), ("eps_dev", C.c_void_p)]


class Pillars3D(C.Structure):
    _fields_ = [("n", C.c_int32), ("centers_dev", C.c_void_p), ("widths_dev", C.c_void_p),
                ("eps_bg", C.c_double), ("eps_sub", C.c_double), ("eps_pillar", C.c_double),
                ("sub_layers", C.c_int32), ("pillar_k0", C.c_int32), ("pillar_layers", C.c_int32)]


class Objective3D(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i_f", C.c_int32), ("j_f", C.c_int32), ("k_f", C.c_int32),
                ("k_m", C.c_int32), ("theta", C.c_double), ("azimuth", C.c_double),
                ("n_m", C.c_double)]


class Light3D(C.Structure):
    _fields_ = [("k_s", C.c_int32), ("n_s", C.c_double), ("ndir", C.c_int32),
                ("dirs_dev", C.c_void_p)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_residual", C.c_double)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("samples", C.c_int64), ("ms", C.c_double),
                ("work", C.c_double)]


NKCLASS = 8
KCLASS_NAMES = ["gj_panel", "gj_update", "schur", "block_gemv", "block_gemm", "gj_last",
                "dense_zgemm", "engine"]


class RecipError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(str(LIB_PATH))
    P = C.POINTER
    vp, i32, f64, sz = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
    sig = {
        "rcp_eps_from_widths": (C.c_int, [P(Grid), P(Pillars), vp, vp]),
        "rcp_factor_bytes": (sz, [P(Grid), i32]),
        "rcp_factor": (C.c_int, [P(Grid), i32, vp, sz, vp, P(vp)]),
        "rcp_factor_batch": (C.c_int, [i32, P(Grid), i32, P(vp), sz, vp, P(vp)]),
        "rcp_factor_batch_async": (C.c_int, [i32, P(Grid), i32, P(vp), sz, vp, P(vp)]),
        "rcp_factors_status": (C.c_int, [vp, vp]),
        "rcp_factors_status_dev": (vp, [vp]),
        "rcp_solve_multi_rhs": (C.c_int, [vp, i32, vp, vp, i32, f64, i32, vp, P(SolveStats)]),
        "rcp_reciprocal_average": (C.c_int, [vp, P(Objective), P(Light), vp, vp, vp, vp]),
        "rcp_brute_force_work_bytes": (sz, [vp, i32, i32]),
        "rcp_brute_force_average": (C.c_int, [vp, P(Objective), P(Light), i32, i32, vp, sz, vp,
                                              vp, vp]),
        "rcp_adjoint_grad": (C.c_int, [vp, P(Objective), P(Light), vp, vp, vp]),
        "rcp_adjoint_grad_batch": (C.c_int, [i32, P(vp), P(Objective), P(Light), vp, P(vp), vp]),
        "rcp_broadband_grad": (C.c_int, [i32, P(vp), P(Objective), P(Light), P(f64), vp, vp, vp]),
        "rcp_width_grad": (C.c_int, [P(Grid), P(Pillars), vp, vp, vp]),
        "rcp_reciprocal_many_work_bytes": (sz, [vp, i32]),
        "rcp_reciprocal_average_many": (C.c_int, [vp, i32, P(Objective), P(Light), vp, vp, sz, vp]),
        "rcp_reciprocal_average_many_noalloc": (C.c_int, [vp, i32, P(Objective), P(Light), vp,
                                                          vp]),
        "rcp_dense_work_bytes": (sz, [vp, i32, i32]),
        "rcp_reciprocal_average_dense": (C.c_int, [vp, i32, P(Objective), P(Light), vp, vp, vp,
                                                   vp, sz, vp]),
        "rcp_adjoint_grad_dense": (C.c_int, [vp, i32, P(Objective), P(Light), vp, vp, vp, vp,
                                             sz, vp]),
        "rcp_correlation_work_bytes": (sz, [i32, i32]),
        "rcp_correlation_matrix": (C.c_int, [P(Grid), P(Light), i32, vp, vp, vp, vp, sz, vp]),
        "rcp_engine_create": (C.c_int, [i32, P(vp)]),
        "rcp_engine_destroy": (None, [vp]),
        "rcp_engine_add": (C.c_int, [vp, P(Grid), vp, sz, vp, P(vp)]),
        "rcp_engine_step": (C.c_int, [vp, i32, vp, P(vp), P(i32), i32, P(i32), P(i32)]),
        "rcp_eps3d_from_pillars": (C.c_int, [P(Grid3D), P(Pillars3D), vp, vp]),
        "rcp_factor3d_bytes": (sz, [P(Grid3D)]),
        "rcp_factor3d": (C.c_int, [P(Grid3D), vp, sz, vp, P(vp)]),
        "rcp_solve3d": (C.c_int, [vp, vp, vp, i32, vp]),
        "rcp_average3d_work_bytes": (sz, [vp, P(Objective3D), P(Light3D)]),
        "rcp_reciprocal_average3d": (C.c_int, [vp, P(Objective3D), P(Light3D), vp, vp, sz, vp]),
        "rcp_brute_force_average3d": (C.c_int, [vp, P(Objective3D), P(Light3D), vp, vp, vp, sz,
                                                vp]),
        "rcp_factors_release": (None, [vp]),
        "rcp_last_error": (C.c_char_p, []),
        "rcp_last_solve_stats": (C.c_int, [vp, P(SolveStats)]),
        "rcp_factors_info": (C.c_int, [vp, P(i32), P(i32), P(i32), P(i32), P(i32)]),
        "rcp_timing_start": (C.c_int, [i32]),
        "rcp_timing_stop": (C.c_int, [P(KernelStat), i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(code: int) -> None:
    if code != RCP_OK:
        raise RecipError(code, lib.rcp_last_error().decode())
