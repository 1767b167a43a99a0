"""ctypes binding of libpsm.so: the C entry points under the same names.

Argument marshalling only; every step of the hot path runs in the library's
HIP kernels.  Importing this module loads the library and raises if it has not
been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsm.so")

PSM_OK, PSM_EINVAL, PSM_ESIZE, PSM_EUNSUP, PSM_EHIP = 0, -1, -2, -3, -4
PSM_F64, PSM_F32, PSM_F16 = 0, 1, 2
PSM_PERIODIC, PSM_WALL, PSM_INLET, PSM_OUTLET = 0, 1, 2, 3
PSM_BUF_PDF, PSM_BUF_B, PSM_BUF_WORK, PSM_BUF_ADJOINT, PSM_BUF_GRAD_B, PSM_BUF_OBSTACLE = 0, 1, 2, 3, 4, 5
PSM_SHAPE_ELLIPSOID, PSM_SHAPE_CUBE = 0, 1
PSM_COLL_TRT, PSM_COLL_CUMULANT = 0, 1
PSM_MAP_SUBSAMPLES, PSM_MAP_BLOCK = 0, 1
PSM_LAYOUT_SOA, PSM_LAYOUT_BLOCKED = 0, 1
PSM_OPT_GENERAL_PATH, PSM_OPT_XCD_REMAP, PSM_OPT_MAP_LIST, PSM_OPT_SOLID_GRID, PSM_OPT_CONCURRENT = 1, 2, 4, 8, 16
PSM_MAX_BODIES = 8
PSM_STATIC_WORK_BYTES = 16 << 20

# every symbol include/psm.h declares
EXPORTS = [
    "psm_last_error", "psm_required_bytes", "psm_lattice", "psm_body_pose", "pdf_field_create",
    "pdf_field_destroy", "psm_field_reset", "psm_geometry_box", "psm_voxelize_host", "psm_analytic_host",
    "geometry_field_create", "geometry_field_create_analytic", "geometry_field_destroy", "geometry_map_step",
    "psm_stream_collide", "body_force_torque", "psm_mass_fp64", "psm_macroscopic", "psm_error_flags",
    "psm_set_option", "psm_stream_copy", "psm_set_fraction_offset", "psm_adjoint_step", "psm_adjoint_omega",
    "psm_step", "lbm_set_obstacle", "psm_rigid_body", "psm_rigid_advance", "psm_coupled_step", "psm_pdf_stride", "psm_adjoint_gather", "psm_step_ahead", "psm_fractions",
    "pdf_field_create_noalloc", "psm_pdf_layout", "psm_pdf_gather", "psm_pdf_scatter",
]


class psm_rigid(C.Structure):
    _fields_ = [("m", C.c_double), ("I", C.c_double * 3), ("F_ext", C.c_double * 3), ("X", C.c_double * 3),
                ("V", C.c_double * 3), ("R", C.c_double * 9), ("W", C.c_double * 3), ("ft_prev", C.c_double * 6),
                ("average", C.c_int32), ("reserved", C.c_int32)]


class psm_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("q", C.c_int32),
                ("storage", C.c_int32), ("psm", C.c_int32), ("sc", C.c_int32), ("b_form", C.c_int32),
                ("slots", C.c_int32), ("max_bodies", C.c_int32), ("bc", C.c_int32 * 6),
                ("tau", C.c_double), ("magic", C.c_double), ("force", C.c_double * 3),
                ("u_in", C.c_double * 3), ("collision", C.c_int32), ("map_reading", C.c_int32),
                ("layout", C.c_int32), ("block_rows", C.c_int32), ("map_ahead", C.c_int32)]


class psm_body(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("X", C.c_double * 3), ("V", C.c_double * 3), ("W", C.c_double * 3)]


class psm_motion(C.Structure):
    _fields_ = [("axis", C.c_double * 3), ("theta0", C.c_double), ("omega", C.c_double),
                ("x0", C.c_double * 3), ("v", C.c_double * 3)]


class PSMError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2502_20049_amd/build.py; "
                          "there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, sz, i64, dp = C.c_void_p, C.c_size_t, C.c_int64, C.POINTER(C.c_double)
    i32p = C.POINTER(C.c_int32)
    u32p = C.POINTER(C.c_uint32)
    sig = {
        "psm_last_error": (C.c_char_p, []),
        "psm_required_bytes": (C.c_int, [C.POINTER(psm_config), C.c_int, C.POINTER(C.c_size_t)]),
        "psm_lattice": (C.c_int, [C.c_int, i32p, dp, i32p]),
        "psm_body_pose": (C.c_int, [C.POINTER(psm_motion), i64, C.POINTER(psm_body)]),
        "pdf_field_create": (C.c_int, [C.POINTER(psm_config), vp, sz, vp, sz, vp, sz, vp, C.POINTER(vp)]),
        "pdf_field_create_noalloc": (C.c_int, [C.POINTER(psm_config), vp, sz, vp, sz, vp, C.POINTER(vp)]),
        "pdf_field_destroy": (C.c_int, [vp]),
        "psm_field_reset": (C.c_int, [vp, vp]),
        "psm_geometry_box": (C.c_int, [C.c_int, dp, dp, i64, C.c_int, i32p, i32p, C.POINTER(C.c_size_t)]),
        "psm_voxelize_host": (C.c_int, [dp, i64, i32p, i64, C.c_int, i32p, i32p, u32p]),
        "psm_analytic_host": (C.c_int, [C.c_int, dp, C.c_int, i32p, i32p, u32p]),
        "geometry_field_create": (C.c_int, [dp, i64, i32p, i64, C.c_int, vp, sz, vp, C.POINTER(vp)]),
        "geometry_field_create_analytic": (C.c_int, [C.c_int, dp, C.c_int, vp, sz, vp, C.POINTER(vp)]),
        "geometry_field_destroy": (C.c_int, [vp]),
        "geometry_map_step": (C.c_int, [vp, C.POINTER(psm_body), C.POINTER(vp), C.c_int, vp]),
        "psm_stream_collide": (C.c_int, [vp, C.POINTER(psm_body), C.c_int, i64, vp]),
        "psm_step": (C.c_int, [vp, C.POINTER(psm_body), C.POINTER(psm_body), C.POINTER(vp), C.c_int, i64, vp, vp]),
        "psm_step_ahead": (C.c_int, [vp, C.POINTER(psm_body), C.POINTER(psm_body), C.POINTER(psm_body), C.POINTER(vp),
                                     C.c_int, i64, vp, vp]),
        "psm_fractions": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]),
        "body_force_torque": (C.c_int, [vp, C.c_int, vp, vp]),
        "psm_mass_fp64": (C.c_int, [vp, i64, vp, vp]),
        "psm_macroscopic": (C.c_int, [vp, i64, vp, vp, vp]),
        "psm_error_flags": (C.c_int, [vp, vp, vp]),
        "psm_set_option": (C.c_int, [vp, C.c_int, C.c_int]),
        "psm_stream_copy": (C.c_int, [vp, vp, sz, vp]),
        "psm_set_fraction_offset": (C.c_int, [vp, vp]),
        "psm_adjoint_step": (C.c_int, [vp, vp, i64, vp, vp, vp, C.POINTER(psm_body), dp, C.c_double, vp]),
        "psm_adjoint_omega": (C.c_int, [vp, vp, vp]),
        "lbm_set_obstacle": (C.c_int, [vp, vp, vp, sz, C.POINTER(i64), vp]),
        "psm_rigid_body": (C.c_int, [C.POINTER(psm_rigid), C.POINTER(psm_body)]),
        "psm_rigid_advance": (C.c_int, [C.POINTER(psm_rigid), dp, C.c_double]),
        "psm_coupled_step": (C.c_int, [vp, C.POINTER(psm_rigid), C.POINTER(vp), C.c_int, i64, vp, dp, vp]),
        "psm_pdf_stride": (C.c_int, [C.POINTER(psm_config), C.POINTER(i64)]),
        "psm_adjoint_gather": (C.c_int, [vp, vp, vp, vp]),
        "psm_pdf_layout": (C.c_int, [C.POINTER(psm_config), i32p, C.POINTER(i64), C.POINTER(i64)]),
        "psm_pdf_gather": (C.c_int, [vp, vp, vp]),
        "psm_pdf_scatter": (C.c_int, [vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def check(rc: int, what: str = ""):
    if rc != PSM_OK:
        msg = lib.psm_last_error().decode()
        raise PSMError(f"{what or 'psm call'} failed ({rc}): {msg}")
    return rc


def last_error() -> str:
    return lib.psm_last_error().decode()
