"""ctypes mirror of include/tbsma.h and the loader of libtbsma.so.

Argument marshalling only: every computation runs in the HIP library.  The
library must have been built (``paper_1311_3890_amd.build.build()``); there is
no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtbsma.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tbsma.h")

TILE = 64


def shape(tiles_per_block: int, stage_class: int) -> int:
    """TBSMA_SHAPE of include/tbsma.h."""
    return int(tiles_per_block) | (int(stage_class) << 4)


SHAPE_DEFAULT = shape(4, 1)
NOBS = 10
OK, EINVAL, ECAPACITY, EHIP, EDEVICE = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
DYN, GRIP_FIXED, GRIP_PULL, PAD = 0, 1, 2, 3
ST_OVERFLOW, ST_NONFINITE, ST_OUTSIDE, ST_RUPTURED, ST_REBUILT, ST_DONE = 1, 2, 4, 8, 16, 32
OBS_STEP, OBS_EPOT, OBS_KE, OBS_T, OBS_WZZ, OBS_SZZ, OBS_STRAIN, OBS_GAP, OBS_D, \
    OBS_STATUS = range(10)

vp = C.c_void_p


class Params(C.Structure):
    _fields_ = [("A", C.c_double), ("xi", C.c_double), ("p", C.c_double), ("q", C.c_double),
                ("r0", C.c_double), ("r_tail", C.c_double), ("r_cut", C.c_double),
                ("skin", C.c_double), ("cell", C.c_double), ("mass", C.c_double),
                ("precision", C.c_int32), ("qbits", C.c_int32), ("prune", C.c_double),
                ("gather", C.c_int32), ("rebuild_exact", C.c_int32)]


class System(C.Structure):
    _fields_ = [("R", C.c_int32), ("max_zbins", C.c_int32), ("N", C.c_int64), ("C", C.c_int64),
                ("rep_off_h", vp), ("cell_off_h", vp), ("rep_off", vp), ("cell_off", vp),
                ("tile_rep", vp), ("grid_dim", vp), ("grid_lo", vp), ("rep_id", vp),
                ("x", vp), ("y", vp), ("z", vp), ("vx", vp), ("vy", vp), ("vz", vp),
                ("z0", vp), ("flag", vp), ("qpos", vp), ("tag", vp),
                ("shape_h", vp), ("shape", vp)]


class Cells(C.Structure):
    _fields_ = [("cell_start", vp), ("cell_atoms", vp)]


class NList(C.Structure):
    _fields_ = [("nl", vp), ("nn", vp), ("k_cap", C.c_int32), ("reserved", C.c_int32),
                ("x_ref", vp), ("y_ref", vp), ("z_ref", vp), ("nact", vp), ("nl_lane", vp)]


class ForcesOut(C.Structure):
    _fields_ = [("fx", vp), ("fy", vp), ("fz", vp), ("e_atom", vp), ("g", vp),
                ("rep_energy", vp), ("rep_wzz", vp)]


class MD(C.Structure):
    _fields_ = [("dt", C.c_double), ("gamma", C.c_double), ("lab_frame", C.c_int32),
                ("n_log", C.c_int32), ("n_slots", C.c_int32), ("reserved", C.c_int32),
                ("T", vp), ("v_pull", vp), ("z_lo", vp), ("z_hi", vp), ("vol", vp), ("L0", vp),
                ("seed", vp), ("dof", vp), ("step", vp), ("obs", vp), ("status", vp),
                ("retire", C.c_double), ("dfail", vp), ("nh_tau", C.c_double), ("nh_xi", vp),
                ("nh_eta", vp), ("grip_step", C.c_double), ("grip_hold", C.c_int64),
                ("T_start", vp), ("ramp_begin", C.c_int64), ("ramp_steps", C.c_int64),
                ("baro_mass", C.c_double), ("baro_load", C.c_double), ("baro_damp", C.c_double),
                ("baro_s", vp)]


P = C.POINTER
SIGNATURES = {
    "tbsma_workspace_query": (C.c_int, [P(Params), P(System), P(C.c_size_t)]),
    "tbsma_workspace_init": (C.c_int, [P(Params), P(System), vp, vp]),
    "tbsma_build_wire": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                   C.c_double, vp, vp, vp, vp, C.c_int64, P(C.c_int64)]),
    "tbsma_init_state": (C.c_int, [P(Params), P(System), P(MD), vp, C.c_double, vp]),
    "tbsma_replica_constants": (C.c_int, [P(Params), P(System), vp, vp, vp, vp, vp]),
    "tbsma_rebase": (C.c_int, [P(Params), P(System), vp, vp, vp]),
    "tbsma_build_cells": (C.c_int, [P(Params), P(System), P(Cells), vp, vp]),
    "tbsma_neighbors": (C.c_int, [P(Params), P(System), P(Cells), P(NList), vp,
                                  P(C.c_int32), vp]),
    "tbsma_forces": (C.c_int, [P(Params), P(System), P(NList), P(ForcesOut), vp, vp]),
    "tbsma_forces_pass": (C.c_int, [P(Params), P(System), P(NList), P(ForcesOut), vp, C.c_int32,
                                    vp]),
    "tbsma_step": (C.c_int, [P(Params), P(System), P(Cells), P(NList), P(ForcesOut), P(MD),
                             vp, C.c_int64, vp]),
    "tbsma_run_batch": (C.c_int, [P(Params), P(System), P(Cells), P(NList), P(ForcesOut),
                                  P(MD), vp, C.c_int64, C.c_int32, vp]),
    "tbsma_step_noalloc": (C.c_int, [P(Params), P(System), P(Cells), P(NList), P(ForcesOut),
                                     P(MD), C.c_int64, vp]),
    "tbsma_list_stats": (C.c_int, [P(Params), P(System), P(NList), vp, P(C.c_int64), vp]),
    "tbsma_rng_fill": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_int64,
                                 vp, vp, vp]),
    "tbsma_rng_normals_f32": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32,
                                        C.c_int64, vp, vp]),
    "tbsma_event_counts": (C.c_int, [P(Params), P(System), vp, P(C.c_int64), vp]),
    "tbsma_last_error": (C.c_char_p, []),
}


class TbsmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtbsma error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libtbsma.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1311_3890_amd.build.build() "
                "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != OK:
        raise TbsmaError(code, lib().tbsma_last_error().decode())
    return code
