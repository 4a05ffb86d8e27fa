"""ctypes view of ``libpotato.so`` (include/potato.h), argument marshalling only.

Loading fails loudly if the library was not built: there is no fallback
implementation of the simulator anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpotato.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "potato.h")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = range(5)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EUNSUPPORTED"}
OPEN_LOOP, CLOSED_LOOP = 0, 1
FORM_AUTO, FORM_PLAIN, FORM_FUSED = 0, 1, 2

TYPE_FIELDS = ("mass", "Ixx", "Iyy", "Izz", "arm", "alpha", "k_f", "k_m", "tau_m", "drag",
               "w_max", "w_ref", "radius")
LIMIT_FIELDS = ("g", "r_sat", "ipos_max", "iatt_max", "irate_max", "az_min_frac")


class TypeParams(C.Structure):
    _fields_ = [(f, C.c_float) for f in TYPE_FIELDS] + [
        ("gains", C.c_float * 9), ("step_budget", C.c_int32), ("kind", C.c_int32),
        ("veh", C.c_float * 12)]


class Limits(C.Structure):
    _fields_ = [(f, C.c_float) for f in LIMIT_FIELDS]


class Options(C.Structure):
    _fields_ = [("mode", C.c_int32), ("form", C.c_int32), ("block", C.c_int32),
                ("steps_per_launch", C.c_int32), ("grid_blocks", C.c_int32),
                ("use_graph", C.c_int32)]


class State(C.Structure):
    _fields_ = [("rows", C.c_void_p), ("ld", C.c_int64), ("carry", C.c_void_p), ("carry_ld", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("type", C.c_void_p), ("perm", C.c_void_p), ("gains", C.c_void_p),
                ("gains_ld", C.c_int64), ("alive", C.c_void_p)]


class Cmds(C.Structure):
    _fields_ = [("motor_cmd", C.c_void_p), ("wp", C.c_void_p), ("n_epochs", C.c_int32),
                ("resample_every", C.c_int32), ("ld", C.c_int64), ("step0", C.c_int64)]


class PotatoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/potato.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(potato_[a-z_]+)\s*\(", text)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(the simulator has no non-HIP implementation)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.potato_create.argtypes = [C.POINTER(C.c_void_p), P, I32, P, P]
    L.potato_destroy.argtypes = [P]
    L.potato_set_options.argtypes = [P, P]
    L.potato_step.argtypes = [P, P, P, P, F, I64, I32, P, I32, P]
    L.potato_autotune.argtypes = [P, P, P, P, F, I64, I32, I32, P, P]
    L.potato_order_workspace_bytes.argtypes = [I64, I32]
    L.potato_order_workspace_bytes.restype = I64
    L.potato_order_by_type.argtypes = [P, P, I64, P, P, I64, P]
    L.potato_backward_workspace_bytes.argtypes = [P, P, I64, I32]
    L.potato_backward_workspace_bytes.restype = I64
    L.potato_step_backward.argtypes = [P, P, P, F, I64, I32, P, I32, I64, P, P, P, P, P, I64, P]
    L.potato_collision_workspace_bytes.argtypes = [I64]
    L.potato_collision_workspace_bytes.restype = I64
    L.potato_detect_collisions.argtypes = [P, P, P, I64, P, P, P, I64, P]
    L.potato_detect_collisions_noalloc.argtypes = [P, P, P, I64, P, P, P]
    L.potato_pipe_create.argtypes = [P, I64, C.POINTER(C.c_void_p)]
    L.potato_pipe_push.argtypes = [P, P]
    L.potato_pipe_run.argtypes = [P, P, P, F, I32, I32, P, P]
    L.potato_pipe_wait_snapshots.argtypes = [P, I64]
    L.potato_pipe_sync.argtypes = [P]
    L.potato_pipe_stats.argtypes = [P, C.POINTER(I64), C.POINTER(I64)]
    L.potato_pipe_destroy.argtypes = [P]
    L.potato_count_nonfinite.argtypes = [P, P, I64, P, P]
    L.potato_last_error.argtypes = [P]
    L.potato_last_error.restype = C.c_char_p
    L.potato_version.argtypes = []
    L.potato_version.restype = C.c_char_p
    for fn in ("potato_create", "potato_destroy", "potato_set_options", "potato_step",
               "potato_autotune", "potato_order_by_type", "potato_step_backward",
               "potato_detect_collisions", "potato_detect_collisions_noalloc", "potato_pipe_create",
               "potato_pipe_push", "potato_pipe_run", "potato_pipe_wait_snapshots", "potato_pipe_sync",
               "potato_pipe_stats", "potato_pipe_destroy", "potato_count_nonfinite"):
        getattr(L, fn).restype = C.c_int
    _lib = L
    return L


def check(status: int):
    if status != OK:
        raise PotatoError(status, load().potato_last_error(None).decode())


def make_type_params(types) -> C.Array:
    """potato_type_params of type dicts: a quadrotor (kind 0, the default)
    gives every field of TYPE_FIELDS; a car or fixed-wing aircraft (kind 1,
    2) gives mass, drag, radius and ``veh`` (other fields are sent as 0)."""
    arr = (TypeParams * len(types))()
    for i, t in enumerate(types):
        kind = int(t.get("kind", 0))
        arr[i].kind = kind
        for f in TYPE_FIELDS:
            if kind == 0:
                v = t.get(f, t["arm"]) if f == "radius" else t[f]
            else:
                v = t.get(f, 0.0)
            setattr(arr[i], f, float(v))
        for k in range(9):
            arr[i].gains[k] = float(t["gains"][k])
        if kind != 0:
            for k, v in enumerate(t.get("veh", ())):
                arr[i].veh[k] = float(v)
        arr[i].step_budget = int(min(int(t.get("budget", 2**31 - 1)), 2**31 - 1))
    return arr


def make_limits(g) -> Limits:
    lim = Limits()
    for f in LIMIT_FIELDS:
        setattr(lim, f, float(g[f]))
    return lim
