"""ctypes binding of the FP64 CPU reference (``oracle.cpp`` for the
quadrotors, ``vehicles.cpp`` for the cars and fixed-wing aircraft).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the simulator.  It imports nothing
from the simulator package; callers hand it plain numpy arrays and dicts
(the seeded generator's output widened to float64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.cpp")
SOURCES = (SRC_PATH, os.path.join(HERE, "vehicles.cpp"))

TYPE_FIELDS = ("mass", "Ixx", "Iyy", "Izz", "arm", "alpha", "k_f", "k_m",
               "tau_m", "drag", "w_max", "w_ref")
GLOBAL_FIELDS = ("g", "r_sat", "ipos_max", "iatt_max", "irate_max", "az_min_frac")


class OracleType(C.Structure):
    _fields_ = [(f, C.c_double) for f in TYPE_FIELDS] + [
        ("gains", C.c_double * 9), ("step_budget", C.c_int64)]


class OracleVehicle(C.Structure):
    _fields_ = [("kind", C.c_int64), ("mass", C.c_double), ("drag", C.c_double),
                ("veh", C.c_double * 12), ("step_budget", C.c_int64)]


class OracleGlobals(C.Structure):
    _fields_ = [(f, C.c_double) for f in GLOBAL_FIELDS]


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (FP64, no contraction, OpenMP)."""
    newest = max(os.path.getmtime(p) for p in SOURCES)
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < newest:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", *SOURCES, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.oracle_rollout.argtypes = [P, I, P, I, I, P, I64, I64, P, P, I64, P, P, I, I, I64,
                                     I64, D, I64, I]
        L.oracle_jacobian.argtypes = [P, I, P, P, I64, I64, P, P, I64, P, I, I, I64, I64, D,
                                      I64, P, I]
        L.oracle_derivative.argtypes = [P, D, P, P, P]
        L.oracle_controller.argtypes = [P, P, P, P, P, P, D, P]
        L.oracle_allocation.argtypes = [P, P, P]
        L.oracle_count_ops.argtypes = [P, P, I, D, P]
        L.oracle_detect_collisions.argtypes = [P, I64, I64, P, P, I, P]
        L.oracle_detect_collisions.restype = C.c_int64
        L.oracle_collides.argtypes = [P, I64, I64, P, P, I, P, P, I64, P, I]
        L.oracle_collides.restype = C.c_int
        L.oracle_vehicle_rollout.argtypes = [P, I, D, I, P, I64, I64, P, P, P, I, I, I64, I64, D,
                                             I64, I]
        L.oracle_vehicle_derivative.argtypes = [P, D, P, P, P]
        L.oracle_vehicle_guidance.argtypes = [P, D, P, P, P]
        for fn in ("oracle_vehicle_rollout", "oracle_vehicle_derivative", "oracle_vehicle_guidance"):
            getattr(L, fn).restype = C.c_int
        for fn in ("oracle_rollout", "oracle_jacobian", "oracle_derivative", "oracle_controller",
                   "oracle_allocation", "oracle_count_ops", "oracle_max_threads"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def make_type(t: dict) -> OracleType:
    """Widen one type dict (float32 scalars, gains, budget) to FP64."""
    o = OracleType()
    for f in TYPE_FIELDS:
        setattr(o, f, float(t[f]))
    for k in range(9):
        o.gains[k] = float(t["gains"][k])
    o.step_budget = int(t["budget"])
    return o


def make_types(types) -> C.Array:
    arr = (OracleType * len(types))()
    for i, t in enumerate(types):
        arr[i] = make_type(t)
    return arr


def make_vehicle(t: dict) -> OracleVehicle:
    """Widen one car or fixed-wing type dict to FP64."""
    o = OracleVehicle()
    o.kind = int(t["kind"])
    o.mass, o.drag = float(t["mass"]), float(t["drag"])
    for k, v in enumerate(t["veh"]):
        o.veh[k] = float(v)
    o.step_budget = int(t["budget"])
    return o


def make_globals(g: dict) -> OracleGlobals:
    o = OracleGlobals()
    for f in GLOBAL_FIELDS:
        setattr(o, f, float(g[f]))
    return o


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def threads_default() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def rollout(state, types, glob, mode, dt, n_steps, *, type_idx=None, gains=None,
            motor_cmd=None, wp=None, resample_every=0, step0=0, renorm=True, threads=None):
    """Advance a copy of ``state`` ([30, N], widened to FP64) and return it."""
    s = np.array(state, dtype=np.float64, copy=True, order="C")
    n = s.shape[1]
    ti = None if type_idx is None else np.ascontiguousarray(type_idx, dtype=np.int32)
    gn, mc, w = _f64(gains), _f64(motor_cmd), _f64(wp)
    ne = 0 if w is None else w.shape[0]
    cmd_ld = n
    tarr, garr = make_types(types), make_globals(glob)
    rc = lib().oracle_rollout(C.addressof(tarr), len(types), C.addressof(garr), int(mode),
                              int(bool(renorm)), _p(s), n, n, _p(ti), _p(gn), n, _p(mc), _p(w),
                              ne, int(resample_every), cmd_ld, int(step0), float(dt),
                              int(n_steps), int(threads or threads_default()))
    if rc != 0:
        raise ValueError("oracle_rollout rejected its arguments")
    return s


def kind_of(t: dict) -> int:
    """Vehicle kind of a type dict: 0 quadrotor (the default), 1 car, 2 fixed wing."""
    return int(t.get("kind", 0))


def vehicle_rollout(state, types, g, mode, dt, n_steps, *, type_idx=None, motor_cmd=None, wp=None,
                    resample_every=0, step0=0, threads=None):
    """Advance a copy of ``state`` ([30, N]) of cars and fixed-wing aircraft
    (every type in ``types`` of kind 1 or 2) and return it."""
    s = np.array(state, dtype=np.float64, copy=True, order="C")
    n = s.shape[1]
    ti = None if type_idx is None else np.ascontiguousarray(type_idx, dtype=np.int32)
    mc, w = _f64(motor_cmd), _f64(wp)
    ne = 0 if w is None else w.shape[0]
    arr = (OracleVehicle * len(types))()
    for i, t in enumerate(types):
        arr[i] = make_vehicle(t)
    rc = lib().oracle_vehicle_rollout(C.addressof(arr), len(types), float(g), int(mode), _p(s), n, n, _p(ti),
                                      _p(mc), _p(w), ne, int(resample_every), n, int(step0), float(dt),
                                      int(n_steps), int(threads or threads_default()))
    if rc != 0:
        raise ValueError("oracle_vehicle_rollout rejected its arguments")
    return s


def rollout_kinds(state, types, glob, mode, dt, n_steps, *, type_idx=None, gains=None, motor_cmd=None,
                  wp=None, resample_every=0, step0=0, threads=None):
    """``rollout`` of a swarm that mixes vehicle kinds: each kind's agents go
    through its own reference (quadrotors through ``oracle_rollout``, cars
    and fixed-wing aircraft through ``oracle_vehicle_rollout``) with the
    type table restricted to that kind; per-agent gains apply to the
    quadrotors."""
    s = np.array(state, dtype=np.float64, copy=True, order="C")
    n = s.shape[1]
    ti = np.zeros(n, dtype=np.int64) if type_idx is None else np.asarray(type_idx, dtype=np.int64)
    kinds = np.array([kind_of(t) for t in types])
    agent_kind = kinds[np.minimum(ti, len(types) - 1)]
    cols = lambda a, idx, ax: None if a is None else np.ascontiguousarray(np.take(a, idx, axis=ax))
    for group in ((0,), (1, 2)):
        tsel = [k for k in range(len(types)) if kinds[k] in group]
        idx = np.where(np.isin(agent_kind, group))[0]
        if idx.size == 0:
            continue
        remap = np.full(len(types), -1, dtype=np.int64)
        remap[tsel] = np.arange(len(tsel))
        sub_ti = remap[ti[idx]]
        sub_types = [types[k] for k in tsel]
        kw = dict(type_idx=sub_ti, motor_cmd=cols(motor_cmd, idx, 1), wp=cols(wp, idx, 2),
                  resample_every=resample_every, step0=step0, threads=threads)
        if group == (0,):
            out = rollout(s[:, idx], sub_types, glob, mode, dt, n_steps, gains=cols(gains, idx, 1), **kw)
        else:
            out = vehicle_rollout(s[:, idx], sub_types, glob["g"], mode, dt, n_steps, **kw)
        s[:, idx] = out
    return s


def vehicle_derivative(t: dict, g: float, x, u):
    """Right-hand side of one car or fixed-wing aircraft: x[7], u[3] -> dx[7]."""
    x = _f64(x); u = _f64(u); dx = np.zeros(7)
    o = make_vehicle(t)
    if lib().oracle_vehicle_derivative(C.byref(o), float(g), _p(x), _p(u), _p(dx)) != 0:
        raise ValueError("oracle_vehicle_derivative rejected its arguments")
    return dx


def vehicle_guidance(t: dict, g: float, x, wp):
    """Closed-loop inputs u[3] of one car or fixed-wing aircraft."""
    x = _f64(x); w = _f64(wp); u = np.zeros(3)
    o = make_vehicle(t)
    if lib().oracle_vehicle_guidance(C.byref(o), float(g), _p(x), _p(w), _p(u)) != 0:
        raise ValueError("oracle_vehicle_guidance rejected its arguments")
    return u


def jacobian(state, types, glob, dt, n_steps, *, wp, type_idx=None, gains=None,
             resample_every=0, step0=0, threads=None):
    """Closed-loop rollout with forward-mode dual numbers.

    Returns (final state [30, N], jac [N, 30, 39]) where jac[a, r, c] is
    d x_N[r] / d (x0[0..29], gains[0..8])[c] of agent a.
    """
    s = np.array(state, dtype=np.float64, copy=True, order="C")
    n = s.shape[1]
    jac = np.zeros((n, 30, 39), dtype=np.float64)
    ti = None if type_idx is None else np.ascontiguousarray(type_idx, dtype=np.int32)
    gn, w = _f64(gains), _f64(wp)
    tarr, garr = make_types(types), make_globals(glob)
    rc = lib().oracle_jacobian(C.addressof(tarr), len(types), C.addressof(garr), _p(s), n, n,
                               _p(ti), _p(gn), n, _p(w), w.shape[0], int(resample_every), n,
                               int(step0), float(dt), int(n_steps), _p(jac),
                               int(threads or threads_default()))
    if rc != 0:
        raise ValueError("oracle_jacobian rejected its arguments")
    return s, jac


def derivative(t: dict, g: float, x, wcmd):
    """f(x) of one agent; x[18] with absolute rotor speeds (rows 13-16) and J last."""
    x = _f64(x); wc = _f64(wcmd); dx = np.zeros(18)
    o = make_type(t)
    if lib().oracle_derivative(C.byref(o), float(g), _p(x), _p(wc), _p(dx)) != 0:
        raise ValueError("oracle_derivative failed")
    return dx


def controller(t: dict, glob: dict, x, mem, wp, dt, gains=None):
    """One controller evaluation; returns (absolute rotor commands[4], new memory[12])."""
    x = _f64(x); m = np.array(mem, dtype=np.float64, copy=True); w = _f64(wp)
    gn = _f64(gains); out = np.zeros(4)
    o, gl = make_type(t), make_globals(glob)
    if lib().oracle_controller(C.byref(o), C.byref(gl), _p(gn), _p(x), _p(m), _p(w), float(dt),
                               _p(out)) != 0:
        raise ValueError("oracle_controller failed")
    return out, m


def allocation(t: dict):
    """(G, G^-1) of eq. (3) for one type."""
    G = np.zeros((4, 4)); Gi = np.zeros((4, 4))
    o = make_type(t)
    if lib().oracle_allocation(C.byref(o), _p(G), _p(Gi)) != 0:
        raise ValueError("singular allocation matrix")
    return G, Gi


PARTS = ("controller", "derivative", "rk4", "renorm")
OP_KINDS = ("add", "mul", "div", "sqrt", "cmp", "rev")


def count_ops(t: dict, glob: dict, mode: int, dt: float) -> dict:
    """Operations of one agent-step, by part (the counting rules are stated
    at ``oracle_count_ops``): ``{part: {add, mul, div, sqrt, cmp, rev,
    flops}}`` for the controller, one right-hand-side evaluation, the RK4
    arithmetic outside the four evaluations and the renormalisation, plus
    ``"flops"`` (forward flops of the whole step: controller + 4 f + RK4 +
    renormalisation) and ``"rev_flops"`` (flops of the whole step's reverse
    sweep)."""
    c = np.zeros(24, dtype=np.int64)
    o, gl = make_type(t), make_globals(glob)
    if lib().oracle_count_ops(C.byref(o), C.byref(gl), int(mode), float(dt), _p(c)) != 0:
        raise ValueError("oracle_count_ops failed")
    out = {}
    for p, part in enumerate(PARTS):
        d = dict(zip(OP_KINDS, (int(v) for v in c[6 * p:6 * p + 6])))
        d["flops"] = d["add"] + d["mul"] + d["div"] + d["sqrt"]
        out[part] = d
    mult = {"controller": 1, "derivative": 4, "rk4": 1, "renorm": 1}
    out["flops"] = sum(mult[p] * out[p]["flops"] for p in PARTS)
    out["rev_flops"] = sum(mult[p] * out[p]["rev"] for p in PARTS)
    out["sqrt"] = sum(mult[p] * out[p]["sqrt"] for p in PARTS)
    return out


def detect_collisions(rows, radius, alive, type_idx=None):
    """Brute-force FP32 collision check; returns (new alive mask, number that died)."""
    r = np.ascontiguousarray(np.asarray(rows)[:3], dtype=np.float32)
    n = r.shape[1]
    a = np.array(alive, dtype=np.uint8, copy=True)
    rad = np.ascontiguousarray(radius, dtype=np.float32)
    ti = None if type_idx is None else np.ascontiguousarray(type_idx, dtype=np.int32)
    died = lib().oracle_detect_collisions(_p(r), n, n, _p(ti), _p(rad), int(rad.size), _p(a))
    if died < 0:
        raise ValueError("oracle_detect_collisions rejected its arguments")
    return a, int(died)


def collides(rows, radius, alive, query, type_idx=None, threads=None):
    """Collision decision of the agents ``query`` against all alive agents."""
    r = np.ascontiguousarray(np.asarray(rows)[:3], dtype=np.float32)
    n = r.shape[1]
    a = np.ascontiguousarray(alive, dtype=np.uint8)
    rad = np.ascontiguousarray(radius, dtype=np.float32)
    ti = None if type_idx is None else np.ascontiguousarray(type_idx, dtype=np.int32)
    qi = np.ascontiguousarray(query, dtype=np.int64)
    hit = np.zeros(qi.size, dtype=np.uint8)
    if lib().oracle_collides(_p(r), n, n, _p(ti), _p(rad), int(rad.size), _p(a), _p(qi), qi.size,
                             _p(hit), int(threads or threads_default())) != 0:
        raise ValueError("oracle_collides rejected its arguments")
    return hit


def max_threads() -> int:
    return int(lib().oracle_max_threads())
