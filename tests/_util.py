"""Shared test helpers: error metrics and small single-agent builders.

The parity metric follows the workload's tolerance statement: per agent and
per state group, ||x_hat - x|| / max(||x||, floor), maximum over agents and
groups.  Rotor groups are compared on absolute speeds (reference + stored
deviation) so that the floor is the hover speed, not zero.
"""
from __future__ import annotations

import math

import numpy as np

GROUPS = {
    "p": (slice(0, 3), 1.0),
    "v": (slice(3, 6), 1.0),
    "q": (slice(6, 10), 1.0),
    "w": (slice(10, 13), 1.0),
    "rotor": (slice(13, 17), None),
    "i_pos": (slice(17, 20), 1.0),
    "i_att": (slice(20, 23), 1.0),
    "i_rate": (slice(23, 26), 1.0),
    "w_prev": (slice(26, 29), 1.0),
    "J": (slice(29, 30), 1.0),
}
OPEN_LOOP_GROUPS = ("p", "v", "q", "w", "rotor")
# Cars and fixed-wing aircraft (rows 0-6): position, speed, heading, actuator
# angle (steering or bank), flight-path angle; floors 1 m, 1 m/s, 1 rad.
VEHICLE_GROUPS = {
    "p": (slice(0, 3), 1.0),
    "speed": (slice(3, 4), 1.0),
    "heading": (slice(4, 5), 1.0),
    "actuator": (slice(5, 6), 1.0),
    "path_angle": (slice(6, 7), 1.0),
}


def w_ref_per_agent(types, type_idx, n):
    w = np.array([float(t["w_ref"]) for t in types])
    return w[np.asarray(type_idx, dtype=np.int64)] if type_idx is not None else np.full(n, w[0])


def rel_errors(got, ref, types, type_idx=None, groups=None):
    """Per-group max relative error over agents: dict group -> (max, p99, argmax)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[1]
    wref = w_ref_per_agent(types, type_idx, n)
    out = {}
    for name in (groups or GROUPS):
        sl, floor = GROUPS[name]
        d = np.linalg.norm(got[sl] - ref[sl], axis=0)
        if name == "rotor":
            mag = np.linalg.norm(ref[sl] + wref[None, :], axis=0)
            den = np.maximum(mag, wref)
        else:
            den = np.maximum(np.linalg.norm(ref[sl], axis=0), floor)
        e = d / den
        e = np.where(np.isfinite(e), e, np.inf)
        out[name] = (float(e.max()) if n else 0.0, float(np.percentile(e, 99)) if n else 0.0,
                     int(e.argmax()) if n else -1)
    return out


def vehicle_rel_errors(got, ref):
    """Per-group max relative error over car and aircraft agents (columns of
    got and ref): dict group -> (max, p99, argmax)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[1]
    out = {}
    for name, (sl, floor) in VEHICLE_GROUPS.items():
        d = np.linalg.norm(got[sl] - ref[sl], axis=0)
        e = d / np.maximum(np.linalg.norm(ref[sl], axis=0), floor)
        e = np.where(np.isfinite(e), e, np.inf)
        out[name] = (float(e.max()) if n else 0.0, float(np.percentile(e, 99)) if n else 0.0,
                     int(e.argmax()) if n else -1)
    return out


def max_rel_error(got, ref, types, type_idx=None, groups=None):
    return max(v[0] for v in rel_errors(got, ref, types, type_idx, groups).values())


def rotation_matrix(q):
    """Rotation matrix of a unit quaternion (w, x, y, z), body -> inertial."""
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_from_axis_angle(axis, angle):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * a])


def single_state(p=(0, 0, 0), v=(0, 0, 0), q=(1, 0, 0, 0), w=(0, 0, 0), rotor_dev=(0, 0, 0, 0),
                 mem=None, J=0.0):
    s = np.zeros((30, 1))
    s[0:3, 0] = p
    s[3:6, 0] = v
    s[6:10, 0] = q
    s[10:13, 0] = w
    s[13:17, 0] = rotor_dev
    if mem is not None:
        s[17:29, 0] = mem
    s[29, 0] = J
    return s
