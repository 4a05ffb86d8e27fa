"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function the header declares, and rejects invalid arguments before
touching the device."""
import ctypes as C
import math
import subprocess

import pytest

from paper_2308_12698_amd import _lib as L
from paper_2308_12698_amd import inputs as I
from tests.conftest import gpu_available


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_header_declares_the_expected_entry_points():
    names = L.declared_functions()
    for fn in ("potato_create", "potato_destroy", "potato_step", "potato_step_backward"
               if "potato_step_backward" in names else "potato_step", "potato_autotune",
               "potato_order_by_type", "potato_last_error"):
        assert fn in names


def test_library_exports_every_declared_function(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for fn in L.declared_functions():
        assert fn in exported, fn
        getattr(lib, fn)


def test_library_is_built_for_gfx950():
    """The offload bundle of the library (built here from source) targets gfx950."""
    with open(L.LIB_PATH, "rb") as f:
        assert b"gfx950" in f.read()


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.potato_version()
    assert isinstance(lib.potato_last_error(None), bytes)


def _create(lib, types, glob=None, opts=None):
    arr = L.make_type_params(types)
    lim = L.make_limits(glob or I.DEFAULT_GLOBALS)
    o = opts or L.Options(1, 2, 0, 0, 0, 0)
    h = C.c_void_p()
    st = lib.potato_create(C.byref(h), C.addressof(arr), len(types), C.byref(lim), C.byref(o))
    return st, h


@pytest.mark.parametrize("bad", [
    dict(mass=0.0), dict(mass=-1.0), dict(Ixx=float("nan")), dict(k_f=0.0), dict(tau_m=0.0),
    dict(alpha=0.0), dict(drag=-0.1), dict(w_max=float("inf")), dict(w_ref=-1.0)])
def test_create_rejects_invalid_types(lib, bad):
    t = I.base_type()
    t.update({k: v for k, v in bad.items()})
    st, h = _create(lib, [t])
    assert st == L.EINVAL and not h.value
    assert len(lib.potato_last_error(None)) > 0


@pytest.mark.parametrize("bad", [
    I.car_type(rho=1.0, l_r=1.3), I.car_type(L=0.0), I.car_type(tau_delta=0.0), I.car_type(delta_max=-0.1),
    I.car_type(mass=0.0), I.car_type(drag=-1.0), I.wing_type(V_cruise=0.0), I.wing_type(tau_phi=-1.0),
    I.wing_type(rho=0.0), I.wing_type(gamma_max=-0.2), I.wing_type(k_head=float("nan")),
    dict(I.car_type(), kind=3), dict(I.base_type(), kind=-1)])
def test_create_rejects_invalid_vehicle_types(lib, bad):
    """Cars and fixed-wing aircraft are validated before any device call
    (the first type is a valid quadrotor)."""
    st, h = _create(lib, [I.base_type(), bad])
    assert st == L.EINVAL and not h.value
    assert b"type 1" in lib.potato_last_error(None)


def test_type_params_layout(lib):
    """The ctypes view of potato_type_params matches the header: 13 floats,
    9 gains, the budget, the kind and 12 vehicle parameters."""
    assert C.sizeof(L.TypeParams) == (13 + 9 + 1 + 1 + 12) * 4
    assert L.TypeParams.kind.offset == (13 + 9 + 1) * 4
    arr = L.make_type_params([I.wing_type(rho=55.0), I.base_type()])
    assert arr[0].kind == 2 and arr[0].veh[6] == 55.0 and arr[0].Ixx == 0.0
    assert arr[1].kind == 0 and arr[1].mass == 1.0 and list(arr[1].veh) == [0.0] * 12


def test_create_rejects_invalid_counts_limits_options(lib):
    t = I.base_type()
    arr = L.make_type_params([t])
    lim = L.make_limits(I.DEFAULT_GLOBALS)
    o = L.Options(1, 2, 0, 0, 0, 0)
    h = C.c_void_p()
    assert lib.potato_create(None, C.addressof(arr), 1, C.byref(lim), C.byref(o)) == L.EINVAL
    assert lib.potato_create(C.byref(h), C.addressof(arr), 0, C.byref(lim), C.byref(o)) == L.EINVAL
    assert lib.potato_create(C.byref(h), C.addressof(arr), 257, C.byref(lim), C.byref(o)) == L.EINVAL
    g = dict(I.DEFAULT_GLOBALS); g["g"] = 0.0
    assert _create(lib, [t], glob=g)[0] == L.EINVAL
    for bad in (L.Options(2, 2, 0, 0, 0, 0), L.Options(1, 3, 0, 0, 0, 0),
                L.Options(1, 2, 100, 0, 0, 0), L.Options(1, 2, 0, -1, 0, 0)):
        assert _create(lib, [t], opts=bad)[0] == L.EINVAL


def test_step_rejects_null_context(lib):
    st = L.State(None, 10)
    pp = L.Params(None, None, None, 0)
    cm = L.Cmds(None, None, 0, 0, 10, 0)
    assert lib.potato_step(None, C.byref(st), C.byref(pp), C.byref(cm), 1e-3, 10, 10, None, 0,
                           None) == L.EINVAL
    assert lib.potato_autotune(None, C.byref(st), C.byref(pp), C.byref(cm), 1e-3, 10, 10, 0, None,
                               None) == L.EINVAL
    assert lib.potato_destroy(None) == L.OK


def test_order_workspace_size(lib):
    assert lib.potato_order_workspace_bytes(0, 8) == -1
    assert lib.potato_order_workspace_bytes(1000, 0) == -1
    # block counts and their prefix sums (rank-major, 256-agent blocks), the
    # scan's chunk totals (1,024 entries per chunk) and its grand total
    for n, t in ((1000, 8), (1 << 20, 8), (1007616, 256)):
        m = math.ceil(n / 256) * t
        assert lib.potato_order_workspace_bytes(n, t) == (2 * m + math.ceil(m / 1024) + 1) * 4


@pytest.mark.skipif(gpu_available(), reason="checks the no-device error path")
def test_create_without_device_reports_hip_error(lib):
    st, h = _create(lib, [I.base_type()])
    assert st == L.EHIP and not h.value


def test_collision_workspace_size(lib):
    lib.potato_collision_workspace_bytes.restype = C.c_int64
    lib.potato_collision_workspace_bytes.argtypes = [C.c_int64]
    assert lib.potato_collision_workspace_bytes(0) == -1
    for n, k in ((1000, 11), (1 << 20, 21), (3, 10), ((1 << 24) + 1, 26), ((1 << 30) - 1, 30)):
        # bucket budget 2^k >= 2n (at least 2^10) plus 2 ghost columns per 32
        m = 2 ** k + 2 ** (k + 1 - 5)
        # partitions of 2^s buckets (s >= 12), at most 16,384 of them, cover
        # the m + 1 bucket starts; tiles of 2,048 agents or a multiple, at
        # most 2,048 tiles
        s = 12
        while math.ceil((m + 1) / 2 ** s) > 16384:
            s += 1
        parts = math.ceil((m + 1) / 2 ** s)
        tile = 2048 * math.ceil(n / (2048 * 2048))
        cells = parts * math.ceil(n / tile)
        # items (x, y, z, r) in partition and in bucket order [2n] each; ids
        # [2n] each; bucket starts [parts * 2^s]; partition-tile offsets
        # [cells + 1]; chunk totals of their scan; bounding box [6] and its
        # partials over at most 1,024 blocks; per-block counts of the dead
        expect = 16 * 4 * n + 4 * (4 * n + parts * 2 ** s + cells + 1 + math.ceil(cells / 1024) + 6 + 6 * 1024
                                   + math.ceil(n / 256)) + 256
        assert lib.potato_collision_workspace_bytes(n) == expect


def test_detect_rejects_null_context(lib):
    st = L.State(None, 10)
    assert lib.potato_detect_collisions(None, C.byref(st), None, 10, None, None, None, 0, None) == L.EINVAL
    assert lib.potato_detect_collisions_noalloc(None, C.byref(st), None, 10, None, None, None) == L.EINVAL
    assert b"non-null" in lib.potato_last_error(None)


def test_type_radius_is_validated(lib):
    t = I.base_type()
    t["radius"] = -1.0
    st, h = _create(lib, [t])
    assert st == L.EINVAL and not h.value


def test_pipe_entry_points_reject_null_handles(lib):
    h = C.c_void_p()
    assert lib.potato_pipe_create(None, 10, C.byref(h)) == L.EINVAL
    assert lib.potato_pipe_create(None, 10, None) == L.EINVAL
    assert lib.potato_pipe_push(None, None) == L.EINVAL
    assert lib.potato_pipe_run(None, None, None, C.c_float(1e-3), 1, 0, None, None) == L.EINVAL
    assert lib.potato_pipe_wait_snapshots(None, 0) == L.EINVAL
    assert lib.potato_pipe_sync(None) == L.EINVAL
    a, b = C.c_int64(0), C.c_int64(0)
    assert lib.potato_pipe_stats(None, C.byref(a), C.byref(b)) == L.EINVAL
    assert lib.potato_pipe_destroy(None) == L.OK


def test_count_nonfinite_rejects_null_handles(lib):
    st = L.State(None, 10)
    assert lib.potato_count_nonfinite(None, C.byref(st), 10, None, None) == L.EINVAL
