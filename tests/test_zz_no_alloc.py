"""The allocation-free collision entry point, through the C ABI.

potato_detect_collisions_noalloc must take the same decisions as
potato_detect_collisions (bit for bit: the mask is integer output) on
consecutive calls that share the library's static workspace, the second
with a smaller swarm than the first, so stale contents of the larger call
must not leak into the smaller one.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2308_12698_amd import _lib as L
from paper_2308_12698_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def dense_state(n, box, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * np.asarray(box, dtype=np.float64)[:, None]
    return I.hover_state(pos)


class Ctx:
    def __init__(self, types):
        self.lib = L.load()
        self.types = L.make_type_params(types)
        self.lim = L.make_limits(I.globals_f32())
        self.opts = L.Options(L.CLOSED_LOOP, L.FORM_FUSED, 0, 0, 0, 0)
        h = C.c_void_p()
        L.check(self.lib.potato_create(C.byref(h), C.addressof(self.types), len(types), C.byref(self.lim),
                                       C.byref(self.opts)))
        self.h = h

    def close(self):
        self.lib.potato_destroy(self.h)


def run_both(torch, dev, ctx, state, alive, type_idx=None):
    """(mask, died) of the workspace entry point and of the allocation-free
    one on the same inputs."""
    n = state.shape[1]
    st = torch.from_numpy(state).to(dev)
    S = L.State(C.c_void_p(st.data_ptr()), st.stride(0), None, 0)
    ti = None if type_idx is None else torch.from_numpy(type_idx).to(dev)
    P = L.Params(None if ti is None else C.c_void_p(ti.data_ptr()), None, None, 0, None)
    out = []
    for noalloc in (False, True):
        a = torch.from_numpy(alive.copy()).to(dev)
        died = torch.zeros(1, dtype=torch.int64, device=dev)
        if noalloc:
            rc = ctx.lib.potato_detect_collisions_noalloc(ctx.h, C.byref(S), C.byref(P), n,
                                                          C.c_void_p(a.data_ptr()), C.c_void_p(died.data_ptr()),
                                                          None)
        else:
            nbytes = int(ctx.lib.potato_collision_workspace_bytes(n))
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            rc = ctx.lib.potato_detect_collisions(ctx.h, C.byref(S), C.byref(P), n, C.c_void_p(a.data_ptr()),
                                                  C.c_void_p(died.data_ptr()), C.c_void_p(ws.data_ptr()), nbytes,
                                                  None)
        L.check(rc)
        torch.cuda.synchronize()
        out.append((a.cpu().numpy(), int(died.item())))
    return out


def test_noalloc_matches_the_workspace_entry_point(oracle, torch_dev):
    torch, dev = torch_dev
    print("no-alloc collisions: 1,048,576 then 30,001 agents", flush=True)
    ctx = Ctx([I.base_type()])
    try:
        # first call at the static workspace's limit, densely packed
        n1 = 1 << 20
        state1 = dense_state(n1, (120, 120, 20), seed=5)
        alive1 = (np.random.default_rng(6).random(n1) > 0.02).astype(np.uint8)
        (ref1, rd1), (got1, gd1) = run_both(torch, dev, ctx, state1, alive1)
        assert np.array_equal(got1, ref1) and gd1 == rd1 and rd1 > 0
        # second call, smaller: stale buckets and sorted slots of the first
        # call must not change its decisions; the brute-force reference
        # anchors both entry points
        n2 = 30001
        state2 = dense_state(n2, (60, 60, 10), seed=n2)
        alive2 = (np.random.default_rng(1).random(n2) > 0.05).astype(np.uint8)
        (ref2, rd2), (got2, gd2) = run_both(torch, dev, ctx, state2, alive2)
        assert np.array_equal(got2, ref2) and gd2 == rd2
        bf, bf_died = oracle.detect_collisions(state2, [I.base_type()["radius"]], alive2)
        assert np.array_equal(got2, bf) and gd2 == bf_died
    finally:
        ctx.close()


def test_noalloc_with_type_radii_and_a_second_context(torch_dev):
    """A second context on the same GPU shares the static workspace; per-type
    radii go through the type index as in the workspace entry point."""
    torch, dev = torch_dev
    types = I.hetero_types()
    a, b = Ctx(types), Ctx([I.base_type()])
    try:
        n = 15000
        state = dense_state(n, (25, 25, 5), seed=7)
        ti = np.random.default_rng(3).integers(0, 8, n).astype(np.uint8)
        (ref, rd), (got, gd) = run_both(torch, dev, a, state, np.ones(n, np.uint8), ti)
        assert np.array_equal(got, ref) and gd == rd
        state = dense_state(4000, (10, 10, 3), seed=8)
        (ref, rd), (got, gd) = run_both(torch, dev, b, state, np.ones(4000, np.uint8))
        assert np.array_equal(got, ref) and gd == rd
    finally:
        a.close()
        b.close()


def test_noalloc_rejects_swarms_beyond_its_limit(torch_dev):
    """Host-detected: nothing is enqueued for n_agents above the limit."""
    torch, dev = torch_dev
    ctx = Ctx([I.base_type()])
    try:
        n = (1 << 20) + 1
        st = torch.zeros((30, n), dtype=torch.float32, device=dev)
        S = L.State(C.c_void_p(st.data_ptr()), n, None, 0)
        P = L.Params(None, None, None, 0, None)
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        rc = ctx.lib.potato_detect_collisions_noalloc(ctx.h, C.byref(S), C.byref(P), n, C.c_void_p(a.data_ptr()),
                                                      None, None)
        assert rc == L.EINVAL
        assert b"exceeds" in ctx.lib.potato_last_error(None)
        torch.cuda.synchronize()
        assert int(a.min().item()) == 1
    finally:
        ctx.close()
