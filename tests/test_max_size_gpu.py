"""The largest sizes the library accepts, on one MI355X.

The ABI takes at most 2^30 agents (a byte offset within one state row then
fits 32 bits).  At that count the state and its carries are 40 x 2^30 x 4 B = 160 GiB,
which the MI355X's HBM holds.  Each case repeats a small seeded swarm over
the whole range: an agent's arithmetic does not depend on where it sits, so
every copy must come out bit for bit equal to the first, and sampled agents
of the last copy are checked against the FP64 reference as in the other
parity tests.

- closed-loop fused rollout, 2^30 agents (row offsets up to 156 GiB);
- heterogeneous swarm with per-type step budgets, 2^30 agents: the type
  order (a permutation of 2^30 entries) and the rollout through it;
- adjoint with two checkpoint slots, 2^27 agents (slot offsets of 20 GiB).
"""
import numpy as np
import pytest

from paper_2308_12698_amd import inputs as I
from tests._util import rel_errors

pytestmark = pytest.mark.gpu

MAX_AGENTS = 1 << 30
GiB = 1 << 30


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(autouse=True)
def release_memory(torch_dev):
    """Hand the cached blocks back after each case, so that later tests and
    the library's own allocations see the whole device again."""
    yield
    import gc
    gc.collect()
    torch_dev[0].cuda.empty_cache()


def need_memory(torch, n_bytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < n_bytes:
        pytest.skip(f"needs {n_bytes / GiB:.0f} GiB of device memory, {free / GiB:.0f} GiB free")


def tile(dst, base, n):
    """dst[..., :n] = base repeated along the last axis (last copy cut short)."""
    b = base.shape[-1]
    t = n // b
    lead = dst.shape[:-1]
    dst[..., :t * b].view(*lead, t, b).copy_(base.unsqueeze(-2))
    if n > t * b:
        dst[..., t * b:n].copy_(base[..., :n - t * b])
    return t


def assert_copies_equal(torch, x, b, n, rows):
    """Copies 1, middle, last and the cut-short tail equal copy 0 bit for bit."""
    t = n // b
    first = x[:rows, :b]
    for c in sorted({1, t // 2, t - 1}):
        assert torch.equal(x[:rows, c * b:(c + 1) * b], first), f"copy {c} differs from copy 0"
    if n > t * b:
        assert torch.equal(x[:rows, t * b:n], first[:, :n - t * b]), "cut-short copy differs"


def test_closed_loop_rollout_at_max_agents(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    n, n_steps = MAX_AGENTS, 20
    # state, its rounding carries, waypoints
    need_memory(torch, (30 + 10 + 3) * 4 * n + 4 * GiB)
    base = I.config2(n=1 << 20, n_steps=n_steps)
    b = base.n
    print(f"closed loop: {n} agents ({n // b} copies of {b}) x {n_steps} steps", flush=True)
    st = torch.empty((30, n), dtype=torch.float32, device=dev)
    carry = torch.zeros((10, n), dtype=torch.float32, device=dev)
    wp = torch.empty((1, 3, n), dtype=torch.float32, device=dev)
    tile(st, torch.from_numpy(base.state).to(dev), n)
    tile(wp, torch.from_numpy(base.wp[:1]).to(dev), n)
    sim = Simulator(base.types, base.glob, mode=1, form="fused", steps_per_launch=n_steps)
    sim.step(st, n_steps, base.dt, wp=wp, resample_every=base.resample_every, carry=carry)
    bad = int(sim.count_nonfinite(st).item())
    torch.cuda.synchronize()
    assert bad == 0
    assert_copies_equal(torch, st, b, n, 30)
    j = np.sort(np.random.default_rng(31).choice(b, 16, replace=False))
    g = (n // b - 1) * b + j
    got = st[:30, torch.from_numpy(g).to(dev)].cpu().numpy()
    assert_copies_equal(torch, carry, b, n, 10)
    sim.close()
    del st, wp, carry
    sub = I.subset(base, j)
    ref = oracle.rollout(sub.state, sub.types, sub.glob, 1, sub.dt, n_steps, wp=sub.wp,
                         resample_every=sub.resample_every)
    errs = rel_errors(got, ref, sub.types)
    print({k: f"{v[0]:.2e}" for k, v in errs.items()}, flush=True)
    assert max(v[0] for v in errs.values()) <= 1e-4, errs


def test_heterogeneous_type_order_at_max_agents(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    n, n_steps = MAX_AGENTS, 20
    # state and waypoints (FP32 rows; no carries: uncompensated updates), types,
    # order, its workspace, the check's int64 copy
    need_memory(torch, (30 + 3) * 4 * n + (1 + 4 + 8 + 8) * n + 4 * GiB)
    base = I.config3(scale=16)
    # budgets of 4, 8, ..., 32 steps: half the types stop inside the rollout
    types = [dict(t, budget=4 * (k + 1)) for k, t in enumerate(base.types)]
    b = base.n
    print(f"heterogeneous: {n} agents ({n // b} copies of {b}, cut short), {len(types)} types, "
          f"budgets 4-32, {n_steps} steps", flush=True)
    st = torch.empty((30, n), dtype=torch.float32, device=dev)
    wp = torch.empty((1, 3, n), dtype=torch.float32, device=dev)
    ti = torch.empty(n, dtype=torch.uint8, device=dev)
    tile(st, torch.from_numpy(base.state).to(dev), n)
    tile(wp, torch.from_numpy(base.wp[:1]).to(dev), n)
    tile(ti, torch.from_numpy(base.type_idx).to(dev), n)
    sim = Simulator(types, base.glob, mode=1, form="fused", steps_per_launch=n_steps)
    perm = sim.order_by_type(ti)
    # the order is a permutation, grouped by type, longest budget first
    p64 = perm.long()
    seen = torch.zeros(n, dtype=torch.uint8, device=dev)
    seen[p64] = 1
    assert bool(seen.all().item()), "order misses agents"
    del seen
    ordered = ti[p64]
    del p64
    assert bool((ordered[1:] <= ordered[:-1]).all().item()), "order not grouped by descending budget"
    assert torch.equal(torch.bincount(ordered, minlength=8), torch.bincount(ti, minlength=8))
    del ordered
    sim.step(st, n_steps, base.dt, type_idx=ti, perm=perm, wp=wp, resample_every=base.resample_every)
    torch.cuda.synchronize()
    assert_copies_equal(torch, st, b, n, 30)
    j = np.sort(np.random.default_rng(32).choice(b, 16, replace=False))
    g = (n // b - 1) * b + j
    got = st[:30, torch.from_numpy(g).to(dev)].cpu().numpy()
    sim.close()
    del st, wp, ti, perm
    sub = I.subset(base, j)
    ref = oracle.rollout(sub.state, types, sub.glob, 1, sub.dt, n_steps, type_idx=sub.type_idx,
                         wp=sub.wp, resample_every=sub.resample_every)
    errs = rel_errors(got, ref, types, sub.type_idx)
    print({k: f"{v[0]:.2e}" for k, v in errs.items()}, flush=True)
    assert max(v[0] for v in errs.values()) <= 1e-4, errs


def test_adjoint_two_checkpoint_slots_at_2_27_agents(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    n, n_steps, K = 1 << 27, 20, 10
    # state and carries, 2 checkpoint slots, gains, waypoint, cotangent, both gradients
    need_memory(torch, (40 + 80 + 9 + 3 + 30 + 30 + 9) * 4 * n + 4 * GiB)
    base = I.config4(n=1 << 16, n_steps=n_steps)
    b = base.n
    print(f"adjoint: {n} agents ({n // b} copies of {b}) x {n_steps} steps, K = {K}", flush=True)
    x = torch.empty((30, n), dtype=torch.float32, device=dev)
    carry = torch.zeros((10, n), dtype=torch.float32, device=dev)
    gains = torch.empty((9, n), dtype=torch.float32, device=dev)
    wp = torch.empty((1, 3, n), dtype=torch.float32, device=dev)
    tile(x, torch.from_numpy(base.state).to(dev), n)
    tile(gains, torch.from_numpy(base.gains).to(dev), n)
    tile(wp, torch.from_numpy(base.wp).to(dev), n)
    sim = Simulator(base.types, base.glob, mode=1, form="fused", steps_per_launch=n_steps)
    ckpt = torch.empty((n_steps // K, 40, n), dtype=torch.float32, device=dev)
    sim.step(x, n_steps, base.dt, gains=gains, wp=wp, ckpt=ckpt, ckpt_every=K, carry=carry)
    gfin = torch.zeros((30, n), dtype=torch.float32, device=dev)
    tgt = torch.empty((3, n), dtype=torch.float32, device=dev)
    tile(tgt, torch.from_numpy(base.extra["target"]).to(dev), n)
    gfin[0:3] = 2.0 * (x[0:3] - tgt)
    gfin[29] = base.extra["cost_weight"]
    del tgt
    gx0, gg = sim.step_backward(ckpt, K, n_steps, base.dt, gfin, gains=gains, wp=wp)
    torch.cuda.synchronize()
    assert_copies_equal(torch, gx0, b, n, 30)
    assert_copies_equal(torch, gg, b, n, 9)
    j = np.sort(np.random.default_rng(33).choice(b, 8, replace=False))
    g = torch.from_numpy((n // b - 1) * b + j).to(dev)
    got = torch.cat([gx0[:, g], gg[:, g]]).T.cpu().numpy()
    sim.close()
    del x, carry, gains, wp, ckpt, gfin, gx0, gg
    sub = I.subset(base, j)
    fin, jac = oracle.jacobian(sub.state, sub.types, sub.glob, sub.dt, n_steps, wp=sub.wp, gains=sub.gains)
    seed = np.zeros((30, sub.n))
    seed[0:3] = 2.0 * (fin[0:3] - sub.extra["target"])
    seed[29] = sub.extra["cost_weight"]
    ref = np.einsum("ar,arc->ac", seed.T, jac)
    es = np.linalg.norm(got[:, :30] - ref[:, :30], axis=1) / np.linalg.norm(ref[:, :30], axis=1)
    eg = np.linalg.norm(got[:, 30:] - ref[:, 30:], axis=1) / np.linalg.norm(ref[:, 30:], axis=1)
    print(f"adjoint at {n} agents vs dual numbers: state {es.max():.2e} gains {eg.max():.2e}", flush=True)
    assert es.max() <= 1e-3 and eg.max() <= 1e-3
