"""Collision detection on the GPU (hashed grid) against the brute-force
reference, and dead agents excluded from the step and the adjoint.

The collision decision is integer output, so parity is bit-exact: both sides
take the FP32 decision with the same operation order.
"""
import numpy as np
import pytest

from paper_2308_12698_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def dense_swarm(n, box, seed):
    """Hovering swarm packed densely enough that many pairs overlap."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * np.asarray(box, dtype=np.float64)[:, None]
    return I.hover_state(pos)


def gpu_detect(torch_dev, state, types, alive, type_idx=None):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sim = Simulator(types, I.globals_f32(), mode=1)
    st = torch.from_numpy(state).to(dev)
    a = torch.from_numpy(alive.copy()).to(dev)
    died = torch.zeros(1, dtype=torch.int64, device=dev)
    ti = None if type_idx is None else torch.from_numpy(type_idx).to(dev)
    sim.detect_collisions(st, a, type_idx=ti, died=died)
    torch.cuda.synchronize()
    sim.close()
    return a.cpu().numpy(), int(died.item())


@pytest.mark.parametrize("n,box", [(1, (1, 1, 1)), (20000, (20, 20, 5)), (30001, (60, 60, 10))])
def test_detection_matches_brute_force(oracle, torch_dev, n, box):
    state = dense_swarm(n, box, seed=n)
    t = I.base_type()
    alive = (np.random.default_rng(1).random(n) > 0.05).astype(np.uint8)
    got, died = gpu_detect(torch_dev, state, [t], alive)
    ref, ref_died = oracle.detect_collisions(state, [t["radius"]], alive)
    assert np.array_equal(got, ref) and died == ref_died
    print(f"collisions n={n}: {ref_died} died", flush=True)


def test_detection_degenerate_geometry(oracle, torch_dev):
    """Coincident agents (one cell holds 1,500), pairs far from the origin,
    huge negative coordinates, NaN and infinite positions: the same
    decisions as the brute-force reference (a NaN or infinite position never
    passes the distance test)."""
    rng = np.random.default_rng(99)
    n = 4000
    pos = np.empty((3, n))
    pos[:, 0:1500] = np.array([[10.0], [10.0], [10.0]])
    base = np.stack([rng.uniform(-1e5, 1e5, 250), rng.uniform(-1e5, 1e5, 250), np.full(250, 5e4)])
    pos[:, 1500:2000:2] = base
    pos[:, 1501:2000:2] = base + np.array([[0.2], [0.0], [0.0]])
    pos[:, 2000:3000] = rng.uniform(-3e6, -2.9e6, size=(3, 1000))
    pos[:, 3000:3100] = rng.uniform(0.0, 50.0, size=(3, 100))
    pos[0, 3000:3050] = np.nan
    pos[1, 3050:3100] = np.nan
    pos[:, 3100:3200] = rng.uniform(0.0, 50.0, size=(3, 100))
    pos[2, 3100:3150] = np.inf
    pos[0, 3150:3200] = -np.inf
    pos[:, 3200:] = rng.uniform(0.0, 50.0, size=(3, n - 3200))
    state = I.hover_state(pos.astype(np.float32).astype(np.float64))
    alive = np.ones(n, np.uint8)
    alive[::97] = 0
    t = I.base_type()
    got, died = gpu_detect(torch_dev, state, [t], alive)
    ref, ref_died = oracle.detect_collisions(state, [t["radius"]], alive)
    assert np.array_equal(got, ref) and died == ref_died
    assert not got[0:1500][alive[0:1500] == 1].any()           # the coincident cluster
    assert got[3000:3200][alive[3000:3200] == 1].all()          # NaN / infinite positions
    print(f"degenerate geometry: {ref_died} died", flush=True)


def test_detection_dense_cluster(oracle, torch_dev):
    """5,000 agents at one point among 7,000 spread ones: the cluster's bucket
    partition holds more items than the sort assembles in LDS, so it takes
    the two-read placement; the same decisions as the brute-force
    reference."""
    rng = np.random.default_rng(5)
    n = 12000
    pos = np.empty((3, n))
    pos[:, :5000] = np.array([[10.0], [10.0], [5.0]])
    pos[:, 5000:] = rng.uniform(0.0, 1.0, size=(3, n - 5000)) * np.array([[50.0], [50.0], [10.0]])
    state = I.hover_state(pos.astype(np.float32).astype(np.float64))
    alive = (rng.random(n) > 0.1).astype(np.uint8)
    t = I.base_type()
    got, died = gpu_detect(torch_dev, state, [t], alive)
    ref, ref_died = oracle.detect_collisions(state, [t["radius"]], alive)
    assert np.array_equal(got, ref) and died == ref_died
    assert not got[:5000].any()


def test_detection_thin_line(oracle, torch_dev):
    """6,000 agents along a 1 km line of cells: two per cell, at opposite
    corners of its y-z section, one cell apart along x with +-5 cm of
    jitter, so neighbours along the line collide or not by the jitter.  The
    grid then has one y row and one z layer (the 9 row ranges of every
    query coincide), and one bucket partition holds more items than the sort
    assembles in LDS, spread over 3,000 buckets.  The same decisions as the
    brute-force reference."""
    rng = np.random.default_rng(6)
    t = I.base_type()
    h = np.float32(2.02) * np.float32(t["radius"])          # cell edge
    n = 6000
    cells = np.repeat(np.arange(n // 2), 2)
    pos = np.empty((3, n))
    pos[0] = (cells + 0.5) * h + rng.uniform(-0.05, 0.05, n)
    pos[1] = np.where(np.arange(n) % 2 == 0, 8.05, 8.95) * h
    pos[2] = np.where(np.arange(n) % 2 == 0, 20.05, 20.95) * h
    state = I.hover_state(pos.astype(np.float32).astype(np.float64))
    alive = (rng.random(n) > 0.05).astype(np.uint8)
    got, died = gpu_detect(torch_dev, state, [t], alive)
    ref, ref_died = oracle.detect_collisions(state, [t["radius"]], alive)
    assert np.array_equal(got, ref) and died == ref_died
    assert 0 < died < int(alive.sum())


def test_detection_with_type_radii(oracle, torch_dev):
    n = 15000
    state = dense_swarm(n, (25, 25, 5), seed=7)
    types = I.hetero_types()
    ti = np.random.default_rng(3).integers(0, 8, n).astype(np.uint8)
    alive = np.ones(n, np.uint8)
    got, died = gpu_detect(torch_dev, state, types, alive, ti)
    radii = [t["radius"] for t in types]
    ref, ref_died = oracle.detect_collisions(state, radii, alive, type_idx=ti)
    assert np.array_equal(got, ref) and died == ref_died


def test_detection_full_size_sampled(oracle, torch_dev):
    """The 1,048,576-agent scale swarm: every agent's decision for a sample of
    4,096 agents, each against all others, from the reference."""
    sw = I.config2()
    alive = np.ones(sw.n, np.uint8)
    got, died = gpu_detect(torch_dev, sw.state, sw.types, alive)
    q = np.random.default_rng(9).choice(sw.n, 4096, replace=False)
    hit = oracle.collides(sw.state, [sw.types[0]["radius"]], alive, q)
    assert np.array_equal(got[q] == 0, hit == 1)
    assert died == int((got == 0).sum()) > 0


def test_detection_two_sort_windows_per_partition(oracle, torch_dev):
    """16,777,217 agents at the scale swarm's density: the sort's bucket
    partitions then hold two windows of 4,096 buckets each (one window per
    partition would take more than 16,384 partitions).  Every decision of a
    sample of 512 agents, each against all others, and of the first and
    last agent."""
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    n = (1 << 24) + 1
    rng = np.random.default_rng(24)
    pos = rng.random((3, n), dtype=np.float32) * np.array([[400.0], [400.0], [20.0]], np.float32)
    t = I.base_type()
    sim = Simulator([t], I.globals_f32(), mode=1)
    st = torch.zeros((30, n), dtype=torch.float32, device=dev)
    st[:3] = torch.from_numpy(pos).to(dev)
    a = torch.ones(n, dtype=torch.uint8, device=dev)
    died = torch.zeros(1, dtype=torch.int64, device=dev)
    sim.detect_collisions(st, a, died=died)
    torch.cuda.synchronize()
    got = a.cpu().numpy()
    sim.close()
    del st
    q = np.concatenate([[0, n - 1], rng.choice(n, 512, replace=False)])
    hit = oracle.collides(pos, [t["radius"]], np.ones(n, np.uint8), q)
    assert np.array_equal(got[q] == 0, hit == 1)
    assert died.item() == int((got == 0).sum()) > 0 and hit.any() and not hit.all()
    print(f"collisions n={n}: {died.item()} died", flush=True)


def test_died_accumulates_over_calls_on_one_workspace(oracle, torch_dev):
    """Three passes over one workspace that starts filled with 0xff bytes:
    each pass adds its own count of dead agents to ``died`` and matches the
    reference."""
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    n = 20000
    state = dense_swarm(n, (20, 20, 5), seed=11)
    t = I.base_type()
    sim = Simulator([t], I.globals_f32(), mode=1)
    st = torch.from_numpy(state).to(dev)
    ws = torch.full((int(sim._lib.potato_collision_workspace_bytes(n)),), 255, dtype=torch.uint8, device=dev)
    died = torch.zeros(1, dtype=torch.int64, device=dev)
    total = 0
    for seed in range(3):
        alive = (np.random.default_rng(seed).random(n) > 0.3).astype(np.uint8)
        a = torch.from_numpy(alive).to(dev)
        sim.detect_collisions(st, a, died=died, workspace=ws)
        ref, ref_died = oracle.detect_collisions(state, [t["radius"]], alive)
        assert np.array_equal(a.cpu().numpy(), ref)
        total += ref_died
        assert died.item() == total > 0
    sim.close()


def test_second_pass_is_a_fixed_point(torch_dev):
    """After one pass no two alive agents overlap, so a second pass kills none."""
    state = dense_swarm(20000, (20, 20, 5), seed=2)
    t = I.base_type()
    a1, d1 = gpu_detect(torch_dev, state, [t], np.ones(20000, np.uint8))
    a2, d2 = gpu_detect(torch_dev, state, [t], a1)
    assert d1 > 0 and d2 == 0 and np.array_equal(a1, a2)


def test_dead_agents_are_not_advanced(torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config1(n=3000)
    alive = (np.arange(sw.n) % 4 != 0).astype(np.uint8)
    sim = Simulator(sw.types, sw.glob, mode=1, steps_per_launch=64)
    st = torch.from_numpy(sw.state).to(dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    sim.step(st, 300, sw.dt, wp=wp, alive=torch.from_numpy(alive).to(dev))
    ref = torch.from_numpy(sw.state).to(dev)
    sim.step(ref, 300, sw.dt, wp=wp)
    torch.cuda.synchronize()
    got, ref = st.cpu().numpy(), ref.cpu().numpy()
    dead = alive == 0
    assert np.array_equal(got[:, dead], sw.state[:, dead])
    assert np.array_equal(got[:, ~dead], ref[:, ~dead])
    sim.close()


def test_dead_agents_pass_the_cotangent_through(torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config4(n=512, n_steps=100)
    alive = (np.arange(sw.n) % 3 != 0).astype(np.uint8)
    at = torch.from_numpy(alive).to(dev)
    sim = Simulator(sw.types, sw.glob, mode=1, steps_per_launch=50)
    x = torch.from_numpy(sw.state).to(dev)
    gains = torch.from_numpy(sw.gains).to(dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    ckpt = torch.empty((2, 40, sw.n), device=dev)
    sim.step(x, 100, sw.dt, gains=gains, wp=wp, ckpt=ckpt, ckpt_every=50, alive=at,
             carry=torch.zeros_like(x[:10]))
    lam = torch.randn(30, sw.n, device=dev)
    gx0, gg = sim.step_backward(ckpt, 50, 100, sw.dt, lam, gains=gains, wp=wp, alive=at)
    x2 = torch.from_numpy(sw.state).to(dev)
    ck2 = torch.empty((2, 40, sw.n), device=dev)
    sim.step(x2, 100, sw.dt, gains=gains, wp=wp, ckpt=ck2, ckpt_every=50, carry=torch.zeros_like(x2[:10]))
    gx2, gg2 = sim.step_backward(ck2, 50, 100, sw.dt, lam, gains=gains, wp=wp)
    torch.cuda.synchronize()
    dead = torch.from_numpy(alive == 0).to(dev)
    assert torch.equal(gx0[:, dead], lam[:, dead]) and torch.all(gg[:, dead] == 0)
    assert torch.equal(gx0[:, ~dead], gx2[:, ~dead]) and torch.equal(gg[:, ~dead], gg2[:, ~dead])
    sim.close()


def test_graph_replay_reads_the_current_mask(torch_dev):
    """A cached graph reads the mask at run time: killing agents between two
    replays freezes them from then on."""
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config1(n=2000)
    sim = Simulator(sw.types, sw.glob, mode=1, steps_per_launch=50, use_graph=True)
    st = torch.from_numpy(sw.state).to(dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    alive = torch.ones(sw.n, dtype=torch.uint8, device=dev)
    sim.step(st, 100, sw.dt, wp=wp, alive=alive)
    alive[::2] = 0
    before = st.clone()
    sim.step(st, 100, sw.dt, wp=wp, alive=alive)
    torch.cuda.synchronize()
    assert torch.equal(st[:, ::2], before[:, ::2])
    assert not torch.equal(st[:, 1::2], before[:, 1::2])
    sim.close()
