"""Parity at the benchmark's full sizes and launch configurations, checked on
sampled agents the FP64 reference can compute one by one.

- scale swarm: 1,048,576 agents x 10,000 steps, waypoints redrawn every
  2,000 steps, fused kernel at the autotuner's recorded launch shape
  replayed from a hipGraph (what bench.py times); 4,096 sampled agents,
  relative error <= 1e-4;
- heterogeneous swarm: 1,007,616 agents, 8 types, budgets 1,000-8,000, one
  launch in the type order; 4,096 sampled agents, <= 1e-4;
- differentiable rollout scaled to 1,048,576 agents (the bench's fwd_bwd
  form): adjoint gradients of 32 sampled agents against the reference's
  dual numbers, <= 1e-3.
"""
import numpy as np
import pytest

from paper_2308_12698_amd import inputs as I
from tests._util import rel_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def sampled_parity(oracle, sw, got, idx, n_steps, tol=1e-4):
    sub = I.subset(sw, idx)
    ref = oracle.rollout(sub.state, sub.types, sub.glob, 1, sub.dt, n_steps, type_idx=sub.type_idx,
                         gains=sub.gains, wp=sub.wp, resample_every=sub.resample_every)
    errs = rel_errors(got[:30, idx], ref, sub.types, sub.type_idx)
    worst = max(v[0] for v in errs.values())
    print(sw.name, {k: f"{v[0]:.2e}" for k, v in errs.items()}, flush=True)
    assert worst <= tol, errs


def test_scale_swarm_10000_steps_bench_configuration(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config2()
    print(f"scale swarm: {sw.n} agents x {sw.n_steps} steps", flush=True)
    st = torch.from_numpy(sw.state).to(dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    carry = torch.zeros((10, sw.n), device=dev)
    sim = Simulator(sw.types, sw.glob, mode=1, form="fused", use_graph=True)
    # the launch shape bench.py uses: the autotuner's recorded result for this build
    import bench
    tuned = sim.autotune(st, sw.dt, 1000, wp=wp, resample_every=sw.resample_every, carry=carry,
                         cache=bench.LAUNCH_SHAPES)
    print(f"launch shape {tuned} ({'recorded' if sim.tuned_from_cache else 'timed now'})", flush=True)
    sim.set_options(form="fused", use_graph=True, **tuned)
    sim.step(st, sw.n_steps, sw.dt, wp=wp, resample_every=sw.resample_every, carry=carry)
    torch.cuda.synchronize()
    got = st.cpu().numpy().astype(np.float64)
    sim.close()
    assert np.isfinite(got).all()
    idx = np.sort(np.random.default_rng(21).choice(sw.n, 4096, replace=False))
    sampled_parity(oracle, sw, got, idx, sw.n_steps)


def test_heterogeneous_swarm_full_size(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config3()
    print(f"heterogeneous swarm: {sw.n} agents, {sw.n_steps} steps", flush=True)
    sim = Simulator(sw.types, sw.glob, mode=1, form="fused", steps_per_launch=sw.n_steps)
    st = torch.from_numpy(sw.state).to(dev)
    ti = torch.from_numpy(sw.type_idx).to(dev)
    perm = sim.order_by_type(ti)
    sim.step(st, sw.n_steps, sw.dt, type_idx=ti, perm=perm, wp=torch.from_numpy(sw.wp).to(dev),
             resample_every=sw.resample_every, carry=torch.zeros((10, sw.n), device=dev))
    torch.cuda.synchronize()
    got = st.cpu().numpy().astype(np.float64)
    sim.close()
    idx = np.sort(np.random.default_rng(22).choice(sw.n, 4096, replace=False))
    sampled_parity(oracle, sw, got, idx, sw.n_steps)


def test_adjoint_at_one_million_agents(oracle, torch_dev):
    torch, dev = torch_dev
    from paper_2308_12698_amd.sim import Simulator
    sw = I.config4(n=1 << 20)
    K = sw.extra["ckpt_every"]
    print(f"differentiable rollout: {sw.n} agents x {sw.n_steps} steps, K = {K}", flush=True)
    sim = Simulator(sw.types, sw.glob, mode=1, form="fused", steps_per_launch=100)
    x = torch.from_numpy(sw.state).to(dev)
    gains = torch.from_numpy(sw.gains).to(dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    ckpt = torch.empty((sw.n_steps // K, 40, sw.n), device=dev)
    sim.step(x, sw.n_steps, sw.dt, gains=gains, wp=wp, ckpt=ckpt, ckpt_every=K,
             carry=torch.zeros((10, sw.n), device=dev))
    tgt = torch.from_numpy(sw.extra["target"]).to(dev)
    gfin = torch.zeros((30, sw.n), device=dev)
    gfin[0:3] = 2.0 * (x[0:3] - tgt)
    gfin[29] = sw.extra["cost_weight"]
    gx0, gg = sim.step_backward(ckpt, K, sw.n_steps, sw.dt, gfin, gains=gains, wp=wp)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(23).choice(sw.n, 32, replace=False))
    gx0 = gx0[:, idx].cpu().numpy()
    gg = gg[:, idx].cpu().numpy()
    sim.close()
    del ckpt
    sub = I.subset(sw, idx)
    fin, jac = oracle.jacobian(sub.state, sub.types, sub.glob, sub.dt, sub.n_steps, wp=sub.wp,
                               gains=sub.gains)
    seed = np.zeros((30, sub.n))
    seed[0:3] = 2.0 * (fin[0:3] - sub.extra["target"])
    seed[29] = sub.extra["cost_weight"]
    ref = np.einsum("ar,arc->ac", seed.T, jac)
    got = np.concatenate([gx0.T, gg.T], axis=1)
    es = np.linalg.norm(got[:, :30] - ref[:, :30], axis=1) / np.linalg.norm(ref[:, :30], axis=1)
    eg = np.linalg.norm(got[:, 30:] - ref[:, 30:], axis=1) / np.linalg.norm(ref[:, 30:], axis=1)
    print(f"adjoint at 1M vs dual: state {es.max():.2e} gains {eg.max():.2e}", flush=True)
    assert es.max() <= 1e-3 and eg.max() <= 1e-3
