"""Throughput benchmark of the batched quadrotor step on one MI355X.

Workload (one bench "step"): the closed-loop scale swarm -- 1,048,576
quadrotors hovering in a 100 x 100 x 20 m box, random waypoints redrawn
every 2,000 steps, cascaded PID + X mixer + rotor lag + quaternion rigid
body + RK4 at dt = 1 ms, 10,000 time steps, FP32 structure of arrays, fused
kernel (many steps per launch, state in registers) replayed from a hipGraph,
launch shape from the autotuner.  value = agent-steps per second over the K
timed rollouts, inputs resident in HBM.

Also reported, on the same GPU: the plain one-step-per-launch kernel on the
same swarm, the fused form without the graph, the heterogeneous 8-type batch
in one launch per rollout, collision detection over the swarm's positions,
the rollout driven through the command/snapshot pipeline (host decisions
outside the loop, positions streamed out), and forward+backward of the
differentiable rollout.  cpu_baseline times the FP64 reference on a bounded
sample of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "quadrotor agent-steps/s at 1M agents (fwd, fwd+bwd) vs plain kernel, 1e-4"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (256 CUs, 2.4 GHz)
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
# Algorithmic flops of one closed-loop agent-step, counted by hand per part
# of the step and pinned against the reference's operation-counting scalar
# (tests/test_bench_host.py): controller 197, right-hand side f(x) 109 (four
# evaluations per step), RK4 stage and combination arithmetic 234,
# renormalisation 12.  A multiplication by a structural zero (the scalar
# part of (0, w), the fourth component of the desired-attitude quaternion)
# or by G's row of ones is not counted, nor is a sign flip; f_c/m and the
# squared rotor speeds are formed once per evaluation.  The kernels do the
# same mathematics in fewer instructions (reciprocals, closed-form G^-1, FMA).
FLOPS_PER_AGENT_STEP = 197 + 4 * 109 + 234 + 12            # 879
FLOPS_PER_AGENT_STEP_OPEN_LOOP = 4 * 109 + 234 + 12         # 682
# The backward pass recomputes each step from its checkpoint (879 flops) and
# then runs the step's reverse sweep: the vector-Jacobian product of every
# forward operation by the elementary reverse-mode rules (per part:
# controller 539, f(x) 282 (x4), RK4 468, renormalisation 45), 2,180 flops.
REV_FLOPS_PER_AGENT_STEP = 539 + 4 * 282 + 468 + 45        # 2180
BWD_FLOPS_PER_AGENT_STEP = FLOPS_PER_AGENT_STEP + REV_FLOPS_PER_AGENT_STEP   # 3059
# Rows per agent-step of the adjoint's recomputation tape (written once and
# read once per agent-step).
TAPE_ROWS = 31            # step-start state without J and w_prev (26), held command (4), branch bits (1)
# Algorithmic HBM bytes per agent of one collision pass (collisions_form).
COLLISION_BYTES_PER_AGENT = 141
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
# The autotuner's results for these workloads on this build (keyed by device,
# build digest, variant, agent count and probe length): a hit fixes the launch
# shape, so the committed profiles and the bench line share it; a miss (new
# kernels, another device) times the candidates and records the result.
LAUNCH_SHAPES = os.environ.get("POTATO_AUTOTUNE_CACHE") or os.path.join(
    ROOT, "paper_2308_12698_amd", "launch_shapes.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2308_12698_amd", "csrc", f)
                  for f in ("quad_step.h", "kernels.hip", "kernels.h")]
# Sources whose code the other recorded kernels run (the rollout's are
# KERNEL_SOURCES).
TRAFFIC_SOURCES = {
    "collisions": [os.path.join(ROOT, "paper_2308_12698_amd", "csrc", f)
                   for f in ("collide.hip", "scan.h", "kernels.h")],
    "adjoint": [os.path.join(ROOT, "paper_2308_12698_amd", "csrc", f)
                for f in ("quad_adjoint.h", "quad_step.h", "kernels.hip", "kernels.h")],
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str = "fused") -> str:
    """Hash of a recorded kernel's sources with comments and blank space
    removed, so that only code changes mark its recorded counters as stale."""
    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES.get(kernel, KERNEL_SOURCES):
        with open(p) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed rollouts")
    ap.add_argument("--warmup", type=int, default=1, help="untimed rollouts")
    ap.add_argument("--agents", type=int, default=1 << 20)
    ap.add_argument("--sim-steps", type=int, default=10000)
    ap.add_argument("--no-extra", action="store_true", help="skip the other forms")
    ap.add_argument("--forms", default="plain,fused_eager,hetero,kinds,collisions,pipeline,fwd_bwd",
                    help="comma-separated subset of the other forms to run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--sweep", action="store_true",
                    help="time per round against the number of agents (the paper's protocol: "
                         "500 warm-up rounds, 2,000 timed rounds, 3 executions), GPU plain and "
                         "fused forms and the FP64 reference on 1 and all host threads; prints "
                         "one JSON line per point and exits")
    ap.add_argument("--oracle-table", action="store_true",
                    help="time the FP64 reference on each workload on 1 and all host threads "
                         "(bounded samples), print one JSON line per row and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of known size (for scaling "
                         "HBM byte counters) and exit")
    ap.add_argument("--shape", default="",
                    help="block,steps_per_launch,grid_blocks of the headline rollout instead of "
                         "autotuning (profiler runs at a fixed launch shape)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.sweep:
        sweep()
        return
    if args.oracle_table:
        oracle_table()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the quadrotor step has no cross-agent coupling, "
              "so a multi-GPU run is N independent copies of this one, each on its share of "
              "the agents.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    sw = I.config2(n=args.agents, n_steps=args.sim_steps)
    N, T = sw.n, args.sim_steps
    log(f"inputs: {N} agents, {T} steps, {sw.wp.shape[0]} waypoint epochs")
    state = torch.from_numpy(sw.state).to(dev)
    # rounding carries of the compensated integrator (the 10,000-step parity
    # bound needs them); they are read and written once per launch
    carry = torch.zeros((10, N), dtype=torch.float32, device=dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    sim = Simulator(sw.types, sw.glob, mode=1, form="fused", use_graph=True)
    if args.shape:
        b, s_, g = (int(v) for v in args.shape.split(","))
        tuned = {"block": b, "steps_per_launch": s_, "grid_blocks": g}
        log(f"launch shape given: {tuned}")
    else:
        tuned = sim.autotune(state, sw.dt, min(1000, T), wp=wp, resample_every=sw.resample_every,
                             carry=carry, cache=LAUNCH_SHAPES)
        log(f"autotuned launch shape: {tuned} "
            f"({'recorded result' if sim.tuned_from_cache else 'timed now'}, {os.path.relpath(LAUNCH_SHAPES, ROOT)})")
    sim_tuned_from_cache = getattr(sim, "tuned_from_cache", False)
    sim.set_options(form="fused", use_graph=True, **tuned)
    launches = -(-T // tuned["steps_per_launch"])

    def rollout():
        sim.step(state, T, sw.dt, wp=wp, resample_every=sw.resample_every, carry=carry)

    for _ in range(args.warmup):
        rollout()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        rollout()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [a.elapsed_time(b) for a, b in ev]
    value = N * T * args.steps / wall
    log(f"fused+graph: {value:.4e} agent-steps/s, rollout {np.mean(ev_ms):.2f} ms (events)")
    assert torch.isfinite(state).all().item(), "non-finite state after the rollouts"

    # roofline of the fused kernel: ALU bound, algorithmic flops per agent-step
    launch_ms = float(np.mean(ev_ms)) / launches
    achieved_tflops = FLOPS_PER_AGENT_STEP * N * tuned["steps_per_launch"] / (launch_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                "traffic": measured_traffic("fused"),
                "kernel": "k_rollout<closed loop> (fused)",
                "flops_per_agent_step": FLOPS_PER_AGENT_STEP,
                "avg_launch_ms": round(launch_ms, 4), "agents_per_launch": N,
                "steps_per_launch": tuned["steps_per_launch"]}

    forms = {"fused_graph": {"agent_steps_per_s": value, "rollout_ms": float(np.mean(ev_ms)),
                             "rollout_ms_sd": float(np.std(ev_ms)), "rollouts": len(ev_ms)}}
    if not args.no_extra:
        forms.update(extra_forms(torch, dev, stream, sim, state, carry, wp, sw, T,
                                 set(args.forms.split(","))))
    sim.close()

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O      # the CPU baseline times the reference itself
        cpu = cpu_baseline(O, sw)

    out = {
        "metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"closed-loop scale swarm: {N} quadrotors, {T} RK4 steps at dt=1 ms, "
                               "waypoints redrawn every 2,000 steps; fused kernel in a hipGraph",
                   "n_agents": N, "sim_steps": T, **tuned,
                   "shape_source": "given" if args.shape else
                   ("autotuner, recorded result" if sim_tuned_from_cache else "autotuner, timed in this run")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "env": run_environment(torch),
    }
    print(json.dumps(out), flush=True)


def extra_forms(torch, dev, stream, sim, state, carry, wp, sw, T, which):
    res = {}
    N = sw.n

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # plain: one launch per step, state round-trips HBM every step
    if "plain" in which:
        res.update(plain_form(timed, sw, state, carry, wp, N))
    # fused without the graph (host launches)
    sim.set_options(form="fused", use_graph=False, block=sim.opts.block,
                    steps_per_launch=sim.opts.steps_per_launch, grid_blocks=sim.opts.grid_blocks)
    if "fused_eager" in which:
        ms = timed(lambda: sim.step(state, 2000, sw.dt, wp=wp, resample_every=sw.resample_every,
                                    carry=carry))
        res["fused_eager"] = {"agent_steps_per_s": N * 2000 / (ms * 1e-3), "steps_timed": 2000,
                              "roofline": alu_roofline(N * 2000 / (ms * 1e-3))}
        log(f"fused eager: {res['fused_eager']['agent_steps_per_s']:.4e} agent-steps/s")
    if "hetero" in which:
        res.update(hetero_form(torch, dev, timed))
    if "kinds" in which:
        res.update(kinds_form(torch, dev, timed, N))
    if "collisions" in which:
        res["collisions"] = collisions_form(torch, dev, timed, N)
    if "pipeline" in which:
        res["pipeline"] = pipeline_form(torch, dev, sim, sw, T)
        log(f"pipeline: {res['pipeline']['agent_steps_per_s']:.4e} agent-steps/s, "
            f"{res['pipeline']['overhead_vs_resident']:+.3f} vs resident")
    if "fwd_bwd" in which:
        res.update(fwd_bwd_form(torch, dev, timed, N))
    return res


def plain_form(timed, sw, state, carry, wp, N):
    """One launch per step: the state round-trips HBM every step.  Without
    carries a closed-loop agent-step moves the method's own bytes, 30 rows
    in and out plus the 3 waypoint rows (252 B); with the compensated
    integrator's 10 carry rows in and out as well, 332 B."""
    from paper_2308_12698_amd.sim import Simulator
    res = {}
    steps_plain = 1000
    plain = Simulator(sw.types, sw.glob, mode=1, form="plain", use_graph=True)
    for key, c, bytes_step in (("plain", None, (30 + 30 + 3) * 4),
                               ("plain_carry", carry, (40 + 40 + 3) * 4)):
        ms = timed(lambda: plain.step(state, steps_plain, sw.dt, wp=wp, resample_every=sw.resample_every,
                                      carry=c))
        launch_ms = ms / steps_plain
        gbs = bytes_step * N / (launch_ms * 1e-3) / 1e9
        res[key] = {"agent_steps_per_s": N * steps_plain / (ms * 1e-3), "steps_timed": steps_plain,
                    "avg_launch_ms": launch_ms,
                    "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                                 "bytes_per_agent_step": bytes_step,
                                 "traffic": measured_traffic(key)}}
        log(f"{key}: {res[key]['agent_steps_per_s']:.4e} agent-steps/s, {gbs:.0f} GB/s "
            f"({bytes_step} B per agent-step)")
    plain.close()
    res["plain"]["hbm_reference"] = hbm_reference(timed, state)
    log(f"torch copy {res['plain']['hbm_reference']['torch_copy_GBps']:.0f}, "
        f"triad {res['plain']['hbm_reference']['torch_triad_GBps']:.0f} GB/s")
    return res


def hbm_reference(timed, like):
    """What torch's own elementwise kernels reach on this HBM, as context for
    the plain kernel's rate: a device copy (read + write) and a triad
    y = x + z / 2 (two reads, one write) over 1 GiB FP32 buffers."""
    import torch
    n = (1 << 30) // 4
    x = torch.ones(n, device=like.device)
    z = torch.full((n,), 2.0, device=like.device)
    y = torch.empty(n, device=like.device)
    copy_ms = timed(lambda: y.copy_(x), reps=20)
    triad_ms = timed(lambda: torch.add(x, z, alpha=0.5, out=y), reps=20)
    return {"torch_copy_GBps": round(2 * 4 * n / (copy_ms * 1e-3) / 1e9, 1),
            "torch_triad_GBps": round(3 * 4 * n / (triad_ms * 1e-3) / 1e9, 1),
            "buffer_bytes": 4 * n}


def hetero_form(torch, dev, timed):
    """8 types, budgets 1,000..8,000, one launch per rollout, with and
    without the type-grouped processing order."""
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator
    res = {}
    hw = I.config3()
    hsim = Simulator(hw.types, hw.glob, mode=1, form="fused", steps_per_launch=hw.n_steps)
    hs = torch.from_numpy(hw.state).to(dev)
    ti = torch.from_numpy(hw.type_idx).to(dev)
    hwp = torch.from_numpy(hw.wp).to(dev)
    work = sum(int(c) * hw.types[t]["budget"] for t, c in enumerate(hw.extra["counts"]))
    for label, perm in (("hetero_unordered", None), ("hetero", hsim.order_by_type(ti))):
        s0 = hs.clone()
        c0 = torch.zeros((10, hw.n), dtype=torch.float32, device=dev)
        ms = timed(lambda: hsim.step(s0, hw.n_steps, hw.dt, type_idx=ti, perm=perm, wp=hwp,
                                     resample_every=hw.resample_every, carry=c0), reps=1)
        res[label] = {"agent_steps_per_s": work / (ms * 1e-3), "agent_steps": work,
                      "n_agents": hw.n, "rollout_ms": ms,
                      "roofline": alu_roofline(work / (ms * 1e-3))}
        log(f"{label}: {res[label]['agent_steps_per_s']:.4e} agent-steps/s")
    hsim.close()
    return res


def kinds_form(torch, dev, timed, N, steps=2000):
    """Quadrotors, cars and fixed-wing aircraft in one launch (half, a
    quarter, a quarter; labels shuffled), closed loop, in index order and in
    the type order; and the same launch with only the quadrotors alive, so
    that the cars' and aircraft's share of the time shows."""
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator
    kw = I.config_kinds(n=N, n_steps=steps)
    ksim = Simulator(kw.types, kw.glob, mode=1, form="fused", steps_per_launch=1000, use_graph=True)
    ks = torch.from_numpy(kw.state).to(dev)
    ti = torch.from_numpy(kw.type_idx).to(dev)
    kwp = torch.from_numpy(kw.wp).to(dev)
    perm = ksim.order_by_type(ti)
    quads_only = torch.from_numpy((kw.type_idx == 0).astype(np.uint8)).to(dev)
    res = {}
    for label, order, alive in (("kinds_unordered", None, None), ("kinds", perm, None),
                                ("kinds_quads_only", perm, quads_only)):
        s0 = ks.clone()
        c0 = torch.zeros((10, kw.n), dtype=torch.float32, device=dev)
        ms = timed(lambda: ksim.step(s0, steps, kw.dt, type_idx=ti, perm=order, wp=kwp,
                                     resample_every=kw.resample_every, carry=c0, alive=alive), reps=2)
        n_adv = kw.n if alive is None else int(kw.extra["counts"][0])
        res[label] = {"agent_steps_per_s": n_adv * steps / (ms * 1e-3), "n_agents": kw.n,
                      "agents_advanced": n_adv, "sim_steps": steps, "rollout_ms": ms,
                      "counts_quad_car_wing": [int(kw.extra["counts"][0]),
                                               int(sum(kw.extra["counts"][1:3])),
                                               int(sum(kw.extra["counts"][3:5]))]}
        log(f"{label}: {res[label]['agent_steps_per_s']:.4e} agent-steps/s ({ms:.2f} ms)")
    ksim.close()
    return res


def collisions_form(torch, dev, timed, N):
    """Collision detection on the scale swarm's positions (all alive on entry)."""
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator
    cw = I.config2(n=N, n_steps=1)
    cstate = torch.from_numpy(cw.state).to(dev)
    csim = Simulator(cw.types, cw.glob, mode=1)
    alive0 = torch.ones(N, dtype=torch.uint8, device=dev)
    alive = alive0.clone()
    ws = torch.empty(int(csim._lib.potato_collision_workspace_bytes(N)), dtype=torch.uint8, device=dev)
    died = torch.zeros(1, dtype=torch.int64, device=dev)

    def detect():
        alive.copy_(alive0)
        csim.detect_collisions(cstate, alive, workspace=ws, died=died)

    ms = timed(detect, reps=5)
    # algorithmic bytes of a pass: positions and mask read by the bounding
    # box, the tile counts and the tile pass (13 B each); the items (x, y, z,
    # r and id, 20 B) written by the tile pass, read and written by the
    # window sort and read by the query (80 B); the bucket starts (2.13 per
    # agent) written by the sort and read by the query (17 B); the tile
    # counts written, scanned and read (about 4 B); the mask written (1 B).
    # Per agent: 39 + 80 + 17 + 4 + 1 = 141 B.
    gbs = COLLISION_BYTES_PER_AGENT * N / (ms * 1e-3) / 1e9
    out = {"agents_per_s": N / (ms * 1e-3), "n_agents": N, "ms": ms,
           "died_per_pass": int(died.item()) // 6,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_agent": COLLISION_BYTES_PER_AGENT,
                        "traffic": measured_traffic("collisions")}}
    log(f"collisions: {N / (ms * 1e-3):.4e} agents/s ({ms:.3f} ms per pass, "
        f"{out['died_per_pass']} collided)")
    csim.close()
    return out


def fwd_bwd_form(torch, dev, timed, N):
    """Forward (with checkpoints) + hand-written adjoint of the differentiable
    rollout: 500 steps at dt = 2 ms, checkpoints every 50 steps, at the
    workload's own 65,536 agents and at N agents."""
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator
    res = {}
    for n_agents in (65536, N):
        dw = I.config4(n=n_agents)
        K = dw.extra["ckpt_every"]
        dsim = Simulator(dw.types, dw.glob, mode=1, form="fused")
        x0 = torch.from_numpy(dw.state).to(dev)
        x = x0.clone()
        carry = torch.zeros((10, dw.n), dtype=torch.float32, device=dev)
        gains = torch.from_numpy(dw.gains).to(dev)
        dwp = torch.from_numpy(dw.wp).to(dev)
        # the forward's launch shape is the autotuner's, as for the other
        # forms, timed on the checkpointing variant that this forward runs
        tuned = dsim.autotune(x0, dw.dt, dw.n_steps, gains=gains, wp=dwp, carry=carry, ckpt_every=K,
                              cache=LAUNCH_SHAPES)
        dsim.set_options(form="fused", **tuned)
        tgt = torch.from_numpy(dw.extra["target"]).to(dev)
        ckpt = torch.empty((dw.n_steps // K, 40, dw.n), device=dev)
        # cotangent of the final state: the cost's rows (0-2 from the final
        # position, 29 a constant) are written per call, the others stay zero
        gfin = torch.zeros((30, dw.n), device=dev)
        gfin[29] = dw.extra["cost_weight"]
        ws = None

        def fwd():
            x.copy_(x0)
            carry.zero_()
            dsim.step(x, dw.n_steps, dw.dt, gains=gains, wp=dwp, ckpt=ckpt, ckpt_every=K, carry=carry)

        def bwd():
            torch.sub(x[0:3], tgt, out=gfin[0:3]).mul_(2.0)
            return dsim.step_backward(ckpt, K, dw.n_steps, dw.dt, gfin, gains=gains, wp=dwp,
                                      workspace=ws)

        fwd(); gx, gg = bwd()
        torch.cuda.synchronize()
        ms_f = timed(fwd)
        ms_fb = timed(lambda: (fwd(), bwd()))
        key = "fwd_bwd" if n_agents == N else "fwd_bwd_65536"
        # backward pass roofline: the algorithm is ALU bound (per agent-step a
        # recomputation of the step from its checkpoint and the step's reverse
        # sweep, BWD_FLOPS_PER_AGENT_STEP; its only algorithmic HBM traffic is
        # one 40-row checkpoint read per segment and the cotangents).  The
        # implementation's recomputation tape (TAPE_ROWS written and read per
        # agent-step) is reported beside it.
        ms_b = ms_fb - ms_f
        bwd_tf = BWD_FLOPS_PER_AGENT_STEP * dw.n * dw.n_steps / (ms_b * 1e-3) / 1e12
        tape_bytes = 2 * TAPE_ROWS * 4 + 40 * 4 / K
        gbs = dw.n * dw.n_steps * tape_bytes / (ms_b * 1e-3) / 1e9
        res[key] = {"agent_steps_per_s": dw.n * dw.n_steps / (ms_fb * 1e-3), "n_agents": dw.n,
                    "sim_steps": dw.n_steps, "ckpt_every": K, "fwd_launch_shape": tuned, "fwd_ms": ms_f,
                    "fwd_bwd_ms": ms_fb, "bwd_ms": ms_b,
                    "fwd_roofline": alu_roofline(dw.n * dw.n_steps / (ms_f * 1e-3)),
                    "bwd_roofline": {"bound": "alu", "achieved": round(bwd_tf, 3), "peak": PEAK_FP32_TFLOPS,
                                     "unit": "TFLOP/s", "frac": round(bwd_tf / PEAK_FP32_TFLOPS, 4),
                                     "flops_per_agent_step": BWD_FLOPS_PER_AGENT_STEP},
                    "bwd_tape": {"GBps": round(gbs, 1), "frac_of_hbm": round(gbs / PEAK_HBM_GBS, 4),
                                 "bytes_per_agent_step": round(tape_bytes, 1),
                                 "traffic": measured_traffic("adjoint") if key == "fwd_bwd" else None}}
        log(f"{key}: {res[key]['agent_steps_per_s']:.4e} agent-steps/s (fwd {ms_f:.2f} ms, "
            f"fwd+bwd {ms_fb:.2f} ms)")
        dsim.close()
        del ckpt, x, x0
    return res


def pipeline_form(torch, dev, sim, sw, T, snap_every=500):
    """Decision loop outside the simulation: every 2,000-step epoch the host
    computes the next waypoints from the positions streamed out one epoch
    earlier and pushes them while the GPU keeps simulating; positions of all
    agents are downloaded every `snap_every` steps.  Compared by wall clock
    with the same steps launched eagerly with the waypoints resident."""
    from paper_2308_12698_amd.sim import Pipe
    N, es = sw.n, sw.resample_every
    E = max(1, T // es)        # a shorter run (profiler passes) still times one epoch
    per = es // snap_every
    x0 = torch.from_numpy(sw.state).to(dev)
    state = x0.clone()
    carry = torch.zeros((10, N), dtype=torch.float32, device=dev)
    wp = torch.from_numpy(sw.wp).to(dev)
    pipe = Pipe(sim, N)
    snaps = torch.empty((E, per, 3, N), dtype=torch.float32, pin_memory=True)
    offsets = (sw.wp - sw.state[None, 0:3]).astype(np.float32)      # [E, 3, N]

    def pipelined():
        state.copy_(x0)
        carry.zero_()
        base = pipe.n_snaps
        pipe.push(sw.wp[0])
        for e in range(E):
            pipe.run(state, es, sw.dt, snap_every=snap_every, snaps=snaps[e], carry=carry)
            if e + 1 == E:
                break
            if e == 0:
                observed = sw.state[0:3]
            else:
                pipe.wait_snapshots(base + e * per)
                observed = snaps[e - 1, per - 1].numpy()
            pipe.push(observed + offsets[e + 1])
        pipe.sync()
        torch.cuda.synchronize()

    def resident():
        state.copy_(x0)
        carry.zero_()
        sim.step(state, E * es, sw.dt, wp=wp, resample_every=es, carry=carry)
        torch.cuda.synchronize()

    out = {}
    for label, fn in (("pipelined", pipelined), ("resident", resident)):
        fn()
        t0 = time.perf_counter()
        for _ in range(2):
            fn()
        out[label] = (time.perf_counter() - t0) / 2
    pipe.close()
    steps = E * es
    return {"agent_steps_per_s": N * steps / out["pipelined"], "sim_steps": steps, "epochs": E,
            "snap_every": snap_every, "snapshots": E * per,
            "snapshot_bytes": E * per * 3 * N * 4, "command_bytes": E * 3 * N * 4,
            "wall_ms": out["pipelined"] * 1e3, "resident_wall_ms": out["resident"] * 1e3,
            "overhead_vs_resident": out["pipelined"] / out["resident"] - 1.0}


SWEEP_SIZES = (1000, 2048, 4096, 5000, 8192, 10000, 16384, 65536, 262144, 1048576)


def sweep(sizes=SWEEP_SIZES, warm=500, rounds=2000, execs=3, cpu_budget_s=4.0):
    """Closed-loop swarm of each size, hovering with one random waypoint.
    One round = one time step of every agent.  GPU forms: plain (one launch
    per round, replayed from a hipGraph) and fused (autotuned, hipGraph);
    after the warm-up rounds one untimed call of `rounds` rounds captures the
    graph that the timed executions replay (one waypoint epoch and no step
    budget, so the step index does not change the work).
    The reference runs the same swarm for as many rounds as fit in about
    cpu_budget_s seconds (at least one)."""
    import torch
    from oracle import oracle as O
    from paper_2308_12698_amd import inputs as I
    from paper_2308_12698_amd.sim import Simulator
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    all_threads = max(1, min(16, os.cpu_count() or 1))
    cpu_rate = {}
    for n in sizes:
        sw = I.config1(n=n)
        wp = torch.from_numpy(sw.wp).to(dev)
        for form in ("plain", "fused"):
            state = torch.from_numpy(sw.state).to(dev)
            # the fused form keeps the rounding carries as the headline rollout
            # does; the plain form moves the state rows only
            carry = torch.zeros((10, n), dtype=torch.float32, device=dev) if form == "fused" else None
            sim = Simulator(sw.types, sw.glob, mode=1, form=form, use_graph=True)
            if form == "fused":
                tuned = sim.autotune(state, sw.dt, 1000, wp=wp, carry=carry, cache=LAUNCH_SHAPES)
                sim.set_options(form="fused", use_graph=True, **tuned)
            sim.step(state, warm, sw.dt, wp=wp, carry=carry)
            sim.step(state, rounds, sw.dt, wp=wp, carry=carry)     # captures the graph timed below
            ms = []
            for e in range(execs):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                sim.step(state, rounds, sw.dt, wp=wp, carry=carry)
                b.record(stream)
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b) / rounds)
            sim.close()
            print(json.dumps({"sweep": "gpu", "form": form, "n_agents": n, "ms_per_round": float(np.mean(ms)),
                              "sd_ms": float(np.std(ms)), "agent_steps_per_s": n / (np.mean(ms) * 1e-3),
                              "warmup_rounds": warm, "rounds": rounds, "executions": execs}), flush=True)
        for threads in (1, all_threads):
            # rate from the previous size sets the number of rounds that fit the budget
            guess = cpu_rate.get(threads, 2e6 * threads)
            r = int(max(1, min(rounds, cpu_budget_s * guess / n)))
            t0 = time.perf_counter()
            O.rollout(sw.state, sw.types, sw.glob, 1, sw.dt, r, wp=sw.wp, threads=threads)
            dt = time.perf_counter() - t0
            cpu_rate[threads] = n * r / dt
            print(json.dumps({"sweep": "oracle", "threads": threads, "n_agents": n, "rounds": r,
                              "ms_per_round": dt / r * 1e3, "agent_steps_per_s": n * r / dt}), flush=True)


def oracle_table(budget_s=8.0):
    """The reference on each workload, single thread and all host threads.
    Each row runs the workload's agents (or a prefix of them) for as many
    steps as fit in about budget_s seconds, scaled from a short probe."""
    from oracle import oracle as O
    from paper_2308_12698_amd import inputs as I
    all_threads = max(1, min(16, os.cpu_count() or 1))

    def run(label, sw, n_steps, threads, agents=None):
        sub = sw if agents is None or agents >= sw.n else I.subset(sw, np.arange(agents))
        kw = dict(type_idx=sub.type_idx, gains=sub.gains, motor_cmd=sub.motor_cmd, wp=sub.wp,
                  resample_every=sub.resample_every, threads=threads)
        probe = max(1, min(n_steps, 20))
        t0 = time.perf_counter()
        O.rollout(sub.state, sub.types, sub.glob, sub.mode, sub.dt, probe, **kw)
        rate = sub.n * probe / max(time.perf_counter() - t0, 1e-6)
        steps = int(max(1, min(n_steps, budget_s * rate / sub.n)))
        t0 = time.perf_counter()
        O.rollout(sub.state, sub.types, sub.glob, sub.mode, sub.dt, steps, **kw)
        dt = time.perf_counter() - t0
        print(json.dumps({"oracle": label, "threads": threads, "agents": sub.n, "steps": steps,
                          "of_steps": n_steps, "seconds": dt, "agent_steps_per_s": sub.n * steps / dt}),
              flush=True)

    rows = [("open loop, 1,000 agents", I.config0(), 1000, None),
            ("closed loop, 5,000 agents", I.config1(), 1000, None),
            ("scale swarm, 1,048,576 agents", I.config2(), 1000, None),
            ("heterogeneous, 1,007,616 agents (first 1,000 steps)", I.config3(), 1000, None),
            ("differentiable forward, 65,536 agents", I.config4(), 500, None)]
    for label, sw, n_steps, agents in rows:
        for threads in (1, all_threads):
            run(label, sw, n_steps, threads, agents)
    # forward-mode dual-number gradients of the differentiable rollout, 64 agents
    dw = I.config4()
    sub = I.subset(dw, np.arange(64))
    for threads in (1, all_threads):
        t0 = time.perf_counter()
        O.jacobian(sub.state, sub.types, sub.glob, sub.dt, sub.n_steps, wp=sub.wp, gains=sub.gains,
                   threads=threads)
        dt = time.perf_counter() - t0
        print(json.dumps({"oracle": "dual-number Jacobian (39 directions), 64 agents x 500 steps",
                          "threads": threads, "agents": 64, "steps": sub.n_steps, "seconds": dt,
                          "agent_steps_per_s": 64 * sub.n_steps / dt}), flush=True)


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain copy of `nbytes` bytes, `reps` times: each dispatch moves
    exactly nbytes in and nbytes out of HBM, which calibrates the FETCH_SIZE
    and WRITE_SIZE counters of a profiler run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def cpu_baseline(O, sw, sample_agents=262144, sample_steps=4000, single_agents=16384, single_steps=1000):
    """FP64 reference on the host cores, bounded samples of the same workload:
    all threads (up to 16) on the first sample_agents agents x sample_steps
    steps, and one thread on the first single_agents agents x single_steps."""
    from paper_2308_12698_amd import inputs as I
    threads = max(1, min(16, os.cpu_count() or 1))
    sub = I.subset(sw, np.arange(min(sample_agents, sw.n)))
    t0 = time.perf_counter()
    O.rollout(sub.state, sub.types, sub.glob, 1, sub.dt, sample_steps, wp=sub.wp,
              resample_every=sub.resample_every, threads=threads)
    dt = time.perf_counter() - t0
    v = sub.n * sample_steps / dt
    one = I.subset(sw, np.arange(min(single_agents, sw.n)))
    t0 = time.perf_counter()
    O.rollout(one.state, one.types, one.glob, 1, one.dt, single_steps, wp=one.wp,
              resample_every=one.resample_every, threads=1)
    dt1 = time.perf_counter() - t0
    v1 = one.n * single_steps / dt1
    log(f"cpu baseline: {v:.4e} agent-steps/s on {threads} threads ({dt:.1f} s), "
        f"{v1:.4e} on 1 thread ({dt1:.1f} s)")
    return {"value": v, "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sub.n} agents of the same swarm x {sample_steps} steps, FP64, "
                      f"{dt:.1f} s wall",
            "single_thread": {"value": v1, "cores": 1,
                              "sample": f"first {one.n} agents x {single_steps} steps, FP64, {dt1:.1f} s wall"},
            "host": host_cpu()}


def run_environment(torch) -> dict:
    """Software versions and the device the numbers were taken on."""
    from paper_2308_12698_amd import _lib
    p = torch.cuda.get_device_properties(0)
    return {"device": p.name, "gcn_arch": getattr(p, "gcnArchName", ""), "compute_units": p.multi_processor_count,
            "torch": torch.__version__, "hip": torch.version.hip,
            "library": _lib.load().potato_version().decode(), "seeds": "numpy PCG64, 12698 + 100 config + stream"}


def alu_roofline(agent_steps_per_s: float) -> dict:
    """Algorithmic FP32 rate of a closed-loop form against the FP32 peak."""
    tf = FLOPS_PER_AGENT_STEP * agent_steps_per_s / 1e12
    return {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / PEAK_FP32_TFLOPS, 4)}


def host_cpu() -> str:
    """CPU model and logical CPU count of the host the reference ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs"



if __name__ == "__main__":
    main()
