"""Seeded synthetic swarms shaped like the paper's quadrotor workloads.

This module is the only code that both the HIP path and the FP64 reference
see.  It produces data and nothing else: initial states, commands,
waypoints, per-type physical parameters and gains, all drawn from numpy
PCG64 streams and rounded to float32 so that both sides start from the same
bits.  It performs none of the simulator's arithmetic (no controller, no
dynamics, no integration).

The paper benchmarks a batch of identical nonlinear quadrotors flying under
a PID body-rate controller (Sec. III, Table I and Fig. "run_time"); it
publishes no dataset, so every workload here is synthetic.

State layout (structure of arrays, ``float32[30][ld]``, one column per agent):

====== ===================================================================
rows   meaning
====== ===================================================================
0-2    position p, inertial ENU frame [m]
3-5    velocity v, inertial frame [m/s]
6-9    attitude quaternion q = (w, x, y, z), body FLU -> inertial, Hamilton
10-12  body rates omega [rad/s]
13-16  rotor speeds, stored as the deviation from the type's reference
       speed ``w_ref`` [rad/s]
17-19  position-loop integral
20-22  attitude-loop integral
23-25  rate-loop integral
26-28  body rates at the previous control step (rate-loop derivative)
29     running cost J = integral of the sum of squared rotor speeds
====== ===================================================================

The simulator's optional rounding carries (a separate ``[10][ld]`` buffer)
are zero for every state generated here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_ROWS = 30
N_GAINS = 9
SEED_BASE = 12698

# Base airframe of the homogeneous workloads (mass, inertia, arm, rotor
# coefficients, motor time constant, linear drag, speed limit).
BASE_QUAD = dict(mass=1.0, Ixx=0.0082, Iyy=0.0082, Izz=0.0149, arm=0.17,
                 alpha=math.pi / 4.0, k_f=6.1e-6, k_m=1.5e-7, tau_m=0.02,
                 drag=0.1, w_max=2500.0)
# Cascade gains [kpp, kip, kdp, kpa, kia, kda, kpr, kir, kdr].
DEFAULT_GAINS = (2.0, 0.1, 2.0, 8.0, 0.2, 0.1, 25.0, 2.0, 0.02)
# Controller limits shared by all types.
DEFAULT_GLOBALS = dict(g=9.81, r_sat=2.0, ipos_max=5.0, iatt_max=1.0,
                       irate_max=1.0, az_min_frac=0.5)
NO_BUDGET = 2**31 - 1
BOX = (100.0, 100.0, 20.0)

TYPE_FIELDS = ("mass", "Ixx", "Iyy", "Izz", "arm", "alpha", "k_f", "k_m",
               "tau_m", "drag", "w_max", "w_ref")


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def rng(config: int, stream: int) -> np.random.Generator:
    """PCG64 stream ``SEED_BASE + 100*config + stream``."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * config + stream))


@dataclass
class Swarm:
    """One synthetic workload.  Every float array is float32."""
    name: str
    mode: int                      # 0 open loop (motor commands), 1 closed loop
    dt: float
    n_steps: int
    state: np.ndarray              # [30, N]
    types: list                    # list of dicts, float32 scalars + gains + budget
    glob: dict                     # controller limits, float32 scalars
    type_idx: np.ndarray | None = None     # uint8 [N]
    gains: np.ndarray | None = None        # [9, N] per-agent gains
    motor_cmd: np.ndarray | None = None    # [4, N] deviation from w_ref
    wp: np.ndarray | None = None           # [E, 3, N]
    resample_every: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.state.shape[1]


def hover_reference_speed(mass, k_f, g) -> np.float32:
    """Rotor speed at which four rotors carry the weight, rounded to float32.

    Used only to pick the reference point of the stored rotor-speed
    deviation and the hovering initial condition; any reference works.
    """
    return np.float32(math.sqrt(float(mass) * float(g) / (4.0 * float(k_f))))


def make_type(mass, Ixx, Iyy, Izz, arm, k_f, k_m, tau_m=0.02, drag=0.1,
              w_max=2500.0, alpha=math.pi / 4.0, gains=DEFAULT_GAINS,
              budget=NO_BUDGET, g=DEFAULT_GLOBALS["g"], w_ref=None) -> dict:
    t = dict(mass=mass, Ixx=Ixx, Iyy=Iyy, Izz=Izz, arm=arm, alpha=alpha,
             k_f=k_f, k_m=k_m, tau_m=tau_m, drag=drag, w_max=w_max)
    t = {k: np.float32(v) for k, v in t.items()}
    if w_ref is None:
        w_ref = hover_reference_speed(t["mass"], t["k_f"], np.float32(g))
    t["w_ref"] = np.float32(w_ref)
    t["radius"] = t["arm"]          # collision radius: rotor hub distance
    t["gains"] = f32(gains)
    t["budget"] = int(budget)
    return t


def base_type(**over) -> dict:
    kw = dict(BASE_QUAD)
    kw.update(over)
    return make_type(**kw)


def globals_f32(**over) -> dict:
    d = dict(DEFAULT_GLOBALS)
    d.update(over)
    return {k: np.float32(v) for k, v in d.items()}


def _box_positions(r: np.random.Generator, n: int) -> np.ndarray:
    return np.stack([r.uniform(0.0, BOX[0], n), r.uniform(0.0, BOX[1], n),
                     r.uniform(0.0, BOX[2], n)])


def hover_state(pos: np.ndarray) -> np.ndarray:
    """Level, at rest, rotors at the reference speed, controller memory zero."""
    n = pos.shape[1]
    s = np.zeros((N_ROWS, n), dtype=np.float64)
    s[0:3] = pos
    s[6] = 1.0
    return f32(s)


def config0(n: int = 1000, n_steps: int = 1000, drag: float | None = None) -> Swarm:
    """Open-loop plain swarm: identical quads, per-motor commands uniform
    within +/-10 % of hover, constant over the rollout."""
    r = rng(0, 0)
    t = base_type() if drag is None else base_type(drag=drag)
    state = hover_state(_box_positions(r, n))
    u = r.uniform(0.9, 1.1, size=(4, n))
    cmd = f32((u - 1.0) * float(t["w_ref"]))
    return Swarm("open-loop", 0, 1e-3, n_steps, state, [t], globals_f32(), motor_cmd=cmd)


def config1(n: int = 5000, n_steps: int = 10000) -> Swarm:
    """Closed-loop plain swarm: hovering in the box, one random waypoint each."""
    r = rng(1, 0)
    state = hover_state(_box_positions(r, n))
    wp = f32(_box_positions(r, n)[None])
    return Swarm("closed-loop", 1, 1e-3, n_steps, state, [base_type()], globals_f32(),
                 wp=wp, resample_every=0)


def config2(n: int = 1 << 20, n_steps: int = 10000, resample_every: int = 2000) -> Swarm:
    """Scale workload: closed loop, waypoints redrawn every ``resample_every`` steps."""
    r = rng(2, 0)
    state = hover_state(_box_positions(r, n))
    n_ep = max(1, -(-n_steps // resample_every))
    wp = f32(np.stack([_box_positions(r, n) for _ in range(n_ep)]))
    return Swarm("scale", 1, 1e-3, n_steps, state, [base_type()], globals_f32(),
                 wp=wp, resample_every=resample_every)


HETERO_COUNTS = (1024, 4096, 16384, 65536, 131072, 262144, 524288, 3072)
# Base airframe inertia divided by mass*arm^2 (x, y, z).
INERTIA_SHAPE = (0.0082 / (1.0 * 0.17**2), 0.0082 / (1.0 * 0.17**2), 0.0149 / (1.0 * 0.17**2))


def hetero_types(n_types: int = 8, seed_stream: int = 0) -> list:
    """Eight airframes: mass U[0.3, 3] kg, arm U[0.08, 0.35] m, inertia
    mass*arm^2 times the base shape, rotor coefficients for a thrust to
    weight ratio of 2 at the speed limit, budgets 1000*(t+1) steps."""
    r = rng(3, seed_stream)
    g = DEFAULT_GLOBALS["g"]
    types = []
    for t in range(n_types):
        m = float(np.float32(r.uniform(0.3, 3.0)))
        L = float(np.float32(r.uniform(0.08, 0.35)))
        w_max = 2500.0
        k_f = m * g / (2.0 * w_max**2)
        k_m = k_f * (1.5e-7 / 6.1e-6)
        I = [m * L * L * s for s in INERTIA_SHAPE]
        types.append(make_type(m, I[0], I[1], I[2], L, k_f, k_m, w_max=w_max,
                               budget=1000 * (t + 1)))
    return types


def config3(scale: int = 1, counts=HETERO_COUNTS) -> Swarm:
    """Heterogeneous swarm: 8 types with uneven counts and step budgets.

    Type t has counts[t] agents and a budget of 1000*(t+1) steps; ``scale``
    divides every count (for small parity cases).  The per-agent type labels
    are shuffled (seeded), so neighbouring agents generally differ in type.
    """
    r = rng(3, 1)
    types = hetero_types()
    counts = [max(1, c // scale) for c in counts]
    labels = np.concatenate([np.full(c, t, dtype=np.uint8) for t, c in enumerate(counts)])
    r.shuffle(labels)
    n = labels.size
    state = hover_state(_box_positions(r, n))
    # Reference speed is per type; the hovering state stores deviation 0.
    n_steps = max(t["budget"] for t in types)
    n_ep = -(-n_steps // 2000)
    wp = f32(np.stack([_box_positions(r, n) for _ in range(n_ep)]))
    return Swarm("hetero", 1, 1e-3, n_steps, state, types, globals_f32(),
                 type_idx=labels, wp=wp, resample_every=2000,
                 extra=dict(counts=counts))


def config4(n: int = 65536, n_steps: int = 500, dt: float = 2e-3) -> Swarm:
    """Differentiable rollout: per-agent gains (defaults x U[0.8, 1.2]),
    target = start + U[-1, 1]^3, waypoint = target."""
    r = rng(4, 0)
    pos = _box_positions(r, n)
    state = hover_state(pos)
    target = f32(pos + r.uniform(-1.0, 1.0, size=(3, n)))
    gains = f32(np.asarray(DEFAULT_GAINS)[:, None] * r.uniform(0.8, 1.2, size=(N_GAINS, n)))
    return Swarm("diff", 1, dt, n_steps, state, [base_type()], globals_f32(),
                 gains=gains, wp=target[None].copy(), resample_every=0,
                 extra=dict(target=target, ckpt_every=50, cost_weight=1e-4))


def limits_swarm(n_group: int = 64, n_steps: int = 1000) -> Swarm:
    """Agents driven into the controller's limits (a parity case, not a
    workload of the paper), four groups of ``n_group``:

    - climbers: waypoint 10 km above, stiff position loop (k_pp in [60, 120],
      no I or D), so every rotor is commanded at the speed limit;
    - descenders: waypoint 10 km below (k_pp in [8, 15], no I or D), so the
      commanded vertical acceleration sits at its floor;
    - yawed: level, yawed by up to 150 degrees, waypoint at the position,
      attitude and rate integrals 1e-4 short of their clamps (rotors hit 0
      and the speed limit);
    - tumbling: tilted by up to 60 degrees about a random axis, body rates up
      to 5 rad/s, waypoint 1 km away in a random direction.
    Gains are per agent (default gains outside the first two groups).
    """
    r = rng(5, 0)
    n = 4 * n_group
    pos = _box_positions(r, n)
    s = np.zeros((N_ROWS, n), dtype=np.float64)
    s[0:3] = pos
    s[6] = 1.0
    gains = np.tile(np.asarray(DEFAULT_GAINS, dtype=np.float64)[:, None], (1, n))
    wp = pos.copy()
    up, down, yaw, tumble = (slice(k * n_group, (k + 1) * n_group) for k in range(4))
    wp[2, up] += 1e4
    gains[0, up] = r.uniform(60.0, 120.0, n_group)
    gains[1:3, up] = 0.0
    wp[2, down] -= 1e4
    gains[0, down] = r.uniform(8.0, 15.0, n_group)
    gains[1:3, down] = 0.0
    psi = r.uniform(-150.0, 150.0, n_group) * math.pi / 180.0
    s[6, yaw], s[9, yaw] = np.cos(psi / 2), np.sin(psi / 2)
    s[22, yaw] = -np.sign(psi) * (DEFAULT_GLOBALS["iatt_max"] - 1e-4)     # i_att z
    s[25, yaw] = -np.sign(psi) * (DEFAULT_GLOBALS["irate_max"] - 1e-4)   # i_rate z
    axis = r.normal(size=(3, n_group))
    axis /= np.linalg.norm(axis, axis=0)
    ang = r.uniform(0.0, 60.0, n_group) * math.pi / 180.0
    s[6, tumble] = np.cos(ang / 2)
    s[7:10, tumble] = axis * np.sin(ang / 2)
    s[10:13, tumble] = r.uniform(-5.0, 5.0, (3, n_group))
    d = r.normal(size=(3, n_group))
    wp[:, tumble] += 1e3 * d / np.linalg.norm(d, axis=0)
    return Swarm("limits", 1, 1e-3, n_steps, f32(s), [base_type()], globals_f32(),
                 gains=f32(gains), wp=f32(wp[None]), resample_every=0,
                 extra=dict(groups=("climb", "descend", "yaw", "tumble")))


# ---------------------------------------------------------------------------
# Cars and fixed-wing aircraft (vehicle kinds 1 and 2)
# ---------------------------------------------------------------------------
KIND_QUAD, KIND_CAR, KIND_WING = 0, 1, 2
# Per-kind parameter vector ``veh`` (12 entries, the last unused):
CAR_FIELDS = ("L", "l_r", "tau_delta", "delta_max", "a_max", "v_cruise", "rho", "lam",
              "k_orb", "k_head", "k_speed")
WING_FIELDS = ("tau_V", "tau_phi", "tau_gamma", "phi_max", "gamma_max", "V_cruise", "rho",
               "lam", "k_orb", "k_head", "k_alt")
# A passenger-car-sized vehicle circling at 8 m/s on a 25 m orbit, and a
# small fixed-wing aircraft at 18 m/s on an 80 m orbit.
CAR_DEFAULTS = dict(L=2.6, l_r=1.3, tau_delta=0.1, delta_max=0.5, a_max=3.0, v_cruise=8.0,
                    rho=25.0, lam=1.0, k_orb=2.0, k_head=1.5, k_speed=0.5)
WING_DEFAULTS = dict(tau_V=1.0, tau_phi=0.3, tau_gamma=0.5, phi_max=0.6, gamma_max=0.25,
                     V_cruise=18.0, rho=80.0, lam=1.0, k_orb=1.5, k_head=1.2, k_alt=0.05)
WING_ALTITUDE = (40.0, 60.0)


def vehicle_type(kind: int, mass: float, drag: float, radius: float, budget: int = NO_BUDGET,
                 **params) -> dict:
    """A car (kind 1) or fixed-wing (kind 2) type dict: float32 mass, linear
    drag coefficient (cars: longitudinal, N s/m), collision radius and the
    12-entry parameter vector ``veh`` in the order of CAR_FIELDS or
    WING_FIELDS.  Quadrotor fields are absent (the binding sends zeros)."""
    fields, defaults = (CAR_FIELDS, CAR_DEFAULTS) if kind == KIND_CAR else (WING_FIELDS, WING_DEFAULTS)
    unknown = set(params) - set(fields)
    if unknown:
        raise ValueError(f"unknown parameters {sorted(unknown)}")
    vals = dict(defaults)
    vals.update(params)
    veh = np.zeros(12, dtype=np.float32)
    veh[:len(fields)] = f32([vals[f] for f in fields])
    return dict(kind=int(kind), mass=np.float32(mass), drag=np.float32(drag), radius=np.float32(radius),
                veh=veh, gains=np.zeros(N_GAINS, dtype=np.float32), budget=int(budget))


def car_type(mass: float = 1200.0, drag: float = 60.0, radius: float = 1.5, budget: int = NO_BUDGET,
             **params) -> dict:
    return vehicle_type(KIND_CAR, mass, drag, radius, budget, **params)


def wing_type(mass: float = 2.0, radius: float = 0.8, budget: int = NO_BUDGET, **params) -> dict:
    return vehicle_type(KIND_WING, mass, 0.0, radius, budget, **params)


def veh_param(t: dict, name: str) -> float:
    fields = CAR_FIELDS if t["kind"] == KIND_CAR else WING_FIELDS
    return float(t["veh"][fields.index(name)])


def orbit_starts(r: np.random.Generator, t: dict, centre: np.ndarray) -> np.ndarray:
    """Initial rows 0-6 of vehicles of type ``t`` around orbit centres
    ``centre`` [3, n]: at a distance U[0.5, 1.5] x rho in a uniform
    direction theta, heading along the orbit's direction of travel
    (theta + lambda pi/2) give or take U[-pi/3, pi/3], so every start has a
    course error well inside (-pi, pi); cars on the ground at rest to
    cruise speed with the wheels straight, aircraft within 5 m of the orbit
    altitude at 0.9-1.1 x cruise speed, wings level."""
    n = centre.shape[1]
    rho, lam = veh_param(t, "rho"), veh_param(t, "lam")
    d = r.uniform(0.5, 1.5, n) * rho
    th = r.uniform(0.0, 2.0 * math.pi, n)
    x = np.zeros((7, n))
    x[0] = centre[0] + d * np.cos(th)
    x[1] = centre[1] + d * np.sin(th)
    x[4] = th + lam * 0.5 * math.pi + r.uniform(-math.pi / 3.0, math.pi / 3.0, n)
    if t["kind"] == KIND_CAR:
        x[2] = 0.0
        x[3] = veh_param(t, "v_cruise") * r.uniform(0.0, 1.0, n)
    else:
        x[2] = centre[2] + r.uniform(-5.0, 5.0, n)
        x[3] = veh_param(t, "V_cruise") * r.uniform(0.9, 1.1, n)
    return x


KINDS_FRACTIONS = (0.5, 0.25, 0.25)


def config_kinds(n: int = 1 << 20, n_steps: int = 10000, resample_every: int = 2000,
                 fractions=KINDS_FRACTIONS) -> Swarm:
    """Quadrotors, cars and fixed-wing aircraft in one batch (the three
    robot kinds of Sec. II-B; the aircraft circle as in the first demo of
    Sec. IV).  Types: 0 the base quadrotor, 1-2 cars circling
    counter-clockwise / clockwise, 3-4 aircraft likewise.  ``fractions``
    splits the agents between quadrotors, cars and aircraft (each vehicle
    kind evenly between its two directions); labels are shuffled.
    Quadrotors hover in the box and get new waypoints every
    ``resample_every`` steps as in the scale workload; a car's or
    aircraft's waypoint is its orbit centre (uniform in the box's
    footprint, on the ground for cars, at 40-60 m for aircraft), the same
    in every epoch."""
    r = rng(6, 0)
    types = [base_type(), car_type(lam=1.0), car_type(lam=-1.0), wing_type(lam=1.0), wing_type(lam=-1.0)]
    n_q = int(round(fractions[0] * n))
    n_c = int(round(fractions[1] * n))
    n_w = n - n_q - n_c
    counts = [n_q, n_c - n_c // 2, n_c // 2, n_w - n_w // 2, n_w // 2]
    labels = np.concatenate([np.full(c, t, dtype=np.uint8) for t, c in enumerate(counts)])
    r.shuffle(labels)
    n_ep = max(1, -(-n_steps // resample_every))
    pos = _box_positions(r, n)
    s = np.zeros((N_ROWS, n), dtype=np.float64)
    s[0:3] = pos
    s[6] = 1.0
    wp = np.stack([_box_positions(r, n) for _ in range(n_ep)])
    for t in range(1, len(types)):
        idx = np.where(labels == t)[0]
        if idx.size == 0:
            continue
        centre = np.stack([r.uniform(0.0, BOX[0], idx.size), r.uniform(0.0, BOX[1], idx.size),
                           np.zeros(idx.size) if types[t]["kind"] == KIND_CAR
                           else r.uniform(*WING_ALTITUDE, idx.size)])
        s[:, idx] = 0.0
        s[0:7, idx] = orbit_starts(r, types[t], centre)
        wp[:, :, idx] = centre[None]
    return Swarm("kinds", 1, 1e-3, n_steps, f32(s), types, globals_f32(), type_idx=labels,
                 wp=f32(wp), resample_every=resample_every, extra=dict(counts=counts))


def subset(sw: Swarm, idx: np.ndarray) -> Swarm:
    """The same workload restricted to the agents ``idx`` (column gather)."""
    idx = np.asarray(idx)
    pick = lambda a, ax: None if a is None else np.ascontiguousarray(np.take(a, idx, axis=ax))
    extra = dict(sw.extra)
    if "target" in extra:
        extra["target"] = pick(extra["target"], 1)
    return Swarm(sw.name, sw.mode, sw.dt, sw.n_steps, pick(sw.state, 1), sw.types, sw.glob,
                 type_idx=pick(sw.type_idx, 0), gains=pick(sw.gains, 1),
                 motor_cmd=pick(sw.motor_cmd, 1), wp=pick(sw.wp, 2),
                 resample_every=sw.resample_every, extra=extra)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}
