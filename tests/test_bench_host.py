"""Host-side logic of bench.py (no GPU): the algorithmic flop count it
prices the roofline with, the staleness check of the recorded HBM
counters, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2308_12698_amd import inputs as I  # noqa: E402


# Hand count of one agent-step, per part (add/sub, mul, div, sqrt), from the
# operation list of the step.  Rules: a product with a structural zero (the
# scalar part of (0, w), the last component of the desired-attitude
# quaternion) or with G's row of ones costs nothing, a sign flip costs
# nothing, f_c/m and the squared rotor speeds are formed once per f(x).
HAND_COUNT = {
    # e = wp - p (3 sub); |e| (3 mul, 2 add, sqrt); integral e dt + i (3 mul,
    # 3 add); a = kpp e + kip i - kdp v (9 mul, 6 add); + g (1 add); body z
    # axis (9 mul, 4 add); f_c = m (a . z) (4 mul, 2 add); |a| (3 mul, 2 add,
    # sqrt); n = a/|a| (3 div); 1 + n_z (1 add); |q_des| (3 mul, 2 add, sqrt);
    # q_des/|q_des| (3 div); conj(q) o q_des with q_des[3] = 0 (12 mul,
    # 8 add); e_att = 2 q_e (3 mul); attitude integral (3 mul, 3 add); w_des
    # (9 mul, 6 add); e_w = w_des - w (3 add); rate integral (3 mul, 3 add);
    # alpha = kpr e_w + kir i - kdr (w - w_prev)/dt (9 mul, 9 add, 3 div);
    # I w (3 mul); tau = I alpha + w x I w (9 mul, 6 add); G^-1 [f_c, tau]
    # (16 mul, 12 add); W = sqrt(f/k_f) (4 div, 4 sqrt)
    "controller": (76, 101, 13, 7),
    # W^2 (4 mul); k_f W^2 (4 mul); G f with row 0 a plain sum (12 mul,
    # 12 add); body z (9 mul, 4 add); f_c/m (1 div); f_c/m z - (c_d/m) v
    # (6 mul, 3 add) and - g (1 add); q o (0, w) (12 mul, 8 add) times 1/2
    # (4 mul); I w (3 mul); w x I w (6 mul, 3 add); (tau - w x I w)/I (3 add,
    # 3 div); (W_cmd - W)/tau_m (4 add, 4 div); J' = sum W^2 (3 add)
    "derivative": (41, 60, 8, 0),
    # three stage states x + c h k over 18 components (54 mul, 54 add);
    # x + h/6 (k1 + 2 k2 + 2 k3 + k4) over 18 (54 mul, 72 add)
    "rk4": (126, 108, 0, 0),
    # |q| (4 mul, 3 add, sqrt), q/|q| (4 div)
    "renorm": (3, 4, 4, 1),
}
# Reverse sweep (vector-Jacobian product) per part, by the elementary
# reverse-mode rules; checked by hand for the renormalisation (4 squares
# 4 flops each, 3 sums 2 each, sqrt 3, 4 quotients of two variables 5 each)
# and the RK4 arithmetic (a scaled stage rate plus a state: 4 per component,
# 3 x 18; the combination: 14 per component, 18).
HAND_REV = {"renorm": 45, "rk4": 468}


def test_flop_count_is_the_hand_count(oracle):
    sw = I.config2(n=8, n_steps=10)
    ops = oracle.count_ops(sw.types[0], sw.glob, 1, sw.dt)
    for part, (add, mul, div, sqrt) in HAND_COUNT.items():
        got = ops[part]
        assert (got["add"], got["mul"], got["div"], got["sqrt"]) == (add, mul, div, sqrt), part
    for part, rev in HAND_REV.items():
        assert ops[part]["rev"] == rev, part
    hand = sum(HAND_COUNT["controller"]) + 4 * sum(HAND_COUNT["derivative"]) + \
        sum(HAND_COUNT["rk4"]) + sum(HAND_COUNT["renorm"])
    assert ops["flops"] == hand == bench.FLOPS_PER_AGENT_STEP == 879
    assert ops["rev_flops"] == bench.REV_FLOPS_PER_AGENT_STEP
    assert bench.BWD_FLOPS_PER_AGENT_STEP == bench.FLOPS_PER_AGENT_STEP + ops["rev_flops"]
    assert ops["controller"]["rev"] + 4 * ops["derivative"]["rev"] + ops["rk4"]["rev"] + \
        ops["renorm"]["rev"] == ops["rev_flops"]
    # open loop: the same step without the controller
    o0 = oracle.count_ops(sw.types[0], sw.glob, 0, sw.dt)
    assert o0["flops"] == bench.FLOPS_PER_AGENT_STEP_OPEN_LOOP == hand - sum(HAND_COUNT["controller"])


def test_flop_count_does_not_depend_on_parameter_values(oracle):
    """Only structural constants are free: an airframe with unit mass and one
    with another mass count the same."""
    a = oracle.count_ops(I.base_type(), I.globals_f32(), 1, 1e-3)
    b = oracle.count_ops(I.base_type(mass=1.3), I.globals_f32(), 1, 1e-3)
    assert a["flops"] == b["flops"] and a["rev_flops"] == b["rev_flops"]


def test_source_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // add one\n}\n/* block\n comment */\n")
    b.write_text("int f(int x)\n{\n\treturn x + 1;\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a)])
    h1 = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(b)])
    assert bench.kernel_source_hash() == h1
    b.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h1


def test_traffic_is_reported_only_for_the_current_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fused") is None                    # no file
    f.write_text(json.dumps({"fused": {"source_hash": "0" * 16, "bytes_per_launch": 123}}))
    assert bench.measured_traffic("fused") is None                    # stale counters
    f.write_text(json.dumps({"fused": {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 123}}))
    assert bench.measured_traffic("fused") == 123
    assert bench.measured_traffic("plain") is None                    # not recorded


@pytest.mark.timeout(120)
def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=100)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_host_cpu_is_described():
    text = bench.host_cpu()
    assert "logical CPUs" in text and text.split(",")[0].strip()


def test_alu_roofline_prices_the_flop_count():
    r = bench.alu_roofline(1e11)
    assert r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP32_TFLOPS
    assert abs(r["achieved"] - 87.9) < 1e-9 and abs(r["frac"] - round(87.9 / 157.3, 4)) < 1e-12
