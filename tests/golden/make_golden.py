"""Write the oracle regression fixture ``oracle_small.json``.

Calls only the FP64 reference (``oracle/``) on seeded inputs; no value here
comes from the HIP path.  Rerun only when the reference's arithmetic is
deliberately changed, and name the passage that justifies the change.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2308_12698_amd import inputs as I  # noqa: E402

AGENTS = [0, 1, 17, 500, 999]


def cases():
    c0 = I.subset(I.config0(), np.array(AGENTS))
    c1 = I.subset(I.config1(), np.array(AGENTS))
    out = {}
    s = O.rollout(c0.state, c0.types, c0.glob, 0, c0.dt, 1000, motor_cmd=c0.motor_cmd, threads=1)
    out["open_loop_1000"] = dict(agents=AGENTS, n_steps=1000, final=s[:30].tolist())
    s = O.rollout(c1.state, c1.types, c1.glob, 1, c1.dt, 1000, wp=c1.wp, threads=1)
    out["closed_loop_1000"] = dict(agents=AGENTS, n_steps=1000, final=s[:30].tolist())
    return out


if __name__ == "__main__":
    data = dict(source="oracle/oracle.cpp via tests/golden/make_golden.py", **cases())
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(data, f, indent=1)
