"""Writes the oracle's answers for the full-size synthetic workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators;
nothing here touches the GPU library.  Usage:
    python tests/golden/make_golden.py [name ...]
Each result goes to tests/golden/oracle_<name>.json.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_31425_amd import inputs  # noqa: E402

WORKLOADS = {
    # name: (generator, args, description)
    "points_1e4_d10": (inputs.points_normal, (10000, 10, 1), "points, m=10,000, d=10, centers N(0,I), seed 1"),
    "balls_1e6_d100": (inputs.balls_uniform, (1000000, 100, 2),
                       "balls, m=1,000,000, d=100, centers U[-1,1]^d, radii U[0,0.1], seed 2"),
    "balls_2e5_d1000": (inputs.balls_normal, (200000, 1000, 3),
                        "balls, m=200,000, d=1000, centers N(0,I), radii |N(0,0.05^2)|, seed 3"),
    "points_1e7_d10": (inputs.points_ball_sphere, (10000000, 10, 4),
                       "points, m=10,000,000, d=10, 90% uniform in the unit ball, 10% on the sphere, seed 4"),
}


def make(name):
    gen, args, desc = WORKLOADS[name]
    C, R = gen(*args)
    t = time.time()
    r, c, st = oracle.ripalm(C, R, tol=1e-12)
    el = time.time() - t
    out = dict(name=name, description=desc, generator=gen.__name__, args=list(args), r_fixed=st["r_fixed"],
               rbar=r, c=c.tolist(), kkt=st["kkt"], kkt_parts=st["kkt_parts"], outer=st["outer"],
               inner=st["inner"], ls_evals=st["ls_evals"], L=st["L"], oracle_seconds=el,
               oracle_tol=1e-12, note="oracle ripALM (FP64, long-double sums), stall-stopped at its rounding floor")
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, r, st["r_fixed"], st["kkt"], f"{el:.1f}s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(WORKLOADS)):
        make(n)
