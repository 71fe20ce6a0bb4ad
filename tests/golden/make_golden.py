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


# The instances of the paper's experiments (Section 5, "Test instances"):
# the Figure 2 / Table 1 grid and the Figure 3 high-dimensional shapes up to
# the dimensions this build supports.
LCG_SHAPES = [(d, m) for d in (20, 30, 40, 50) for m in (1000, 5000, 10000, 50000, 100000)] + \
             [(d, m) for d in (100, 500, 1000) for m in (1000, 5000)]


def make_lcg():
    out = dict(description="LCG instances of Section 5 (psi_0 = 7, psi_{j+1} = (445 psi_j + 1) mod 4096, "
                           "values psi_j / 40.96 as r_1, c_1, r_2, c_2, ...)",
               oracle_tol=1e-12, instances=[])
    for d, m in LCG_SHAPES:
        C, R = inputs.lcg_instance(m, d)
        t = time.time()
        r, c, st = oracle.ripalm(C, R, tol=1e-12)
        el = time.time() - t
        out["instances"].append(dict(d=d, m=m, r_fixed=st["r_fixed"], rbar=r, kkt=st["kkt"], outer=st["outer"],
                                     inner=st["inner"], oracle_seconds=el, c=c.tolist() if d <= 50 else None))
        print("lcg", d, m, st["r_fixed"], st["kkt"], f"{el:.1f}s", flush=True)
    with open(os.path.join(HERE, "oracle_lcg.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(WORKLOADS) + ["lcg"]):
        if n == "lcg":
            make_lcg()
        else:
            make(n)
