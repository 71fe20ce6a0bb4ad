"""The full-size synthetic workloads on the GPU against the oracle's stored
answers (tests/golden/oracle_<workload>.json, written by make_golden.py
from the CPU oracle only).

Bar: relative radius error <= 1e-8 and no ball violated by more than
1e-10 (1 + r), both modes.  The inputs are regenerated from the same seeded
generators the stored answers were computed from.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2605_31425_amd import inputs
from tests.gpu_common import dev, gpu

pytestmark = gpu

HERE = os.path.dirname(os.path.abspath(__file__))

WORKLOADS = {
    "balls_1e6_d100": (inputs.balls_uniform, (1000000, 100, 2)),
    "points_1e7_d10": (inputs.points_ball_sphere, (10000000, 10, 4)),
    "balls_2e5_d1000": (inputs.balls_normal, (200000, 1000, 3)),
}

_cache = {}


def _instance(name):
    if name not in _cache:
        _cache.clear()
        gen, args = WORKLOADS[name]
        C, R = gen(*args)
        with open(os.path.join(HERE, "golden", f"oracle_{name}.json")) as f:
            g = json.load(f)
        assert g["args"] == list(args)
        _cache[name] = (C, R, dev(C), dev(R), g)
    return _cache[name]


def _max_reach(C, R, c):
    out = -np.inf
    for i0 in range(0, C.shape[0], 1 << 18):
        blk = C[i0:i0 + (1 << 18)]
        reach = np.linalg.norm(blk - c, axis=1) + (0 if R is None else R[i0:i0 + (1 << 18)])
        out = max(out, reach.max())
    return out


@pytest.mark.parametrize("mode", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_workload_matches_oracle(name, mode):
    from paper_2605_31425_amd import meb
    print(f"workload {name} {mode}", flush=True)
    C, R, Cd, Rd, g = _instance(name)
    r, c, st = meb.solve(Cd, Rd, mode=mode)
    assert st["rc"] == 0, st
    r_ref = g["r_fixed"]
    assert abs(r - r_ref) <= 1e-8 * r_ref, (r, r_ref)
    assert _max_reach(C, R, c) - r <= 1e-10 * (1 + r)
    if mode == "mixed":
        assert 0 < st["n_red"] <= C.shape[0]


@pytest.mark.parametrize("d", [5, 7])
def test_small_d_many_batches_modes_agree(d):
    # short rows (several balls per lane group step); 9e6 points give every
    # wave more than 64 batches of 64 balls, so FP32 partial sums are
    # flushed several times per pass
    from paper_2605_31425_amd import meb
    m = 9_000_000
    print(f"small d={d} m={m}", flush=True)
    C, R = inputs.points_ball_sphere(m, d, 11 + d)
    Cd = torch.from_numpy(C).cuda()
    r64, c64, s64 = meb.solve(Cd, None, mode="fp64")
    rmx, cmx, smx = meb.solve(Cd, None, mode="mixed")
    assert s64["rc"] == 0 and smx["rc"] == 0, (s64, smx)
    assert abs(rmx - r64) <= 1e-8 * r64, (rmx, r64)
    for r, c in ((r64, c64), (rmx, cmx)):
        assert _max_reach(C, None, c) - r <= 1e-10 * (1 + r)
