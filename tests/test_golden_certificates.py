"""Weak-duality certificates of the stored oracle answers (CPU only).

The golden radii of the full-size workloads come from the oracle's ripALM,
so their accuracy would otherwise rest on that algorithm alone.  This test
bounds the true minimum radius r* from below without using the oracle:

For multipliers (u_i, v_i) in the second-order cone with sum u_i = 1, the
Lagrangian of the conic form (Section 2) gives, at the optimum (r*, c*),
    r* >= sum_i u_i r_i + sum_i <v_i, c_i - c_hat> - <sum_i v_i, c* - c_hat>
for any point c_hat (every term u_i (r* - r_i) + <v_i, c* - c_i> is an inner
product of two elements of the self-dual cone, hence >= 0).  Taking
v_i = u_i (c_i - c_hat) / ||c_i - c_hat|| puts (u_i, v_i) on the cone's
boundary, and ||c* - c_hat|| <= r_out since both centers lie in the stored
ball (c* is in the convex hull of the centers, each within r_out of c_hat):
    r* >= LB = sum_i u_i (r_i + ||c_i - c_hat||) - r_out ||sum_i v_i||.
The weights u come from a non-negative least-squares fit that makes
sum_i v_i small over the balls whose reach is within delta of r_out.  The
stored radius r_out = max_i (r_i + ||c_i - c_hat||) is an upper bound (it is
recomputed here), so r* lies in [LB, r_out]; the test asserts the bracket is
within 1e-10 r_out, the solve tolerance of the workloads being 1e-8.
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import nnls

from paper_2605_31425_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def certificate(C, R, c_hat, r_out, deltas=(1e-12, 1e-11, 1e-10, 1e-9, 1e-8, 1e-7)):
    E = C - c_hat[None, :]
    dist = np.sqrt(np.einsum("ij,ij->i", E, E))
    reach = dist + (0.0 if R is None else R)
    best = -np.inf
    for dl in deltas:
        S = np.nonzero(reach >= r_out - dl * r_out)[0]
        if len(S) == 0:
            continue
        cap = 40 * (C.shape[1] + 1)  # a support has at most d + 1 balls; keep the fit small
        if len(S) > cap:  # a seeded spread-out subset (the top reaches can cluster on one side)
            S = np.sort(np.random.default_rng(0).choice(S, cap, replace=False))
        W = (E[S] / dist[S, None]).T  # unit vectors, d x k
        for big in (1.0, 10.0, 100.0, 1000.0):  # weight of the row sum u_i = 1
            A = np.vstack([W, big * np.ones((1, len(S)))])
            b = np.zeros(W.shape[0] + 1)
            b[-1] = big
            u, _ = nnls(A, b, maxiter=50 * len(S))
            if u.sum() <= 0:
                continue
            u = u / u.sum()
            rho = W @ u
            lb = float(u @ reach[S]) - r_out * float(np.linalg.norm(rho))
            best = max(best, lb)
    return best, float(reach.max())


@pytest.mark.slow
@pytest.mark.parametrize("name", ["balls_1e6_d100", "balls_2e5_d1000", "points_1e4_d10", "points_1e7_d10"])
def test_golden_radius_bracket(name):
    g = json.load(open(os.path.join(HERE, "golden", f"oracle_{name}.json")))
    C, R = getattr(inputs, g["generator"])(*g["args"])
    c = np.asarray(g["c"])
    lb, reach = certificate(C, R, c, g["r_fixed"])
    # the stored radius is the largest reach from the stored center
    assert reach == pytest.approx(g["r_fixed"], rel=1e-15, abs=0)
    assert lb <= g["r_fixed"]
    gap = (g["r_fixed"] - lb) / g["r_fixed"]
    print(f"{name}: r_out {g['r_fixed']:.17g} lower bound {lb:.17g} relative gap {gap:.2e}")
    assert gap <= 1e-10


@pytest.mark.parametrize("d,m", [(20, 1000), (30, 5000), (40, 1000), (50, 100000)])
def test_lcg_golden_radius_bracket(d, m):
    # the paper's LCG instances (Section 5): the stored oracle radius is
    # bracketed the same way
    g = {(e["d"], e["m"]): e for e in json.load(open(os.path.join(HERE, "golden", "oracle_lcg.json")))["instances"]}
    e = g[(d, m)]
    C, R = inputs.lcg_instance(m, d)
    lb, reach = certificate(C, R, np.asarray(e["c"]), e["r_fixed"])
    assert reach == pytest.approx(e["r_fixed"], rel=1e-15, abs=0)
    assert lb <= e["r_fixed"]
    assert (e["r_fixed"] - lb) / e["r_fixed"] <= 1e-10, (e["r_fixed"] - lb) / e["r_fixed"]
