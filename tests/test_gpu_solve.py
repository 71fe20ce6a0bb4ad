"""meb_solve on the GPU against the CPU oracle and the closed forms (GPU).

Bar: relative radius error <= 1e-8 against the oracle's FP64 answer on the
same seeded inputs, and no ball violated by more than 1e-10 (1 + r) in an
FP64 check on the host.  Both the plain FP64 path and the mixed path
(FP32 screening run, FP64 refinement, full check, reinsertion) are checked.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2605_31425_amd import inputs
from tests.gpu_common import dev, gpu

pytestmark = gpu


def _check(C, R, r, c, r_ref, rel=1e-8):
    reach = np.linalg.norm(C - c, axis=1) + (0 if R is None else R)
    assert reach.max() - r <= 1e-10 * (1 + r), (reach.max() - r)
    assert abs(r - r_ref) <= rel * abs(r_ref), (r, r_ref, abs(r - r_ref) / r_ref)


def _solve(C, R, mode, **kw):
    from paper_2605_31425_amd import meb
    return meb.solve(dev(C), dev(R), mode=mode, **kw)


MODES = ["fp64", "mixed"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed,m,d,balls", [(1, 3, 2, False), (2, 50, 2, True), (3, 1000, 3, True),
                                           (4, 2049, 10, False), (5, 777, 33, True), (6, 3000, 100, True)])
def test_solve_matches_oracle(mode, seed, m, d, balls):
    print(f"solve {mode} m={m} d={d}", flush=True)
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(m, d))
    R = rng.uniform(0, 0.3, m) if balls else None
    r_ref, c_ref, st_ref = oracle.ripalm(C, R, tol=1e-12)
    r, c, st = _solve(C, R, mode)
    assert st["rc"] == 0, st
    _check(C, R, r, c, st_ref["r_fixed"])
    assert np.abs(c - c_ref).max() <= 1e-6 * (1 + r_ref)


@pytest.mark.parametrize("mode", MODES)
def test_solve_single_ball_and_points(mode):
    r, c, st = _solve(np.array([[1.0, 2.0, 3.0]]), np.array([0.5]), mode)
    assert abs(r - 0.5) <= 1e-12 and np.allclose(c, [1, 2, 3], atol=1e-10)
    r, c, st = _solve(np.tile([[2.0, -1.0]], (10, 1)), None, mode)
    assert r == 0.0 and np.array_equal(c, [2.0, -1.0])


@pytest.mark.parametrize("mode", MODES)
def test_solve_two_balls_closed_form(mode):
    C = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    R = np.array([1.0, 2.0])
    r, c, st = _solve(C, R, mode)
    rs = (5.0 + 1.0 + 2.0) / 2
    _check(C, R, r, c, rs)
    assert np.allclose(c, C[0] + (rs - 1.0) * (C[1] - C[0]) / 5.0, atol=1e-7)


@pytest.mark.parametrize("mode", MODES)
def test_solve_cube_and_cross_polytope(mode):
    C = np.array(list(itertools.product([-1.0, 1.0], repeat=10)))
    r, c, st = _solve(C, None, mode)
    _check(C, None, r, c, np.sqrt(10))
    P, _ = inputs.points_ball_sphere(20000, 10, 9)
    C = inputs.with_cross_polytope(P * 0.999)
    r, c, st = _solve(C, None, mode)
    _check(C, None, r, c, 1.0)


@pytest.mark.parametrize("mode", MODES)
def test_points_workload_full_size(mode):
    """The 10,000 Gaussian points in R^10 workload (seed 1) at full size."""
    C, R = inputs.points_normal(10000, 10, 1)
    r_ref, c_ref, st_ref = oracle.ripalm(C, R, tol=1e-12)
    r, c, st = _solve(C, R, mode)
    assert st["rc"] == 0
    _check(C, R, r, c, st_ref["r_fixed"])


def test_forced_reinsertion_gives_same_answer():
    """A negative screening margin keeps only the balls that the crude FP32
    ball violates and discards touching ones; the full check must find them
    and the re-solve must reach the same ball."""
    C, R = inputs.balls_uniform(20000, 20, 17)
    r_ref, c_ref, st_ref = oracle.ripalm(C, R, tol=1e-12)
    r, c, st = _solve(C, R, "mixed", tol_red=-0.01, tol_kkt_low=0.3)
    assert st["rc"] == 0
    _check(C, R, r, c, st_ref["r_fixed"])
    assert st["reinsert_rounds"] >= 1


def test_fp64_trajectory_follows_oracle():
    """Same algorithm, same parameters: after a few outer iterations the
    plain FP64 path and the oracle are at the same iterate."""
    C, R = inputs.balls_uniform(3000, 8, 23)
    for k in [1, 2, 3]:
        r_ref, c_ref, st_ref = oracle.ripalm(C, R, max_outer=k, tol=0.0)
        r, c, st = _solve(C, R, "fp64", max_outer=k, tol_kkt=0.0)
        assert st["outer"][1] == k
        assert abs(st["rbar"] - r_ref) <= 1e-9 * r_ref, (k, st["rbar"], r_ref)
        assert np.abs(c - c_ref).max() <= 1e-9 * (1 + r_ref)


def test_solve_deterministic():
    C, R = inputs.balls_uniform(50000, 30, 29)
    a = _solve(C, R, "mixed")
    b = _solve(C, R, "mixed")
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_progress_printing_driver_matches():
    """The driver observes the end of a run through a mode word written by
    the control step, or, when it prints progress, through a copy of the
    state header; both see the same steps, so the results are identical."""
    C, R = inputs.balls_uniform(20000, 12, 31)
    for mode in MODES:
        a = _solve(C, R, mode)
        b = _solve(C, R, mode, verbose=1)
        assert a[2]["rc"] == 0 and b[2]["rc"] == 0
        assert a[0] == b[0] and np.array_equal(a[1], b[1]), mode


@pytest.mark.parametrize("mode", MODES)
def test_solve_fp32_input_is_the_solve_of_the_widened_data(mode):
    # FP32 input is widened exactly into the workspace: the answer is bitwise
    # the one of meb_solve on the same values given as FP64
    import torch
    from paper_2605_31425_amd import meb
    print(f"fp32 input {mode}", flush=True)
    rng = np.random.default_rng(21)
    C = rng.normal(size=(4001, 12)).astype(np.float32)
    R = rng.uniform(0, 0.2, 4001).astype(np.float32)
    r32, c32, st32 = meb.solve(dev(C, torch.float32), dev(R, torch.float32), mode=mode)
    r64, c64, st64 = meb.solve(dev(C.astype(np.float64)), dev(R.astype(np.float64)), mode=mode)
    assert st32["rc"] == 0 and r32 == r64 and np.array_equal(c32, c64)
    r_ref, c_ref, st_ref = oracle.ripalm(C.astype(np.float64), R.astype(np.float64), tol=1e-12)
    _check(C.astype(np.float64), R.astype(np.float64), r32, c32, st_ref["r_fixed"])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("bad", ["negative_radius", "nan_center", "inf_radius"])
def test_solve_rejects_bad_input(mode, bad):
    from paper_2605_31425_amd import meb
    print(f"bad input {bad} {mode}", flush=True)
    rng = np.random.default_rng(22)
    C = rng.normal(size=(3000, 5))
    R = rng.uniform(0, 0.2, 3000)
    if bad == "negative_radius":
        R[1234] = -1e-3
    elif bad == "nan_center":
        C[2999, 3] = np.nan
    else:
        R[7] = np.inf
    with pytest.raises(meb.MebError) as e:
        meb.solve(dev(C), dev(R), mode=mode)
    assert e.value.code == meb.MEB_ERR_ARG


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("fo", [1, 4])
def test_first_order_inner_solver_early_outer_iterations(mode, fo):
    # the accelerated gradient method as inner solver of the first `fo`
    # outer iterations (Section 4.1), semismooth Newton after: same answer
    from paper_2605_31425_amd import meb
    print(f"first-order {fo} {mode}", flush=True)
    rng = np.random.default_rng(31 + fo)
    C = rng.normal(size=(20000, 20))
    R = rng.uniform(0, 0.2, 20000)
    r_ref, c_ref, st_ref = oracle.ripalm(C, R, tol=1e-12)
    r, c, st = meb.solve(dev(C), dev(R), mode=mode, first_order_outer=fo)
    assert st["rc"] == 0, st
    assert sum(st["first_order_steps"]) > 0
    _check(C, R, r, c, st_ref["r_fixed"])



@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed,m,d", [(51, 20000, 20), (52, 6000, 300), (53, 2000, 500)])
def test_newton_cg_solver_matches_oracle(mode, seed, m, d):
    # matrix-free Newton directions (preconditioned CG with Hessian-vector
    # products, Section 4.1): the same ball
    from paper_2605_31425_amd import meb
    print(f"newton-cg {mode} m={m} d={d}", flush=True)
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(m, d))
    R = rng.uniform(0, 0.1, m)
    r_ref, c_ref, st_ref = oracle.ripalm(C, R, tol=1e-12)
    r, c, st = meb.solve(dev(C), dev(R), mode=mode, newton="cg", cg_max_iter=40, cg_tol=1e-3)
    assert st["rc"] == 0, st
    assert sum(st["cg_iterations"]) > 0
    _check(C, R, r, c, st_ref["r_fixed"])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed,m,d", [(54, 2000, 400), (55, 1500, 700)])
def test_dense_newton_large_d_matches_oracle(mode, seed, m, d):
    # Newton systems of d + 1 >= 320 unknowns: the Cholesky factorization
    # across many workgroups, one launch per panel phase
    from paper_2605_31425_amd import meb
    print(f"dense newton {mode} m={m} d={d}", flush=True)
    C, R, r_ref = _large_d_instance(seed, m, d)
    r, c, st = meb.solve(dev(C), dev(R), mode=mode)
    assert st["rc"] == 0, st
    _check(C, R, r, c, r_ref)


_large_d = {}


def _large_d_instance(seed, m, d):
    # the oracle's answer, computed once for both modes
    if seed not in _large_d:
        rng = np.random.default_rng(seed)
        C = rng.normal(size=(m, d))
        R = rng.uniform(0, 0.1, m)
        _large_d[seed] = (C, R, oracle.ripalm(C, R, tol=1e-12)[2]["r_fixed"])
    return _large_d[seed]
