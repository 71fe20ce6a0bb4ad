"""Pins of the oracle's ripALM solve (CPU only).

The answer of (MEB) is unique (Section 2), so the oracle is checked on
(r, c) against: closed forms (one ball, two balls, d = 1, cube vertices,
cross-polytope, nested and duplicated balls, collinear centers), the
exhaustive support-set enumeration of ``oracle.brute`` on tiny instances,
the KKT certificate of its own multipliers (dual feasibility, complementarity,
c in the convex hull of the touching centers), weak duality, and
invariance under translation, scaling, permutation and rotation.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2605_31425_amd import inputs

TOL = 1e-12


def solve(C, R=None, **kw):
    kw.setdefault("tol", TOL)
    return oracle.ripalm(C, R, **kw)


def test_single_ball():
    r, c, st = solve(np.array([[1.0, -2.0, 3.0]]), np.array([0.7]))
    np.testing.assert_allclose(r, 0.7, rtol=1e-12)
    np.testing.assert_allclose(c, [1.0, -2.0, 3.0], atol=1e-12)


def test_single_point_and_identical_points():
    r, c, st = solve(np.tile([[2.0, 5.0]], (5, 1)))
    assert r == 0.0 and np.array_equal(c, [2.0, 5.0])


@pytest.mark.parametrize("seed", range(6))
def test_two_balls_closed_form(seed):
    g = np.random.default_rng(seed)
    d = int(g.integers(1, 6))
    C = g.normal(size=(2, d)) * 3
    R = g.uniform(0, 1, 2)
    D = np.linalg.norm(C[0] - C[1])
    if D > abs(R[0] - R[1]):
        rs = (D + R[0] + R[1]) / 2
        cs = C[0] + (rs - R[0]) * (C[1] - C[0]) / D
    else:
        k = int(np.argmax(R))
        rs, cs = R[k], C[k]
    r, c, st = solve(C, R)
    np.testing.assert_allclose(r, rs, rtol=1e-11)
    np.testing.assert_allclose(c, cs, atol=1e-10 * (1 + rs))


def test_nested_balls_answer_is_container():
    C = np.array([[0.0, 0.0], [0.5, 0.2], [-0.3, 0.1], [0.1, -0.6]])
    R = np.array([2.0, 0.3, 0.5, 0.2])
    r, c, st = solve(C, R)
    np.testing.assert_allclose(r, 2.0, rtol=1e-11)
    np.testing.assert_allclose(c, [0.0, 0.0], atol=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_one_dimension_closed_form(seed):
    g = np.random.default_rng(100 + seed)
    C = g.normal(size=(50, 1)) * 4
    R = g.uniform(0, 1, 50)
    hi, lo = np.max(C[:, 0] + R), np.min(C[:, 0] - R)
    r, c, st = solve(C, R)
    np.testing.assert_allclose(r, (hi - lo) / 2, rtol=1e-11)
    np.testing.assert_allclose(c, [(hi + lo) / 2], atol=1e-10)


def test_collinear_centers_in_3d():
    g = np.random.default_rng(7)
    a, b = np.array([1.0, 2.0, -1.0]), np.array([0.3, -0.5, 0.8])
    tt = g.normal(size=30)
    R = g.uniform(0, 0.4, 30)
    C = a + tt[:, None] * b / np.linalg.norm(b)
    hi, lo = np.max(tt + R), np.min(tt - R)
    r, c, st = solve(C, R)
    np.testing.assert_allclose(r, (hi - lo) / 2, rtol=1e-11)
    np.testing.assert_allclose(c, a + (hi + lo) / 2 * b / np.linalg.norm(b), atol=1e-10)


@pytest.mark.parametrize("d", [2, 5, 10])
def test_cube_vertices(d):
    C = np.array(list(itertools.product([-1.0, 1.0], repeat=d)))
    r, c, st = solve(C)
    np.testing.assert_allclose(r, np.sqrt(d), rtol=1e-11)
    np.testing.assert_allclose(c, np.zeros(d), atol=1e-10)


@pytest.mark.parametrize("d", [3, 10])
def test_cross_polytope_with_interior_points(d):
    g = np.random.default_rng(d)
    P = g.normal(size=(500, d))
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    P *= g.uniform(0, 1, (500, 1))
    C = inputs.with_cross_polytope(P)
    r, c, st = solve(C)
    np.testing.assert_allclose(r, 1.0, rtol=1e-11)
    np.testing.assert_allclose(c, np.zeros(d), atol=1e-10)


def test_duplicated_balls_do_not_change_answer():
    g = np.random.default_rng(3)
    C = g.normal(size=(30, 4))
    R = g.uniform(0, 0.2, 30)
    r1, c1, _ = solve(C, R)
    r2, c2, _ = solve(np.concatenate([C, C, C]), np.concatenate([R, R, R]))
    np.testing.assert_allclose(r2, r1, rtol=1e-11)
    np.testing.assert_allclose(c2, c1, atol=1e-10)


@pytest.mark.parametrize("seed", range(24))
def test_brute_force_tiny(seed):
    g = np.random.default_rng(1000 + seed)
    d = 2 + seed % 2
    m = 3 + seed % 6
    C = g.normal(size=(m, d)) * g.uniform(0.5, 3)
    R = None if seed % 3 == 0 else g.uniform(0, 0.6, m)
    rb, cb, S = brute.meb(C, R)
    r, c, st = solve(C, R)
    np.testing.assert_allclose(r, rb, rtol=1e-10)
    np.testing.assert_allclose(c, cb, atol=1e-9 * (1 + rb))


def _certificate(C, R, r, c, U, V, tol):
    m, d = C.shape
    R0 = np.zeros(m) if R is None else R
    # dual feasibility (Section 2, dual problem)
    assert abs(U.sum() - 1) <= tol
    assert np.linalg.norm(V.sum(0)) <= tol
    assert np.all(np.linalg.norm(V, axis=1) <= U + tol)
    # complementarity: u_i > 0 only where the ball touches
    reach = np.linalg.norm(C - c, axis=1) + R0
    assert np.all(U * (r - reach) <= tol * (1 + r))
    # c is a convex combination of the touching centers (derived from the
    # KKT system: v_i = u_i (c_i - c)/||c_i - c|| on touching balls)
    act = U > 1e-9
    dist = np.linalg.norm(C[act] - c, axis=1)
    lam = np.where(dist > 0, U[act] / np.maximum(r - R0[act], 1e-300), 0)
    lam /= lam.sum()
    np.testing.assert_allclose(lam @ C[act], c, atol=1e3 * tol * (1 + np.abs(c).max()))
    # weak duality: the dual objective bounds r* from below
    dual = U @ R0 + np.einsum("ij,ij->", V, C)
    assert dual <= r + 1e3 * tol * (1 + r)
    assert r - dual <= 1e3 * tol * (1 + r)


@pytest.mark.parametrize("kind", ["points", "balls", "sphere"])
def test_kkt_certificate(kind):
    if kind == "points":
        C, R = inputs.points_normal(3000, 6, 11)
    elif kind == "balls":
        C, R = inputs.balls_uniform(3000, 20, 12)
    else:
        C, R = inputs.points_ball_sphere(5000, 5, 13)
    # at very large sigma the multipliers of a degenerate support pick up
    # rounding of order sigma * eps per touching ball, so the certificate is
    # taken at the printed tolerance scale (KKT_max <= 1e-9)
    r, c, st, U, V = solve(C, R, want_mult=True, tol=1e-9)
    assert st["kkt"] <= 1e-9
    _certificate(C, R, r, c, U, V, 1e-8)
    # the fixed-up radius is feasible and within the KKT level of rbar
    # (numpy's norm rounds differently from the oracle's by an ulp or two)
    reach = np.linalg.norm(C - c, axis=1) + (0 if R is None else R)
    assert st["r_fixed"] >= reach.max() * (1 - 8 * np.finfo(float).eps)
    assert st["r_fixed"] - r <= 1e-8 * r


def test_support_set_certificate_points_full_size():
    """On the 10,000 x 10 Gaussian points workload, re-solve the touching set
    exactly with ``oracle.brute.candidates_for`` and check that this ball
    encloses every point and that its center is a convex combination of the
    touching points: then it is the exact optimum, and the oracle must agree."""
    C, R = inputs.points_normal(10000, 10, 1)
    r, c, st, U, V = solve(C, R, want_mult=True)
    S = np.flatnonzero(U > 1e-8)
    assert 2 <= len(S) <= 11
    cands = brute.candidates_for(C[S], np.zeros(len(S)))
    assert len(cands) == 1
    rx, cx = cands[0]
    assert (np.linalg.norm(C - cx, axis=1)).max() <= rx * (1 + 1e-13)
    lam = np.linalg.lstsq(np.vstack([C[S].T, np.ones(len(S))]), np.append(cx, 1.0), rcond=None)[0]
    assert lam.min() > 0
    np.testing.assert_allclose(r, rx, rtol=1e-11)
    np.testing.assert_allclose(c, cx, atol=1e-10)


def test_invariances():
    g = np.random.default_rng(5)
    C, R = inputs.balls_normal(400, 5, 21)
    r, c, _ = solve(C, R)
    # translation and scaling
    shift, scale = g.normal(size=5) * 10, 3.5
    r2, c2, _ = solve(C * scale + shift, R * scale)
    np.testing.assert_allclose(r2, r * scale, rtol=1e-11)
    np.testing.assert_allclose(c2, c * scale + shift, atol=1e-9 * scale)
    # permutation
    p = g.permutation(400)
    r3, c3, _ = solve(C[p], R[p])
    np.testing.assert_allclose(r3, r, rtol=1e-11)
    # rotation
    Q, _ = np.linalg.qr(g.normal(size=(5, 5)))
    r4, c4, _ = solve(C @ Q.T, R)
    np.testing.assert_allclose(r4, r, rtol=1e-11)
    np.testing.assert_allclose(c4, Q @ c, atol=1e-9)


def test_warm_start_reaches_same_answer():
    C, R = inputs.balls_uniform(2000, 8, 31)
    r, c, st, U, V = solve(C, R, want_mult=True)
    x0 = np.concatenate([[r * 1.01], c + 0.01])
    r2, c2, st2 = solve(C, R, x0=x0, U0=U, V0=V)
    np.testing.assert_allclose(r2, r, rtol=1e-11)
