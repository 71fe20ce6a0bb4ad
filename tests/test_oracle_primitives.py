"""Pins of the oracle's cone primitives and per-ball evaluator (CPU only).

Each check compares against something fixed independently of the oracle's
code: the closed-form projection cases (Section 2), the Moreau
decomposition of a self-dual cone, finite differences of Psi and of its
gradient (Section 4 defines g and H as the gradient and a generalized
Hessian of Psi), and numpy's dense solver for the Newton system.
"""
import numpy as np
import pytest

import oracle

rng = np.random.default_rng(12345)


def test_projection_cases_closed_form():
    # interior: ||s|| <= t  -> unchanged
    pt, ps, case = oracle.soc_project(5.0, [3.0, 4.0])
    assert case == 0 and pt == 5.0 and np.array_equal(ps, [3.0, 4.0])
    # polar: ||s|| <= -t -> 0
    pt, ps, case = oracle.soc_project(-5.0, [3.0, 4.0])
    assert case == 1 and pt == 0.0 and np.array_equal(ps, [0.0, 0.0])
    # otherwise: (t + n)/2 (1, s/n);  t = 1, s = (3, 4): n = 5 -> 3 (1, 0.6, 0.8)
    pt, ps, case = oracle.soc_project(1.0, [3.0, 4.0])
    assert case == 2
    np.testing.assert_allclose([pt, *ps], [3.0, 1.8, 2.4], rtol=0, atol=1e-15)
    # apex tie (0, 0) counts as interior
    pt, ps, case = oracle.soc_project(0.0, [0.0, 0.0])
    assert case == 0 and pt == 0.0


@pytest.mark.parametrize("d", [1, 2, 5, 40])
def test_projection_moreau(d):
    for _ in range(50):
        t = rng.normal() * 2
        s = rng.normal(size=d)
        pt, ps, _ = oracle.soc_project(t, s)
        qt, qs, _ = oracle.soc_project(-t, -s)
        # z = Pi(z) - Pi(-z) and <Pi(z), Pi(-z)> = 0 for a self-dual cone
        np.testing.assert_allclose(pt - qt, t, atol=1e-13)
        np.testing.assert_allclose(ps - qs, s, atol=1e-13)
        assert abs(pt * qt + ps @ qs) <= 1e-12
        # Pi(z) lies in Q and Pi is idempotent
        assert np.linalg.norm(ps) <= pt * (1 + 1e-14) + 1e-15
        p2t, p2s, _ = oracle.soc_project(pt, ps)
        np.testing.assert_allclose([p2t, *p2s], [pt, *ps], atol=1e-14)
        # distance to Q equals ||z - Pi(z)||
        dist = np.sqrt((t - pt) ** 2 + np.sum((s - ps) ** 2))
        np.testing.assert_allclose(oracle.soc_dist(t, s), dist, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("d", [1, 3, 8])
def test_jacobian_matches_finite_differences(d):
    h = 1e-6
    for _ in range(30):
        t = rng.normal()
        s = rng.normal(size=d)
        n = np.linalg.norm(s)
        if min(abs(n - t), abs(n + t)) < 1e-3:  # stay away from the kinks
            continue
        P, case = oracle.soc_jacobian(t, s)
        z = np.concatenate([[t], s])
        J = np.empty((d + 1, d + 1))
        for k in range(d + 1):
            zp, zm = z.copy(), z.copy()
            zp[k] += h
            zm[k] -= h
            a = oracle.soc_project(zp[0], zp[1:])
            b = oracle.soc_project(zm[0], zm[1:])
            J[:, k] = (np.concatenate([[a[0]], a[1]]) - np.concatenate([[b[0]], b[1]])) / (2 * h)
        np.testing.assert_allclose(P, J, atol=1e-7)
        np.testing.assert_allclose(P, P.T, atol=0)
        ev = np.linalg.eigvalsh(P)
        assert ev.min() >= -1e-14 and ev.max() <= 1 + 1e-14


def _instance(m, d, balls=True):
    C = rng.normal(size=(m, d))
    R = rng.uniform(0, 0.3, m) if balls else None
    return C, R


@pytest.mark.parametrize("d,balls", [(2, False), (3, True), (7, True)])
def test_al_eval_gradient_and_hessian_by_finite_differences(d, balls):
    m = 40
    C, R = _instance(m, d, balls)
    sigma, tau = 1.7, 0.6
    # multipliers in the cone, some zero
    U = np.abs(rng.normal(size=m)) * (rng.uniform(size=m) < 0.5)
    V = rng.normal(size=(m, d))
    V *= (U / np.maximum(np.linalg.norm(V, axis=1), 1e-300) * rng.uniform(size=m))[:, None]
    x = np.concatenate([[1.5], rng.normal(size=d) * 0.3])
    xbar = x + rng.normal(size=d + 1) * 0.1
    ev = oracle.al_eval(C, R, U, V, x, xbar, sigma, tau)
    h = 1e-6
    gfd = np.empty(d + 1)
    Hfd = np.empty((d + 1, d + 1))
    for k in range(d + 1):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        a = oracle.al_eval(C, R, U, V, xp, xbar, sigma, tau)
        b = oracle.al_eval(C, R, U, V, xm, xbar, sigma, tau)
        gfd[k] = (a["psi"] - b["psi"]) / (2 * h)
        Hfd[:, k] = (a["g"] - b["g"]) / (2 * h)
    np.testing.assert_allclose(ev["g"], gfd, atol=1e-7 * (1 + np.abs(gfd).max()))
    np.testing.assert_allclose(ev["H"], Hfd, atol=1e-6 * (1 + np.abs(Hfd).max()))
    H = ev["H"]
    np.testing.assert_allclose(H, H.T, atol=0)
    assert np.linalg.eigvalsh(H).min() >= tau / sigma * (1 - 1e-12)
    # the multiplier update is sigma * Pi(z_i) and the gradient is
    # (1, 0) - sum (u+, v+) + tau/sigma (x - xbar)
    g2 = np.concatenate([[1.0 - ev["U"].sum()], -ev["V"].sum(0)]) + tau / sigma * (x - xbar)
    np.testing.assert_allclose(ev["g"], g2, atol=1e-12)
    dm = np.sum((ev["U"] - U) ** 2) + np.sum((ev["V"] - V) ** 2)
    np.testing.assert_allclose(ev["dmult"], dm, rtol=1e-12)
    assert ev["counts"].sum() == m


def test_al_eval_psi_at_far_feasible_point():
    # far inside every constraint with zero multipliers every z_i is in the
    # polar cone: Psi = r + tau/(2 sigma)||x - xbar||^2, g = (1,0) + tau/sigma (x - xbar)
    C, R = _instance(30, 4)
    x = np.array([100.0, 0.1, 0.0, -0.2, 0.3])
    xbar = np.array([99.0, 0.0, 0.0, 0.0, 0.0])
    ev = oracle.al_eval(C, R, None, None, x, xbar, 2.0, 3.0)
    assert ev["counts"][1] == 30
    np.testing.assert_allclose(ev["psi"], 100.0 + 3.0 / 4.0 * np.sum((x - xbar) ** 2), rtol=1e-15)
    np.testing.assert_allclose(ev["g"], np.eye(5)[0] + 1.5 * (x - xbar), rtol=1e-15)
    np.testing.assert_allclose(ev["H"], 1.5 * np.eye(5), rtol=1e-15)


@pytest.mark.parametrize("n", [1, 5, 33, 101])
def test_chol_solve_matches_numpy(n):
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)
    b = rng.normal(size=n)
    np.testing.assert_allclose(oracle.chol_solve(A, b), np.linalg.solve(A, b), rtol=1e-11, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.chol_solve(-np.eye(n), b)


def test_kkt_max_at_exact_two_point_solution():
    # Two points p1, p2: c = midpoint, r = |p1 - p2|/2, u_i = 1/2 and
    # v_i = u_i (c_i - c)/||c_i - c|| (so sum v = 0 and (u_i, v_i) on the
    # boundary of Q, orthogonal to (r, c - c_i)).
    p1, p2 = np.array([0.0, 0.0, 1.0]), np.array([2.0, 0.0, 1.0])
    C = np.stack([p1, p2])
    c = (p1 + p2) / 2
    r = 1.0
    U = np.array([0.5, 0.5])
    V = np.stack([0.5 * (p1 - c), 0.5 * (p2 - c)])
    k, parts = oracle.kkt_max(C, None, U, V, np.concatenate([[r], c]))
    assert k <= 1e-15
    # flipping v breaks complementarity by r * u * 2 = 1 per ball
    k2, parts2 = oracle.kkt_max(C, None, U, -V, np.concatenate([[r], c]))
    assert abs(parts2[4] - 1.0) < 1e-15
    # shrinking r by 0.1 violates both: dist = 0.1/sqrt(2)
    k3, parts3 = oracle.kkt_max(C, None, U, V, np.concatenate([[0.9], c]))
    np.testing.assert_allclose(parts3[2], 0.1 / np.sqrt(2), rtol=1e-14)


def test_check_feasible_and_screen_known_values():
    # unit circle points plus the origin, ball (r=1, c=0): every circle point is tight
    ang = np.linspace(0, 2 * np.pi, 8, endpoint=False)
    C = np.concatenate([np.stack([np.cos(ang), np.sin(ang)], 1), [[0.0, 0.0], [3.0, 0.0]]])
    R = np.zeros(len(C))
    R[-1] = 0.5
    dmax, am, viol = oracle.check_feasible(C, R, 1.0, np.zeros(2), 1e-9)
    np.testing.assert_allclose(dmax, 2.5, rtol=1e-15)  # ball 9: 0.5 + 3 - 1
    assert am == 9 and list(viol) == [9]
    keep, slack = oracle.screen(C, R, 1.0, np.zeros(2), 0.5)
    # slack: circle points ~0, origin 1, far ball -2.5
    assert list(keep) == [0, 1, 2, 3, 4, 5, 6, 7, 9]
    np.testing.assert_allclose(slack[8], 1.0)
    # ties in the maximum go to the smallest index
    dmax, am, viol = oracle.check_feasible(C[:8], None, 0.5, np.zeros(2), 0.1)
    np.testing.assert_allclose(dmax, 0.5, rtol=1e-15)
    assert am == 0 and len(viol) == 8


def test_lcg_generator_first_values():
    from paper_2605_31425_amd import inputs
    rows = [l.split() for l in open(__file__.replace("test_oracle_primitives.py", "golden/lcg_first_values.txt"))
            if l.strip() and not l.startswith("#")]
    C, R = inputs.lcg_instance(1, 3)
    vals = [R[0], *C[0]]
    for (j, psi, v), got in zip(rows, vals):
        assert float(v) == got and int(psi) / 40.96 == got
    # period 4096 (Hull-Dobell): value 4097 repeats value 1
    Cb, Rb = inputs.lcg_instance(4097 * 2, 1)  # 8194 scalars
    flat = np.stack([Rb, Cb[:, 0]], 1).ravel()
    assert flat[4096] == flat[0] and len(set(flat[:4096])) == 4096


def _three_case_instance():
    """Three balls in R^2 whose z_i = (r_i - r + u_i/sigma, c_i - c + v_i/sigma)
    fall in the three projection cases at x = (1, 0, 0), sigma = 2, tau = 1,
    xbar = (0.5, 0, 1), each with a non-zero multiplier (u_i, v_i) in Q:
      A (third case): c = (2.4, 3.2), r = 1,   w = (2, 1.2, 1.6)  -> z = (1, 3, 4)
      B (interior):   c = (0.5, 0),   r = 1.5, w = (1, 0.5, 0)    -> z = (1, 0.75, 0)
      C (polar):      c = (0, 0.2),   r = 0,   w = (0.5, 0, 0.4)  -> z = (-0.75, 0, 0.4)
    """
    C = np.array([[2.4, 3.2], [0.5, 0.0], [0.0, 0.2]])
    R = np.array([1.0, 1.5, 0.0])
    U = np.array([2.0, 1.0, 0.5])
    V = np.array([[1.2, 1.6], [0.5, 0.0], [0.0, 0.4]])
    return C, R, U, V, np.array([1.0, 0.0, 0.0]), np.array([0.5, 0.0, 1.0]), 2.0, 1.0


def test_al_eval_three_cases_worked_by_hand():
    # Worked out by hand from the closed-form projection (Section 2), Psi of
    # the proximal subproblem (Section 3), its gradient and the generalized
    # Hessian (Section 4) and the multiplier update (Algorithm 1):
    #   A: t = 1, s = (3, 4), n = 5: Pi = 3 (1, 0.6, 0.8) = (3, 1.8, 2.4), ||Pi||^2 = 18,
    #      sigma Pi = (6, 3.6, 4.8), change (4, 2.4, 3.2): 32;  ||w||^2 = 4 + 1.44 + 2.56 = 8
    #   B: Pi = z = (1, 0.75, 0), ||Pi||^2 = 1.5625, sigma Pi = (2, 1.5, 0), change (1, 1, 0): 2;
    #      ||w||^2 = 1.25
    #   C: Pi = 0, change -w: 0.41;  ||w||^2 = 0.41
    #   Psi = r + sigma/2 * 19.5625 - 9.66 / (2 sigma) + tau/(2 sigma) * 1.25
    #       = 1 + 19.5625 - 2.415 + 0.3125 = 18.46
    #   g = (1, 0, 0) - sigma (4, 2.55, 2.4) + tau/sigma (0.5, 0, -1) = (-6.75, -5.1, -5.3)
    #   H = tau/sigma I + sigma (I + P_A), P_A = 1/2 [[1, w^T], [w, 1.2 I - 0.2 w w^T]], w = (0.6, 0.8)
    C, R, U, V, x, xbar, sigma, tau = _three_case_instance()
    ev = oracle.al_eval(C, R, U, V, x, xbar, sigma, tau)
    assert list(ev["counts"]) == [1, 1, 1]
    np.testing.assert_allclose(ev["psi"], 18.46, rtol=0, atol=1e-13)
    np.testing.assert_allclose(ev["g"], [-6.75, -5.1, -5.3], rtol=0, atol=1e-13)
    np.testing.assert_allclose(ev["dmult"], 34.41, rtol=0, atol=1e-13)
    H = np.array([[3.5, 0.6, 0.8], [0.6, 3.628, -0.096], [0.8, -0.096, 3.572]])
    np.testing.assert_allclose(ev["H"], H, rtol=0, atol=1e-13)
    np.testing.assert_allclose(ev["U"], [6.0, 2.0, 0.0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(ev["V"], [[3.6, 4.8], [1.5, 0.0], [0.0, 0.0]], rtol=0, atol=1e-14)


@pytest.mark.parametrize("ball,psi,dmult", [(0, 1 + 18 - 2 + 0.3125, 32.0), (1, 1 + 1.5625 - 0.3125 + 0.3125, 2.0),
                                            (2, 1 + 0 - 0.1025 + 0.3125, 0.41)])
def test_al_eval_single_case_multiplier_terms(ball, psi, dmult):
    # each ball alone: the -||w||^2 / (2 sigma) term and the multiplier change
    # carry the case's hand value (a sign or factor slip in either fails)
    C, R, U, V, x, xbar, sigma, tau = _three_case_instance()
    sl = slice(ball, ball + 1)
    ev = oracle.al_eval(C[sl], R[sl], U[sl], V[sl], x, xbar, sigma, tau)
    np.testing.assert_allclose(ev["psi"], psi, rtol=0, atol=1e-13)
    np.testing.assert_allclose(ev["dmult"], dmult, rtol=0, atol=1e-13)
