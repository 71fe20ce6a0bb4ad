"""Helpers shared by the GPU parity tests (instance builders and
normwise error scales).  Nothing here computes the method."""
import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def cone_multipliers(rng, m, d, frac=0.5):
    """Random multipliers in the second-order cone, some exactly zero."""
    U = np.abs(rng.normal(size=m)) * (rng.uniform(size=m) < frac)
    V = rng.normal(size=(m, d))
    V *= (U / np.maximum(np.linalg.norm(V, axis=1), 1e-300) * rng.uniform(0, 1, m))[:, None]
    return U, V


def near_point(rng, C, R):
    """A point close to the optimum region so that all three projection
    cases occur: center near the mean, radius around the typical reach."""
    c = C.mean(0) + rng.normal(size=C.shape[1]) * 0.05
    reach = np.linalg.norm(C - c, axis=1) + (0 if R is None else R)
    r = np.quantile(reach, 0.9)
    return np.concatenate([[r], c])


def ball_terms(C, R, U, V, y, sigma):
    """Per-ball projection inputs of an evaluation at y: t_i, the rows s_i
    and n_i = ||s_i|| (z_i = (r_i - y_r, c_i - y_c) + (u_i, v_i) / sigma)."""
    m = C.shape[0]
    t = (np.zeros(m) if R is None else R) - y[0] + (0 if U is None else U / sigma)
    S = C - y[1:] + (0 if V is None else V / sigma)
    return t, S, np.linalg.norm(S, axis=1)


def hess_scale(C, R, U, V, y, sigma, tau):
    """Per-component sum of magnitudes of the terms of the generalized
    Hessian tau/sigma I + sigma sum_i P_i at y: the error scale of each entry.
    Interior balls add sigma on the diagonal; a ball in the third case adds
    sigma/2 [[1, |w|^T], [|w|, |1 + t/n| I + |t/n| |w||w|^T]], w = s / n."""
    t, S, n = ball_terms(C, R, U, V, y, sigma)
    d = C.shape[1]
    inter = n <= t
    mid = ~inter & ~(n <= -t)
    sc = np.zeros((d + 1, d + 1))
    sc += tau / sigma * np.eye(d + 1)
    sc += sigma * inter.sum() * np.eye(d + 1)
    if mid.any():
        nm, tm = n[mid], t[mid]
        W = np.abs(S[mid]) / nm[:, None]
        r = np.abs(tm / nm)
        sc[0, 0] += sigma / 2 * mid.sum()
        sc[0, 1:] += sigma / 2 * W.sum(0)
        sc[1:, 0] += sigma / 2 * W.sum(0)
        sc[1:, 1:] += sigma / 2 * (np.abs(1 + tm / nm).sum() * np.eye(d) + (W * r[:, None]).T @ W)
    return sc


def mult_scale(C, R, U, V, y, sigma):
    """Per-ball magnitude of the terms that form the updated multiplier
    sigma Pi(z_i): sigma times the magnitudes of the inputs of t_i and s_i
    (|r_i| + |y_r| + |u_i| / sigma + ||c_i|| + ||y_c|| + ||v_i|| / sigma), so
    that rounding of the inputs in the working precision is covered."""
    m = C.shape[0]
    a = (np.zeros(m) if R is None else np.abs(R)) + abs(y[0]) + np.linalg.norm(C, axis=1) + np.linalg.norm(y[1:])
    if U is not None:
        a = a + (np.abs(U) + np.linalg.norm(V, axis=1)) / sigma
    return sigma * a


def case_allowance(C, R, U, V, y, sigma, rel):
    """Additive error allowance of the generalized Hessian for balls whose
    projection case is decided within `rel` of a case boundary (||s|| = t or
    ||s|| = -t): there the working precision may pick either case, and the
    element of the generalized Jacobian jumps (Pi itself is continuous, so
    g, Psi and the multipliers do not).  Either choice is correct; each such
    ball may change H by up to sigma (|w^||w^|^T + I), w^ = (1, s / ||s||)."""
    t, S, n = ball_terms(C, R, U, V, y, sigma)
    gap = np.minimum(np.abs(n - t), np.abs(n + t)) / (np.abs(t) + n + 1e-300)
    amb = gap <= rel
    d = C.shape[1]
    al = np.zeros((d + 1, d + 1))
    if amb.any():
        W = np.concatenate([np.ones((amb.sum(), 1)), np.abs(S[amb]) / (n[amb][:, None] + 1e-300)], axis=1)
        al += sigma * (W.T @ W + amb.sum() * np.eye(d + 1))
    return al
