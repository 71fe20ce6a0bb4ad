"""Seeded synthetic MEB instances.

Random numbers only: nothing here evaluates the method.  Every generator is
deterministic in its seed (numpy PCG64 via ``default_rng``) and returns FP64
host arrays ``(C, R)`` with C of shape (m, d) row-major and R of shape (m,)
(``R is None`` for point sets).
"""
import numpy as np


def points_normal(m, d, seed):
    """Points, centers iid N(0, I)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, d)), None


def balls_uniform(m, d, seed, rmax=0.1):
    """Balls, centers uniform in [-1, 1]^d, radii uniform in [0, rmax]."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(-1.0, 1.0, (m, d))
    R = rng.uniform(0.0, rmax, m)
    return C, R


def balls_normal(m, d, seed, rstd=0.05):
    """Balls, centers iid N(0, I), radii |N(0, rstd^2)|."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, d))
    R = np.abs(rng.normal(0.0, rstd, m))
    return C, R


def points_ball_sphere(m, d, seed, sphere_frac=0.1):
    """Points: a fraction uniform in the unit ball, the rest on the unit
    sphere, randomly interleaved (many near-boundary candidates)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    n_in = m - int(round(sphere_frac * m))
    rad = rng.uniform(size=n_in) ** (1.0 / d)
    perm = rng.permutation(m)
    inside = perm[:n_in]
    g[inside] *= rad[:, None]
    return g, None


def with_cross_polytope(C):
    """Appends +-e_k for every axis k; if every input row has norm <= 1 the
    minimum enclosing ball of the result is exactly the unit ball at 0."""
    m, d = C.shape
    E = np.concatenate([np.eye(d), -np.eye(d)])
    return np.concatenate([C, E])


def lcg_instance(m, d):
    """The deterministic instances of the experiments (Section 5, "Test
    instances"): psi_0 = 7, psi_{j+1} = (445 psi_j + 1) mod 4096, values
    psi_j / 40.96 for j >= 1, filled in the order r_1, c_1(1..d), r_2, ..."""
    n = m * (d + 1)
    vals = np.empty(n)
    psi = 7
    for j in range(n):
        psi = (445 * psi + 1) % 4096
        vals[j] = psi / 40.96
    vals = vals.reshape(m, d + 1)
    return np.ascontiguousarray(vals[:, 1:]), np.ascontiguousarray(vals[:, 0])


def serving_requests(n, seed, dims=(2, 3, 10, 50, 200), log_m=(3.0, 6.0), rmax=0.05):
    """Shapes of a request stream: m = floor(10^U[log_m]), d uniform over
    dims.  Returns a list of (m, d, instance_seed); the instance itself is
    drawn by ``serving_instance``."""
    rng = np.random.default_rng(seed)
    ms = np.floor(10.0 ** rng.uniform(log_m[0], log_m[1], n)).astype(np.int64)
    ds = rng.choice(np.asarray(dims), n)
    return [(int(ms[i]), int(ds[i]), seed * (1 << 32) + i) for i in range(n)]


def serving_instance(m, d, seed, rmax=0.05):
    """One request: centers N(0, I), radii uniform in [0, rmax]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, d)), rng.uniform(0.0, rmax, m)


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of a Poisson stream of n requests at `rate` per s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def serving_bank_device(n_doubles, n_radii, seed, rmax=0.05, device="cuda"):
    """Device-resident random numbers for a long request stream: iid N(0, 1)
    FP64 values (request centers are row-major windows of it) and radii
    uniform in [0, rmax].  Drawn on the device from torch's seeded generator,
    so a multi-gigabyte stream needs no host-side generation."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    Z = torch.randn(int(n_doubles), dtype=torch.float64, device=device, generator=g)
    Rb = torch.rand(int(n_radii), dtype=torch.float64, device=device, generator=g) * rmax
    return Z, Rb
