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
