"""meb_check_feasible_noalloc (fixed library scratch, no workspace) against
meb_check_feasible (caller workspace): the same maximum, argmax, violator
count and violator list, on two calls in a row, the second one smaller.
Index outputs must agree exactly (same FP64 arithmetic on both sides)."""
import numpy as np
import pytest
import torch

from tests.gpu_common import gpu

pytestmark = gpu


def _case(m, d, seed, frac):
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(m, d))
    R = rng.uniform(0, 0.05, size=m)
    c = rng.normal(size=d) * 0.01
    reach = np.linalg.norm(C - c, axis=1) + R
    r = float(np.quantile(reach, 1.0 - frac))  # about frac of the balls violate
    return C, R, c, r


def _compare(C, R, c, r, eps, cap, dtype):
    from paper_2605_31425_amd import meb
    Cd = torch.as_tensor(C, device="cuda:0").to(dtype)
    Rd = torch.as_tensor(R, device="cuda:0").to(dtype)
    dm_ref, am_ref, viol_ref, nv_ref = meb.check_feasible(Cd, Rd, r, c, eps, viol_cap=cap)
    out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device="cuda:0")
    dm, am, nv = meb.check_feasible_noalloc(Cd, Rd, r, c, eps, viol_idx=out if cap > 0 else None)
    assert dm == dm_ref and am == am_ref and nv == nv_ref, (dm, dm_ref, am, am_ref, nv, nv_ref)
    k = min(nv, cap)
    assert torch.equal(out[:k].cpu(), viol_ref[:k].cpu())
    if cap > k:
        assert (out[k:cap] == -7).all()  # nothing written past the count
    # and against the plain definition (ascending violated indices)
    Ch = Cd.double().cpu().numpy()
    Rh = Rd.double().cpu().numpy()
    reach = np.linalg.norm(Ch - c, axis=1) + Rh - r
    assert nv == int((reach > eps).sum())
    return nv


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_workspace_entry_point_twice(dtype):
    C, R, c, r = _case(300_001, 37, 11, 0.02)
    n1 = _compare(C, R, c, r, 1e-12, 4000, dtype)   # cap below the count: truncated list
    assert n1 > 4000
    C2, R2, c2, r2 = _case(5_003, 8, 12, 0.1)         # second call, smaller input
    n2 = _compare(C2, R2, c2, r2, 1e-12, 5_003, dtype)
    assert 0 < n2 < 5_003


def test_noalloc_no_violator_and_no_list():
    C, R, c, r = _case(70_000, 16, 13, 0.0)
    from paper_2605_31425_amd import meb
    Cd = torch.as_tensor(C, device="cuda:0")
    Rd = torch.as_tensor(R, device="cuda:0")
    out = torch.full((16,), -7, dtype=torch.int64, device="cuda:0")
    dm, am, nv = meb.check_feasible_noalloc(Cd, Rd, r + 1.0, c, 1e-12, viol_idx=out)
    assert nv == 0 and dm < 0 and (out == -7).all()
    dm2, am2, nv2 = meb.check_feasible_noalloc(Cd, Rd, r, c, 1e-12)   # no list requested
    dm_ref, am_ref, _, nv_ref = meb.check_feasible(Cd, Rd, r, c, 1e-12, viol_cap=0)
    assert (dm2, am2, nv2) == (dm_ref, am_ref, nv_ref)
