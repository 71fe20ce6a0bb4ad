"""Per-kernel parity of the HIP path against the CPU oracle (GPU).

meb_al_eval is compared with the oracle's direct per-ball evaluator on the
same seeded inputs: FP64 to 1e-12 and FP32 to 1e-5, normwise (the error of
each output is measured against the sum of magnitudes of the terms that
make it up, since g -> 0 near the optimum).  The screening and feasibility
index sets are compared exactly, except for balls whose slack lies within
rounding of the threshold, where either decision is correct.  Sizes span
several waves and a ragged tail; d covers every lane-group configuration.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import case_allowance, cone_multipliers, dev, gpu, hess_scale, mult_scale, near_point

pytestmark = gpu

SHAPES = [(1, 3), (7, 1), (130, 2), (1000, 3), (1500, 5), (2222, 7), (4097, 10), (3001, 17), (2500, 64),
          (1999, 100), (601, 129), (300, 512), (150, 1001)]


def _inst(seed, m, d, balls=True):
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(m, d))
    R = rng.uniform(0, 0.2, m) if balls else None
    return rng, C, R


@pytest.mark.parametrize("m,d", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_al_eval_parity(m, d, dtype):
    from paper_2605_31425_amd import meb
    print(f"al_eval m={m} d={d} {dtype}", flush=True)
    rng, C, R = _inst(m * 1000 + d, m, d, balls=(m % 2 == 1))
    U, V = cone_multipliers(rng, m, d)
    x = near_point(rng, C, R)
    xbar = x + rng.normal(size=d + 1) * 0.01
    direction = rng.normal(size=d + 1) * 0.02
    sigma, tau = 3.0, 0.7
    etas = [1.0, 0.5, 0.25, 0.125, 0.0]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":  # the oracle sees exactly the FP32 inputs
        C, U, V = C.astype(np.float32).astype(np.float64), U.astype(np.float32).astype(np.float64), \
            V.astype(np.float32).astype(np.float64)
        R = None if R is None else R.astype(np.float32).astype(np.float64)
    tol = 1e-12 if dtype == "f64" else 1e-5
    # the FP64-accumulating contraction (the matrix-core forms have tests of their own)
    out = meb.al_eval(dev(C, tdt), dev(R, tdt), dev(U, tdt), dev(V, tdt), x, xbar, sigma, tau, direction=direction,
                      etas=etas, want=meb.WANT_ALL | (meb.MEB_HESS_F64 << 8))
    y = x + direction
    ref = oracle.al_eval(C, R, U, V, y, xbar, sigma, tau)
    # scales: sums of magnitudes of the terms
    Up, Vp = ref["U"], ref["V"]
    sg = 1.0 + np.concatenate([[np.abs(Up).sum()], np.abs(Vp).sum(0)]) + tau / sigma * np.abs(y - xbar)
    assert np.all(np.abs(out["g"] - ref["g"]) <= tol * sg), np.abs(out["g"] - ref["g"]).max()
    # H per component against the sum of magnitudes of its terms (plus, for
    # balls on a case boundary to working precision, either case's element)
    sH = hess_scale(C, R, U, V, y, sigma, tau)
    aH = case_allowance(C, R, U, V, y, sigma, 10 * tol)
    assert np.all(np.abs(out["H"] - ref["H"]) <= tol * sH + aH), (np.abs(out["H"] - ref["H"]) / sH).max()
    spsi = abs(y[0]) + sigma / 2 * (np.sum((Up / sigma) ** 2) + np.sum((Vp / sigma) ** 2)) + \
        (np.sum(U ** 2) + np.sum(V ** 2)) / (2 * sigma) + tau / (2 * sigma) * np.sum((y - xbar) ** 2) + 1.0
    assert abs(out["psi"] - ref["psi"]) <= tol * spsi
    for eta, pv in zip(etas, out["psi_trial"]):
        rt = oracle.al_eval(C, R, U, V, x + eta * direction, xbar, sigma, tau, want_h=False)
        assert abs(pv - rt["psi"]) <= 10 * tol * spsi, (eta, pv, rt["psi"])
    sdm = np.sum(Up ** 2) + np.sum(Vp ** 2) + np.sum(U ** 2) + np.sum(V ** 2) + 1e-300
    assert abs(out["dmult"] - ref["dmult"]) <= tol * sdm
    Un, Vn = out["U"].double().cpu().numpy(), out["V"].double().cpu().numpy()
    sw = np.abs(Up).max() + 1
    # updated multipliers per ball against the magnitude of their terms
    su = mult_scale(C, R, U, V, y, sigma) + 1e-300
    assert np.all(np.abs(Un - Up) <= tol * su), (np.abs(Un - Up) / su).max()
    assert np.all(np.abs(Vn - Vp) <= tol * su[:, None]), (np.abs(Vn - Vp) / su[:, None]).max()
    k_ref, parts = oracle.kkt_max(C, R, Up, Vp, y)
    scale_k = [1 + np.abs(Up).sum(), 1 + np.abs(Vp).sum(), 1 + np.abs(y).max() + np.abs(C).max(), 1 + sw,
               (1 + np.abs(y).max() + np.abs(C).max()) * sw]
    for a, b, s in zip(out["kkt"], parts, scale_k):
        assert abs(a - b) <= 10 * tol * s, (out["kkt"], parts)


@pytest.mark.parametrize("m,d", SHAPES)
def test_check_feasible_parity(m, d):
    from paper_2605_31425_amd import meb
    print(f"check m={m} d={d}", flush=True)
    rng, C, R = _inst(7 * m + d, m, d)
    x = near_point(rng, C, R)
    eps = 1e-3
    dmax, am, viol, nv = meb.check_feasible(dev(C), dev(R), x[0], x[1:], eps)
    rd, ra, rv = oracle.check_feasible(C, R, x[0], x[1:], eps)
    scale = np.abs(C).max() * np.sqrt(d) + 1
    assert abs(dmax - rd) <= 1e-14 * scale
    reach = np.linalg.norm(C - x[1:], axis=1) + R - x[0]
    tie = np.abs(reach - reach.max()) <= 1e-14 * scale
    assert am == ra or tie[am]
    got = set(viol.cpu().numpy().tolist())
    exp = set(rv.tolist())
    border = set(np.flatnonzero(np.abs(reach - eps) <= 1e-13 * scale).tolist())
    assert (got ^ exp) <= border
    assert nv == len(got)
    v = viol.cpu().numpy()
    assert np.all(np.diff(v) > 0)
    # a capacity smaller than the count keeps the first indices
    if nv > 2:
        _, _, v2, nv2 = meb.check_feasible(dev(C), dev(R), x[0], x[1:], eps, viol_cap=2)
        assert nv2 == nv and np.array_equal(v2.cpu().numpy(), v[:2])


@pytest.mark.parametrize("m,d", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_screen_parity(m, d, dtype):
    from paper_2605_31425_amd import meb
    print(f"screen m={m} d={d} {dtype}", flush=True)
    rng, C, R = _inst(11 * m + d, m, d, balls=(d % 2 == 0))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        C = C.astype(np.float32).astype(np.float64)
        R = None if R is None else R.astype(np.float32).astype(np.float64)
    x = near_point(rng, C, R)
    tol = 0.3
    keep, slack = meb.screen(dev(C, tdt), dev(R, tdt), x[0], x[1:], tol, want_slack=True)
    rk, rs = oracle.screen(C, R, x[0], x[1:], tol)
    scale = np.abs(C).max() * np.sqrt(d) + 1
    assert np.abs(slack.cpu().numpy() - rs).max() <= 1e-14 * scale
    border = set(np.flatnonzero(np.abs(rs - tol) <= 1e-13 * scale).tolist())
    got = keep.cpu().numpy()
    assert np.all(np.diff(got) > 0)
    assert (set(got.tolist()) ^ set(rk.tolist())) <= border


@pytest.mark.parametrize("m,d", [(1, 1), (333, 7), (5000, 100), (257, 1000)])
def test_prepare_f32_bit_exact(m, d):
    from paper_2605_31425_amd import meb
    rng, C, R = _inst(m + d, m, d)
    C = C * 50 + 1000.0  # offset data: the shift matters
    origin = C[0].copy()
    C32, R32, L = meb.prepare_f32(dev(C), dev(R), origin)
    rc, rr, rL = oracle.prepare_f32(C, R, origin)
    assert np.array_equal(C32.cpu().numpy(), rc)
    assert np.array_equal(R32.cpu().numpy(), rr)
    assert abs(L - rL) <= 1e-14 * rL


# n >= 320: the factorization across many workgroups (one launch per phase)
@pytest.mark.parametrize("n", [1, 2, 3, 11, 63, 64, 65, 101, 127, 128, 141, 300, 320, 353, 1001, 1025])
def test_chol_solve_parity(n):
    from paper_2605_31425_amd import meb
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)
    b = rng.normal(size=n)
    y = meb.chol_solve(dev(A), dev(b)).cpu().numpy()
    ref = oracle.chol_solve(A, b)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(meb.MebError):
        meb.chol_solve(dev(-np.eye(n)), dev(b))


@pytest.mark.parametrize("n", [5, 64, 101, 127, 400])
def test_chol_solve_ill_conditioned_backward_error(n):
    # condition number 1e10, like the Hessians late in a run: compare the
    # backward error (residual), which a stable solve keeps near eps
    from paper_2605_31425_amd import meb
    rng = np.random.default_rng(100 + n)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = (Q * np.logspace(0, 10, n)) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.normal(size=n)
    y = meb.chol_solve(dev(A), dev(b)).cpu().numpy()
    res = np.abs(A @ y - b).max()
    assert res <= 64 * n * np.finfo(float).eps * np.abs(A).max() * np.abs(y).max()


@pytest.mark.parametrize("n", [2, 40, 101, 127, 333, 700])
def test_chol_solve_detects_late_negative_pivot(n):
    # positive diagonal, one negative eigenvalue: the failure shows only in a
    # later pivot
    from paper_2605_31425_amd import meb
    rng = np.random.default_rng(200 + n)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.linspace(1.0, 2.0, n)
    ev[rng.integers(n)] = -1.0
    A = (Q * ev) @ Q.T
    A = 0.5 * (A + A.T)
    assert np.all(np.diag(A) > 0) or n == 2
    if n == 2:
        A = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(meb.MebError):
        meb.chol_solve(dev(A), dev(rng.normal(size=n)))


def test_al_eval_deterministic_bitwise():
    from paper_2605_31425_amd import meb
    rng, C, R = _inst(5, 20000, 50)
    U, V = cone_multipliers(rng, 20000, 50)
    x = near_point(rng, C, R)
    a = meb.al_eval(dev(C), dev(R), dev(U), dev(V), x, x, 2.0, 1.0)
    b = meb.al_eval(dev(C), dev(R), dev(U), dev(V), x, x, 2.0, 1.0)
    assert a["psi"] == b["psi"] and np.array_equal(a["g"], b["g"]) and np.array_equal(a["H"], b["H"])


# ---------------------------------------------------------------------------
# The rank-one Hessian contraction in each arithmetic (MEB_HESS_*), against
# the oracle per component, relative to the sum of magnitudes of the terms:
# FP64 inputs (vector FMAs or FP64 matrix cores) 1e-12; FP32 inputs with
# FP32 matrix-core accumulation 1e-5; BF16 inputs (8 significant bits, two
# roundings per product) with FP32 accumulation 1.5e-2.
# ---------------------------------------------------------------------------
HESS_CASES = [("f64", "f64", 1e-12), ("f64", "mfma_f64", 1e-12), ("f32", "f64", 1e-5), ("f32", "mfma_f32", 1e-5),
              ("f32", "mfma_bf16", 1.5e-2)]


@pytest.mark.parametrize("m,d", [(4001, 5), (3001, 64), (2500, 100), (1201, 129), (700, 300), (301, 1001)])
@pytest.mark.parametrize("dtype,hess,tol", HESS_CASES)
def test_hessian_contraction_arithmetics(m, d, dtype, hess, tol):
    from paper_2605_31425_amd import meb
    print(f"hess m={m} d={d} {dtype} {hess}", flush=True)
    rng, C, R = _inst(7 * m + d, m, d)
    U, V = cone_multipliers(rng, m, d)
    x = near_point(rng, C, R)
    xbar = x + rng.normal(size=d + 1) * 0.01
    sigma, tau = 2.0, 0.9
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        C, R, U, V = (a.astype(np.float32).astype(np.float64) for a in (C, R, U, V))
    code = meb._HESS[hess]
    out = meb.al_eval(dev(C, tdt), dev(R, tdt), dev(U, tdt), dev(V, tdt), x, xbar, sigma, tau,
                      want=meb.WANT_HESS | (code << 8))
    ref = oracle.al_eval(C, R, U, V, x, xbar, sigma, tau)
    assert ref["counts"][2] > 0  # balls in the third projection case exist
    sH = hess_scale(C, R, U, V, x, sigma, tau)
    aH = case_allowance(C, R, U, V, x, sigma, 1e-5 if dtype == "f32" else 1e-12)
    err = np.maximum(np.abs(out["H"] - ref["H"]) - aH, 0.0) / sH
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))
    # symmetric to rounding (the two triangles of a diagonal tile multiply the
    # coefficient into different factors)
    assert np.all(np.abs(out["H"] - out["H"].T) <= 2 * tol * sH)


# ---------------------------------------------------------------------------
# Full-size evaluation passes: shapes at which every wave streams many batches
# through its LDS ring (the ring wraps, full 64-ball batches, the FP32 partial
# sums flushed every 64 balls, the radii and multipliers copied a batch
# ahead), checked against the oracle's evaluator to the same bars.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,d", [(200_000, 100), (2_000_000, 5), (300_001, 36)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_al_eval_full_size(m, d, dtype):
    from paper_2605_31425_amd import meb
    print(f"al_eval full m={m} d={d} {dtype}", flush=True)
    rng = np.random.default_rng(m + d)
    C = rng.uniform(-1, 1, size=(m, d))
    R = rng.uniform(0, 0.1, m)
    # multipliers on about 1% of the balls (as late in a run)
    U, V = cone_multipliers(rng, m, d, frac=0.01)
    x = near_point(rng, C, R)
    xbar = x + rng.normal(size=d + 1) * 0.01
    direction = rng.normal(size=d + 1) * 0.02
    sigma, tau = 3.0, 0.7
    etas = [1.0, 0.5, 0.25, 0.0]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        C, R, U, V = (a.astype(np.float32).astype(np.float64) for a in (C, R, U, V))
    tol = 1e-12 if dtype == "f64" else 1e-5
    out = meb.al_eval(dev(C, tdt), dev(R, tdt), dev(U, tdt), dev(V, tdt), x, xbar, sigma, tau, direction=direction,
                      etas=etas, want=meb.WANT_ALL | (meb.MEB_HESS_F64 << 8))
    y = x + direction
    ref = oracle.al_eval(C, R, U, V, y, xbar, sigma, tau)
    Up, Vp = ref["U"], ref["V"]
    sg = 1.0 + np.concatenate([[np.abs(Up).sum()], np.abs(Vp).sum(0)]) + tau / sigma * np.abs(y - xbar)
    assert np.all(np.abs(out["g"] - ref["g"]) <= tol * sg), np.abs(out["g"] - ref["g"]).max()
    sH = hess_scale(C, R, U, V, y, sigma, tau)
    aH = case_allowance(C, R, U, V, y, sigma, 10 * tol)
    assert np.all(np.abs(out["H"] - ref["H"]) <= tol * sH + aH), (np.abs(out["H"] - ref["H"]) / sH).max()
    spsi = abs(y[0]) + sigma / 2 * (np.sum((Up / sigma) ** 2) + np.sum((Vp / sigma) ** 2)) + \
        (np.sum(U ** 2) + np.sum(V ** 2)) / (2 * sigma) + tau / (2 * sigma) * np.sum((y - xbar) ** 2) + 1.0
    assert abs(out["psi"] - ref["psi"]) <= tol * spsi
    for eta, pv in zip(etas, out["psi_trial"]):
        rt = oracle.al_eval(C, R, U, V, x + eta * direction, xbar, sigma, tau, want_h=False)
        assert abs(pv - rt["psi"]) <= 10 * tol * spsi, (eta, pv, rt["psi"])
    sdm = np.sum(Up ** 2) + np.sum(Vp ** 2) + np.sum(U ** 2) + np.sum(V ** 2) + 1e-300
    assert abs(out["dmult"] - ref["dmult"]) <= tol * sdm
    su = mult_scale(C, R, U, V, y, sigma) + 1e-300
    Un, Vn = out["U"].double().cpu().numpy(), out["V"].double().cpu().numpy()
    assert np.all(np.abs(Un - Up) <= tol * su), (np.abs(Un - Up) / su).max()
    assert np.all(np.abs(Vn - Vp) <= tol * su[:, None]), (np.abs(Vn - Vp) / su[:, None]).max()


# ---------------------------------------------------------------------------
# The matrix-free Hessian-vector product (meb_hess_vec, the product the CG
# Newton solver iterates with) against the oracle's H times q, per component
# relative to the sum of magnitudes of the terms (|H| |q| with the scale of
# each entry of H).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,d", [(4001, 5), (3001, 64), (2500, 100), (700, 300), (301, 1001), (200_000, 100)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hess_vec_parity(m, d, dtype):
    from paper_2605_31425_amd import meb
    print(f"hess_vec m={m} d={d} {dtype}", flush=True)
    rng, C, R = _inst(11 * m + d, m, d)
    U, V = cone_multipliers(rng, m, d, frac=0.3)
    x = near_point(rng, C, R)
    q = rng.normal(size=d + 1)
    sigma, tau = 2.5, 0.8
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        C, R, U, V = (a.astype(np.float32).astype(np.float64) for a in (C, R, U, V))
    tol = 1e-12 if dtype == "f64" else 1e-5
    out = meb.hess_vec(dev(C, tdt), dev(R, tdt), dev(U, tdt), dev(V, tdt), x, sigma, tau, q)
    ref = oracle.al_eval(C, R, U, V, x, x, sigma, tau)
    Hq = ref["H"] @ q
    sc = hess_scale(C, R, U, V, x, sigma, tau) @ np.abs(q)
    al = case_allowance(C, R, U, V, x, sigma, 10 * tol) @ np.abs(q)
    err = np.abs(out - Hq)
    assert np.all(err <= tol * sc + al), (err / sc).max()
