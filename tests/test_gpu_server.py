"""Multi-instance server on the GPU: every result equals meb_solve's on the
same input bitwise, alone and in the mix, and matches the oracle.

The server batches the solver steps of all requests inside a ripALM run into
shared launches; each request keeps its own launch shape and reduction
order, so the results are reproducible whatever else is in flight.
"""
import time

import numpy as np
import pytest
import torch

from paper_2605_31425_amd import inputs, meb
from tests.gpu_common import dev, gpu

pytestmark = gpu

# (m, d, seed): the serving dimensions, small enough for the oracle
MIX = [(1500, 2, 1), (4000, 3, 2), (2500, 10, 3), (900, 50, 4), (700, 200, 5), (20000, 10, 6), (3000, 2, 7),
       (1200, 50, 8), (5000, 3, 9), (1000, 200, 10), (8000, 50, 11), (600, 10, 12)]


def _instances(cases):
    out = []
    for m, d, s in cases:
        C, R = inputs.serving_instance(m, d, 1000 + s)
        out.append((C, R, dev(C), dev(R)))
    return out


def _solve_alone(inst):
    res = []
    for _, _, Cd, Rd in inst:
        r, c, st = meb.solve(Cd, Rd, mode="mixed")
        res.append((r, c))
    torch.cuda.synchronize()
    return res


def _serve(inst, pool_bytes=1 << 30, max_active=64, order=None, gaps=None):
    srv = meb.Server(pool_bytes, max_active=max_active, max_d=256, mode="mixed")
    try:
        order = range(len(inst)) if order is None else order
        tickets = {}
        for k, i in enumerate(order):
            if gaps is not None:
                time.sleep(gaps[k])
            _, _, Cd, Rd = inst[i]
            tickets[srv.submit(Cd, Rd, tag=i)] = i
        got = {}
        t0 = time.time()
        while len(got) < len(inst):
            for r in srv.poll(wait_ms=200):
                got[r["tag"]] = r
            assert time.time() - t0 < 120, srv.info()
        info = srv.info()
    finally:
        srv.close()
    return got, info


def test_server_results_equal_solve_bitwise():
    inst = _instances(MIX)
    alone = _solve_alone(inst)
    got, info = _serve(inst)
    assert info["completed"] == len(MIX) and info["failed"] == 0
    assert info["mean_tick_items"] > 1.0  # requests really shared ticks
    for i, (r, c) in enumerate(alone):
        g = got[i]
        assert g["status"] >= 0, g["message"]
        assert g["r"] == r, (MIX[i], g["r"], r)
        np.testing.assert_array_equal(g["c"], c)


def test_server_alone_equals_in_mix():
    inst = _instances(MIX[:6])
    mix, _ = _serve(inst, order=[5, 4, 3, 2, 1, 0])
    for i in (0, 4):
        one, info = _serve([inst[i]])
        assert info["completed"] == 1
        assert one[0]["r"] == mix[i]["r"]
        np.testing.assert_array_equal(one[0]["c"], mix[i]["c"])


def test_server_matches_oracle():
    import oracle
    cases = [(1500, 2, 1), (2500, 10, 3), (900, 50, 4), (700, 200, 5)]
    inst = _instances(cases)
    got, _ = _serve(inst)
    for i, (C, R, _, _) in enumerate(inst):
        ro, co, st = oracle.ripalm(C, R, tol=1e-12)
        r_ref = st["r_fixed"]
        g = got[i]
        assert abs(g["r"] - r_ref) <= 1e-8 * r_ref, (cases[i], g["r"], r_ref)
        reach = np.linalg.norm(C - g["c"], axis=1) + R
        assert reach.max() - g["r"] <= 1e-10 * (1 + g["r"])


def test_server_small_pool_admits_in_order():
    # a pool that holds about two requests: admission waits for room, and the
    # results are still those of meb_solve
    cases = [(3000, 10, 21), (3000, 10, 22), (3000, 10, 23), (3000, 10, 24), (3000, 10, 25)]
    inst = _instances(cases)
    alone = _solve_alone(inst)
    nb = meb.lib.meb_workspace_size
    import ctypes
    b = ctypes.c_size_t()
    meb._check(nb(3000, 10, meb.MEB_F64, ctypes.byref(meb.options(mode="mixed")), ctypes.byref(b)))
    got, info = _serve(inst, pool_bytes=int(2.5 * b.value) + (1 << 20), max_active=8)
    assert info["pool_peak"] <= info["pool_capacity"]
    admits = [got[i]["t_admit_ms"] for i in range(len(cases))]
    assert admits == sorted(admits)
    for i, (r, c) in enumerate(alone):
        assert got[i]["r"] == r
        np.testing.assert_array_equal(got[i]["c"], c)


def test_server_poisson_stream_feasible():
    reqs = inputs.serving_requests(40, 7, log_m=(3.0, 4.3))
    arr = inputs.poisson_arrivals(len(reqs), 400.0, 8)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    inst = [(C, R, dev(C), dev(R)) for C, R in (inputs.serving_instance(m, d, s) for m, d, s in reqs)]
    got, info = _serve(inst, gaps=gaps)
    assert info["completed"] == len(reqs) and info["failed"] == 0
    lat = []
    for i, (C, R, _, _) in enumerate(inst):
        g = got[i]
        assert g["status"] >= 0
        reach = np.linalg.norm(C - g["c"], axis=1) + R
        assert reach.max() - g["r"] <= 1e-10 * (1 + g["r"])
        lat.append(g["t_done_ms"] - g["t_submit_ms"])
    assert np.percentile(lat, 99) > 0


def test_server_rejects_request_larger_than_pool():
    srv = meb.Server(1 << 22, max_active=4, max_d=256)
    try:
        C = torch.zeros((200000, 50), dtype=torch.float64, device="cuda")
        with pytest.raises(meb.MebError):
            srv.submit(C, None)
        with pytest.raises(meb.MebError):
            srv.submit(torch.zeros((10, 300), dtype=torch.float64, device="cuda"), None)
    finally:
        srv.close()
