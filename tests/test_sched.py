"""Admission policy of the multi-instance server, on a simulated clock.

meb_sched_simulate runs the server's own FIFO / first-fit admission code
with caller-given arrival and service times (an injected executor), so the
policy is checked on the CPU: pool budget and slot limits never exceeded,
regions of concurrent requests disjoint, admission in arrival order, and a
request admitted as soon as the pool allows when it reaches the head.
"""
import numpy as np
import pytest

from paper_2605_31425_amd import meb

GRAN = 256


def _events(ta, td):
    """(time, +1/-1, id) sorted with departures before arrivals at equal times."""
    ev = [(t, 1, i) for i, t in enumerate(ta)] + [(t, -1, i) for i, t in enumerate(td)]
    ev.sort(key=lambda e: (e[0], e[1]))
    return ev


def _check_invariants(arrival, service, nbytes, pool, slots, ta, td, off):
    n = len(arrival)
    rb = (np.asarray(nbytes, dtype=np.int64) + GRAN - 1) // GRAN * GRAN
    assert np.all(ta >= arrival - 1e-12)
    np.testing.assert_allclose(td - ta, service)
    # FIFO: admission times are non-decreasing in arrival order
    assert np.all(np.diff(ta) >= 0)
    # at every instant: slot count, bytes, disjoint regions inside the pool
    live = {}
    for t, kind, i in _events(ta, td):
        if kind < 0:
            live.pop(i)
            continue
        for j, (o, b) in live.items():
            assert off[i] + rb[i] <= o or o + b <= off[i], (i, j)
        assert off[i] + rb[i] <= pool
        live[i] = (int(off[i]), int(rb[i]))
        assert len(live) <= slots
        assert sum(b for _, b in live.values()) <= pool
    assert not live


def _random_case(seed, n=400, pool=1 << 24, slots=16):
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0, n))
    service = rng.exponential(8.0, n)
    nbytes = rng.integers(1, pool // 3, n).astype(np.uint64)
    return arrival, service, nbytes, pool, slots


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_invariants_random(seed):
    arrival, service, nbytes, pool, slots = _random_case(seed)
    ta, td, off = meb.sched_simulate(arrival, service, nbytes, pool, slots)
    _check_invariants(arrival, service, nbytes, pool, slots, ta, td, off)


def test_idle_server_admits_at_arrival():
    # well-separated arrivals: every request finds the server empty
    n = 50
    arrival = np.arange(n) * 10.0
    service = np.full(n, 1.0)
    nbytes = np.full(n, 1000, dtype=np.uint64)
    ta, td, off = meb.sched_simulate(arrival, service, nbytes, 1 << 20, 4)
    np.testing.assert_array_equal(ta, arrival)
    assert np.all(off == 0)


def test_slot_limit_serializes():
    # one slot: each request starts when the previous one ends
    n = 20
    arrival = np.zeros(n)
    service = np.arange(1, n + 1, dtype=float)
    ta, td, _ = meb.sched_simulate(arrival, service, np.full(n, 64, dtype=np.uint64), 1 << 20, 1)
    np.testing.assert_allclose(ta[1:], td[:-1])
    np.testing.assert_allclose(td[-1], service.sum())


def test_head_of_line_blocks_smaller_requests():
    # the big request at the head waits for room; the small one behind it
    # waits too (FIFO), although it alone would fit
    pool = 100 * GRAN
    arrival = np.array([0.0, 1.0, 2.0])
    service = np.array([10.0, 5.0, 1.0])
    nbytes = np.array([60 * GRAN, 60 * GRAN, 10 * GRAN], dtype=np.uint64)
    ta, td, _ = meb.sched_simulate(arrival, service, nbytes, pool, 8)
    assert ta[0] == 0.0
    assert ta[1] == 10.0  # waits for the first to leave
    assert ta[2] == 10.0  # FIFO behind the second, admitted right after it


def test_pool_reuse_after_release():
    # two requests of exactly the pool size run back to back at offset 0
    pool = 64 * GRAN
    ta, td, off = meb.sched_simulate([0.0, 0.0], [3.0, 3.0], np.array([pool, pool], dtype=np.uint64), pool, 4)
    assert list(ta) == [0.0, 3.0]
    assert list(off) == [0, 0]


def test_first_fit_reuses_freed_hole():
    # A (40) B (40) C (20) fill the pool; A leaves; D (30) takes A's hole at 0
    g = GRAN
    pool = 100 * g
    arrival = [0.0, 0.0, 0.0, 1.0]
    service = [2.0, 10.0, 10.0, 1.0]
    nbytes = np.array([40 * g, 40 * g, 20 * g, 30 * g], dtype=np.uint64)
    ta, td, off = meb.sched_simulate(arrival, service, nbytes, pool, 8)
    assert list(off[:3]) == [0, 40 * g, 80 * g]
    assert ta[3] == 2.0 and off[3] == 0


def test_oversized_request_rejected():
    with pytest.raises(meb.MebError):
        meb.sched_simulate([0.0], [1.0], np.array([1 << 21], dtype=np.uint64), 1 << 20, 4)


def test_unsorted_arrivals_rejected():
    with pytest.raises(meb.MebError):
        meb.sched_simulate([1.0, 0.0], [1.0, 1.0], np.array([1, 1], dtype=np.uint64), 1 << 20, 4)
