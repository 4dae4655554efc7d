"""Admission of the serving loop (host logic, no GPU): requests enter by
footprint within the budget; a later request that fits may pass an older one
that does not, at most `max_bypass` times per older request, after which the
line holds until the older one fits; an oversized request fails at once."""
import threading
import time

import pytest

from paper_2206_00708_amd import serve


def _run(adm, needs, releases):
    """Requests 0..n-1 arrive in order; request 0 is admitted first; then each
    request asks in order (thread per request, 30 ms apart); `releases` lists
    (time, request) at which an admitted request finishes."""
    for rid in range(len(needs)):
        adm.arrive(rid)
    threads = []
    for rid, nb in enumerate(needs):
        t = threading.Thread(target=adm.admit, args=(rid, nb))
        t.start()
        threads.append(t)
        time.sleep(0.03)
    t0 = time.perf_counter()
    for at, rid in releases:
        time.sleep(max(0.0, t0 + at - time.perf_counter()))
        adm.release(needs[rid])
    for t in threads:
        t.join(timeout=5)
        assert not t.is_alive(), "a request never got in"
    return adm.order


def test_bounded_out_of_order_admission():
    # budget 10: request 0 (4) runs; request 1 (8) does not fit beside it;
    # requests 2 and 3 (2 each) pass it; request 4 (2) would fit too but
    # request 1 has been passed twice (the bound), so the line holds until
    # requests 0 and 2 finish and request 1 fits
    adm = serve.Admission(10, max_bypass=2)
    order = _run(adm, [4, 8, 2, 2, 2, 2], [(0.05, 0), (0.10, 2), (0.15, 3), (0.20, 1)])
    assert order[:4] == [0, 2, 3, 1], order
    assert sorted(order) == list(range(6))


def test_arrival_order_when_everything_fits():
    adm = serve.Admission(100, max_bypass=2)
    order = _run(adm, [10, 10, 10, 10], [])
    assert order == [0, 1, 2, 3]


def test_no_bypass_with_zero_bound():
    adm = serve.Admission(10, max_bypass=0)
    order = _run(adm, [4, 8, 2, 2], [(0.05, 0), (0.10, 1), (0.15, 2)])
    assert order == [0, 1, 2, 3], order


def test_oversized_request_fails():
    adm = serve.Admission(10)
    adm.arrive(0)
    with pytest.raises(Exception) as e:
        adm.admit(0, 11)
    assert "budget" in str(e.value)
    adm.arrive(1)
    adm.admit(1, 10)   # the failed request left the line
    assert adm.order == [1]
