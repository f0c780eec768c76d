"""Admission and scheduling of the serving form, without a GPU (fake work)."""
import threading
import time

import pytest

from paper_1604_01713_amd import serving as sv


def _req(rid, arrival=0.0, nbytes=1, nsys=1):
    r = sv.Request(rid=rid, arrival=arrival, n=10, p=1, nnz=10, nsys=nsys, system=lambda i: None)
    r._bytes = nbytes
    return r


def _run_fake(durations):
    def run(req, res):
        time.sleep(durations[req.rid])
        res.stats = [{} for _ in range(req.nsys)]
    return run


def test_slots_budget_and_fifo_are_respected():
    reqs = [_req(i, nbytes=b) for i, b in enumerate([4, 3, 3, 2, 5, 1, 2])]
    events = []
    lock = threading.Lock()

    def on_event(kind, rid, t, running, used):
        with lock:
            events.append((kind, rid, running, used))

    res = sv.serve(reqs, _run_fake({i: 0.02 * (1 + i % 3) for i in range(7)}), budget_bytes=8, slots=3,
                   bytes_of=lambda r: r._bytes, realtime=False, on_event=on_event)
    assert all(r.error is None for r in res)
    admits = [e[1] for e in events if e[0] == "admit"]
    assert admits == sorted(admits), "admission must follow arrival order"
    assert max(e[2] for e in events) <= 3
    assert max(e[3] for e in events) <= 8


def test_admission_is_continuous_not_batched():
    # slots = 2: request 0 is long, 1 is short; 2 must start when 1 ends, long before 0 ends
    reqs = [_req(0), _req(1), _req(2)]
    res = sv.serve(reqs, _run_fake({0: 0.5, 1: 0.05, 2: 0.05}), budget_bytes=10, slots=2,
                   bytes_of=lambda r: 1, realtime=False)
    by = {r.rid: r for r in res}
    assert by[2].admitted >= by[1].finished - 1e-3
    assert by[2].finished < by[0].finished


def test_requests_wait_for_their_arrival_and_oversized_are_rejected():
    reqs = [_req(0, arrival=0.0), _req(1, arrival=0.15), _req(2, arrival=0.0, nbytes=100)]
    res = sv.serve(reqs, _run_fake({0: 0.01, 1: 0.01, 2: 0.01}), budget_bytes=10, slots=4,
                   bytes_of=lambda r: r._bytes, realtime=True)
    by = {r.rid: r for r in res}
    assert by[1].admitted >= 0.15 - 1e-3
    assert by[2].error is not None and "budget" in by[2].error
    assert by[0].error is None and by[1].error is None


def test_worker_failure_is_reported_per_request():
    reqs = [_req(0), _req(1)]

    def run(req, res):
        if req.rid == 0:
            raise RuntimeError("boom")
        res.stats = [{}]

    res = sv.serve(reqs, run, budget_bytes=10, slots=2, bytes_of=lambda r: 1, realtime=False)
    by = {r.rid: r for r in res}
    assert "boom" in by[0].error and by[1].error is None


def test_device_bytes_follow_the_library_footprint():
    pytest.importorskip("ctypes")
    r64 = sv.Request(rid=0, arrival=0, n=100000, p=8, nnz=700000, nsys=1, system=None, precision=0)
    r32 = sv.Request(rid=1, arrival=0, n=100000, p=8, nnz=700000, nsys=1, system=None, precision=1)
    b64 = sv.device_bytes(r64, sv.library_footprint)
    b32 = sv.device_bytes(r32, sv.library_footprint)
    # basis, W, recycle pair in FP32 for the precision form: clearly smaller
    assert 0 < b32 < b64
    # at least the basis (m blocks) and the CSR
    assert b64 > 10 * 100000 * 8 * 8 + 12 * 700000
