"""Serving form: continuous batching of sequences of related systems on one GPU.

A request is a sequence of related sparse systems A^[i] X = B^[i] that share
one recycle space (U_k, C_k); the sequence's workspaces and recycle pair stay on
the device from its first system to its last (the stored U of Algorithm 1 is
reused by the next solve).  The server

* admits requests in arrival order (FIFO: a request never overtakes an earlier
  one) as soon as a slot is free and its device footprint fits in the HBM
  budget next to the requests already running;
* runs every admitted request in a worker thread of its own with its own HIP
  stream and sequence handle, so that the solves of different requests overlap
  on the device (the library call releases the interpreter lock); each
  request's host-side dense work runs in its worker thread;
* reports per-request latency (completion minus arrival, including the upload
  of the request's matrices and right-hand sides) and systems per second.

Results do not depend on what else runs: every kernel's reduction order is
fixed by its launch shape, which depends only on the request's own sizes.

The admission and scheduling logic (`serve`) takes the work as a callable, so
it is exercised without a GPU by the tests; `gpu_runner` supplies the real work
through the C ABI.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence as Seq

import numpy as np


@dataclass
class Request:
    """One sequence of related systems; `system(i)` returns (A scipy CSR, B ndarray n x p)."""
    rid: int
    arrival: float              # seconds after the start of the stream
    n: int
    p: int
    nnz: int
    nsys: int
    system: Callable[[int], tuple]
    m: int = 10
    k: int = 20
    tol: float = 1e-8
    precision: int = 0          # BGCR_PLAIN_FP64 or BGCR_MIXED_FP32
    dtype: int = 0              # BGCR_F64


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    stats: list = field(default_factory=list)
    solutions: list = field(default_factory=list)
    error: Optional[str] = None

    @property
    def latency(self):
        return self.finished - self.arrival


def device_bytes(req: Request, footprint: Callable[[Request], int]) -> int:
    """Bytes a request holds on the device while it runs: the library's
    workspaces and recycle pair (bgcr_footprint_bytes) plus one system's CSR
    matrix (int32 indices), right-hand side and solution."""
    sv = 16 if req.dtype == 1 else 8
    return int(footprint(req)) + 4 * (req.n + 1) + (4 + sv) * req.nnz + 2 * sv * req.n * req.p


def serve(requests: Seq[Request], run: Callable[[Request, Result], None], budget_bytes: int, slots: int,
          bytes_of: Callable[[Request], int], realtime: bool = True, clock=time.perf_counter,
          on_event: Optional[Callable[[str, int, float, int, int], None]] = None) -> List[Result]:
    """Continuous batching: admit each request (in arrival order) as soon as it
    has arrived, a slot is free and its bytes fit next to the running ones.
    `run(req, result)` does the work in a worker thread.  With `realtime`
    False every request counts as arrived at time 0.  A request larger than
    the whole budget is rejected (result.error set) without running.
    `on_event(kind, rid, t, running, used_bytes)` observes admissions and
    completions."""
    order = sorted(requests, key=lambda r: (r.arrival if realtime else 0.0, r.rid))
    results = {r.rid: Result(r.rid, r.arrival if realtime else 0.0) for r in order}
    cv = threading.Condition()
    state = {"running": 0, "used": 0}
    pending = list(order)
    threads = []
    t0 = clock()

    def worker(req, res, nbytes):
        try:
            run(req, res)
        except Exception as e:  # reported per request; the server keeps going
            res.error = f"{type(e).__name__}: {e}"
        with cv:
            res.finished = clock() - t0
            state["running"] -= 1
            state["used"] -= nbytes
            if on_event:
                on_event("done", req.rid, res.finished, state["running"], state["used"])
            cv.notify_all()

    with cv:
        while pending or state["running"] > 0:
            now = clock() - t0
            while pending:
                req = pending[0]
                arr = req.arrival if realtime else 0.0
                if arr > now:
                    break
                nb = bytes_of(req)
                if nb > budget_bytes:
                    pending.pop(0)
                    res = results[req.rid]
                    res.error = f"needs {nb} device bytes, over the budget of {budget_bytes}"
                    res.admitted = res.finished = now
                    continue
                if state["running"] >= slots or state["used"] + nb > budget_bytes:
                    break
                pending.pop(0)
                res = results[req.rid]
                res.admitted = now
                state["running"] += 1
                state["used"] += nb
                if on_event:
                    on_event("admit", req.rid, now, state["running"], state["used"])
                th = threading.Thread(target=worker, args=(req, res, nb), daemon=True)
                threads.append(th)
                th.start()
            if not pending and state["running"] == 0:
                break
            timeout = None
            if pending:
                arr = pending[0].arrival if realtime else 0.0
                if arr > now:
                    timeout = arr - now
            cv.wait(timeout)
    for th in threads:
        th.join()
    return [results[r.rid] for r in order]


def gpu_runner(device="cuda:0", keep_solutions=False, precision: Optional[int] = None):
    """Work of one request on the GPU: its own stream and sequence, systems
    solved in order with the recycle space kept on the device in between."""
    import torch

    from . import BGCR_BREAKDOWN_DEFLATED, BGCR_OK, DeviceCSR, Sequence, bgcr_strerror

    def run(req: Request, res: Result):
        stream = torch.cuda.Stream(device=device)
        prec = req.precision if precision is None else precision
        with torch.cuda.stream(stream):
            seq = Sequence(req.n, req.p, req.m, req.k, dtype=req.dtype, precision=prec, stream=stream)
            try:
                for i in range(req.nsys):
                    A, B = req.system(i)
                    dA = DeviceCSR.from_scipy(A, device)
                    dB = torch.from_numpy(np.ascontiguousarray(B)).to(device)
                    dX = torch.zeros_like(dB)
                    st = seq.solve(dA, dB, dX, req.tol)
                    res.stats.append(st.as_dict())
                    if keep_solutions:
                        res.solutions.append(dX.cpu().numpy())
                    # only a converged system counts (OK, or converged after
                    # handling a rank-deficient block)
                    if st.status not in (BGCR_OK, BGCR_BREAKDOWN_DEFLATED):
                        res.error = f"system {i}: status {st.status} ({bgcr_strerror(st.status)})"
                        break
                stream.synchronize()
            finally:
                seq.release()

    return run


def summarize(results: Seq[Result], wall: float) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    # systems of requests that finished without error; every one converged
    nsys = sum(len(r.stats) for r in ok)
    return {"requests": len(results), "failed": len(results) - len(ok), "systems": nsys,
            "wall_s": round(wall, 3), "systems_per_s": round(nsys / wall, 4) if wall > 0 else 0.0,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4)}


def library_footprint(req: Request) -> int:
    """bgcr_footprint_bytes for the request's sequence parameters."""
    from . import bgcr_footprint_bytes, bgcr_params

    prm = bgcr_params(req.p, req.m, req.k, req.dtype, req.precision, 1000, 0, 0)
    return bgcr_footprint_bytes(prm, req.n, req.nnz)
