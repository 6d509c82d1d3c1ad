"""Continuous-batching executor for independent Floquet solves.

Requests (a problem, its times, t0) arrive over time.  The executor keeps a
fixed number of slots; each slot owns a HIP stream (default priority) and a
worker thread.  A request is admitted when it has arrived, a slot is free
and its HBM footprint (Floquet matrix, eigensolver and evolution
workspaces) fits in the budget next to the requests already on the device;
its whole solve (assemble -> eigh -> U(t) -> P) is then enqueued on the
slot's stream, so solves of different slots overlap on the GPU.  Results
(eigenvalues, P, U) stay on the device until the caller reads them.
Latency is measured from a request's arrival to the moment its stream has
finished.  Every step runs in the library's kernels (libmmf.so); this
module only schedules.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import (DeviceProblem, build_floquet, eigh, evolve, avg_prob, eigh_workspace_bytes, call,
               MMF_C128)


def footprint_bytes(M: int, D: int, T: int, prec: int = MMF_C128) -> int:
    """HBM bytes a solve holds while in flight (matrix + workspaces + outputs)."""
    S = M // D
    ev = T * S * 16 + T * D * M * 16 + ((M + 2047) // 2048) * T * D * D * 16
    return 16 * M * M + eigh_workspace_bytes(M, prec) + ev + 8 * M + 16 * T * D * D + 4096


@dataclass
class Request:
    rid: int
    arrival: float
    problem: object
    times: np.ndarray
    t0: float = 0.0
    prec: int = MMF_C128
    # filled by the executor
    admitted: float = -1.0
    done: float = -1.0
    result: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Executor:
    def __init__(self, slots: int = 4, hbm_budget: int | None = None, device: str = "cuda",
                 keep_eigenvectors: bool = False):
        import torch
        self.torch = torch
        self.device = device
        self.slots = slots
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
        self.keep_vectors = keep_eigenvectors
        self._lock = threading.Condition()
        self._in_use = 0
        self._pending: list[Request] = []
        self._finished: list[Request] = []
        self._closed = False
        self._t0 = None
        dev = torch.device(device)
        self._dev_index = dev.index if dev.index is not None else torch.cuda.current_device()
        self._errors: list[BaseException] = []
        self._streams = [torch.cuda.Stream(device=self._dev_index) for _ in range(slots)]
        self._threads = [threading.Thread(target=self._worker, args=(k,), daemon=True) for k in range(slots)]
        self.rejected: list[Request] = []

    # ------------------------------------------------------------------ worker
    def _solve(self, req: Request, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            dp = DeviceProblem(req.problem, self.device)
            tt = torch.as_tensor(np.asarray(req.times, dtype=np.float64), device=self.device)
            HF = build_floquet(dp, stream=stream)
            w, Pt, info = eigh(HF, prec=req.prec, stream=stream)
            U = evolve(dp, Pt, w, req.t0, tt, stream=stream)
            P = avg_prob(dp, Pt, stream=stream)
        stream.synchronize()
        res = {"w": w, "U": U, "P": P, "info": info, "M": dp.M}
        if self.keep_vectors:
            res["Pt"] = Pt
        return res

    def _worker(self, k: int):
        torch = self.torch
        stream = self._streams[k]
        torch.cuda.set_device(self._dev_index)
        while True:
            with self._lock:
                req = None
                while req is None:
                    if self._closed and not self._pending:
                        return
                    now = self._now()
                    for idx, r in enumerate(self._pending):
                        if r.arrival > now:
                            break                       # pending is sorted by arrival
                        need = r._fp
                        if self._in_use + need <= self.budget:
                            req = self._pending.pop(idx)
                            self._in_use += need
                            break
                    if req is None:
                        self._lock.wait(timeout=0.0005)
                req.admitted = self._now()
            try:
                req.result = self._solve(req, stream)
            except BaseException as exc:          # surfaced by run()
                with self._lock:
                    self._errors.append(exc)
                    self._closed = True
                    self._pending.clear()
            finally:
                with self._lock:
                    req.done = self._now()
                    self._in_use -= req._fp
                    self._finished.append(req)
                    self._lock.notify_all()

    def _now(self) -> float:
        return time.perf_counter() - self._t0

    # ------------------------------------------------------------------ API
    def run(self, requests: list[Request]) -> list[Request]:
        """Serve the requests (arrival times in seconds from start); returns
        them with latencies filled in, in completion order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            D = int(np.asarray(r.problem.E).shape[0])
            M = D
            for n in r.problem.N:
                M *= 2 * int(n) + 1
            r._fp = footprint_bytes(M, D, len(r.times), r.prec)
            if r._fp > self.budget:
                self.rejected.append(r)
        reqs = [r for r in reqs if r._fp <= self.budget]
        self._pending = reqs
        self._finished = []
        self._closed = True
        self._t0 = time.perf_counter()
        for t in self._threads:
            t.start()
        for t in self._threads:
            t.join()
        if self._errors:
            raise self._errors[0]
        return self._finished


def latency_stats(done: list[Request]) -> dict:
    lat = np.array([r.latency for r in done])
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"count": len(done), "solves_per_s": len(done) / span, "makespan_s": span,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}
