"""Continuous-batching executor for independent Floquet solves.

Requests (a problem, its times, t0) arrive over time.  The executor keeps a
fixed number of slots; each slot owns a HIP stream (default priority) and a
worker thread.  A free slot takes the oldest arrived request and, with it,
every other arrived request of the same size class and precision (classes
are octaves of the Floquet dimension M, so a batch's largest solve costs at
most eight times its smallest), up to `max_batch` requests and as long as
their HBM footprints (Floquet matrix, eigensolver and evolution workspaces)
fit in the budget next to the work already on the device.  The batch is
solved with one grouped eigensolve (each kernel launch advances every matrix
of the batch), then U(t) and the averaged P per request, all on the slot's
stream; batches of different slots overlap on the GPU.  A request's result
does not depend on the batch it joined (the grouped kernels do the same
arithmetic per matrix as a single solve).  A request whose mixed-precision
eigensolve reports non-convergence is solved again in complex128 on the
same stream (its result then says `retried_c128`), unless the executor was
made with retry_c128=False.  With `band_min` set, a complex128 request whose
Floquet matrix is banded within its 64th subdiagonal (one drive with
D h + D - 1 <= 64) and of order at least band_min is solved alone through the
band-aware eigensolver (mmf_eigh_band: no dense -> band stage).  That routing
is off by default: the 2000-request serving benchmark with it ended in a GPU
memory fault whose cause has not been found.  A batch whose workspace the caching allocator
cannot place (fragmented free blocks) is solved one request at a time.
Results stay on the device until
the caller reads them.  Latency runs from a request's arrival to the moment
its batch's stream has finished.  Every step runs in the library's kernels
(libmmf.so); this module only schedules.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import (DeviceProblem, build_floquet, eigh, eigh_band, eigh_batched, evolve, avg_prob, eigh_workspace_bytes,
               eigh_band_workspace_bytes, floquet_half_bandwidth, call, MMF_C128)

BAND_MAX = 64          # widest native half-bandwidth the band-aware eigensolver takes


def footprint_bytes(M: int, D: int, T: int, prec: int = MMF_C128, band: int | None = None) -> int:
    """HBM bytes a solve holds while in flight (matrix + workspaces + outputs;
    for a mixed-precision request also what its complex128 retry needs; with
    `band`, the band-aware eigensolver's workspace)."""
    S = M // D
    ev = T * S * 16 + T * D * M * 16 + ((M + 2047) // 2048) * T * D * D * 16
    ws = eigh_band_workspace_bytes(M, band) if band is not None else eigh_workspace_bytes(M, prec)
    if prec != MMF_C128:
        ws = max(ws, eigh_workspace_bytes(M, MMF_C128))
    return 16 * M * M + ws + ev + 8 * M + 16 * T * D * D + 4096


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
                 max_batch: int = 64, progress=None, retry_c128: bool = True, limits: dict | None = None,
                 band_min: int | None = None):
        """slots: streams (and worker threads); hbm_budget: bytes of admitted
        footprints at once (default 0.8 of the free HBM); max_batch: requests
        per grouped eigensolve; progress: callable(done_count) called as
        batches finish; retry_c128: solve a mixed-precision request again in
        complex128 when its eigensolve reports non-convergence; limits:
        iteration limits of mmf_eigh_ex (e.g. {"refine_max_iters": 1}) to
        force the failure handling from the host; with limits every request
        is solved alone (the grouped eigensolver takes none); band_min: order
        from which narrow-band complex128 requests take the band-aware
        eigensolver (None, the default: never; the serving benchmark with
        band_min = 1024 ended in a GPU fault whose cause is not known)."""
        import torch
        self.torch = torch
        self.retry_c128 = retry_c128
        self.limits = limits
        self.band_min = band_min if limits is None else None
        if limits is not None:
            max_batch = 1
        self.device = device
        self.slots = slots
        self.max_batch = max(1, int(max_batch))
        self.progress = progress          # optional callable(done_count), called as batches finish
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
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
        self.batches: list[int] = []

    # ------------------------------------------------------------------ worker
    def _solve(self, reqs: list[Request], stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            dps = [DeviceProblem(r.problem, self.device) for r in reqs]
            HFs = [build_floquet(dp, stream=stream) for dp in dps]
            if len(reqs) == 1 and reqs[0]._band is not None:
                w, Pt, info = eigh_band(HFs[0], reqs[0]._band, stream=stream)
                ws, Pts, infos = [w], [Pt], [info]
            elif len(reqs) == 1:
                w, Pt, info = eigh(HFs[0], prec=reqs[0].prec, stream=stream, limits=self.limits)
                ws, Pts, infos = [w], [Pt], [info]
            else:
                ws, Pts, info = eigh_batched(HFs, prec=reqs[0].prec, stream=stream)
                infos = [info[k:k + 1] for k in range(len(reqs))]
            out = []
            for r, dp, w, Pt, inf in zip(reqs, dps, ws, Pts, infos):
                tt = torch.as_tensor(np.asarray(r.times, dtype=np.float64), device=self.device)
                U = evolve(dp, Pt, w, r.t0, tt, stream=stream)
                P, pstat = avg_prob(dp, Pt, w, stream=stream)
                # results keep no M x M buffer, so a finished request frees its whole footprint
                out.append({"w": w, "U": U, "P": P, "P_status": pstat, "info": inf, "M": dp.M})
        stream.synchronize()
        HFs = Pts = Pt = None             # the M x M buffers go before any retry allocates its own
        if self.retry_c128 and reqs[0].prec != MMF_C128:
            for k, (r, dp) in enumerate(zip(reqs, dps)):
                if int(out[k]["info"].item()) == 0:
                    continue
                with torch.cuda.stream(stream):
                    HF = build_floquet(dp, stream=stream)
                    w, Pt, inf = eigh(HF, prec=MMF_C128, stream=stream)
                    tt = torch.as_tensor(np.asarray(r.times, dtype=np.float64), device=self.device)
                    U = evolve(dp, Pt, w, r.t0, tt, stream=stream)
                    P, pstat = avg_prob(dp, Pt, w, stream=stream)
                    out[k] = {"w": w, "U": U, "P": P, "P_status": pstat, "info": inf, "M": dp.M,
                              "retried_c128": True}
                    del HF, Pt
                stream.synchronize()
        return out

    def _take(self, now: float) -> list[Request]:
        """Oldest arrived request plus arrived requests of its class (lock held)."""
        if not self._pending or self._pending[0].arrival > now:
            return []
        head = None
        for idx, r in enumerate(self._pending):
            if r.arrival > now:
                break                                  # pending is sorted by arrival
            if self._in_use + r._fp <= self.budget:
                head = idx
                break
        if head is None:
            return []
        first = self._pending[head]
        batch, room = [head], self.budget - self._in_use - first._fp
        for idx in range(head + 1, len(self._pending)):
            if len(batch) >= self.max_batch:
                break
            r = self._pending[idx]
            if r.arrival > now:
                break
            if r._cls == first._cls and r.prec == first.prec and r._fp <= room:
                batch.append(idx)
                room -= r._fp
        taken = [self._pending[i] for i in batch]
        for i in reversed(batch):
            self._pending.pop(i)
        self._in_use += sum(r._fp for r in taken)
        return taken

    def _worker(self, k: int):
        torch = self.torch
        stream = self._streams[k]
        torch.cuda.set_device(self._dev_index)
        while True:
            with self._lock:
                reqs = []
                while not reqs:
                    if self._closed and not self._pending:
                        return
                    reqs = self._take(self._now())
                    if not reqs:
                        self._lock.wait(timeout=0.0005)
                t_adm = self._now()
                for r in reqs:
                    r.admitted = t_adm
                self.batches.append(len(reqs))
            try:
                results = None
                try:
                    results = self._solve(reqs, stream)
                except torch.OutOfMemoryError:
                    pass                          # (leaves the handler, so the failed frame's buffers go)
                if results is None:
                    # the admitted footprints fit the budget, but the caching
                    # allocator's free blocks may be too fragmented for one
                    # batch workspace: solve one at a time (smaller pieces).
                    # The cache is not returned to the driver here: other
                    # slots' streams may still be using blocks that their
                    # threads have already released to it.
                    stream.synchronize()
                    results = [self._solve([r], stream)[0] for r in reqs]
                for r, res in zip(reqs, results):
                    r.result = res
            except BaseException as exc:          # surfaced by run()
                with self._lock:
                    self._errors.append(exc)
                    self._closed = True
                    self._pending.clear()
            finally:
                with self._lock:
                    t_done = self._now()
                    for r in reqs:
                        r.done = t_done
                        self._in_use -= r._fp
                        self._finished.append(r)
                    done = len(self._finished)
                    self._lock.notify_all()
                if self.progress is not None:
                    self.progress(done)

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
            b = floquet_half_bandwidth(r.problem)
            r._band = (b if self.band_min is not None and r.prec == MMF_C128 and b <= BAND_MAX
                       and M >= self.band_min else None)
            r._fp = footprint_bytes(M, D, len(r.times), r.prec, r._band)
            # octave of M; a band-aware request is a class of its own (solved alone)
            r._cls = int(M).bit_length() if r._band is None else ("band", id(r))
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
