"""Batched Floquet solves replayed as one recorded HIP graph.

A parameter sweep solves many small, unevenly sized Floquet problems again
and again (the frequency scans of the paper's examples).  `BatchPlan` holds
every buffer of such a batch on the device (Floquet matrices, eigenpairs,
workspaces, U(t), averaged probabilities) and enqueues one pass as

  1. one batched assembly launch for every H_F (from device copies of E, V);
  2. the eigensolves in groups, each group one batched call, the groups
     dealt to four streams (forked from the plan's stream and joined back)
     by load, so that they run side by side: orders <= 64 in one group on the
     one-workgroup LDS solver (a persistent launch over a work queue), larger
     orders in groups of one octave of the order (at most 64 problems) on
     the grouped Householder / divide-and-conquer path;
  3. one batched pass for U(t, t0) and the averaged probabilities of every
     problem (five launches whatever the batch size).

The pass is recorded once as a graph (with its stream fork and join) and
replayed.  Every step runs in the library's kernels; the graph only removes
the host's per-launch cost, and the recording holds no memset (the library
clears its flags and counters with its own kernels).
"""
from __future__ import annotations

import ctypes as C
import numpy as np

from . import (DeviceProblem, eigh_batched, eigh_batched_workspace_bytes, call, MMF_C128, _workspace, _stream,
               _ptr)
from ._lib import MMFProblem


def size_classes(sizes, small_max: int = 64, group_max: int = 64, lanes: int = 4):
    """The eigensolve's schedule: a list of lanes (one stream each), each an
    ordered list of groups of problem indices, every group one batched call.
    Orders <= small_max form one group (the LDS solver, one launch).  Larger
    orders are grouped by octave of the order (a grouped call advances all its
    problems step by step, so similar orders waste little), an octave cut into
    groups of at most group_max problems; the groups, largest first, go to
    the lane with the least estimated time so far (sequential steps plus
    work), so that the largest octave's groups run side by side."""
    octaves = {}
    for k, m in enumerate(sizes):
        if m > small_max:
            octaves.setdefault(int(m - 1).bit_length(), []).append(k)
    groups = []
    for key in sorted(octaves, reverse=True):
        ks = sorted(octaves[key], key=lambda k: -sizes[k])
        groups += [ks[i:i + group_max] for i in range(0, len(ks), group_max)]
    # time of a grouped call: its sequential steps (about 40 us per column of
    # its largest order) plus its work at about 10 TFLOP/s of the nominal
    # (40/3) M^3 flops per problem
    def cost(g):
        return 4e-5 * max(float(sizes[k]) for k in g) + 1.33e-12 * sum(float(sizes[k]) ** 3 for k in g)
    groups.sort(key=lambda g: -cost(g))
    plan = [[] for _ in range(lanes)]
    load = [0.0] * lanes
    small = [k for k, m in enumerate(sizes) if m <= small_max]
    for g in groups + ([small] if small else []):
        j = min(range(lanes), key=lambda i: load[i])
        plan[j].append(g)
        load[j] += cost(g)
    return [lane for lane in plan if lane]


class BatchPlan:
    """All device state of one batch of Floquet solves, and its recorded graph.

    problems: list of host problem statements (D <= 64, at most 4 fundamentals
    and 8 couplings); times: the evaluation times of U(t, t0), one array for
    the whole batch or one per problem (equal lengths); tiles: the batched
    eigensolver's tile table (None: the library's rule); graph: record and
    replay a graph (else each run() launches eagerly); group_max: largest
    number of problems per grouped eigensolver call."""

    def __init__(self, problems, times, t0: float = 0.0, prec: int = MMF_C128, tiles=None, graph: bool = True,
                 device: str = "cuda", group_max: int = 64):
        import torch
        self.torch = torch
        self.prec, self.tiles, self.t0 = prec, tiles, float(t0)
        self.dps = [p if isinstance(p, DeviceProblem) else DeviceProblem(p, device) for p in problems]
        count = len(self.dps)
        self.sizes = [dp.M for dp in self.dps]
        if len(times) == count and np.ndim(times[0]) == 1:
            self.tt = [torch.as_tensor(np.asarray(t, dtype=np.float64), device=device) for t in times]
        else:
            one = torch.as_tensor(np.asarray(times, dtype=np.float64), device=device)
            self.tt = [one] * count
        T = int(self.tt[0].shape[0])
        assert all(int(t.shape[0]) == T for t in self.tt), "every problem needs the same number of times"
        self.T = T
        self.HF = [torch.empty((m, m), dtype=torch.complex128, device=device) for m in self.sizes]
        self.w = [torch.empty(m, dtype=torch.float64, device=device) for m in self.sizes]
        self.U = [torch.empty((T, dp.D, dp.D), dtype=torch.complex128, device=device) for dp in self.dps]
        self.P = [torch.empty((dp.D, dp.D), dtype=torch.float64, device=device) for dp in self.dps]
        self.pstat = torch.zeros(count, dtype=torch.int32, device=device)
        # host-side argument arrays of the batched calls, built once
        self.probs = (MMFProblem * count)(*[dp.struct for dp in self.dps])

        def ptrs(ts):
            return (C.c_void_p * count)(*[t.data_ptr() for t in ts])
        self.a_EV, self.a_HF, self.a_w = ptrs([dp.ev_work for dp in self.dps]), ptrs(self.HF), ptrs(self.w)
        self.a_t, self.a_U, self.a_P = ptrs(self.tt), ptrs(self.U), ptrs(self.P)
        self.a_ld = (C.c_int64 * count)(*[max(m, 1) for m in self.sizes])
        b = C.c_size_t(0)
        call("mmf_batched_workspace", C.c_int64(count), self.probs, C.c_int32(T), C.byref(b))
        self.bwork = _workspace(b.value, device)
        # eigensolve lanes (one stream each) of groups, each group with its
        # workspace and status words
        self.lanes = size_classes(self.sizes, group_max=group_max)
        self.classes = [g for lane in self.lanes for g in lane]
        self.cls_work = [_workspace(eigh_batched_workspace_bytes([self.sizes[k] for k in cl], prec), device)
                         for cl in self.classes]
        self.cls_info = [torch.zeros(len(cl), dtype=torch.int32, device=device) for cl in self.classes]
        self.stream = torch.cuda.Stream(device=device)
        self.lane_streams = [torch.cuda.Stream(device=device) for _ in self.lanes]
        self.graph = None
        # one eager pass first: it also performs the library's one-time set-up
        # (code loading, kernel attributes), which a recording must not contain
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            self._enqueue()
        self.stream.synchronize()
        if graph:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=self.stream):
                self._enqueue()
            self.stream.synchronize()

    def _enqueue(self):
        torch = self.torch
        count = len(self.dps)
        main = torch.cuda.current_stream()
        call("mmf_build_floquet_batched", C.c_int64(count), self.probs, self.a_EV, self.a_HF, self.a_ld,
             _ptr(self.bwork), C.c_size_t(self.bwork.numel()), _stream(main))
        g = 0
        for lane, s in zip(self.lanes, self.lane_streams):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                for cl in lane:
                    eigh_batched([self.HF[k] for k in cl], self.prec, ws=[self.w[k] for k in cl],
                                 work=self.cls_work[g], info=self.cls_info[g], tiles=self.tiles, stream=s)
                    g += 1
        for s in self.lane_streams:
            main.wait_stream(s)
        call("mmf_observables_batched", C.c_int64(count), self.probs, self.a_HF, self.a_ld, self.a_w,
             C.c_double(self.t0), C.c_int32(self.T), self.a_t, self.a_U, self.a_P, _ptr(self.pstat),
             _ptr(self.bwork), C.c_size_t(self.bwork.numel()), _stream(main))

    def run(self):
        """One pass over the batch on the plan's stream (graph replay or eager
        launches); returns when it is enqueued.  Results: results()."""
        with self.torch.cuda.stream(self.stream):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._enqueue()

    def synchronize(self):
        self.stream.synchronize()

    def info(self):
        """Eigensolver status of every problem (device int32 [count])."""
        out = self.torch.zeros(len(self.dps), dtype=self.torch.int32, device=self.pstat.device)
        for cl, inf in zip(self.classes, self.cls_info):
            out[cl] = inf
        return out

    def results(self):
        """Per problem: eigenvalues w, eigenvectors Pt (row a), U[tau, i, j],
        P[i, j], eigensolver info and averaged-probability status (views of
        the plan's buffers: the next run() overwrites them)."""
        info = self.info()
        return [{"w": self.w[k], "Pt": self.HF[k], "U": self.U[k].transpose(1, 2), "P": self.P[k].T,
                 "info": info[k:k + 1], "P_status": self.pstat[k:k + 1], "dp": self.dps[k]}
                for k in range(len(self.dps))]
