"""Autotuner of the batched eigensolver's tile table.

For every order bucket of the one-workgroup LDS solver (orders 1-8, 9-16, ...,
57-64) it times a batch of random Hermitian matrices of the bucket's largest
order with each candidate -- the LDS solver at 64, 128, 256 and 512 threads
per workgroup, and the grouped Householder / divide-and-conquer path (0) --
and keeps the fastest (median of repeated runs after a warm-up).  The table
(mmf_batch_opts.small_threads) is written as JSON next to this module and
read by load_table(); the measured times are kept with it.

    python -m paper_2005_03426_amd.autotune [--count 256] [--reps 5] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")
CANDIDATES = (0, 64, 128, 256, 512)


def load_table(path: str = TABLE_PATH, prec: str = "c128"):
    """The tuned 8-entry table, or None when no table has been written."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    ent = t.get(prec)
    return None if ent is None else [int(x) for x in ent["small_threads"]]


def _time_bucket(mmf, torch, n: int, count: int, reps: int, seed: int):
    rng = np.random.default_rng(seed)
    mats = []
    for _ in range(count):
        A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        H = (A + A.conj().T) / 2
        mats.append(torch.from_numpy(np.ascontiguousarray(H.T)).to("cuda"))
    work = torch.empty(mmf.eigh_batched_workspace_bytes([n] * count), dtype=torch.uint8, device="cuda")
    info = torch.zeros(count, dtype=torch.int32, device="cuda")
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(count)]
    scratch = [torch.empty_like(m) for m in mats]
    out = {}
    for cand in CANDIDATES:
        tiles = [cand] * 8
        times = []
        for r in range(reps + 1):
            for s, m in zip(scratch, mats):
                s.copy_(m)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mmf.eigh_batched(scratch, mmf.MMF_C128, ws=ws, work=work, info=info, tiles=tiles)
            torch.cuda.synchronize()
            if r:                                        # the first run is a warm-up
                times.append(time.perf_counter() - t0)
        if int(info.ne(0).sum().item()):
            continue                                     # a candidate that reports failure is not taken
        out[cand] = float(np.median(times)) * 1e3
    return out


def tune(count: int = 256, reps: int = 5, out_path: str = TABLE_PATH, seed: int = 0) -> dict:
    import torch
    import paper_2005_03426_amd as mmf
    assert torch.cuda.is_available(), "the autotuner measures on the GPU"
    table, timings = [], {}
    for b in range(8):
        n = 8 * (b + 1)
        t = _time_bucket(mmf, torch, n, count, reps, seed + b)
        best = min(t, key=t.get)
        table.append(int(best))
        timings[str(n)] = {str(k): v for k, v in t.items()}
        print(f"[autotune] order {n}: " + ", ".join(f"{k}: {v:.3f} ms" for k, v in t.items()) + f" -> {best}",
              flush=True)
    rec = {"device": torch.cuda.get_device_name(0), "count_per_bucket": count, "reps": reps,
           "c128": {"small_threads": table, "ms_per_batch": timings}}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=TABLE_PATH)
    a = ap.parse_args()
    tune(a.count, a.reps, a.out)
