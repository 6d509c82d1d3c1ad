"""Benchmark of the multimode Floquet hot path on one MI355X.

One step = one whole Floquet solve of the workload: assemble H_F -> dense
Hermitian eigensolve -> U(t, t0) at the workload's times -> averaged
transition probabilities, with every input already resident in HBM.

Default workload: 8-level ladder under two incommensurate drives
(w = 1, golden ratio), truncation +-25 on both axes, Floquet dimension
M = 20808 (complex128), U at 256 times; the default run also solves the
16-level spectrum at M = 41616 once and times the CPU oracle on a bounded
sample.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--no-large] [--no-cpu-baseline]
                  [--workload ladder20808|spec41616|tls82|ladder_N<n>|band20816|precision41616|
                              sweep512|batch512|serve|lattice_sweep|window_lattice|band_window20816]
                  [--band]   (band20816 and the other single solves: mmf_eigh_band at the
                              workload's Floquet half-bandwidth)
                  [--batch-mode executor|grouped|plan] [--prec c128|c64_refined|c64_raw]
                  [--sync-every N]   (launch throttle for rocprofv3 counter runs)
"""
from __future__ import annotations

import ctypes as C
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 counter runs
# (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0, the factors a 1 GiB device
# copy gives), with the sha256 prefixes of the sources that define the kernel
# when they were taken: a changed kernel reports null.
TRAFFIC = {
    ("bt2", "ladder20808"): {
        "bytes_per_launch": 1.9180e9 + 1.8857e9,
        "sources": {"paper_2005_03426_amd/csrc/hb2st.hip": "14affd338dc97d86",
                    "paper_2005_03426_amd/csrc/twostage.h": "a20ae151221be86a"},
        "profile": "profiles/hbm_bytes_ladder20808_counters.md",
    },
}


def counter_traffic(kernel, workload_name):
    """Counter-measured HBM bytes per launch, or None if none were taken for
    this (kernel, workload) or a defining source changed since."""
    import hashlib
    rec = TRAFFIC.get((kernel, workload_name))
    if rec is None:
        return None
    for path, h in rec["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != h:
                return None
    return rec["bytes_per_launch"]


def workload(name):
    from workloads import cfg1_tls, cfg2_large
    if name == "ladder20808":
        p, ts, t0 = cfg2_large()
    elif name == "tls82":
        p, ts, t0 = cfg1_tls()
    elif name == "spec41616":
        from workloads import cfg4_precision
        p, ts, t0 = cfg4_precision()
    elif name.startswith("ladder_N"):
        n = int(name[len("ladder_N"):])
        p, ts, t0 = cfg2_large(N=(n, n))
    elif name == "band20816":
        from workloads import one_drive_band
        p, ts, t0 = one_drive_band()
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, ts, t0


def cpu_baseline(Ns=12):
    """The FP64 oracle, as it stands, on a bounded sample of the same system
    (same ladder and drives, truncation +-Ns: M = 8 (2 Ns + 1)^2, 5000 for the
    default), timed stage by stage and extrapolated to the full dimension
    (eigh ~ M^3, the other stages ~ M^2).  The result is an extrapolation,
    labelled as such."""
    import oracle
    from workloads import cfg2_large
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    p, ts, t0 = cfg2_large(N=(Ns, Ns))
    t_a = time.perf_counter()
    H = oracle.build_floquet(p)
    t_b = time.perf_counter()
    w, Phi = oracle.eigh(H)
    t_c = time.perf_counter()
    oracle.evolve(p, Phi, w, t0, ts)
    t_d = time.perf_counter()
    oracle.avg_prob(p, Phi)
    t_e = time.perf_counter()
    Ms = H.shape[0]
    M = 8 * 51 * 51
    r = M / Ms
    full = (t_b - t_a) * r ** 2 + (t_c - t_b) * r ** 3 + (t_d - t_c) * r ** 2 + (t_e - t_d) * r ** 2
    return {
        "value": 1.0 / full, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
        "extrapolated": True,
        "sample": (f"same ladder/drives at truncation +-{Ns} (M={Ms}, 256 times), measured: build "
                   f"{t_b - t_a:.2f}s, eigh {t_c - t_b:.2f}s, U {t_d - t_c:.2f}s, P {t_e - t_d:.2f}s; "
                   f"extrapolated to M={M} with eigh ~M^3 (x{r ** 3:.0f}) and the other stages ~M^2"),
        "sample_solves_per_s": 1.0 / (t_e - t_a),
        "sample_seconds": t_e - t_a,
    }


def run_executor_bench(args, torch, mmf):
    """Batched (all requests at t = 0) or served (Poisson arrivals) solves
    through the continuous-batching executor; FP64 and refined mixed precision."""
    from paper_2005_03426_amd import serve
    from workloads import cfg3_batch, cfg5_serving
    if args.workload == "batch512":
        items = [(0.0, p, ts, t0) for p, ts, t0 in cfg3_batch()]
        cfg = {"workload": "batch512", "requests": len(items), "dims": "22..1995", "times": 32}
    else:
        items = cfg5_serving(R=args.requests or 2000)
        cfg = {"workload": "serve", "requests": len(items), "rate_per_s": 200.0, "dims": "50..12000",
               "times": 32}
    out_runs = {}
    for prec_name, prec in (("c128", mmf.MMF_C128), ("c64_refined", mmf.MMF_C64_REFINED)):
        if args.prec_only and prec_name != args.prec_only:
            continue
        if args.warmup:
            ex = serve.Executor(slots=args.slots, max_batch=args.max_batch)
            ex.run([serve.Request(rid=-1, arrival=0.0, problem=items[0][1], times=items[0][2], prec=prec)])
        reqs = [serve.Request(rid=k, arrival=a, problem=p, times=ts, t0=t0, prec=prec)
                for k, (a, p, ts, t0) in enumerate(items)]
        step = max(1, len(reqs) // 20)
        marks = {"next": step}

        def progress(done, name=prec_name, total=len(reqs)):
            # printed as batches of requests complete
            if done >= marks["next"]:
                marks["next"] = (done // step + 1) * step
                print(f"[bench] {args.workload} {name}: {done}/{total} requests done", file=sys.stderr, flush=True)
        ex = serve.Executor(slots=args.slots, max_batch=args.max_batch, progress=progress)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        done = ex.run(reqs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_a
        st = serve.latency_stats(done)
        failed = [(r.rid, int(r.result["M"]), int(r.problem.D), len(r.problem.N), int(r.result["info"].item()))
                  for r in done if int(r.result["info"].item()) != 0]
        bad = len(failed)
        flops = sum((40.0 / 3.0) * float(r.result["M"]) ** 3 for r in done)
        retried = [(r.rid, int(r.result["M"]), int(r.problem.D), len(r.problem.N))
                   for r in done if r.result.get("retried_c128")]
        st.update({"wall_s": wall, "eigh_tflops": flops / wall / 1e12, "failed": bad,
                   "failed_rid_M_D_F_info": failed[:64], "retried_c128": len(retried),
                   "retried_rid_M_D_F": retried[:64],
                   "band_path": sum(1 for r in done if getattr(r, "_band", None) is not None),
                   "rejected": len(ex.rejected), "batches": len(ex.batches),
                   "mean_batch": float(np.mean(ex.batches)) if ex.batches else 0.0})
        print(f"[bench] {args.workload} {prec_name}: {st}", file=sys.stderr, flush=True)
        out_runs[prec_name] = st
    main_run = out_runs.get("c128") or next(iter(out_runs.values()))
    out = {
        "metric": "Floquet eigensolves/s", "value": main_run["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": args.warmup, "ms_per_step": main_run["makespan_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic", "config": dict(cfg, slots=args.slots, max_batch=args.max_batch),
        "p50_ms": main_run["p50_ms"], "p99_ms": main_run["p99_ms"], "runs": out_runs,
    }
    print(json.dumps(out), flush=True)


def run_grouped_batch(args, torch, mmf):
    """The 512 uneven solves as one batch: every H_F assembled, one grouped
    eigensolve over all of them, then U(t) and averaged P per problem."""
    from workloads import cfg3_batch
    items = cfg3_batch()
    dev = "cuda"
    dps = [mmf.DeviceProblem(p, dev) for p, _, _ in items]
    tts = [torch.as_tensor(np.asarray(ts), dtype=torch.float64, device=dev) for _, ts, _ in items]
    sizes = [dp.M for dp in dps]
    HFs = [torch.empty((m, m), dtype=torch.complex128, device=dev) for m in sizes]
    ws = [torch.empty(m, dtype=torch.float64, device=dev) for m in sizes]
    info = torch.zeros(len(dps), dtype=torch.int32, device=dev)
    out_runs = {}
    for prec_name, prec in (("c128", mmf.MMF_C128), ("c64_refined", mmf.MMF_C64_REFINED)):
        if args.prec_only and prec_name != args.prec_only:
            continue
        work = torch.empty(mmf.eigh_batched_workspace_bytes(sizes, prec), dtype=torch.uint8, device=dev)
        ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))

        def step():
            for dp, HF in zip(dps, HFs):
                mmf.build_floquet(dp, out=HF)
            ev0.record()
            mmf.eigh_batched(HFs, prec, ws=ws, work=work, info=info)
            ev1.record()
            res = []
            for (p, ts, t0), dp, tt, HF, w in zip(items, dps, tts, HFs, ws):
                res.append((mmf.evolve(dp, HF, w, t0, tt), mmf.avg_prob(dp, HF, w)[0]))
            ev2.record()
            return res

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        eig_ms = 0.0
        for _ in range(args.steps):
            res = step()
            torch.cuda.synchronize()
            eig_ms += ev0.elapsed_time(ev1)
        wall = time.perf_counter() - t_a
        bad = int(info.ne(0).sum().item())
        flops = sum((40.0 / 3.0) * float(m) ** 3 for m in sizes)
        st = {"solves_per_s": len(dps) * args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
              "eigh_ms_per_step": eig_ms / args.steps, "eigh_tflops": flops / (eig_ms / args.steps * 1e-3) / 1e12,
              "failed": bad}
        if not args.no_check:
            # sampled problems: eigen residual / orthogonality against a freshly
            # assembled H_F, and sum_i P(i, j) = 1 (exact for orthonormal eigenvectors)
            st["max_residual"] = st["max_orth_err"] = st["max_colsum_err"] = 0.0
            for k in (0, len(dps) // 2, len(dps) - 1):
                H = mmf.build_floquet(dps[k]).T          # H_F (row-major view)
                Phi = HFs[k].T                           # columns = eigenvectors
                w = ws[k]
                r = torch.linalg.norm(H @ Phi - Phi * w) / torch.linalg.norm(H)
                eye = torch.eye(sizes[k], dtype=Phi.dtype, device=dev)
                o = (Phi.conj().T @ Phi - eye).abs().max()
                P = res[k][1]
                c = (P.sum(0) - 1).abs().max()
                st["max_residual"] = max(st["max_residual"], float(r))
                st["max_orth_err"] = max(st["max_orth_err"], float(o))
                st["max_colsum_err"] = max(st["max_colsum_err"], float(c))
        print(f"[bench] batch512 grouped {prec_name}: {st}", file=sys.stderr, flush=True)
        out_runs[prec_name] = st
        del work
    main_run = out_runs.get("c128") or next(iter(out_runs.values()))
    out = {
        "metric": "Floquet eigensolves/s", "value": main_run["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "batch512", "requests": len(dps), "dims": f"{min(sizes)}..{max(sizes)}",
                   "times": 32, "mode": "grouped"},
        "runs": out_runs,
    }
    print(json.dumps(out), flush=True)


def run_plan_bench(args, torch, mmf):
    """A batch of solves as one BatchPlan: all device state resident, the
    whole launch sequence recorded once as a graph and replayed per step.
    Compared on the same GPU with the same plan launched eagerly and with the
    small orders sent to the grouped path (tile table of zeros)."""
    from paper_2005_03426_amd.batch import BatchPlan
    from paper_2005_03426_amd import autotune
    from workloads import cfg3_batch, cfg3_uniform_sweep
    items = cfg3_uniform_sweep() if args.workload == "sweep512" else cfg3_batch()
    probs = [p for p, _, _ in items]
    times = [ts for _, ts, _ in items]
    t0 = items[0][2]
    tuned = autotune.load_table()
    variants = [("graph_tuned", tuned, True), ("eager_tuned", tuned, False), ("graph_grouped_only", [0] * 8, True)]
    runs = {}
    sizes = None
    for name, tiles, graph in variants:
        plan = BatchPlan(probs, times, t0, tiles=tiles, graph=graph, group_max=args.group_max)
        sizes = plan.sizes
        for _ in range(args.warmup):
            plan.run()
        plan.synchronize()
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for _ in range(args.steps):
            plan.run()
        plan.synchronize()
        wall = time.perf_counter() - t_a
        bad = int(plan.info().ne(0).sum().item())
        flops = sum((40.0 / 3.0) * float(m) ** 3 for m in sizes)
        runs[name] = {"solves_per_s": len(probs) * args.steps / wall, "ms_per_batch": wall * 1e3 / args.steps,
                      "eigh_tflops_nominal_over_batch": flops * args.steps / wall / 1e12, "failed": bad,
                      "tiles": list(tiles) if tiles is not None else "library rule"}
        print(f"[bench] {args.workload} {name}: {runs[name]}", file=sys.stderr, flush=True)
        del plan
        torch.cuda.empty_cache()
    main_run = runs["graph_tuned"]
    out = {
        "metric": "Floquet eigensolves/s", "value": main_run["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": args.workload, "requests": len(probs), "dims": f"{min(sizes)}..{max(sizes)}",
                   "times": len(times[0]), "mode": "BatchPlan (recorded graph)"},
        "runs": runs,
        "graph_gain_vs_eager": runs["graph_tuned"]["solves_per_s"] / runs["eager_tuned"]["solves_per_s"],
        "small_solver_gain_vs_grouped": runs["graph_tuned"]["solves_per_s"] / runs["graph_grouped_only"]["solves_per_s"],
    }
    print(json.dumps(out), flush=True)


def run_lattice_sweep(args, torch, mmf):
    """Quasienergy scan of the driven lattice (D = 256, +-10, M = 5376) over
    64 drive frequencies in [0.2, 1]: every H_F assembled, then one grouped
    eigenvalue-only solve (reduction + bisection)."""
    from workloads import lattice_sweep
    dev = "cuda"
    prec = {"c128": mmf.MMF_C128, "c64_raw": mmf.MMF_C64_RAW}.get(args.prec)
    assert prec is not None, "the eigenvalue-only scan runs in c128 or c64_raw"
    probs = lattice_sweep(count=args.requests or 64)
    dps = [mmf.DeviceProblem(p, dev) for p in probs]
    M = dps[0].M
    sizes = [dp.M for dp in dps]
    HFs = [torch.empty((m, m), dtype=torch.complex128, device=dev) for m in sizes]
    ws = [torch.empty(m, dtype=torch.float64, device=dev) for m in sizes]
    info = torch.zeros(len(dps), dtype=torch.int32, device=dev)
    work = torch.empty(mmf.eigvalsh_batched_workspace_bytes(sizes, prec), dtype=torch.uint8, device=dev)
    print(f"[bench] lattice sweep: {len(dps)} frequencies, M={M}", file=sys.stderr, flush=True)

    def step():
        for dp, HF in zip(dps, HFs):
            mmf.build_floquet(dp, out=HF)
        mmf.eigvalsh_batched(HFs, prec, ws=ws, work=work, info=info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not args.no_ktimer:
        mmf.call("mmf_ktimer_arm", b"hemv" if prec == mmf.MMF_C128 else b"hemv_c64")
    t_a = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_a
    out = {
        "metric": "Floquet eigensolves/s", "value": len(dps) * args.steps / elapsed, "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if prec == mmf.MMF_C128 else "c64", "data": "synthetic",
        "config": {"workload": "lattice_sweep", "D": 256, "M": M, "frequencies": len(dps),
                   "omega": [0.2, 1.0], "truncation": 10, "outputs": "eigenvalues only"},
        "eigvalsh_tflops": len(dps) * (16.0 / 3.0) * M ** 3 / (elapsed / args.steps) / 1e12,
    }
    if not args.no_ktimer:
        nl, tms, wb = C.c_int64(0), C.c_double(0.0), C.c_double(0.0)
        mmf.call("mmf_ktimer_read", C.byref(nl), C.byref(tms), C.byref(wb))
        if nl.value:
            per = wb.value / nl.value
            avg_ms = tms.value / nl.value
            gbs = per / (avg_ms / 1e3) / 1e9
            out["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "ht_hemv (grouped)",
                               "launches": int(nl.value), "avg_launch_us": avg_ms * 1e3,
                               "algorithmic_bytes_per_launch": per,
                               "share_of_step": tms.value / (elapsed * 1e3)}
    if not args.no_check:
        assert not info.any().item()
        # every spectrum ascending; the undriven closed form is a CPU pin, here
        # the trace identity: sum of quasienergies = tr H_F = 0 for this model
        out["check"] = {"max_abs_trace": max(abs(float(w.sum())) for w in ws),
                        "ascending": all(bool((w[1:] >= w[:-1]).all()) for w in ws)}
    if not args.no_cpu_baseline:
        import os
        import oracle
        print("[bench] cpu baseline (oracle, one frequency) ...", file=sys.stderr, flush=True)
        t_c = time.perf_counter()
        q = oracle.quasienergies(probs[len(probs) // 2])
        dt = time.perf_counter() - t_c
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count() or 1
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
                               "sample": f"one frequency of the same scan (M={M}, eigenvalues only): {dt:.1f} s"}
        qg = ws[len(probs) // 2].cpu().numpy()
        out.setdefault("check", {})["max_dev_vs_oracle"] = float(np.abs(qg - q).max())
    print(json.dumps(out), flush=True)


def run_window(args, torch, mmf):
    """Partial spectrum vs full eigensolve on one lattice Floquet matrix
    (D = 256, +-10, M = 5376, omega = 0.6): the Brillouin-zone window
    [-omega/2, omega/2) holds the 256 Floquet states."""
    from workloads import lattice_problem
    dev = "cuda"
    p = lattice_problem(0.6, D=256, N=10)
    dp = mmf.DeviceProblem(p, dev)
    M = dp.M
    HF = torch.empty((M, M), dtype=torch.complex128, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def one(window):
        mmf.build_floquet(dp, out=HF)
        ev[0].record()
        if window:
            out = mmf.eigh_window(HF, -0.3, 0.3, 256)
        else:
            out = mmf.eigh(HF)
        ev[1].record()
        return out

    res = {}
    for name, window in (("window", True), ("full", False)):
        for _ in range(args.warmup):
            one(window)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            out = one(window)
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        res[name] = float(np.median(ms))
        if window:
            res["count"] = int(out[2].item())
    out = {
        "metric": "Floquet eigensolves/s", "value": 1e3 / res["window"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["window"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "window_lattice", "D": 256, "M": M, "omega": 0.6, "window": [-0.3, 0.3],
                   "states": res["count"]},
        "full_eigh_ms": res["full"], "window_eigh_ms": res["window"], "speedup": res["full"] / res["window"],
    }
    print(json.dumps(out), flush=True)


def run_band_window(args, torch, mmf):
    """Floquet states of the one-drive workload (16 levels, harmonics 1 and 2,
    +-650, M = 20816, half-bandwidth 47): the window [-omega/2, omega/2)
    through the band-aware partial-spectrum solver, against the band-aware
    full solve and the dense partial-spectrum solver on the same matrix."""
    from workloads import one_drive_band
    dev = "cuda"
    p, ts, t0 = one_drive_band()
    dp = mmf.DeviceProblem(p, dev)
    M = dp.M
    b = mmf.floquet_half_bandwidth(p)
    HF = torch.empty((M, M), dtype=torch.complex128, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def one(kind):
        mmf.build_floquet(dp, out=HF)
        ev[0].record()
        if kind == "band_window":
            out = mmf.eigh_band_window(HF, b, -0.5, 0.5, 64)
        elif kind == "band_full":
            out = mmf.eigh_band(HF, b)
        else:
            out = mmf.eigh_window(HF, -0.5, 0.5, 64)
        ev[1].record()
        return out

    res = {}
    for kind in ("band_window", "band_full", "dense_window"):
        for _ in range(args.warmup):
            one(kind)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            out = one(kind)
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        res[kind] = float(np.median(ms))
        if kind == "band_window":
            res["count"] = int(out[2].item())
        print(f"[bench] band window: {kind} {res[kind]:.1f} ms", file=sys.stderr, flush=True)
    out = {
        "metric": "Floquet eigensolves/s", "value": 1e3 / res["band_window"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["band_window"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "band_window20816", "D": dp.D, "M": M, "half_bandwidth": b, "window": [-0.5, 0.5],
                   "states": res["count"]},
        "band_window_ms": res["band_window"], "band_full_ms": res["band_full"],
        "dense_window_ms": res["dense_window"],
    }
    print(json.dumps(out), flush=True)


def run_precision(args, torch, mmf):
    """16-level spectrum under two drives, M = 41616: the complex64 paths
    (raw, and refined in FP64) against the plain complex128 solve on the same
    GPU.  The oracle does not reach this size, so the complex128 GPU result
    (matched to the oracle at smaller sizes) is the reference; errors are
    reported for quasienergies, U(t) at 256 times and the averaged P."""
    from workloads import cfg4_precision
    dev = "cuda"
    p, ts, t0 = cfg4_precision()
    dp = mmf.DeviceProblem(p, dev)
    M, D = dp.M, dp.D
    tt = torch.as_tensor(np.asarray(ts), dtype=torch.float64, device=dev)
    print(f"[bench] precision workload: M={M} D={D}", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    ref = None
    for name, prec in (("c128", mmf.MMF_C128), ("c64_refined", mmf.MMF_C64_REFINED), ("c64_raw", mmf.MMF_C64_RAW)):
        if args.prec_only and name not in ("c128", args.prec_only):
            continue
        HF = mmf.build_floquet(dp)
        work = torch.empty(mmf.eigh_workspace_bytes(M, prec), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        ev0.record()
        w, Pt, info = mmf.eigh(HF, prec, work=work)
        ev1.record()
        t_wait = time.perf_counter()
        while not ev1.query():                       # a progress line while the long solve runs
            time.sleep(1.0)
            if time.perf_counter() - t_wait > 30.0:
                print(f"[bench] precision {name}: solving ...", file=sys.stderr, flush=True)
                t_wait = time.perf_counter()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        del work
        U = mmf.evolve(dp, Pt, w, t0, tt)
        P, _ = mmf.avg_prob(dp, Pt, w)
        g = torch.Generator(device="cpu").manual_seed(0)
        idx = torch.randperm(M, generator=g)[:32].to(dev)
        H = mmf.build_floquet(dp).T
        Phi = Pt[idx].T.contiguous()
        resid = float((H @ Phi - Phi * w[idx][None, :]).abs().max()) / torch.linalg.matrix_norm(H, ord=1).item()
        del H, Phi
        r = {"eigh_s": ms / 1e3, "eigh_tflops_nominal": (40.0 / 3.0) * M ** 3 / (ms / 1e3) / 1e12,
             "info": int(info.item()), "sampled_residual": resid}
        if ref is None:
            ref = (w.clone(), U.clone(), P.clone())
        else:
            scale = max(1.0, float(ref[0].abs().max()))
            r["eps_err_vs_c128"] = float((w - ref[0]).abs().max()) / scale
            r["U_err_vs_c128"] = float((U - ref[1]).abs().max())
            r["P_err_vs_c128"] = float((P - ref[2]).abs().max())
        print(f"[bench] precision {name}: {r}", file=sys.stderr, flush=True)
        res[name] = r
        del HF, Pt, w, U, P
        torch.cuda.empty_cache()
    main_name = "c64_refined" if "c64_refined" in res else "c128"
    out = {
        "metric": "Floquet eigensolves/s", "value": 1.0 / res[main_name]["eigh_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": res[main_name]["eigh_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64" if main_name == "c64_refined" else "c128", "data": "synthetic",
        "config": {"workload": "precision41616", "D": D, "M": M, "times": len(ts),
                   "drives": [float(x) for x in p.omega], "truncation": [int(x) for x in p.N],
                   "reference": "complex128 solve on the same GPU"},
        "runs": res,
    }
    print(json.dumps(out), flush=True)


def run_single(args, torch, mmf, name, steps, warmup, prec, ktimer=True, check_enabled=True):
    """K timed steps of one whole Floquet solve (assemble -> eigh -> U -> P)
    of the named workload; returns the result dictionary (no printing)."""
    dev = "cuda"
    p, ts, t0 = workload(name)
    dp = mmf.DeviceProblem(p, dev)
    M, D, T = dp.M, dp.D, len(ts)
    print(f"[bench] workload {name}: D={D} M={M} T={T}", file=sys.stderr, flush=True)
    tt = torch.as_tensor(np.asarray(ts), dtype=torch.float64, device=dev)
    HF = torch.empty((M, M), dtype=torch.complex128, device=dev)
    w = torch.empty(M, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    band = getattr(args, "band", False) and prec == mmf.MMF_C128
    bw = mmf.floquet_half_bandwidth(p)
    if band:
        print(f"[bench] band path: half-bandwidth {bw}", file=sys.stderr, flush=True)
        ework = torch.empty(mmf.eigh_band_workspace_bytes(M, bw), dtype=torch.uint8, device=dev)
    else:
        ework = torch.empty(mmf.eigh_workspace_bytes(M, prec), dtype=torch.uint8, device=dev)

    b = C.c_size_t(0)
    mmf.call("mmf_evolve_workspace", dp.ref, C.c_int32(T), C.byref(b))
    uwork = torch.empty(b.value, dtype=torch.uint8, device=dev)
    mmf.call("mmf_avg_prob_workspace", dp.ref, C.byref(b))
    pwork = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    pstat = torch.zeros(1, dtype=torch.int32, device=dev)

    stages = ("assemble", "eigh", "evolve", "avg_prob")

    def step(ev=None):
        if ev: ev[0].record()
        mmf.build_floquet(dp, out=HF)
        if ev: ev[1].record()
        if band:
            mmf.eigh_band(HF, bw, w=w, work=ework, info=info)
        else:
            mmf.eigh(HF, prec=prec, w=w, work=ework, info=info)
        if ev: ev[2].record()
        U = mmf.evolve(dp, HF, w, t0, tt, work=uwork)
        if ev: ev[3].record()
        P, _ = mmf.avg_prob(dp, HF, w, work=pwork, status=pstat)
        if ev: ev[4].record()
        return U, P

    if args.calib_copy:
        # plain copy of a known size: calibrates the HBM byte counters of a
        # --pmc run (FETCH_SIZE / WRITE_SIZE of this kernel vs 1 GiB each way)
        src = torch.ones(1 << 26, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    L = mmf.lib()
    torch.cuda.synchronize()
    # dominant kernel: the HEMV of the one-stage reduction, or the
    # back-transformation by the bulge-chasing reflectors of the two-stage one
    two_stage = prec == mmf.MMF_C128 and (M >= mmf.eigh_two_stage_min() or (band and bw <= 64))
    if ktimer:
        mmf.call("mmf_ktimer_arm", b"bt2" if two_stage else b"hemv")
    t_start = time.perf_counter()
    for k in range(steps):
        U, P = step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kt = None
    if ktimer:
        nl, tms, wb = C.c_int64(0), C.c_double(0.0), C.c_double(0.0)
        mmf.call("mmf_ktimer_read", C.byref(nl), C.byref(tms), C.byref(wb))
        kt = {"launches": int(nl.value), "total_ms": tms.value, "bytes": wb.value}
    per_stage = {s: [] for s in stages}
    step_ms = []
    for ev in evs:
        for j, s in enumerate(stages):
            per_stage[s].append(ev[j].elapsed_time(ev[j + 1]))
        step_ms.append(ev[0].elapsed_time(ev[4]))
    med = {s: float(np.median(v)) for s, v in per_stage.items()}
    print(f"[bench] {name}: timed {steps} steps: {elapsed:.3f}s; stages(ms) {med}", file=sys.stderr, flush=True)

    eigh_flops = (40.0 / 3.0) * M ** 3
    t_eigh = med["eigh"] / 1e3
    eigh_tflops = eigh_flops / t_eigh / 1e12

    check = {}
    if check_enabled:
        assert int(info.item()) == 0, "eigensolver reported non-convergence"
        g = torch.Generator(device="cpu").manual_seed(0)
        idx = torch.randperm(M, generator=g)[:64].to(dev)
        H = mmf.build_floquet(dp)                       # H_F again (storage = H^T)
        Hm = H.T                                        # logical H_F (view)
        Phi_s = HF[idx].T.contiguous()                  # columns of sampled eigenvectors (M x 64)
        R = Hm @ Phi_s - Phi_s * w[idx][None, :]
        hn = torch.linalg.matrix_norm(Hm, ord=1).item()
        check["eig_residual_rel"] = float(R.abs().max().item() / hn)
        G = HF.conj() @ Phi_s                           # rows a: <phi_a | phi_idx>
        G[idx, torch.arange(64, device=dev)] -= 1.0
        check["orth_max"] = float(G.abs().max().item())
        check["trace_rel"] = float(abs(w.sum().item() - torch.diagonal(Hm).real.sum().item()) / hn)
        check["colsum_P_max_dev"] = float((P.sum(dim=0) - 1.0).abs().max().item())
        Ud = U.conj().transpose(1, 2) @ U - torch.eye(D, dtype=U.dtype, device=dev)
        # a truncation diagnostic, not a numerical error: U of a finite Fourier
        # box is unitary only as the truncation converges (the oracle on the
        # same ladder: 0.27, 0.10, 0.032, 0.012 at truncation 6, 8, 10, 12)
        check["truncation_unitarity_defect_U"] = float(Ud.abs().max().item())
        del H, R, G

    value = steps / elapsed
    out = {
        "metric": "Floquet eigensolves/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prec == mmf.MMF_C128 else ("c64+f64" if prec == mmf.MMF_C64_REFINED else "c64"),
        "data": "synthetic",
        "config": {"workload": name, "precision": args.prec, "D": D, "M": M, "times": T,
                   "drives": [float(x) for x in p.omega], "truncation": [int(x) for x in p.N],
                   "reduction": (f"band (chase from the native half-bandwidth {bw})" if band
                                 else "two-stage" if two_stage else "one-stage")},
        "eigh_tflops": eigh_tflops,
        "eigh_frac_fp64_peak": eigh_tflops / FP64_MFMA_PEAK_TFLOPS,
        "stage_ms": med,
        "step_ms_p50": float(np.percentile(step_ms, 50)),
        "step_ms_p99": float(np.percentile(step_ms, 99)),
        "check": check,
    }
    if kt and kt["launches"] and two_stage:
        per_launch_flops = kt["bytes"] / kt["launches"]
        avg_ms = kt["total_ms"] / kt["launches"]
        tfs = per_launch_flops / (avg_ms / 1e3) / 1e12
        out["roofline"] = {
            "bound": "mfma", "achieved": tfs, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tfs / FP64_MFMA_PEAK_TFLOPS, "traffic": counter_traffic("bt2", name),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "kernel": "bt2_apply (back-transformation by the bulge-chasing reflectors: compact-WY groups "
                      "of 16 on the FP64 matrix cores; achieved counts the algorithmic flops, the kernel "
                      "executes 1.25 times as many in the usual count, forming each complex product from "
                      "three real ones)",
            "launches": kt["launches"], "avg_launch_us": avg_ms * 1e3,
            "algorithmic_flops_per_launch": per_launch_flops,
            "share_of_step": kt["total_ms"] / (elapsed * 1e3),
        }
    elif kt and kt["launches"]:
        per_launch_bytes = kt["bytes"] / kt["launches"]
        avg_ms = kt["total_ms"] / kt["launches"]
        gbs = per_launch_bytes / (avg_ms / 1e3) / 1e9
        out["roofline"] = {
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "kernel": "ht_hemv (Hermitian matrix-vector product of the tridiagonal reduction)",
            "launches": kt["launches"], "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "share_of_step": kt["total_ms"] / (elapsed * 1e3),
        }
    # the two-stage path executes (16/3 + 10 + 8) M^3 real flops in the usual
    # count of four real products per complex one (band reduction, stage-2
    # back-transformation with its zero triangles, stage-1 back-transformation;
    # its GEMMs and the stage-2 kernel form each complex product from three
    # real ones, which this count does not discount); the one-stage path the
    # nominal (40/3) M^3
    # (the band path: only the stage-2 back-transformation's 10 M^3)
    exec_flops = (10.0 * M ** 3 if band else (16.0 / 3.0 + 10.0 + 8.0) * M ** 3 if two_stage else eigh_flops)
    out["eigh_executed_tflops"] = exec_flops / t_eigh / 1e12
    out["eigh_executed_frac_fp64_peak"] = out["eigh_executed_tflops"] / FP64_MFMA_PEAK_TFLOPS
    out["eigh_roofline"] = {
        "bound": "mfma", "achieved": eigh_tflops, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": eigh_tflops / FP64_MFMA_PEAK_TFLOPS,
        "note": "whole mmf_eigh call at the nominal (40/3) M^3 flops of reduction + back-transformation",
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ladder20808")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the one-solve M = 41616 measurement")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-ktimer", action="store_true")
    ap.add_argument("--band", action="store_true",
                    help="solve with mmf_eigh_band at the workload's Floquet half-bandwidth")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--sync-every", type=int, default=0,
                    help="profiling aid: the library waits for the device after every n launches")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--group-max", type=int, default=64, help="problems per grouped eigensolver call (BatchPlan)")
    ap.add_argument("--requests", type=int, default=0, help="serve: requests (default 2000); lattice: frequencies (64)")
    ap.add_argument("--prec-only", default="")
    ap.add_argument("--batch-mode", default="executor", choices=["grouped", "executor", "plan"])
    ap.add_argument("--prec", default="c128", choices=["c128", "c64_refined", "c64_raw"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import torch
    import paper_2005_03426_amd as mmf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda"
    if args.sync_every:
        mmf.call("mmf_profile_sync_every", C.c_int64(args.sync_every))
    if args.workload == "precision41616":
        run_precision(args, torch, mmf)
        return
    if args.workload == "band_window20816":
        run_band_window(args, torch, mmf)
        return
    if args.workload == "window_lattice":
        run_window(args, torch, mmf)
        return
    if args.workload == "lattice_sweep":
        run_lattice_sweep(args, torch, mmf)
        return
    if args.workload == "sweep512" or (args.workload == "batch512" and args.batch_mode == "plan"):
        run_plan_bench(args, torch, mmf)
        return
    if args.workload == "batch512" and args.batch_mode == "grouped":
        run_grouped_batch(args, torch, mmf)
        return
    if args.workload in ("batch512", "serve"):
        run_executor_bench(args, torch, mmf)
        return
    prec = {"c128": mmf.MMF_C128, "c64_refined": mmf.MMF_C64_REFINED, "c64_raw": mmf.MMF_C64_RAW}[args.prec]
    out = run_single(args, torch, mmf, args.workload, args.steps, args.warmup, prec,
                     ktimer=not args.no_ktimer, check_enabled=not args.no_check)
    if args.workload == "ladder20808" and not args.no_large:
        # the 16-level, M = 41616 configuration on which the eigensolve's
        # fraction of the FP64 peak is quoted: one timed solve (the library is
        # already warm), same stages, same checks
        torch.cuda.empty_cache()
        big = run_single(args, torch, mmf, "spec41616", 1, 0, prec, ktimer=not args.no_ktimer,
                         check_enabled=not args.no_check)
        keep = ("value", "ms_per_step", "stage_ms", "eigh_tflops", "eigh_frac_fp64_peak", "eigh_executed_tflops",
                "eigh_executed_frac_fp64_peak", "check", "roofline", "config")
        out["at_41616"] = {k: big[k] for k in keep if k in big}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline and args.workload == "ladder20808":
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
