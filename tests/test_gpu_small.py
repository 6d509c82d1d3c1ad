"""The one-workgroup LDS eigensolver (orders <= 64) and the batch machinery
around it, against the oracle.

* single matrices of every awkward order (1, 2, odd, bucket edges, 64):
  eigenvalues within 1e-12 normwise of LAPACK, residual and orthogonality at
  the FP64 level, spectral projectors of simple eigenvalues within 1e-10;
* degenerate and diagonal inputs (exact multiplicities, the static limit);
* a batch of uneven small and large orders through every workgroup size of
  the tile table and through the grouped path, each problem against the
  oracle, and the default batch bitwise equal to single calls;
* the uniform two-level frequency sweep (512 x M = 34) through the recorded
  graph of a BatchPlan: every replay, with eager work and synchronisations in
  between, bitwise equal to the eager pass, and sampled solves (w, U, P)
  within 1e-10 of the oracle.
"""
import numpy as np
import pytest

import oracle
from workloads import gue, cfg3_uniform_sweep, random_problem
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu


def _check_pairs(H, w, Phi, tol_w=1e-12):
    wo, Po = oracle.eigh(H)
    n = H.shape[0]
    scale = max(1.0, np.abs(wo).max())
    assert np.abs(w - wo).max() <= tol_w * scale
    assert np.linalg.norm(H @ Phi - Phi * w) <= 1e-13 * max(1.0, np.linalg.norm(H)) * max(1, n)
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-13 * max(1, n)
    gaps = np.diff(wo)
    for a in range(n):
        left = gaps[a - 1] if a > 0 else np.inf
        right = gaps[a] if a < n - 1 else np.inf
        if min(left, right) > 1e-6 * scale:
            Pg = np.outer(Phi[:, a], Phi[:, a].conj())
            Pr = np.outer(Po[:, a], Po[:, a].conj())
            assert np.abs(Pg - Pr).max() < 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 9, 16, 17, 31, 33, 48, 63, 64])
def test_small_single_random(n):
    torch, mmf = require_gpu()
    H = gue(np.random.default_rng(500 + n), n, 1.0)
    w, Pt, info = mmf.eigh(to_dev_cm(torch, H))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    _check_pairs(H, w.cpu().numpy(), from_dev_cm(Pt))


@pytest.mark.parametrize("kind", ["degenerate", "diagonal", "zero", "scaled"])
def test_small_structured(kind):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(7)
    n = 40
    if kind == "degenerate":
        d = np.repeat([-1.0, 0.25, 2.0, 3.5], 10)
        U, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
        H = (U * d) @ U.conj().T
        H = (H + H.conj().T) / 2
    elif kind == "diagonal":
        H = np.diag(rng.permutation(np.arange(n) % 7).astype(float)).astype(np.complex128)
    elif kind == "zero":
        H = np.zeros((n, n), np.complex128)
    else:
        H = 1e6 * gue(rng, n, 1.0)
    w, Pt, info = mmf.eigh(to_dev_cm(torch, H))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w, Phi = w.cpu().numpy(), from_dev_cm(Pt)
    wo = oracle.eigvalsh(H)
    scale = max(1.0, np.abs(wo).max())
    log(f"small {kind}: eig err {np.abs(w - wo).max() / scale:.2e}")
    assert np.abs(w - wo).max() <= 1e-12 * scale
    assert np.linalg.norm(H @ Phi - Phi * w) <= 1e-12 * max(1.0, np.linalg.norm(H))
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("tiles", [None, [64] * 8, [128] * 8, [256] * 8, [512] * 8, [0] * 8,
                                   [64, 64, 128, 128, 0, 256, 512, 256]])
def test_batched_tile_tables_against_oracle(tiles):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(99)
    sizes = [1, 5, 8, 9, 20, 33, 47, 64, 64, 65, 130, 12, 3, 40]
    Hs = [gue(rng, n, 1.0) for n in sizes]
    mats = [to_dev_cm(torch, H) for H in Hs]
    ws, mats, info = mmf.eigh_batched(mats, tiles=tiles)
    torch.cuda.synchronize()
    assert not info.any().item()
    for H, w, Pt in zip(Hs, ws, mats):
        _check_pairs(H, w.cpu().numpy(), from_dev_cm(Pt))
    if tiles is None:
        # the library's rule in a batch gives the single call's result bit for bit
        for H, w, Pt in zip(Hs, ws, mats):
            w1, P1, _ = mmf.eigh(to_dev_cm(torch, H))
            torch.cuda.synchronize()
            assert torch.equal(w1, w) and torch.equal(P1, Pt)


def test_batched_tile_table_rejects_bad_entry():
    torch, mmf = require_gpu()
    with pytest.raises(mmf.MMFError) as e:
        mmf.eigh_batched([to_dev_cm(torch, np.eye(3, dtype=np.complex128))], tiles=[96] + [0] * 7)
    assert e.value.code == -7


def test_uniform_sweep_graph_replays_against_eager_and_oracle():
    torch, mmf = require_gpu()
    from paper_2005_03426_amd.batch import BatchPlan
    items = cfg3_uniform_sweep()
    probs = [p for p, _, _ in items]
    times = [ts for _, ts, _ in items]
    t0 = items[0][2]
    assert len(probs) == 512 and all(p.E.shape[0] * (2 * p.N[0] + 1) == 34 for p in probs)
    eager = BatchPlan(probs, times, t0, graph=False)
    eager.run()
    eager.synchronize()
    ref = [{k: v.clone() for k, v in r.items() if k != "dp"} for r in eager.results()]
    plan = BatchPlan(probs, times, t0, graph=True)
    for rep in range(3):
        # eager work of the program between replays, and synchronisations
        eager.run()
        eager.synchronize()
        plan.run()
        plan.synchronize()
        torch.cuda.synchronize()
        for k, r in enumerate(plan.results()):
            for key in ("w", "Pt", "U", "P", "info"):
                assert torch.equal(r[key], ref[k][key]), (rep, k, key)
    log("uniform sweep: 3 graph replays bitwise equal to the eager pass")
    for k in (0, 137, 511):
        p = probs[k]
        H = oracle.build_floquet(p)
        wo, Po = oracle.eigh(H)
        r = plan.results()[k]
        assert np.abs(r["w"].cpu().numpy() - wo).max() < 1e-10 * max(1.0, np.abs(wo).max())
        assert np.abs(r["U"].cpu().numpy() - oracle.evolve(p, Po, wo, t0, times[k])).max() < 1e-10
        assert np.abs(r["P"].cpu().numpy() - oracle.avg_prob(p, Po)).max() < 1e-10


def test_uneven_batch_graph_against_eager():
    """A mixed batch (one-workgroup solver, grouped path, several workgroup
    sizes) recorded and replayed: bitwise equal to its eager pass."""
    torch, mmf = require_gpu()
    from paper_2005_03426_amd.batch import BatchPlan
    probs = [random_problem(2, (3,), seed=1), random_problem(3, (8,), seed=2), random_problem(2, (6, 3), seed=3),
             random_problem(4, (4, 2), seed=4), random_problem(5, (2,), seed=5)]
    ts = np.linspace(0.0, 3.0, 5)
    eager = BatchPlan(probs, ts, 0.0, graph=False)
    eager.run()
    eager.synchronize()
    ref = [{k: v.clone() for k, v in r.items() if k != "dp"} for r in eager.results()]
    plan = BatchPlan(probs, ts, 0.0, graph=True)
    for rep in range(2):
        plan.run()
        plan.synchronize()
        for k, r in enumerate(plan.results()):
            for key in ("w", "Pt", "U", "P"):
                assert torch.equal(r[key], ref[k][key]), (rep, k, key)
    for k, p in enumerate(probs):
        H = oracle.build_floquet(p)
        wo, Po = oracle.eigh(H)
        r = plan.results()[k]
        assert np.abs(r["w"].cpu().numpy() - wo).max() < 1e-10 * max(1.0, np.abs(wo).max())
        assert np.abs(r["U"].cpu().numpy() - oracle.evolve(p, Po, wo, 0.0, ts)).max() < 1e-10


def test_batched_assembly_bitwise_and_observables_against_single_calls():
    """mmf_build_floquet_batched gives the single assembly's H_F bit for bit;
    mmf_observables_batched gives the single calls' U(t) and P to rounding."""
    torch, mmf = require_gpu()
    from paper_2005_03426_amd.batch import BatchPlan
    probs = [random_problem(3, (4, 2), seed=11), random_problem(2, (10,), seed=12),
             random_problem(8, (3, 3), seed=13), random_problem(1, (5,), seed=14)]
    ts = np.linspace(0.2, 7.0, 9)
    plan = BatchPlan(probs, ts, 0.2, graph=False)
    plan.run()
    plan.synchronize()
    for k, r in enumerate(plan.results()):
        dp = r["dp"]
        H1 = mmf.build_floquet(dp)
        w1, P1t, info1 = mmf.eigh(H1)
        U1 = mmf.evolve(dp, P1t, w1, 0.2, torch.as_tensor(ts, device="cuda"))
        Pr1, st1 = mmf.avg_prob(dp, P1t, w1)
        torch.cuda.synchronize()
        # eigenvalues of the same H_F by the same rule: bitwise; then U, P to rounding
        assert torch.equal(w1, r["w"])
        assert (U1 - r["U"]).abs().max().item() < 1e-13
        assert (Pr1 - r["P"]).abs().max().item() < 1e-14
        assert int(st1.item()) == int(r["P_status"].item())
        Hb = torch.empty_like(H1)
        mmf.build_floquet_dev(dp, Hb)
        torch.cuda.synchronize()
        assert torch.equal(Hb, mmf.build_floquet(dp))
