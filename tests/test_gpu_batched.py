"""GPU tests of the grouped (batched) eigensolver and batched Floquet solves.

A batch of uneven Hermitian matrices (orders that span several tiles, ragged
tails, the 1x1 and empty cases) goes through mmf_eigh_batched in one call.
Each problem's kernels do the same arithmetic in the same order as a single
mmf_eigh call, so results must match the single call bit for bit; they are
also checked against the FP64 oracle (eigenvalues within 1e-10 relative,
residual and orthogonality within 1e-12).  Batched Floquet solves are
compared with the oracle's U(t,t0) and averaged probabilities (1e-10).
"""
import numpy as np
import pytest

import oracle
from workloads import random_problem, cfg1_tls, tls_problem, gue
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu

SIZES = [65, 1, 17, 0, 130, 2, 300, 64, 257, 33]


def _hermitian(n, seed):
    rng = np.random.default_rng(seed)
    return gue(rng, n, 1.0) if n else np.zeros((0, 0), complex)


@pytest.mark.parametrize("prec", [0, 2, 1], ids=["c128", "c64_raw", "c64_refined"])
def test_batched_equals_single_calls(prec):
    torch, mmf = require_gpu()
    Hs = [_hermitian(n, 500 + k) for k, n in enumerate(SIZES)]
    log(f"batched eigh prec={prec} sizes={SIZES}")
    mats = [to_dev_cm(torch, H) if H.size else torch.empty((0, 0), dtype=torch.complex128, device="cuda")
            for H in Hs]
    ws, Pts, info = mmf.eigh_batched(mats, prec)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(SIZES)
    for k, H in enumerate(Hs):
        n = H.shape[0]
        if n == 0:
            continue
        w1, P1, i1 = mmf.eigh(to_dev_cm(torch, H), prec)
        torch.cuda.synchronize()
        assert int(i1.item()) == 0
        assert torch.equal(ws[k], w1), f"eigenvalues differ from the single call, n={n}"
        assert torch.equal(Pts[k], P1), f"eigenvectors differ from the single call, n={n}"


def test_batched_against_oracle():
    torch, mmf = require_gpu()
    Hs = [_hermitian(n, 900 + k) for k, n in enumerate(SIZES) if n]
    log(f"batched eigh vs oracle, {len(Hs)} problems")
    ws, Pts, info = mmf.eigh_batched([to_dev_cm(torch, H) for H in Hs])
    torch.cuda.synchronize()
    assert not info.any().item()
    for H, w, Pt in zip(Hs, ws, Pts):
        n = H.shape[0]
        w = w.cpu().numpy()
        Phi = from_dev_cm(Pt)
        wo, _ = oracle.eigh(H)
        scale = max(1.0, np.abs(wo).max())
        assert np.all(np.diff(w) >= 0)
        assert np.abs(w - wo).max() <= 1e-10 * scale
        assert np.linalg.norm(H @ Phi - Phi * w) / max(1.0, np.linalg.norm(H)) < 1e-12
        assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-12


def test_batched_uniform_many_small():
    """A scan of many equal small problems (one grouped launch per step)."""
    torch, mmf = require_gpu()
    count = 300
    Hs = [_hermitian(40, 7000 + k) for k in range(count)]
    log(f"batched eigh {count} x n=40")
    ws, Pts, info = mmf.eigh_batched([to_dev_cm(torch, H) for H in Hs])
    torch.cuda.synchronize()
    assert not info.any().item()
    for k in (0, 1, 150, count - 1):
        wo, _ = oracle.eigh(Hs[k])
        assert np.abs(ws[k].cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
        Phi = from_dev_cm(Pts[k])
        assert np.linalg.norm(Hs[k] @ Phi - Phi * ws[k].cpu().numpy()) < 1e-12 * max(1.0, np.linalg.norm(Hs[k]))


def test_solve_batched_floquet_against_oracle():
    """Uneven Floquet problems (two-level sweep plus random multimode ones)."""
    torch, mmf = require_gpu()
    p1, ts, t0 = cfg1_tls()
    probs = [p1, tls_problem(1.0, 0.3, 1.2, 12), random_problem(3, (3, 2), seed=41),
             random_problem(2, (5,), seed=42), random_problem(4, (2, 2), seed=43)]
    log("solve_batched on 5 Floquet problems")
    outs = mmf.solve_batched(probs, ts, t0)
    torch.cuda.synchronize()
    for p, out in zip(probs, outs):
        assert int(out["info"].item()) == 0
        H = oracle.build_floquet(p)
        wo, Phio = oracle.eigh(H)
        assert np.abs(out["w"].cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
        Uo = oracle.evolve(p, Phio, wo, t0, ts)
        assert np.abs(out["U"].cpu().numpy() - Uo).max() < 1e-10
        Po = oracle.avg_prob(p, Phio)
        assert np.abs(out["P"].cpu().numpy() - Po).max() < 1e-10


@pytest.mark.skip(reason="the batched two-stage path is switched off (BATCHED_TWO_STAGE in csrc/eigh.hip): the "
                         "serving benchmark with it ended in a GPU fault whose cause has not been found")
def test_batched_routes_large_orders_to_the_two_stage_path(monkeypatch):
    """With the two-stage threshold lowered to 100, the batch's problems of
    order >= 100 are solved one by one by the two-stage path inside the
    batched call: bitwise equal to single calls under the same setting (which
    take the two-stage path too), and against the oracle; the rest stay on
    the grouped and one-workgroup paths."""
    torch, mmf = require_gpu()
    monkeypatch.setenv("MMF_EIGH_TWO_STAGE_MIN", "100")
    assert mmf.eigh_two_stage_min() == 100
    sizes = [40, 150, 99, 100, 257, 7]
    Hs = [_hermitian(n, 900 + k) for k, n in enumerate(sizes)]
    ws, Pts, info = mmf.eigh_batched([to_dev_cm(torch, H) for H in Hs])
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(sizes)
    for H, w, Pt in zip(Hs, ws, Pts):
        w1, P1, info1 = mmf.eigh(to_dev_cm(torch, H))
        torch.cuda.synchronize()
        assert int(info1.item()) == 0
        assert torch.equal(w1, w) and torch.equal(P1, Pt)
        wo, _ = oracle.eigh(H)
        n = H.shape[0]
        Phi = from_dev_cm(Pt)
        assert np.abs(w.cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
        assert np.linalg.norm(H @ Phi - Phi * w.cpu().numpy()) <= 1e-12 * max(1.0, np.linalg.norm(H)) * n
        assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-12 * max(1, n)
    log("batched: orders >= 100 through the two-stage path, bitwise equal to single calls")
