"""Checks at the benchmark's full size (8-level ladder, two drives, M = 20808)
in the launch configuration bench.py times.

The oracle cannot diagonalise this matrix in test time, so the checks are the
properties that hold at any size, plus an independent algorithm on the GPU:
eigen-residual and orthogonality of sampled eigenvectors (1e-12), the trace
identity sum(eps) = tr H_F, column sums of the averaged probabilities
(1e-12), the eigenvalues against the eigenvalue-only solver (Householder +
Sturm bisection, 1e-12 normwise), and the refined mixed-precision path
against the FP64 path at the stated 1e-9 (quasienergies and U(t)).
"""
import numpy as np
import pytest

from workloads import cfg2_large
from gpu_util import require_gpu, log

pytestmark = pytest.mark.gpu


def _solve(mmf, torch, dp, tt, t0, prec):
    HF = mmf.build_floquet(dp)
    w, Pt, info = mmf.eigh(HF, prec)
    U = mmf.evolve(dp, Pt, w, t0, tt)
    P, _ = mmf.avg_prob(dp, Pt, w)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    return w, Pt, U, P


def test_ladder_full_size():
    torch, mmf = require_gpu()
    p, ts, t0 = cfg2_large()
    dp = mmf.DeviceProblem(p)
    M = dp.M
    assert M == 20808
    tt = torch.as_tensor(np.asarray(ts), dtype=torch.float64, device="cuda")
    log("ladder M=20808 complex128")
    w, Pt, U, P = _solve(mmf, torch, dp, tt, t0, mmf.MMF_C128)
    H = mmf.build_floquet(dp).T
    g = torch.Generator(device="cpu").manual_seed(1)
    idx = torch.randperm(M, generator=g)[:64].to("cuda")
    Phi = Pt[idx].T.contiguous()
    hn = torch.linalg.matrix_norm(H, ord=1).item()
    assert float((H @ Phi - Phi * w[idx][None, :]).abs().max()) / hn < 1e-12
    G = Pt.conj() @ Phi
    G[idx, torch.arange(64, device="cuda")] -= 1.0
    assert float(G.abs().max()) < 1e-12
    assert abs(float(w.sum()) - float(torch.diagonal(H).real.sum())) / hn < 1e-10
    assert float((P.sum(dim=0) - 1.0).abs().max()) < 1e-12
    assert bool((w[1:] >= w[:-1]).all())
    del H, G, Phi
    log("ladder M=20808 eigenvalue-only solver")
    wb, _ = mmf.eigvalsh_batched([mmf.build_floquet(dp)])
    torch.cuda.synchronize()
    assert float((wb[0] - w).abs().max()) <= 1e-12 * max(1.0, float(w.abs().max()))
    log("ladder M=20808 complex64 + FP64 refinement")
    w2, Pt2, U2, P2 = _solve(mmf, torch, dp, tt, t0, mmf.MMF_C64_REFINED)
    scale = max(1.0, float(w.abs().max()))
    assert float((w2 - w).abs().max()) <= 1e-9 * scale
    assert float((U2 - U).abs().max()) <= 1e-9
    assert float((P2 - P).abs().max()) <= 1e-9
