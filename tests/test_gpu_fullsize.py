"""Checks at the benchmark's full size (8-level ladder, two drives, M = 20808)
in the launch configuration bench.py times.

The oracle cannot diagonalise this matrix in test time, so the checks are the
properties that hold at any size, plus an independent algorithm on the GPU:
eigen-residual and orthogonality of sampled eigenvectors (1e-12), the trace
identity sum(eps) = tr H_F, column sums of the averaged probabilities
(1e-12), the eigenvalues against the eigenvalue-only solver (Householder +
Sturm bisection, 1e-12 normwise), and the refined mixed-precision path
against the FP64 path at the stated 1e-9 (quasienergies and U(t)).

Spot checks against the oracle at both full sizes (the ladder, M = 20808, and
the 16-level spectrum, M = 41616), with the oracle's routes that need no
full diagonalisation: sampled rows of H_F bitwise against the oracle's sparse
assembly; the quasienergies nearest three shifts against the oracle's
shift-invert solver (1e-10 normwise, and no GPU eigenvalue missing or extra in
between); 64 sampled eigenpairs' residuals against the oracle's H_F (1e-12 of
its 1-norm); U(t, t0) at two times against the oracle's sparse propagator
(1e-10).  The refined mixed-precision path (complex64 eigensolve + FP64
refinement) takes the same checks on the ladder at its stated 1e-9.
"""
import numpy as np
import pytest

import oracle
from workloads import cfg2_large, cfg4_precision
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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which,prec", [("ladder20808", "c128"), ("spec41616", "c128"),
                                        ("ladder20808", "c64_refined")])
def test_full_size_spot_checks_against_oracle(which, prec):
    """The refined mixed-precision case holds the same checks at its stated
    1e-9 (quasienergies normwise, U(t)) and 1e-12 residuals."""
    torch, mmf = require_gpu()
    refined = prec == "c64_refined"
    tol = 1e-9 if refined else 1e-10
    p, ts, t0 = cfg2_large() if which == "ladder20808" else cfg4_precision()
    dp = mmf.DeviceProblem(p)
    M = dp.M
    assert M == (20808 if which == "ladder20808" else 41616)
    log(f"{which}: oracle sparse H_F")
    Hs = oracle.build_floquet_sparse(p)
    rng = np.random.default_rng(17)
    HF = mmf.build_floquet(dp)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(M, 32, replace=False))
    got = HF[:, torch.as_tensor(rows, device="cuda")].T.cpu().numpy()      # rows of H_F
    assert np.array_equal(got, Hs[rows].toarray())
    log(f"{which}: GPU eigensolve ({prec})")
    w, Pt, info = mmf.eigh(HF, mmf.MMF_C64_REFINED if refined else mmf.MMF_C128)
    times = np.array([ts[1], ts[5]])
    U = mmf.evolve(dp, Pt, w, t0, torch.as_tensor(times, device="cuda"))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = w.cpu().numpy()
    scale = max(1.0, np.abs(w).max())
    hn = float(abs(Hs).sum(axis=0).max())
    cols = np.sort(rng.choice(M, 64, replace=False))
    Phi = Pt[torch.as_tensor(cols, device="cuda")].T.cpu().numpy()        # eigenvectors as columns
    res = np.abs(Hs @ Phi - Phi * w[cols][None, :]).max() / hn
    log(f"{which}: sampled residuals against the oracle's H_F {res:.2e}")
    assert res < 1e-12
    del Pt, HF
    for sigma in (-7.1, 3.3, 15.2):
        wo = oracle.quasienergies_near(Hs, sigma, 8)
        inside = w[(w >= wo[0] - 1e-9 * scale) & (w <= wo[-1] + 1e-9 * scale)]
        assert inside.shape[0] == 8, (sigma, inside, wo)
        err = np.abs(inside - wo).max() / scale
        log(f"{which}: quasienergies near {sigma}: {err:.2e} normwise")
        assert err < tol
    Uo = oracle.evolve_expm_sparse(p, Hs, t0, times)
    err_u = np.abs(U.cpu().numpy() - Uo).max()
    log(f"{which}: U(t) against the sparse propagator {err_u:.2e}")
    assert err_u < tol
