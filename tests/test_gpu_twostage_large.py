"""The default (two-stage) eigensolve against the oracle above the order from
which a step of the second back-transformation needs more than one launch
(more than 64 active blocks of 64 sweeps: n > 8194): the 8-level ladder of the
benchmark at truncation +-16, M = 8712.

The oracle's full eigendecomposition of this matrix takes minutes on the host,
so the comparison uses the oracle's cheaper routes to the same quantities:
every quasienergy against LAPACK's eigenvalue-only solver (1e-10 normwise),
U(t, t0) at three times against the sparse action of exp(-i H_F t) on the zero
Fourier block (no eigendecomposition at all, 1e-10), and the averaged
probabilities against the oracle's table stored by
tests/golden/make_ladder8712_pbar.py (1e-10; the oracle found no
near-degenerate quasienergies sharing weight, so the table is unique), plus
the identities that hold for any orthonormal eigenvector set (column sums 1
to 1e-12, entries in [0, 1]).
"""
import os

import numpy as np
import pytest

import oracle
from workloads import cfg2_large
from gpu_util import require_gpu, log

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_two_stage_ladder_8712_against_oracle():
    torch, mmf = require_gpu()
    p, ts, t0 = cfg2_large(N=(16, 16))
    dp = mmf.DeviceProblem(p)
    M = dp.M
    assert M == 8712 and M >= mmf.eigh_two_stage_min()
    times = np.array([0.0, ts[37], ts[128]])
    log(f"two-stage ladder M={M}: GPU solve")
    out = mmf.solve(p, times, t0)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 0
    w = out["w"].cpu().numpy()
    U = out["U"].cpu().numpy()
    P = out["P"].cpu().numpy()
    H = oracle.build_floquet(p)
    log("  oracle eigenvalues (LAPACK eigvalsh)")
    wo = oracle.eigvalsh(H)
    scale = max(1.0, np.abs(wo).max())
    err_w = np.abs(w - wo).max() / scale
    log(f"  quasienergies: {err_w:.2e} normwise")
    assert err_w < 1e-10
    log("  oracle U(t) (sparse propagator)")
    Uo = oracle.evolve_expm_sparse(p, H, t0, times)
    err_u = np.abs(U - Uo).max()
    log(f"  U(t): {err_u:.2e}")
    assert err_u < 1e-10
    assert np.abs(P.sum(axis=0) - 1.0).max() < 1e-12
    assert P.min() >= -1e-14 and P.max() <= 1.0 + 1e-12
    golden = os.path.join(os.path.dirname(__file__), "golden", "ladder8712_pbar.txt")
    with open(golden) as f:
        assert "degenerate_clusters_share_weight 0" in f.read()
    Po = np.loadtxt(golden)
    assert int(out["P_status"].item()) == 0
    err_p = np.abs(P - Po).max()
    log(f"  P against the stored oracle table: {err_p:.2e}")
    assert err_p < 1e-10
