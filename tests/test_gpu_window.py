"""GPU parity of the partial-spectrum (quasienergy window) eigensolve.

mmf_eigh_window against the oracle's LAPACK eigenpairs: the count of
eigenvalues in [vl, vu) exactly, eigenvalues within 1e-10 normwise,
eigenvectors up to phase (|<phi_oracle, phi_gpu>| = 1 within 1e-10 on a
nondegenerate window) and residual ||A z - w z|| / ||A|| < 1e-12.  Cases:
random matrices (window inside the spectrum, truncated to kmax, empty), the
driven lattice's Brillouin-zone window (one state per orbit) at small size and
at the scan's size (M = 5376).
"""
import numpy as np
import pytest

import oracle
from workloads import lattice_problem, gue
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu


def _check(H, vl, vu, kmax, w, Zt, count, info):
    wo, Vo = oracle.eigh(H)
    sel = np.nonzero((wo >= vl) & (wo < vu))[0]
    assert int(info.item()) == 0
    assert int(count.item()) == len(sel)
    k = min(len(sel), kmax)
    wg = w.cpu().numpy()[:k]
    Z = Zt.cpu().numpy()[:k].T                      # columns = eigenvectors
    scale = max(1.0, np.abs(wo).max())
    assert np.abs(wg - wo[sel[:k]]).max(initial=0.0) <= 1e-10 * scale
    if k:
        ov = np.abs(np.sum(Vo[:, sel[:k]].conj() * Z, axis=0))
        assert np.abs(ov - 1.0).max() < 1e-10
        assert np.linalg.norm(H @ Z - Z * wg) / max(1.0, np.linalg.norm(H)) < 1e-12
    return k


@pytest.mark.parametrize("n,vl,vu,kmax", [(300, -0.5, 0.7, 300), (300, -0.5, 0.7, 10), (257, 50.0, 60.0, 5),
                                          (65, -100.0, 100.0, 65)])
def test_window_random(n, vl, vu, kmax):
    torch, mmf = require_gpu()
    H = gue(np.random.default_rng(40 + n), n, 1.0)
    log(f"window n={n} [{vl},{vu}) kmax={kmax}")
    out = mmf.eigh_window(to_dev_cm(torch, H), vl, vu, kmax)
    torch.cuda.synchronize()
    _check(H, vl, vu, kmax, *out)


def test_window_lattice_brillouin_zone_small():
    torch, mmf = require_gpu()
    p = lattice_problem(0.6, D=32, N=4)
    H = oracle.build_floquet(p)
    out = mmf.eigh_window(mmf.build_floquet(mmf.DeviceProblem(p)), -0.3, 0.3, 64)
    torch.cuda.synchronize()
    assert _check(H, -0.3, 0.3, 64, *out) == 32


def test_window_lattice_full_size():
    torch, mmf = require_gpu()
    p = lattice_problem(0.6, D=256, N=10)
    dp = mmf.DeviceProblem(p)
    log("window lattice D=256 N=10 (M=5376)")
    w, Zt, count, info = mmf.eigh_window(mmf.build_floquet(dp), -0.3, 0.3, 512)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and int(count.item()) == 256
    q = oracle.quasienergies(p)
    qo = q[(q >= -0.3) & (q < 0.3)]
    assert np.abs(w[:256].cpu().numpy() - qo).max() <= 1e-10 * max(1.0, np.abs(q).max())
    H = mmf.build_floquet(dp).T                        # logical H_F
    Z = Zt[:256].T
    r = torch.linalg.norm(H @ Z - Z * w[:256][None, :]) / torch.linalg.norm(H)
    G = Z.conj().T @ Z - torch.eye(256, dtype=Z.dtype, device=Z.device)
    assert float(r) < 1e-12 and float(G.abs().max()) < 1e-12
