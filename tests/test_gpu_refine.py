"""GPU checks of the refinement's cluster handling and of the iteration-limit
reports.

* a 40-fold exactly degenerate level (a static Floquet problem: diagonal H_F,
  complex64 eigenvectors exact unit vectors, every gap inside the level 0)
  must give finite eigenpairs, info 0 and the oracle's quasienergies and U(t);
* a near-degenerate run of 40 and of 100 eigenvalues (spread 4e-9 and 1e-8,
  longer than one Rayleigh-Ritz chunk for the second) must give finite output,
  and the reported status must be honest: info 0 only with eigenvalues within
  1e-9 of the oracle, residual and orthogonality at the FP64 level;
* limits forced from the host (mmf_eigh_ex: one refinement iteration, one
  secular step, one QL step) must set dev_info to MMF_ERR_NO_CONVERGENCE while
  every kernel still ends normally.
"""
import numpy as np
import pytest

import oracle
from workloads import Problem, gue
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu


def _near_run(n, run, spread, seed):
    rng = np.random.default_rng(seed)
    d = np.concatenate([0.5 + spread * np.arange(run) / run, rng.uniform(-3.0, 3.0, n - run)])
    U, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    H = (U * d) @ U.conj().T
    return (H + H.conj().T) / 2


def _solve(H, prec, limits=None):
    torch, mmf = require_gpu()
    At = to_dev_cm(torch, H)
    w, Pt, info = mmf.eigh(At, prec=prec, limits=limits)
    torch.cuda.synchronize()
    return w.cpu().numpy(), from_dev_cm(Pt), int(info.item())


def test_refined_degenerate_level_of_40():
    torch, mmf = require_gpu()
    D = 44
    E = np.diag(np.concatenate([np.full(40, 0.5), [-1.0, 0.1, 1.7, 2.2]])).astype(np.complex128)
    p = Problem(E=E, omega=[1.3], N=[1], axis=[0], harm=[1], V=[np.zeros((D, D))])
    ts = np.linspace(0.0, 5.0, 7)
    log("refined: 40-fold degenerate level, M=132")
    out = mmf.solve(p, ts, 0.0, prec=mmf.MMF_C64_REFINED)
    torch.cuda.synchronize()
    w = out["w"].cpu().numpy()
    U = out["U"].cpu().numpy()
    assert np.isfinite(w).all() and np.isfinite(U).all()
    assert int(out["info"].item()) == 0
    H = oracle.build_floquet(p)
    wo, Phio = oracle.eigh(H)
    assert np.abs(w - wo).max() <= 1e-12 * max(1.0, np.abs(wo).max())
    assert np.abs(U - oracle.evolve(p, Phio, wo, 0.0, ts)).max() < 1e-9
    # the averaged probabilities are basis dependent here, and the status says so
    assert int(out["P_status"].item()) == mmf.MMF_ERR_DEGENERATE


@pytest.mark.parametrize("run,spread", [(40, 4e-9), (100, 1e-8)])
def test_refined_near_degenerate_run(run, spread):
    torch, mmf = require_gpu()
    n = 240
    H = _near_run(n, run, spread, seed=run)
    log(f"refined: near-degenerate run of {run}, n={n}")
    w, Phi, info = _solve(H, mmf.MMF_C64_REFINED)
    assert np.isfinite(w).all() and np.isfinite(Phi).all()
    wo, Po = oracle.eigh(H)
    scale = max(1.0, np.abs(wo).max())
    err = np.abs(w - wo).max() / scale
    res = np.linalg.norm(H @ Phi - Phi * w) / np.linalg.norm(H)
    orth = np.abs(Phi.conj().T @ Phi - np.eye(n)).max()
    log(f"  info {info}: eig err {err:.2e}, residual {res:.2e}, orthogonality {orth:.2e}")
    if run <= 64:
        assert info == 0
    if info == 0:
        assert err <= 1e-9 and res < 1e-12 and orth < 1e-12
        # the run's invariant subspace (gauge invariant) against the oracle
        sel = slice(int(np.searchsorted(wo, 0.5 - 1e-7)), int(np.searchsorted(wo, 0.5 + spread + 1e-7)))
        assert sel.stop - sel.start == run
        Pg = Phi[:, sel] @ Phi[:, sel].conj().T
        Pr = Po[:, sel] @ Po[:, sel].conj().T
        assert np.abs(Pg - Pr).max() < 1e-9
    else:
        assert info == mmf.MMF_ERR_NO_CONVERGENCE


def test_refinement_limit_reports_no_convergence():
    torch, mmf = require_gpu()
    H = _near_run(150, 8, 1e-6, seed=3)
    w, Phi, info = _solve(H, mmf.MMF_C64_REFINED, limits={"refine_max_iters": 1})
    assert info == mmf.MMF_ERR_NO_CONVERGENCE
    assert np.isfinite(w).all() and np.isfinite(Phi).all()
    # the default budget converges on the same input
    w, Phi, info = _solve(H, mmf.MMF_C64_REFINED)
    assert info == 0


@pytest.mark.parametrize("lim", [{"secular_max_iters": 1}, {"leaf_max_iters": 1}])
def test_divide_and_conquer_limits_report_no_convergence(lim):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(11)
    H = gue(rng, 300, 1.0)
    w, Phi, info = _solve(H, mmf.MMF_C128, limits=lim)
    log(f"c128 with {lim}: info {info}")
    assert info == mmf.MMF_ERR_NO_CONVERGENCE
    w, Phi, info = _solve(H, mmf.MMF_C128, limits={})
    assert info == 0
    wo, _ = oracle.eigh(H)
    assert np.abs(w - wo).max() < 1e-12 * max(1.0, np.abs(wo).max())


def test_eigh_ex_argument_errors():
    torch, mmf = require_gpu()
    import ctypes as C
    L = mmf.lib()
    n = 8
    A = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = torch.empty(mmf.eigh_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    bad = mmf.MMFEighOpts(refine_max_iters=65)
    ok = mmf.MMFEighOpts()

    def call(opts, nbytes=None, inf=info):
        return L.mmf_eigh_ex(C.c_int64(n), C.c_void_p(A.data_ptr()), C.c_int64(n), C.c_void_p(w.data_ptr()), 0,
                             C.byref(opts) if opts is not None else None, C.c_void_p(work.data_ptr()),
                             C.c_size_t(work.numel() if nbytes is None else nbytes),
                             C.c_void_p(inf.data_ptr()) if inf is not None else None, None)
    assert call(bad) == -6
    assert call(ok, nbytes=16) == -8
    assert call(ok, inf=None) == -9
    assert call(None) == 0 and call(ok) == 0
