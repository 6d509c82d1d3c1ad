"""GPU parity of the two-stage eigensolver (dense -> band -> real tridiagonal
by bulge chasing, then the two back-transformations) against the oracle.

mmf_eigh takes this path from order MMF_EIGH_TWO_STAGE_MIN up (default 5888);
the tests lower the threshold to 0 so that small orders, which the oracle
solves in milliseconds, exercise every edge of the band reduction: partial
last panels, sweeps shorter than the bandwidth, single-element reflectors,
matrices that are already banded or diagonal, padded leading dimensions.
At n = 2100 the back-transformation by the chase reflectors has more column
tiles than workgroups, so each workgroup walks several (reading the next
tile's window ahead), also for a window of 650 eigenvectors.
Tolerances as for the one-stage solver: eigenvalues within 1e-10 of the
oracle (relative to max(1, max|w|)), residual and orthogonality 1e-12.
"""
import numpy as np
import pytest

import oracle
from workloads import Problem, cfg2_large, random_problem
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log
from test_gpu_parity import _check_eigh

pytestmark = pytest.mark.gpu


@pytest.fixture
def two_stage(monkeypatch):
    monkeypatch.setenv("MMF_EIGH_TWO_STAGE_MIN", "0")


def _herm(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return (A + A.conj().T) / 2


@pytest.mark.parametrize("n", [2, 3, 5, 63, 64, 65, 66, 127, 128, 129, 130, 193, 200, 257, 300, 513, 1100, 2100])
def test_two_stage_random_hermitian(two_stage, n):
    log(f"two-stage eigh random n={n}")
    _check_eigh(_herm(n, 2000 + n))


@pytest.mark.parametrize("name,mk", [
    ("ladder_small", lambda: cfg2_large(N=(4, 4))[0]),
    ("d4_f2", lambda: random_problem(4, (6, 5), seed=2)),
    ("diag_static", lambda: Problem(E=np.diag([0.3, -0.2, 1.1]).astype(complex), omega=[1.0], N=[40],
                                    axis=[0], harm=[1], V=[np.zeros((3, 3))])),
])
def test_two_stage_floquet(two_stage, name, mk):
    log(f"two-stage eigh floquet {name}")
    _check_eigh(mk())


def test_two_stage_block_diagonal(two_stage):
    """Two decoupled blocks: whole panels and sweeps meet columns that are
    already reduced (identity reflectors)."""
    n = 260
    H = np.zeros((n, n), complex)
    H[:130, :130] = _herm(130, 5)
    H[130:, 130:] = _herm(130, 6)
    log("two-stage block diagonal")
    _check_eigh(H)


def test_two_stage_padded_ld(two_stage):
    torch, mmf = require_gpu()
    n, pad = 150, 9
    H = _herm(n, 77)
    buf = torch.zeros((n, n + pad), dtype=torch.complex128, device="cuda")
    buf[:, :n] = to_dev_cm(torch, H)
    At = buf[:, :n]
    log("two-stage padded ld")
    w, Pt, info = mmf.eigh(At)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Phi = from_dev_cm(Pt)
    wo, _ = oracle.eigh(H)
    assert np.abs(w.cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
    assert np.linalg.norm(H @ Phi - Phi * w.cpu().numpy()) / np.linalg.norm(H) < 1e-12


def test_two_stage_matches_one_stage_spectrum():
    """Both reductions of the same matrix give the same eigenvalues (1e-12)."""
    torch, mmf = require_gpu()
    import os
    n = 700
    H = _herm(n, 31)
    out = []
    for thr in ("0", str(10 ** 9)):
        os.environ["MMF_EIGH_TWO_STAGE_MIN"] = thr
        try:
            w, Pt, info = mmf.eigh(to_dev_cm(torch, H))
            torch.cuda.synchronize()
            assert int(info.item()) == 0
            out.append(w.cpu().numpy())
        finally:
            del os.environ["MMF_EIGH_TWO_STAGE_MIN"]
    assert np.abs(out[0] - out[1]).max() <= 1e-12 * max(1.0, np.abs(out[1]).max())


@pytest.mark.parametrize("n,kmax", [(300, 40), (129, 200), (2100, 700)])
def test_two_stage_window(two_stage, n, kmax):
    torch, mmf = require_gpu()
    H = _herm(n, 900 + n)
    wo, Phio = oracle.eigh(H)
    nsel = 26 if n < 1000 else 650
    vl, vu = wo[n // 3] - 1e-9, wo[n // 3 + nsel - 1] + 1e-9
    log(f"two-stage window n={n}")
    w, Zt, count, info = mmf.eigh_window(to_dev_cm(torch, H), vl, vu, kmax)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = int(count.item())
    assert k == nsel
    kk = min(k, kmax)
    sel = wo[(wo >= vl) & (wo < vu)][:kk]
    assert np.abs(w.cpu().numpy()[:kk] - sel).max() <= 1e-10 * max(1.0, np.abs(wo).max())
    Z = Zt.cpu().numpy()[:kk].T
    assert np.linalg.norm(H @ Z - Z * w.cpu().numpy()[:kk]) / np.linalg.norm(H) < 1e-12
    assert np.abs(Z.conj().T @ Z - np.eye(kk)).max() < 1e-12


@pytest.mark.parametrize("thr", ["0", "200"], ids=["all_two_stage", "mixed"])
def test_two_stage_eigvalsh_batched(monkeypatch, thr):
    """Grouped two-stage reduction + Sturm bisection over mixed orders (with
    threshold 200 one call holds one-stage and two-stage problems)."""
    torch, mmf = require_gpu()
    monkeypatch.setenv("MMF_EIGH_TWO_STAGE_MIN", thr)
    sizes = [65, 1, 0, 130, 2, 300, 64, 513, 3, 257]
    Hs = [_herm(n, 4000 + n) if n else np.zeros((0, 0), complex) for n in sizes]
    mats = [to_dev_cm(torch, H) if n else torch.empty((0, 0), dtype=torch.complex128, device="cuda")
            for H, n in zip(Hs, sizes)]
    log(f"two-stage eigvalsh batched threshold {thr}")
    ws, info = mmf.eigvalsh_batched(mats, 0)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(sizes)
    for H, w in zip(Hs, ws):
        if H.shape[0] == 0:
            continue
        wo, _ = oracle.eigh(H)
        wg = w.cpu().numpy()
        assert np.all(np.diff(wg) >= 0)
        assert np.abs(wg - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max()), H.shape[0]
