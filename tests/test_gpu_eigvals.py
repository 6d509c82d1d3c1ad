"""GPU parity of the eigenvalue-only batched solver (quasienergy scans).

mmf_eigvalsh_batched (grouped Householder reduction + FP64 Sturm bisection)
against the oracle's LAPACK eigenvalues: complex128 within 1e-10 normwise
(relative to max(1, max|eps|)); the complex64 reduction within 2e-5.  The
driven-lattice scan of Sec. 4.2 is checked at small size over a frequency
sweep and at the benchmark's size (D = 256, +-10, M = 5376) for one drive
frequency; the undriven lattice against its closed form.
"""
import numpy as np
import pytest

import oracle
from workloads import lattice_problem, gue
from gpu_util import require_gpu, to_dev_cm, log

pytestmark = pytest.mark.gpu

SIZES = [65, 1, 17, 0, 130, 2, 300, 64, 257, 33]


def _mats(torch, seed0):
    Hs = []
    for k, n in enumerate(SIZES):
        Hs.append(gue(np.random.default_rng(seed0 + k), n, 1.0) if n else np.zeros((0, 0), complex))
    mats = [to_dev_cm(torch, H) if H.size else torch.empty((0, 0), dtype=torch.complex128, device="cuda")
            for H in Hs]
    return Hs, mats


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 2e-5)], ids=["c128", "c64_raw"])
def test_eigvalsh_batched_random(prec, tol):
    torch, mmf = require_gpu()
    Hs, mats = _mats(torch, 300)
    log(f"eigvalsh batched prec={prec} sizes={SIZES}")
    ws, info = mmf.eigvalsh_batched(mats, prec)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(SIZES)
    worst = 0.0
    for H, w in zip(Hs, ws):
        if H.shape[0] == 0:
            continue
        wo = oracle.eigvalsh(H)
        wg = w.cpu().numpy()
        assert np.all(np.diff(wg) >= 0)
        err = np.abs(wg - wo).max() / max(1.0, np.abs(wo).max())
        worst = max(worst, err)
        assert err <= tol, (H.shape[0], err)
    log(f"  worst normwise error {worst:.2e}")


def test_eigvalsh_agrees_with_eigh():
    torch, mmf = require_gpu()
    H = gue(np.random.default_rng(11), 400, 1.0)
    ws, _ = mmf.eigvalsh_batched([to_dev_cm(torch, H)])
    w2, _, _ = mmf.eigh(to_dev_cm(torch, H))
    torch.cuda.synchronize()
    scale = max(1.0, float(w2.abs().max()))
    assert float((ws[0] - w2).abs().max()) <= 1e-12 * scale


def test_lattice_scan_small_against_oracle():
    torch, mmf = require_gpu()
    probs = [lattice_problem(float(w), D=32, N=4) for w in np.linspace(0.2, 1.0, 9)]
    log("lattice scan D=32 N=4, 9 frequencies")
    ws = mmf.quasienergy_scan(probs)
    torch.cuda.synchronize()
    for p, w in zip(probs, ws):
        qo = oracle.quasienergies(p)
        assert np.abs(w.cpu().numpy() - qo).max() <= 1e-10 * max(1.0, np.abs(qo).max())


def test_undriven_lattice_closed_form():
    torch, mmf = require_gpu()
    D, N, w = 128, 3, 0.45
    p = lattice_problem(w, D=D, V=0.0, N=N)
    j = np.arange(1, D // 2 + 1)
    r = np.sqrt(0.25 ** 2 + 4 * 0.125 ** 2 * np.cos(np.pi * j / (D + 1)) ** 2)
    st = np.concatenate([-r, r])
    expect = np.sort(np.concatenate([st + n * w for n in range(-N, N + 1)]))
    q = mmf.quasienergy_scan([p])[0].cpu().numpy()
    assert np.abs(q - expect).max() <= 1e-12 * max(1.0, np.abs(expect).max())


def test_lattice_full_size_one_frequency():
    """The scan's launch shape at the figure's size: D = 256, +-10, M = 5376."""
    torch, mmf = require_gpu()
    p = lattice_problem(0.6, D=256, N=10)
    log("lattice D=256 N=10 (M=5376) on the GPU")
    q = mmf.quasienergy_scan([p])[0].cpu().numpy()
    log("lattice D=256 N=10 oracle (CPU eigvalsh)")
    qo = oracle.quasienergies(p)
    assert q.shape == qo.shape == (5376,)
    assert np.abs(q - qo).max() <= 1e-10 * max(1.0, np.abs(qo).max())
