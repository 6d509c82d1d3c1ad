"""GPU parity of the band-aware eigensolver (mmf_eigh_band) against the oracle.

A Hermitian matrix whose entries vanish below its b-th subdiagonal, b <= 64,
goes straight to the bulge chase: no dense -> band stage and no first
back-transformation (Q = Q2); orders up to 64 take the one-workgroup LDS
solver as in mmf_eigh.  Checks, as for the other eigensolvers:
eigenvalues within 1e-10 of the oracle's (relative to max(1, max|w|)),
residual and orthogonality 1e-12.  Cases: random banded matrices of widths
0 .. 64 at orders that cover a single entry, sweeps shorter than the band,
partial last chase blocks and several launch steps of the second
back-transformation; a width stated wider than the matrix; one-drive Floquet
matrices (half-width D h_max + D - 1); b > 64, which is the dense call bit for
bit.  At the full size of the one-drive workload (M = 20816, b = 47): the
oracle's shift-invert quasienergies near three shifts and 64 sampled
eigenpairs' residuals against its sparse H_F.
"""
import numpy as np
import pytest

import oracle
from workloads import one_drive_band, random_problem, tls_problem
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu


def _banded(n, b, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = (A + A.conj().T) / 2
    i, j = np.indices((n, n))
    A[np.abs(i - j) > b] = 0.0
    return A


def _check(H, b):
    torch, mmf = require_gpu()
    n = H.shape[0]
    w, Pt, info = mmf.eigh_band(to_dev_cm(torch, H), b)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = w.cpu().numpy()
    Phi = from_dev_cm(Pt)
    wo, _ = oracle.eigh(H)
    scale = max(1.0, np.abs(wo).max())
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wo).max() <= 1e-10 * scale
    hn = max(np.linalg.norm(H), 1.0)
    assert np.linalg.norm(H @ Phi - Phi * w[None, :]) / hn < 1e-12 * max(1.0, n / 100)
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-12 * max(1.0, n / 100)


@pytest.mark.parametrize("n,b", [(2, 1), (5, 10), (64, 3), (65, 0), (65, 1), (65, 64), (66, 60), (129, 64),
                                 (130, 17), (200, 64), (300, 1), (300, 40), (1100, 31), (1100, 64)])
def test_band_random(n, b):
    log(f"band eigh random n={n} b={b}")
    _check(_banded(n, b, 500 + n + b), b)


@pytest.mark.parametrize("name,mk", [
    ("tls", lambda: tls_problem(1.0, 0.7, 0.9, 40)),
    ("d4_two_harmonics", lambda: random_problem(4, (60,), seed=4, harmonics=[(0, 1), (0, 2)])),
    ("one_drive_small", lambda: one_drive_band(N=40)[0]),
])
def test_band_floquet(name, mk):
    torch, mmf = require_gpu()
    p = mk()
    b = mmf.floquet_half_bandwidth(p)
    H = oracle.build_floquet(p)
    log(f"band eigh floquet {name}: M={H.shape[0]} b={b}")
    assert b <= 64
    _check(H, b)


def test_band_wider_than_64_is_the_dense_call():
    torch, mmf = require_gpu()
    n = 300
    H = _banded(n, 100, 9)
    log("band eigh b=100 against mmf_eigh")
    w1, P1, i1 = mmf.eigh_band(to_dev_cm(torch, H), 100)
    w2, P2, i2 = mmf.eigh(to_dev_cm(torch, H))
    torch.cuda.synchronize()
    assert int(i1.item()) == 0 and int(i2.item()) == 0
    assert torch.equal(w1, w2) and torch.equal(P1, P2)


def test_band_argument_errors():
    torch, mmf = require_gpu()
    import ctypes as C
    L = mmf.lib()
    n = 8
    A = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = mmf.eigh_band_workspace_bytes(n, 3)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")

    def call(M=n, a=A, lda=n, b=3, ww=w, wk=work, nbytes=nb, inf=info):
        ptr = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
        return L.mmf_eigh_band(C.c_int64(M), ptr(a), C.c_int64(lda), C.c_int64(b), ptr(ww), ptr(wk),
                               C.c_size_t(nbytes), ptr(inf), None)
    assert call(M=-1) == -1
    assert call(a=None) == -2
    assert call(lda=n - 1) == -3
    assert call(b=-1) == -4
    assert call(ww=None) == -5
    assert call(wk=None) == -6
    assert call(nbytes=16) == -7
    assert call(inf=None) == -8
    assert call() == 0
    out = C.c_size_t(0)
    assert L.mmf_eigh_band_workspace(C.c_int64(-1), C.c_int64(3), C.byref(out)) == -1
    assert L.mmf_eigh_band_workspace(C.c_int64(n), C.c_int64(-1), C.byref(out)) == -2
    assert L.mmf_eigh_band_workspace(C.c_int64(n), C.c_int64(3), None) == -3
    torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_band_full_size_spot_checks_against_oracle():
    torch, mmf = require_gpu()
    p, ts, t0 = one_drive_band()
    dp = mmf.DeviceProblem(p)
    M = dp.M
    b = mmf.floquet_half_bandwidth(p)
    assert M == 20816 and b == 47
    log("one-drive band M=20816: oracle sparse H_F")
    Hs = oracle.build_floquet_sparse(p)
    log("one-drive band M=20816: GPU band eigensolve")
    w, Pt, info = mmf.eigh_band(mmf.build_floquet(dp), b)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = w.cpu().numpy()
    assert np.all(np.diff(w) >= 0)
    scale = max(1.0, np.abs(w).max())
    hn = float(abs(Hs).sum(axis=0).max())
    rng = np.random.default_rng(23)
    cols = np.sort(rng.choice(M, 64, replace=False))
    Phi = Pt[torch.as_tensor(cols, device="cuda")].T.cpu().numpy()
    res = np.abs(Hs @ Phi - Phi * w[cols][None, :]).max() / hn
    log(f"  sampled residuals against the oracle's H_F {res:.2e}")
    assert res < 1e-12
    G = Pt.conj() @ torch.as_tensor(Phi, device="cuda")
    G[torch.as_tensor(cols, device="cuda"), torch.arange(64, device="cuda")] -= 1.0
    assert float(G.abs().max()) < 1e-12
    del Pt, G
    for sigma in (-120.3, 2.7, 95.1):
        wo = oracle.quasienergies_near(Hs, sigma, 8)
        inside = w[(w >= wo[0] - 1e-9 * scale) & (w <= wo[-1] + 1e-9 * scale)]
        assert inside.shape[0] == 8, (sigma, inside, wo)
        err = np.abs(inside - wo).max() / scale
        log(f"  quasienergies near {sigma}: {err:.2e} normwise")
        assert err < 1e-10


# ------------------------------------------------------------ partial spectrum
def _check_window(H, vl, vu, kmax, w, Zt, count, info):
    wo, _ = oracle.eigh(H)
    sel = np.nonzero((wo >= vl) & (wo < vu))[0]
    assert int(info.item()) == 0
    assert int(count.item()) == len(sel)
    k = min(len(sel), kmax)
    wg = w.cpu().numpy()[:k]
    Z = Zt.cpu().numpy()[:k].T                      # columns = eigenvectors
    scale = max(1.0, np.abs(wo).max())
    assert np.abs(wg - wo[sel[:k]]).max(initial=0.0) <= 1e-10 * scale
    if k:
        assert np.linalg.norm(H @ Z - Z * wg) / max(1.0, np.linalg.norm(H)) < 1e-12
        assert np.abs(Z.conj().T @ Z - np.eye(k)).max() < 1e-12
    return k


@pytest.mark.parametrize("n,b,vl,vu,kmax", [(300, 17, -0.5, 0.7, 300), (300, 17, -0.5, 0.7, 10),
                                            (1100, 64, -1.0, 1.0, 1100), (129, 3, 50.0, 60.0, 5),
                                            (65, 0, -100.0, 100.0, 65), (200, 40, -3.0, 3.0, 0)])
def test_band_window_random(n, b, vl, vu, kmax):
    torch, mmf = require_gpu()
    H = _banded(n, b, 900 + n + b)
    At = to_dev_cm(torch, H)
    A0 = At.clone()
    log(f"band window n={n} b={b} [{vl},{vu}) kmax={kmax}")
    out = mmf.eigh_band_window(At, b, vl, vu, kmax)
    torch.cuda.synchronize()
    _check_window(H, vl, vu, kmax, *out)
    assert torch.equal(At, A0)                      # the band path only reads A


def test_band_window_floquet_states_match_the_full_band_solve():
    torch, mmf = require_gpu()
    p = one_drive_band(N=40)[0]
    b = mmf.floquet_half_bandwidth(p)
    dp = mmf.DeviceProblem(p)
    H = oracle.build_floquet(p)
    log(f"band window floquet: M={dp.M} b={b}")
    out = mmf.eigh_band_window(mmf.build_floquet(dp), b, -0.5, 0.5, 64)
    wf, _, info = mmf.eigh_band(mmf.build_floquet(dp), b)
    torch.cuda.synchronize()
    k = _check_window(H, -0.5, 0.5, 64, *out)
    assert k > 0 and int(info.item()) == 0
    sel = (wf >= -0.5) & (wf < 0.5)
    assert torch.equal(out[0][:k], wf[sel])          # the same tridiagonal and divide and conquer


def test_band_window_wider_than_64_is_the_dense_window():
    torch, mmf = require_gpu()
    H = _banded(300, 100, 19)
    log("band window b=100 against mmf_eigh_window")
    w1, Z1, c1, i1 = mmf.eigh_band_window(to_dev_cm(torch, H), 100, -2.0, 2.0, 300)
    w2, Z2, c2, i2 = mmf.eigh_window(to_dev_cm(torch, H), -2.0, 2.0, 300)
    torch.cuda.synchronize()
    assert int(i1.item()) == 0 and int(c1.item()) == int(c2.item())
    assert torch.equal(w1, w2) and torch.equal(Z1, Z2)


def test_band_window_argument_errors():
    torch, mmf = require_gpu()
    import ctypes as C
    L = mmf.lib()
    n, kmax = 80, 8
    A = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    w = torch.empty(kmax, dtype=torch.float64, device="cuda")
    Z = torch.empty((kmax, n), dtype=torch.complex128, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = C.c_size_t(0)
    assert L.mmf_eigh_band_window_workspace(C.c_int64(n), C.c_int64(3), C.c_int64(kmax), C.byref(nb)) == 0
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    ptr = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)

    def call(M=n, a=A, lda=n, b=3, vl=-1.0, vu=1.0, km=kmax, ww=w, zz=Z, ldz=n, c=cnt, wk=work,
             nbytes=nb.value, inf=info):
        return L.mmf_eigh_band_window(C.c_int64(M), ptr(a), C.c_int64(lda), C.c_int64(b), C.c_double(vl),
                                      C.c_double(vu), C.c_int64(km), ptr(ww), ptr(zz), C.c_int64(ldz), ptr(c),
                                      ptr(wk), C.c_size_t(nbytes), ptr(inf), None)
    assert call(M=-1) == -1
    assert call(a=None) == -2
    assert call(lda=n - 1) == -3
    assert call(b=-1) == -4
    assert call(vl=1.0, vu=1.0) == -5
    assert call(km=-1) == -7
    assert call(ww=None) == -8
    assert call(zz=None) == -9
    assert call(ldz=n - 1) == -10
    assert call(c=None) == -11
    assert call(wk=None) == -12
    assert call(nbytes=16) == -13
    assert call(inf=None) == -14
    assert call() == 0
    out = C.c_size_t(0)
    assert L.mmf_eigh_band_window_workspace(C.c_int64(-1), C.c_int64(3), C.c_int64(1), C.byref(out)) == -1
    assert L.mmf_eigh_band_window_workspace(C.c_int64(n), C.c_int64(-1), C.c_int64(1), C.byref(out)) == -2
    assert L.mmf_eigh_band_window_workspace(C.c_int64(n), C.c_int64(3), C.c_int64(-1), C.byref(out)) == -3
    assert L.mmf_eigh_band_window_workspace(C.c_int64(n), C.c_int64(3), C.c_int64(1), None) == -4
    torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_band_window_full_size_against_oracle():
    torch, mmf = require_gpu()
    p, ts, t0 = one_drive_band()
    dp = mmf.DeviceProblem(p)
    M = dp.M
    b = mmf.floquet_half_bandwidth(p)
    log("one-drive band window M=20816: oracle sparse H_F")
    Hs = oracle.build_floquet_sparse(p)
    log("one-drive band window M=20816: GPU window [-0.5, 0.5)")
    w, Zt, count, info = mmf.eigh_band_window(mmf.build_floquet(dp), b, -0.5, 0.5, 64)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = int(count.item())
    assert 0 < k <= 64
    w = w.cpu().numpy()[:k]
    Z = Zt.cpu().numpy()[:k].T
    hn = float(abs(Hs).sum(axis=0).max())
    res = np.abs(Hs @ Z - Z * w[None, :]).max() / hn
    log(f"  {k} states, residual against the oracle's H_F {res:.2e}")
    assert res < 1e-12
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() < 1e-12
    wo = oracle.quasienergies_near(Hs, 0.0, k + 8)
    wo = wo[(wo >= -0.5) & (wo < 0.5)]
    assert wo.shape[0] == k
    err = np.abs(w - wo).max() / max(1.0, np.abs(w).max())
    log(f"  quasienergies against the oracle's shift-invert solver {err:.2e}")
    assert err < 1e-10


def test_band_padded_leading_dimensions():
    """A and Z inside larger buffers (lda, ldz > M)."""
    torch, mmf = require_gpu()
    import ctypes as C
    n, b, pad = 150, 20, 9
    H = _banded(n, b, 77)
    buf = torch.zeros((n, n + pad), dtype=torch.complex128, device="cuda")
    buf[:, :n] = to_dev_cm(torch, H)
    log("band eigh padded ld")
    w, Pt, info = mmf.eigh_band(buf[:, :n], b)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Phi = from_dev_cm(Pt[:, :n])
    wo, _ = oracle.eigh(H)
    assert np.abs(w.cpu().numpy() - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
    assert np.linalg.norm(H @ Phi - Phi * w.cpu().numpy()) / np.linalg.norm(H) < 1e-12
    assert float(buf[:, n:].abs().max()) == 0.0                  # the padding is not written
    log("band window padded ld and ldz")
    A = torch.zeros((n, n + pad), dtype=torch.complex128, device="cuda")
    A[:, :n] = to_dev_cm(torch, H)
    kmax = 40
    wv = torch.zeros(kmax, dtype=torch.float64, device="cuda")
    Zb = torch.zeros((kmax, n + 5), dtype=torch.complex128, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    inf = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = C.c_size_t(0)
    mmf.call("mmf_eigh_band_window_workspace", C.c_int64(n), C.c_int64(b), C.c_int64(kmax), C.byref(nb))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    mmf.call("mmf_eigh_band_window", C.c_int64(n), C.c_void_p(A.data_ptr()), C.c_int64(n + pad), C.c_int64(b),
             C.c_double(-1.0), C.c_double(1.0), C.c_int64(kmax), C.c_void_p(wv.data_ptr()),
             C.c_void_p(Zb.data_ptr()), C.c_int64(n + 5), C.c_void_p(cnt.data_ptr()), C.c_void_p(work.data_ptr()),
             C.c_size_t(work.numel()), C.c_void_p(inf.data_ptr()), None)
    torch.cuda.synchronize()
    _check_window(H, -1.0, 1.0, kmax, wv, Zb[:, :n], cnt, inf)
    assert float(Zb[:, n:].abs().max()) == 0.0
