"""GPU parity of every C-ABI entry point against the CPU oracle.

Inputs are seeded and synthetic; the oracle runs on the host with the same
inputs.  Tolerances: assembly is bit-exact (copies plus one FP64 add chain
per diagonal element, done in the same order on both sides); eigenvalues
within 1e-10 relative to max(1, max|eps|); U(t,t0) and the averaged
probabilities within 1e-10 of the oracle on converged inputs (gauge-free
quantities, eigenvector phases are never compared).
"""
import math
import numpy as np
import pytest

import oracle
from workloads import Problem, random_problem, cfg1_tls, cfg2_large, tls_problem, gue
from gpu_util import require_gpu, to_dev_cm, from_dev_cm, log

pytestmark = pytest.mark.gpu

ASSEMBLY_CASES = [
    ("tls", lambda: cfg1_tls()[0]),
    ("d3_f2", lambda: random_problem(3, (2, 3), seed=5, harmonics=[(0, 1), (1, 1), (0, 2), (1, 3)])),
    ("dup_axis_h", lambda: random_problem(2, (3,), seed=6, harmonics=[(0, 1), (0, 1), (0, 2)])),
    ("beyond_box", lambda: random_problem(2, (1,), seed=3, harmonics=[(0, 1), (0, 3)])),
    ("f3", lambda: random_problem(2, (2, 1, 2), seed=8)),
    # four fundamentals, one truncated at N = 0 (a one-site axis the column
    # walk always carries through), D = 3 so column blocks start mid-site
    ("f4_zero_axis", lambda: random_problem(3, (1, 0, 2, 1), seed=10)),
    ("static_f0", lambda: Problem(E=gue(np.random.default_rng(1), 4, 1.0), omega=[], N=[], axis=[],
                                  harm=[], V=np.zeros((0, 4, 4)))),
    ("d16", lambda: random_problem(16, (2, 2), seed=9)),
]


@pytest.mark.parametrize("name,mk", ASSEMBLY_CASES, ids=[c[0] for c in ASSEMBLY_CASES])
def test_build_floquet_bitwise(name, mk):
    torch, mmf = require_gpu()
    p = mk()
    log(f"assembly {name}")
    dp = mmf.DeviceProblem(p)
    HFt = mmf.build_floquet(dp)
    torch.cuda.synchronize()
    H = oracle.build_floquet(p)
    assert dp.M == H.shape[0]
    got = from_dev_cm(HFt)
    assert np.array_equal(got, H), f"max diff {np.abs(got - H).max()}"


def test_build_floquet_padded_ld():
    torch, mmf = require_gpu()
    p = random_problem(3, (2, 1), seed=2)
    dp = mmf.DeviceProblem(p)
    M = dp.M
    buf = torch.full((M, M + 7), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    mmf.build_floquet(dp, out=buf)
    torch.cuda.synchronize()
    H = oracle.build_floquet(p)
    assert np.array_equal(buf[:, :M].T.cpu().numpy(), H)
    assert torch.all(buf[:, M:] == complex(7.0, 7.0))


def _oracle_solve(p):
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    return H, w, Phi


@pytest.mark.parametrize("mk", [lambda: cfg1_tls()[0], lambda: random_problem(3, (3, 2), seed=4),
                                lambda: random_problem(5, (4,), seed=12)])
def test_avg_prob_on_oracle_eigenvectors(mk):
    torch, mmf = require_gpu()
    p = mk()
    H, w, Phi = _oracle_solve(p)
    dp = mmf.DeviceProblem(p)
    P, st = mmf.avg_prob(dp, to_dev_cm(torch, Phi), torch.as_tensor(w, device="cuda"))
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and not oracle.avg_prob_degenerate(p, Phi, w)
    np.testing.assert_allclose(P.cpu().numpy(), oracle.avg_prob(p, Phi), rtol=0, atol=1e-13)


def _rot(Phi, a, b, theta=0.6):
    R = Phi.copy()
    c, s = math.cos(theta), math.sin(theta)
    R[:, a] = c * Phi[:, a] + s * Phi[:, b]
    R[:, b] = -s * Phi[:, a] + c * Phi[:, b]
    return R


@pytest.mark.parametrize("case", ["same_site", "same_site_rotated", "cross_site", "cross_site_rotated"])
def test_avg_prob_degenerate_flag_matches_oracle(case):
    """The device status of mmf_avg_prob against the oracle's degeneracy rule
    on static problems with exactly degenerate quasienergies, in the pure
    eigenbasis and with a degenerate pair mixed; P itself matches the oracle
    on the same (flagged or not) eigenvectors."""
    torch, mmf = require_gpu()
    if case.startswith("same_site"):
        p = Problem(E=np.diag([0.3, 0.3, -0.5]).astype(np.complex128), omega=[1.1], N=[2], axis=[0], harm=[1],
                    V=[np.zeros((3, 3))])
    else:
        p = Problem(E=np.diag([0.0, 1.0]).astype(np.complex128), omega=[1.0], N=[3], axis=[0], harm=[1],
                    V=[np.zeros((2, 2))])
    H, w, Phi = _oracle_solve(p)
    if case.endswith("rotated"):
        D, s0 = p.D, oracle.zero_site(p.N)
        row = np.argmax(np.abs(Phi) ** 2, axis=0)
        # a degenerate pair whose second member sits on the zero site
        b = int(np.nonzero(row == D * s0 + (0 if case.startswith("same") else 1))[0][0])
        a = [k for k in range(len(w)) if k != b and abs(w[k] - w[b]) < 1e-12][0]
        Phi = _rot(Phi, a, b)
    expect = oracle.avg_prob_degenerate(p, Phi, w)
    assert expect == (case != "cross_site")
    dp = mmf.DeviceProblem(p)
    P, st = mmf.avg_prob(dp, to_dev_cm(torch, Phi), torch.as_tensor(w, device="cuda"))
    torch.cuda.synchronize()
    log(f"avg_prob degeneracy {case}: status {int(st.item())}")
    assert int(st.item()) == (mmf.MMF_ERR_DEGENERATE if expect else 0)
    np.testing.assert_allclose(P.cpu().numpy(), oracle.avg_prob(p, Phi), rtol=0, atol=1e-13)


@pytest.mark.parametrize("mk", [lambda: cfg1_tls()[0], lambda: random_problem(3, (3, 2), seed=4),
                                lambda: random_problem(2, (5, 1, 1), seed=7)])
def test_evolve_on_oracle_eigenvectors(mk):
    torch, mmf = require_gpu()
    p = mk()
    H, w, Phi = _oracle_solve(p)
    dp = mmf.DeviceProblem(p)
    ts = np.linspace(-3.0, 40.0, 37)
    t0 = 0.7
    U = mmf.evolve(dp, to_dev_cm(torch, Phi), torch.from_numpy(w).cuda(), t0, torch.from_numpy(ts).cuda())
    torch.cuda.synchronize()
    Uo = oracle.evolve(p, Phi, w, t0, ts)
    assert np.abs(U.cpu().numpy() - Uo).max() < 1e-11


def test_micromotion_on_oracle_eigenvectors():
    torch, mmf = require_gpu()
    p = cfg1_tls()[0]
    H, w, Phi = _oracle_solve(p)
    dp = mmf.DeviceProblem(p)
    ts = np.array([0.0, 1.3, 7.7])
    UF, eps, sel, info = mmf.micromotion(dp, to_dev_cm(torch, Phi), torch.from_numpy(w).cuda(),
                                         torch.from_numpy(ts).cuda())
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    UFo, epso = oracle.micromotion(p, Phi, w, ts)
    assert list(sel.cpu().numpy()) == list(oracle.micromotion_select(p, Phi, w))
    np.testing.assert_allclose(eps.cpu().numpy(), epso, rtol=0, atol=0)
    assert np.abs(UF.cpu().numpy() - UFo).max() < 1e-12


# --------------------------------------------------------------- eigensolver stages
STEDC_SIZES = [1, 2, 3, 17, 64, 65, 100, 129, 257, 600]


@pytest.mark.parametrize("n", STEDC_SIZES)
def test_stedc_random(n):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(100 + n)
    d = rng.normal(size=n)
    e = rng.normal(size=max(n - 1, 0))
    log(f"stedc random n={n}")
    wg, Zt, info = mmf.stedc(torch.from_numpy(d.copy()).cuda(),
                             torch.from_numpy(e if n > 1 else np.zeros(1)).cuda())
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = wg.cpu().numpy()
    Z = from_dev_cm(Zt)
    wo, _ = oracle.tridiag_eigh(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    nrm = max(1.0, np.abs(wo).max())
    assert np.abs(w - wo).max() <= 1e-12 * nrm * max(1, math.log2(n + 1))
    assert np.abs(T @ Z - Z * w).max() <= 1e-12 * nrm * max(1, math.log2(n + 1))
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-12 * max(1, math.log2(n + 1))


@pytest.mark.parametrize("kind", ["glued", "constant", "wilkinson", "zero_offdiag", "floquet", "glued_2000",
                                  "mixed_2000"])
def test_stedc_structured(kind):
    """Deflation-heavy tridiagonals: clusters, exact degeneracy, split matrix;
    at n = 2000 the merges' deflation scans and gathers span many 64-entry and
    256-column chunks."""
    torch, mmf = require_gpu()
    n = 2000 if kind.endswith("_2000") else 300
    if kind == "mixed_2000":
        # half the spectrum in tight clusters, half spread: both deflation kinds
        rng = np.random.default_rng(11)
        d = np.where(np.arange(n) % 2 == 0, np.round(rng.normal(size=n), 1), rng.normal(size=n))
        e = np.where(np.arange(n - 1) % 3 == 0, 1e-10, rng.normal(size=n - 1))
    elif kind.startswith("glued"):
        d = np.ones(n); e = np.full(n - 1, 1e-9)
    elif kind == "constant":
        d = np.full(n, 2.0); e = np.full(n - 1, -1.0)
    elif kind == "wilkinson":
        d = np.abs(np.arange(n) - (n - 1) / 2.0); e = np.ones(n - 1)
    elif kind == "zero_offdiag":
        rng = np.random.default_rng(3); d = rng.normal(size=n); e = rng.normal(size=n - 1); e[::7] = 0.0
    else:
        p = random_problem(3, (10, 4), seed=1)
        H = oracle.build_floquet(p)
        import scipy.linalg as sl
        Tm = sl.hessenberg(H)
        n = H.shape[0]
        d = np.real(np.diag(Tm)).copy(); e = np.abs(np.diag(Tm, -1)).copy()
    log(f"stedc {kind} n={n}")
    wg, Zt, info = mmf.stedc(torch.from_numpy(d.copy()).cuda(), torch.from_numpy(e.copy()).cuda())
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = wg.cpu().numpy(); Z = from_dev_cm(Zt)
    wo, _ = oracle.tridiag_eigh(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    nrm = max(1.0, np.abs(wo).max())
    assert np.abs(w - wo).max() <= 1e-12 * nrm
    assert np.abs(T @ Z - Z * w).max() <= 1e-11 * nrm
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-11


@pytest.mark.parametrize("n", [1, 2, 3, 31, 33, 64, 65, 100, 257])
def test_hetrd_defining_identity(n):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = A + A.conj().T
    log(f"hetrd n={n}")
    At = to_dev_cm(torch, A)
    d, e, tau = mmf.hetrd(At)
    torch.cuda.synchronize()
    V = from_dev_cm(At)
    refl = np.zeros((n, n), complex)
    for i in range(n - 1):
        refl[i + 1, i] = 1.0
        refl[i + 2:, i] = V[i + 2:, i]
        assert V[i + 1, i] == 1.0
    Q, T = oracle.householder_tridiag_apply(d.cpu().numpy(), e.cpu().numpy()[:n - 1], refl,
                                            tau.cpu().numpy()[:n - 1])
    scale = np.abs(A).max()
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-13 * max(1, n / 10)
    assert np.abs(Q @ T @ Q.conj().T - A).max() < 1e-13 * scale * max(1, n / 10)


@pytest.mark.parametrize("n", [2, 5, 64, 65, 129, 130, 200, 257, 300])
def test_unmtr_against_oracle_reflectors(n):
    torch, mmf = require_gpu()
    rng = np.random.default_rng(7 + n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = A + A.conj().T
    At = to_dev_cm(torch, A)
    d, e, tau = mmf.hetrd(At)
    Vt = At.clone()
    Zt = torch.from_numpy(np.ascontiguousarray(np.linalg.qr(rng.normal(size=(n, n)))[0].T)).cuda()
    Phi_t = mmf.unmtr(Vt, tau, Zt)
    torch.cuda.synchronize()
    V = from_dev_cm(Vt)
    refl = np.zeros((n, n), complex)
    for i in range(n - 1):
        refl[i + 1, i] = 1.0
        refl[i + 2:, i] = V[i + 2:, i]
    Q, _ = oracle.householder_tridiag_apply(d.cpu().numpy(), e.cpu().numpy()[:n - 1], refl,
                                            tau.cpu().numpy()[:n - 1])
    expect = Q @ from_dev_cm(Zt)
    assert np.abs(from_dev_cm(Phi_t) - expect).max() < 1e-13 * max(1, n / 10)


# --------------------------------------------------------------- full eigensolve
def _check_eigh(p_or_H, tol_eps=1e-10):
    torch, mmf = require_gpu()
    H = p_or_H if isinstance(p_or_H, np.ndarray) else oracle.build_floquet(p_or_H)
    n = H.shape[0]
    At = to_dev_cm(torch, H)
    w, Pt, info = mmf.eigh(At)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = w.cpu().numpy()
    Phi = from_dev_cm(Pt)
    wo, _ = oracle.eigh(H)
    scale = max(1.0, np.abs(wo).max())
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wo).max() <= tol_eps * scale
    assert np.linalg.norm(H @ Phi - Phi * w) / max(1.0, np.linalg.norm(H)) < 1e-12
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-12
    return w, Phi


@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 64, 65, 97, 200, 513])
def test_eigh_random_hermitian(n):
    rng = np.random.default_rng(1000 + n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    log(f"eigh random n={n}")
    _check_eigh((A + A.conj().T) / 2)


@pytest.mark.parametrize("name,mk", [
    ("tls_cfg", lambda: cfg1_tls()[0]),
    ("ladder_small", lambda: cfg2_large(N=(4, 4))[0]),
    ("d4_f2", lambda: random_problem(4, (6, 5), seed=2)),
    ("diag_static", lambda: Problem(E=np.diag([0.3, -0.2, 1.1]).astype(complex), omega=[1.0], N=[30],
                                    axis=[0], harm=[1], V=[np.zeros((3, 3))])),
])
def test_eigh_floquet(name, mk):
    log(f"eigh floquet {name}")
    _check_eigh(mk())


def test_full_pipeline_cfg1_against_oracle():
    """assemble -> eigh -> U(100 times) -> P on the GPU vs the oracle (1e-10)."""
    torch, mmf = require_gpu()
    p, ts, t0 = cfg1_tls()
    out = mmf.solve(p, ts, t0)
    torch.cuda.synchronize()
    H, wo, Phio = _oracle_solve(p)
    w = out["w"].cpu().numpy()
    assert np.abs(w - wo).max() <= 1e-10 * max(1.0, np.abs(wo).max())
    Uo = oracle.evolve(p, Phio, wo, t0, ts)
    U = out["U"].cpu().numpy()
    assert np.abs(U - Uo).max() < 1e-10
    dev = max(np.abs(U[q].conj().T @ U[q] - np.eye(2)).max() for q in range(len(ts)))
    assert dev < 1e-10
    P = out["P"].cpu().numpy()
    assert np.abs(P - oracle.avg_prob(p, Phio)).max() < 1e-10
    np.testing.assert_allclose(P.sum(axis=0), 1.0, atol=1e-12)


def test_deterministic_repeat():
    """Same input twice gives bitwise-equal eigenpairs, U and P."""
    torch, mmf = require_gpu()
    p = random_problem(3, (5, 3), seed=31)
    ts = np.linspace(0, 10, 9)
    a = mmf.solve(p, ts, 0.0)
    b = mmf.solve(p, ts, 0.0)
    torch.cuda.synchronize()
    for k in ("w", "Pt", "U", "P"):
        assert torch.equal(a[k], b[k]), k


def test_argument_errors():
    torch, mmf = require_gpu()
    import ctypes as C
    L = mmf.lib()
    M = C.c_int64(0)
    assert L.mmf_floquet_dim(None, C.byref(M)) == -1
    p = cfg1_tls()[0]
    dp = mmf.DeviceProblem(p)
    buf = torch.empty((dp.M, dp.M), dtype=torch.complex128, device="cuda")
    ev = C.c_void_p(dp.ev_work.data_ptr())
    evn = C.c_size_t(dp.ev_work.numel())
    assert L.mmf_build_floquet(dp.ref, C.c_void_p(buf.data_ptr()), C.c_int64(dp.M - 1), ev, evn, None) == -3
    assert L.mmf_build_floquet(dp.ref, None, C.c_int64(dp.M), ev, evn, None) == -2
    assert L.mmf_build_floquet(dp.ref, C.c_void_p(buf.data_ptr()), C.c_int64(dp.M), None, evn, None) == -4
    assert L.mmf_build_floquet(dp.ref, C.c_void_p(buf.data_ptr()), C.c_int64(dp.M), ev, C.c_size_t(16),
                               None) == -5
    w = torch.empty(dp.M, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert L.mmf_eigh(C.c_int64(dp.M), C.c_void_p(buf.data_ptr()), C.c_int64(dp.M), C.c_void_p(w.data_ptr()),
                      0, C.c_void_p(small.data_ptr()), C.c_size_t(16), C.c_void_p(info.data_ptr()), None) == -7
    assert L.mmf_eigh(C.c_int64(dp.M), C.c_void_p(buf.data_ptr()), C.c_int64(dp.M), C.c_void_p(w.data_ptr()),
                      9, C.c_void_p(small.data_ptr()), C.c_size_t(16), C.c_void_p(info.data_ptr()), None) == -5


# --------------------------------------------------------------- precision layer
def _eigh_prec(H, prec):
    torch, mmf = require_gpu()
    At = to_dev_cm(torch, H)
    w, Pt, info = mmf.eigh(At, prec=prec)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    return w.cpu().numpy(), from_dev_cm(Pt)


@pytest.mark.parametrize("n", [5, 64, 129, 400])
def test_eigh_c64_raw_is_single_precision(n):
    """Unrefined complex64 path: error reported, only sanity-bounded."""
    torch, mmf = require_gpu()
    rng = np.random.default_rng(2000 + n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = (A + A.conj().T) / 2
    w, Phi = _eigh_prec(H, mmf.MMF_C64_RAW)
    wo, _ = oracle.eigh(H)
    err = np.abs(w - wo).max() / max(1.0, np.abs(wo).max())
    log(f"c64 raw n={n}: eigenvalue error {err:.2e}")
    assert err < 1e-4
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-3


@pytest.mark.parametrize("n", [1, 2, 5, 64, 129, 400])
def test_eigh_c64_refined_random(n):
    """Refined mixed path: eigenvalues within 1e-9, eigenpairs at FP64 level."""
    torch, mmf = require_gpu()
    rng = np.random.default_rng(3000 + n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = (A + A.conj().T) / 2
    w, Phi = _eigh_prec(H, mmf.MMF_C64_REFINED)
    wo, _ = oracle.eigh(H)
    scale = max(1.0, np.abs(wo).max())
    log(f"c64 refined n={n}: eig err {np.abs(w - wo).max() / scale:.2e}")
    assert np.abs(w - wo).max() <= 1e-9 * scale
    assert np.linalg.norm(H @ Phi - Phi * w) / max(1.0, np.linalg.norm(H)) < 1e-11
    assert np.abs(Phi.conj().T @ Phi - np.eye(n)).max() < 1e-11


@pytest.mark.parametrize("name,mk", [
    ("tls_cfg", lambda: cfg1_tls()),
    ("ladder_small", lambda: cfg2_large(N=(5, 5))),
])
def test_refined_pipeline_against_oracle(name, mk):
    """Precision-layer solve: eigenvalues, U(t,t0) and P within 1e-9 of the FP64 oracle."""
    torch, mmf = require_gpu()
    p, ts, t0 = mk()
    ts = ts[:40]
    out = mmf.solve(p, ts, t0, prec=mmf.MMF_C64_REFINED)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 0
    H, wo, Phio = _oracle_solve(p)
    w = out["w"].cpu().numpy()
    ew = np.abs(w - wo).max() / max(1.0, np.abs(wo).max())
    Uo = oracle.evolve(p, Phio, wo, t0, ts)
    eu = np.abs(out["U"].cpu().numpy() - Uo).max()
    ep = np.abs(out["P"].cpu().numpy() - oracle.avg_prob(p, Phio)).max()
    log(f"refined pipeline {name}: eps {ew:.2e} U {eu:.2e} P {ep:.2e}")
    assert ew <= 1e-9 and eu <= 1e-9 and ep <= 1e-9


def test_refined_ladder_medium_against_oracle():
    """Refined mixed path on a 3528-dimensional two-drive ladder (dense
    quasienergy spectrum with close pairs): eigenvalues and U within 1e-9."""
    torch, mmf = require_gpu()
    p, ts, t0 = cfg2_large(N=(10, 10))
    ts = ts[::32]
    out = mmf.solve(p, ts, t0, prec=mmf.MMF_C64_REFINED)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 0
    H, wo, Phio = _oracle_solve(p)
    w = out["w"].cpu().numpy()
    ew = np.abs(w - wo).max() / max(1.0, np.abs(wo).max())
    Uo = oracle.evolve(p, Phio, wo, t0, ts)
    eu = np.abs(out["U"].cpu().numpy() - Uo).max()
    ep = np.abs(out["P"].cpu().numpy() - oracle.avg_prob(p, Phio)).max()
    log(f"refined ladder M=3528: eps {ew:.2e} U {eu:.2e} P {ep:.2e}")
    assert ew <= 1e-9 and eu <= 1e-9
