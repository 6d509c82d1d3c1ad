"""Pins of the oracle's eigensolve, U(t,t0), micromotion and averaged
transition probabilities against closed forms, brute force and invariants."""
import math
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import jv

import oracle
from workloads import Problem, random_problem, cfg1_tls, tls_problem, gue

SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]], complex)
SZ = np.array([[1, 0], [0, -1]], complex)
SM = np.array([[0, 0], [1, 0]], complex)     # sigma_- = |down><up| (basis up, down)


def _solve(p):
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    return H, w, Phi


# ----------------------------------------------------------------- eigensolve
def test_jacobi_agrees_with_lapack():
    p = random_problem(2, (4, 2), seed=9)          # M = 2*9*5 = 90
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    wj, Vj = oracle.jacobi_eigh(H)
    scale = max(1.0, np.abs(w).max())
    assert np.abs(w - wj).max() <= 1e-12 * scale
    # spectral projectors of well-separated eigenvalues agree
    gaps = np.minimum(np.r_[np.inf, np.diff(w)], np.r_[np.diff(w), np.inf])
    for a in np.nonzero(gaps > 1e-3)[0][:20]:
        P1 = np.outer(Phi[:, a], Phi[:, a].conj())
        P2 = np.outer(Vj[:, a], Vj[:, a].conj())
        assert np.abs(P1 - P2).max() < 1e-10


def test_eigvalsh_agrees_with_jacobi():
    """The eigenvalue-only library route against the oracle's own Jacobi
    method (an independent algorithm), on a Floquet matrix with a cluster."""
    p = random_problem(3, (5, 1), seed=12)        # M = 3*11*3 = 99
    H = oracle.build_floquet(p)
    wj, _ = oracle.jacobi_eigh(H)
    w = oracle.eigvalsh(H)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wj).max() <= 1e-12 * max(1.0, np.abs(wj).max())


def test_eigh_residual_and_orthogonality():
    p = random_problem(3, (3, 3), seed=4)
    H, w, Phi = _solve(p)
    assert np.linalg.norm(H @ Phi - Phi * w) / np.linalg.norm(H) < 1e-13
    assert np.abs(Phi.conj().T @ Phi - np.eye(len(w))).max() < 1e-12


def test_omega_translation_symmetry_cfg1():
    """Central quasienergies repeat at eps + w (extended-space translation)."""
    p, _, _ = cfg1_tls()
    H, w, Phi = _solve(p)
    n = oracle.sites(p.N)[:, 0].astype(float)
    weight = (np.abs(Phi) ** 2).reshape(len(n), 2, -1).sum(axis=1)
    c = n @ weight
    om = p.omega[0]
    checked = 0
    for a in range(len(w)):
        if abs(c[a]) <= p.N[0] - 10:
            assert np.min(np.abs(w - (w[a] + om))) < 1e-12
            checked += 1
    assert checked >= 30


# ------------------------------------------------------------ closed forms
def test_static_limit_evolution_and_average():
    rng = np.random.default_rng(2)
    D = 3
    E = gue(rng, D, 1.0)
    p = Problem(E=E, omega=[1.3], N=[2], axis=[0], harm=[1], V=[np.zeros((D, D))])
    H, w, Phi = _solve(p)
    ts = np.array([0.0, 0.37, 2.5, 11.0])
    U = oracle.evolve(p, Phi, w, 0.4, ts)
    for q, t in enumerate(ts):
        np.testing.assert_allclose(U[q], expm(-1j * E * (t - 0.4)), atol=1e-13)
    e, B = np.linalg.eigh(E)
    expect = (np.abs(B) ** 2) @ (np.abs(B) ** 2).T
    np.testing.assert_allclose(oracle.avg_prob(p, Phi), expect, atol=1e-13)


def test_bessel_diagonal_drive():
    """E = diag(E_i), drive sum_l a_il cos(w_l t) on the diagonal: exact phases
    (Jacobi-Anger), Bessel-weighted Fourier components, P = I."""
    Ei = np.array([0.3, -0.8])
    a = np.array([[0.9, 0.4], [0.5, 1.1]])         # a[i, l]
    w = np.array([1.0, 1.618])
    N = [18, 18]
    V = [np.diag(a[:, 0]) / 2, np.diag(a[:, 1]) / 2]
    p = Problem(E=np.diag(Ei), omega=w, N=N, axis=[0, 1], harm=[1, 1], V=V)
    H, eps, Phi = _solve(p)
    t0 = 0.6
    ts = np.array([0.6, 1.9, 7.3, 20.0])
    U = oracle.evolve(p, Phi, eps, t0, ts)
    for q, t in enumerate(ts):
        for i in range(2):
            ph = -Ei[i] * (t - t0) - sum(a[i, l] / w[l] * (math.sin(w[l] * t) - math.sin(w[l] * t0)) for l in range(2))
            assert abs(U[q, i, i] - np.exp(1j * ph)) < 1e-12
        assert abs(U[q, 0, 1]) < 1e-13 and abs(U[q, 1, 0]) < 1e-13
    np.testing.assert_allclose(oracle.avg_prob(p, Phi), np.eye(2), atol=1e-12)
    # eigenvector of the central orbit of level i=0: |Phi[(0,n)]|^2 = prod_l J_{n_l}(a_0l/w_l)^2
    n = oracle.sites(N)
    s0 = oracle.zero_site(N)
    col = np.argmax(np.abs(Phi[2 * s0, :]))
    assert abs(eps[col] - Ei[0]) < 1e-12
    weights = np.abs(Phi[0::2, col]) ** 2
    expect = jv(n[:, 0], a[0, 0] / w[0]) ** 2 * jv(n[:, 1], a[0, 1] / w[1]) ** 2
    np.testing.assert_allclose(weights, expect, atol=1e-13)


def test_circular_drive_exact_rabi():
    """H = (w0/2) sz + g s- e^{iwt} + g s+ e^{-iwt}: rotating frame is exact."""
    w0, g, w = 1.0, 0.07, 0.93
    p = Problem(E=(w0 / 2) * SZ, omega=[w], N=[12], axis=[0], harm=[1], V=[g * SM])
    H, eps, Phi = _solve(p)
    Delta = w0 - w
    Om = math.sqrt(Delta ** 2 + 4 * g * g)
    Hp = (Delta / 2) * SZ + g * SX
    t0 = 1.3
    ts = np.linspace(0, 40, 9)
    U = oracle.evolve(p, Phi, eps, t0, ts)
    for q, t in enumerate(ts):
        R = lambda s: expm(1j * w * s * SZ / 2)
        expect = R(t).conj().T @ expm(-1j * Hp * (t - t0)) @ R(t0)
        np.testing.assert_allclose(U[q], expect, atol=1e-12)
    P = oracle.avg_prob(p, Phi)
    assert abs(P[0, 1] - 2 * g * g / Om ** 2) < 1e-12
    assert abs(P[1, 0] - 2 * g * g / Om ** 2) < 1e-12
    # quasienergies w/2 +- Om/2 modulo w
    for target in (w / 2 + Om / 2, w / 2 - Om / 2):
        folded = np.mod(eps - target + w / 2, w) - w / 2
        assert np.min(np.abs(folded)) < 1e-12


def _folded_splitting(p):
    _, eps, Phi = _solve(p)
    s0 = oracle.zero_site(p.N)
    wt = (np.abs(Phi[2 * s0:2 * s0 + 2, :]) ** 2).sum(axis=0)
    top = np.argsort(wt)[-2:]
    de = abs(eps[top[0]] - eps[top[1]])
    om = p.omega[0]
    de = de % om
    return min(de, om - de), oracle.avg_prob(p, Phi)


def test_rwa_and_bloch_siegert_asymptotics():
    """Linear drive on a TLS: RWA error ~ Omega^2, Bloch-Siegert error ~ Omega^4."""
    w0, w = 1.0, 1.1
    err_rwa, err_bs = [], []
    for Om in (0.4, 0.2, 0.1, 0.05):
        split, P = _folded_splitting(tls_problem(w0, Om, w, 20))
        Delta = w0 - w
        rwa = math.sqrt(Delta ** 2 + Om ** 2 / 4)
        g = Om / 4
        d_eff = Delta + 2 * g * g / (w0 + w)
        bs = math.sqrt(d_eff ** 2 + 4 * g * g)
        err_rwa.append(abs(split - rwa))
        err_bs.append(abs(split - bs))
        assert abs(P.sum(axis=0) - 1).max() < 1e-12
    for k in range(3):
        assert err_rwa[k] / err_rwa[k + 1] >= 2.5
        assert err_bs[k] / err_bs[k + 1] >= 8.0
    assert err_bs[1] <= err_rwa[1] / 10


def test_cfg1_values_and_unitarity():
    p, ts, t0 = cfg1_tls()
    H, eps, Phi = _solve(p)
    U = oracle.evolve(p, Phi, eps, t0, ts)
    dev = max(np.abs(U[q].conj().T @ U[q] - np.eye(2)).max() for q in range(len(ts)))
    assert dev < 1e-10
    P = oracle.avg_prob(p, Phi)
    np.testing.assert_allclose(P.sum(axis=0), 1.0, atol=1e-12)
    np.testing.assert_allclose(P, P.T, atol=1e-10)
    split, _ = _folded_splitting(p)
    # exact value lies between the RWA (0.14142) and just below Bloch-Siegert (0.13975)
    assert 0.1390 < split < 0.1398


# ------------------------------------------------------------ brute force
def test_rk4_matches_floquet_evolution():
    """Two fundamentals, weak drive, converged truncation: RK4 (h = 1e-3)."""
    rng = np.random.default_rng(21)
    D = 2
    E = np.diag([0.4, -0.4]).astype(complex) + 0.05 * gue(rng, D, 1.0)
    V = [0.12 * (rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D))) for _ in range(2)]
    p = Problem(E=E, omega=[1.0, 1.414], N=[9, 9], axis=[0, 1], harm=[1, 1], V=V)
    H, eps, Phi = _solve(p)
    t0 = 0.35
    ts = np.array([1.0, 3.7, 6.0])
    U = oracle.evolve(p, Phi, eps, t0, ts)
    Ur = oracle.rk4_evolve(p, t0, ts, h=1e-3)
    assert np.abs(U - Ur).max() < 1e-9


def test_expm_route_matches_eigen_route():
    p = random_problem(2, (3, 2), seed=13)
    H, eps, Phi = _solve(p)
    ts = np.array([0.0, 0.8, 3.3])
    np.testing.assert_allclose(oracle.evolve(p, Phi, eps, 0.2, ts),
                               oracle.evolve_expm(p, H, 0.2, ts), atol=1e-12)


def test_micromotion_route():
    """U_F(t) diag(e^{-i eps (t-t0)}) U_F(t0)^H reproduces U(t,t0); U_F unitary."""
    p, _, _ = cfg1_tls()
    H, eps, Phi = _solve(p)
    ts = np.array([0.0, 2.1, 9.9])
    t0 = 0.5
    U = oracle.evolve(p, Phi, eps, t0, ts)
    UF, esel = oracle.micromotion(p, Phi, eps, ts)
    UF0, _ = oracle.micromotion(p, Phi, eps, [t0])
    for q, t in enumerate(ts):
        assert np.abs(UF[q].conj().T @ UF[q] - np.eye(2)).max() < 1e-10
        alt = UF[q] @ np.diag(np.exp(-1j * esel * (t - t0))) @ UF0[0].conj().T
        assert np.abs(alt - U[q]).max() < 1e-10
    assert np.all(np.abs(esel) < p.omega[0])


def test_time_average_monte_carlo():
    """Brute-force average of |U_ij(t0 + tau, t0)|^2 over random t0 and tau."""
    p = tls_problem(1.0, 0.6, 1.2, 12)
    H, eps, Phi = _solve(p)
    P = oracle.avg_prob(p, Phi)
    rng = np.random.default_rng(0)
    acc = np.zeros((2, 2))
    nsamp = 4000
    t0s = rng.uniform(0, 2 * math.pi / 1.2, nsamp)
    taus = rng.uniform(0, 1e4, nsamp)
    for t0, tau in zip(t0s, taus):
        acc += np.abs(oracle.evolve(p, Phi, eps, t0, [t0 + tau])[0]) ** 2
    acc /= nsamp
    assert np.abs(acc - P).max() < 2e-2
