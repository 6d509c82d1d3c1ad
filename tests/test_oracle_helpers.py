"""Pins of the oracle's helper routines that the GPU stage tests compare with:
the tridiagonal eigensolver (reference of the divide-and-conquer tests), the
reflector product (reference of the reduction and back-transformation tests)
and the degeneracy rule of the averaged probabilities.

Each is checked against something other than itself: closed forms of the
constant tridiagonal matrix, the independent Jacobi eigensolver, reflectors
built in the test from the defining property of a Householder matrix, and the
exact time average of a static problem."""
import math

import numpy as np
import pytest

import oracle
from workloads import Problem, cfg1_tls, gue


# ------------------------------------------------------------ tridiag_eigh
@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_tridiag_eigh_constant_closed_form(n):
    """tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(k pi / (n+1)), eigenvectors
    sqrt(2/(n+1)) sin(j k pi / (n+1)) (discrete sine transform)."""
    w, Z = oracle.tridiag_eigh(np.full(n, 2.0), np.full(n - 1, -1.0))
    k = np.arange(1, n + 1)
    np.testing.assert_allclose(w, 2.0 - 2.0 * np.cos(k * math.pi / (n + 1)), rtol=0, atol=1e-13)
    j = np.arange(1, n + 1)[:, None]
    S = math.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * math.pi / (n + 1))
    # same columns up to sign
    np.testing.assert_allclose(np.abs(np.sum(S * Z, axis=0)), 1.0, rtol=0, atol=1e-12)


def test_tridiag_eigh_invariances():
    """For a random (d, e): a diagonal shift moves every eigenvalue by the
    shift, flipping the sign of e leaves the spectrum alone (similarity by
    diag(+-1)), and the trace and Frobenius identities hold; a one-sided use
    of e breaks the last one."""
    rng = np.random.default_rng(5)
    d = rng.normal(size=25)
    e = rng.normal(size=24)
    w0, _ = oracle.tridiag_eigh(d, e)
    w1, _ = oracle.tridiag_eigh(d + 3.25, e)
    w2, _ = oracle.tridiag_eigh(d, -e)
    np.testing.assert_allclose(w1, w0 + 3.25, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w2, w0, rtol=0, atol=1e-13)
    # trace and Frobenius identities of T
    assert abs(w0.sum() - d.sum()) < 1e-12
    assert abs((w0 ** 2).sum() - ((d ** 2).sum() + 2 * (e ** 2).sum())) < 1e-11


def test_tridiag_eigh_against_jacobi():
    rng = np.random.default_rng(9)
    n = 30
    d = rng.normal(size=n)
    e = rng.normal(size=n - 1)
    w, Z = oracle.tridiag_eigh(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    wj, Vj = oracle.jacobi_eigh(T.astype(np.complex128))
    np.testing.assert_allclose(w, wj, rtol=0, atol=1e-12)
    # spectral projectors of the (simple) eigenvalues agree
    for a in (0, n // 2, n - 1):
        Pa = np.outer(Z[:, a], Z[:, a])
        Pj = np.outer(Vj[:, a], Vj[:, a].conj())
        assert np.abs(Pa - Pj).max() < 1e-10
    # residual and orthogonality of the returned pairs
    assert np.abs(T @ Z - Z * w).max() < 1e-12
    assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12


# ------------------------------------------------------------ householder_tridiag_apply
def _reflector(x):
    """Complex Householder reflector built in the test from its defining
    property: H = I - tau v v^H with v[0] = 1 and H^H x = beta e_1, beta real
    (Golub and Van Loan Sec. 5.1 with the complex phase choice)."""
    alpha = x[0]
    nrm = np.linalg.norm(x)
    if nrm == 0.0 or (np.linalg.norm(x[1:]) == 0.0 and alpha.imag == 0.0):
        return np.eye(len(x), dtype=np.complex128)[:, 0], 0.0 + 0.0j, alpha.real
    beta = -math.copysign(nrm, alpha.real)
    tau = (beta - alpha) / beta
    v = np.concatenate([[1.0 + 0j], x[1:] / (alpha - beta)])
    return v, tau, beta


def test_householder_single_reflector_maps_to_beta_e1():
    rng = np.random.default_rng(3)
    n = 6
    x = rng.normal(size=n - 1) + 1j * rng.normal(size=n - 1)
    v, tau, beta = _reflector(x)
    refl = np.zeros((n, n - 1), dtype=np.complex128)
    refl[1:, 0] = v
    taus = np.zeros(n - 1, dtype=np.complex128)
    taus[0] = tau
    Q, _ = oracle.householder_tridiag_apply(np.zeros(n), np.zeros(n - 1), refl, taus)
    y = np.concatenate([[0.7 + 0.1j], x])
    out = Q.conj().T @ y
    expect = np.zeros(n, dtype=np.complex128)
    expect[0] = y[0]
    expect[1] = beta
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n), rtol=0, atol=1e-13)


def test_householder_zero_taus_give_identity_and_tridiagonal():
    n = 5
    d = np.arange(1.0, n + 1)
    e = np.array([0.5, -0.25, 2.0, 1.5])
    refl = np.zeros((n, n - 1), dtype=np.complex128)
    Q, T = oracle.householder_tridiag_apply(d, e, refl, np.zeros(n - 1, dtype=np.complex128))
    np.testing.assert_array_equal(Q, np.eye(n))
    np.testing.assert_array_equal(np.diag(T), d)
    np.testing.assert_array_equal(np.diag(T, 1), e)
    np.testing.assert_array_equal(np.diag(T, -1), e)
    assert np.count_nonzero(np.triu(T, 2)) == 0 and np.count_nonzero(np.tril(T, -2)) == 0


@pytest.mark.parametrize("n", [3, 6, 11])
def test_householder_defining_identity_of_a_textbook_reduction(n):
    """Reduce a random Hermitian A in the test (reflector i from column i
    below the diagonal, two-sided application), then the helper's Q and T
    must satisfy A = Q T Q^H.  Reversing the product order or conjugating
    tau in the helper breaks this identity for n >= 3."""
    rng = np.random.default_rng(n)
    A = gue(rng, n, 1.0)
    B = A.copy()
    refl = np.zeros((n, n - 1), dtype=np.complex128)
    taus = np.zeros(n - 1, dtype=np.complex128)
    for i in range(n - 1):
        v, tau, beta = _reflector(B[i + 1:, i].copy())
        H = np.eye(n - i - 1, dtype=np.complex128) - tau * np.outer(v, v.conj())
        B[i + 1:, :] = H.conj().T @ B[i + 1:, :]
        B[:, i + 1:] = B[:, i + 1:] @ H
        refl[i + 1:, i] = v
        taus[i] = tau
    d = np.diag(B).real.copy()
    e = np.diag(B, -1).copy()
    assert np.abs(e.imag).max() < 1e-13
    Q, T = oracle.householder_tridiag_apply(d, e.real, refl, taus)
    np.testing.assert_allclose(Q @ T @ Q.conj().T, A, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n), rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(A), rtol=0, atol=1e-12)


# ------------------------------------------------------------ degeneracy rule of the averaged P
def _static(E, omega, N):
    D = E.shape[0]
    return Problem(E=E, omega=[omega], N=[N], axis=[0], harm=[1], V=[np.zeros((D, D))])


def _rotate(Phi, a, b, theta=0.6):
    R = Phi.copy()
    c, s = math.cos(theta), math.sin(theta)
    R[:, a] = c * Phi[:, a] + s * Phi[:, b]
    R[:, b] = -s * Phi[:, a] + c * Phi[:, b]
    return R


def test_degenerate_same_site_is_flagged_and_basis_dependent():
    """Two equal levels of a static E: U = exp(-iEt) is diagonal, so the exact
    average of |U_ij|^2 is the identity.  The eigen form gives it in the pure
    basis and something else in a rotated basis of the degenerate pair; the
    rule flags both bases (both columns sit on the zero site)."""
    p = _static(np.diag([0.3, 0.3, -0.5]).astype(np.complex128), 1.1, 2)
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    s0 = oracle.zero_site(p.N)
    z = (np.abs(Phi[3 * s0:3 * s0 + 3]) ** 2).sum(0)
    pair = [a for a in range(len(w)) if abs(w[a] - 0.3) < 1e-12 and z[a] > 0.5]
    assert len(pair) == 2
    np.testing.assert_allclose(oracle.avg_prob(p, Phi), np.eye(3), atol=1e-14)
    assert oracle.avg_prob_degenerate(p, Phi, w)
    Rot = _rotate(Phi, *pair)
    assert np.abs(oracle.avg_prob(p, Rot) - np.eye(3)).max() > 0.1
    assert oracle.avg_prob_degenerate(p, Rot, w)


def test_degenerate_across_sites_flagged_only_when_weight_is_shared():
    """E = diag(0, 1), w = 1: level 0 at n = +1 and level 1 at n = 0 are
    degenerate, but only the second has weight on the zero site.  In the pure
    basis the eigen form equals the exact average (the identity) and the rule
    stays silent; mixing the pair puts weight of both on the zero site, the
    eigen form goes wrong and the rule fires."""
    p = _static(np.diag([0.0, 1.0]).astype(np.complex128), 1.0, 3)
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    np.testing.assert_allclose(oracle.avg_prob(p, Phi), np.eye(2), atol=1e-14)
    assert not oracle.avg_prob_degenerate(p, Phi, w)
    s0 = oracle.zero_site(p.N)
    s1 = oracle.sites(p.N).tolist().index([1])           # site of n = +1
    row = np.argmax(np.abs(Phi) ** 2, axis=0)            # row of each unit eigenvector
    a = int(np.nonzero(row == 2 * s1 + 0)[0][0])         # level 0 at n = +1
    b = int(np.nonzero(row == 2 * s0 + 1)[0][0])         # level 1 at n = 0
    assert abs(w[a] - w[b]) < 1e-14
    Rot = _rotate(Phi, a, b)
    assert np.abs(oracle.avg_prob(p, Rot) - np.eye(2)).max() > 0.1
    assert oracle.avg_prob_degenerate(p, Rot, w)


def test_nondegenerate_driven_problem_not_flagged():
    p, _, _ = cfg1_tls()
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    assert not oracle.avg_prob_degenerate(p, Phi, w)


# ------------------------------------------------------------ sparse propagator route
def test_evolve_expm_sparse_matches_eigen_and_dense_routes():
    """The sparse action-of-the-exponential route gives the same truncated
    U(t, t0) as the eigen expansion and the dense matrix exponential (three
    independent computations of one object), on a two-drive problem."""
    from workloads import random_problem
    p = random_problem(3, (4, 3), seed=21)
    H = oracle.build_floquet(p)
    w, Phi = oracle.eigh(H)
    ts = np.array([0.3, 2.9, 11.0])
    Ue = oracle.evolve(p, Phi, w, 0.3, ts)
    Us = oracle.evolve_expm_sparse(p, H, 0.3, ts)
    Ud = oracle.evolve_expm(p, H, 0.3, ts)
    assert np.abs(Us - Ue).max() < 1e-12
    assert np.abs(Us - Ud).max() < 1e-12
    # U(t0, t0) is the identity exactly up to rounding
    np.testing.assert_allclose(Us[0], np.eye(3), atol=1e-14)


# ------------------------------------------------ sparse assembly, spot spectra
@pytest.mark.parametrize("case", ["one_axis", "two_axes", "three_axes_harmonic", "duplicate_coupling"])
def test_build_floquet_sparse_equals_dense_definition(case):
    """The sparse assembly stores exactly the dense assembly's entries (which
    the Appendix-A layout and the closed forms pin), including a second
    harmonic and two couplings on the same (axis, h), summed."""
    from workloads import random_problem
    if case == "one_axis":
        p = random_problem(3, (7,), seed=21)
    elif case == "two_axes":
        p = random_problem(4, (3, 2), seed=22)
    elif case == "three_axes_harmonic":
        p = random_problem(2, (2, 3, 1), seed=23, harmonics=[(0, 1), (1, 1), (2, 1), (0, 2)])
    else:
        p = random_problem(3, (4, 2), seed=24, harmonics=[(0, 1), (1, 1), (0, 1)])
    Hs = oracle.build_floquet_sparse(p)
    assert Hs.shape == (oracle.floquet_dim(p),) * 2
    assert np.array_equal(Hs.toarray(), oracle.build_floquet(p))


def test_quasienergies_near_static_closed_form():
    """Undriven problem: the quasienergies are E_i + n . w exactly, so the k
    closest to a shift are known in closed form."""
    E = np.diag([0.0, 0.37, 1.3]).astype(np.complex128)
    w = np.array([1.0, math.sqrt(2.0)])
    N = [6, 5]
    p = Problem(E=E, omega=w, N=N, axis=[0, 1], harm=[1, 1], V=[np.zeros((3, 3)), np.zeros((3, 3))])
    Hs = oracle.build_floquet_sparse(p)
    n0, n1 = np.meshgrid(np.arange(-6, 7), np.arange(-5, 6), indexing="ij")
    all_eps = np.sort((np.diag(E).real[:, None] + (n0 * w[0] + n1 * w[1]).reshape(1, -1)).reshape(-1))
    for sigma in (0.11, -2.9, 4.05):
        got = oracle.quasienergies_near(Hs, sigma, 6)
        ref = np.sort(all_eps[np.argsort(np.abs(all_eps - sigma))[:6]])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_quasienergies_near_driven_against_lapack():
    """Driven problem with non-Hermitian V: the shift-invert values equal the
    k eigenvalues of LAPACK's full solve closest to the shift."""
    from workloads import random_problem
    p = random_problem(3, (6, 4), seed=11)
    wl = np.linalg.eigvalsh(oracle.build_floquet(p))
    Hs = oracle.build_floquet_sparse(p)
    for sigma in (0.37, 2.2, -1.75):
        got = oracle.quasienergies_near(Hs, sigma, 7)
        ref = np.sort(wl[np.argsort(np.abs(wl - sigma))[:7]])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
