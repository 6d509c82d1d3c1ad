"""Pins of the oracle's Floquet-matrix assembly (Eq. 6, Appendix A)."""
import os
import numpy as np
import pytest

import oracle
from workloads import Problem, random_problem, cfg1_tls, gue

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_a_layout.txt")


def _parse_layout(path):
    sections, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            sections[cur] = []
            continue
        sections[cur].append(line.split())
    return sections


def _appendix_a_problem(seed=11):
    rng = np.random.default_rng(seed)
    D = 2
    H0 = gue(rng, D, 1.0)
    V11, V12, V21 = [(rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D))) for _ in range(3)]
    w1, w2 = 1.3, 0.77
    p = Problem(E=H0, omega=[w1, w2], N=[3, 3], axis=[0, 0, 1], harm=[1, 2, 1],
                V=[V11, V12, V21])
    return p, dict(H0=H0, V11=V11, V12=V12, V21=V21, w1=w1, w2=w2)


def _expand(tok, blocks, inner=None):
    D = blocks["H0"].shape[0]
    if tok == "0":
        n = D if inner is None else inner.shape[0]
        return np.zeros((n, n), complex)
    herm = tok.endswith("^H")
    base = tok[:-2] if herm else tok
    if base.startswith("H0") or base.startswith("H1"):
        mat = blocks["H0"] if base.startswith("H0") else inner
        k = int(base[2:-2])
        w = blocks["w1"] if base.endswith("w1") else blocks["w2"]
        out = mat.copy()
        out[np.diag_indices(out.shape[0])] += k * w
        return out
    if base == "V21" and inner is not None:
        out = np.kron(np.eye(7), blocks["V21"])
    else:
        out = blocks[base].copy()
    return out.conj().T if herm else out


def test_appendix_a_layout_exact():
    """Every block lands where Appendix A prints it (incl. the seven copies of
    V^{2,1} in the outer coupling block)."""
    lay = _parse_layout(GOLDEN)
    p, blocks = _appendix_a_problem()
    inner = np.block([[_expand(t, blocks) for t in row] for row in lay["inner"]])
    full = np.block([[_expand(t, blocks, inner) for t in row] for row in lay["outer"]])
    H = oracle.build_floquet(p)
    assert H.shape == full.shape == (98, 98)
    np.testing.assert_allclose(H, full, rtol=0, atol=1e-14)


def test_exact_hermiticity_and_entries():
    p = random_problem(3, (2, 3), seed=5, harmonics=[(0, 1), (1, 1), (0, 2), (1, 3)])
    H = oracle.build_floquet(p)
    assert np.array_equal(H, H.conj().T)
    rng = np.random.default_rng(0)
    M = H.shape[0]
    for _ in range(400):
        r, c = rng.integers(0, M, size=2)
        assert oracle.floquet_entry(p, int(r), int(c)) == H[r, c]


def test_trace_and_frobenius_identities():
    """tr H_F = S tr E (n.w sums to zero over the symmetric box) and
    ||H_F||_F^2 = S||E||_F^2 + D sum_s (n_s.w)^2 (+ cross term) + 2 sum_k pairs_k ||V_k||^2."""
    p = random_problem(3, (4, 2), seed=7)
    H = oracle.build_floquet(p)
    n = oracle.sites(p.N)
    S = n.shape[0]
    assert abs(np.trace(H) - S * np.trace(p.E)) < 1e-11
    shifts = n @ p.omega
    # diagonal contributions: |E_ii + x|^2 summed = ||E||^2 + 2 x Re tr E + D x^2
    diag_part = sum(np.linalg.norm(p.E) ** 2 + 2 * x * np.trace(p.E).real + p.D * x * x for x in shifts)
    coup = 0.0
    for k in range(p.K):
        l, h = int(p.axis[k]), int(p.harm[k])
        pairs = sum(1 for v in n if abs(v[l] - h) <= p.N[l]) if h <= 2 * p.N[l] else 0
        coup += 2 * pairs * np.linalg.norm(p.V[k]) ** 2
    assert abs(np.linalg.norm(H) ** 2 - (diag_part + coup)) < 1e-9 * np.linalg.norm(H) ** 2


def test_harmonic_beyond_box_contributes_nothing():
    p = random_problem(2, (1,), seed=3, harmonics=[(0, 1), (0, 3)])
    H = oracle.build_floquet(p)
    q = Problem(E=p.E, omega=p.omega, N=p.N, axis=p.axis[:1], harm=p.harm[:1], V=p.V[:1])
    assert np.array_equal(H, oracle.build_floquet(q))


def test_static_limit_spectrum():
    """No drive: H_F is block diagonal and eps = eig(E) + n.w exactly as a set."""
    rng = np.random.default_rng(1)
    D = 3
    E = gue(rng, D, 1.0)
    p = Problem(E=E, omega=[1.7, 0.45], N=[2, 1], axis=[0], harm=[1], V=[np.zeros((D, D))])
    H = oracle.build_floquet(p)
    w, _ = oracle.eigh(H)
    e0 = np.linalg.eigvalsh(E)
    n = oracle.sites(p.N)
    expect = np.sort((e0[None, :] + (n @ p.omega)[:, None]).ravel())
    np.testing.assert_allclose(w, expect, rtol=0, atol=1e-13)


def test_cfg1_dimension_and_band():
    p, _, _ = cfg1_tls()
    H = oracle.build_floquet(p)
    assert H.shape == (82, 82)
    # top block is H0 + 20 w (descending n, App. A)
    np.testing.assert_allclose(np.diag(H)[:2].real, [0.5 + 20 * 1.1, -0.5 + 20 * 1.1], rtol=0, atol=1e-13)
    assert H[0, 3] == 0.05 and H[2, 1] == 0.05          # V = 0.05 sx above the diagonal
    assert np.count_nonzero(np.abs(np.triu(H, 4))) == 0
