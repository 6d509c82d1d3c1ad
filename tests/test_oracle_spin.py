"""Oracle pins for the spin front end (Sec. 3.4: Eq. 7 and the two-spin
dipole system) and parity of the library's host-side builders with it.

* angular-momentum algebra: [S_x, S_y] = i S_z (and cyclic), S^2 = s(s+1),
  S_z = diag(s .. -s);
* dipole interaction A S_1.S_2: eigenvalues A/2 [F(F+1) - s1(s1+1) - s2(s2+1)]
  with multiplicity 2F + 1, F = |s1 - s2| .. s1 + s2;
* spin s in a circularly polarised drive omega0 S_z + Omega (S_x cos wt +
  S_y sin wt): in the frame rotating at w the Hamiltonian is static,
  (omega0 - w) S_z + Omega S_x, so the Floquet exponents are
  m Omega_R (m = -s..s, Omega_R = sqrt((omega0 - w)^2 + Omega^2)), shifted by
  w/2 for half-integer s (the frame rotation by 2 pi is -1), modulo w.
"""
import math
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("s", [0.5, 1, 1.5, 2, 3.5])
def test_spin_algebra(s):
    Sx, Sy, Sz = oracle.spin_ops(s)
    D = int(round(2 * s)) + 1
    I = np.eye(D)
    for A, B, Cm in ((Sx, Sy, Sz), (Sy, Sz, Sx), (Sz, Sx, Sy)):
        assert np.abs(A @ B - B @ A - 1j * Cm).max() < 1e-13
    assert np.abs(Sx @ Sx + Sy @ Sy + Sz @ Sz - s * (s + 1) * I).max() < 1e-12
    assert np.allclose(np.diag(Sz).real, s - np.arange(D))
    for A in (Sx, Sy, Sz):
        assert np.abs(A - A.conj().T).max() == 0


@pytest.mark.parametrize("s1,s2", [(0.5, 0.5), (0.5, 1.5), (1, 1), (1.5, 2)])
def test_dipole_multiplets(s1, s2):
    A = 0.7
    S1 = [np.kron(a, np.eye(int(2 * s2 + 1))) for a in oracle.spin_ops(s1)]
    S2 = [np.kron(np.eye(int(2 * s1 + 1)), b) for b in oracle.spin_ops(s2)]
    H = A * sum(a @ b for a, b in zip(S1, S2))
    ev = np.linalg.eigvalsh(H)
    expect = []
    F = abs(s1 - s2)
    while F <= s1 + s2 + 1e-9:
        expect += [A / 2 * (F * (F + 1) - s1 * (s1 + 1) - s2 * (s2 + 1))] * int(round(2 * F + 1))
        F += 1
    assert np.abs(ev - np.sort(expect)).max() < 1e-12


@pytest.mark.parametrize("s", [1, 1.5])
def test_circular_drive_quasienergies(s):
    w0, Om, w, N = 1.0, 0.2, 0.9, 14
    S = oracle.spin_ops(s)
    # Omega (S_x cos wt + S_y sin wt) = Omega cos(wt) S_x + Omega cos(wt - pi/2) S_y
    V = oracle.spin_drive(S, (Om, Om, 0.0), (0.0, -math.pi / 2, 0.0))

    class P:
        pass
    p = P()
    p.E, p.D, p.F, p.K = w0 * S[2], S[2].shape[0], 1, 1
    p.omega, p.N, p.axis, p.harm, p.V = [w], [N], [0], [1], [V]
    q = oracle.quasienergies(p)
    OmR = math.hypot(w0 - w, Om)
    D = p.D
    shift = 0.5 * w if (2 * s) % 2 == 1 else 0.0
    expect = np.sort(np.mod(np.array([m * OmR + shift for m in np.arange(-s, s + 1)]) + w / 2, w) - w / 2)
    central = np.sort(q[(q >= -w / 2) & (q < w / 2)])
    assert len(central) == D
    assert np.abs(central - expect).max() < 1e-9


def test_front_end_builders_match_the_oracle():
    from paper_2005_03426_amd import spin
    for s in (0.5, 1, 1.5, 2):
        for a, b in zip(spin.spin_matrices(s), oracle.spin_ops(s)):
            assert np.abs(a - b).max() < 1e-15
        S = oracle.spin_ops(s)
        amp, ph = (0.3, -0.2, 0.05), (0.1, 1.2, -0.7)
        assert np.abs(spin.drive_coupling(spin.spin_matrices(s), amp, ph) - oracle.spin_drive(S, amp, ph)).max() < 1e-15
    p = spin.two_spin_problem(0.5, 1.5, 0.7, static1=(0, 0, 0.3), static2=(0, 0, -0.1),
                              drives=[(0.8, (0.1, 0, 0), (0.02, 0, 0))], N=[3])
    S1 = [np.kron(a, np.eye(4)) for a in oracle.spin_ops(0.5)]
    S2 = [np.kron(np.eye(2), b) for b in oracle.spin_ops(1.5)]
    E = 0.7 * sum(a @ b for a, b in zip(S1, S2)) + 0.3 * S1[2] - 0.1 * S2[2]
    assert np.abs(p.E - E).max() < 1e-14
    V = oracle.spin_drive(S1, (0.1, 0, 0), (0, 0, 0)) + oracle.spin_drive(S2, (0.02, 0, 0), (0, 0, 0))
    assert np.abs(p.V[0] - V).max() < 1e-15
