"""Oracle pins for evolution in a dressed basis (Sec. 4.1, Fig. 4).

* Without the probe the full problem is the dressing subset itself, so its
  evolution seen in the subset's dressed basis is diagonal with the dressed
  quasienergies: U_dressed(t, t0) = diag(exp(-i eps_b (t - t0))) (the
  micromotion factorisation of Eq. 4), up to the truncation error.
* Resonant dressing (omega_D = omega0) of a qubit with S = sigma/2 splits the
  dressed states by Omega_X / 2 (quasienergies +-(omega0 + Omega_X/2)/2 modulo
  omega_D); a weak probe on S_z then drives complete transitions between the
  dressed states exactly when omega_P = Omega_X / 2, the resonance the paper
  points out, and only partial ones 0.002 away from it.
"""
import numpy as np

import oracle
from workloads import dressed_qubit


def test_restrict_modes_keeps_static_part_and_subset_couplings():
    p = dressed_qubit(0.0125)
    q = oracle.restrict_modes(p, [0])
    assert q.omega == [1.0] and q.N == [4] and q.axis == [0] and q.harm == [1]
    assert np.array_equal(q.V[0], np.asarray(p.V[0])) and np.array_equal(q.E, p.E)
    r = oracle.restrict_modes(p, [1])
    assert r.omega == [0.0125] and r.axis == [0] and np.array_equal(r.V[0], np.asarray(p.V[1]))


def test_dressed_evolution_without_probe_is_diagonal_phase():
    p = dressed_qubit(0.0125, Omega_Px=0.0, Omega_Pz=0.0, N=(6, 2))
    ts = np.linspace(0.0, 800.0, 41)
    t0 = 0.37
    Ud, U, eps = oracle.dressed_evolution(p, [0], ts, t0)
    expect = np.array([np.diag(np.exp(-1j * eps * (t - t0))) for t in ts])
    assert np.abs(Ud - expect).max() < 1e-9
    # the dressed splitting is Omega_X / 2 modulo omega_D
    assert abs(abs(eps[1] - eps[0]) - 1.0 - 0.0125) < 1e-6


def test_weak_probe_resonance_at_half_dressing_rabi_frequency():
    ts = np.linspace(0.0, 30000.0, 601)
    peak = {}
    for wP in (0.0105, 0.0125, 0.0145):
        p = dressed_qubit(wP, Omega_Px=0.0005, Omega_Pz=0.0025, N=(4, 4))
        Ud, _, _ = oracle.dressed_evolution(p, [0], ts, 0.0)
        peak[wP] = float((np.abs(Ud[:, 1, 0]) ** 2).max())
    assert peak[0.0125] > 0.99
    assert peak[0.0105] < 0.35 and peak[0.0145] < 0.35
