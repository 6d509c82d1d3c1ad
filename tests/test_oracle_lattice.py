"""Oracle pins for the driven-lattice quasienergy scan (Sec. 4.2, the unnumbered lattice Hamiltonian).

The open chain's hopping phases t exp(i cos(2 pi m / D)) are a pure gauge
(a diagonal unitary removes them bond by bond), so the static spectrum is
that of uniform hopping t with staggered energies +-V0:
    +- sqrt(V0^2 + 4 t^2 cos^2(pi j / (D + 1))),  j = 1 .. D/2.
Without the drive the Floquet spectrum is that set shifted by every n w,
n in [-N, N]; the oracle's assembly + eigenvalue routine must reproduce it.
"""
import numpy as np
import pytest

import oracle
from workloads import lattice_problem


def _static_closed_form(D, V0, t):
    j = np.arange(1, D // 2 + 1)
    r = np.sqrt(V0 ** 2 + 4 * t ** 2 * np.cos(np.pi * j / (D + 1)) ** 2)
    return np.sort(np.concatenate([-r, r]))


@pytest.mark.parametrize("D", [8, 256])
def test_static_lattice_spectrum_is_gauge_free_closed_form(D):
    p = lattice_problem(0.4, D=D, V=0.0, N=1)
    ev = np.linalg.eigvalsh(p.E)
    assert np.abs(ev - _static_closed_form(D, 0.25, 0.125)).max() < 1e-13


@pytest.mark.parametrize("w,N", [(0.4, 2), (0.6, 1)])
def test_undriven_floquet_spectrum_is_shifted_static_spectrum(w, N):
    D = 64
    p = lattice_problem(w, D=D, V=0.0, N=N)
    q = oracle.quasienergies(p)
    st = _static_closed_form(D, 0.25, 0.125)
    expect = np.sort(np.concatenate([st + n * w for n in range(-N, N + 1)]))
    assert q.shape == (D * (2 * N + 1),)
    assert np.abs(q - expect).max() < 1e-13


def test_driven_lattice_spectrum_invariants():
    """tr H_F = 0 (staggered energies cancel, n w cancels over the box) and the
    drive's Frobenius weight 2 * #bonds * (V/2)^2 * (site pairs) enters
    sum eps^2 = ||H_F||_F^2."""
    D, N, V, w = 16, 3, 0.0625, 0.5
    p = lattice_problem(w, D=D, V=V, N=N)
    q = oracle.quasienergies(p)
    S = 2 * N + 1
    assert abs(q.sum()) < 1e-12
    static_f2 = np.sum(np.abs(p.E) ** 2)
    shift_f2 = D * sum((n * w) ** 2 for n in range(-N, N + 1))
    drive_f2 = 2 * (S - 1) * 2 * (D - 1) * (V / 2) ** 2
    assert abs(np.sum(q ** 2) - (S * static_f2 + shift_f2 + drive_f2)) < 1e-11


@pytest.mark.parametrize("w,shift", [(0.4, 0.0), (0.6, 0.0), (0.6, 0.11), (0.9, -0.2)])
def test_window_of_one_drive_period_holds_one_state_per_orbit(w, shift):
    """omega-translation symmetry: a converged single-drive truncation has one
    quasienergy per orbit in any central window of width omega."""
    D = 32
    q = oracle.quasienergies(lattice_problem(w, D=D, N=4))
    lo = -w / 2 + shift
    assert int(((q >= lo) & (q < lo + w)).sum()) == D
