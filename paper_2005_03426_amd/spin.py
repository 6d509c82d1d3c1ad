"""Problem builders for spin systems (Sec. 3.4 of the paper: the spin
couplings of Eq. 7 and the two-spin dipole system).

These build the *inputs* of a Floquet problem -- the D x D matrices E and
V_k of the problem statement (D = 2s + 1, or (2s1 + 1)(2s2 + 1) for two
spins) -- on the host, once per problem; everything from the Floquet matrix
onward runs in the library's kernels.

Conventions:
  * angular-momentum matrices in the |s, m> basis ordered m = s, s-1, ..., -s
    (S_z diagonal, S_+ |m> = sqrt(s(s+1) - m(m+1)) |m+1>, S_x = (S_+ + S_-)/2,
    S_y = (S_+ - S_-)/(2i), hbar = 1);
  * a drive is given per Cartesian axis by a cos amplitude and a phase,
    H(t) ∋ sum_i A_i cos(h w t + phi_i) S_i (Eq. 7 with the missing i in the
    exponent and the axis set x, y, z), which enters the problem statement as
    the Fourier coefficient V = sum_i (A_i / 2) e^{i phi_i} S_i (the same
    reading as the dressed-qubit example of Sec. 4.1, Eq. 8);
  * two spins use the uncoupled basis |m1, m2> = |m1> (x) |m2> (index
    i = i1 * (2 s2 + 1) + i2) with the dipole interaction A S_1 . S_2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def spin_matrices(s: float):
    """(S_x, S_y, S_z) for spin s (integer or half-integer), basis m = s .. -s."""
    twos = int(round(2 * s))
    if twos < 0 or abs(twos - 2 * s) > 1e-12:
        raise ValueError("s must be a non-negative integer or half-integer")
    D = twos + 1
    m = s - np.arange(D)                       # s, s-1, ..., -s
    Sz = np.diag(m).astype(np.complex128)
    Sp = np.zeros((D, D), np.complex128)       # raising: <m+1| S_+ |m>
    for k in range(1, D):                      # column k holds m[k]; row k-1 holds m[k] + 1
        Sp[k - 1, k] = np.sqrt(s * (s + 1) - m[k] * (m[k] + 1))
    Sm = Sp.conj().T
    Sx = 0.5 * (Sp + Sm)
    Sy = -0.5j * (Sp - Sm)
    return Sx, Sy, Sz


@dataclass
class SpinProblem:
    """A problem statement (the fields the library's DeviceProblem reads)."""
    E: np.ndarray
    omega: list
    N: list
    axis: list = field(default_factory=list)
    harm: list = field(default_factory=list)
    V: list = field(default_factory=list)

    @property
    def D(self):
        return int(self.E.shape[0])

    @property
    def F(self):
        return len(self.omega)

    @property
    def K(self):
        return len(self.axis)


def drive_coupling(S, amplitudes, phases=(0.0, 0.0, 0.0)):
    """Fourier coefficient of sum_i A_i cos(w t + phi_i) S_i for S = (S_x, S_y, S_z)."""
    V = np.zeros_like(S[0])
    for Si, a, ph in zip(S, amplitudes, phases):
        V = V + (0.5 * a * np.exp(1j * ph)) * Si
    return V


def spin_problem(s: float, static=(0.0, 0.0, 0.0), drives=(), N=()):
    """Spin s with static field terms sum_i static_i S_i and drives
    (omega, amplitudes (x, y, z), phases (x, y, z), harmonic) on fundamentals
    0, 1, ... (one per drive), truncations N."""
    S = spin_matrices(s)
    E = sum(b * Si for b, Si in zip(static, S))
    p = SpinProblem(E=np.asarray(E, np.complex128), omega=[], N=list(N))
    for k, d in enumerate(drives):
        w, amp = d[0], d[1]
        ph = d[2] if len(d) > 2 else (0.0, 0.0, 0.0)
        h = d[3] if len(d) > 3 else 1
        p.omega.append(float(w))
        p.axis.append(k)
        p.harm.append(int(h))
        p.V.append(drive_coupling(S, amp, ph))
    return p


def two_spin_matrices(s1: float, s2: float):
    """Spin operators of both spins in the uncoupled basis |m1, m2>."""
    A = spin_matrices(s1)
    B = spin_matrices(s2)
    I1 = np.eye(A[0].shape[0])
    I2 = np.eye(B[0].shape[0])
    return [np.kron(a, I2) for a in A], [np.kron(I1, b) for b in B]


def two_spin_problem(s1: float, s2: float, A_dip: float, static1=(0.0, 0.0, 0.0), static2=(0.0, 0.0, 0.0),
                     drives=(), N=()):
    """Two spins with the dipole interaction A_dip S_1 . S_2, static field
    terms on each spin and drives; a drive is (omega, amplitudes on spin 1,
    amplitudes on spin 2, phases (x, y, z), harmonic), one fundamental each."""
    S1, S2 = two_spin_matrices(s1, s2)
    E = A_dip * sum(a @ b for a, b in zip(S1, S2))
    E = E + sum(b * Si for b, Si in zip(static1, S1)) + sum(b * Si for b, Si in zip(static2, S2))
    p = SpinProblem(E=np.asarray(E, np.complex128), omega=[], N=list(N))
    for k, d in enumerate(drives):
        w, a1, a2 = d[0], d[1], d[2]
        ph = d[3] if len(d) > 3 else (0.0, 0.0, 0.0)
        h = d[4] if len(d) > 4 else 1
        p.omega.append(float(w))
        p.axis.append(k)
        p.harm.append(int(h))
        p.V.append(drive_coupling(S1, a1, ph) + drive_coupling(S2, a2, ph))
    return p


def dipole_basis(s1: float, s2: float, A_dip: float, device="cuda"):
    """Eigenbasis of the dipole interaction A_dip S_1 . S_2 (columns, eigenvalues
    ascending), computed by the library's eigensolver; returns (W, energies) as
    device tensors with W[i, b] = <m1 m2 | b>."""
    import torch
    from . import eigh
    S1, S2 = two_spin_matrices(s1, s2)
    Hd = A_dip * sum(a @ b for a, b in zip(S1, S2))
    At = torch.from_numpy(np.ascontiguousarray(Hd.T)).to(device)
    w, Pt, info = eigh(At)
    return Pt.T, w


def change_basis(U, W):
    """U' [t] = W^H U[t] W for every time (U: [T, D, D] device tensor, W: [D, D]),
    through the library's dressed-basis kernel with a time-independent basis."""
    import torch
    import ctypes as C
    from . import call, _ptr, _stream
    T, D, _ = U.shape
    Us = U.transpose(1, 2).contiguous()                    # column-major per time
    Ws = W.T.contiguous()                                  # column-major
    W2 = Ws.unsqueeze(0).expand(T, D, D).contiguous()
    out = torch.empty((T, D, D), dtype=torch.complex128, device=U.device)
    call("mmf_dressed_evolution", C.c_int32(D), C.c_int32(T), _ptr(W2), _ptr(Us), _ptr(Ws), _ptr(out),
         _stream(None))
    return out.transpose(1, 2)
