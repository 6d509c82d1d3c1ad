"""Seeded synthetic inputs for the multimode Floquet hot path.

This module only *describes problems*: the bare Hamiltonian E, the harmonic
couplings V_k with the fundamental each one oscillates at, the fundamental
frequencies and the per-fundamental Fourier truncations (Eq. 1 and the data
structures of Sec. 3.1 of the paper: ATOM, MODES_NUMBER, MODE).  It contains
none of the method's arithmetic (no Floquet matrix, no eigenpairs, no time
evolution); both the CPU oracle and the GPU library consume what it returns.

Conventions (shared by every consumer):
  * H(t) = E + sum_k [ V_k exp(+i h_k w_{axis_k} t) + V_k^H exp(-i h_k w_{axis_k} t) ]
    (hbar = 1).  A drive written as C cos(w t + phi) enters as V = (C/2) e^{i phi}.
  * Fourier truncation: n_l in [-N_l, N_l] on every fundamental axis l.

The named workloads follow the sizes, value distributions and draw order that
the benchmark configurations state (a two-level atom under one drive; an
8-level ladder under two incommensurate drives; a batch of 512 uneven solves;
a 16-level spectrum under two drives; a Poisson stream of served requests).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np

__all__ = [
    "Problem", "gue", "tls_problem", "cfg1_tls", "cfg2_large", "cfg3_batch",
    "cfg3_uniform_sweep", "cfg4_precision", "cfg5_serving", "random_problem",
    "time_grid", "floquet_dim_of", "lattice_problem", "lattice_sweep", "dressed_qubit",
]


@dataclass
class Problem:
    """A multimode-driven D-level system (host arrays, numpy)."""
    E: np.ndarray                 # (D, D) complex128, Hermitian
    omega: np.ndarray             # (F,) float64 fundamental angular frequencies
    N: np.ndarray                 # (F,) int32 truncations
    axis: np.ndarray              # (K,) int32 fundamental index of each coupling
    harm: np.ndarray              # (K,) int32 harmonic order h >= 1
    V: np.ndarray                 # (K, D, D) complex128 coupling matrices
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.E = np.ascontiguousarray(self.E, dtype=np.complex128)
        self.omega = np.ascontiguousarray(self.omega, dtype=np.float64).reshape(-1)
        self.N = np.ascontiguousarray(self.N, dtype=np.int32).reshape(-1)
        self.axis = np.ascontiguousarray(self.axis, dtype=np.int32).reshape(-1)
        self.harm = np.ascontiguousarray(self.harm, dtype=np.int32).reshape(-1)
        V = np.asarray(self.V, dtype=np.complex128)
        if V.size == 0:
            V = np.zeros((0, self.E.shape[0], self.E.shape[0]), np.complex128)
        self.V = np.ascontiguousarray(V)

    @property
    def D(self) -> int:
        return int(self.E.shape[0])

    @property
    def F(self) -> int:
        return int(self.omega.shape[0])

    @property
    def K(self) -> int:
        return int(self.axis.shape[0])


def floquet_dim_of(p: Problem) -> int:
    """Number of rows of the truncated Floquet matrix: D * prod(2 N_l + 1).

    A sizing helper (no arithmetic of the method)."""
    s = 1
    for n in p.N:
        s *= 2 * int(n) + 1
    return p.D * s


def gue(rng: np.random.Generator, D: int, sigma: float) -> np.ndarray:
    """Random Hermitian matrix: A, B ~ N(0, sigma^2) drawn in that order,
    C = (A + iB)/sqrt(2), return (C + C^H)/sqrt(2)."""
    A = rng.normal(0.0, sigma, size=(D, D))
    B = rng.normal(0.0, sigma, size=(D, D))
    C = (A + 1j * B) / math.sqrt(2.0)
    return (C + C.conj().T) / math.sqrt(2.0)


def time_grid(t_end: float, T: int) -> np.ndarray:
    """T inclusive uniform times in [0, t_end]."""
    return np.linspace(0.0, t_end, T)


def tls_problem(w0: float, Omega: float, w: float, N: int) -> Problem:
    """Two-level atom H = (w0/2) sz + (Omega/2) sx cos(w t).

    The drive (Omega/2) sx cos(w t) has Fourier coefficient V = (Omega/4) sx."""
    sx = np.array([[0, 1], [1, 0]], np.complex128)
    E = np.diag([w0 / 2.0, -w0 / 2.0]).astype(np.complex128)
    return Problem(E=E, omega=[w], N=[N], axis=[0], harm=[1],
                   V=[(Omega / 4.0) * sx], name=f"tls_w{w}_N{N}")


def dressed_qubit(omega_P: float, Omega_X: float = 0.025, omega_D: float = 1.0, Omega_Px: float = 0.005,
                  Omega_Pz: float = 0.025, omega0: float = 1.0, N=(4, 12)) -> Problem:
    """Bichromatically driven qubit of Sec. 4.1 (Eq. 8, S = sigma / 2, all
    phases zero): H = omega0 S_z + Omega_X cos(omega_D t) S_x
    + cos(omega_P t) (Omega_Px S_x + Omega_Pz S_z).  Fundamental 0 is the
    dressing drive (omega_D), fundamental 1 the probe (omega_P); truncations
    N = (N_D, N_P).  Defaults: the figure's parameters (Omega_X = 0.025,
    resonant dressing omega_D = omega0 = 1, Omega_Px = 0.005, Omega_Pz = 0.025)."""
    Sx = 0.5 * np.array([[0, 1], [1, 0]], np.complex128)
    Sz = 0.5 * np.array([[1, 0], [0, -1]], np.complex128)
    return Problem(E=omega0 * Sz, omega=[omega_D, omega_P], N=list(N), axis=[0, 1], harm=[1, 1],
                   V=[(Omega_X / 2.0) * Sx, (Omega_Px / 2.0) * Sx + (Omega_Pz / 2.0) * Sz],
                   name=f"dressed_qubit_wP{omega_P:.5f}")


def lattice_problem(omega: float, D: int = 256, V0: float = 0.25, t: float = 0.125, V: float = 0.0625,
                    phi: float = 0.0, N: int = 10) -> Problem:
    """Driven 1-D lattice of Sec. 4.2 (its unnumbered lattice Hamiltonian): D sites (D/2 two-site cells)
    with on-site energies (-1)^m V0 (m = 1..D), static hopping
    t exp(i cos(2 pi m / D)) from site m+1 to site m, and a uniform hopping
    modulation V cos(omega t + phi) on every bond.  The drive's Fourier
    coefficient is (V/2) e^{i phi} times the bond matrix.  Defaults: the
    figure's parameters D = 256, V0 = 0.25, t = 0.125, V = 0.0625, phi = 0,
    truncation +-10 (Floquet dimension 5376)."""
    m = np.arange(1, D + 1)
    E = np.diag(((-1.0) ** m) * V0).astype(np.complex128)
    B = np.zeros((D, D), np.complex128)
    for k in range(1, D):                      # bond between sites k and k+1 (1-based)
        h = t * np.exp(1j * np.cos(2.0 * np.pi * k / D))
        E[k - 1, k] = h
        E[k, k - 1] = np.conj(h)
        B[k - 1, k] = 1.0
        B[k, k - 1] = 1.0
    Vk = (V / 2.0) * np.exp(1j * phi) * B
    return Problem(E=E, omega=[omega], N=[N], axis=[0], harm=[1], V=[Vk],
                   name=f"lattice_D{D}_w{omega:.4f}_N{N}")


def lattice_sweep(count: int = 64, lo: float = 0.2, hi: float = 1.0, D: int = 256, N: int = 10):
    """Frequency scan of the driven lattice: `count` drive frequencies
    uniform in [lo, hi] (the quasienergy-versus-frequency plot of Sec. 4.2)."""
    return [lattice_problem(float(w), D=D, N=N) for w in np.linspace(lo, hi, count)]


def cfg1_tls() -> tuple[Problem, np.ndarray, float]:
    """Two-level system w0 = 1, one drive (Omega/2) sx cos(w t), Omega = 0.2,
    w = 1.1, truncation +-20 (Floquet dimension 82); 100 uniform times in
    [0, 20 pi / w], t0 = 0."""
    p = tls_problem(1.0, 0.2, 1.1, 20)
    p.name = "tls_N20_M82"
    return p, time_grid(20.0 * math.pi / 1.1, 100), 0.0


def _ladder(rng, D, top):
    return np.diag(np.sort(rng.uniform(0.0, top, size=D))).astype(np.complex128)


def cfg2_large(seed: int = 2, N=(25, 25), T: int = 256) -> tuple[Problem, np.ndarray, float]:
    """8-level ladder (level energies uniform in [0,10), sorted), two
    incommensurate drives w = (1, golden ratio), random Hermitian couplings
    C_l = GUE(8, 0.3) (cos amplitudes, so V_l = C_l / 2), truncations +-25 on
    both axes: Floquet dimension 8*51*51 = 20808.  256 times in [0, 20 pi]."""
    rng = np.random.default_rng(seed)
    D = 8
    E = _ladder(rng, D, 10.0)
    C0 = gue(rng, D, 0.3)
    C1 = gue(rng, D, 0.3)
    w = np.array([1.0, (1.0 + math.sqrt(5.0)) / 2.0])
    p = Problem(E=E, omega=w, N=list(N), axis=[0, 1], harm=[1, 1],
                V=[C0 / 2.0, C1 / 2.0], name=f"ladder8_2drive_N{N[0]}x{N[1]}")
    return p, time_grid(20.0 * math.pi / w[0], T), 0.0


def cfg4_precision(seed: int = 4, N=(25, 25), T: int = 256) -> tuple[Problem, np.ndarray, float]:
    """16-level random spectrum in [0,20), two drives w = (1, sqrt 2),
    couplings C_l = GUE(16, 0.5), V_l = C_l/2, truncations +-25: dimension 41616."""
    rng = np.random.default_rng(seed)
    D = 16
    E = _ladder(rng, D, 20.0)
    C0 = gue(rng, D, 0.5)
    C1 = gue(rng, D, 0.5)
    w = np.array([1.0, math.sqrt(2.0)])
    p = Problem(E=E, omega=w, N=list(N), axis=[0, 1], harm=[1, 1],
                V=[C0 / 2.0, C1 / 2.0], name=f"spec16_2drive_N{N[0]}x{N[1]}")
    return p, time_grid(20.0 * math.pi / w[0], T), 0.0


def one_drive_band(seed: int = 6, D: int = 16, N: int = 650, T: int = 256) -> tuple[Problem, np.ndarray, float]:
    """16-level random spectrum in [0,20) under one strong drive w = 1 with a
    coupling C = GUE(16, 2.0) (V = C/2) and its second harmonic C2 = GUE(16,
    0.5) (V2 = C2/2), truncation +-650 (strong driving needs many photon
    blocks): dimension 16*1301 = 20816, a banded Floquet matrix of half-width
    16*2 + 15 = 47 in the block order of App. A.  256 times in [0, 20 pi]."""
    rng = np.random.default_rng(seed)
    E = _ladder(rng, D, 20.0)
    C1 = gue(rng, D, 2.0)
    C2 = gue(rng, D, 0.5)
    p = Problem(E=E, omega=np.array([1.0]), N=[N, ], axis=[0, 0], harm=[1, 2],
                V=[C1 / 2.0, C2 / 2.0], name=f"spec{D}_1drive_N{N}")
    return p, time_grid(20.0 * math.pi, T), 0.0


def _scaled_gue(rng, D, a):
    G = gue(rng, D, 1.0)
    return a * G / np.linalg.norm(G, 2)


def cfg3_batch(seed: int = 3, count: int = 512, max_dim: int = 2000, T: int = 32):
    """Seeded parameter sweep of `count` independent solves of uneven size.

    D ~ U{2..8}; K ~ U{1,2,3} couplings: K=1 -> one axis; K=2 -> two axes
    (h=1 each); K=3 -> two axes plus the second harmonic of axis 0 (whose
    fundamental is then drawn in [0.5, 1.5] so that 2 w_0 <= 3).  w_l ~ U[0.5,3],
    amplitudes a_k ~ U[0.01, 1] with C_k = a_k G/||G||_2, G = GUE(D,1),
    V_k = C_k/2, E = diag(sort(U[0,3)^D)), N_l ~ U{5..15}; redraw while the
    Floquet dimension exceeds max_dim.  Each solve carries T times in
    [0, 20 pi / w_0]."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        D = int(rng.integers(2, 9))
        K = int(rng.integers(1, 4))
        F = min(K, 2)
        Ns = [int(rng.integers(5, 16)) for _ in range(F)]
        M = D
        for n in Ns:
            M *= 2 * n + 1
        if M > max_dim:
            continue
        hi0 = 1.5 if K == 3 else 3.0
        w = [float(rng.uniform(0.5, hi0))] + [float(rng.uniform(0.5, 3.0)) for _ in range(F - 1)]
        E = _ladder(rng, D, 3.0)
        axes = [0, 1, 0][:K] if F == 2 else [0]
        harms = [1, 1, 2][:K] if F == 2 else [1]
        Vs = []
        for _ in range(K):
            a = float(rng.uniform(0.01, 1.0))
            Vs.append(_scaled_gue(rng, D, a) / 2.0)
        p = Problem(E=E, omega=w, N=Ns, axis=axes, harm=harms, V=Vs,
                    name=f"batch{len(out)}_D{D}_K{K}")
        out.append((p, time_grid(20.0 * math.pi / w[0], T), 0.0))
    return out


def cfg3_uniform_sweep(count: int = 512, N: int = 8, T: int = 32):
    """Uniform sweep of a driven qubit: w0 = 1, (Omega/2) sx cos(w t) with
    Omega = 2, w = 0.2 + 2 m / count, truncation N (dimension 2(2N+1))."""
    out = []
    for m in range(count):
        w = 0.2 + 2.0 * m / count
        p = tls_problem(1.0, 2.0, w, N)
        out.append((p, time_grid(32.0 * math.pi / w, T), 0.0))
    return out


def cfg5_serving(seed: int = 5, R: int = 2000, rate: float = 200.0,
                 lo: int = 50, hi: int = 12000, T: int = 32):
    """Poisson stream of solve requests: inter-arrival ~ Exp(1/rate); target
    dimension M* ~ logU[lo, hi]; D ~ U{2..16}; F ~ U{1,2,3}; L = odd-rounded
    (M*/D)^(1/F) (L >= 3), N_l = (L-1)/2, M = D L^F; D, F redrawn (keeping M*)
    until M lies in [lo, hi].  One h=1 coupling per axis with C = a GUE/||.||_2,
    a ~ U[0.01,1], w ~ U[0.5,3], E = diag(sort(U[0,3)^D)).  Returns a list of
    (arrival_time_s, problem, times, t0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(R):
        t += float(rng.exponential(1.0 / rate))
        Mt = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        while True:
            D = int(rng.integers(2, 17))
            F = int(rng.integers(1, 4))
            L = (Mt / D) ** (1.0 / F)
            L = max(3, int(2 * round((L - 1) / 2) + 1))
            M = D * L ** F
            if lo <= M <= hi:
                break
        w = [float(rng.uniform(0.5, 3.0)) for _ in range(F)]
        E = _ladder(rng, D, 3.0)
        Vs = []
        for _ in range(F):
            a = float(rng.uniform(0.01, 1.0))
            Vs.append(_scaled_gue(rng, D, a) / 2.0)
        N = [(L - 1) // 2] * F
        p = Problem(E=E, omega=w, N=N, axis=list(range(F)), harm=[1] * F, V=Vs,
                    name=f"req{r}_D{D}_F{F}_L{L}")
        out.append((t, p, time_grid(20.0 * math.pi / w[0], T), 0.0))
    return out


def random_problem(D: int, N, K: int | None = None, seed: int = 0, amp: float = 0.3,
                   spread: float = 3.0, harmonics=None) -> Problem:
    """Generic random problem for tests: F = len(N) axes, one h=1 coupling per
    axis unless `harmonics` (list of (axis, h)) is given; E a random Hermitian
    matrix (not diagonal) with spectrum of width ~spread; couplings GUE(D, amp)/2
    plus a random non-Hermitian part so that V != V^H is exercised."""
    rng = np.random.default_rng(seed)
    N = list(N)
    F = len(N)
    if harmonics is None:
        harmonics = [(l, 1) for l in range(F)]
    if K is not None:
        harmonics = harmonics[:K]
    E = np.diag(np.sort(rng.uniform(0.0, spread, size=D))).astype(np.complex128) + 0.1 * gue(rng, D, 1.0)
    w = np.sort(rng.uniform(0.7, 2.5, size=F))[::-1].copy() if F else np.zeros(0)
    Vs = []
    for _ in harmonics:
        H = gue(rng, D, amp) / 2.0
        X = 0.3 * amp * (rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D)))
        Vs.append(H + X)
    axes = [a for a, _ in harmonics]
    hs = [h for _, h in harmonics]
    return Problem(E=E, omega=w, N=N, axis=axes, harm=hs, V=Vs if Vs else np.zeros((0, D, D)),
                   name=f"rand_D{D}_N{'x'.join(map(str, N))}_s{seed}")
