"""CPU oracle for the multimode Floquet hot path (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the GPU library: it imports nothing
from it, and the GPU library imports nothing from here.

Every function states the passage of the paper (G. A. Sinuco-Leon, "OPENMMF: a
library for multimode driven quantum systems", arXiv:2005.03426) it follows.
Units: hbar = 1.

Model (Sec. 2, Eq. 1):
    H(t) = E + sum_k [ V_k e^{+i h_k w_{l_k} t} + V_k^H e^{-i h_k w_{l_k} t} ]
with harmonic couplings k given by (axis l_k, harmonic h_k >= 1, matrix V_k).

Floquet matrix (Eq. 6 with the conjugate-term index read as U^{n-m}; block
layout of Appendix A):
    H_F[(i,n),(j,m)] = H^{[n-m]}_{ij} + delta_{nm} delta_{ij} (n . w)
with H^{[0]} = E, H^{[+h e_l]} = sum of V_k with (l_k, h_k) = (l, h),
H^{[-h e_l]} = sum of V_k^H over the same k, and zero for any other offset.
Rows are ordered r = i + D s with the site index
    s = sum_l (N_l - n_l) prod_{l' < l} (2 N_{l'} + 1)
(descending n, fundamental 0 innermost), which puts H_0 + N w_1 in the top
block and V above the block diagonal exactly as Appendix A prints it.

Sign convention: the paper writes the micromotion series with e^{-i n.w t}
and the diagonal E - n.w (Eqs. 5-6); substituting n -> -n gives the same
matrix with E + n.w, used here, paired with U_F(t) = sum_n Phi^n e^{+i n.w t}.
The brute-force Schroedinger integration (`rk4_evolve`) fixes this pairing.

Parity status: every function below is pinned by the CPU tests (closed forms,
invariants, brute force, the Appendix-A layout); none is "parity unpinned".
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "sites", "floquet_dim", "floquet_entry", "build_floquet", "eigh", "site_phases",
    "evolve", "evolve_expm", "micromotion_select", "micromotion", "avg_prob",
    "hamiltonian_at", "rk4_evolve", "jacobi_eigh", "householder_tridiag_apply",
    "zero_site", "tridiag_eigh", "quasienergies", "restrict_modes", "dressed_evolution",
    "spin_ops", "spin_drive", "avg_prob_degenerate", "evolve_expm_sparse",
    "build_floquet_sparse", "quasienergies_near", "eigvalsh",
]


# ---------------------------------------------------------------------------
# Index set of the truncated Fourier expansion (Sec. 2 after Eq. 6; App. A)
# ---------------------------------------------------------------------------
def sites(N) -> np.ndarray:
    """Fourier index vectors n (one row per site s), in site order.

    Truncation n_l in [-N_l, N_l] (the "number of Floquet manifolds" of each
    fundamental, App. A uses N_F = 3 -> 7 blocks per axis).  Site s decodes as
    a mixed-radix number, digit q_l = (N_l - n_l) with radix 2 N_l + 1 and
    axis 0 the least significant digit."""
    N = [int(x) for x in N]
    F = len(N)
    S = 1
    for n in N:
        S *= 2 * n + 1
    out = np.zeros((S, F), dtype=np.int64)
    for s in range(S):
        rem = s
        for l in range(F):
            L = 2 * N[l] + 1
            q = rem % L
            rem //= L
            out[s, l] = N[l] - q
    return out


def zero_site(N) -> int:
    """Site index of n = 0 (each digit q_l = N_l)."""
    s, stride = 0, 1
    for n in N:
        s += int(n) * stride
        stride *= 2 * int(n) + 1
    return s


def floquet_dim(p) -> int:
    """M = D * prod_l (2 N_l + 1)."""
    return p.D * len(sites(p.N))


def _offset_block(p, delta):
    """H^{[delta]} of the definition above, or None when it is zero.

    delta is the integer vector n - m.  Couplings sharing (axis, h) are
    summed in ascending k."""
    nz = [l for l in range(len(delta)) if delta[l] != 0]
    if not nz:
        return p.E.copy()
    if len(nz) != 1:
        return None
    l = nz[0]
    d = int(delta[l])
    blk = None
    for k in range(p.K):
        if int(p.axis[k]) != l:
            continue
        h = int(p.harm[k])
        if d == h:
            term = p.V[k]
        elif d == -h:
            term = p.V[k].conj().T
        else:
            continue
        blk = term.copy() if blk is None else blk + term
    return blk


def _diag_shift(E_ii: float, n, omega) -> float:
    """E_ii + n . w as the chain ((E_ii + n_0 w_0) + n_1 w_1) + ... in FP64,
    each product n_l * w_l rounded once (ascending l)."""
    x = float(E_ii)
    for l in range(len(n)):
        x = x + float(n[l]) * float(omega[l])
    return x


def floquet_entry(p, r: int, c: int) -> complex:
    """One element H_F[r, c] straight from the definition (Eq. 6, App. A).

    Used to check sampled entries of full-size matrices one by one."""
    D = p.D
    N = [int(x) for x in p.N]
    i, sr = r % D, r // D
    j, sc = c % D, c // D

    def dec(s):
        v = []
        for n in N:
            L = 2 * n + 1
            v.append(n - s % L)
            s //= L
        return v
    nr, nc = dec(sr), dec(sc)
    delta = [a - b for a, b in zip(nr, nc)]
    blk = _offset_block(p, delta)
    if blk is None:
        return 0j
    val = complex(blk[i, j])
    if all(x == 0 for x in delta) and i == j:
        val = complex(_diag_shift(val.real, nr, p.omega), val.imag)
    return val


def build_floquet(p) -> np.ndarray:
    """Dense truncated Floquet matrix H_F (M x M complex128), Eq. 6 / App. A.

    Row site loop; for each row site the only nonzero column sites are the
    site itself (block E + n.w) and its neighbours at offsets +-h e_l of the
    couplings (blocks V, V^H), as the definition states."""
    n = sites(p.N)
    S, F, D = n.shape[0], n.shape[1], p.D
    M = D * S
    index = {tuple(v): s for s, v in enumerate(n.tolist())}
    offsets = [tuple([0] * F)]
    for k in range(p.K):
        for sgn in (+1, -1):
            o = [0] * F
            o[int(p.axis[k])] = sgn * int(p.harm[k])
            if tuple(o) not in offsets:
                offsets.append(tuple(o))
    H = np.zeros((M, M), dtype=np.complex128)
    for sr in range(S):
        for o in offsets:
            m = tuple(int(a) - b for a, b in zip(n[sr], o))   # delta = n - m = o
            sc = index.get(m)
            if sc is None:
                continue
            blk = _offset_block(p, o)
            if blk is None:
                continue
            blk = blk.copy()
            if all(x == 0 for x in o):
                for i in range(D):
                    blk[i, i] = complex(_diag_shift(blk[i, i].real, n[sr], p.omega), blk[i, i].imag)
            H[D * sr:D * sr + D, D * sc:D * sc + D] = blk
    return H


# ---------------------------------------------------------------------------
# Dense Hermitian eigensolve (the paper delegates it to LAPACK, Sec. 3.2)
# ---------------------------------------------------------------------------
def build_floquet_sparse(p):
    """The same truncated H_F (Eq. 6 / App. A) as a SciPy CSR matrix, for
    orders whose dense form would not fit the host comfortably.  The same
    row-site loop as `build_floquet`: each row site's nonzero column sites
    are itself (block E + n.w) and its neighbours at the couplings' offsets
    +-h e_l (blocks V, V^H); every stored block entry is kept, zeros
    included, so the values equal the dense form's entry for entry."""
    from scipy.sparse import csr_matrix
    n = sites(p.N)
    S, F, D = n.shape[0], n.shape[1], p.D
    M = D * S
    index = {tuple(v): s for s, v in enumerate(n.tolist())}
    offsets = [tuple([0] * F)]
    for k in range(p.K):
        for sgn in (+1, -1):
            o = [0] * F
            o[int(p.axis[k])] = sgn * int(p.harm[k])
            if tuple(o) not in offsets:
                offsets.append(tuple(o))
    blocks = {o: _offset_block(p, o) for o in offsets}
    ii = np.repeat(np.arange(D), D)
    jj = np.tile(np.arange(D), D)
    rows, cols, vals = [], [], []
    for sr in range(S):
        for o in offsets:
            m = tuple(int(a) - b for a, b in zip(n[sr], o))   # delta = n - m = o
            sc = index.get(m)
            blk = blocks[o]
            if sc is None or blk is None:
                continue
            blk = blk.copy()
            if all(x == 0 for x in o):
                for i in range(D):
                    blk[i, i] = complex(_diag_shift(blk[i, i].real, n[sr], p.omega), blk[i, i].imag)
            rows.append(D * sr + ii)
            cols.append(D * sc + jj)
            vals.append(blk.reshape(-1))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals).astype(np.complex128)
    return csr_matrix((v, (r, c)), shape=(M, M))


def quasienergies_near(H, sigma: float, k: int) -> np.ndarray:
    """The k eigenvalues of the Hermitian (sparse) H_F closest to sigma,
    ascending, for spot checks of spectra too large for a full
    diagonalisation: shift-invert Arnoldi through SciPy's ARPACK interface,
    the inverse of H_F - sigma I applied by LAPACK's banded LU (H_F is
    banded: its nonzero blocks sit at most one coupling offset from the
    diagonal in the site order)."""
    from scipy.linalg import lapack
    from scipy.sparse import coo_matrix
    from scipy.sparse.linalg import LinearOperator, eigsh
    A = coo_matrix(H)
    M = A.shape[0]
    kl = int(max(0, (A.row - A.col).max()))
    ku = int(max(0, (A.col - A.row).max()))
    ab = np.zeros((2 * kl + ku + 1, M), dtype=np.complex128)
    ab[kl + ku + A.row - A.col, A.col] = A.data
    ab[kl + ku, :] -= sigma
    lu, piv, info = lapack.zgbtrf(ab, kl, ku)
    if info != 0:
        raise ValueError(f"shift {sigma} is an eigenvalue to working precision (zgbtrf info {info})")

    def solve(x):
        y, inf = lapack.zgbtrs(lu, kl, ku, np.asarray(x, dtype=np.complex128).reshape(M, -1), piv)
        return y

    op = LinearOperator((M, M), matvec=solve, dtype=np.complex128)
    w = eigsh(A.tocsr(), k=k, sigma=sigma, which="LM", OPinv=op, return_eigenvectors=False, tol=0.0)
    return np.sort(np.asarray(w).real.astype(np.float64))


def eigh(H: np.ndarray):
    """Eigenvalues (ascending) and orthonormal eigenvectors (columns) of the
    Hermitian H_F: LAPACK zheevd through NumPy, the library routine the
    paper's wrapper calls (Sec. 3.2)."""
    w, Phi = np.linalg.eigh(H)
    return w, Phi


def eigvalsh(H: np.ndarray) -> np.ndarray:
    """All eigenvalues (ascending) of a Hermitian matrix, without eigenvectors:
    LAPACK's eigenvalue-only Hermitian solver through NumPy (the paper's
    LAPACK_FULLEIGENVALUES call, Sec. 3.2)."""
    return np.linalg.eigvalsh(H)


def quasienergies(p) -> np.ndarray:
    """All eigenvalues (ascending) of the truncated H_F, without eigenvectors
    (the paper's LAPACK_FULLEIGENVALUES call on the Floquet matrix, Sec. 4.2)."""
    return eigvalsh(build_floquet(p))


def jacobi_eigh(H: np.ndarray, sweeps: int = 30, tol: float = 1e-15):
    """Cyclic complex Jacobi eigensolver (textbook method), for small matrices.

    Each rotation first removes the phase of a_pq with a diagonal unitary,
    then applies the real symmetric Jacobi rotation that zeroes the now-real
    2x2 off-diagonal.  Used to pin `eigh` independently of LAPACK."""
    A = np.array(H, dtype=np.complex128, copy=True)
    n = A.shape[0]
    V = np.eye(n, dtype=np.complex128)
    scale = max(np.linalg.norm(A), 1e-300)
    for _ in range(sweeps):
        off = math.sqrt(max(np.linalg.norm(A) ** 2 - np.sum(np.abs(np.diag(A)) ** 2), 0.0))
        if off <= tol * scale:
            break
        for p_ in range(n - 1):
            for q in range(p_ + 1, n):
                apq = A[p_, q]
                r = abs(apq)
                if r <= 1e-300:
                    continue
                ph = apq / r                            # a_pq = r e^{i phi}
                app, aqq = A[p_, p_].real, A[q, q].real
                theta = (aqq - app) / (2.0 * r)
                t = (1.0 if theta >= 0 else -1.0) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                # J = diag(1, conj(ph)) . [[c, s], [-s, c]] on columns p, q
                J = np.array([[c, s], [-s * np.conj(ph), c * np.conj(ph)]], dtype=np.complex128)
                cols = A[:, [p_, q]] @ J
                A[:, p_], A[:, q] = cols[:, 0], cols[:, 1]
                rows = J.conj().T @ A[[p_, q], :]
                A[p_, :], A[q, :] = rows[0], rows[1]
                A[p_, q] = A[q, p_] = 0.0
                vc = V[:, [p_, q]] @ J
                V[:, p_], V[:, q] = vc[:, 0], vc[:, 1]
    w = np.diag(A).real.copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def householder_tridiag_apply(d, e, refl, tau):
    """Rebuild Q from Householder reflectors and the tridiagonal T = Q^H A Q.

    refl[:, i] holds v_i (v_i[i+1] = 1, zeros above), Q = H_0 H_1 ... with
    H_i = I - tau_i v_i v_i^H.  Returns (Q, T) with T real symmetric
    tridiagonal from d (diagonal) and e (off-diagonal).  Used to check a
    tridiagonal reduction by its defining identity A = Q T Q^H."""
    n = len(d)
    Q = np.eye(n, dtype=np.complex128)
    for i in range(n - 1):
        v = refl[:, i]
        Hi = np.eye(n, dtype=np.complex128) - tau[i] * np.outer(v, v.conj())
        Q = Q @ Hi
    T = np.diag(np.asarray(d, float)) + np.diag(np.asarray(e, float), 1) + np.diag(np.asarray(e, float), -1)
    return Q, T


# ---------------------------------------------------------------------------
# Time evolution and micromotion (Eqs. 3-5)
# ---------------------------------------------------------------------------
def site_phases(p, t: float) -> np.ndarray:
    """e^{+i n_s . w t} for every site s (the Fourier factors of Eq. 5 in the
    sign convention stated in the module docstring)."""
    n = sites(p.N).astype(np.float64)
    return np.exp(1j * (n @ p.omega) * t)


def evolve(p, Phi: np.ndarray, eps: np.ndarray, t0: float, ts) -> np.ndarray:
    """Bare-basis time-evolution operators U(t, t0) for every t in ts.

    Eqs. 3-5 written over all M eigenpairs of H_F (the extended-space form
    the paper cites, Sec. 2 after Eq. 6):
        U_ij(t, t0) = sum_n e^{i n.w t} sum_a Phi[(i,n),a] e^{-i eps_a (t-t0)} conj(Phi[(j,0),a])
    Returns U with U[tau, i, j] (i final, j initial)."""
    D = p.D
    M = Phi.shape[0]
    S = M // D
    Phi3 = Phi.reshape(S, D, M)                 # row r = i + D s
    Phi0 = Phi3[zero_site(p.N)]                 # (D, M): rows of the n = 0 block
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    U = np.zeros((len(ts), D, D), dtype=np.complex128)
    for q, t in enumerate(ts):
        B = site_phases(p, t)                   # (S,)
        A = np.einsum("s,sia->ia", B, Phi3)     # (D, M)
        ph = np.exp(-1j * eps * (t - t0))       # (M,)
        U[q] = (A * ph[None, :]) @ Phi0.conj().T
    return U


def evolve_expm(p, H: np.ndarray, t0: float, ts) -> np.ndarray:
    """Same object as `evolve` with no eigendecomposition: the propagator
    exp(-i H_F (t - t0)) applied to the n = 0 block columns, then the Fourier
    sum over sites."""
    from scipy.linalg import expm
    D = p.D
    M = H.shape[0]
    S = M // D
    s0 = zero_site(p.N)
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    U = np.zeros((len(ts), D, D), dtype=np.complex128)
    for q, t in enumerate(ts):
        G = expm(-1j * H * (t - t0))[:, D * s0:D * s0 + D]      # (M, D)
        B = site_phases(p, t)
        U[q] = np.einsum("s,sij->ij", B, G.reshape(S, D, D))
    return U


def evolve_expm_sparse(p, H: np.ndarray, t0: float, ts) -> np.ndarray:
    """`evolve_expm` for large truncations: H_F is sparse (at most D (1 + 2K)
    nonzeros per row), so exp(-i H_F (t - t0)) is applied to the D columns
    of the n = 0 block by SciPy's action-of-the-exponential routine (the
    truncated Taylor method of Al-Mohy and Higham, 2011) on a sparse copy of
    H_F, then the same Fourier sum over sites."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.linalg import expm_multiply
    D = p.D
    M = H.shape[0]
    S = M // D
    s0 = zero_site(p.N)
    Hs = csr_matrix(H)
    B0 = np.zeros((M, D), dtype=np.complex128)
    B0[D * s0:D * s0 + D, :] = np.eye(D)
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    U = np.zeros((len(ts), D, D), dtype=np.complex128)
    for q, t in enumerate(ts):
        G = expm_multiply(-1j * (t - t0) * Hs, B0)                # (M, D)
        B = site_phases(p, t)
        U[q] = np.einsum("s,sij->ij", B, G.reshape(S, D, D))
    return U


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def micromotion_select(p, Phi: np.ndarray, eps: np.ndarray):
    """Pick one eigenvector per w-translation orbit (Eq. 5 needs D of them).

    Fourier centre of mass c_a = sum_n n sum_i |Phi[(i,n),a]|^2 (F-vector);
    keep the eigenvectors whose centre rounds (half away from zero) to the
    zero vector; if more than D qualify keep the D of smallest |eps_a|, ties
    by lower index.  Returns the selected column indices in ascending order,
    or raises when fewer than D qualify (truncation not converged)."""
    D = p.D
    M = Phi.shape[0]
    S = M // D
    n = sites(p.N).astype(np.float64)           # (S, F)
    w = (np.abs(Phi) ** 2).reshape(S, D, M).sum(axis=1)   # (S, M) site weights
    c = n.T @ w                                             # (F, M)
    ok = np.all(_round_half_away(c) == 0, axis=0) if n.shape[1] else np.ones(M, bool)
    cand = np.nonzero(ok)[0]
    if len(cand) < D:
        raise ValueError(f"micromotion: only {len(cand)} orbit representatives found, need {D}")
    if len(cand) > D:
        key = sorted(cand.tolist(), key=lambda a: (abs(float(eps[a])), a))
        cand = np.array(sorted(key[:D]))
    return cand


def micromotion(p, Phi: np.ndarray, eps: np.ndarray, ts):
    """Micromotion operator U_F(t) (Eq. 5): U_F(t)_{i b} = sum_n Phi[(i,n),b] e^{i n.w t}
    over the D selected representatives b; returns (UF[tau, i, b], eps_sel[b])."""
    sel = micromotion_select(p, Phi, eps)
    D = p.D
    M = Phi.shape[0]
    S = M // D
    Phi3 = Phi[:, sel].reshape(S, D, D)
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    UF = np.zeros((len(ts), D, D), dtype=np.complex128)
    for q, t in enumerate(ts):
        UF[q] = np.einsum("s,sib->ib", site_phases(p, t), Phi3)
    return UF, eps[sel].copy()


# ---------------------------------------------------------------------------
# Evolution in a dressed basis (Sec. 4.1, DRESSEDBASIS_SUBSET + Eq. 4)
# ---------------------------------------------------------------------------
class _Restricted:
    pass


def restrict_modes(p, axes):
    """The problem with only the fundamentals in `axes` kept (in that order):
    the static Hamiltonian plus the couplings oscillating on those axes (the
    paper's subset of dressing modes, which always includes the static mode)."""
    q = _Restricted()
    q.E = np.asarray(p.E, dtype=np.complex128)
    q.D = q.E.shape[0]
    new_index = {int(a): i for i, a in enumerate(axes)}
    q.omega = [float(p.omega[int(a)]) for a in axes]
    q.N = [int(p.N[int(a)]) for a in axes]
    q.axis, q.harm, q.V = [], [], []
    for k in range(len(p.axis)):
        a = int(p.axis[k])
        if a in new_index:
            q.axis.append(new_index[a])
            q.harm.append(int(p.harm[k]))
            q.V.append(np.asarray(p.V[k], dtype=np.complex128))
    q.F = len(q.omega)
    q.K = len(q.axis)
    return q


def dressed_evolution(p, axes, ts, t0: float):
    """U_dressed(t, t0) = U_F^sub(t)^H U(t, t0) U_F^sub(t0): the bare evolution
    of the full problem (Shirley form over all its eigenpairs) seen in the
    dressed basis of the subset `axes` (micromotion operator of the subset's
    Floquet problem, one representative per orbit).  Returns
    (Ud[tau, i, j], U[tau, i, j], eps_dressed)."""
    sub = restrict_modes(p, axes)
    Hs = build_floquet(sub)
    ws, Phis = eigh(Hs)
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    UF, eps_d = micromotion(sub, Phis, ws, np.concatenate([ts, [t0]]))
    H = build_floquet(p)
    w, Phi = eigh(H)
    U = evolve(p, Phi, w, t0, ts)
    Ud = np.zeros_like(U)
    for q in range(len(ts)):
        Ud[q] = UF[q].conj().T @ U[q] @ UF[-1]
    return Ud, U, eps_d


# ---------------------------------------------------------------------------
# Spin couplings (Sec. 3.4, Eq. 7)
# ---------------------------------------------------------------------------
def spin_ops(s: float):
    """(S_x, S_y, S_z) of spin s from the matrix elements of the standard
    angular-momentum algebra, basis ordered m = s, s-1, ..., -s:
        <m +- 1| S_x |m> = sqrt((s -+ m)(s +- m + 1)) / 2,
        <m +- 1| S_y |m> = -+ i sqrt((s -+ m)(s +- m + 1)) / 2,   <m|S_z|m> = m."""
    D = int(round(2 * s)) + 1
    ms = [s - k for k in range(D)]
    Sx = np.zeros((D, D), complex)
    Sy = np.zeros((D, D), complex)
    Sz = np.zeros((D, D), complex)
    for c, m in enumerate(ms):
        Sz[c, c] = m
        for r, mp in enumerate(ms):
            if abs(mp - (m + 1)) < 1e-9:
                a = math.sqrt((s - m) * (s + m + 1)) / 2.0
                Sx[r, c] += a
                Sy[r, c] += -1j * a
            elif abs(mp - (m - 1)) < 1e-9:
                a = math.sqrt((s + m) * (s - m + 1)) / 2.0
                Sx[r, c] += a
                Sy[r, c] += 1j * a
    return Sx, Sy, Sz


def spin_drive(S, amplitudes, phases):
    """Fourier coefficient of sum_i A_i cos(w t + phi_i) S_i (Eq. 7 read with
    an imaginary exponent and axes x, y, z; cos amplitude -> half, as R8)."""
    return sum(0.5 * a * np.exp(1j * ph) * Si for a, ph, Si in zip(amplitudes, phases, S))


# ---------------------------------------------------------------------------
# Time- and phase-averaged transition probability (MULTIMODETRANSITIONAVG)
# ---------------------------------------------------------------------------
def avg_prob(p, Phi: np.ndarray) -> np.ndarray:
    """P[i, j] = long-time and drive-phase average of |U_ij(t, t0)|^2.

    Averaging the eigen expansion of `evolve` over t - t0 and t0 keeps only
    the diagonal terms of a nondegenerate spectrum:
        P[i, j] = sum_a ( sum_n |Phi[(i,n),a]|^2 ) |Phi[(j,0),a]|^2 ."""
    D = p.D
    M = Phi.shape[0]
    S = M // D
    A2 = (np.abs(Phi) ** 2).reshape(S, D, M)
    W = A2.sum(axis=0)                          # (D, M)
    Z = A2[zero_site(p.N)]                      # (D, M)
    return W @ Z.T


def avg_prob_degenerate(p, Phi: np.ndarray, eps, rel: float = 1e-8, shared: float = 1e-20) -> bool:
    """True when `avg_prob` has no unique value for these eigenpairs.

    The time average of |U_ij|^2 drops the cross terms of a pair of
    eigenvectors a != b only if eps_a != eps_b; for a degenerate pair the
    surviving cross terms (size up to sqrt(z_a z_b), z_a the weight of
    column a on the zero Fourier site, the only site U's initial index sees)
    depend on the basis chosen inside the degenerate subspace.  Reading of
    the paper's averaged-probability routine, which also receives the
    quasienergies: a pair counts as degenerate when
    |eps_b - eps_a| <= rel * max(1, max|eps|), and it matters when
    z_a z_b > shared.  Written as a plain loop over all pairs."""
    eps = np.asarray(eps, dtype=np.float64)
    D = p.D
    s0 = zero_site(p.N)
    z = (np.abs(Phi[D * s0:D * s0 + D, :]) ** 2).sum(axis=0)
    tol = rel * max(1.0, float(np.abs(eps).max()))
    M = len(eps)
    for a in range(M):
        for b in range(a + 1, M):
            if abs(eps[b] - eps[a]) <= tol and z[a] * z[b] > shared:
                return True
    return False


# ---------------------------------------------------------------------------
# Brute-force Schroedinger integration (independent of the Floquet matrix)
# ---------------------------------------------------------------------------
def hamiltonian_at(p, t: float) -> np.ndarray:
    """H(t) of Eq. 1 in the convention of the module docstring."""
    H = p.E.astype(np.complex128).copy()
    for k in range(p.K):
        ph = np.exp(1j * int(p.harm[k]) * float(p.omega[int(p.axis[k])]) * t)
        H = H + p.V[k] * ph + p.V[k].conj().T * np.conj(ph)
    return H


def rk4_evolve(p, t0: float, ts, h: float = 1e-3) -> np.ndarray:
    """U(t, t0) from classical fourth-order Runge-Kutta on i dU/dt = H(t) U,
    U(t0) = I, with steps no longer than h (each interval [t0, t] split
    evenly).  Returns U[tau, i, j]."""
    D = p.D
    ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
    out = np.zeros((len(ts), D, D), dtype=np.complex128)
    order = np.argsort(ts)
    U = np.eye(D, dtype=np.complex128)
    tc = float(t0)

    def f(t, X):
        return -1j * (hamiltonian_at(p, t) @ X)
    for q in order:
        T = float(ts[q])
        nsteps = max(1, int(math.ceil(abs(T - tc) / h)))
        dt = (T - tc) / nsteps
        for _ in range(nsteps):
            k1 = f(tc, U)
            k2 = f(tc + dt / 2, U + dt / 2 * k1)
            k3 = f(tc + dt / 2, U + dt / 2 * k2)
            k4 = f(tc + dt, U + dt * k3)
            U = U + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
            tc += dt
        tc = T
        out[q] = U
    return out


def tridiag_eigh(d, e):
    """Eigenpairs of the real symmetric tridiagonal matrix with diagonal d and
    off-diagonal e (dense LAPACK solve of the matrix written out)."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    return np.linalg.eigh(T)
