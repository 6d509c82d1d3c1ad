"""Host-side checks that need no GPU: the library loads and exports every
symbol declared in include/mmf.h, and the host-only calls validate input."""
import ctypes as C
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mmf.h")).read()
    return sorted(set(re.findall(r"\b(mmf_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2005_03426_amd as mmf
    L = mmf.lib()
    names = _declared()
    assert "mmf_eigh" in names and "mmf_build_floquet" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mmf.EXPORTED)


def test_floquet_dim_and_argument_checks_host_only():
    import paper_2005_03426_amd as mmf
    from paper_2005_03426_amd._lib import MMFProblem
    L = mmf.lib()
    omega = np.array([1.0, 1.5]); N = np.array([3, 2], np.int32)
    axis = np.array([0, 1], np.int32); harm = np.array([1, 1], np.int32)
    dummy = C.c_void_p(16)     # device pointers are never dereferenced by host-only calls
    p = MMFProblem(4, 2, 2, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                   dummy, dummy)
    M = C.c_int64(0)
    assert L.mmf_floquet_dim(C.byref(p), C.byref(M)) == 0 and M.value == 4 * 7 * 5
    assert L.mmf_floquet_dim(None, C.byref(M)) == -1
    assert L.mmf_floquet_dim(C.byref(p), None) == -2
    bad_axis = np.array([0, 2], np.int32)
    q = MMFProblem(4, 2, 2, omega.ctypes.data, N.ctypes.data, bad_axis.ctypes.data, harm.ctypes.data,
                   dummy, dummy)
    assert L.mmf_floquet_dim(C.byref(q), C.byref(M)) == -1
    bad_h = np.array([0, 1], np.int32)
    q = MMFProblem(4, 2, 2, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, bad_h.ctypes.data,
                   dummy, dummy)
    assert L.mmf_floquet_dim(C.byref(q), C.byref(M)) == -1
    big = np.array([40000, 40000], np.int32)
    q = MMFProblem(4, 2, 2, omega.ctypes.data, big.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                   dummy, dummy)
    assert L.mmf_floquet_dim(C.byref(q), C.byref(M)) == 6      # MMF_ERR_TOO_LARGE
    b = C.c_size_t(0)
    assert L.mmf_eigh_workspace(C.c_int64(1000), 0, C.byref(b)) == 0 and b.value > 16 * 1000 * 1000
    assert L.mmf_eigh_workspace(C.c_int64(-1), 0, C.byref(b)) == -1
    assert L.mmf_eigh_workspace(C.c_int64(10), 7, C.byref(b)) == -2
    assert L.mmf_strerror(4).decode().startswith("iteration")


def test_batched_argument_checks_host_only():
    """Every argument error of mmf_eigh_batched is found before any device work."""
    import paper_2005_03426_amd as mmf
    L = mmf.lib()
    dummy = 16                                  # never dereferenced on these paths
    n = (C.c_int64 * 2)(4, 5)
    bad = (C.c_int64 * 2)(4, -1)
    Ap = (C.c_void_p * 2)(dummy, dummy)
    Anull = (C.c_void_p * 2)(dummy, None)
    wp = (C.c_void_p * 2)(dummy, dummy)
    ld = (C.c_int64 * 2)(5, 5)
    ld_bad = (C.c_int64 * 2)(5, 4)
    b = C.c_size_t(0)
    assert L.mmf_eigh_batched_workspace(C.c_int64(2), n, 0, C.byref(b)) == 0
    one = C.c_size_t(0)
    assert L.mmf_eigh_workspace(C.c_int64(5), 0, C.byref(one)) == 0
    assert b.value > one.value
    assert L.mmf_eigh_batched_workspace(C.c_int64(-1), n, 0, C.byref(b)) == -1
    assert L.mmf_eigh_batched_workspace(C.c_int64(2), bad, 0, C.byref(b)) == -2
    assert L.mmf_eigh_batched_workspace(C.c_int64(2), n, 5, C.byref(b)) == -3
    assert L.mmf_eigh_batched_workspace(C.c_int64(2), n, 0, None) == -4
    assert L.mmf_eigh_batched_workspace(C.c_int64(2), n, 0, C.byref(b)) == 0

    def call(count=2, nn=n, A=Ap, lda=ld, w=wp, prec=0, work=dummy, nbytes=None, info=dummy):
        nb = b.value if nbytes is None else nbytes
        return L.mmf_eigh_batched(C.c_int64(count), nn, A, lda, w, prec, C.c_void_p(work), C.c_size_t(nb),
                                  C.c_void_p(info), None)
    assert call(count=-1) == -1
    assert call(count=0) == 0
    assert call(nn=None) == -2
    assert call(nn=bad) == -2
    assert call(A=None) == -3
    assert call(A=Anull) == -3
    assert call(lda=ld_bad) == -4
    assert call(w=None) == -5
    assert call(prec=9) == -6
    assert call(work=0) == -7
    assert call(nbytes=b.value - 1) == -8
    assert call(info=0) == -9


def test_eigvalsh_batched_argument_checks_host_only():
    import paper_2005_03426_amd as mmf
    L = mmf.lib()
    dummy = 16
    n = (C.c_int64 * 2)(4, 5)
    Ap = (C.c_void_p * 2)(dummy, dummy)
    wp = (C.c_void_p * 2)(dummy, dummy)
    ld = (C.c_int64 * 2)(5, 5)
    b = C.c_size_t(0)
    assert L.mmf_eigvalsh_batched_workspace(C.c_int64(2), n, 0, C.byref(b)) == 0 and b.value > 0
    assert L.mmf_eigvalsh_batched_workspace(C.c_int64(2), n, 1, C.byref(b)) == -3     # refined: no
    assert L.mmf_eigvalsh_batched_workspace(C.c_int64(2), n, 2, C.byref(b)) == 0
    assert L.mmf_eigvalsh_batched_workspace(C.c_int64(2), n, 0, C.byref(b)) == 0

    def call(count=2, A=Ap, lda=ld, prec=0, nbytes=None, info=dummy):
        nb = b.value if nbytes is None else nbytes
        return L.mmf_eigvalsh_batched(C.c_int64(count), n, A, lda, wp, prec, C.c_void_p(dummy),
                                      C.c_size_t(nb), C.c_void_p(info), None)
    assert call(count=-1) == -1
    assert call(A=None) == -3
    assert call(lda=(C.c_int64 * 2)(3, 5)) == -4
    assert call(prec=1) == -6
    assert call(nbytes=b.value - 1) == -8
    assert call(info=0) == -9


def test_large_bare_dimension_limits_host_only():
    """D up to 4096 assembles and diagonalises; the D x D on-chip calls stop at 64."""
    import paper_2005_03426_amd as mmf
    from paper_2005_03426_amd._lib import MMFProblem
    L = mmf.lib()
    omega = np.array([0.5]); N = np.array([2], np.int32)
    axis = np.array([0], np.int32); harm = np.array([1], np.int32)
    dummy = C.c_void_p(16)
    M = C.c_int64(0)
    b = C.c_size_t(0)
    big = MMFProblem(256, 1, 1, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                     dummy, dummy)
    assert L.mmf_floquet_dim(C.byref(big), C.byref(M)) == 0 and M.value == 256 * 5
    assert L.mmf_avg_prob_workspace(C.byref(big), C.byref(b)) == 6          # MMF_ERR_TOO_LARGE
    assert L.mmf_evolve_workspace(C.byref(big), 4, C.byref(b)) == 6
    huge = MMFProblem(5000, 1, 1, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                      dummy, dummy)
    assert L.mmf_floquet_dim(C.byref(huge), C.byref(M)) == -1


def test_dressed_evolution_argument_checks_host_only():
    import paper_2005_03426_amd as mmf
    L = mmf.lib()
    d = C.c_void_p(16)
    assert L.mmf_dressed_evolution(0, 4, d, d, d, d, None) == -1
    assert L.mmf_dressed_evolution(65, 4, d, d, d, d, None) == -1
    assert L.mmf_dressed_evolution(2, -1, d, d, d, d, None) == -2
    assert L.mmf_dressed_evolution(2, 0, None, None, None, None, None) == 0     # nothing to do
    assert L.mmf_dressed_evolution(2, 4, None, d, d, d, None) == -3
    assert L.mmf_dressed_evolution(2, 4, d, None, d, d, None) == -4
    assert L.mmf_dressed_evolution(2, 4, d, d, None, d, None) == -5
    assert L.mmf_dressed_evolution(2, 4, d, d, d, None, None) == -6


def test_eigh_window_argument_checks_host_only():
    import paper_2005_03426_amd as mmf
    L = mmf.lib()
    d = C.c_void_p(16)
    b = C.c_size_t(0)
    assert L.mmf_eigh_window_workspace(C.c_int64(100), C.c_int64(10), C.byref(b)) == 0 and b.value > 0
    assert L.mmf_eigh_window_workspace(C.c_int64(-1), C.c_int64(10), C.byref(b)) == -1

    def call(M=100, A=d, lda=100, vl=0.0, vu=1.0, kmax=10, w=d, Z=d, ldz=100, cnt=d, work=d, nb=None, info=d):
        return L.mmf_eigh_window(C.c_int64(M), A, C.c_int64(lda), C.c_double(vl), C.c_double(vu),
                                 C.c_int64(kmax), w, Z, C.c_int64(ldz), cnt, work,
                                 C.c_size_t(b.value if nb is None else nb), info, None)
    assert call(M=-1) == -1
    assert call(A=None) == -2
    assert call(lda=99) == -3
    assert call(vl=1.0, vu=1.0) == -4
    assert call(kmax=-1) == -6
    assert call(w=None) == -7
    assert call(Z=None) == -8
    assert call(ldz=50) == -9
    assert call(cnt=None) == -10
    assert call(work=None) == -11
    assert call(nb=16) == -12
    assert call(info=None) == -13


def test_build_floquet_rejects_non_hermitian_E_host_only():
    """E is host memory in the problem statement and is validated before
    anything is enqueued: an imaginary diagonal entry or an off-diagonal pair
    that is not conjugate makes the problem invalid (-1)."""
    import paper_2005_03426_amd as mmf
    from paper_2005_03426_amd._lib import MMFProblem
    L = mmf.lib()
    omega = np.array([1.1]); N = np.array([2], np.int32)
    axis = np.array([0], np.int32); harm = np.array([1], np.int32)
    V = np.zeros((1, 2, 2), np.complex128)
    d = C.c_void_p(16)                          # never dereferenced on these paths

    def rc(E):
        Ec = np.ascontiguousarray(E.T.astype(np.complex128))
        p = MMFProblem(2, 1, 1, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                       Ec.ctypes.data, V.ctypes.data)
        b = C.c_size_t(0)
        assert L.mmf_build_floquet_workspace(C.byref(p), C.byref(b)) == 0 and b.value == 2 * 4 * 16
        return L.mmf_build_floquet(C.byref(p), d, C.c_int64(10), d, C.c_size_t(b.value), None)
    assert rc(np.array([[0.5, 0.1 + 0.2j], [0.1 - 0.2j, -0.5]])) != -1      # Hermitian: passes the check
    assert rc(np.array([[0.5 + 1e-9j, 0.0], [0.0, -0.5]])) == -1           # complex diagonal
    assert rc(np.array([[0.5, 0.1 + 0.2j], [0.1 + 0.2j, -0.5]])) == -1     # not conjugate
    assert rc(np.array([[0.5, 0.1], [0.1 + 1e-12, -0.5]])) == -1           # asymmetric beyond 1e-14
    assert rc(np.array([[0.5, 0.1], [0.1 + 1e-16, -0.5]])) != -1           # within 1e-14 max|E|
    assert rc(np.array([[np.nan, 0.0], [0.0, -0.5]])) == -1


def test_avg_prob_argument_checks_host_only():
    import paper_2005_03426_amd as mmf
    from paper_2005_03426_amd._lib import MMFProblem
    L = mmf.lib()
    omega = np.array([1.1]); N = np.array([3], np.int32)
    axis = np.array([0], np.int32); harm = np.array([1], np.int32)
    E = np.eye(2, dtype=np.complex128); V = np.zeros((1, 2, 2), np.complex128)
    p = MMFProblem(2, 1, 1, omega.ctypes.data, N.ctypes.data, axis.ctypes.data, harm.ctypes.data,
                   E.ctypes.data, V.ctypes.data)
    b = C.c_size_t(0)
    assert L.mmf_avg_prob_workspace(C.byref(p), C.byref(b)) == 0 and b.value >= 14 * 4 * 8
    d = C.c_void_p(16)

    def call(Phi=d, ld=14, w=d, P=d, st=d, work=d, nb=None):
        return L.mmf_avg_prob(C.byref(p), Phi, C.c_int64(ld), w, P, st, work,
                              C.c_size_t(b.value if nb is None else nb), None)
    assert call(Phi=None) == -2
    assert call(ld=13) == -3
    assert call(w=None) == -4
    assert call(P=None) == -5
    assert call(st=None) == -6
    assert call(work=None) == -7
    assert call(nb=b.value - 1) == -8
    assert L.mmf_strerror(7).decode().startswith("averaged probabilities")
