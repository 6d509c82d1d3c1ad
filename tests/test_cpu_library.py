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
