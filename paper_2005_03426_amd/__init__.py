"""MI355X-native multimode Floquet hot path (arXiv:2005.03426, OPENMMF).

Python surface over the C ABI of libmmf.so (include/mmf.h).  Functions take
and return torch tensors on the GPU; this layer only marshals pointers,
sizes and streams -- every step of the computation (assembly of the Floquet
matrix, its Hermitian eigendecomposition, U(t,t0), micromotion, averaged
transition probabilities) runs in the library's HIP kernels.

Storage conventions (the C ABI is column-major):
  * an M x M matrix X is held in a torch tensor Xt of shape (M, M) with
    Xt[c, r] = X[r, c]; so H_F = HFt.T and eigenvector a is the row Pt[a];
  * U(t,t0) comes back as U[tau, i, j] (a transposed view of the raw buffer).
"""
from __future__ import annotations

import ctypes as C
import numpy as np

from ._lib import (lib, call, check, MMFProblem, MMFEighOpts, MMFBatchOpts, MMFError, EXPORTED, LIB_PATH, MMF_ERR_DEGENERATE,
                   MMF_C128, MMF_C64_REFINED, MMF_C64_RAW, MMF_OK, MMF_ERR_HIP, MMF_ERR_WORKSPACE,
                   MMF_ERR_NOT_IMPLEMENTED, MMF_ERR_NO_CONVERGENCE, MMF_ERR_SELECTION, MMF_ERR_TOO_LARGE)

__all__ = [
    "DeviceProblem", "floquet_dim", "build_floquet", "eigh", "eigh_workspace_bytes", "hetrd",
    "stedc", "unmtr", "evolve", "micromotion", "avg_prob", "solve", "MMFError", "lib",
    "MMF_C128", "MMF_C64_REFINED", "MMF_C64_RAW", "EXPORTED", "LIB_PATH",
]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class DeviceProblem:
    """A problem statement (see workloads.Problem) prepared for the library:
    E and V as column-major host arrays (the library validates E and stages
    both on the device when it assembles H_F, into `ev_work`), frequencies,
    truncations and the coupling table as host arrays kept alive for the
    ctypes structure."""

    def __init__(self, problem, device="cuda"):
        torch = _torch()
        self.D = int(problem.E.shape[0])
        self.F = int(len(problem.omega))
        self.K = int(len(problem.axis))
        self.omega = np.ascontiguousarray(problem.omega, dtype=np.float64)
        self.N = np.ascontiguousarray(problem.N, dtype=np.int32)
        self.axis = np.ascontiguousarray(problem.axis, dtype=np.int32)
        self.harm = np.ascontiguousarray(problem.harm, dtype=np.int32)
        # column-major storage: the transposed array in C order
        self.E = np.ascontiguousarray(np.asarray(problem.E, dtype=np.complex128).T)
        if self.K:
            V = np.asarray(problem.V, dtype=np.complex128)
            self.V = np.ascontiguousarray(V.transpose(0, 2, 1))
        else:
            self.V = None
        self.struct = MMFProblem(
            self.D, self.F, self.K,
            self.omega.ctypes.data if self.F else None, self.N.ctypes.data if self.F else None,
            self.axis.ctypes.data if self.K else None, self.harm.ctypes.data if self.K else None,
            self.E.ctypes.data, self.V.ctypes.data if self.K else None)
        self.M = floquet_dim(self)
        self.device = device
        b = C.c_size_t(0)
        call("mmf_build_floquet_workspace", self.ref, C.byref(b))
        self.ev_work = _workspace(b.value, device)
        # the device copy of E and V in the workspace's layout (E, then each
        # V_k, column-major), for mmf_build_floquet_dev
        ev = [self.E.ravel()] + ([self.V.ravel()] if self.K else [])
        ev = np.ascontiguousarray(np.concatenate(ev)).view(np.uint8)
        self.ev_work[:ev.size].copy_(torch.from_numpy(ev))
        S = self.M // self.D
        s0, stride = 0, 1
        for n in self.N:
            s0 += int(n) * stride
            stride *= 2 * int(n) + 1
        self.S, self.s0 = S, s0

    @property
    def ref(self):
        return C.byref(self.struct)


def floquet_dim(dp: DeviceProblem) -> int:
    M = C.c_int64(0)
    call("mmf_floquet_dim", dp.ref, C.byref(M))
    return int(M.value)


def build_floquet(dp: DeviceProblem, out=None, stream=None):
    """H_F in column-major storage: returns HFt with H_F = HFt.T."""
    torch = _torch()
    M = dp.M
    if out is None:
        out = torch.empty((M, M), dtype=torch.complex128, device=dp.device)
    call("mmf_build_floquet", dp.ref, _ptr(out), C.c_int64(out.stride(0)), _ptr(dp.ev_work),
         C.c_size_t(dp.ev_work.numel()), _stream(stream))
    return out


def build_floquet_dev(dp: DeviceProblem, out, stream=None):
    """H_F from the device copy of E and V held by dp (one kernel launch, no
    host copy: usable under stream capture).  out: preallocated (M, M)
    complex128 tensor, H_F = out.T."""
    call("mmf_build_floquet_dev", dp.ref, _ptr(dp.ev_work), _ptr(out), C.c_int64(out.stride(0)), _stream(stream))
    return out


def eigh_workspace_bytes(M: int, prec: int = MMF_C128) -> int:
    b = C.c_size_t(0)
    call("mmf_eigh_workspace", C.c_int64(M), C.c_int(prec), C.byref(b))
    return int(b.value)


def eigh_two_stage_min() -> int:
    """Order from which eigh / eigh_window use the two-stage reduction."""
    return int(lib().mmf_eigh_two_stage_min())


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def eigh(At, prec: int = MMF_C128, w=None, work=None, info=None, stream=None, limits=None):
    """In-place eigendecomposition of the Hermitian matrix held (column-major)
    in At.  Returns (w, At, info): eigenvalues ascending; At's row a is the
    eigenvector of w[a]; info a device int32 (0 = converged).  `limits`, a
    dict with any of refine_max_iters / secular_max_iters / leaf_max_iters,
    selects mmf_eigh_ex with those iteration limits."""
    torch = _torch()
    M = At.shape[0]
    dev = At.device
    if w is None:
        w = torch.empty(M, dtype=torch.float64, device=dev)
    if work is None:
        work = _workspace(eigh_workspace_bytes(M, prec), dev)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=dev)
    if limits is None:
        call("mmf_eigh", C.c_int64(M), _ptr(At), C.c_int64(At.stride(0) if M else 1), _ptr(w), C.c_int(prec),
             _ptr(work), C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    else:
        opts = MMFEighOpts(**{k: int(v) for k, v in limits.items()})
        call("mmf_eigh_ex", C.c_int64(M), _ptr(At), C.c_int64(At.stride(0) if M else 1), _ptr(w), C.c_int(prec),
             C.byref(opts), _ptr(work), C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return w, At, info


def eigh_batched_workspace_bytes(sizes, prec: int = MMF_C128) -> int:
    n = (C.c_int64 * max(len(sizes), 1))(*[int(m) for m in sizes])
    b = C.c_size_t(0)
    call("mmf_eigh_batched_workspace", C.c_int64(len(sizes)), n, C.c_int(prec), C.byref(b))
    return int(b.value)


def eigh_batched(mats, prec: int = MMF_C128, ws=None, work=None, info=None, stream=None, tiles=None):
    """In-place eigendecomposition of every Hermitian matrix of the list
    `mats` (column-major like eigh's argument) in one grouped call.  Returns
    (ws, mats, info): eigenvalue tensors, the matrices now holding the
    eigenvectors (row a = eigenvector a), and a device int32 [count].
    `tiles`: the 8-entry tile table of mmf_batch_opts (workgroup size of the
    one-workgroup solver per order bucket, 0 = grouped path), e.g. from
    autotune.load_table(); None keeps the library's built-in rule."""
    torch = _torch()
    count = len(mats)
    if count == 0:
        return [], mats, None
    dev = mats[0].device
    sizes = [int(A.shape[0]) for A in mats]
    if ws is None:
        ws = [torch.empty(m, dtype=torch.float64, device=dev) for m in sizes]
    if work is None:
        work = _workspace(eigh_batched_workspace_bytes(sizes, prec), dev)
    if info is None:
        info = torch.zeros(count, dtype=torch.int32, device=dev)
    n = (C.c_int64 * count)(*sizes)
    ld = (C.c_int64 * count)(*[int(A.stride(0)) if m else 1 for A, m in zip(mats, sizes)])
    Ap = (C.c_void_p * count)(*[A.data_ptr() for A in mats])
    wp = (C.c_void_p * count)(*[w.data_ptr() for w in ws])
    if tiles is None:
        call("mmf_eigh_batched", C.c_int64(count), n, Ap, ld, wp, C.c_int(prec), _ptr(work),
             C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    else:
        opts = MMFBatchOpts((C.c_int32 * 8)(*[int(x) for x in tiles]))
        call("mmf_eigh_batched_ex", C.c_int64(count), n, Ap, ld, wp, C.c_int(prec), C.byref(opts), _ptr(work),
             C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return ws, mats, info


def eigh_window(At, vl: float, vu: float, kmax: int, work=None, stream=None):
    """Eigenpairs of the Hermitian matrix in At (column-major, destroyed)
    with eigenvalue in [vl, vu).  Returns (w, Zt, count, info): w[:k] and the
    rows Zt[:k] (row t = eigenvector of w[t]) are valid for
    k = min(count, kmax)."""
    torch = _torch()
    M = At.shape[0]
    dev = At.device
    kmax = int(min(kmax, M))
    w = torch.zeros(max(kmax, 1), dtype=torch.float64, device=dev)
    Zt = torch.zeros((max(kmax, 1), M), dtype=torch.complex128, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        b = C.c_size_t(0)
        call("mmf_eigh_window_workspace", C.c_int64(M), C.c_int64(kmax), C.byref(b))
        work = _workspace(b.value, dev)
    call("mmf_eigh_window", C.c_int64(M), _ptr(At), C.c_int64(At.stride(0) if M else 1), C.c_double(vl),
         C.c_double(vu), C.c_int64(kmax), _ptr(w), _ptr(Zt), C.c_int64(max(M, 1)), _ptr(count), _ptr(work),
         C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return w[:kmax], Zt[:kmax], count, info


def eigh_band_workspace_bytes(M: int, b: int) -> int:
    nb = C.c_size_t(0)
    call("mmf_eigh_band_workspace", C.c_int64(M), C.c_int64(b), C.byref(nb))
    return int(nb.value)


def eigh_band(At, b: int, w=None, work=None, info=None, stream=None):
    """In-place eigendecomposition (complex128) of the Hermitian matrix held
    column-major in At whose entries vanish below its b-th subdiagonal (see
    mmf_eigh_band; b = D h_max for a one-drive Floquet matrix).  Returns
    (w, At, info) as eigh."""
    torch = _torch()
    M = At.shape[0]
    dev = At.device
    if w is None:
        w = torch.empty(M, dtype=torch.float64, device=dev)
    if work is None:
        work = _workspace(eigh_band_workspace_bytes(M, b), dev)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=dev)
    call("mmf_eigh_band", C.c_int64(M), _ptr(At), C.c_int64(At.stride(0) if M else 1), C.c_int64(b), _ptr(w),
         _ptr(work), C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return w, At, info


def eigh_band_window(At, b: int, vl: float, vu: float, kmax: int, work=None, stream=None):
    """Eigenpairs with eigenvalue in [vl, vu) of the banded Hermitian matrix
    in At (column-major, half-bandwidth b; kept when b <= 64, see
    mmf_eigh_band_window).  Returns (w, Zt, count, info) as eigh_window."""
    torch = _torch()
    M = At.shape[0]
    dev = At.device
    kmax = int(min(kmax, M))
    w = torch.zeros(max(kmax, 1), dtype=torch.float64, device=dev)
    Zt = torch.zeros((max(kmax, 1), M), dtype=torch.complex128, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        nb = C.c_size_t(0)
        call("mmf_eigh_band_window_workspace", C.c_int64(M), C.c_int64(b), C.c_int64(kmax), C.byref(nb))
        work = _workspace(nb.value, dev)
    call("mmf_eigh_band_window", C.c_int64(M), _ptr(At), C.c_int64(At.stride(0) if M else 1), C.c_int64(b),
         C.c_double(vl), C.c_double(vu), C.c_int64(kmax), _ptr(w), _ptr(Zt), C.c_int64(max(M, 1)), _ptr(count),
         _ptr(work), C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return w[:kmax], Zt[:kmax], count, info


def floquet_half_bandwidth(p) -> int:
    """Half-bandwidth of the Floquet matrix of a problem statement (workloads.
    Problem) in the block order of App. A: a coupling of harmonic h on axis l
    sits h * prod_{l' < l} (2 N_l' + 1) blocks of D rows off the diagonal (none
    when h > 2 N_l), so the farthest entry is D - 1 rows beyond that block
    offset times D."""
    import numpy as np
    D = int(np.asarray(p.E).shape[0])
    stride = [1]
    for n in p.N:
        stride.append(stride[-1] * (2 * int(n) + 1))
    far = 0
    for ax, h in zip(p.axis, p.harm):
        if int(h) <= 2 * int(p.N[ax]):
            far = max(far, int(h) * stride[ax])
    return D * far + (D - 1)


def eigvalsh_batched_workspace_bytes(sizes, prec: int = MMF_C128) -> int:
    n = (C.c_int64 * max(len(sizes), 1))(*[int(m) for m in sizes])
    b = C.c_size_t(0)
    call("mmf_eigvalsh_batched_workspace", C.c_int64(len(sizes)), n, C.c_int(prec), C.byref(b))
    return int(b.value)


def eigvalsh_batched(mats, prec: int = MMF_C128, ws=None, work=None, info=None, stream=None):
    """Eigenvalues (ascending) of every Hermitian matrix of `mats` (column-
    major like eigh's argument; destroyed for complex128, kept for
    MMF_C64_RAW).  Returns (ws, info)."""
    torch = _torch()
    count = len(mats)
    if count == 0:
        return [], None
    dev = mats[0].device
    sizes = [int(A.shape[0]) for A in mats]
    if ws is None:
        ws = [torch.empty(m, dtype=torch.float64, device=dev) for m in sizes]
    if work is None:
        work = _workspace(eigvalsh_batched_workspace_bytes(sizes, prec), dev)
    if info is None:
        info = torch.zeros(count, dtype=torch.int32, device=dev)
    n = (C.c_int64 * count)(*sizes)
    ld = (C.c_int64 * count)(*[int(A.stride(0)) if m else 1 for A, m in zip(mats, sizes)])
    Ap = (C.c_void_p * count)(*[A.data_ptr() for A in mats])
    wp = (C.c_void_p * count)(*[w.data_ptr() for w in ws])
    call("mmf_eigvalsh_batched", C.c_int64(count), n, Ap, ld, wp, C.c_int(prec), _ptr(work),
         C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return ws, info


def quasienergy_scan(problems, prec: int = MMF_C128, device="cuda", stream=None):
    """Quasienergy spectra of many Floquet problems (e.g. a frequency scan):
    assemble every H_F, then one grouped eigenvalue-only solve.  Returns the
    list of eigenvalue tensors."""
    torch = _torch()
    import contextlib
    ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
    with ctx:
        dps = [p if isinstance(p, DeviceProblem) else DeviceProblem(p, device) for p in problems]
        HFs = [build_floquet(dp, stream=stream) for dp in dps]
        ws, info = eigvalsh_batched(HFs, prec, stream=stream)
    return ws


def hetrd(At, work=None, stream=None):
    """Stage 1: returns (d, e, tau); At's column i (row i of the tensor) keeps
    the reflector v_i below the diagonal."""
    torch = _torch()
    n = At.shape[0]
    dev = At.device
    d = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    tau = torch.empty(max(n - 1, 1), dtype=torch.complex128, device=dev)
    if work is None:
        work = _workspace(eigh_workspace_bytes(n), dev)
    call("mmf_hetrd", C.c_int64(n), _ptr(At), C.c_int64(At.stride(0)), _ptr(d), _ptr(e), _ptr(tau),
         _ptr(work), C.c_size_t(work.numel()), _stream(stream))
    return d, e, tau


def stedc(d, e, work=None, stream=None):
    """Stage 2: eigenpairs of the real symmetric tridiagonal (d, e).  Returns
    (w, Zt, info) with Z = Zt.T (column a = eigenvector a); d is overwritten."""
    torch = _torch()
    n = d.shape[0]
    dev = d.device
    Zt = torch.empty((n, n), dtype=torch.float64, device=dev)
    if work is None:
        work = _workspace(eigh_workspace_bytes(n), dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    call("mmf_stedc", C.c_int64(n), _ptr(d), _ptr(e), _ptr(Zt), C.c_int64(n), _ptr(work),
         C.c_size_t(work.numel()), _ptr(info), _stream(stream))
    return d, Zt, info


def unmtr(Vt, tau, Zt, out=None, work=None, stream=None):
    """Stage 3: Phi = Q Z (column-major tensors as elsewhere)."""
    torch = _torch()
    n = Vt.shape[0]
    dev = Vt.device
    if out is None:
        out = torch.empty((n, n), dtype=torch.complex128, device=dev)
    if work is None:
        work = _workspace(eigh_workspace_bytes(n), dev)
    call("mmf_unmtr", C.c_int64(n), _ptr(Vt), C.c_int64(Vt.stride(0)), _ptr(tau), _ptr(Zt),
         C.c_int64(Zt.stride(0)), _ptr(out), C.c_int64(out.stride(0)), _ptr(work),
         C.c_size_t(work.numel()), _stream(stream))
    return out


def evolve(dp: DeviceProblem, Pt, w, t0: float, t, work=None, stream=None, out=None):
    """U(t, t0) for every time in t (device float64).  Returns U[tau, i, j]
    (a transposed view of `out`, a preallocated (T, D, D) complex128 tensor
    if given)."""
    torch = _torch()
    T = int(t.shape[0])
    D = dp.D
    U = out if out is not None else torch.empty((T, D, D), dtype=torch.complex128, device=Pt.device)
    if work is None:
        b = C.c_size_t(0)
        call("mmf_evolve_workspace", dp.ref, C.c_int32(T), C.byref(b))
        work = _workspace(b.value, Pt.device)
    call("mmf_evolve", dp.ref, _ptr(Pt), C.c_int64(Pt.stride(0)), _ptr(w), C.c_double(t0),
         C.c_int32(T), _ptr(t), _ptr(U), _ptr(work), C.c_size_t(work.numel()), _stream(stream))
    return U.transpose(1, 2)


def micromotion(dp: DeviceProblem, Pt, w, t, work=None, stream=None):
    """U_F(t) over one representative per orbit.  Returns (UF[tau, i, b],
    eps_sel[b], sel[b], info)."""
    torch = _torch()
    T = int(t.shape[0])
    D = dp.D
    dev = Pt.device
    UF = torch.empty((T, D, D), dtype=torch.complex128, device=dev)
    eps = torch.empty(D, dtype=torch.float64, device=dev)
    sel = torch.empty(D, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        b = C.c_size_t(0)
        call("mmf_evolve_workspace", dp.ref, C.c_int32(max(T, 1)), C.byref(b))
        work = _workspace(b.value, dev)
    call("mmf_micromotion", dp.ref, _ptr(Pt), C.c_int64(Pt.stride(0)), _ptr(w), C.c_int32(T), _ptr(t),
         _ptr(UF), _ptr(eps), _ptr(sel), _ptr(work), C.c_size_t(work.numel()), _ptr(info),
         _stream(stream))
    return UF.transpose(1, 2), eps, sel, info


class _ModeSubset:
    """The problem restricted to the fundamentals `axes` (static part plus
    the couplings on those axes), axes renumbered in the given order."""

    def __init__(self, problem, axes):
        axes = [int(a) for a in axes]
        pos = {a: i for i, a in enumerate(axes)}
        keep = [k for k in range(len(problem.axis)) if int(problem.axis[k]) in pos]
        self.E = problem.E
        self.omega = [problem.omega[a] for a in axes]
        self.N = [problem.N[a] for a in axes]
        self.axis = [pos[int(problem.axis[k])] for k in keep]
        self.harm = [problem.harm[k] for k in keep]
        V = np.asarray(problem.V)
        self.V = V[keep] if len(keep) else np.zeros((0,) + np.asarray(problem.E).shape, np.complex128)


def dressed_evolution(problem, dressing_axes, t, t0: float = 0.0, prec: int = MMF_C128, device="cuda",
                      stream=None):
    """Evolution of the full problem in the dressed basis of a subset of its
    modes (the static Hamiltonian plus the drives on `dressing_axes`):
    U_dressed(t, t0) = U_F^sub(t)^H U(t, t0) U_F^sub(t0).  Returns a dict with
    'U_dressed' and 'U_bare' [T, D, D] (final, initial), the subset's
    micromotion operators 'UF' [T, D, D] and dressed energies 'eps_dressed'."""
    torch = _torch()
    import contextlib
    ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
    with ctx:
        full = DeviceProblem(problem, device)          # problem: a host problem statement
        sub = DeviceProblem(_ModeSubset(problem, dressing_axes), device)
        dev = full.device
        tt = t if torch.is_tensor(t) else torch.as_tensor(np.asarray(t, dtype=np.float64), device=dev)
        T = int(tt.shape[0])
        # subset: eigenpairs, then U_F at the times t and at t0 (one call, t0 last)
        Hs = build_floquet(sub, stream=stream)
        ws, Ps, _ = eigh(Hs, prec, stream=stream)
        tt1 = torch.cat([tt, torch.full((1,), float(t0), dtype=torch.float64, device=dev)])
        UF, eps, sel, minfo = micromotion(sub, Ps, ws, tt1, stream=stream)
        # full problem: U(t, t0)
        Hf = build_floquet(full, stream=stream)
        wf, Pf, info = eigh(Hf, prec, stream=stream)
        U = evolve(full, Pf, wf, t0, tt, stream=stream)
        D = full.D
        UFs = UF.transpose(1, 2)                 # storage [T+1][b][i] = column-major per time
        Us = U.transpose(1, 2)
        Ud = torch.empty((T, D, D), dtype=torch.complex128, device=dev)
        call("mmf_dressed_evolution", C.c_int32(D), C.c_int32(T), _ptr(UFs), _ptr(Us), _ptr(UFs[T]),
             _ptr(Ud), _stream(stream))
    return {"U_dressed": Ud.transpose(1, 2), "U_bare": U, "UF": UF[:T], "eps_dressed": eps,
            "info": info, "selection_info": minfo}


def avg_prob(dp: DeviceProblem, Pt, w, work=None, status=None, stream=None, out=None):
    """Averaged transition probabilities P[i, j] (i final, j initial) from
    the eigenvectors (rows of Pt) and their ascending eigenvalues w.  Returns
    (P, status): status is a device int32, MMF_ERR_DEGENERATE when degenerate
    quasienergies share weight (P then depends on the eigenvector basis).
    out: optional preallocated (D, D) float64 tensor (P is its transpose)."""
    torch = _torch()
    D = dp.D
    P = out if out is not None else torch.empty((D, D), dtype=torch.float64, device=Pt.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=Pt.device)
    if work is None:
        b = C.c_size_t(0)
        call("mmf_avg_prob_workspace", dp.ref, C.byref(b))
        work = _workspace(b.value, Pt.device)
    call("mmf_avg_prob", dp.ref, _ptr(Pt), C.c_int64(Pt.stride(0)), _ptr(w), _ptr(P), _ptr(status),
         _ptr(work), C.c_size_t(work.numel()), _stream(stream))
    return P.T, status


def avg_prob_noalloc(dp: DeviceProblem, Pt, w, P=None, status=None, stream=None):
    """avg_prob through the entry point that allocates nothing (the
    library's own fixed device array holds the partial sums).  P and status
    may be passed in so that the call itself allocates nothing either."""
    torch = _torch()
    D = dp.D
    if P is None:
        P = torch.empty((D, D), dtype=torch.float64, device=Pt.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=Pt.device)
    call("mmf_avg_prob_noalloc", dp.ref, _ptr(Pt), C.c_int64(Pt.stride(0)), _ptr(w), _ptr(P), _ptr(status),
         _stream(stream))
    return P.T, status


def solve(problem, t, t0: float = 0.0, prec: int = MMF_C128, device="cuda"):
    """One Floquet solve: assemble -> eigh -> U at times t -> averaged P.
    Returns a dict of device tensors (w, Pt, U, P, info)."""
    torch = _torch()
    dp = problem if isinstance(problem, DeviceProblem) else DeviceProblem(problem, device)
    tt = t if torch.is_tensor(t) else torch.as_tensor(np.asarray(t, dtype=np.float64), device=dp.device)
    HF = build_floquet(dp)
    w, Pt, info = eigh(HF, prec)
    U = evolve(dp, Pt, w, t0, tt)
    P, pstat = avg_prob(dp, Pt, w)
    return {"w": w, "Pt": Pt, "U": U, "P": P, "P_status": pstat, "info": info, "dp": dp}


def solve_batched(problems, t, t0: float = 0.0, prec: int = MMF_C128, device="cuda", stream=None):
    """Many Floquet solves with one grouped eigensolve: assemble each H_F,
    diagonalise them all together, then U(t) and averaged P per problem.
    Returns a list of dicts like solve()."""
    torch = _torch()
    import contextlib
    ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
    with ctx:          # temporaries are then allocated and freed in the order of `stream`
        dps = [p if isinstance(p, DeviceProblem) else DeviceProblem(p, device) for p in problems]
        if not dps:
            return []
        dev = dps[0].device
        tt = t if torch.is_tensor(t) else torch.as_tensor(np.asarray(t, dtype=np.float64), device=dev)
        HFs = [build_floquet(dp, stream=stream) for dp in dps]
        ws, Pts, info = eigh_batched(HFs, prec, stream=stream)
        out = []
        for k, (dp, w, Pt) in enumerate(zip(dps, ws, Pts)):
            U = evolve(dp, Pt, w, t0, tt, stream=stream)
            P, pstat = avg_prob(dp, Pt, w, stream=stream)
            out.append({"w": w, "Pt": Pt, "U": U, "P": P, "P_status": pstat, "info": info[k:k + 1], "dp": dp})
    return out
