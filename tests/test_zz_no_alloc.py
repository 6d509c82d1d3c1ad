"""mmf_avg_prob_noalloc (no workspace, the library's fixed device array)
against mmf_avg_prob with its workspace, called through the C ABI: two calls
in a row on one GPU, the second with a smaller problem (the array keeps the
first call's contents), for a bare dimension whose partials fit the array
(same partition: bitwise equal) and one whose partials do not (fewer
workgroups: equal up to rounding).  The degeneracy status must agree too."""
import ctypes as C

import numpy as np
import pytest

from workloads import random_problem
from gpu_util import require_gpu, log

pytestmark = pytest.mark.gpu


def _both(torch, mmf, p, seed):
    dp = mmf.DeviceProblem(p)
    M = dp.M
    g = torch.Generator(device="cuda").manual_seed(seed)
    Pt = torch.randn((M, M), dtype=torch.complex128, device="cuda", generator=g)
    Pt /= torch.linalg.vector_norm(Pt, dim=1, keepdim=True)       # unit columns (rows of Pt)
    w = torch.sort(torch.randn(M, dtype=torch.float64, device="cuda", generator=g)).values
    w[1] = w[0]                                                    # one exactly degenerate pair
    L = mmf.lib()
    b = C.c_size_t(0)
    assert L.mmf_avg_prob_workspace(dp.ref, C.byref(b)) == 0
    work = torch.empty(b.value, dtype=torch.uint8, device="cuda")
    Pa = torch.empty((dp.D, dp.D), dtype=torch.float64, device="cuda")
    Pb = torch.full((dp.D, dp.D), float("nan"), dtype=torch.float64, device="cuda")
    sa = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    sb = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ld = C.c_int64(Pt.stride(0))
    assert L.mmf_avg_prob(dp.ref, C.c_void_p(Pt.data_ptr()), ld, C.c_void_p(w.data_ptr()),
                          C.c_void_p(Pa.data_ptr()), C.c_void_p(sa.data_ptr()), C.c_void_p(work.data_ptr()),
                          C.c_size_t(work.numel()), s) == 0
    assert L.mmf_avg_prob_noalloc(dp.ref, C.c_void_p(Pt.data_ptr()), ld, C.c_void_p(w.data_ptr()),
                                  C.c_void_p(Pb.data_ptr()), C.c_void_p(sb.data_ptr()), s) == 0
    torch.cuda.synchronize()
    return dp, Pa.cpu().numpy(), Pb.cpu().numpy(), int(sa.item()), int(sb.item())


@pytest.mark.parametrize("D,N1,N2", [(3, (20, 12), (4, 3)), (52, (20,), (6,))])
def test_avg_prob_noalloc_matches_workspace_form(D, N1, N2):
    torch, mmf = require_gpu()
    for k, N in enumerate((N1, N2)):                 # second call: smaller input
        p = random_problem(D, N, seed=40 + k)
        dp, Pa, Pb, sa, sb = _both(torch, mmf, p, seed=7 + k)
        log(f"no-alloc avg_prob D={D} M={dp.M}: max diff {np.abs(Pa - Pb).max():.2e}, status {sa}/{sb}")
        assert np.isfinite(Pb).all()
        if D <= 45:
            assert np.array_equal(Pa, Pb)
        else:
            assert np.abs(Pa - Pb).max() <= 1e-13 * max(1.0, np.abs(Pa).max())
        assert sa == sb


def test_avg_prob_noalloc_argument_errors():
    torch, mmf = require_gpu()
    L = mmf.lib()
    p = random_problem(2, (3,), seed=1)
    dp = mmf.DeviceProblem(p)
    d = C.c_void_p(16)
    assert L.mmf_avg_prob_noalloc(None, d, C.c_int64(dp.M), d, d, d, None) == -1
    assert L.mmf_avg_prob_noalloc(dp.ref, None, C.c_int64(dp.M), d, d, d, None) == -2
    assert L.mmf_avg_prob_noalloc(dp.ref, d, C.c_int64(dp.M - 1), d, d, d, None) == -3
    assert L.mmf_avg_prob_noalloc(dp.ref, d, C.c_int64(dp.M), None, d, d, None) == -4
    assert L.mmf_avg_prob_noalloc(dp.ref, d, C.c_int64(dp.M), d, None, d, None) == -5
    assert L.mmf_avg_prob_noalloc(dp.ref, d, C.c_int64(dp.M), d, d, None, None) == -6
