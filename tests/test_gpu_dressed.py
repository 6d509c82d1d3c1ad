"""GPU parity of the dressed-basis evolution (Sec. 4.1, Fig. 4).

The whole chain runs in the library: the dressing subset's Floquet matrix,
eigenpairs and micromotion operator at every time and at t0, the full
problem's bare evolution, then mmf_dressed_evolution.  Compared element by
element with the oracle (1e-10), plus the resonance pin evaluated on the GPU
result.
"""
import numpy as np
import pytest

import oracle
from workloads import dressed_qubit
from gpu_util import require_gpu, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wP", [0.0100, 0.0125])
def test_dressed_evolution_against_oracle(wP):
    torch, mmf = require_gpu()
    p = dressed_qubit(wP)                               # the figure's parameters, N = (4, 12)
    ts = np.linspace(0.0, 3000.0, 64)
    t0 = 0.0
    log(f"dressed qubit wP={wP}")
    out = mmf.dressed_evolution(p, [0], ts, t0)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 0 and int(out["selection_info"].item()) == 0
    Ud_o, U_o, eps_o = oracle.dressed_evolution(p, [0], ts, t0)
    assert np.abs(out["eps_dressed"].cpu().numpy() - eps_o).max() < 1e-10
    assert np.abs(out["U_bare"].cpu().numpy() - U_o).max() < 1e-10
    assert np.abs(out["U_dressed"].cpu().numpy() - Ud_o).max() < 1e-10


def test_dressed_resonance_on_gpu():
    torch, mmf = require_gpu()
    ts = np.linspace(0.0, 30000.0, 601)
    peak = {}
    for wP in (0.0105, 0.0125, 0.0145):
        p = dressed_qubit(wP, Omega_Px=0.0005, Omega_Pz=0.0025, N=(4, 4))
        Ud = mmf.dressed_evolution(p, [0], ts, 0.0)["U_dressed"]
        peak[wP] = float((Ud[:, 1, 0].abs() ** 2).max())
    log(f"dressed transition peaks {peak}")
    assert peak[0.0125] > 0.99
    assert peak[0.0105] < 0.35 and peak[0.0145] < 0.35


def test_dressed_without_probe_is_diagonal():
    torch, mmf = require_gpu()
    p = dressed_qubit(0.0125, Omega_Px=0.0, Omega_Pz=0.0, N=(6, 2))
    ts = np.linspace(0.0, 800.0, 41)
    t0 = 0.37
    out = mmf.dressed_evolution(p, [0], ts, t0)
    eps = out["eps_dressed"].cpu().numpy()
    expect = np.array([np.diag(np.exp(-1j * eps * (t - t0))) for t in ts])
    assert np.abs(out["U_dressed"].cpu().numpy() - expect).max() < 1e-9
