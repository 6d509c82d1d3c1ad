"""The binding's Floquet half-bandwidth (the b that mmf_eigh_band is called
with) against the widest nonzero offset of the oracle's assembled H_F."""
import numpy as np
import pytest

import oracle
import paper_2005_03426_amd as mmf
from workloads import cfg1_tls, cfg2_large, one_drive_band, random_problem


@pytest.mark.parametrize("name,mk", [
    ("tls", lambda: cfg1_tls()[0]),
    ("ladder_2drive", lambda: cfg2_large(N=(4, 4))[0]),
    ("one_drive", lambda: one_drive_band(N=12)[0]),
    ("d3_h2_axis0_h1_axis1", lambda: random_problem(3, (5, 2), seed=3, harmonics=[(0, 2), (1, 1)])),
    ("harmonic_beyond_box", lambda: random_problem(2, (1,), seed=5, harmonics=[(0, 1), (0, 3)])),
    ("static", lambda: random_problem(3, (0,), seed=6)),
])
def test_floquet_half_bandwidth(name, mk):
    p = mk()
    H = oracle.build_floquet(p)
    idx = np.argwhere(np.abs(H) > 0)
    assert mmf.floquet_half_bandwidth(p) == int(np.max(np.abs(idx[:, 0] - idx[:, 1])))
