"""Writes ladder8712_pbar.txt: the oracle's time- and phase-averaged
transition probabilities (Eqs. 3-5 averaged over time and the drive phases)
for the 8-level two-drive ladder at truncation +-16 (Floquet dimension 8712),
with the oracle's verdict on near-degenerate quasienergies sharing weight.

The oracle's full eigendecomposition at this order takes minutes on the host,
too long for a test; the stored 8 x 8 table stands in for it.  Only the oracle
and the seeded input generator are called.

    python tests/golden/make_ladder8712_pbar.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import cfg2_large  # noqa: E402


def main():
    p, _, _ = cfg2_large(N=(16, 16))
    H = oracle.build_floquet(p)
    eps, Phi = oracle.eigh(H)
    P = oracle.avg_prob(p, Phi)
    degenerate = oracle.avg_prob_degenerate(p, Phi, eps)
    out = os.path.join(HERE, "ladder8712_pbar.txt")
    with open(out, "w") as f:
        f.write("# oracle time- and phase-averaged transition probabilities P[i, j] = average |U_ij|^2 (j: initial level),\n")
        f.write("# 8-level two-drive ladder, truncation +-16 per mode (M = 8712); written by make_ladder8712_pbar.py\n")
        f.write(f"# degenerate_clusters_share_weight {int(degenerate)}\n")
        f.write(f"# quasienergy_min {eps.min():.17e} quasienergy_max {eps.max():.17e}\n")
        np.savetxt(f, P, fmt="%.17e")
    print(out, "degenerate", degenerate)


if __name__ == "__main__":
    main()
