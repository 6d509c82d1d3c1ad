"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2005_03426_amd as mmf
    mmf.lib()          # fails loudly if libmmf.so is missing
    return torch, mmf


def to_dev_cm(torch, X):
    """numpy matrix -> device tensor in column-major storage (Xt[c, r] = X[r, c])."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(X).T)).to("cuda")


def from_dev_cm(Xt):
    return Xt.T.cpu().numpy()


def log(msg):
    print(msg, flush=True)
