"""Helpers shared by the GPU tests (not collected by pytest)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def M():
    import paper_2408_04440_amd.mpchol as mod

    mod.lib()  # raises if libmpchol.so is missing
    return mod


def factor_dense(h, n):
    """Copy the factor's represented values to a host FP64 array."""
    torch = torch_cuda()
    mod = M()
    Lg = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    mod.mpchol_get_factor(h, Lg.T, n)
    torch.cuda.synchronize()
    return Lg.T.cpu().numpy()


def tile_rel(A, B, b):
    """max over lower tiles of ||A_IJ - B_IJ||_F / ||B_IJ||_F (zero tiles skipped)."""
    n = A.shape[0]
    nt = (n + b - 1) // b
    worst = 0.0
    for I in range(nt):
        for J in range(I + 1):
            a = A[I * b:(I + 1) * b, J * b:(J + 1) * b]
            c = B[I * b:(I + 1) * b, J * b:(J + 1) * b]
            den = np.linalg.norm(c)
            if den > 0:
                worst = max(worst, np.linalg.norm(a - c) / den)
    return worst
