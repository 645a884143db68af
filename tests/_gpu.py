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


def tile_residual_levels(tr_g, tr_o, A, b, lo=0.25, hi=4.0, floor_rel=1e-13):
    """Per lower tile, the residual norm of one valid execution against
    another's: sqrt(tr_g / tr_o) within [lo, hi] wherever either is above the
    FP64 floor (floor_rel * ||A_IJ||_F).  The residual of tile (I, J) depends
    only on that tile's class, so two executions of the same map leave every
    tile at the same error level; a tile computed or decoded in the wrong
    class moves by orders of magnitude.  Returns (worst low ratio, worst high
    ratio, tiles compared)."""
    n = A.shape[0]
    nt = (n + b - 1) // b
    rmin, rmax, cnt = np.inf, 0.0, 0
    for I in range(nt):
        for J in range(I + 1):
            fl = (floor_rel * np.linalg.norm(A[I * b:(I + 1) * b, J * b:(J + 1) * b])) ** 2
            if max(tr_g[I, J], tr_o[I, J]) <= fl:
                continue
            r = np.sqrt(max(tr_g[I, J], fl) / max(tr_o[I, J], fl))
            rmin, rmax, cnt = min(rmin, r), max(rmax, r), cnt + 1
            assert lo <= r <= hi, f"tile ({I},{J}): residual ratio {r:.3g} outside [{lo}, {hi}]"
    return rmin, rmax, cnt


def same_factor_residuals(be_g, tr_g, be_o, tr_o, A, b, rel=1e-6, floor_rel=1e-13):
    """The residual kernel against the oracle's residual of the same factor:
    total within `rel`, and every lower tile within `rel` plus the FP64 floor."""
    assert abs(be_g - be_o) <= rel * be_o, (be_g, be_o)
    n = A.shape[0]
    nt = (n + b - 1) // b
    worst = 0.0
    for I in range(nt):
        for J in range(I + 1):
            fl = (floor_rel * np.linalg.norm(A[I * b:(I + 1) * b, J * b:(J + 1) * b])) ** 2
            d = abs(tr_g[I, J] - tr_o[I, J])
            assert d <= rel * tr_o[I, J] + fl, f"tile ({I},{J}): {tr_g[I, J]:.6e} vs {tr_o[I, J]:.6e}"
            worst = max(worst, d / (rel * tr_o[I, J] + fl))
    # the upper part carries nothing
    assert np.all(np.triu(tr_g, 1) == 0)
    return worst
