"""mpchol_sample_noalloc (draws without any allocation, for callers that
cannot allocate) against mpchol_sample on the same factor and seed: the two
must agree bit for bit.  Two calls in a row, the second with a smaller input;
the first spans more than one pass through the library's fixed draw buffer
(n * ndraws above its 16,777,216 values)."""
import numpy as np
import pytest

import synth
from _gpu import M, log, torch_cuda

pytestmark = pytest.mark.gpu

BUFFER_VALUES = 1 << 24


def _factor(mod, L, tile, eps):
    n = L * L
    sigma, x = synth.workload(L)
    h = mod.mpchol_create(n, tile)
    mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
    mod.mpchol_precision_map(h, mod.RULE_NORM, eps)
    assert mod.mpchol_factor(h) == 0
    return h, n


def _both(torch, mod, h, n, ndraws, seed):
    Ya = torch.full((ndraws, n), float("nan"), dtype=torch.float32, device="cuda")
    Yb = torch.full((ndraws, n), float("nan"), dtype=torch.float32, device="cuda")
    mod.mpchol_sample(h, ndraws, seed, Ya.T, n)
    mod.mpchol_sample_noalloc(h, ndraws, seed, Yb.T, n)
    torch.cuda.synchronize()
    return Ya, Yb


def test_sample_noalloc_matches_sample():
    torch = torch_cuda()
    mod = M()
    # first call: n = 36,864 (band limit 192, tile 1024, mixed map), 600 draws = 2 passes
    h, n = _factor(mod, 192, 1024, 1e-9)
    try:
        assert n * 600 > BUFFER_VALUES
        log(f"noalloc: n={n} ndraws=600 seed=2")
        Ya, Yb = _both(torch, mod, h, n, 600, 2)
        assert not torch.isnan(Ya).any() and torch.isfinite(Ya).all()
        assert torch.equal(Ya, Yb)
        # the same handle again with fewer draws: the buffer's old contents do not leak
        log(f"noalloc: n={n} ndraws=100 seed=5")
        Ya, Yb = _both(torch, mod, h, n, 100, 5)
        assert torch.equal(Ya, Yb)
    finally:
        mod.mpchol_destroy(h)
    # second call: a smaller input (n = 1,024, tile 128, 50 draws), one pass
    h, n = _factor(mod, 32, 128, 1e-6)
    try:
        log(f"noalloc: n={n} ndraws=50 seed=7")
        Ya, Yb = _both(torch, mod, h, n, 50, 7)
        assert torch.equal(Ya, Yb)
        # a leading dimension larger than n: rows beyond n are left untouched
        Yc = torch.full((50, n + 64), -3.0, dtype=torch.float32, device="cuda")
        mod.mpchol_sample_noalloc(h, 50, 7, Yc.T, n)
        torch.cuda.synchronize()
        assert torch.equal(Yc[:, :n], Ya)
        assert bool((Yc[:, n:] == -3.0).all())
    finally:
        mod.mpchol_destroy(h)


def test_sample_noalloc_errors():
    torch = torch_cuda()
    mod = M()
    n, tile = 1024, 128
    sigma, x = synth.workload(32)
    h = mod.mpchol_create(n, tile)
    try:
        Y = torch.zeros((4, n), dtype=torch.float32, device="cuda")
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        rc = mod.lib().mpchol_sample_noalloc(h, 4, 1, mod._ptr(Y), n)
        assert rc == mod.EORDER  # before a factor
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        assert mod.lib().mpchol_sample_noalloc(h, 0, 1, mod._ptr(Y), n) == mod.EINVAL
        assert mod.lib().mpchol_sample_noalloc(h, 4, 1, mod._ptr(Y), n - 1) == mod.EINVAL
        assert mod.lib().mpchol_sample_noalloc(h, 4, 1, None, n) == mod.EINVAL
    finally:
        mod.mpchol_destroy(h)
