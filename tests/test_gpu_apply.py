"""Solve, Philox draws and emulation draws Y = L Z against the oracle."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(orc, L, tile, rho=5.0, nugget=1e-8, rule=0, eps=1e-9):
    n = L * L
    sigma, x = synth.workload(L)
    mod = M()
    h = mod.mpchol_create(n, tile)
    mod.mpchol_set_generator(h, sigma, x, rho, nugget)
    mod.mpchol_precision_map(h, rule, eps)
    assert mod.mpchol_factor(h) == 0
    return mod, h, n, sigma, x


@pytest.mark.parametrize("L,tile,nrhs,rule,eps", [(32, 128, 1, 0, 1e-9), (24, 128, 3, 0, 1e-9), (32, 128, 17, 1, 1e-6),
                                                  (32, 256, 2, 1, 1e-4)])
def test_solve(orc, L, tile, nrhs, rule, eps):
    torch = torch_cuda()
    mod, h, n, sigma, x = _setup(orc, L, tile, rule=rule, eps=eps)
    try:
        A = orc.cov_dense(sigma, x, 5.0, 1e-8)
        B = synth.rhs(n, nrhs)
        Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
        mod.mpchol_solve(h, Bt.T, n)
        torch.cuda.synchronize()
        X = Bt.T.cpu().numpy()
        be_fac = mod.mpchol_backward_error(h)
    finally:
        mod.mpchol_destroy(h)
    berr = np.linalg.norm(B - A @ X) / (np.linalg.norm(A) * np.linalg.norm(X) + np.linalg.norm(B))
    Xc = orc.markov_solve(sigma, x, 5.0, 1e-8, B)
    fwd = np.linalg.norm(X - Xc) / np.linalg.norm(Xc)
    log(f"  solve n={n} nrhs={nrhs} rule={rule}: berr={berr:.2e} fwd={fwd:.2e} factor be={be_fac:.2e}")
    if rule == 0:
        assert berr <= 1e-13
    else:
        assert berr <= 10 * max(be_fac, 1e-15)


def test_solve_full_size_16rhs(orc):
    """L=128 (N=16384, tile 512), 16 right-hand sides, FP64."""
    torch = torch_cuda()
    mod, h, n, sigma, x = _setup(orc, 128, 512)
    try:
        B = synth.rhs(n, 16)
        Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
        mod.mpchol_solve(h, Bt.T, n)
        torch.cuda.synchronize()
        X = Bt.T.cpu().numpy()
    finally:
        mod.mpchol_destroy(h)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    berr = np.linalg.norm(B - A @ X) / (np.linalg.norm(A) * np.linalg.norm(X) + np.linalg.norm(B))
    Xc = orc.markov_solve(sigma, x, 5.0, 1e-8, B)
    log(f"  solve N=16384: berr={berr:.2e} fwd={np.linalg.norm(X - Xc) / np.linalg.norm(Xc):.2e}")
    assert berr <= 1e-13


@pytest.mark.parametrize("count,seed", [(4099, 2), (1 << 16, 12345678901234)])
def test_philox_draws(orc, count, seed):
    torch = torch_cuda()
    mod = M()
    h = mod.mpchol_create(256, 128)
    try:
        z = torch.zeros(count, dtype=torch.float32, device="cuda")
        raw = torch.zeros(count, dtype=torch.int32, device="cuda")
        mod.mpchol_normal_draws(h, count, seed, z, raw)
        torch.cuda.synchronize()
    finally:
        mod.mpchol_destroy(h)
    zo, rawo = orc.normal_draws(seed, count)
    assert np.array_equal(raw.cpu().numpy().view(np.uint32), rawo)
    err = np.abs(z.cpu().numpy().astype(np.float64) - zo)
    assert np.all(err <= 4e-6 * np.maximum(1.0, np.abs(zo)))


@pytest.mark.parametrize("rule,eps", [(0, 1e-9), (1, 1e-4)])
def test_sample_z_matches_oracle_product(orc, rule, eps):
    torch = torch_cuda()
    L, tile, nd = 32, 128, 200
    mod, h, n, sigma, x = _setup(orc, L, tile, rule=rule, eps=eps)
    try:
        Lg = factor_dense(h, n)
        Z = synth.draws(n, nd)
        Zt = torch.tensor(np.ascontiguousarray(Z.T), device="cuda")
        Yt = torch.zeros((nd, n), dtype=torch.float32, device="cuda")
        mod.mpchol_sample_z(h, Zt.T, Yt.T, n)
        torch.cuda.synchronize()
        Y = Yt.T.cpu().numpy().astype(np.float64)
        be = mod.mpchol_backward_error(h)
    finally:
        mod.mpchol_destroy(h)
    # the oracle's FP64 product of the GPU's own factor (its represented
    # values) with the same draws: only the FP32 products and accumulation
    # of the draws kernel differ (about 1e-7)
    Yg = orc.lower_matmul(Lg, Z.astype(np.float64))
    rel = np.linalg.norm(Y - Yg) / np.linalg.norm(Yg)
    # for information: the distance to the product with the exact factor
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    Lo, _ = orc.potrf(A)
    Yo = orc.lower_matmul(Lo, Z.astype(np.float64))
    log(f"  sample_z rule={rule}: rel to L_gpu Z {rel:.2e}; to L_exact Z {np.linalg.norm(Y - Yo) / np.linalg.norm(Yo):.2e}")
    assert rel <= 1e-5


@pytest.mark.parametrize("n,kind", [(4096, "integer"), (3600, "integer"), (3600, "covariance")])
def test_sample_z_tile1024_mixed(orc, n, kind):
    """Y = L Z at the benchmark's tile size, 1024, with FP32, FP16 and FP8
    tiles (the second and third cases have a 528-row last tile): against the
    oracle's FP64 product of the GPU's own factor (its represented values) to
    1e-5, as a whole and row tile by row tile.  "integer": A = L0 L0^T with a
    user map cycling the three lower classes below the diagonal (the factor
    is L0 exactly); "covariance": the band-limit-60 covariance under the norm
    rule at eps = 1e-5."""
    torch = torch_cuda()
    tile, nd = 1024, 64
    nt = (n + tile - 1) // tile
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        if kind == "integer":
            L0 = synth.int_lower(n, 29)
            mod.mpchol_set_matrix(h, L0 @ L0.T)
            um = np.zeros((nt, nt), np.uint8)
            for J in range(nt):
                for I in range(J + 1, nt):
                    um[I, J] = 1 + (I + J) % 3
            mp = mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.asfortranarray(um))
        else:
            L = int(round(np.sqrt(n)))
            sigma, x = synth.workload(L)
            mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
            mp = mod.mpchol_precision_map(h, mod.RULE_NORM, 1e-5)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        Z = synth.draws(n, nd, 31)
        Zt = torch.tensor(np.ascontiguousarray(Z.T), device="cuda")
        Yt = torch.zeros((nd, n), dtype=torch.float32, device="cuda")
        mod.mpchol_sample_z(h, Zt.T, Yt.T, n)
        torch.cuda.synchronize()
        Y = Yt.T.cpu().numpy().astype(np.float64)
    finally:
        mod.mpchol_destroy(h)
    hist = np.bincount(mp[np.tril_indices(nt, -1)], minlength=4)
    if kind == "integer":
        assert np.array_equal(Lg, L0) and np.all(hist[1:] > 0)
    else:
        assert np.count_nonzero(hist) >= 2
    Yg = orc.lower_matmul(Lg, Z.astype(np.float64))
    rel = np.linalg.norm(Y - Yg) / np.linalg.norm(Yg)
    worst = max(np.linalg.norm(Y[r:r + tile] - Yg[r:r + tile]) / np.linalg.norm(Yg[r:r + tile])
                for r in range(0, n, tile))
    log(f"  sample_z tile 1024 n={n} {kind}: hist={hist} rel={rel:.2e} worst row tile {worst:.2e}")
    assert rel <= 1e-5 and worst <= 1e-5


def test_sample_is_philox_then_product(orc):
    """mpchol_sample(seed) equals mpchol_sample_z on the draws of the same seed,
    and the draws have the covariance of Sigma (per-coordinate variances)."""
    torch = torch_cuda()
    L, tile, nd = 32, 128, 1000
    mod, h, n, sigma, x = _setup(orc, L, tile)
    try:
        Y = torch.zeros((nd, n), dtype=torch.float32, device="cuda")
        mod.mpchol_sample(h, nd, 2, Y.T, n)
        Z = torch.zeros((nd, n), dtype=torch.float32, device="cuda")
        mod.mpchol_normal_draws(h, n * nd, 2, Z.reshape(-1), None)
        Y2 = torch.zeros((nd, n), dtype=torch.float32, device="cuda")
        mod.mpchol_sample_z(h, Z.T, Y2.T, n)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y2)
        Yh = Y.cpu().numpy().astype(np.float64)  # (nd, n)
    finally:
        mod.mpchol_destroy(h)
    var = Yh.var(axis=0)
    sii = sigma ** 2 + 1e-8
    ratio = var / sii
    log(f"  sample variance ratio mean={ratio.mean():.4f} min={ratio.min():.3f} max={ratio.max():.3f}")
    assert abs(ratio.mean() - 1.0) < 0.03
    assert ratio.min() > 0.7 and ratio.max() < 1.3
