"""The residual kernel (backward error ||Sigma - L L^T||_F / ||Sigma||_F and its
per-tile squared norms, which also drive the selector labels) pinned by
planted perturbations and against the oracle's residual of the same factor."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, same_factor_residuals, torch_cuda

pytestmark = pytest.mark.gpu


def _planted(n, b, I, J, seed):
    """Small-integer perturbation confined to tile (I, J) (symmetric when
    I == J), as a full symmetric n x n matrix."""
    u = synth.uniform01(seed, b * b).reshape(b, b)
    E = np.zeros((n, n))
    blk = np.floor(u * 9.0) - 4.0
    r0, c0 = I * b, J * b
    r1, c1 = min(n, r0 + b), min(n, c0 + b)
    blk = blk[:r1 - r0, :c1 - c0]
    if I == J:
        blk = np.tril(blk) + np.tril(blk, -1).T
    E[r0:r1, c0:c1] = blk
    if I != J:
        E[c0:c1, r0:r1] = blk.T
    return E


@pytest.mark.parametrize("n,tile,I,J,umap", [(1000, 128, 5, 2, False), (1024, 128, 7, 7, True), (1280, 256, 4, 1, True)])
def test_planted_perturbation_exact(n, tile, I, J, umap):
    """A0 = L0 L0^T with small integers factors to L0 exactly (in every class);
    the residual against A0 + tau E, E integer and confined to tile (I, J),
    tau = 2^-10, is exactly tau E: all of it lands in tile (I, J) (tau^2
    ||E_IJ||^2, bit for bit) and none elsewhere."""
    torch = torch_cuda()
    L0 = synth.int_lower(n, 23)
    A0 = L0 @ L0.T
    nt = (n + tile - 1) // tile
    tau = 2.0 ** -10
    E = _planted(n, tile, I, J, 71)
    A = A0 + tau * E
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_matrix(h, A0)
        if umap:
            u = synth.uniform01(37, nt * nt).reshape(nt, nt)
            um = np.asfortranarray(np.tril(np.floor(u * 4).astype(np.uint8), -1))
            mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, um)
        else:
            mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        assert np.array_equal(factor_dense(h, n), L0)
        be0, tr0 = mod.mpchol_backward_error(h, tiles=True)
        be_h, tr_h = mod.mpchol_backward_error_matrix(h, A, tiles=True)
        Ad = torch.tensor(np.ascontiguousarray(A.T), device="cuda")
        be_d, tr_d = mod.mpchol_backward_error_matrix(h, Ad.T, tiles=True)
        be_k = mod.mpchol_backward_error_matrix(h, A0)
    finally:
        mod.mpchol_destroy(h)
    log(f"  planted n={n} tile=({I},{J}) umap={umap}: be={be_h:.6e}")
    assert be0 == 0.0 and np.all(tr0 == 0.0) and be_k == 0.0
    want = np.zeros((nt, nt))
    blk = E[I * tile:(I + 1) * tile, J * tile:(J + 1) * tile]
    # a diagonal tile counts its strict-lower entries twice (both triangles)
    want[I, J] = tau ** 2 * (np.sum(blk ** 2) if I != J else np.sum(np.tril(blk) ** 2) + np.sum(np.tril(blk, -1) ** 2))
    assert np.array_equal(tr_h, want)
    assert np.array_equal(tr_d, tr_h) and be_d == be_h
    expect = tau * np.linalg.norm(E) / np.linalg.norm(A)
    assert abs(be_h - expect) <= 1e-12 * expect


@pytest.mark.parametrize("L,tile,rho,tau", [(32, 128, 5.0, 1e-10), (40, 256, 2.0, 1e-12)])
def test_planted_perturbation_of_covariance(orc, L, tile, rho, tau):
    """The paper's covariance factored in FP64, judged against Sigma + tau E0
    (E0 symmetric N(0,1)): the backward error returns tau ||E0|| / ||Sigma +
    tau E0|| to 1e-3 relative, and equals the oracle's residual of the same
    factor against the same matrix."""
    n = L * L
    sigma, x = synth.workload(L)
    S = orc.cov_dense(sigma, x, rho, 1e-8)
    g = synth.draws(n, n).astype(np.float64)
    E0 = (g + g.T) / np.sqrt(2.0)
    A = S + tau * E0
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be, tr = mod.mpchol_backward_error_matrix(h, A, tiles=True)
    finally:
        mod.mpchol_destroy(h)
    expect = tau * np.linalg.norm(E0) / np.linalg.norm(A)
    log(f"  planted covariance L={L} tau={tau}: be={be:.6e} expected {expect:.6e}")
    assert abs(be - expect) <= 1e-3 * expect
    same_factor_residuals(be, tr, orc.backward_error(A, Lg), orc.tile_residual2(A, Lg, tile), A, tile)


@pytest.mark.parametrize("L,tile,rho,eps", [(32, 128, 5.0, 1e-9), (48, 256, 5.0, 1e-7), (30, 128, 2.0, 1e-5),
                                            (64, 512, 20.0, 1e-8)])
def test_residual_same_factor_mixed(orc, L, tile, rho, eps):
    """Mixed maps with backward errors from 1e-10 to 1e-5: the residual kernel
    (generator source) and the caller-matrix call both against the oracle's
    residual of the GPU's own factor, in total and tile by tile."""
    n = L * L
    sigma, x = synth.workload(L)
    A = orc.cov_dense(sigma, x, rho, 1e-8)
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
        mp = mod.mpchol_precision_map(h, mod.RULE_NORM, eps)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be, tr = mod.mpchol_backward_error(h, tiles=True)
        be_m, tr_m = mod.mpchol_backward_error_matrix(h, A, tiles=True)
    finally:
        mod.mpchol_destroy(h)
    be_o, tr_o = orc.backward_error(A, Lg), orc.tile_residual2(A, Lg, tile)
    hist = np.bincount(mp[np.tril_indices(mp.shape[0], -1)], minlength=4)
    w = same_factor_residuals(be, tr, be_o, tr_o, A, tile)
    w2 = same_factor_residuals(be_m, tr_m, be_o, tr_o, A, tile)
    log(f"  same factor L={L} eps={eps} hist={hist}: be_gpu={be:.6e} be_oracle={be_o:.6e} "
        f"worst tile {w:.2e}/{w2:.2e} of the tolerance")
