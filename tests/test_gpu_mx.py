"""Block-scaled FP8 copies (lo8 = MX: one E8M0 scale per 32 consecutive K
elements of a row, applied inside the block-scaled FP8 MFMA) against the
oracle's definition of the copies and its replay of the tile algorithm."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, same_factor_residuals, tile_rel, tile_residual_levels

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,tile,kind,lo8", [(1000, 128, "all8", 1), (1000, 128, "mixed", 1), (1500, 256, "mixed", 1),
                                             (3648, 1024, "mixed", 1), (3648, 1024, "all8", 1),
                                             (1000, 128, "mixed", 0), (3648, 1024, "mixed", 0)])
def test_graded_integer_factor_bit_exact(n, tile, kind, lo8):
    """A = L0 L0^T with graded integers: magnitudes change from row to row and
    from one 32-column block of a row to the next, so the block scales of a
    copy differ (E8M0 exponents 4..7 within a row).  Every value is exact in
    every class, so the factor must be L0 bit for bit -- with the per-tile
    scales as well as the block scales; a block read at another block's
    scale, or a scale byte read from the wrong lane, would not give L0."""
    log(f"graded integer n={n} tile={tile} kind={kind} lo8={lo8}")
    L0 = synth.int_lower(n, 17, graded=True)
    A = L0 @ L0.T
    nt = (n + tile - 1) // tile
    if kind == "mixed":
        u = synth.uniform01(23, nt * nt).reshape(nt, nt)
        um = np.tril(np.floor(u * 4).astype(np.uint8), -1)
        um[1:, 0] = 0  # the first panel column stored in FP64: FP8 updates read its block-scaled copies
    else:
        um = np.tril(np.full((nt, nt), 3, np.uint8), -1)
    mod = M()
    h = mod.mpchol_create(n, tile, lo8=lo8, band=0)
    try:
        mod.mpchol_set_matrix(h, A)
        cmap = mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.asfortranarray(um))
        assert np.array_equal(cmap, um)
        log("  factor")
        assert mod.mpchol_factor(h) == 0
        log("  factor done; read back")
        Lg = factor_dense(h, n)
        be = mod.mpchol_backward_error(h)
    finally:
        mod.mpchol_destroy(h)
    log(f"  max |L - L0| = {np.max(np.abs(Lg - L0)):.3e}, backward error {be:.3e}")
    assert np.array_equal(Lg, L0)
    assert be == 0.0


@pytest.mark.parametrize("n,tile,seed,lo16,lo32", [(1000, 128, 61, 0, 0), (1200, 256, 62, 1, 1), (3648, 1024, 63, 0, 1)])
def test_mx_against_replay(orc, n, tile, seed, lo16, lo32):
    """A random map over every class (band 0) on a covariance, with
    block-scaled FP8 copies: against O2 with the same copies, stored scales
    bit-equal, global distance within 8x the order spread, worst tile within
    8x the worst tile spread, every tile's residual at O2's level, backward
    errors within 25%; the residual kernel against the oracle on the GPU's own
    factor."""
    olo = orc.F16 if lo16 == 0 else orc.BF16
    L = int(np.ceil(np.sqrt(n)))
    sigma, x = synth.workload(L)
    sigma, x = sigma[:n], x[:n]
    A = orc.cov_dense(sigma, x, 5.0, 1e-2)
    nt = (n + tile - 1) // tile
    u = synth.uniform01(seed, nt * nt).reshape(nt, nt)
    um = np.asfortranarray(np.tril(np.floor(u * 4).astype(np.uint8), -1))
    log(f"mx replay n={n} tile={tile} seed={seed} lo16={lo16} lo32={lo32}")
    mod = M()
    h = mod.mpchol_create(n, tile, lo16=lo16, lo32=lo32, lo8=mod.LO8_MX, band=0)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, um)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        tg = mod.mpchol_get_tile_scales(h, nt)
        be_g, tr_g = mod.mpchol_backward_error(h, tiles=True)
    finally:
        mod.mpchol_destroy(h)
    same_factor_residuals(be_g, tr_g, orc.backward_error(A, Lg), orc.tile_residual2(A, Lg, tile), A, tile)
    L0, i0, t0 = orc.mp_factor(A, tile, um, lo16=olo, order=0, lo32=lo32, lo8=1)
    L1, i1, _ = orc.mp_factor(A, tile, um, lo16=olo, order=1, lo32=lo32, lo8=1)
    assert i0 == 0 and i1 == 0
    assert np.array_equal(tg, t0)
    d_oo = np.linalg.norm(L0 - L1) / np.linalg.norm(L0)
    d_go = np.linalg.norm(Lg - L0) / np.linalg.norm(L0)
    be_o = orc.backward_error(A, L0)
    lo_r, hi_r, cnt = tile_residual_levels(tr_g, orc.tile_residual2(A, L0, tile), A, tile)
    log(f"  be_gpu={be_g:.3e} be_O2={be_o:.3e} |G-O2|={d_go:.2e} |O2-O2'|={d_oo:.2e} "
        f"tile residual GPU/O2 [{lo_r:.3f}, {hi_r:.3f}] over {cnt}")
    assert d_go <= 8.0 * d_oo + 1e-14
    assert tile_rel(Lg, L0, tile) <= 8.0 * max(tile_rel(L1, L0, tile), 1e-14) + 1e-13
    assert abs(be_g - be_o) <= 0.25 * be_o


def test_full_size_mx_129600(orc):
    """The headline workload (L = 360, N = 129,600, tile 1024) under the norm
    rule with block-scaled FP8 copies: exact backward error <= 1e-9 and logdet
    against the closed form <= 1e-8."""
    L, tile = 360, 1024
    n = L * L
    sigma, x = synth.workload(L)
    mod = M()
    h = mod.mpchol_create(n, tile, lo8=mod.LO8_MX)
    try:
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        mp = mod.mpchol_precision_map(h, mod.RULE_NORM, 1e-9)
        assert mod.mpchol_factor(h) == 0
        be = mod.mpchol_backward_error(h)
        ld = mod.mpchol_logdet(h)
        st = mod.mpchol_get_stats(h)
    finally:
        mod.mpchol_destroy(h)
    ref = orc.markov_logdet(sigma, x, 5.0, 1e-8)
    hist = np.bincount(mp[np.tril_indices(mp.shape[0], -1)], minlength=4)
    log(f"  N=129600 norm, MX copies: hist={hist} be={be:.3e} logdet rel={abs(ld - ref) / abs(ref):.2e} "
        f"t_factor={st['t_factor_ms']:.0f} ms")
    assert hist[3] > 0
    assert be <= 1e-9
    assert abs(ld - ref) / abs(ref) <= 1e-8
