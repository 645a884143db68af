"""FP64-class updates formed from exact integer products on the INT8 MFMA
(lo64 = INT8, the Ozaki scheme II) against the oracle's definition of the
same products: bit for bit where every other step is exact, and at FP64
level on the covariance."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, same_factor_residuals, tile_rel, tile_residual_levels

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,tile", [(384, 128), (3072, 1024), (2624, 1024)])
def test_int8_product_bit_exact(orc, n, tile):
    """Three tile columns with A00 = I and integer A10 (so L10 = A10 and
    L11 = I exactly): tile (2,1) of the factor is A21 - D(A20, A10) with D the
    emulated product, bit for bit against the oracle's definition (A20 and
    A21 arbitrary doubles; the last case has a 576-row last tile)."""
    b = tile
    n2 = n - 2 * b
    A10 = np.floor(synth.uniform01(62, b * b).reshape(b, b) * 7.0) - 3.0
    A20 = synth.normal(63, n2 * b).reshape(n2, b) * np.logspace(-2, 1, b)[None, :]
    A21 = synth.normal(64, n2 * b).reshape(n2, b)
    A = np.zeros((n, n))
    A[:b, :b] = np.eye(b)
    A[b:2 * b, :b] = A10
    A[b:2 * b, b:2 * b] = np.eye(b) + A10 @ A10.T
    A[2 * b:, :b] = A20
    A[2 * b:, b:2 * b] = A21
    A[2 * b:, 2 * b:] = 1e9 * np.eye(n2)
    A = np.tril(A) + np.tril(A, -1).T
    mod = M()
    h = mod.mpchol_create(n, tile, band=0, lo64=mod.LO64_INT8)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.zeros((3, 3), np.uint8))
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
    finally:
        mod.mpchol_destroy(h)
    assert np.array_equal(Lg[:b, :b], np.eye(b)) and np.array_equal(Lg[b:2 * b, b:2 * b], np.eye(b))
    assert np.array_equal(Lg[b:2 * b, :b], A10) and np.array_equal(Lg[2 * b:, :b], A20)
    want = A21 - orc.ozaki_gemm(A20, A10)
    got = Lg[2 * b:, b:2 * b]
    log(f"  int8 product n={n} tile={tile}: max |got - want| = {np.abs(got - want).max():.3e}, "
        f"distance to the FP64 product {np.abs(want - (A21 - A20 @ A10.T)).max():.3e}")
    assert np.array_equal(got.view(np.int64), want.view(np.int64))


@pytest.mark.parametrize("n,tile,mixed", [(1024, 128, False), (1000, 128, True), (1280, 256, True)])
def test_int8_integer_factor_bit_exact(n, tile, mixed):
    """A = L0 L0^T with small integers: every scaled entry is an exact
    integer and the products are exact, so the factor equals L0 bit for bit
    (FP64 map with band 0, and a random map over every class)."""
    L0 = synth.int_lower(n, 17)
    A = L0 @ L0.T
    nt = (n + tile - 1) // tile
    if mixed:
        u = synth.uniform01(43, nt * nt).reshape(nt, nt)
        um = np.asfortranarray(np.tril(np.floor(u * 4).astype(np.uint8), -1))
    else:
        um = np.zeros((nt, nt), np.uint8)
    mod = M()
    h = mod.mpchol_create(n, tile, band=0, lo64=mod.LO64_INT8)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, um)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be = mod.mpchol_backward_error(h)
    finally:
        mod.mpchol_destroy(h)
    assert np.array_equal(Lg, L0) and be == 0.0


@pytest.mark.parametrize("L,tile,rho,band", [(32, 128, 5.0, 0), (40, 256, 2.0, 1), (30, 128, 20.0, 0)])
def test_int8_fp64_parity(orc, L, tile, rho, band):
    """The covariance with every tile FP64, the off-band products formed from
    INT8 products: backward error at FP64 level (<= 1e-14), logdet against the
    closed form <= 1e-12, the distance to the exact factor no more than 4x
    that of the FP64-MFMA path, and within rounding of the oracle's replay of
    the same arithmetic."""
    n = L * L
    nt = (n + tile - 1) // tile
    sigma, x = synth.workload(L)
    A = orc.cov_dense(sigma, x, rho, 1e-8)
    mod = M()
    out = {}
    for lo64 in (mod.LO64_FP64, mod.LO64_INT8):
        h = mod.mpchol_create(n, tile, band=band, lo64=lo64)
        try:
            mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
            mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.zeros((nt, nt), np.uint8))
            assert mod.mpchol_factor(h) == 0
            out[lo64] = (factor_dense(h, n), mod.mpchol_backward_error(h), mod.mpchol_logdet(h))
        finally:
            mod.mpchol_destroy(h)
    ref = orc.markov_logdet(sigma, x, rho, 1e-8)
    Lo, _ = orc.potrf(A)
    L2, i2, _ = orc.mp_factor(A, tile, np.zeros((nt, nt), np.uint8), lo64=1, band=band)
    assert i2 == 0
    (Lf, bef, _), (Lg, be, ld) = out[mod.LO64_FP64], out[mod.LO64_INT8]
    nrm = np.linalg.norm(Lo)
    d_g, d_f, d_o2 = (np.linalg.norm(Lg - Lo) / nrm, np.linalg.norm(Lf - Lo) / nrm,
                      np.linalg.norm(Lg - L2) / np.linalg.norm(L2))
    d_2 = np.linalg.norm(L2 - Lo) / nrm
    log(f"  int8 fp64 L={L} band={band}: be={be:.2e} (FP64 MFMA {bef:.2e}) logdet rel={abs(ld - ref) / abs(ref):.2e} "
        f"|G-O1|={d_g:.2e} |G_fp64-O1|={d_f:.2e} |O2-O1|={d_2:.2e} |G-O2|={d_o2:.2e}")
    assert be <= 1e-14
    assert abs(ld - ref) <= 1e-12 * abs(ref)
    assert d_g <= 4.0 * max(d_f, d_2) + 1e-15
    assert d_o2 <= 4.0 * max(d_f, d_2) + 1e-15


@pytest.mark.parametrize("L,tile,rho,eps,lo16", [(32, 128, 5.0, 1e-9, 0), (32, 128, 2.0, 1e-5, 1),
                                                 (48, 256, 5.0, 1e-7, 0)])
def test_int8_mixed_against_replay(orc, L, tile, rho, eps, lo16):
    """Norm-rule maps with the FP64-class products from INT8 products, against
    O2 replaying the same arithmetic: map equal, global and worst-tile
    distance within 8x the order spread, every tile's residual at O2's level,
    residual kernel on the GPU's own factor, logdet."""
    n = L * L
    nt = (n + tile - 1) // tile
    olo = orc.F16 if lo16 == 0 else orc.BF16
    sigma, x = synth.workload(L)
    A = orc.cov_dense(sigma, x, rho, 1e-8)
    mod = M()
    h = mod.mpchol_create(n, tile, lo16=lo16, lo32=mod.LO32_FP32, lo64=mod.LO64_INT8)
    try:
        mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
        mg = mod.mpchol_precision_map(h, mod.RULE_NORM, eps)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be_g, tr_g = mod.mpchol_backward_error(h, tiles=True)
    finally:
        mod.mpchol_destroy(h)
    same_factor_residuals(be_g, tr_g, orc.backward_error(A, Lg), orc.tile_residual2(A, Lg, tile), A, tile)
    L0, i0, _ = orc.mp_factor(A, tile, mg, lo16=olo, order=0, lo64=1, band=1)
    L1, i1, _ = orc.mp_factor(A, tile, mg, lo16=olo, order=1, lo64=1, band=1)
    assert i0 == 0 and i1 == 0
    d_oo = np.linalg.norm(L0 - L1) / np.linalg.norm(L0)
    d_go = np.linalg.norm(Lg - L0) / np.linalg.norm(L0)
    lo_r, hi_r, cnt = tile_residual_levels(tr_g, orc.tile_residual2(A, L0, tile), A, tile)
    hist = np.bincount(mg[np.tril_indices(nt, -1)], minlength=4)
    log(f"  int8 mixed L={L} eps={eps}: hist={hist} be={be_g:.3e} |G-O2|={d_go:.2e} |O2-O2'|={d_oo:.2e} "
        f"tile residual GPU/O2 [{lo_r:.3f}, {hi_r:.3f}] over {cnt}")
    assert d_go <= 8.0 * d_oo + 1e-14
    assert tile_rel(Lg, L0, tile) <= 8.0 * max(tile_rel(L1, L0, tile), 1e-14) + 1e-13
    assert be_g <= max(eps, 1e-13) or eps > 1e-9


def test_int8_rejects_large_tiles():
    mod = M()
    with pytest.raises(Exception):
        mod.mpchol_create(4096, 2048, lo64=mod.LO64_INT8)
