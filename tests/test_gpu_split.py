"""FP32-class updates from three-way BF16 splits (lo32 = BF16x3): exactness on
integer factors, parity with the oracle's split replay, and the accuracy
budget of the norm rule at full size."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, same_factor_residuals, tile_rel, tile_residual_levels

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,tile,kind", [(1024, 128, "all32"), (1000, 128, "mixed"), (1280, 256, "mixed")])
def test_split_integer_factor_bit_exact(n, tile, kind):
    """A = L0 L0^T with small integers: the split of every FP32 operand is
    exact and so are the part products, so the factor equals L0 bit for bit
    (covers the split copies' layout, the six part pairs and the pairs of
    steps)."""
    log(f"split integer exact n={n} tile={tile} kind={kind}")
    L0 = synth.int_lower(n, 17)
    A = L0 @ L0.T
    nt = (n + tile - 1) // tile
    if kind == "mixed":
        u = synth.uniform01(31, nt * nt).reshape(nt, nt)
        um = np.tril(np.floor(u * 4).astype(np.uint8), -1)
    else:
        um = np.tril(np.ones((nt, nt), np.uint8), -1)
    mod = M()
    h = mod.mpchol_create(n, tile, lo32=mod.LO32_BF16X3)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.asfortranarray(um))
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be = mod.mpchol_backward_error(h)
    finally:
        mod.mpchol_destroy(h)
    assert np.array_equal(Lg, L0)
    assert be == 0.0


@pytest.mark.parametrize("n,tile,seed,lo16", [(1024, 128, 31, 0), (1000, 128, 32, 1), (1280, 256, 33, 0)])
def test_split_user_map_against_replay(orc, n, tile, seed, lo16):
    """A map using every class on a well-conditioned covariance, against the
    oracle replay with the same split products; tolerance as for the plain
    FP32 path (eight times the spread between two summation orders)."""
    olo = orc.F16 if lo16 == 0 else orc.BF16
    L = int(np.ceil(np.sqrt(n)))
    sigma, x = synth.workload(L)
    sigma, x = sigma[:n], x[:n]
    A = orc.cov_dense(sigma, x, 5.0, 1e-2)
    nt = (n + tile - 1) // tile
    u = synth.uniform01(seed, nt * nt).reshape(nt, nt)
    um = np.asfortranarray(np.tril(np.floor(u * 4).astype(np.uint8), -1))
    mod = M()
    h = mod.mpchol_create(n, tile, lo16=lo16, lo32=mod.LO32_BF16X3)
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
    L0, _, t0 = orc.mp_factor(A, tile, um, lo16=olo, order=0, lo32=1)
    L1, _, _ = orc.mp_factor(A, tile, um, lo16=olo, order=1, lo32=1)
    assert np.array_equal(tg, t0)
    d_oo = np.linalg.norm(L0 - L1) / np.linalg.norm(L0)
    d_go = np.linalg.norm(Lg - L0) / np.linalg.norm(L0)
    be_o = orc.backward_error(A, L0)
    log(f"  split user map n={n}: be_gpu={be_g:.3e} be_O2={be_o:.3e} |G-O2|={d_go:.2e} |O2-O2'|={d_oo:.2e}")
    assert d_go <= 8.0 * d_oo + 1e-14
    assert tile_rel(Lg, L0, tile) <= 8.0 * max(tile_rel(L1, L0, tile), 1e-14) + 1e-13
    assert abs(be_g - be_o) <= 0.25 * be_o
    tile_residual_levels(tr_g, orc.tile_residual2(A, L0, tile), A, tile)


@pytest.mark.parametrize("rho,eps", [(2.0, 1e-9), (5.0, 1e-9)])
def test_split_full_size_65536(orc, rho, eps):
    """The norm rule at N = 65,536 (FP64/FP32/BF16) with the split FP32-class
    products: the same map as the FP32 path, backward error <= eps and logdet
    within 1e-8 of the closed form."""
    L, tile = 256, 1024
    n = L * L
    sigma, x = synth.workload(L)
    mod = M()
    res = {}
    for lo32 in (mod.LO32_FP32, mod.LO32_BF16X3):
        h = mod.mpchol_create(n, tile, lo16=mod.LO16_BF16, allowed=0b0111, lo32=lo32)
        try:
            mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
            mp = mod.mpchol_precision_map(h, mod.RULE_NORM, eps)
            assert mod.mpchol_factor(h) == 0
            be = mod.mpchol_backward_error(h)
            ld = mod.mpchol_logdet(h)
            st = mod.mpchol_get_stats(h)
        finally:
            mod.mpchol_destroy(h)
        res[lo32] = (mp, be, ld, st["t_factor_ms"])
    ref = orc.markov_logdet(sigma, x, rho, 1e-8)
    (mp0, be0, ld0, t0), (mp1, be1, ld1, t1) = res[0], res[1]
    log(f"  N=65536 rho={rho}: FP32 be={be0:.3e} {t0:.0f} ms; split be={be1:.3e} {t1:.0f} ms, "
        f"logdet rel {abs(ld1 - ref) / abs(ref):.2e}")
    assert np.array_equal(mp0, mp1)
    assert be1 <= eps
    assert abs(ld1 - ref) / abs(ref) <= 1e-8
