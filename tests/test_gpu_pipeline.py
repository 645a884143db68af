"""The built rows chained as in the paper's pipeline (Sec. III.A.1 -> III.A.3):
fields -> SHT coefficient vectors -> their covariance (the producer, with the
vectors themselves standing in for the VAR residuals) -> factorization ->
log-determinant, against the oracle chained the same way."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,nth,nph,T,tile,mixed", [(12, 13, 24, 300, 128, False), (20, 21, 40, 500, 128, False),
                                                     (24, 25, 48, 700, 128, True)])
def test_fields_to_factor(orc, sht_orc, L, nth, nph, T, tile, mixed):
    torch = torch_cuda()
    mod = M()
    n = L * L
    Z = synth.sht_fields(T, nth, nph, seed=80 + L)
    scale, nugget = 1.0 / T, 1e-6
    s = mod.mpchol_sht_create(L, nth, nph, T)
    h = mod.mpchol_create(n, tile)
    try:
        f = torch.empty((T, n), dtype=torch.float64, device="cuda")
        mod.mpchol_sht_forward(s, torch.tensor(Z, device="cuda"), f, L)
        torch.cuda.synchronize()
        # f is T x n row-major, i.e. the n x T column-major sample matrix
        mod.mpchol_set_samples(h, f.T, scale, nugget)
        nt = (n + tile - 1) // tile
        if mixed:
            mp = mod.mpchol_precision_map(h, mod.RULE_NORM, 1e-6)
        else:
            mp = mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        ld = mod.mpchol_logdet(h)
        be = mod.mpchol_backward_error(h)
        fg = f.cpu().numpy()
    finally:
        mod.mpchol_destroy(h)
        mod.mpchol_sht_destroy(s)
    D = sht_orc.wigner_table(L)
    fo = np.array([sht_orc.sht_forward_real(Z[t], L, D) for t in range(T)])
    assert np.abs(fg - fo).max() <= 1e-12 * np.abs(fo).max()
    S = orc.cov_samples(np.asfortranarray(fo.T), scale, nugget)
    Lo, info = orc.potrf(S)
    assert info == 0
    ld_o = orc.logdet(Lo)
    beo = orc.backward_error(S, Lg)
    log(f"  pipeline L={L} T={T} mixed={mixed}: logdet {ld:.6f} vs {ld_o:.6f}, be vs oracle Sigma {beo:.2e}, "
        f"be {be:.2e}, classes {np.bincount(mp[np.tril_indices(nt, -1)], minlength=4).tolist()}")
    if mixed:
        assert beo <= 1e-6 and be <= 1e-6
        assert abs(ld - ld_o) <= 1e-4 * abs(ld_o)
    else:
        assert beo <= 1e-13
        assert abs(ld - ld_o) <= 1e-11 * abs(ld_o)
