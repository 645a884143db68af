"""Covariance from samples (mpchol_set_samples): Sigma = scale * Xi Xi^T +
nugget I on the GPU, against the oracle's definition."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,tile,kind", [(1000, 128, "fp64"), (1000, 128, "mixed"), (1152, 256, "fp64")])
def test_hadamard_samples_give_exact_factor(n, tile, kind):
    """Xi = L0 H_n (first n rows of a Sylvester-Hadamard matrix of order m,
    H_n H_n^T = m I) with scale 1/m: Sigma = L0 L0^T exactly, so the factor
    equals L0 bit for bit (covers the packing, the padded K range, the tile
    placement and the ragged last tile)."""
    m = 1024 if n <= 1024 else 2048
    log(f"hadamard samples n={n} m={m} tile={tile} {kind}")
    L0 = synth.int_lower(n, 19)
    xi = np.asfortranarray(L0 @ synth.hadamard(m)[:n, :])
    nt = (n + tile - 1) // tile
    if kind == "mixed":
        u = synth.uniform01(29, nt * nt).reshape(nt, nt)
        um = np.asfortranarray(np.tril(np.floor(u * 4).astype(np.uint8), -1))
    else:
        um = np.zeros((nt, nt), np.uint8, order="F")
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_samples(h, xi, 1.0 / m, 0.0)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, um)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be = mod.mpchol_backward_error(h)
        st = mod.mpchol_get_stats(h)
    finally:
        mod.mpchol_destroy(h)
    log(f"  t_samples={st['t_samples_ms']:.2f} ms be={be}")
    assert np.array_equal(Lg, L0)
    assert be == 0.0


@pytest.mark.parametrize("n,m,tile,pad", [(900, 300, 128, 5), (1280, 77, 256, 0), (640, 1000, 128, 3)])
def test_random_samples_match_oracle(orc, n, m, tile, pad):
    """Seeded residual-like samples (m not a multiple of 16, ld > n, a ragged
    last tile, fewer or more samples than n): the FP64 factor of the GPU's
    Sigma has backward error <= 1e-13 against the oracle's Sigma, and the same
    logdet, so the two Sigma agree to FP64 rounding."""
    xi = synth.samples(n, m)
    X = np.zeros((n + pad, m), order="F")
    X[:n] = xi
    scale, nugget = 1.0 / m, 1e-2
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        rc = mod.lib().mpchol_set_samples(h, X.ctypes.data_as(__import__("ctypes").c_void_p), n + pad, m, scale, nugget, 0)
        assert rc == 0
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        ld = mod.mpchol_logdet(h)
    finally:
        mod.mpchol_destroy(h)
    S = orc.cov_samples(xi, scale, nugget)
    be = orc.backward_error(S, Lg)
    Lo, info = orc.potrf(S)
    assert info == 0
    ld_o = orc.logdet(Lo)
    log(f"  samples n={n} m={m}: be vs oracle Sigma {be:.2e}, logdet rel {abs(ld - ld_o) / abs(ld_o):.2e}")
    assert be <= 1e-13
    assert abs(ld - ld_o) <= 1e-12 * abs(ld_o)


def test_device_and_host_samples_agree():
    torch = torch_cuda()
    n, m, tile = 700, 200, 128
    xi = synth.samples(n, m)
    mod = M()
    outs = []
    for dev in (False, True):
        h = mod.mpchol_create(n, tile)
        try:
            if dev:
                Xt = torch.tensor(np.ascontiguousarray(xi.T), device="cuda")  # Xt.T is column-major xi
                mod.mpchol_set_samples(h, Xt.T, 1.0 / m, 1e-3)
            else:
                mod.mpchol_set_samples(h, xi, 1.0 / m, 1e-3)
            mod.mpchol_precision_map(h, mod.RULE_FP64)
            assert mod.mpchol_factor(h) == 0
            outs.append(factor_dense(h, n))
        finally:
            mod.mpchol_destroy(h)
    assert np.array_equal(outs[0], outs[1])


def test_samples_argument_errors():
    import ctypes as C

    mod = M()
    n = 512
    h = mod.mpchol_create(n, 128)
    try:
        X = np.zeros((n, 4), order="F")
        p = X.ctypes.data_as(C.c_void_p)
        L = mod.lib()
        assert L.mpchol_set_samples(h, p, n - 1, 4, 1.0, 0.0, 0) == -1   # ldxi < n
        assert L.mpchol_set_samples(h, p, n, 0, 1.0, 0.0, 0) == -1       # no samples
        assert L.mpchol_set_samples(h, p, n, 4, 0.0, 0.0, 0) == -1       # scale <= 0
        assert L.mpchol_set_samples(h, p, n, 4, 1.0, -1.0, 0) == -1      # nugget < 0
        assert L.mpchol_set_samples(h, None, n, 4, 1.0, 0.0, 0) == -1
    finally:
        mod.mpchol_destroy(h)


def test_samples_sampled_entries_at_8192(orc):
    """n = 8192, m = 2048, tile 512: entries of the factor's product L L^T at
    seeded positions against the oracle's definition evaluated entry by entry
    (scale * sum_k xi_ik xi_jk + nugget delta_ij)."""
    torch = torch_cuda()
    n, m, tile = 8192, 2048, 512
    xi = synth.samples(n, m)
    scale, nugget = 1.0 / m, 1e-3
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_samples(h, xi, scale, nugget)
        st = mod.mpchol_get_stats(h)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
    finally:
        mod.mpchol_destroy(h)
    flops = n * (n + 1) * m
    log(f"  samples n={n} m={m}: {st['t_samples_ms']:.1f} ms, {flops / st['t_samples_ms'] / 1e9:.1f} TFLOP/s")
    u = synth.uniform01(53, 2 * 256).reshape(256, 2)
    idx = np.floor(u * n).astype(np.int64)
    ii, jj = np.maximum(idx[:, 0], idx[:, 1]), np.minimum(idx[:, 0], idx[:, 1])
    ii[:8] = jj[:8]  # some diagonal entries
    sub = orc.cov_samples(np.vstack([xi[ii], xi[jj]]), scale, 0.0)  # entry (p, 256 + p) = scale xi_i . xi_j
    k = len(ii)
    want = np.array([sub[p, k + p] for p in range(k)]) + nugget * (ii == jj)
    got = np.einsum("pk,pk->p", Lg[ii], Lg[jj])
    rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
    log(f"  sampled entries: max |LL^T - Sigma| / max|Sigma| = {rel:.2e}")
    assert rel <= 1e-13
