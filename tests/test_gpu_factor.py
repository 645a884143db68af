"""FP64 path of the HIP tile Cholesky against the oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from _gpu import M, factor_dense, log, tile_rel, torch_cuda

pytestmark = pytest.mark.gpu


def _sun_bound(A, L, be_sum):
    """First-order bound on ||L1 - L2||_F / ||L||_2 for the exact factors of two
    perturbations A + E1, A + E2 with ||E1 - E2||_F <= be_sum ||A||_F
    (Sun 1991): kappa_2(A) / sqrt(2) * ||E||_F / ||A||_2."""
    w = np.linalg.eigvalsh(A)
    kappa = w[-1] / w[0]
    return kappa / np.sqrt(2.0) * be_sum * np.linalg.norm(A) / w[-1]


@pytest.mark.parametrize("L,tile,rho", [(32, 128, 5.0), (24, 128, 5.0), (32, 256, 2.0), (20, 128, 20.0)])
def test_fp64_parity_small(orc, L, tile, rho):
    """Several tiles and (L=24, 20) a ragged last tile."""
    n = L * L
    log(f"fp64 parity n={n} tile={tile} rho={rho}")
    sigma, x = synth.workload(L)
    A = orc.cov_dense(sigma, x, rho, 1e-8)
    Lo, info_o = orc.potrf(A)
    assert info_o == 0
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
        cmap = mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert np.all(cmap == 0)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be_gpu = mod.mpchol_backward_error(h)
        ld = mod.mpchol_logdet(h)
    finally:
        mod.mpchol_destroy(h)
    assert np.all(np.triu(Lg, 1) == 0) and np.all(np.diag(Lg) > 0)
    be_np = np.linalg.norm(A - Lg @ Lg.T) / np.linalg.norm(A)
    be_o = orc.backward_error(A, Lo)
    assert be_gpu <= 1e-13 and be_np <= 1e-13
    # both residuals sit at the FP64 rounding floor, where each is computed to
    # O(1) relative accuracy only: require the same order of magnitude
    assert abs(be_gpu - be_np) <= 0.5 * be_np
    tol = _sun_bound(A, Lo, be_np + be_o)
    diff = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo, 2)
    log(f"  be_gpu={be_gpu:.2e} diff={diff:.2e} bound={tol:.2e}")
    assert diff <= tol
    ref = orc.markov_logdet(sigma, x, rho, 1e-8)
    assert abs(ld - ref) / abs(ref) <= 1e-12


@pytest.mark.parametrize("n,tile,lo16,kind", [
    (1024, 128, 0, "fp64"), (1024, 128, 0, "mixed"), (1024, 128, 1, "mixed"),
    (1000, 128, 0, "mixed"), (1152, 256, 0, "mixed"), (640, 128, 1, "all8"), (777, 128, 0, "all16"),
    (4096, 1024, 0, "mixed"), (3600, 1024, 1, "mixed")])
def test_integer_factor_bit_exact(n, tile, lo16, kind):
    """A = L0 L0^T with small integers: every class computes L0 exactly, so the
    GPU factor must equal L0 bit for bit (covers MFMA layouts, scaling, FP8
    E4M3 and FP16/BF16 codes, conversions and padding)."""
    log(f"integer exact n={n} tile={tile} lo16={lo16} kind={kind}")
    L0 = synth.int_lower(n, 17)
    A = L0 @ L0.T
    nt = (n + tile - 1) // tile
    if kind == "mixed":
        u = synth.uniform01(23, nt * nt).reshape(nt, nt)
        um = np.tril(np.floor(u * 4).astype(np.uint8), -1)
    else:
        c = {"fp64": 0, "all8": 3, "all16": 2}[kind]
        um = np.tril(np.full((nt, nt), c, np.uint8), -1)
    mod = M()
    h = mod.mpchol_create(n, tile, lo16=lo16)
    try:
        mod.mpchol_set_matrix(h, A)
        cmap = mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, np.asfortranarray(um))
        assert np.array_equal(cmap, um)
        assert mod.mpchol_factor(h) == 0
        Lg = factor_dense(h, n)
        be = mod.mpchol_backward_error(h)
        ld = mod.mpchol_logdet(h)
    finally:
        mod.mpchol_destroy(h)
    assert np.array_equal(Lg, L0)
    assert be == 0.0
    ref = 2.0 * np.sum(np.log(np.diag(L0)))
    assert abs(ld - ref) <= 1e-13 * abs(ref)


def test_set_matrix_device_and_host_agree():
    torch = torch_cuda()
    n, tile = 700, 128
    L0 = synth.int_lower(n, 5)
    A = L0 @ L0.T
    mod = M()
    outs = []
    for dev in (False, True):
        h = mod.mpchol_create(n, tile)
        try:
            if dev:
                At = torch.tensor(np.ascontiguousarray(A.T), device="cuda")  # At.T is column-major A
                mod.mpchol_set_matrix(h, At.T)
            else:
                mod.mpchol_set_matrix(h, A)
            mod.mpchol_precision_map(h, mod.RULE_FP64)
            assert mod.mpchol_factor(h) == 0
            outs.append(factor_dense(h, n))
        finally:
            mod.mpchol_destroy(h)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], L0)


@pytest.mark.parametrize("bad,expect", [(300, 301), (0, 1), (1023, 1024), (128, 129)])
def test_not_spd_reports_lapack_info(bad, expect):
    n, tile = 1024, 128
    A = np.eye(n)
    A[bad, bad] = -1.0
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == expect
        with pytest.raises(mod.MpcholError) as e:
            mod.mpchol_logdet(h)
        assert e.value.status == -4
    finally:
        mod.mpchol_destroy(h)


def test_nan_entry_reports_info():
    n, tile = 512, 128
    A = np.eye(n) * 2.0
    A[200, 200] = np.nan
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 201
    finally:
        mod.mpchol_destroy(h)


@pytest.mark.parametrize("cls", [3, 0])
def test_inf_entry_reports_its_column(cls):
    """An Inf below the diagonal (row 300, column 10) in a map of FP8 tiles, or
    of FP64 tiles: the panel solve writes the Inf into column 10 of the factor
    and the call returns MPCHOL_NOT_SPD with info 11 -- also where the E4M3
    code would saturate it to 448."""
    n, tile = 512, 128
    L0 = synth.int_lower(n, 5)
    A = L0 @ L0.T
    A[300, 10] = A[10, 300] = np.inf
    nt = n // tile
    um = np.asfortranarray(np.tril(np.full((nt, nt), cls, np.uint8), -1))
    log(f"inf entry, class {cls}")
    mod = M()
    h = mod.mpchol_create(n, tile, band=0)
    try:
        mod.mpchol_set_matrix(h, A)
        mod.mpchol_precision_map(h, mod.RULE_USER, 1e-9, um)
        assert mod.mpchol_factor(h) == 11
    finally:
        mod.mpchol_destroy(h)


def test_call_order_and_arguments():
    import ctypes as C

    mod = M()
    n, tile = 256, 128
    h = mod.mpchol_create(n, tile)
    lib = mod.lib()
    try:
        v = C.c_double()
        info = C.c_int64()
        assert lib.mpchol_precision_map(h, 0, 1e-9, None, None) == -4  # no matrix yet
        assert lib.mpchol_factor(h, C.byref(info)) == -4
        assert lib.mpchol_logdet(h, C.byref(v)) == -4
        sigma, x = synth.workload(16)
        assert lib.mpchol_set_generator(h, sigma.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p), -1.0, 0.0) == -1
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        assert lib.mpchol_precision_map(h, 9, 1e-9, None, None) == -1
        assert lib.mpchol_precision_map(h, mod.RULE_USER, 1e-9, None, None) == -1
        assert lib.mpchol_precision_map(h, mod.RULE_NORM, -1.0, None, None) == -1
        assert lib.mpchol_precision_map(h, mod.RULE_LEARNED, 1e-9, None, None) == -4  # no selector weights
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        assert lib.mpchol_factor(h, C.byref(info)) == -4  # tiles hold the factor: map again first
        assert lib.mpchol_solve(h, 1, None, n) == -1
        assert lib.mpchol_get_factor(h, None, n) == -1
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
    finally:
        mod.mpchol_destroy(h)


def test_fp64_full_size_16384(orc):
    """The FP64 workload at its full size (L=128, N=16384, tile 512): backward
    error from the residual kernel, logdet against the O(N) closed form, and
    sampled entries of the nugget-free factor against the closed form."""
    L, tile = 128, 512
    n = L * L
    sigma, x = synth.workload(L)
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        be = mod.mpchol_backward_error(h)
        ld = mod.mpchol_logdet(h)
        log(f"  N=16384 be={be:.3e} stats={mod.mpchol_get_stats(h)['t_factor_ms']:.1f} ms")
        assert be <= 1e-13
        ref = orc.markov_logdet(sigma, x, 5.0, 1e-8)
        assert abs(ld - ref) / abs(ref) <= 1e-12
        # nugget 0: the factor has the closed form sigma_i exp(-(x_i - x_j)/rho) s_j
        mod.mpchol_set_generator(h, sigma, x, 5.0, 0.0)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        assert mod.mpchol_factor(h) == 0
        torch = torch_cuda()
        Lg = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        mod.mpchol_get_factor(h, Lg.T, n)
        torch.cuda.synchronize()
        u = synth.uniform01(77, 4000).reshape(2000, 2)
        ii = (u[:, 0] * n).astype(np.int64)
        jj = (u[:, 1] * n).astype(np.int64)
        i, j = np.maximum(ii, jj), np.minimum(ii, jj)
        got = Lg.T[torch.tensor(i), torch.tensor(j)].cpu().numpy()
        want = np.array([orc.markov_L(sigma, x, 5.0, a, c) for a, c in zip(i, j)])
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        log(f"  closed-form sample max err {err:.2e}")
        assert err <= 1e-6
        ld0 = mod.mpchol_logdet(h)
        ref0 = orc.markov_logdet(sigma, x, 5.0, 0.0)
        assert abs(ld0 - ref0) / abs(ref0) <= 1e-11
    finally:
        mod.mpchol_destroy(h)
