"""Spherical harmonic transform on the GPU (mpchol_sht_*) against the oracle:
element by element at sizes the oracle finishes in seconds (several GEMM
row tiles, time batches spanning column tiles, ragged grids), and at the
full L = 360 and ERA5 L = 720 grids through round trips and sampled
coefficients.

Tolerance (FP64): each output sums O(L) products after two FFTs of length
O(L); with unit roundoff 1.1e-16 the error is a few 1e-14 relative to the
largest output at L <= 720.  Element-wise checks use 1e-12 of max|oracle|,
round trips 1e-11."""
import numpy as np
import pytest

import synth
from _gpu import M, log, torch_cuda

pytestmark = pytest.mark.gpu


def run_forward(mod, torch, L, nth, nph, Z, tmax=None):
    T = Z.shape[0]
    s = mod.mpchol_sht_create(L, nth, nph, tmax or max(T, 1))
    try:
        Zd = torch.tensor(Z, device="cuda")
        fd = torch.full((T, L * L), np.nan, dtype=torch.float64, device="cuda")
        mod.mpchol_sht_forward(s, Zd, fd, L)
        torch.cuda.synchronize()
        return fd.cpu().numpy()
    finally:
        mod.mpchol_sht_destroy(s)


def run_inverse(mod, torch, L, nth, nph, f):
    T = f.shape[0]
    s = mod.mpchol_sht_create(L, nth, nph, max(T, 1))
    try:
        fd = torch.tensor(f, device="cuda")
        Zd = torch.full((T, nth, nph), np.nan, dtype=torch.float64, device="cuda")
        mod.mpchol_sht_inverse(s, fd, Zd, L)
        torch.cuda.synchronize()
        return Zd.cpu().numpy()
    finally:
        mod.mpchol_sht_destroy(s)


CASES = [(1, 2, 1, 1), (2, 3, 3, 2), (5, 6, 10, 3), (12, 13, 24, 4), (12, 16, 30, 70), (17, 19, 36, 5),
         (40, 41, 81, 3), (45, 46, 90, 2), (150, 151, 300, 2)]


@pytest.mark.parametrize("L,nth,nph,T", CASES)
def test_forward_matches_oracle(sht_orc, L, nth, nph, T):
    torch = torch_cuda()
    mod = M()
    log(f"sht forward L={L} grid {nth}x{nph} T={T}")
    Z = synth.sht_fields(T, nth, nph)
    fg = run_forward(mod, torch, L, nth, nph, Z)
    D = sht_orc.wigner_table(L)
    fo = np.array([sht_orc.sht_forward_real(Z[t], L, D) for t in range(T)])
    err = np.abs(fg - fo).max()
    log(f"  max |gpu - oracle| = {err:.2e} (max |f| {np.abs(fo).max():.2e})")
    assert np.isfinite(fg).all()
    assert err <= 1e-12 * np.abs(fo).max()


@pytest.mark.parametrize("L,nth,nph,T", CASES)
def test_inverse_matches_oracle(sht_orc, L, nth, nph, T):
    torch = torch_cuda()
    mod = M()
    log(f"sht inverse L={L} grid {nth}x{nph} T={T}")
    f = synth.sht_coeffs(L, T)
    Zg = run_inverse(mod, torch, L, nth, nph, f)
    D = sht_orc.wigner_table(L)
    Zo = np.array([sht_orc.sht_inverse_real(f[t], nth, nph, D) for t in range(T)])
    err = np.abs(Zg - Zo).max()
    log(f"  max |gpu - oracle| = {err:.2e} (max |Z| {np.abs(Zo).max():.2e})")
    assert np.isfinite(Zg).all()
    assert err <= 1e-12 * np.abs(Zo).max()


@pytest.mark.parametrize("L,nth,nph,T,nsample", [(360, 361, 720, 64, 24), (720, 721, 1440, 8, 12)])
def test_full_size_round_trip_and_sampled_coefficients(sht_orc, L, nth, nph, T, nsample):
    """Inverse then forward returns the coefficients (band-limited fields);
    sampled coefficients of a white-noise field against the oracle computed
    one by one."""
    torch = torch_cuda()
    mod = M()
    log(f"sht full size L={L} grid {nth}x{nph} T={T}")
    s = mod.mpchol_sht_create(L, nth, nph, T)
    try:
        info = mod.mpchol_sht_info(s)
        log(f"  tables {info['table_bytes'] / 2**30:.2f} GiB, work {info['work_bytes'] / 2**30:.2f} GiB")
        f = torch.tensor(synth.sht_coeffs(L, T), device="cuda")
        Z = torch.empty((T, nth, nph), dtype=torch.float64, device="cuda")
        f2 = torch.empty_like(f)
        mod.mpchol_sht_inverse(s, f, Z, L)
        mod.mpchol_sht_forward(s, Z, f2, L)
        torch.cuda.synchronize()
        rt = (f2 - f).abs().max().item() / f.abs().max().item()
        log(f"  round trip max rel {rt:.2e}")
        assert rt <= 1e-11
        Zn = synth.sht_fields(1, nth, nph)
        fn = torch.empty((1, L * L), dtype=torch.float64, device="cuda")
        mod.mpchol_sht_forward(s, torch.tensor(Zn, device="cuda"), fn, L)
        torch.cuda.synchronize()
        fg = fn.cpu().numpy()[0]
    finally:
        mod.mpchol_sht_destroy(s)
    u = synth.uniform01(61, 2 * nsample).reshape(nsample, 2)
    ls = np.floor(u[:, 0] * L).astype(int)
    ls[:3] = [0, L - 1, L - 1]
    ms = np.floor(u[:, 1] * (ls + 1)).astype(int)
    ms[1] = L - 1
    lm = [(int(l), int(m)) for l, m in zip(ls, ms)]
    zo = sht_orc.sht_forward_coeffs(Zn[0], L, lm)
    got = np.array([fg[l * l + l] if m == 0 else (fg[l * l + l + m] + 1j * fg[l * l + l - m]) / np.sqrt(2)
                    for l, m in lm])
    err = np.abs(got - zo).max() / np.abs(zo).max()
    log(f"  sampled coefficients: max rel {err:.2e}")
    assert err <= 1e-12


def test_calls_reuse_buffers_with_smaller_batches(sht_orc):
    """Two calls on one object, the second with fewer fields: each result
    equals the oracle's (no stale columns leak into the smaller batch)."""
    torch = torch_cuda()
    mod = M()
    L, nth, nph = 20, 21, 40
    s = mod.mpchol_sht_create(L, nth, nph, 130)
    D = sht_orc.wigner_table(L)
    try:
        for T, seed in [(130, 71), (3, 72)]:
            Z = synth.sht_fields(T, nth, nph, seed)
            fd = torch.empty((T, L * L), dtype=torch.float64, device="cuda")
            mod.mpchol_sht_forward(s, torch.tensor(Z, device="cuda"), fd, L)
            f = synth.sht_coeffs(L, T, seed)
            Zd = torch.empty((T, nth, nph), dtype=torch.float64, device="cuda")
            mod.mpchol_sht_inverse(s, torch.tensor(f, device="cuda"), Zd, L)
            torch.cuda.synchronize()
            fo = np.array([sht_orc.sht_forward_real(Z[t], L, D) for t in range(T)])
            Zo = np.array([sht_orc.sht_inverse_real(f[t], nth, nph, D) for t in range(T)])
            assert np.abs(fd.cpu().numpy() - fo).max() <= 1e-12 * np.abs(fo).max()
            assert np.abs(Zd.cpu().numpy() - Zo).max() <= 1e-12 * np.abs(Zo).max()
    finally:
        mod.mpchol_sht_destroy(s)


def test_batch_limits_and_empty_batch():
    import ctypes as C

    torch = torch_cuda()
    mod = M()
    s = mod.mpchol_sht_create(8, 9, 15, 4)
    try:
        Z = torch.zeros((5, 9, 15), dtype=torch.float64, device="cuda")
        f = torch.zeros((5, 64), dtype=torch.float64, device="cuda")
        L_ = mod.lib()
        assert L_.mpchol_sht_forward(s, C.c_void_p(Z.data_ptr()), 5, C.c_void_p(f.data_ptr())) == mod.EINVAL
        assert L_.mpchol_sht_inverse(s, C.c_void_p(f.data_ptr()), -1, C.c_void_p(Z.data_ptr())) == mod.EINVAL
        assert L_.mpchol_sht_forward(s, None, 0, None) == 0
        assert L_.mpchol_sht_forward(s, None, 2, C.c_void_p(f.data_ptr())) == mod.EINVAL
    finally:
        mod.mpchol_sht_destroy(s)


def test_large_object_still_runs_after_a_smaller_one_is_created():
    """Kernel launch limits set for a small object must not break an object
    created earlier with longer transforms (69 KB of LDS per workgroup at
    N_phi = 720)."""
    torch = torch_cuda()
    mod = M()
    L, nth, nph, T = 360, 361, 720, 4
    big = mod.mpchol_sht_create(L, nth, nph, T)
    small = mod.mpchol_sht_create(8, 9, 15, 2)
    try:
        f = torch.tensor(synth.sht_coeffs(L, T), device="cuda")
        Z = torch.empty((T, nth, nph), dtype=torch.float64, device="cuda")
        f2 = torch.empty_like(f)
        mod.mpchol_sht_inverse(big, f, Z, L)
        mod.mpchol_sht_forward(big, Z, f2, L)
        fs = torch.tensor(synth.sht_coeffs(8, 2), device="cuda")
        Zs = torch.empty((2, 9, 15), dtype=torch.float64, device="cuda")
        mod.mpchol_sht_inverse(small, fs, Zs, 8)
        torch.cuda.synchronize()
        rt = ((f2 - f).abs().max() / f.abs().max()).item()
        log(f"  round trip after a second object: {rt:.2e}")
        assert rt <= 1e-11
    finally:
        mod.mpchol_sht_destroy(small)
        mod.mpchol_sht_destroy(big)
