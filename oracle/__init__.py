"""CPU oracle for the mixed-precision tile Cholesky -- TEST INFRASTRUCTURE ONLY.

Plain, slow reference implementations (FP64 unless stated) of what the HIP
path computes, written from the paper (Sec. III.A.3: the covariance and its
Cholesky factor; Sec. III.B: draws xi = V z; Sec. III.D and Sec. V.A: tile
mixed precision with sender-side conversion) and from textbook definitions.
Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The arithmetic lives in ``oracle.c`` (built to ``liboracle.so`` with gcc); this
module only marshals numpy arrays.  Parity status per function group is given
in ``oracle.c``; the one group without an independent pin is the exact bit
pattern of the mixed-precision factor under a different summation order
("parity unpinned": judged through backward error, logdet and the map).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, BF16, F16, E4M3 = 0, 1, 2, 3, 4
P64, P32, P16, P8 = 0, 1, 2, 3

NPARAM = 8 * 64 + 64 + 64 * 64 + 64 + 4 * 64 + 4


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        d, i64, i32, u32p = C.c_double, C.c_int64, C.c_int, C.POINTER(C.c_uint32)
        dp = C.POINTER(C.c_double)
        L.orc_cov_entry.restype = d
        L.orc_cov_entry.argtypes = [dp, dp, d, d, i64, i64]
        L.orc_cov_dense.argtypes = [i64, dp, dp, d, d, dp, i64]
        L.orc_cov_samples.argtypes = [i64, i64, dp, i64, d, d, dp, i64]
        L.orc_threads.restype = i32
        L.orc_potrf.restype = i64
        L.orc_potrf.argtypes = [i64, dp, i64]
        L.orc_logdet.restype = d
        L.orc_logdet.argtypes = [i64, dp, i64]
        L.orc_potrs.argtypes = [i64, dp, i64, i64, dp, i64]
        L.orc_residual_fro.restype = d
        L.orc_residual_fro.argtypes = [i64, dp, i64, dp, i64, dp]
        L.orc_tile_residual2.argtypes = [i64, i64, dp, i64, dp, i64, dp]
        L.orc_lower_matmul.argtypes = [i64, dp, i64, i64, dp, i64, dp, i64]
        L.orc_markov_L.restype = d
        L.orc_markov_L.argtypes = [dp, dp, d, i64, i64]
        L.orc_markov_logdet.restype = d
        L.orc_markov_logdet.argtypes = [i64, dp, dp, d, d]
        L.orc_markov_solve.argtypes = [i64, dp, dp, d, d, i64, dp, i64]
        L.orc_round.restype = d
        L.orc_round.argtypes = [d, i32]
        L.orc_e4m3_decode.restype = d
        L.orc_e4m3_decode.argtypes = [C.c_uint8]
        L.orc_unit_roundoff.restype = d
        L.orc_unit_roundoff.argtypes = [i32]
        L.orc_scale_exp.restype = i32
        L.orc_scale_exp.argtypes = [d, i32]
        L.orc_tile_norms.restype = d
        L.orc_tile_norms.argtypes = [i64, i64, dp, i64, dp, dp]
        L.orc_map_norm.argtypes = [i64, dp, d, d, i32, C.c_uint, i32, C.POINTER(C.c_uint8)]
        L.orc_map_band.argtypes = [i64, i32, i32, C.c_uint, C.POINTER(C.c_uint8)]
        L.orc_mp_factor.restype = i64
        L.orc_mp_factor.argtypes = [i64, i64, dp, i64, C.POINTER(C.c_uint8), i32, dp, i64, C.POINTER(C.c_int32), i32, i32,
                                    i32, i32, i32]
        L.orc_mx_block_exp.restype = i32
        L.orc_mx_block_exp.argtypes = [d]
        L.orc_mx_quantize.argtypes = [i64, i64, dp, i64, dp, i64, C.POINTER(C.c_int32)]
        L.orc_ozaki_gemm.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        L.orc_ozaki_row_exp.restype = i32
        L.orc_ozaki_row_exp.argtypes = [dp, i64, i64]
        L.orc_split3.restype = C.c_float
        L.orc_split3.argtypes = [d, i32]
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_normal_draws.argtypes = [C.c_uint64, i64, dp, u32p]
        L.orc_mlp_nparam.restype = i64
        L.orc_mlp_forward.argtypes = [dp, i64, dp, dp]
        L.orc_mlp_loss_grad.restype = d
        L.orc_mlp_loss_grad.argtypes = [dp, i64, dp, C.POINTER(C.c_int32), dp, d, dp]
        L.orc_adam_step.argtypes = [i64, dp, dp, dp, dp, i64, d, d, d, d]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _fortran(a):
    return np.asfortranarray(a, dtype=np.float64)


# ---------------------------------------------------------------- workload
def cov_dense(sigma, x, rho, nugget):
    """Sigma_ij = sigma_i sigma_j exp(-|x_i - x_j| / rho) + nugget delta_ij."""
    sigma, x = _f64(sigma), _f64(x)
    n = sigma.size
    A = np.empty((n, n), order="F")
    lib().orc_cov_dense(n, _dp(sigma), _dp(x), rho, nugget, _dp(A), n)
    return A


def cov_samples(xi, scale, nugget):
    """S = scale * xi xi^T + nugget I for samples xi (n x m): the covariance
    estimator of the residual vectors (Sec. III.A.3, constructing the covariance
    matrix)."""
    xi = _fortran(xi)
    n, m = xi.shape
    S = np.empty((n, n), order="F")
    lib().orc_cov_samples(n, m, _dp(xi), n, float(scale), float(nugget), _dp(S), n)
    return S


def cov_entry(sigma, x, rho, nugget, i, j):
    sigma, x = _f64(sigma), _f64(x)
    return lib().orc_cov_entry(_dp(sigma), _dp(x), rho, nugget, int(i), int(j))


# ---------------------------------------------------------------- O1 exact
def potrf(A):
    """(L, info): FP64 lower Cholesky factor by the right-looking definition."""
    L = _fortran(A).copy(order="F")
    n = L.shape[0]
    info = lib().orc_potrf(n, _dp(L), n)
    return L, int(info)


def threads():
    """OpenMP threads the oracle runs with."""
    return int(lib().orc_threads())


def logdet(L):
    L = _fortran(L)
    return lib().orc_logdet(L.shape[0], _dp(L), L.shape[0])


def potrs(L, B):
    L = _fortran(L)
    X = _fortran(B).copy(order="F")
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    n = L.shape[0]
    lib().orc_potrs(n, _dp(L), n, X.shape[1], _dp(X), n)
    return X


def backward_error(A, L):
    """||A - L L^T||_F / ||A||_F."""
    A, L = _fortran(A), _fortran(L)
    n = A.shape[0]
    an = C.c_double(0.0)
    r = lib().orc_residual_fro(n, _dp(A), n, _dp(L), n, C.byref(an))
    return r / an.value


def tile_residual2(A, L, b):
    """Squared Frobenius norms of the residual per tile, nt x nt (lower part)."""
    A, L = _fortran(A), _fortran(L)
    n = A.shape[0]
    nt = (n + b - 1) // b
    out = np.zeros((nt, nt), order="F")
    lib().orc_tile_residual2(n, b, _dp(A), n, _dp(L), n, _dp(out))
    return out


def lower_matmul(L, Z):
    L, Z = _fortran(L), _fortran(Z)
    n, m = Z.shape
    Y = np.empty((n, m), order="F")
    lib().orc_lower_matmul(n, _dp(L), n, m, _dp(Z), n, _dp(Y), n)
    return Y


# ---------------------------------------------------------------- closed forms
def markov_L(sigma, x, rho, i, j):
    sigma, x = _f64(sigma), _f64(x)
    return lib().orc_markov_L(_dp(sigma), _dp(x), rho, int(i), int(j))


def markov_factor(sigma, x, rho):
    sigma, x = _f64(sigma), _f64(x)
    n = sigma.size
    return np.array([[markov_L(sigma, x, rho, i, j) for j in range(n)] for i in range(n)], order="F")


def markov_logdet(sigma, x, rho, nugget):
    sigma, x = _f64(sigma), _f64(x)
    return lib().orc_markov_logdet(sigma.size, _dp(sigma), _dp(x), rho, nugget)


def markov_solve(sigma, x, rho, nugget, B):
    sigma, x = _f64(sigma), _f64(x)
    X = _fortran(B).copy(order="F")
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    lib().orc_markov_solve(sigma.size, _dp(sigma), _dp(x), rho, nugget, X.shape[1], _dp(X), X.shape[0])
    return X


# ---------------------------------------------------------------- formats
def round_to(v, fmt):
    f = lib().orc_round
    return np.array([f(float(t), fmt) for t in np.asarray(v, dtype=np.float64).ravel()]).reshape(np.shape(v))


def e4m3_decode(code):
    return lib().orc_e4m3_decode(int(code))


def unit_roundoff(fmt):
    return lib().orc_unit_roundoff(fmt)


def scale_exp(amax, fmt):
    return int(lib().orc_scale_exp(float(amax), fmt))


# ---------------------------------------------------------------- maps, O2
def tile_norms(A, b):
    """(fro2, amax, total_fro) over the valid part of the lower tiles."""
    A = _fortran(A)
    n = A.shape[0]
    nt = (n + b - 1) // b
    fro2 = np.zeros((nt, nt), order="F")
    amax = np.zeros((nt, nt), order="F")
    tot = lib().orc_tile_norms(n, b, _dp(A), n, _dp(fro2), _dp(amax))
    return fro2, amax, tot


def map_norm(fro2, total, eps, band=1, allowed=0xF, lo16=F16):
    nt = fro2.shape[0]
    fro2 = _fortran(fro2)
    out = np.zeros((nt, nt), dtype=np.uint8, order="F")
    lib().orc_map_norm(nt, _dp(fro2), total, eps, band, allowed, lo16, out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out


def map_band(nt, band=1, variant=3, allowed=0xF):
    """Band rule map (Sec. IV.B variants: 1 DP/SP, 2 DP/SP/HP, 3 DP/HP), nt x nt uint8."""
    out = np.zeros((nt, nt), dtype=np.uint8, order="F")
    lib().orc_map_band(int(nt), int(band), int(variant), int(allowed), out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out


def mp_factor(A, b, cmap, lo16=F16, order=0, lo32=0, lo64=0, band=1, lo8=0):
    """O2: (Lhat, info, tscale) -- the tile algorithm replayed with explicit rounding.

    cmap is an nt x nt class map (lower part used; 0 FP64, 1 FP32, 2 16-bit, 3 FP8);
    order 0/1 sums the update products in increasing/decreasing order;
    lo32 = 1 forms FP32-class products from three-way BF16 splits;
    lo64 = 1 forms the FP64-class products of tiles farther than `band` from
    the diagonal as exact integer products of row-scaled panels (ozaki_gemm);
    lo8 = 1 block-scales the FP8 copies of the panel tiles (mx_quantize).
    """
    A = _fortran(A)
    n = A.shape[0]
    nt = (n + b - 1) // b
    cmap = np.asfortranarray(cmap, dtype=np.uint8)
    assert cmap.shape == (nt, nt)
    Lh = np.zeros((n, n), order="F")
    ts = np.zeros((nt, nt), dtype=np.int32, order="F")
    info = lib().orc_mp_factor(n, b, _dp(A), n, cmap.ctypes.data_as(C.POINTER(C.c_uint8)), lo16, _dp(Lh), n,
                               ts.ctypes.data_as(C.POINTER(C.c_int32)), int(order), int(lo32), int(lo64), int(band),
                               int(lo8))
    return Lh, int(info), ts


def mx_block_exp(amax):
    """Exponent t of a block-scaled FP8 block with largest |value| amax: the
    largest t with amax 2^t <= 448, clamped to [-127, 127] (0 for amax = 0)."""
    return int(lib().orc_mx_block_exp(float(amax)))


def mx_quantize(X):
    """(values, texp): the block-scaled FP8 copy of X (rows x cols) -- per
    row, every 32 consecutive elements (fewer in a row's last block) share a
    power-of-two scale; texp[r, c // 32] are the block exponents."""
    X = _fortran(X)
    rows, cols = X.shape
    out = np.zeros((rows, cols), order="F")
    texp = np.zeros((rows, (cols + 31) // 32), dtype=np.int32, order="F")
    lib().orc_mx_quantize(rows, cols, _dp(X), rows, _dp(out), rows, texp.ctypes.data_as(C.POINTER(C.c_int32)))
    return out, texp


def ozaki_gemm(A, B):
    """D = A B^T with FP64-class products emulated by exact integer products:
    each row scaled by 2^e (row max in [2^52, 2^53)), rounded to integers,
    the integer products summed exactly, the sum rounded once to FP64 and
    scaled back."""
    A, B = _fortran(A), _fortran(B)
    m, k = A.shape
    n = B.shape[0]
    assert B.shape[1] == k
    D = np.empty((m, n), order="F")
    lib().orc_ozaki_gemm(m, n, k, _dp(A), m, _dp(B), n, _dp(D), m)
    return D


def ozaki_row_exp(row):
    """Scale exponent e of a row: max |row| 2^e in [2^52, 2^53) (0 for a zero row)."""
    r = _f64(row)
    return int(lib().orc_ozaki_row_exp(_dp(r), 1, r.size))


def split3(v):
    """(hi, mid, lo): the three-way BF16 split of float(v)."""
    return tuple(float(lib().orc_split3(float(v), p)) for p in range(3))


# ---------------------------------------------------------------- Philox, draws
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normal_draws(seed, count):
    """(z FP64, raw uint32) of the Philox/Box-Muller draw sequence."""
    z = np.empty(count)
    raw = np.empty(count, dtype=np.uint32)
    lib().orc_normal_draws(C.c_uint64(seed), count, _dp(z), raw.ctypes.data_as(C.POINTER(C.c_uint32)))
    return z, raw


# ---------------------------------------------------------------- selector MLP
def mlp_forward(params, X):
    P, X = _f64(params), _f64(X)
    out = np.empty((X.shape[0], 4))
    lib().orc_mlp_forward(_dp(P), X.shape[0], _dp(X), _dp(out))
    return out


def mlp_loss_grad(params, X, y, class_w, alpha):
    P, X, cw = _f64(params), _f64(X), _f64(class_w)
    y = np.ascontiguousarray(y, dtype=np.int32)
    g = np.zeros(NPARAM)
    loss = lib().orc_mlp_loss_grad(_dp(P), X.shape[0], _dp(X), y.ctypes.data_as(C.POINTER(C.c_int32)), _dp(cw),
                                   alpha, _dp(g))
    return loss, g


def adam_step(params, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on params, m, v (FP64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_adam_step(params.size, _dp(params), _dp(g), _dp(m), _dp(v), step, lr, b1, b2, eps)
