"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This module only draws numbers and lays out the workload's coordinates; it
holds none of the factorization's arithmetic (no covariance entries, no
Cholesky, no rounding), so both sides can take their inputs from it without
sharing any of the method.

Workload (a stand-in for the empirical covariance of spherical-harmonic
coefficients, Sec. III.A.3 of the paper; ERA5 and trained emulator
parameters are not available):

* index i runs over (l, m), l = 0..L-1, m = -l..l, in the order i = l^2 + l + m
  (the coefficient vector of Sec. III.A.3, truncated at degree L-1 as in
  Sec. III.A.1);
* coordinate x_i = l + (m + l) / (2l + 1), strictly increasing in i;
* scale sigma_i = (1 + l)^-1 * exp(0.1 * g_i), g_i ~ N(0, 1) (a lognormal(0, 0.1)
  factor), drawn with seed 0;
* right-hand sides B ~ N(0, 1) with seed 1; caller-side draws z ~ N(0, 1) with seed 2.

SHT inputs (Sec. III.A.1 and III.B; the ERA5 fields are not available): real
coefficient vectors f_t of length L^2 in the same index order, N(0,1) scaled
by (1+l)^-1 (seed 5), and white-noise grid fields N(0,1) of N_theta x N_phi
points (seed 6) standing in for the stochastic component, which is not
band-limited.

Random numbers: splitmix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) -> 53-bit uniforms ->
Box-Muller (Box & Muller 1958) in FP64.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED_SIGMA = 0
SEED_RHS = 1
SEED_DRAWS = 2
SEED_MLP_INIT = 3
SEED_SAMPLES = 4
SEED_SHT_COEFFS = 5
SEED_SHT_FIELD = 6


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of splitmix64 started from state `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """Uniforms in (0, 1]: (top 53 bits + 1) * 2^-53."""
    z = splitmix64(seed, count)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """`count` standard normals by Box-Muller on consecutive uniform pairs."""
    npair = (count + 1) // 2
    u = uniform01(seed, 2 * npair)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npair)
    out[0::2] = r * np.cos(2.0 * np.pi * u2)
    out[1::2] = r * np.sin(2.0 * np.pi * u2)
    return out[:count]


def sh_degrees(L: int) -> np.ndarray:
    """Degree l of every coefficient index i = l^2 + l + m (length L^2)."""
    return np.repeat(np.arange(L, dtype=np.int64), 2 * np.arange(L) + 1)


def sh_orders(L: int) -> np.ndarray:
    """Order m of every coefficient index (length L^2)."""
    return np.concatenate([np.arange(-l, l + 1, dtype=np.int64) for l in range(L)])


def sh_coords(L: int) -> np.ndarray:
    """x_i = l + (m + l) / (2l + 1)."""
    l = sh_degrees(L).astype(np.float64)
    m = sh_orders(L).astype(np.float64)
    return l + (m + l) / (2.0 * l + 1.0)


def sh_sigma(L: int, seed: int = SEED_SIGMA) -> np.ndarray:
    """sigma_i = (1 + l)^-1 * lognormal(0, 0.1), one factor per index."""
    l = sh_degrees(L).astype(np.float64)
    return np.exp(0.1 * normal(seed, L * L)) / (1.0 + l)


def workload(L: int, seed: int = SEED_SIGMA):
    """(sigma, x) of the band-limit-L workload, N = L^2 entries each."""
    return sh_sigma(L, seed), sh_coords(L)


def rhs(n: int, nrhs: int, seed: int = SEED_RHS) -> np.ndarray:
    """N(0,1) right-hand sides, column-major (Fortran order) n x nrhs."""
    return np.asfortranarray(normal(seed, n * nrhs).reshape(nrhs, n).T)


def draws(n: int, ndraws: int, seed: int = SEED_DRAWS) -> np.ndarray:
    """Caller-side N(0,1) draws in float32, column-major n x ndraws."""
    return np.asfortranarray(normal(seed, n * ndraws).astype(np.float32).reshape(ndraws, n).T)


def int_lower(n: int, seed: int, lo: int = -3, hi: int = 3, diag_lo: int = 1, diag_hi: int = 4,
              graded: bool = False) -> np.ndarray:
    """Random lower-triangular integer matrix with a positive diagonal.

    Small integer entries keep L0 @ L0.T exactly representable in FP64, so a
    matrix built from it has a known exact Cholesky factor.  graded: entry
    (i, j) below the diagonal is multiplied by 2^((i + j // 32) mod 4), so that
    neighbouring rows and neighbouring 32-column blocks of a row differ in
    magnitude (entries stay integers of at most two significant bits).
    """
    u = uniform01(seed, n * n).reshape(n, n)
    off = np.floor(lo + u * (hi - lo + 1)).astype(np.int64)
    off = np.clip(off, lo, hi)
    if graded:
        i, j = np.indices((n, n))
        off = off << ((i + j // 32) % 4)
    d = np.floor(diag_lo + uniform01(seed + 7919, n) * (diag_hi - diag_lo + 1)).astype(np.int64)
    d = np.clip(d, diag_lo, diag_hi)
    L0 = np.tril(off, -1).astype(np.float64)
    L0[np.arange(n), np.arange(n)] = d
    return L0


def hadamard(m: int) -> np.ndarray:
    """Sylvester-Hadamard matrix of order m (a power of two): entries +-1,
    H H^T = m I."""
    assert m >= 1 and (m & (m - 1)) == 0
    H = np.ones((1, 1))
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


def samples(n: int, m: int, seed: int = SEED_SAMPLES) -> np.ndarray:
    """Residual-like samples for the covariance producer: column-major n x m,
    N(0,1) entries scaled by the SH spectrum (1+l)^-1 of coefficient i."""
    l = sh_degrees(int(np.ceil(np.sqrt(n))))[:n]
    z = normal(seed, n * m).reshape(m, n).T
    return np.asfortranarray(z / (1.0 + l)[:, None])


def features_toy(count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """A separable toy classification set for selector training checks:
    8 features ~ U(-1, 1); class = index of the largest of the first 4."""
    u = uniform01(seed, count * 8).reshape(count, 8) * 2.0 - 1.0
    return u.astype(np.float32), np.argmax(u[:, :4], axis=1).astype(np.int32)


def sht_coeffs(L: int, T: int, seed: int = SEED_SHT_COEFFS) -> np.ndarray:
    """T real coefficient vectors (row t = f_t, length L^2), N(0,1) / (1 + l)."""
    l = sh_degrees(L).astype(np.float64)
    return normal(seed, T * L * L).reshape(T, L * L) / (1.0 + l)[None, :]


def sht_fields(T: int, ntheta: int, nphi: int, seed: int = SEED_SHT_FIELD) -> np.ndarray:
    """T white-noise fields N(0,1) on an N_theta x N_phi grid (longitude fastest)."""
    return normal(seed, T * ntheta * nphi).reshape(T, ntheta, nphi)
