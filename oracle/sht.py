"""CPU oracle of the spherical harmonic transform -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy implementation of the forward SHT (Sec. III.A.1, "Modeling
in the Spherical Harmonic Domain": FFT along longitude, extension of G_m to
colatitudes in (pi, 2 pi), inverse FFT along the extended colatitude for
K_{m,m'}, then the two sums of the coefficient equation with S_{l,m,m''} and
I(q)) and of the inverse SHT used to generate emulations (Sec. III.B).  The
steps are taken in the paper's order with the full index ranges
-(L-1) <= m, m', m'' <= L-1 and no symmetry shortcuts; numpy's FFT and matmul
are the only library steps.  Only tests/, the package smoke check and the
benchmark's CPU leg may import this module.

Conventions (readings, stated once):
* grid: colatitudes theta_j = j pi / (N_theta - 1), j = 0..N_theta-1 (both
  poles), longitudes phi_k = 2 pi k / N_phi; a field is an N_theta x N_phi
  array, longitude fastest.
* Y_lm(theta, phi) carries the Condon-Shortley phase; Y_lm(theta, 0) =
  sqrt((2l+1)/(4 pi)) d^l_{m,0}(theta) with d^l_{m',m}(beta) =
  <l m'| exp(-i beta J_y) |l m>.
* inverse over longitude: Z(theta, phi) = (1 / 2 pi) sum_m G_m(theta) e^{i m phi}
  (the inverse of G_m = int Z e^{-i m phi} dphi).
* poles: the extension G_m(2 pi - theta) = (-1)^m G_m(theta), continued to
  theta = 0 and pi, forces G_m = 0 there for odd m; the pole samples of odd
  orders are taken as zero before the colatitude FFT.  A field that is
  single-valued at the poles (constant along the first and last grid rows),
  in particular any band-limited field, is unaffected.
* real coefficient vector f of length L^2 (the paper's f_t): index l^2 + l holds
  z_{l,0}; for m > 0, index l^2 + l + m holds sqrt(2) Re z_{l,m} and index
  l^2 + l - m holds sqrt(2) Im z_{l,m}.  For a real field z_{l,-m} =
  (-1)^m conj(z_{l,m}), so f determines z and |f|^2 = sum over all (l, m) of
  |z_{l,m}|^2.

Pins (tests/test_oracle_sht.py): Wigner-d at pi/2 against Wigner's explicit
sum in exact rational arithmetic and against orthogonality at large degree;
the Fourier expansion of d^l_{m,0} against scipy's spherical harmonics; I(q)
against numerical quadrature; forward and inverse transforms against fields
synthesized with scipy's spherical harmonics; closed forms (constant, cos
theta, sin theta cos phi).
"""
from __future__ import annotations

import numpy as np


def wigner_d_pi2(l: int) -> np.ndarray:
    """Delta^l[k + l, m + l] = d^l_{k,m}(pi/2) for -l <= k, m <= l.

    Edge value (Wigner's formula with k = l, at beta = pi/2):
        d^l_{l,m} = (-1)^(l-m) 2^-l sqrt(C(2l, l+m)).
    Three-term recursion in the first index, from J_z acting on both sides of
    the rotation (at beta = pi/2 the rotated J_z is a multiple of J_x, whose
    matrix elements couple k to k +- 1):
        sqrt((l+k)(l-k+1)) d_{k-1,m} = 2 m d_{k,m} - sqrt((l-k)(l+k+1)) d_{k+1,m},
    run downward from k = l to k = 0 (the direction in which the wanted
    solution grows out of the edge region), and the reflection
        d^l_{-k,m}(pi/2) = (-1)^(l+m) d^l_{k,m}(pi/2)
    for k < 0 (the recursion continued past the middle would run into the
    decaying region and lose all accuracy).
    """
    ms = np.arange(-l, l + 1)
    D = np.zeros((2 * l + 1, 2 * l + 1))
    # edge row k = l: 2^-l sqrt(C(2l, l+m)) built from m = l downward by the
    # ratio C(2l, l+m) / C(2l, l+m+1) = (l+m+1) / (l-m)
    edge = np.zeros(2 * l + 1)
    edge[2 * l] = 2.0 ** (-l)
    for m in range(l - 1, -l - 1, -1):
        edge[m + l] = edge[m + 1 + l] * np.sqrt((l + m + 1) / (l - m))
    D[2 * l] = edge * np.where((l - ms) % 2 == 0, 1.0, -1.0)
    prev = np.zeros(2 * l + 1)  # d_{k+1, m}
    for k in range(l, 0, -1):
        cur = D[k + l]
        nxt = (2.0 * ms * cur - np.sqrt((l - k) * (l + k + 1.0)) * prev) / np.sqrt((l + k) * (l - k + 1.0))
        D[k - 1 + l] = nxt
        prev = cur
    sgn = np.where((l + ms) % 2 == 0, 1.0, -1.0)
    for k in range(1, l + 1):
        D[-k + l] = sgn * D[k + l]
    return D


def wigner_table(L: int) -> list:
    """[Delta^0, ..., Delta^{L-1}]."""
    return [wigner_d_pi2(l) for l in range(L)]


def I_q(q):
    """I(q) = int_0^pi e^{i q theta} sin theta dtheta (closed form of the paper):
    i q pi / 2 for q = +-1, 0 for other odd q, 2 / (1 - q^2) for even q."""
    q = np.asarray(q)
    out = np.zeros(q.shape, dtype=complex)
    even = q % 2 == 0
    out[even] = 2.0 / (1.0 - q[even].astype(float) ** 2)
    one = np.abs(q) == 1
    out[one] = 1j * q[one] * np.pi / 2.0
    return out


def S_tensor_m(L: int, m: int, D: list) -> np.ndarray:
    """S[l, m'' + L - 1] = i^-m sqrt((2l+1)/(4 pi)) d^l_{m'',0}(pi/2) d^l_{m'',m}(pi/2)
    for |m| <= l < L, |m''| <= l (zero elsewhere)."""
    S = np.zeros((L, 2 * L - 1), dtype=complex)
    ph = (1j) ** (-m)
    for l in range(abs(m), L):
        Dl = D[l]
        k = np.arange(-l, l + 1)
        S[l, k + L - 1] = ph * np.sqrt((2 * l + 1) / (4 * np.pi)) * Dl[k + l, l] * Dl[k + l, m + l]
    return S


def grid(ntheta: int, nphi: int):
    return np.arange(ntheta) * np.pi / (ntheta - 1), 2.0 * np.pi * np.arange(nphi) / nphi


def check_grid(L: int, ntheta: int, nphi: int):
    if ntheta <= L or nphi < 2 * L - 1:
        raise ValueError("the transform needs N_theta > L and N_phi >= 2L - 1")


def G_from_field(Z: np.ndarray, L: int) -> np.ndarray:
    """G[j, m + L - 1] = int Z(theta_j, phi) e^{-i m phi} dphi, exact on the
    equispaced longitudes for a field band-limited at L (N_phi >= 2L - 1)."""
    nphi = Z.shape[1]
    X = np.fft.fft(Z, axis=1) * (2.0 * np.pi / nphi)
    ms = np.arange(-(L - 1), L)
    return X[:, ms % nphi]


def K_from_G(G: np.ndarray, L: int, orders=None) -> np.ndarray:
    """K[i, m' + L - 1] for the order m = orders[i] (default all orders
    -(L-1)..L-1, one per column of G) with G_m(theta) = sum_m' K_{m,m'}
    e^{i m' theta}: G_m extended to 2 N_theta - 2 equispaced colatitudes by
    G_m(2 pi - theta) = (-1)^m G_m(theta), then an inverse DFT."""
    ntheta = G.shape[0]
    M = 2 * ntheta - 2
    ms = np.arange(-(L - 1), L)
    orders = ms if orders is None else np.asarray(orders)
    ext = np.zeros((M, G.shape[1]), dtype=complex)
    ext[:ntheta] = G
    par = np.where(orders % 2 == 0, 1.0, -1.0)
    # the extension's symmetry forces G_m = 0 at both poles for odd m (a
    # field on the sphere, single-valued at a pole, has it); pole samples of
    # odd orders are taken as zero
    ext[0, par < 0] = 0.0
    ext[ntheta - 1, par < 0] = 0.0
    for j in range(ntheta, M):
        ext[j] = par * G[M - j]
    F = np.fft.fft(ext, axis=0) / M  # coefficient of e^{+i m' theta_j}
    return F[ms % M, :].T


def sht_forward(Z: np.ndarray, L: int, D: list | None = None) -> np.ndarray:
    """Complex coefficients zc[l, m + L - 1] (zero for |m| > l) of a field on
    the grid, by the paper's steps: G_m by FFT along phi, K_{m,m'} by the
    extended inverse FFT along theta, J_{m,m''} = sum_m' K_{m,m'} I(m' + m''),
    z_{l,m} = sum_m'' S_{l,m,m''} J_{m,m''}."""
    ntheta, nphi = Z.shape
    check_grid(L, ntheta, nphi)
    D = wigner_table(L) if D is None else D
    G = G_from_field(np.asarray(Z, dtype=float), L)
    K = K_from_G(G, L)
    ms = np.arange(-(L - 1), L)
    H = I_q(ms[:, None] + ms[None, :])  # H[m', m''] = I(m' + m'')
    J = K @ H
    zc = np.zeros((L, 2 * L - 1), dtype=complex)
    for m in ms:
        S = S_tensor_m(L, m, D)
        zc[:, m + L - 1] = S @ J[m + L - 1]
    return zc


def sht_inverse(zc: np.ndarray, ntheta: int, nphi: int, D: list | None = None) -> np.ndarray:
    """Field on the grid from complex coefficients, by the same relations read
    backwards: K_{m,m'} = 2 pi sum_l S_{l,m,m'} z_{l,m}, G_m(theta_j) =
    sum_m' K_{m,m'} e^{i m' theta_j}, Z = (1/2pi) sum_m G_m e^{i m phi} (real
    part; the imaginary part vanishes for coefficients of a real field)."""
    L = zc.shape[0]
    check_grid(L, ntheta, nphi)
    D = wigner_table(L) if D is None else D
    th, ph = grid(ntheta, nphi)
    ms = np.arange(-(L - 1), L)
    K = np.zeros((2 * L - 1, 2 * L - 1), dtype=complex)
    for m in ms:
        S = S_tensor_m(L, m, D)
        K[m + L - 1] = 2.0 * np.pi * (S.T @ zc[:, m + L - 1])
    G = K @ np.exp(1j * np.outer(ms, th))  # G[m, j]
    Z = (G.T @ np.exp(1j * np.outer(ms, ph))) / (2.0 * np.pi)
    return Z.real


def complex_to_real(zc: np.ndarray) -> np.ndarray:
    """f (length L^2) from z_{l,m}, m >= 0 (see the module's layout)."""
    L = zc.shape[0]
    f = np.zeros(L * L)
    for l in range(L):
        f[l * l + l] = zc[l, L - 1].real
        for m in range(1, l + 1):
            z = zc[l, m + L - 1]
            f[l * l + l + m] = np.sqrt(2.0) * z.real
            f[l * l + l - m] = np.sqrt(2.0) * z.imag
    return f


def real_to_complex(f: np.ndarray) -> np.ndarray:
    """z_{l,m} for all -l <= m <= l from f, using z_{l,-m} = (-1)^m conj(z_{l,m})."""
    L = int(round(np.sqrt(f.size)))
    assert L * L == f.size
    zc = np.zeros((L, 2 * L - 1), dtype=complex)
    for l in range(L):
        zc[l, L - 1] = f[l * l + l]
        for m in range(1, l + 1):
            z = (f[l * l + l + m] + 1j * f[l * l + l - m]) / np.sqrt(2.0)
            zc[l, m + L - 1] = z
            zc[l, -m + L - 1] = (-1) ** m * np.conj(z)
    return zc


def sht_forward_real(Z: np.ndarray, L: int, D: list | None = None) -> np.ndarray:
    return complex_to_real(sht_forward(Z, L, D))


def sht_inverse_real(f: np.ndarray, ntheta: int, nphi: int, D: list | None = None) -> np.ndarray:
    return sht_inverse(real_to_complex(f), ntheta, nphi, D)


def sht_forward_coeffs(Z: np.ndarray, L: int, lm: list) -> np.ndarray:
    """Selected coefficients z_{l,m} of one field (same steps, restricted to the
    orders asked for; Wigner-d only at the degrees asked for), for sampled
    checks at sizes where the whole transform is too slow."""
    ntheta, nphi = Z.shape
    check_grid(L, ntheta, nphi)
    G = G_from_field(np.asarray(Z, dtype=float), L)
    ms = np.arange(-(L - 1), L)
    H = I_q(ms[:, None] + ms[None, :])
    out = np.zeros(len(lm), dtype=complex)
    cacheK = {}
    for i, (l, m) in enumerate(lm):
        if m not in cacheK:
            Km = K_from_G(G[:, [m + L - 1]], L, [m])
            cacheK[m] = Km[0] @ H
        Dl = wigner_d_pi2(l)
        k = np.arange(-l, l + 1)
        s = (1j) ** (-m) * np.sqrt((2 * l + 1) / (4 * np.pi)) * Dl[k + l, l] * Dl[k + l, m + l]
        out[i] = s @ cacheK[m][k + L - 1]
    return out
