"""Pins of the SHT oracle against what the mathematics fixes: Wigner's
explicit sum (exact rational arithmetic), orthogonality of d^l(pi/2), scipy's
spherical harmonics (an independent implementation), quadrature of I(q), and
closed-form fields."""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import sht


def wigner_exact(l, k, m):
    """d^l_{k,m}(pi/2) from Wigner's explicit sum, the rational part exact."""
    tot = Fraction(0)
    for s in range(0, 2 * l + 1):
        a, b, c = l + m - s, l - k - s, k - m + s
        if a < 0 or b < 0 or c < 0:
            continue
        tot += Fraction((-1) ** c, factorial(a) * factorial(s) * factorial(b) * factorial(c))
    F = factorial(l + k) * factorial(l - k) * factorial(l + m) * factorial(l - m)
    # sign(tot) * sqrt(tot^2 F) / 2^l, the square root of an exact rational
    v = np.sqrt(float(tot * tot * F))
    return (v if tot >= 0 else -v) / 2.0 ** l


@pytest.mark.parametrize("l", [0, 1, 2, 3, 6, 11, 16])
def test_wigner_pi2_against_explicit_sum(l):
    D = sht.wigner_d_pi2(l)
    E = np.array([[wigner_exact(l, k, m) for m in range(-l, l + 1)] for k in range(-l, l + 1)])
    assert np.abs(D - E).max() <= 1e-15


@pytest.mark.parametrize("l", [40, 150, 359, 719])
def test_wigner_pi2_orthogonal_at_large_degree(l):
    """d^l(pi/2) is a real orthogonal matrix; an unstable recursion or a wrong
    reflection sign breaks this long before the last digit."""
    D = sht.wigner_d_pi2(l)
    assert np.abs(D @ D.T - np.eye(2 * l + 1)).max() <= 2e-13


def test_wigner_known_l1():
    """d^1(beta) at beta = pi/2: d_{1,0} = -1/sqrt2, d_{0,1} = +1/sqrt2, d_{1,1} = 1/2."""
    D = sht.wigner_d_pi2(1)
    assert D[2, 1] == pytest.approx(-np.sqrt(0.5), abs=4e-16)
    assert D[1, 2] == pytest.approx(np.sqrt(0.5), abs=4e-16)
    assert D[2, 2] == pytest.approx(0.5, abs=4e-16)


@pytest.mark.parametrize("l,m,th", [(0, 0, 1.0), (1, 1, 0.3), (3, 2, 0.7), (5, -3, 1.1), (7, 7, 0.3),
                                    (7, -6, 2.9), (20, 13, 0.01), (60, -31, 1.7), (60, 60, 3.1)])
def test_fourier_expansion_of_ylm_matches_scipy(l, m, th):
    """Y_lm(theta, 0) = sqrt((2l+1)/4pi) i^-m sum_m' d_{m',0} d_{m',m} e^{i m' theta}."""
    D = sht.wigner_d_pi2(l)
    k = np.arange(-l, l + 1)
    y = np.sqrt((2 * l + 1) / (4 * np.pi)) * (1j) ** (-m) * np.sum(D[k + l, l] * D[k + l, m + l] * np.exp(1j * k * th))
    assert abs(y - sp.sph_harm_y(l, m, th, 0.0)) <= 1e-14


def test_I_q_against_quadrature():
    for q in range(-9, 10):
        re = si.quad(lambda t: np.cos(q * t) * np.sin(t), 0, np.pi, epsabs=1e-13, limit=200)[0]
        im = si.quad(lambda t: np.sin(q * t) * np.sin(t), 0, np.pi, epsabs=1e-13, limit=200)[0]
        assert abs(sht.I_q(np.array([q]))[0] - (re + 1j * im)) <= 1e-13


def random_coeffs(L, seed):
    rng = np.random.default_rng(seed)
    zc = np.zeros((L, 2 * L - 1), complex)
    for l in range(L):
        zc[l, L - 1] = rng.standard_normal()
        for m in range(1, l + 1):
            z = rng.standard_normal() + 1j * rng.standard_normal()
            zc[l, m + L - 1] = z
            zc[l, -m + L - 1] = (-1) ** m * np.conj(z)
    return zc


def scipy_field(zc, ntheta, nphi):
    L = zc.shape[0]
    th, ph = sht.grid(ntheta, nphi)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    Z = np.zeros((ntheta, nphi), complex)
    for l in range(L):
        for m in range(-l, l + 1):
            Z += zc[l, m + L - 1] * sp.sph_harm_y(l, m, TH, PH)
    assert np.abs(Z.imag).max() <= 1e-12
    return Z.real


@pytest.mark.parametrize("L,ntheta,nphi,seed", [(1, 2, 1, 1), (2, 3, 3, 2), (12, 13, 23, 3), (12, 14, 25, 4),
                                                 (9, 20, 40, 5), (17, 18, 36, 6)])
def test_forward_and_inverse_against_scipy_synthesis(L, ntheta, nphi, seed):
    """A band-limited field synthesized with scipy's Y_lm: the forward
    transform returns its coefficients and the inverse returns the field,
    on the smallest grid the method allows (N_theta = L + 1, N_phi = 2L - 1)
    and on larger ones."""
    zc = random_coeffs(L, seed)
    Z = scipy_field(zc, ntheta, nphi)
    zf = sht.sht_forward(Z, L)
    assert np.abs(zf - zc).max() <= 1e-13 * max(1, L)
    Zi = sht.sht_inverse(zc, ntheta, nphi)
    assert np.abs(Zi - Z).max() <= 1e-13 * max(1, L)


def test_closed_form_fields():
    L, nt, nph = 4, 6, 9
    th, ph = sht.grid(nt, nph)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    want = {}
    for name, Z, nz in [("one", np.ones_like(TH), {(0, 0): np.sqrt(4 * np.pi)}),
                        ("cos", np.cos(TH), {(1, 0): np.sqrt(4 * np.pi / 3)}),
                        ("sincos", np.sin(TH) * np.cos(PH), {(1, 1): -np.sqrt(2 * np.pi / 3), (1, -1): np.sqrt(2 * np.pi / 3)})]:
        zc = sht.sht_forward(Z, L)
        ref = np.zeros_like(zc)
        for (l, m), v in nz.items():
            ref[l, m + L - 1] = v
        assert np.abs(zc - ref).max() <= 1e-14, name
        want[name] = zc


def test_real_layout_is_an_isometry_and_round_trips():
    zc = random_coeffs(10, 7)
    f = sht.complex_to_real(zc)
    assert f.size == 100
    assert f @ f == pytest.approx(np.sum(np.abs(zc) ** 2), rel=1e-14)
    assert np.abs(sht.real_to_complex(f) - zc).max() <= 1e-15
    # index of z_{l,0} and the pair for m = 2 at l = 3
    assert f[9 + 3] == zc[3, 9].real
    assert f[9 + 3 + 2] == pytest.approx(np.sqrt(2) * zc[3, 11].real)
    assert f[9 + 3 - 2] == pytest.approx(np.sqrt(2) * zc[3, 11].imag)


def test_selected_coefficients_match_full_transform():
    L, nt, nph = 15, 16, 30
    Z = scipy_field(random_coeffs(L, 8), nt, nph)
    zf = sht.sht_forward(Z, L)
    lm = [(0, 0), (14, 14), (14, -14), (9, 4), (9, -4), (3, 0), (10, 7)]
    sel = sht.sht_forward_coeffs(Z, L, lm)
    assert np.abs(sel - np.array([zf[l, m + L - 1] for l, m in lm])).max() <= 1e-14


def test_grid_too_small_is_rejected():
    with pytest.raises(ValueError):
        sht.sht_forward(np.zeros((5, 20)), 5)  # N_theta = L
    with pytest.raises(ValueError):
        sht.sht_forward(np.zeros((6, 8)), 5)   # N_phi < 2L - 1


def test_pole_reading_only_drops_odd_orders_at_the_poles():
    """Odd-order longitude content added to the two pole rows changes
    nothing (those samples are taken as zero); even-order content does."""
    L, nt, nph = 7, 9, 14
    rng = np.random.default_rng(11)
    Z = rng.standard_normal((nt, nph))
    base = sht.sht_forward(Z, L)
    _, ph = sht.grid(nt, nph)
    Zo = Z.copy()
    Zo[0] += 0.7 * np.cos(3 * ph) - 0.2 * np.sin(ph)
    Zo[-1] += 0.4 * np.sin(5 * ph)
    assert np.abs(sht.sht_forward(Zo, L) - base).max() <= 1e-14
    Ze = Z.copy()
    Ze[0] += 0.5 * np.cos(2 * ph)
    assert np.abs(sht.sht_forward(Ze, L) - base).max() > 1e-3


def test_odd_q_terms_cancel():
    """The q = +-1 terms of I contribute nothing: K_{m,-m'} = (-1)^m K_{m,m'}
    and S_{l,m,-m''} = (-1)^m S_{l,m,m''} pair each (m', m'') term with a
    (-m', -m'') term of opposite sign.  Flipping their sign leaves the
    transform unchanged (a fact the GPU tables use)."""
    good = sht.I_q
    zc = random_coeffs(8, 9)
    Z = scipy_field(zc, 9, 15)

    def flipped(q):
        out = good(q)
        one = np.abs(np.asarray(q)) == 1
        out[one] = -out[one]
        return out

    a = sht.sht_forward(Z, 8)
    sht_I, sht.I_q = sht.I_q, flipped
    try:
        b = sht.sht_forward(Z, 8)
    finally:
        sht.I_q = sht_I
    assert np.abs(a - b).max() <= 1e-14


@pytest.mark.parametrize("mistake", ["transposed_d", "even_q_sign", "no_extension_parity"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    """Plausible mistakes planted in the oracle break the scipy pin."""
    zc = random_coeffs(8, 10)
    Z = scipy_field(zc, 9, 15)
    if mistake == "transposed_d":
        good = sht.wigner_d_pi2
        monkeypatch.setattr(sht, "wigner_d_pi2", lambda l: good(l).T.copy())
    elif mistake == "even_q_sign":
        good = sht.I_q
        monkeypatch.setattr(sht, "I_q", lambda q: np.where(np.asarray(q) % 2 == 0, -good(q), good(q)))
    else:
        def K_no_parity(G, L, orders=None):
            M = 2 * G.shape[0] - 2
            ext = np.concatenate([G, G[1:-1][::-1]], axis=0)
            ms = np.arange(-(L - 1), L)
            return (np.fft.fft(ext, axis=0) / M)[ms % M, :].T
        monkeypatch.setattr(sht, "K_from_G", K_no_parity)
    assert np.abs(sht.sht_forward(Z, 8) - zc).max() > 1e-3
