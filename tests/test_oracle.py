"""Pins of the CPU oracle against facts fixed outside it: hand-derived factors,
exactly representable constructions, closed forms of the exponential kernel,
LAPACK, numpy's IEEE casts, format bit definitions and published known-answer
vectors.  CPU only."""
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _workload(L, rho, nugget):
    sigma, x = synth.workload(L)
    return sigma, x


# ------------------------------------------------------------------ O1 factor
def test_golden_3x3(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "chol3x3.txt")) if l.strip() and not l.startswith("#")]
    A = np.zeros((3, 3))
    Lref = np.zeros((3, 3))
    for i, j, a, l in rows:
        i, j = int(i), int(j)
        A[i, j] = A[j, i] = float(a)
        Lref[i, j] = float(l)
    L, info = orc.potrf(A)
    assert info == 0
    assert np.array_equal(L, Lref)


def test_2x2_closed_form(orc):
    a, b, c = 2.5, -0.75, 3.0
    L, info = orc.potrf(np.array([[a, b], [b, c]]))
    assert info == 0
    ref = np.array([[np.sqrt(a), 0], [b / np.sqrt(a), np.sqrt(c - b * b / a)]])
    assert np.allclose(L, ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,seed", [(7, 1), (64, 2), (300, 3)])
def test_integer_L0_exact(orc, n, seed):
    L0 = synth.int_lower(n, seed)
    A = L0 @ L0.T  # small integers: exact in FP64
    L, info = orc.potrf(A)
    assert info == 0
    assert np.array_equal(L, L0)


def test_lapack_crosscheck(orc):
    sigma, x = synth.workload(20)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, info = orc.potrf(A)
    assert info == 0
    Lnp = np.linalg.cholesky(A)
    assert np.linalg.norm(L - Lnp) / np.linalg.norm(Lnp) < 1e-12


def test_invariants(orc):
    sigma, x = synth.workload(12)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, info = orc.potrf(A)
    assert info == 0
    assert np.all(np.triu(L, 1) == 0)
    assert np.all(np.diag(L) > 0)
    L4, _ = orc.potrf(4.0 * A)  # scaling by a power of two: exact
    assert np.array_equal(L4, 2.0 * L)
    I, _ = orc.potrf(np.eye(9))
    assert np.array_equal(I, np.eye(9))
    d = np.array([4.0, 9.0, 0.25, 16.0])
    D, _ = orc.potrf(np.diag(d))
    assert np.array_equal(D, np.diag(np.sqrt(d)))


def test_not_spd_info(orc):
    A = np.diag([1.0, 2.0, -1.0, 3.0])
    _, info = orc.potrf(A)
    assert info == 3
    B = np.array([[1.0, 2.0], [2.0, 1.0]])
    _, info = orc.potrf(B)
    assert info == 2
    Cn = np.diag([1.0, np.nan, 1.0])
    _, info = orc.potrf(Cn)
    assert info == 2


def test_markov_closed_form_factor(orc):
    """chol(D K D) from the closed form matches the right-looking definition."""
    sigma, x = synth.workload(16)  # N = 256
    A = orc.cov_dense(sigma, x, 5.0, 0.0)
    L, info = orc.potrf(A)
    assert info == 0
    Lc = orc.markov_factor(sigma, x, 5.0)
    assert np.max(np.abs(L - Lc)) / np.max(np.abs(Lc)) < 1e-11


@pytest.mark.parametrize("rho,nugget", [(5.0, 0.0), (5.0, 1e-8), (2.0, 1e-8), (20.0, 1e-8)])
def test_markov_logdet(orc, rho, nugget):
    sigma, x = synth.workload(16)
    A = orc.cov_dense(sigma, x, rho, nugget)
    L, info = orc.potrf(A)
    assert info == 0
    ld_ref = orc.markov_logdet(sigma, x, rho, nugget)
    assert abs(orc.logdet(L) - ld_ref) / abs(ld_ref) < 1e-11
    sgn, ld_np = np.linalg.slogdet(A)
    assert sgn > 0 and abs(ld_np - ld_ref) / abs(ld_ref) < 1e-11


@pytest.mark.parametrize("nugget", [0.0, 1e-8])
def test_markov_solve(orc, nugget):
    sigma, x = synth.workload(16)
    A = orc.cov_dense(sigma, x, 5.0, nugget)
    B = synth.rhs(A.shape[0], 3)
    Xc = orc.markov_solve(sigma, x, 5.0, nugget, B)
    Xn = np.linalg.solve(A, B)
    assert np.linalg.norm(Xc - Xn) / np.linalg.norm(Xn) < 1e-9
    L, _ = orc.potrf(A)
    Xo = orc.potrs(L, B)
    assert np.linalg.norm(Xo - Xc) / np.linalg.norm(Xc) < 1e-9
    # normwise backward error of the oracle solve
    r = np.linalg.norm(B - A @ Xo) / (np.linalg.norm(A) * np.linalg.norm(Xo) + np.linalg.norm(B))
    assert r < 1e-15


def test_markov_logdet_matches_definition_larger(orc):
    sigma, x = synth.workload(32)  # N = 1024, the small workload
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, info = orc.potrf(A)
    assert info == 0
    ld = orc.logdet(L)
    ref = orc.markov_logdet(sigma, x, 5.0, 1e-8)
    assert abs(ld - ref) / abs(ref) < 1e-10


def test_residual_pins(orc):
    L0 = synth.int_lower(40, 5)
    A = L0 @ L0.T
    assert orc.backward_error(A, L0) == 0.0
    sigma, x = synth.workload(8)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, _ = orc.potrf(A)
    E0 = synth.normal(11, A.size).reshape(A.shape)
    E0 = E0 + E0.T
    tau = 1e-6
    be = orc.backward_error(A + tau * E0, L)
    want = tau * np.linalg.norm(E0) / np.linalg.norm(A + tau * E0)
    assert abs(be - want) / want < 1e-3
    # tile residuals add up to the full residual (strict-lower tiles twice)
    t2 = orc.tile_residual2(A + tau * E0, L, 16)
    tot = sum(t2[i, j] * (1 if i == j else 2) for i in range(t2.shape[0]) for j in range(i + 1))
    full = be * np.linalg.norm(A + tau * E0)
    assert abs(np.sqrt(tot) - full) / full < 1e-10


def test_lower_matmul(orc):
    L0 = np.tril(synth.normal(3, 50 * 50).reshape(50, 50))
    Z = synth.normal(4, 50 * 7).reshape(50, 7)
    assert np.allclose(orc.lower_matmul(L0, Z), L0 @ Z, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ formats
def _rand_doubles(seed, n):
    u = synth.uniform01(seed, n)
    e = np.floor(synth.uniform01(seed + 1, n) * 80 - 50)
    s = np.where(synth.uniform01(seed + 2, n) < 0.5, -1.0, 1.0)
    return s * (0.5 + u) * 2.0 ** e


def test_round_f32_matches_numpy(orc):
    v = np.concatenate([_rand_doubles(1, 2000), [0.0, 1e-45, 3e-39, -7e-46, 3.5e38, 1e39]])
    got = orc.round_to(v, orc.F32)
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, ref)


def test_round_f16_matches_numpy(orc):
    v = np.concatenate([_rand_doubles(5, 3000) * 1e-3, [65504.0, 65519.0, 65520.0, 6e-8, 2.98e-8, 2.99e-8, 1e-9]])
    got = orc.round_to(v, orc.F16)
    with np.errstate(over="ignore"):
        ref = v.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, ref)


def test_e4m3_table_and_rounding(orc):
    codes = [c for c in range(256) if not np.isnan(orc.e4m3_decode(c))]
    vals = np.array(sorted({orc.e4m3_decode(c) for c in codes}))
    assert vals.max() == 448.0 and vals.min() == -448.0
    assert np.min(vals[vals > 0]) == 2.0 ** -9
    assert np.isnan(orc.e4m3_decode(0x7F)) and np.isnan(orc.e4m3_decode(0xFF))
    assert len(codes) == 254
    pos = vals[vals >= 0]
    # brute force nearest with ties to an even code (even mantissa)
    def nearest(a):
        d = np.abs(pos - a)
        best = np.flatnonzero(d == d.min())
        if len(best) == 1:
            return pos[best[0]]
        for bi in best:
            m = [c for c in range(128) if orc.e4m3_decode(c) == pos[bi]][0] & 7
            if m % 2 == 0:
                return pos[bi]
        raise AssertionError
    v = np.abs(_rand_doubles(9, 600)) * 2.0 ** -20
    v = np.concatenate([v, [448.0, 460.0, 480.0, 1e5, 2.0 ** -10, 3 * 2.0 ** -11, 2.0 ** -9 * 1.5, 17.0, 18.0, 19.0]])
    got = orc.round_to(v, orc.E4M3)
    for a, g in zip(v, got):
        want = 448.0 if a >= 448.0 else nearest(a)
        assert g == want, (a, g, want)
    assert orc.round_to(np.array([-17.0]), orc.E4M3)[0] == -16.0  # tie to even


def test_round_bf16_bruteforce(orc):
    v = _rand_doubles(13, 500)
    got = orc.round_to(v, orc.BF16)
    for a, g in zip(v, got):
        e = np.floor(np.log2(abs(a)))
        ulp = 2.0 ** (e - 7)
        lo = np.floor(abs(a) / ulp) * ulp
        cands = [lo, lo + ulp]
        d = [abs(abs(a) - c) for c in cands]
        want = cands[int(np.argmin(d))]
        assert abs(g) == want and np.sign(g) == np.sign(a)


def test_scale_exp(orc):
    for fmt, mx in [(orc.F16, 65504.0), (orc.E4M3, 448.0)]:
        for a in np.abs(_rand_doubles(21, 300)) * 1e-20:
            t = orc.scale_exp(a, fmt)
            assert a * 2.0 ** t <= mx < a * 2.0 ** (t + 1)
        assert orc.scale_exp(0.0, fmt) == 0
    assert orc.scale_exp(1e-30, orc.BF16) == 0 and orc.scale_exp(1e-30, orc.F32) == 0


def test_unit_roundoffs(orc):
    assert orc.unit_roundoff(orc.F64) == 2.0 ** -53
    assert orc.unit_roundoff(orc.F32) == 2.0 ** -24
    assert orc.unit_roundoff(orc.BF16) == 2.0 ** -8
    assert orc.unit_roundoff(orc.F16) == 2.0 ** -11
    assert orc.unit_roundoff(orc.E4M3) == 2.0 ** -4


# ------------------------------------------------------------------ maps
def test_map_norm_rule(orc):
    sigma, x = synth.workload(24)  # N = 576
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    b = 64
    fro2, amax, tot = orc.tile_norms(A, b)
    assert abs(tot - np.linalg.norm(A)) / tot < 1e-13
    nt = fro2.shape[0]
    m0 = orc.map_norm(fro2, tot, 1e-30)
    assert np.all(m0 == 0)
    mh = orc.map_norm(fro2, tot, 1e30)
    for I in range(nt):
        for J in range(I + 1):
            assert mh[I, J] == (3 if I - J > 1 else 0)
    m2 = orc.map_norm(fro2, tot, 1e30, band=3, allowed=0b0011)
    for I in range(nt):
        for J in range(I + 1):
            assert m2[I, J] == (1 if I - J > 3 else 0)
    # the rule: lowest allowed class whose unit roundoff times the tile norm fits the budget
    eps = 1e-9
    m = orc.map_norm(fro2, tot, eps, lo16=orc.F16)
    us = [2.0 ** -53, 2.0 ** -24, 2.0 ** -11, 2.0 ** -4]
    thr = eps * tot / nt
    for I in range(nt):
        for J in range(I - 1):
            f = np.sqrt(fro2[I, J])
            c = m[I, J]
            assert f * us[c] <= thr or c == 0
            if c < 3:
                assert f * us[c + 1] > thr
    # monotone in eps
    m3 = orc.map_norm(fro2, tot, 1e-6, lo16=orc.F16)
    assert np.all(m3 >= m)


# ------------------------------------------------------------------ O2 mixed replay
def _class_map(nt, seed):
    u = synth.uniform01(seed, nt * nt).reshape(nt, nt)
    m = np.floor(u * 4).astype(np.uint8)
    m = np.tril(m, -1)
    return np.asfortranarray(m)


@pytest.mark.parametrize("lo16", [3, 2])
def test_mp_integer_exact_any_map(orc, lo16):
    """With A = L0 L0^T (small integers) every stage is exact in every class,
    so the mixed replay must return L0 bit for bit whatever the map."""
    n, b = 256, 32
    L0 = synth.int_lower(n, 17)
    A = L0 @ L0.T
    nt = n // b
    cmap = _class_map(nt, 23)
    assert set(np.unique(cmap[np.tril_indices(nt, -1)])) == {0, 1, 2, 3}
    Lh, info, ts = orc.mp_factor(A, b, cmap, lo16=lo16)
    assert info == 0
    assert np.array_equal(Lh, L0)


def test_mp_all_fp64_matches_o1(orc):
    sigma, x = synth.workload(16)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, _ = orc.potrf(A)
    nt = (A.shape[0] + 63) // 64
    Lh, info, _ = orc.mp_factor(A, 64, np.zeros((nt, nt), np.uint8))
    assert info == 0
    assert np.linalg.norm(Lh - L) / np.linalg.norm(L) < 1e-13
    assert orc.backward_error(A, Lh) < 1e-15


def test_mp_padding(orc):
    """N not a multiple of b: the identity padding leaves factor and logdet unchanged."""
    sigma, x = synth.workload(15)  # N = 225, b = 64 -> 4 tiles, last has 33 rows
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    L, _ = orc.potrf(A)
    Lh, info, _ = orc.mp_factor(A, 64, np.zeros((4, 4), np.uint8))
    assert info == 0
    assert np.linalg.norm(Lh - L) / np.linalg.norm(L) < 1e-13
    assert abs(orc.logdet(Lh) - orc.markov_logdet(sigma, x, 5.0, 1e-8)) < 1e-9 * abs(orc.logdet(L))


@pytest.mark.parametrize("cls,u", [(1, 2.0 ** -24), (2, 2.0 ** -11), (3, 2.0 ** -4)])
def test_mp_error_scales_with_precision(orc, cls, u):
    """All off-band tiles in one class: the backward error lands at that class's
    rounding level relative to the off-band part of Sigma."""
    sigma, x = synth.workload(16)
    # a well-conditioned variant (larger diagonal perturbation), so that even
    # all-FP8 off-band tiles keep the perturbed matrix positive definite
    A = orc.cov_dense(sigma, x, 5.0, 1e-2)
    b = 32
    nt = A.shape[0] // b
    cmap = np.zeros((nt, nt), np.uint8)
    for I in range(nt):
        for J in range(I - 1):
            cmap[I, J] = cls
    Lh, info, ts = orc.mp_factor(A, b, cmap, lo16=orc.F16)
    assert info == 0
    fro2, _, tot = orc.tile_norms(A, b)
    off = np.sqrt(sum(2 * fro2[I, J] for I in range(nt) for J in range(I - 1)))
    be = orc.backward_error(A, Lh) * tot
    assert be <= 4 * u * off * np.sqrt(nt)
    assert be >= 0.01 * u * off
    # stored low-precision tiles are exactly representable in their format
    if cls >= 2:
        fmt = orc.F16 if cls == 2 else orc.E4M3
        for I in range(2, nt):
            tile = Lh[I * b:(I + 1) * b, 0:b] * 2.0 ** ts[I, 0]
            assert np.array_equal(orc.round_to(tile[:4, :4], fmt), tile[:4, :4])


def test_mp_not_spd(orc):
    A = np.eye(64)
    A[40, 40] = -1.0
    Lh, info, _ = orc.mp_factor(A, 16, np.zeros((4, 4), np.uint8))
    assert info == 41


# ------------------------------------------------------------------ Philox draws
def test_philox_kat(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_normal_draws_moments(orc):
    z, raw = orc.normal_draws(2, 200001)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    o = orc.philox4x32_10([1, 0, 0, 0], [2, 0])
    assert list(raw[4:8]) == o


# ------------------------------------------------------------------ selector MLP
def _params(orc, seed, scale=0.3):
    return np.ascontiguousarray(synth.normal(seed, orc.NPARAM) * scale)


def test_mlp_forward_hand_case(orc):
    P = np.zeros(orc.NPARAM)
    # W1 = [I_8; 0], b1 = 0 -> h1 = relu(x) on the first 8 units
    for i in range(8):
        P[i * 8 + i] = 1.0
    off_w2 = 512 + 64
    for i in range(8):
        P[off_w2 + i * 64 + i] = 2.0  # h2_i = relu(2 h1_i)
    off_b2 = off_w2 + 4096
    off_w3 = off_b2 + 64
    for c in range(4):
        P[off_w3 + c * 64 + c] = 1.0
        P[off_w3 + c * 64 + 4 + c] = -1.0
    P[off_w3 + 256 + 0] = 0.5  # b3
    x = np.array([[1.0, -2.0, 3.0, 0.5, 0.25, 4.0, -1.0, 2.0]])
    z = orc.mlp_forward(P, x)
    r = np.maximum(x[0], 0)
    want = [2 * r[c] - 2 * r[4 + c] for c in range(4)]
    want[0] += 0.5
    assert np.allclose(z[0], want, rtol=0, atol=1e-15)


def test_mlp_grad_finite_difference(orc):
    P = _params(orc, 3)
    X, y = synth.features_toy(16, 5)
    cw = np.array([1.0, 1.5, 2.0, 0.5])
    loss, g = orc.mlp_loss_grad(P, X.astype(np.float64), y, cw, 0.7)
    idx = np.concatenate([np.arange(0, orc.NPARAM, 97), [orc.NPARAM - 1, orc.NPARAM - 2, orc.NPARAM - 4]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (orc.mlp_loss_grad(Pp, X.astype(np.float64), y, cw, 0.7)[0]
              - orc.mlp_loss_grad(Pm, X.astype(np.float64), y, cw, 0.7)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mlp_training_decreases_loss(orc):
    P = _params(orc, 3, 0.2)
    X, y = synth.features_toy(256, 7)
    X = X.astype(np.float64)
    cw = np.ones(4)
    m, v = np.zeros_like(P), np.zeros_like(P)
    l0 = orc.mlp_loss_grad(P, X, y, cw, 0.0)[0]
    for s in range(1, 201):
        _, g = orc.mlp_loss_grad(P, X, y, cw, 0.0)
        orc.adam_step(P, g, m, v, s, lr=3e-3)
    l1 = orc.mlp_loss_grad(P, X, y, cw, 0.0)[0]
    assert l1 < 0.3 * l0
    acc = np.mean(np.argmax(orc.mlp_forward(P, X), axis=1) == y)
    assert acc > 0.9


# ---------------------------------------------------------------- covariance from samples
def test_cov_samples_identity_samples(orc):
    """xi = [I 0]: S = (scale + nugget) I exactly (drops of the scale, the
    nugget or a transposed contraction all fail)."""
    n, m = 7, 12
    xi = np.zeros((n, m))
    xi[:, :n] = np.eye(n)
    S = orc.cov_samples(xi, 0.25, 0.125)
    assert S.shape == (n, n)
    assert np.array_equal(S, 0.375 * np.eye(n))


def test_cov_samples_rank_one_closed_form(orc):
    """xi = u v^T: S = scale |v|^2 u u^T + nugget I."""
    u = synth.normal(5, 9)
    v = synth.normal(6, 13)
    S = orc.cov_samples(np.outer(u, v), 0.5, 1e-3)
    want = 0.5 * float(v @ v) * np.outer(u, u) + 1e-3 * np.eye(9)
    assert np.max(np.abs(S - want)) <= 1e-13 * np.max(np.abs(want))


def test_cov_samples_hadamard_gives_exact_covariance(orc):
    """xi = L0 H_n with H_n the first n rows of a Sylvester-Hadamard matrix of
    order m (H_n H_n^T = m I): with scale 1/m the estimator returns L0 L0^T
    exactly, the population covariance the samples were drawn to have."""
    n, m = 24, 32
    L0 = synth.int_lower(n, 9)
    xi = L0 @ synth.hadamard(m)[:n, :]
    S = orc.cov_samples(xi, 1.0 / m, 0.0)
    assert np.array_equal(S, L0 @ L0.T)


def test_cov_samples_symmetric_psd(orc):
    xi = synth.samples(40, 25)
    S = orc.cov_samples(xi, 1.0 / 25, 1e-6)
    assert np.array_equal(S, S.T)
    assert np.linalg.eigvalsh(S).min() >= 1e-6 * (1 - 1e-6)


# ---------------------------------------------------------------- three-way BF16 split products
def test_split3_reconstructs_every_float(orc):
    """hi + mid + lo == float(v) exactly, each part a BF16 value and each
    smaller than the previous by at least 2^8 (the split that makes the six
    part products carry a float product's information)."""
    z = synth.normal(71, 3000)
    e = synth.uniform01(72, 3000) * 60.0 - 30.0
    for v in z * np.exp(e):
        v32 = float(np.float32(v))
        hi, mid, lo = orc.split3(v)
        assert hi + mid + lo == v32
        for p in (hi, mid, lo):
            assert orc.round_to(p, orc.BF16) == p
        assert abs(mid) <= abs(hi) * 2.0 ** -8 and abs(lo) <= abs(mid) * 2.0 ** -8


def test_mp_factor_split_integer_exact(orc):
    """A = L0 L0^T with small integers and every off-band tile FP32 under the
    split products: the replay returns L0 exactly."""
    n, b = 384, 128
    L0 = synth.int_lower(n, 13)
    A = L0 @ L0.T
    nt = n // b
    cmap = np.tril(np.ones((nt, nt), np.uint8), -1)
    Lh, info, _ = orc.mp_factor(A, b, cmap, lo32=1)
    assert info == 0 and np.array_equal(Lh, L0)


def test_mp_factor_split_close_to_fp32(orc):
    """On a covariance with a map using every class, the split-product replay
    stays within a few times the spread between two summation orders of the
    plain FP32 replay (the three dropped part products are of the order of a
    float rounding)."""
    sigma, x = synth.workload(24)
    A = orc.cov_dense(sigma, x, 5.0, 1e-2)
    b, nt = 64, 9
    u = synth.uniform01(73, nt * nt).reshape(nt, nt)
    cmap = np.tril(np.floor(u * 4).astype(np.uint8), -1)
    L0, _, _ = orc.mp_factor(A, b, cmap, order=0)
    L1, _, _ = orc.mp_factor(A, b, cmap, order=1)
    Ls, info, _ = orc.mp_factor(A, b, cmap, lo32=1)
    assert info == 0
    d_oo = np.linalg.norm(L0 - L1) / np.linalg.norm(L0)
    d_so = np.linalg.norm(Ls - L0) / np.linalg.norm(L0)
    assert 0 < d_so <= 4.0 * d_oo


# ---------------------------------------------------------------- block-scaled FP8 copies
def test_mx_block_exponent_brute_force(orc):
    """The block exponent is the largest t in [-127, 127] (the E8M0 range) with
    max 2^t <= 448, found here by trying every t; 0 for an all-zero block."""
    u = synth.uniform01(91, 200)
    vals = [448.0, 449.0, 447.9, 224.0, 1.0, 3.0, 0.75, 2.0 ** -120, 2.0 ** -140, 2.0 ** 119, 2.0 ** 140, 1e-300,
            1e300, np.nextafter(448.0, 0.0), np.nextafter(448.0, 1e9)]
    vals += list(np.ldexp(0.5 + u[:100], (u[100:] * 80 - 40).astype(int)))
    for a in vals:
        ok = [t for t in range(-127, 128) if a <= np.ldexp(448.0, -t)]
        want = max(ok) if ok else -127
        assert orc.mx_block_exp(a) == want, a
    assert orc.mx_block_exp(0.0) == 0
    # a maximum that is not finite has no exponent: 0, and the call returns
    for fmt in (orc.E4M3, orc.F16):
        assert orc.scale_exp(float("inf"), fmt) == 0 and orc.scale_exp(float("nan"), fmt) == 0
    assert orc.mx_block_exp(float("inf")) == 0


def test_mx_quantize_exact_for_short_significands(orc):
    """Values of at most four significant bits are exact in E4M3 at any scale:
    with a different exponent in every 32-element block of a row (spread over
    2^-40 .. 2^40) the block-scaled copy reproduces them exactly, while one
    scale per row block pair of 64 elements, or per whole array, does not (it
    flushes the small blocks)."""
    rows, cols = 6, 160
    u = synth.uniform01(92, rows * cols).reshape(rows, cols)
    k = np.floor(u * 31).astype(np.int64) - 15                       # -15 .. 15
    d = np.floor(synth.uniform01(93, rows * cols).reshape(rows, cols) * 4).astype(int)   # 0 .. 3
    e = np.floor(synth.uniform01(94, rows * cols // 32).reshape(rows, cols // 32) * 81).astype(int) - 40
    X = np.ldexp(k.astype(float), d + np.repeat(e, 32, axis=1))
    Q, texp = orc.mx_quantize(X)
    assert np.array_equal(Q, X)
    # the exponents follow the 32-element blocks along each row
    for r in range(rows):
        for c in range(cols // 32):
            assert texp[r, c] == orc.mx_block_exp(np.max(np.abs(X[r, 32 * c:32 * c + 32])))
    # a scale shared by 64 elements, or by the whole array, loses the small blocks
    for width in (64, cols):
        Y = np.zeros_like(X)
        for c0 in range(0, cols, width):
            for r in range(rows if width < cols else 1):
                blk = X[r, c0:c0 + width] if width < cols else X
                t = orc.mx_block_exp(np.max(np.abs(blk)))
                q = np.array([np.ldexp(orc.round_to(float(np.float32(np.ldexp(v, t))), orc.E4M3), -t)
                              for v in blk.ravel()]).reshape(blk.shape)
                if width < cols:
                    Y[r, c0:c0 + width] = q
                else:
                    Y = q
        assert not np.array_equal(Y, X)


def test_mx_quantize_equals_tile_copy_when_every_block_holds_the_max(orc):
    """If every block of every row holds the array's largest |value|, every
    block exponent is the per-tile exponent and the copy is the per-tile
    E4M3 copy element for element."""
    rows, cols = 5, 96
    X = (synth.uniform01(95, rows * cols).reshape(rows, cols) - 0.5) * 7.0
    M = 11.3
    for r in range(rows):
        for c in range(0, cols, 32):
            X[r, c + (r * 7 + c) % 32] = M if (r + c) % 3 else -M
    t = orc.scale_exp(M, orc.E4M3)
    tile = np.array([np.ldexp(orc.round_to(float(np.float32(np.ldexp(v, t))), orc.E4M3), -t)
                     for v in X.ravel()]).reshape(X.shape)
    Q, texp = orc.mx_quantize(X)
    assert np.all(texp == t)
    assert np.array_equal(Q, tile)


def test_mx_quantize_error_bound(orc):
    """Every element is within the E4M3 rounding bound of its block: 2^-4 of
    its magnitude in the normal range (plus the float step before it), or
    half the subnormal spacing 2^-9 of the scaled block below it; a row's
    last block may be shorter than 32."""
    rows, cols = 7, 77
    u = synth.uniform01(96, rows * cols).reshape(rows, cols)
    X = (u - 0.5) * np.ldexp(1.0, (synth.uniform01(97, rows * cols).reshape(rows, cols) * 50 - 25).astype(int))
    Q, texp = orc.mx_quantize(X)
    assert texp.shape == (rows, 3)
    for r in range(rows):
        for c in range(cols):
            t = texp[r, c // 32]
            bound = max(2.0 ** -4 * (1 + 2.0 ** -19) * abs(X[r, c]), np.ldexp(1.0, -10 - t))
            assert abs(Q[r, c] - X[r, c]) <= bound


@pytest.mark.parametrize("kind", ["all8", "mixed"])
def test_mp_factor_mx_integer_exact(orc, kind):
    """A = L0 L0^T with graded integers (magnitudes that change from row to row
    and from one 32-column block to the next): with block-scaled FP8 copies
    the replay returns L0 exactly, in an all-FP8 map and in a map over every
    class -- a copy read at the wrong block's scale would not."""
    n, b = 320, 64
    L0 = synth.int_lower(n, 29, graded=True)
    A = L0 @ L0.T
    nt = n // b
    if kind == "all8":
        cmap = np.tril(np.full((nt, nt), 3, np.uint8), -1)
    else:
        u = synth.uniform01(31, nt * nt).reshape(nt, nt)
        cmap = np.tril(np.floor(u * 4).astype(np.uint8), -1)
    Lh, info, _ = orc.mp_factor(A, b, cmap, lo8=1)
    assert info == 0 and np.array_equal(Lh, L0)


def test_mp_factor_mx_invariants(orc):
    """Where block scaling cannot change the replay, it does not: in an all-FP8
    map every panel tile is stored on its tile's E4M3 grid, which every finer
    block scale represents exactly, so the block-scaled copies equal the
    per-tile ones and the factors agree bit for bit; likewise on a map
    without FP8 tiles.  (The copies of panel tiles stored in a higher class do
    differ: the graded integer test above reads them at their block scales.)"""
    sigma, x = synth.workload(20)
    A = orc.cov_dense(sigma, x, 5.0, 1e-1)
    b, nt = 64, 7
    n = b * nt - 20
    A = A[:n, :n]
    cmap = np.tril(np.full((nt, nt), 3, np.uint8), -1)
    Lt, it, tt = orc.mp_factor(A, b, cmap)
    Lm, im, tm = orc.mp_factor(A, b, cmap, lo8=1)
    assert it == 0 and im == 0 and np.array_equal(tt, tm)
    assert np.array_equal(Lm, Lt)
    L, _ = orc.potrf(A)
    assert 0 < np.linalg.norm(Lt - L) / np.linalg.norm(L) <= 2.0 ** -4
    cmap2 = np.tril(np.full((nt, nt), 2, np.uint8), -1)
    La, _, _ = orc.mp_factor(A, b, cmap2)
    Lb, _, _ = orc.mp_factor(A, b, cmap2, lo8=1)
    assert np.array_equal(La, Lb)


# ---------------------------------------------------------------- Adam against hand-derived steps
def test_adam_two_steps_golden(orc):
    """Two Adam steps (Kingma & Ba, with bias correction) against values derived
    by hand in exact rational arithmetic (tests/golden/adam_two_steps.txt).
    eps = 0.5 makes the bias correction and the place of eps visible in every
    step-1 value."""
    rows = [l.split() for l in open(os.path.join(GOLD, "adam_two_steps.txt")) if l.strip() and not l.startswith("#")]
    th0 = np.array([float(r[1]) for r in rows])
    g1 = np.array([float(r[2]) for r in rows])
    g2 = np.array([float(r[3]) for r in rows])
    want1 = np.array([float(r[4]) for r in rows])
    want2 = np.array([float(r[5]) for r in rows])
    P, m, v = th0.copy(), np.zeros(3), np.zeros(3)
    orc.adam_step(P, g1, m, v, 1, lr=0.1, b1=0.5, b2=0.75, eps=0.5)
    assert np.allclose(P, want1, rtol=2e-16, atol=0)
    orc.adam_step(P, g2, m, v, 2, lr=0.1, b1=0.5, b2=0.75, eps=0.5)
    assert np.allclose(P, want2, rtol=4e-16, atol=0)


# ---------------------------------------------------------------- per-tile residual attribution
@pytest.mark.parametrize("I,J", [(0, 0), (2, 1), (4, 0), (4, 4), (3, 3)])
def test_tile_residual2_planted_in_one_tile(orc, I, J):
    """A = L0 L0^T exactly (small integers) plus an integer perturbation E
    planted in the lower part of tile (I, J) only: the per-tile residual of L0
    is exactly the planted tile's ||E||^2 (strict-lower entries of a diagonal
    tile counted twice, as in the symmetric matrix) and exactly zero in every
    other tile.  n = 70, b = 16: the last tile row and column have 6 entries."""
    n, b = 70, 16
    nt = (n + b - 1) // b
    L0 = synth.int_lower(n, 31)
    A = L0 @ L0.T
    E = np.zeros((n, n))
    r0, r1 = I * b, min(n, (I + 1) * b)
    c0, c1 = J * b, min(n, (J + 1) * b)
    vals = np.round(synth.normal(40 + 7 * I + J, (r1 - r0) * (c1 - c0)) * 2).reshape(r1 - r0, c1 - c0)
    vals[vals == 0] = 1.0
    E[r0:r1, c0:c1] = vals
    if I == J:
        E = np.tril(E)
        E = E + np.tril(E, -1).T  # symmetric, so the planted matrix stays a covariance
    t2 = orc.tile_residual2(A + E, L0, b)
    want = np.zeros((nt, nt))
    blk = np.tril(E[r0:r1, c0:c1]) if I == J else E[r0:r1, c0:c1]
    w = np.where(np.eye(r1 - r0, c1 - c0, dtype=bool), 1.0, 2.0) if I == J else 1.0
    want[I, J] = np.sum(w * blk * blk)
    assert np.array_equal(np.tril(t2), want)


# ---------------------------------------------------------------- O2 rounding placement
_E4M3 = None


def _e4m3_table():
    """Every finite non-negative E4M3FN value, indexed by its code, decoded from
    the OCP bit definition (4 exponent bits, bias 7, 3 mantissa bits, no infinity,
    code 0x7F is NaN)."""
    global _E4M3
    if _E4M3 is None:
        t = []
        for c in range(0x7F):
            e, m = c >> 3, c & 7
            t.append(m / 8 * 2.0 ** -6 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
        _E4M3 = np.array(t)
    return _E4M3


def _rne_e4m3(x):
    """Nearest E4M3FN value of the float x, ties to the even code, saturating at 448."""
    tab = _e4m3_table()
    a = min(abs(float(x)), 448.0)
    d = np.abs(tab - a)
    best = np.flatnonzero(d == d.min())
    code = best[0] if len(best) == 1 else [c for c in best if c % 2 == 0][0]
    return float(np.copysign(tab[code], x))


def _rne_bf16(x):
    """float32 x to bfloat16 by round-to-nearest-even on the 16 dropped bits of its encoding."""
    u = int(np.array(x, dtype=np.float32).view(np.uint32))
    low, high = u & 0xFFFF, u >> 16
    if low > 0x8000 or (low == 0x8000 and high & 1):
        high += 1
    return float(np.array(high << 16, dtype=np.uint32).view(np.float32))


def _scale(amax, maxf):
    """Largest integer t with amax * 2^t <= maxf (0 for amax = 0)."""
    if amax == 0.0:
        return 0
    t = 0
    while amax * 2.0 ** t > maxf:
        t -= 1
    while amax * 2.0 ** (t + 1) <= maxf:
        t += 1
    return t


def _o2_replica(A, b, cmap, lo16, lo32):
    """The mixed tile algorithm written out step by step for tiny sizes, with
    rounding by numpy's float32/float16 casts, bfloat16 from the float32
    encoding and E4M3 from its code table: W in FP64 with FP32 work tiles for
    lower classes; POTRF in FP64; TRSM in FP64 then rounded to FP32 (lower
    classes) and stored as fmt(f32(v 2^t)) 2^-t (16-bit/FP8); one copy per
    consumer class made from the stored tile; GEMMs in the tile's class with
    float products and float sums in k order, the FP32 work tile updated in
    float.  f32 = np.float32, so every rounding placement is explicit."""
    f32 = lambda v: float(np.float32(v))
    n = A.shape[0]
    nt = -(-n // b)
    npd = nt * b
    W = np.eye(npd)
    W[:n, :n] = A
    for I in range(nt):
        for J in range(I):
            if cmap[I, J] != 0:
                W[I * b:(I + 1) * b, J * b:(J + 1) * b] = np.float32(W[I * b:(I + 1) * b, J * b:(J + 1) * b])

    def fmt_round(v, q):
        if q == 2 and lo16 == 2:
            return _rne_bf16(v)
        if q == 2:
            return float(np.float16(np.float32(v)))
        return _rne_e4m3(v)

    def maxf(q):
        return None if (q == 2 and lo16 == 2) else (65504.0 if q == 2 else 448.0)

    tsc = np.zeros((nt, nt), np.int32)
    for k in range(nt):
        k0 = k * b
        D = W[k0:k0 + b, k0:k0 + b]
        for c in range(b):  # POTRF, right-looking
            D[c, c] = np.sqrt(D[c, c])
            for i in range(c + 1, b):
                D[i, c] /= D[c, c]
            for j in range(c + 1, b):
                for i in range(j, b):
                    D[i, j] -= D[i, c] * D[j, c]
        copies = {}
        for I in range(k + 1, nt):
            X = W[I * b:(I + 1) * b, k0:k0 + b]
            for c in range(b):  # TRSM, forward substitution in FP64
                for cc in range(c):
                    X[:, c] -= X[:, cc] * D[c, cc]
                X[:, c] /= D[c, c]
            q = cmap[I, k]
            if q != 0:
                X[:] = np.float32(X)
                if maxf(q) is not None or q == 2:
                    t = _scale(np.max(np.abs(X)), maxf(q)) if maxf(q) else 0
                    if q >= 2:
                        tsc[I, k] = t
                        for r in range(b):
                            for c in range(b):
                                X[r, c] = fmt_round(f32(X[r, c] * 2.0 ** t), q) * 2.0 ** -t
            m = np.max(np.abs(X))
            cp = {0: (X.copy(), 0), 1: (np.float32(X).astype(np.float64), 0)}
            for q in (2, 3):
                t = _scale(m, maxf(q)) if maxf(q) else 0
                cp[q] = (np.array([[fmt_round(f32(X[r, c] * 2.0 ** t), q) for c in range(b)] for r in range(b)]), t)
            copies[I] = cp
        for I in range(k + 1, nt):
            for J in range(k + 1, I + 1):
                q = 0 if I == J else cmap[I, J]
                (CI, tI), (CJ, tJ) = copies[I][q], copies[J][q]
                Wt = W[I * b:(I + 1) * b, J * b:(J + 1) * b]
                for r in range(b):
                    for s in range(b):
                        if q == 0:
                            acc = 0.0
                            for c in range(b):
                                acc += CI[r, c] * CJ[s, c]
                            Wt[r, s] -= acc
                            continue
                        acc = np.float32(0.0)
                        if q == 1 and lo32:
                            def parts(v):
                                hi = _rne_bf16(f32(v))
                                mid = _rne_bf16(f32(f32(v) - hi))
                                lo = _rne_bf16(f32(f32(f32(v) - hi) - mid))
                                return (hi, mid, lo)
                            for pa, pb in ((1, 1), (0, 2), (2, 0), (0, 1), (1, 0), (0, 0)):
                                for c in range(b):
                                    acc = np.float32(acc + np.float32(parts(CI[r, c])[pa]) * np.float32(parts(CJ[s, c])[pb]))
                        else:
                            for c in range(b):
                                acc = np.float32(acc + np.float32(CI[r, c]) * np.float32(CJ[s, c]))
                        w = np.float32(Wt[r, s])
                        Wt[r, s] = float(w - acc) if q == 1 else float(w - np.float32(float(acc) * 2.0 ** -(tI + tJ)))
    return np.tril(W[:n, :n]), tsc


@pytest.mark.parametrize("n", [6, 5])
@pytest.mark.parametrize("lo16,lo32", [(3, 0), (2, 0), (3, 1)])
@pytest.mark.parametrize("classes", [(1, 3, 2), (2, 1, 3), (3, 2, 1), (1, 1, 1)])
def test_mp_rounding_placement_tiny(orc, n, lo16, lo32, classes):
    """O2 against the step-by-step replica above, bit for bit, on nt = 3 tiles
    of b = 2 (n = 5: a padded last tile) for maps putting tiles (1,0), (2,0),
    (2,1) in the classes given: each TRSM output's FP32 rounding, storage
    rounding with its scale, each consumer copy and the FP32/16-bit/FP8
    update of tile (2,1) are then fixed by numpy's IEEE casts and the format
    tables, not by the oracle's own rounding routine."""
    M0 = synth.normal(50 + n, 36).reshape(6, 6)
    A = (M0 @ M0.T + 6.0 * np.eye(6))[:n, :n] * 0.37
    cmap = np.zeros((3, 3), np.uint8)
    cmap[1, 0], cmap[2, 0], cmap[2, 1] = classes
    Lh, info, ts = orc.mp_factor(A, 2, cmap, lo16=lo16, lo32=lo32)
    assert info == 0
    Lr, tr = _o2_replica(A, 2, cmap, lo16, lo32)
    assert np.array_equal(Lh, Lr), np.max(np.abs(Lh - Lr))
    assert np.array_equal(np.tril(ts, -1), np.tril(tr, -1))


# ---------------------------------------------------------------- band rule
def test_map_band_hand_case(orc):
    """nt = 8, FP64 band 1: 28 strict-lower tiles, 5% is 1.4 tiles, so the FP32
    band of DP/SP/HP is the single diagonal I - J = 2 (6 tiles)."""
    d = np.subtract.outer(np.arange(8), np.arange(8))
    low = d > 1
    want = {1: np.where(low, 1, 0), 2: np.where(d == 2, 1, np.where(d > 2, 2, 0)), 3: np.where(low, 2, 0)}
    for v, w in want.items():
        assert np.array_equal(orc.map_band(8, 1, v), w.astype(np.uint8)), v


@pytest.mark.parametrize("nt,band", [(127, 1), (64, 1), (157, 1), (20, 2), (40, 0), (3, 1), (2, 1), (1, 1)])
def test_map_band_sp_band_holds_five_percent(orc, nt, band):
    """DP/SP/HP: the FP32 tiles are a band next to the FP64 band, they hold at
    least 5% of the strict-lower tiles and dropping its outermost diagonal
    leaves less than 5% (or there is no room for more; nt = 40 with band 0 holds
    exactly 5% in one diagonal); DP/SP and DP/HP put
    every off-band tile in FP32 / 16-bit; the FP64 band and the diagonal stay FP64."""
    total = nt * (nt - 1) / 2
    d = np.subtract.outer(np.arange(nt), np.arange(nt))
    m = orc.map_band(nt, band, 2)
    assert np.all(m[d <= band] == 0) and np.all(m[d < 0] == 0)
    sp = (m == 1)
    if nt - 1 > band:
        w32 = d[sp].max()
        assert np.array_equal(sp, (d > band) & (d <= w32))
        assert np.all(m[d > w32] == 2)
        assert sp.sum() >= 0.05 * total or w32 == nt - 1
        assert ((d > band) & (d < w32)).sum() < 0.05 * total
    else:
        assert not sp.any()
    assert np.array_equal(orc.map_band(nt, band, 1), np.where(d > band, 1, 0).astype(np.uint8))
    assert np.array_equal(orc.map_band(nt, band, 3), np.where(d > band, 2, 0).astype(np.uint8))


def test_map_band_c4_widths(orc):
    """nt = 127 (N = 129,600, tile 1024): 8001 strict-lower tiles; diagonals 2..5
    hold 125 + 124 + 123 + 122 = 494 >= 400.05 tiles while 2..4 hold 372."""
    m = orc.map_band(127, 1, 2)
    d = np.subtract.outer(np.arange(127), np.arange(127))
    assert np.array_equal(m == 1, (d >= 2) & (d <= 5))
    assert (m == 1).sum() == 494


def test_map_band_allowed_classes_raise(orc):
    """Classes outside the allowed mask move up to the nearest allowed more precise class."""
    d = np.subtract.outer(np.arange(10), np.arange(10))
    assert np.array_equal(orc.map_band(10, 1, 3, allowed=0b0011), np.where(d > 1, 1, 0).astype(np.uint8))
    assert np.array_equal(orc.map_band(10, 1, 1, allowed=0b1101), np.zeros((10, 10), np.uint8))
    m = orc.map_band(10, 1, 2, allowed=0b0101)
    assert set(np.unique(m[d > 1])) == {0, 2}


# ---------------------------------------------------------------- FP64-class products from exact integer products
def _ozaki_py(A, B, rint=round):
    """The definition with Python integers: row exponents from frexp, entries
    rounded to integers (round half to even by default), exact integer sums,
    Python's correctly rounded int-to-float conversion, scaled back."""
    import math

    def exps(X):
        out = []
        for row in X:
            mu = max(abs(float(v)) for v in row)
            out.append(0 if mu == 0 else 53 - math.frexp(mu)[1])
        return out

    ea, eb = exps(A), exps(B)
    ia = [[int(rint(math.ldexp(float(v), e))) for v in row] for row, e in zip(A, ea)]
    ib = [[int(rint(math.ldexp(float(v), e))) for v in row] for row, e in zip(B, eb)]
    D = np.empty((len(A), len(B)))
    for r in range(len(A)):
        for s in range(len(B)):
            P = sum(x * y for x, y in zip(ia[r], ib[s]))
            D[r, s] = math.ldexp(float(P), -(ea[r] + eb[s]))
    return D


def test_ozaki_gemm_brute_force(orc):
    """Bit for bit against the definition worked with Python integers, on
    rows spanning 60 orders of magnitude, a zero row and mixed signs; the data
    is discriminating: truncating instead of rounding to nearest changes it."""
    g = synth.normal(91, 9 * 37).reshape(9, 37)
    A = g[:5] * np.array([1.0, 1e-30, 1e30, 3.0, 0.0])[:, None]
    A[3, ::3] *= 1e-12  # small entries inside a row: rounded relative to the row maximum
    B = g[5:] * np.array([2.0 ** -40, 1.0, 7.0, 1e-8])[:, None]
    D = orc.ozaki_gemm(A, B)
    Dp = _ozaki_py(A, B)
    assert np.array_equal(D.view(np.int64), Dp.view(np.int64))
    assert np.all(D[4] == 0.0)
    Dt = _ozaki_py(A, B, rint=lambda v: int(v))  # truncation toward zero: a plausible mistake
    assert not np.array_equal(D, Dt)
    # and the definition is close to the exact product
    assert np.allclose(D, A @ B.T, rtol=1e-13, atol=0)


def test_ozaki_conversion_rounds_halfway_to_even(orc):
    """The 128-bit sum is rounded once, to nearest with ties to even: row
    [2^52, t] times row [2, 1] scales to integers [2^52, t] and [2^52, 2^51],
    so P = 2^104 + t 2^51 lies exactly halfway between two doubles for t = 1
    and t = 3 (down to 2^104, up to 2^104 + 2^53), and the result is P 2^-51."""
    for t, want in [(1.0, 2.0 ** 53), (3.0, 2.0 ** 53 + 4.0), (2.0, 2.0 ** 53 + 2.0), (5.0, 2.0 ** 53 + 4.0)]:
        A = np.array([[2.0 ** 52, t]])
        B = np.array([[2.0, 1.0]])
        assert orc.ozaki_row_exp(A[0]) == 0 and orc.ozaki_row_exp(B[0]) == 51
        D = orc.ozaki_gemm(A, B)
        assert D[0, 0] == want, (t, D[0, 0], want)
        assert D[0, 0] == _ozaki_py(A, B)[0, 0]


def test_ozaki_integers_exact_and_error_bound(orc):
    """Small integers are exact (every scaled entry is an integer and every
    sum fits); random data stays within the bound of the definition, against
    the exact rational product: each scaled entry moves by at most half a
    unit, 2^-53 of its row maximum, so each term by 2 2^-53 mu_r nu_s (plus
    a second-order part), and the sum is rounded once."""
    from fractions import Fraction

    L0 = synth.int_lower(24, 5)
    assert np.array_equal(orc.ozaki_gemm(L0, L0), L0 @ L0.T)
    k = 64
    A = synth.normal(92, 6 * k).reshape(6, k) * np.logspace(-3, 3, k)
    B = synth.normal(93, 5 * k).reshape(5, k)
    D = orc.ozaki_gemm(A, B)
    for r in range(6):
        for s in range(5):
            exact = sum(Fraction(float(A[r, c])) * Fraction(float(B[s, c])) for c in range(k))
            bound = 2 * k * 2.0 ** -53 * np.abs(A[r]).max() * np.abs(B[s]).max() * (1 + 2.0 ** -52) \
                + abs(float(exact)) * 2.0 ** -53
            assert abs(Fraction(float(D[r, s])) - exact) <= Fraction(bound)


def test_mp_factor_lo64(orc):
    """O2 with emulated FP64-class products: exact on an integer factor for
    every band width; on the covariance at FP64 level (backward error below
    1e-15) and within rounding of the plain O2 for an all-FP64 map."""
    n, b = 384, 64
    L0 = synth.int_lower(n, 41)
    A0 = L0 @ L0.T
    nt = n // b
    z = np.zeros((nt, nt), np.uint8)
    for band in (0, 1, 3):
        Lh, info, _ = orc.mp_factor(A0, b, z, lo64=1, band=band)
        assert info == 0 and np.array_equal(Lh, L0)
    L = 20
    sigma, x = synth.workload(L)
    S = orc.cov_dense(sigma, x, 5.0, 1e-8)
    m = np.zeros((7, 7), np.uint8)
    L1, i1, _ = orc.mp_factor(S, 64, m, lo64=1, band=0)
    L2, i2, _ = orc.mp_factor(S, 64, m, lo64=0)
    assert i1 == 0 and i2 == 0
    assert orc.backward_error(S, L1) <= 1e-15
    assert np.linalg.norm(L1 - L2) <= 1e-12 * np.linalg.norm(L2)
    # the emulated products do not depend on the summation order: only the
    # FP64 sums of SYRK differ between the two orders
    L3, _, _ = orc.mp_factor(S, 64, m, lo64=1, band=0, order=1)
    assert np.linalg.norm(L3 - L1) <= 1e-13 * np.linalg.norm(L1)
