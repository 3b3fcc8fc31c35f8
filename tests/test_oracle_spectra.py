"""Pins of the power-spectrum oracle (section 3.1 eq. (9); section 3.2
eqs. (10), (11); section 3.3: smoothing and eqs. (12), (13)) against
mathematics and libraries that share nothing with it."""

from fractions import Fraction as F
import math

import mpmath
import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import healpix as H
from oracle import spectra as S


def _ring_z(nside, i):
    N = nside
    if i < N:
        return 1 - F(i * i, 3 * N * N)
    if i <= 3 * N:
        return F(4, 3) - F(2 * i, 3 * N)
    ii = 4 * N - i
    return -(1 - F(ii * ii, 3 * N * N))


def _theta_mp(zq):
    # theta from the exact rational z: 2 asin(sqrt((1 - z)/2))
    one_minus = mpmath.mpf((1 - zq).numerator) / (1 - zq).denominator
    return 2 * mpmath.asin(mpmath.sqrt(one_minus / 2))


def test_ring_table_matches_pixel_centres():
    # against the (separately pinned) exact pix2ang of the binning oracle
    for nside in (1, 2, 3, 8):
        start, count, shift, z, st = S.ring_table(nside)
        assert count.sum() == S.npix(nside)
        for r in range(len(start)):
            for j in (0, int(count[r]) - 1):
                zq, phi = H.pix2ang_ring(nside, int(start[r]) + j)
                assert float(zq) == z[r]
                assert math.isclose(math.pi * (2 * j + shift[r]) / count[r], phi, rel_tol=1e-15)
                assert math.isclose(st[r] ** 2 + z[r] ** 2, 1.0, rel_tol=1e-15)


@pytest.mark.parametrize("nside,i,l,m", [
    (16, 21, 47, 0), (16, 3, 47, 13), (64, 4, 191, 100), (64, 128, 191, 191),
    (1024, 1, 3071, 5), (1024, 2, 3071, 2), (1024, 6, 3071, 3000), (1024, 2048, 3071, 1500),
    (1024, 1001, 2000, 1999), (1024, 3000, 3071, 700), (1024, 4090, 3071, 31), (512, 700, 1535, 1000),
])
def test_lambda_against_mpmath(nside, i, l, m):
    # lambda_lm(cos theta) = Y_lm(theta, 0), mpmath at 30 digits at the exact ring
    # colatitude.  The oracle starts from z rounded to a double, which the
    # recurrence amplifies by up to ~l^2 near the poles: the relative bound
    # carries that term.
    mpmath.mp.dps = 30
    zq = _ring_z(nside, i)
    s2 = (1 - zq) * (1 + zq)
    st = math.sqrt(s2.numerator) / math.sqrt(s2.denominator)
    got = S.legendre_lambda(l, m, np.array([float(zq)]), np.array([st]))[l, 0]
    ref = mpmath.spherharm(l, m, _theta_mp(zq), 0).real
    tol = (1e-13 * l + 1.2e-16 * l * l) * abs(float(ref)) + 1e-25 * math.sqrt((2 * l + 1) / (4 * math.pi))
    assert abs(got - float(ref)) <= tol, (got, float(ref))


def test_lambda_rows_against_scipy_low_degree():
    # scipy's sph_harm_y (its own recurrences) for l < 60 at every ring of Nside 16
    _, _, _, z, st = S.ring_table(16)
    theta = np.arctan2(st, z)
    lmax = 59
    for m in (0, 1, 2, 7, 30, 59):
        lam = S.legendre_lambda(lmax, m, z, st)
        for l in range(m, lmax + 1):
            ref = sph_harm_y(l, m, theta, 0.0).real
            np.testing.assert_allclose(lam[l], ref, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("nside", [1, 2])
def test_map2alm_brute_force_mpmath(nside):
    # a_lm = (4 pi / Npix) sum_p map_p conj(Y_lm(centre_p)), pixel by pixel in mpmath
    mpmath.mp.dps = 25
    rng = np.random.default_rng(7 + nside)
    npx = S.npix(nside)
    mp_map = rng.standard_normal(npx)
    lmax = 3 * nside - 1 + 2
    got = S.map2alm(mp_map, nside, lmax)
    w = 4 * mpmath.pi / npx
    for l in range(lmax + 1):
        for m in range(l + 1):
            s = mpmath.mpc(0)
            for p in range(npx):
                zq, phi = H.pix2ang_ring(nside, p)
                s += mp_map[p] * mpmath.conj(mpmath.spherharm(l, m, _theta_mp(zq), phi))
            ref = complex(w * s)
            assert abs(got[m, l] - ref) <= 1e-13 * (1 + abs(ref)), (l, m, got[m, l], ref)


def test_constant_map():
    nside = 8
    c = 1.75
    a = S.map2alm(np.full(S.npix(nside), c), nside)
    # Y_00 = 1/sqrt(4 pi) and the weights sum to 4 pi exactly
    assert abs(a[0, 0] - c * math.sqrt(4 * math.pi)) <= 1e-14 * c
    # every ring holds 4k pixels at phi_j = pi (2j+s)/n: sum_j e^{-i m phi_j} = 0 unless n | m
    for m in range(a.shape[0]):
        if m % 4:
            assert np.abs(a[m]).max() <= 1e-14


def _rotate_quarter(mp, nside):
    # map'(phi) = map(phi - pi/2): within each ring, pixel j takes pixel j - n/4
    start, count, _, _, _ = S.ring_table(nside)
    out = np.empty_like(mp)
    for r in range(len(start)):
        n = int(count[r])
        ring = mp[start[r]:start[r] + n]
        out[start[r]:start[r] + n] = np.roll(ring, n // 4)
    return out


def _mirror(mp, nside):
    # map'(z) = map(-z): ring i takes ring 4N - i (same azimuths)
    start, count, _, _, _ = S.ring_table(nside)
    out = np.empty_like(mp)
    nr = len(start)
    for r in range(nr):
        q = nr - 1 - r
        out[start[r]:start[r] + count[r]] = mp[start[q]:start[q] + count[q]]
    return out


def test_rotation_and_mirror_symmetries():
    nside = 8
    rng = np.random.default_rng(3)
    mp = rng.standard_normal(S.npix(nside))
    a = S.map2alm(mp, nside)
    lmax = a.shape[1] - 1
    scale = np.abs(a).max()
    m = np.arange(lmax + 1)[:, None]
    l = np.arange(lmax + 1)[None, :]
    rot = S.map2alm(_rotate_quarter(mp, nside), nside)
    np.testing.assert_allclose(rot, a * np.exp(-0.5j * np.pi * m), atol=1e-13 * scale)
    mir = S.map2alm(_mirror(mp, nside), nside)
    np.testing.assert_allclose(mir, a * (-1.0) ** (l + m), atol=1e-13 * scale)


def test_band_limited_recovery():
    # map = Re Y_32 + 0.5 Y_10 at the pixel centres: a_32 = 1/2, a_10 = 1/2, the
    # rest zero up to the pixel quadrature's error (~1e-3 at Nside 32)
    nside = 32
    start, count, shift, z, st = S.ring_table(nside)
    th = np.zeros(S.npix(nside))
    ph = np.zeros(S.npix(nside))
    for r in range(len(start)):
        j = np.arange(count[r])
        ph[start[r]:start[r] + count[r]] = np.pi * (2 * j + shift[r]) / count[r]
        th[start[r]:start[r] + count[r]] = math.atan2(st[r], z[r])
    mp = sph_harm_y(3, 2, th, ph).real + 0.5 * sph_harm_y(1, 0, th, ph).real
    a = S.map2alm(mp, nside)
    assert abs(a[2, 3] - 0.5) < 2e-4 and abs(a[0, 1] - 0.5) < 2e-4
    rest = np.abs(a)
    rest[2, 3] = rest[0, 1] = 0
    assert rest.max() < 2e-3


def test_alm2cl_single_modes():
    lmax = 6
    a = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    a[0, 4] = 3.0            # a_40
    a[2, 5] = 1.0 - 2.0j     # a_52 (and a_5,-2 by reality)
    cl = S.alm2cl(a)
    assert cl[4] == pytest.approx(9.0 / 9)
    assert cl[5] == pytest.approx(2 * 5.0 / 11)
    assert cl[[0, 1, 2, 3, 6]].max() == 0.0


def test_pack_alm_index():
    lmax = 5
    a = np.arange((lmax + 1) ** 2).reshape(lmax + 1, lmax + 1).astype(complex)
    v = S.pack_alm(a, lmax)
    assert len(v) == (lmax + 1) * (lmax + 2) // 2
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            assert v[m * (2 * lmax + 1 - m) // 2 + l] == a[m, l]


@pytest.mark.parametrize("ddof", [0, 1])
def test_covariance_against_numpy(ddof):
    rng = np.random.default_rng(11)
    cl = rng.gamma(2.0, 1.0, size=(150, 64)) * np.linspace(1, 2, 64)
    mean, cov, corr = S.cl_covariance(cl, ell_min=4, delta_ell=10, n_bands=6, ddof=ddof)
    X = np.stack([cl[:, 4 + 10 * b:14 + 10 * b].mean(axis=1) for b in range(6)], axis=1)
    np.testing.assert_allclose(mean, X.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(cov, np.cov(X, rowvar=False, ddof=ddof), rtol=1e-12)
    np.testing.assert_allclose(corr, np.corrcoef(X, rowvar=False), rtol=1e-12, atol=1e-15)
    assert np.allclose(np.diag(corr), 1.0)


@pytest.mark.parametrize("l,m,a", [(4, 2, 0.3 - 0.7j), (3, 0, 1.25), (5, 5, -0.2 + 0.1j)])
def test_alm2map_single_mode_against_mpmath(l, m, a):
    # a real field with one coefficient a_lm (and a_{l,-m} = (-1)^m conj(a_lm)):
    # map = a Y_l0 for m = 0, else 2 Re(a_lm Y_lm), at every pixel centre of Nside 2
    mpmath.mp.dps = 25
    nside, lmax = 2, 6
    full = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    full[m, l] = a
    got = S.alm2map(full, nside)
    for p in range(S.npix(nside)):
        zq, phi = H.pix2ang_ring(nside, p)
        y = mpmath.spherharm(l, m, _theta_mp(zq), phi)
        ref = float((a * y).real) if m == 0 else float(2 * (mpmath.mpc(a.real, a.imag) * y).real)
        assert abs(got[p] - ref) <= 1e-14, (p, got[p], ref)


def test_alm2map_is_the_adjoint_of_map2alm():
    # sum_p x_p alm2map(a)_p = (N_pix / 4 pi) Re sum_lm w_m a_lm conj(map2alm(x)_lm),
    # w_0 = 1, w_m = 2: the quadrature of map2alm is the transpose of the synthesis
    rng = np.random.default_rng(1)
    nside = 4
    lmax = 3 * nside - 1
    x = rng.standard_normal(S.npix(nside))
    a = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    for m in range(lmax + 1):
        a[m, m:] = rng.standard_normal(lmax + 1 - m) + (1j * rng.standard_normal(lmax + 1 - m) if m else 0)
    y = S.map2alm(x, nside)
    lhs = float(np.dot(x, S.alm2map(a, nside)))
    w = np.full((lmax + 1, 1), 2.0)
    w[0] = 1.0
    rhs = float((w * (a * np.conj(y))).real.sum()) * S.npix(nside) / (4 * np.pi)
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_gaussian_beam_is_the_transform_of_a_gaussian_profile():
    # b_l = (int K P_l sin) / (int K sin) for K(theta) = exp(-theta^2 / (2 sigma^2)):
    # equals exp(-l(l+1) sigma^2 / 2) up to O(sigma^2) on the sphere
    from scipy.integrate import quad
    from scipy.special import eval_legendre
    sigma = np.radians(10.8 / 60.0)
    b = S.gaussian_beam(sigma, 400)
    norm = quad(lambda t: np.exp(-t * t / (2 * sigma ** 2)) * np.sin(t), 0, 12 * sigma)[0]
    for l in (0, 1, 10, 100, 250, 400):
        num = quad(lambda t: np.exp(-t * t / (2 * sigma ** 2)) * eval_legendre(l, np.cos(t)) * np.sin(t),
                   0, 12 * sigma, limit=400)[0]
        assert num / norm == pytest.approx(b[l], rel=2e-3, abs=1e-12), l


def test_map_moments_against_scipy_and_closed_forms():
    from scipy.stats import moment
    rng = np.random.default_rng(4)
    q = rng.gamma(2.0, 1.5, size=100_001)
    mean, m2, m4, s2, var_s2 = S.map_moments(q)
    assert mean == pytest.approx(q.mean(), rel=1e-14)
    assert m2 == pytest.approx(moment(q, 2), rel=1e-12)
    assert m4 == pytest.approx(moment(q, 4), rel=1e-12)
    assert s2 == m2
    # two-point values +-1: m2 = m4 = 1, var_s2 = ((N-1)^2 - (N-1)(N-3)) / N^3 = 2(N-1)/N^3
    N = 1000
    two = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    mean, m2, m4, s2, var_s2 = S.map_moments(two)
    assert mean == 0.0 and m2 == 1.0 and m4 == 1.0
    assert var_s2 == pytest.approx(2.0 * (N - 1) / N ** 3, rel=1e-14)
