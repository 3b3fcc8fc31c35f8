"""Oracle (test infrastructure only): spherical-harmonic coefficients and power
spectra of HEALPix RING maps, and the covariance of power spectra over
realisations (section 3.1 eq. (9); section 3.2 eqs. (10) and (11)).

Definitions followed:
  * harmonic analysis as ANAFAST does it without iterative refinement: the
    pixel quadrature
        a_lm = (4 pi / N_pix) sum_p map_p conj(Y_lm(theta_p, phi_p))
    over the pixel centres, 0 <= m <= l <= lmax, lmax = 3 Nside - 1 by default
    (section 3.1);
  * Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi},
    lambda_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta), P_l^m with
    the Condon-Shortley phase (-1)^m;
  * C_l = (|a_l0|^2 + 2 sum_{m>=1} |a_lm|^2) / (2l+1): eq. (9)'s ensemble
    average replaced by the average over the 2l+1 coefficients of one map
    (the ANAFAST estimator for a real map);
  * cov(l, l') = average over realisations of (C_l - <C_l>)(C_l' - <C_l'>),
    normalised by R - ddof.  Eq. (10) as printed multiplies two averages (each
    zero); the reading is the average of the product.  corr = cov /
    sqrt(cov(l,l) cov(l',l')) (eq. (11)).  Bands of width dl (the paper bins by
    dl = 4, 10, 24): the plain mean of C_l over l in [l0 + b dl, l0 + (b+1) dl).

lambda_lm is evaluated by the textbook recurrences in l at fixed m,
    lambda_mm      = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},  lambda_00 = 1/sqrt(4 pi)
    lambda_{m+1,m} = sqrt(2m+3) cos(theta) lambda_mm
    lambda_lm      = c_lm (cos(theta) lambda_{l-1,m} - lambda_{l-2,m} / c_{l-1,m}),
                     c_lm = sqrt((4l^2 - 1) / (l^2 - m^2)),
carried as mantissa * 2^E per ring, so sin^m(theta) cannot underflow; a value
is rounded to a double (possibly to zero) only when it is used.

Pixel sums are grouped by ring (every pixel of a ring has the same theta), and
the azimuthal factor is the plain sum sum_j map_j e^{-i m phi_j} with m phi_j
reduced modulo 2 pi in integers: ring r has n_r pixels at
phi_j = pi (2j + s_r) / n_r, so m phi_j = pi ((m (2j + s_r)) mod 2 n_r) / n_r.

Synthesis and smoothing (section 3.3: maps smoothed with a Gaussian beam of
r.m.s. radius sigma before their PDF and moments are taken):
  * map_p = sum_l b_l [a_l0 lambda_l0(z_p) + 2 Re sum_{m>=1} a_lm lambda_lm(z_p) e^{i m phi_p}],
    the real field whose coefficients are a_lm (a_{l,-m} = (-1)^m conj(a_lm)),
    with the Gaussian beam b_l = exp(-l(l+1) sigma^2 / 2);
  * moments of a map of N pixels (eqs. (12), (13)): mean qbar, the central
    sample moments m_k = (1/N) sum (q - qbar)^k; s^2 = m_2 (eq. (12) as
    printed lacks the square), and the variance of the variance estimator
    sigma_{s^2}^2 = (N-1)^2/N^3 mu_4 - (N-1)(N-3)/N^3 mu_2^2 with mu_k -> m_k.

Pins (tests/test_oracle_spectra.py): lambda against mpmath's spherical
harmonics up to l = 3071, a pixel-by-pixel mpmath sum at Nside 1 and 2, the
constant map, the exact rotation and mirror symmetries of the HEALPix grid,
recovery of band-limited maps, C_l of single modes, numpy's cov/corrcoef.
"""

from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np


def npix(nside: int) -> int:
    return 12 * nside * nside


def ring_table(nside: int):
    """Per ring i = 1 .. 4N-1 (index i-1): first pixel, pixel count n_r,
    azimuth offset s_r (phi_j = pi (2j + s_r)/n_r), z = cos(theta) and
    sin(theta), both from the exact rational z of the ring.

    RING geometry (Gorski et al. 2005):
      i < N       : 4i pixels, z = 1 - i^2/(3N^2), phi_j = pi/(2i) (j + 1/2)
      N <= i <= 3N: 4N pixels, z = 4/3 - 2i/(3N),  phi_j = pi/(2N) (j + 1/2) if i-N even else pi/(2N) j
      i > 3N      : mirror of ring 4N - i (z -> -z, same azimuths).
    """
    N = nside
    nring = 4 * N - 1
    start = np.zeros(nring, dtype=np.int64)
    count = np.zeros(nring, dtype=np.int64)
    shift = np.zeros(nring, dtype=np.int64)
    z = np.zeros(nring)
    st = np.zeros(nring)
    for i in range(1, 4 * N):
        if i < N:
            first, n, s = 2 * i * (i - 1), 4 * i, 1
            zq = 1 - F(i * i, 3 * N * N)
        elif i <= 3 * N:
            first, n, s = 2 * N * (N - 1) + 4 * N * (i - N), 4 * N, 1 if (i - N) % 2 == 0 else 0
            zq = F(4, 3) - F(2 * i, 3 * N)
        else:
            ii = 4 * N - i
            first, n, s = 12 * N * N - 2 * ii * (ii + 1), 4 * ii, 1
            zq = -(1 - F(ii * ii, 3 * N * N))
        start[i - 1], count[i - 1], shift[i - 1] = first, n, s
        z[i - 1] = float(zq)
        s2 = (1 - zq) * (1 + zq)          # sin^2(theta), exact
        st[i - 1] = math.sqrt(s2.numerator) / math.sqrt(s2.denominator)
    return start, count, shift, z, st


def ring_sums(maps: np.ndarray, nside: int, ms) -> np.ndarray:
    """G[r, k] = sum_j map[first_r + j] e^{-i ms[k] phi_j}, complex [4N-1, len(ms)]."""
    start, count, shift, _, _ = ring_table(nside)
    ms = np.asarray(ms, dtype=np.int64)
    m = np.asarray(maps, dtype=np.float64)
    out = np.zeros((len(start), len(ms)), dtype=np.complex128)
    for r in range(len(start)):
        n = int(count[r])
        x = m[start[r]:start[r] + n]
        j2s = 2 * np.arange(n, dtype=np.int64) + shift[r]          # phi_j = pi j2s / n
        k = (ms[None, :] * j2s[:, None]) % (2 * n)                  # m phi_j = pi k / n (mod 2 pi)
        ang = np.pi * k.astype(np.float64) / n
        out[r] = (x[:, None] * (np.cos(ang) - 1j * np.sin(ang))).sum(axis=0)
    return out


def legendre_lambda(lmax: int, m: int, z: np.ndarray, st: np.ndarray) -> np.ndarray:
    """lambda_lm(z) for l = 0 .. lmax (rows l < m are zero), shape [lmax+1, len(z)].

    z = cos(theta) and st = sin(theta) per point.  Values too small for a
    double become zero (or subnormal) only at the final conversion.
    """
    z = np.asarray(z, dtype=np.float64)
    st = np.asarray(st, dtype=np.float64)
    out = np.zeros((lmax + 1, len(z)))
    if m > lmax:
        return out
    # lambda_mm as mantissa * 2^E
    mant = np.full(len(z), 1.0 / math.sqrt(4.0 * math.pi))
    E = np.zeros(len(z), dtype=np.int64)
    zero = st == 0.0
    for k in range(1, m + 1):
        mant = mant * (-math.sqrt((2 * k + 1) / (2 * k))) * st
        fr, ex = np.frexp(mant)
        mant, E = fr, E + ex
    if m > 0:
        mant = np.where(zero, 0.0, mant)
    out[m] = np.ldexp(mant, E)
    if m == lmax:
        return out
    prev = mant
    cur = math.sqrt(2 * m + 3) * z * mant                  # lambda_{m+1,m}, same exponent E
    out[m + 1] = np.ldexp(cur, E)
    c_prev = math.sqrt((4.0 * (m + 1) ** 2 - 1.0) / ((m + 1) ** 2 - m * m))
    for l in range(m + 2, lmax + 1):
        c = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        new = c * (z * cur - prev / c_prev)
        _, ex = np.frexp(np.maximum(np.abs(cur), np.abs(new)))   # exponent 0 when both vanish
        prev, cur, E = np.ldexp(cur, -ex), np.ldexp(new, -ex), E + ex
        out[l] = np.ldexp(cur, E)
        c_prev = c
    return out


def map2alm(maps: np.ndarray, nside: int, lmax: int | None = None, ms=None) -> np.ndarray:
    """a[k, l] = a_{l, ms[k]} (zero for l < m), complex [len(ms), lmax+1].

    Default lmax = 3 Nside - 1 and ms = 0 .. lmax (section 3.1).
    """
    if lmax is None:
        lmax = 3 * nside - 1
    if ms is None:
        ms = list(range(lmax + 1))
    _, _, _, z, st = ring_table(nside)
    G = ring_sums(maps, nside, ms)
    w = 4.0 * math.pi / npix(nside)
    out = np.zeros((len(ms), lmax + 1), dtype=np.complex128)
    for k, m in enumerate(ms):
        lam = legendre_lambda(lmax, int(m), z, st)          # [l, ring]
        out[k] = w * (lam @ G[:, k])
    return out


def pack_alm(a_full: np.ndarray, lmax: int) -> np.ndarray:
    """Full [m, l] array (m = 0..lmax) -> m-major packed vector,
    index m (2 lmax + 1 - m) / 2 + l for l >= m."""
    out = []
    for m in range(lmax + 1):
        out.append(a_full[m, m:lmax + 1])
    return np.concatenate(out)


def alm2cl(a_full: np.ndarray) -> np.ndarray:
    """C_l from the full [m, l] coefficient array (m = 0 .. lmax)."""
    lmax = a_full.shape[1] - 1
    cl = np.zeros(lmax + 1)
    for l in range(lmax + 1):
        s = abs(a_full[0, l]) ** 2
        for m in range(1, l + 1):
            s += 2.0 * abs(a_full[m, l]) ** 2
        cl[l] = s / (2 * l + 1)
    return cl


def band_powers(cl: np.ndarray, ell_min: int, delta_ell: int, n_bands: int) -> np.ndarray:
    """Mean of C_l over each band [ell_min + b dl, ell_min + (b+1) dl); cl is [R, n_ell]."""
    cl = np.atleast_2d(np.asarray(cl, dtype=np.float64))
    out = np.zeros((cl.shape[0], n_bands))
    for b in range(n_bands):
        lo = ell_min + b * delta_ell
        out[:, b] = cl[:, lo:lo + delta_ell].sum(axis=1) / delta_ell
    return out


def cl_covariance(cl: np.ndarray, ell_min: int = 0, delta_ell: int = 1, n_bands: int | None = None,
                  ddof: int = 1):
    """(mean [n_bands], cov [n_bands, n_bands], corr) over the R realisations of
    cl [R, n_ell] (eqs. (10), (11)); plain loops over realisations."""
    cl = np.asarray(cl, dtype=np.float64)
    R, n_ell = cl.shape
    if n_bands is None:
        n_bands = (n_ell - ell_min) // delta_ell
    X = band_powers(cl, ell_min, delta_ell, n_bands)
    mean = X.sum(axis=0) / R
    cov = np.zeros((n_bands, n_bands))
    for r in range(R):
        d = X[r] - mean
        cov += np.outer(d, d)
    cov /= (R - ddof)
    sd = np.sqrt(np.diag(cov))
    with np.errstate(divide="ignore", invalid="ignore"):
        corr = cov / np.outer(sd, sd)
    return mean, cov, corr


def gaussian_beam(sigma: float, lmax: int) -> np.ndarray:
    """b_l = exp(-l (l+1) sigma^2 / 2), sigma the r.m.s. radius in radians."""
    l = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * l * (l + 1.0) * sigma * sigma)


def alm2map(a_full: np.ndarray, nside: int, beam=None, rings=None) -> np.ndarray:
    """Real map from the full [m, l] coefficients (m = 0..lmax), optionally
    multiplied by a beam b_l; grouped by ring, azimuths reduced in integers.
    `rings` (indices i-1) restricts the work to those rings; the other pixels
    are left at zero."""
    lmax = a_full.shape[1] - 1
    start, count, shift, z, st = ring_table(nside)
    sel = np.arange(len(start)) if rings is None else np.asarray(rings, dtype=np.int64)
    b = np.ones(lmax + 1) if beam is None else np.asarray(beam, dtype=np.float64)
    # per ring and m: F_r(m) = sum_l b_l a_lm lambda_lm(z_r)
    Fr = np.zeros((len(start), lmax + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        if not a_full[m].any():
            continue                                            # F_r(m) = 0
        lam = legendre_lambda(lmax, m, z[sel], st[sel])        # [l, ring]
        Fr[sel, m] = (b * a_full[m]) @ lam
    out = np.zeros(npix(nside))
    ms = np.arange(lmax + 1, dtype=np.int64)
    for r in sel:
        n = int(count[r])
        j2s = 2 * np.arange(n, dtype=np.int64) + shift[r]      # phi_j = pi j2s / n
        k = (ms[None, :] * j2s[:, None]) % (2 * n)
        ang = np.pi * k.astype(np.float64) / n
        terms = (Fr[r][None, :] * (np.cos(ang) + 1j * np.sin(ang))).real
        out[start[r]:start[r] + n] = terms[:, 0] + 2.0 * terms[:, 1:].sum(axis=1)
    return out


def map_moments(q: np.ndarray):
    """(mean, m2, m4, s2, var_s2) of one map: central sample moments with
    exactly rounded sums (math.fsum), s2 = m2 and eq. (13) with mu_k = m_k."""
    q = np.asarray(q, dtype=np.float64)
    N = q.size
    mean = math.fsum(q) / N
    d = q - mean
    m2 = math.fsum(d * d) / N
    m4 = math.fsum((d * d) * (d * d)) / N
    var_s2 = (N - 1) ** 2 / N ** 3 * m4 - (N - 1) * (N - 3) / N ** 3 * m2 * m2
    return mean, m2, m4, m2, var_s2
