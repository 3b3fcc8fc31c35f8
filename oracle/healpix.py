"""Oracle (test infrastructure only): exact HEALPix RING pixelisation.

The paper pixelises each shell with HEALPix, 12*Nside^2 pixels (section 2.4);
pixel numbering is the RING scheme of Gorski et al. 2005 (ApJ 622, 759).

Everything here is exact or certified:
  * comparisons that involve only the (rational) FP64 coordinates and square
    roots of rationals are decided with Python Fractions;
  * the azimuth enters through tt = 2 phi / pi.  For the eight directions with
    dx = 0, dy = 0 or |dx| = |dy| it is an exact multiple of 1/2.  For every
    other direction phi/pi is transcendental (Niven, Gelfond-Schneider), so no
    floor argument that contains tt can be an exact integer; those floors are
    evaluated with mpmath at rising precision until the value is provably
    farther from an integer than the evaluation error.

Conventions (readings where the definition is silent):
  * boundary points follow floor(), i.e. every floor argument uses [k, k+1);
  * |z| = 2/3 exactly belongs to the equatorial formula;
  * phi = 0 when dx = dy = 0; the zero vector maps to pixel 0.
"""

from __future__ import annotations

import math
from fractions import Fraction as F

import mpmath


class Unresolved(RuntimeError):
    pass


def npix(nside: int) -> int:
    """Number of pixels, 12*Nside^2 (section 2.4)."""
    return 12 * nside * nside


def _special_tt(dx: float, dy: float):
    """tt = 2 phi/pi as an exact Fraction for the axis/diagonal directions, else None."""
    if dy == 0.0:
        return F(2) if dx < 0.0 else F(0)      # includes dx == dy == 0 (phi := 0)
    if dx == 0.0:
        return F(1) if dy > 0.0 else F(3)
    if dx == dy:
        return F(1, 2) if dx > 0.0 else F(5, 2)
    if dx == -dy:
        return F(3, 2) if dx < 0.0 else F(7, 2)
    return None


def _sign_a_minus_u_sqrt_s(a: F, u: F, s: F) -> int:
    """Exact sign of a - u*sqrt(s) for rationals a, u and s >= 0."""
    us_sign = 0 if (u == 0 or s == 0) else (1 if u > 0 else -1)
    if a >= 0 and us_sign <= 0:
        return 0 if (a == 0 and us_sign == 0) else 1
    if a <= 0 and us_sign >= 0:
        return -1
    lhs, rhs = a * a, u * u * s
    if a > 0:  # both positive
        return (lhs > rhs) - (lhs < rhs)
    return (rhs > lhs) - (rhs < lhs)  # both negative


def _certified_floor(fn):
    """floor(fn()) where fn evaluates a non-integer real with mpmath at the current precision."""
    for prec in (160, 320, 640, 1280, 2560):
        with mpmath.workprec(prec):
            v = fn()
            fl = mpmath.floor(v)
            dist = min(v - fl, fl + 1 - v)
            if dist > mpmath.mpf(2) ** (40 - prec) * max(1, abs(v)):
                return int(fl)
    raise Unresolved("floor argument not separated from an integer at 2560 bits")


def _mp_tt(dx: float, dy: float):
    phi = mpmath.atan2(mpmath.mpf(dy), mpmath.mpf(dx))
    if phi < 0:
        phi += 2 * mpmath.pi
    return 2 * phi / mpmath.pi


def _mp_z(dx, dy, dz):
    r = mpmath.sqrt(mpmath.mpf(dx) ** 2 + mpmath.mpf(dy) ** 2 + mpmath.mpf(dz) ** 2)
    return mpmath.mpf(dz) / r


def _floor_c_plus_kz(c: F, k: F, Z: F, r2: F) -> int:
    """Exact floor(c + k * Z / sqrt(r2)) for rationals c, k, Z and r2 > 0."""
    approx = float(c) + float(k) * float(Z) / math.sqrt(float(r2))
    m = math.floor(approx)

    def ge(t):  # c + k Z / sqrt(r2) >= t  <=>  k Z - (t - c) sqrt(r2) >= 0
        return _sign_a_minus_u_sqrt_s(k * Z, t - c, r2) >= 0

    while not ge(F(m)):
        m -= 1
    while ge(F(m + 1)):
        m += 1
    return m


def _floor_h_sigma(h: F, N: int, Zabs: F, r2: F) -> int:
    """Exact floor(h * sigma), sigma = N sqrt(3 (1 - |Z|/sqrt(r2))), h > 0."""
    approx = float(h) * N * math.sqrt(max(0.0, 3.0 * (1.0 - float(Zabs) / math.sqrt(float(r2)))))
    m = max(0, math.floor(approx))

    def ge(t: int) -> bool:  # h sigma >= t  (t >= 0)
        if t <= 0:
            return True
        c = 1 - F(t * t) / (3 * h * h * N * N)   # |Z|/sqrt(r2) <= c
        if c < 0:
            return False
        return _sign_a_minus_u_sqrt_s(Zabs, c, r2) <= 0

    while m > 0 and not ge(m):
        m -= 1
    while ge(m + 1):
        m += 1
    return m


def ang2pix_ring(nside: int, dx: float, dy: float, dz: float) -> int:
    """Exact RING pixel of the direction of the FP64 vector (dx, dy, dz)."""
    N = int(nside)
    X, Y, Z = F(dx), F(dy), F(dz)
    rho2 = X * X + Y * Y
    r2 = rho2 + Z * Z
    if r2 == 0:
        return 0
    tts = _special_tt(dx, dy)
    if 9 * Z * Z <= 4 * r2:                                   # |z| <= 2/3
        if tts is not None:
            c = N * (F(1, 2) + tts)
            jp = _floor_c_plus_kz(c, F(-3 * N, 4), Z, r2)
            jm = _floor_c_plus_kz(c, F(3 * N, 4), Z, r2)
        else:
            jp = _certified_floor(lambda: N * (mpmath.mpf(0.5) + _mp_tt(dx, dy)) - 0.75 * N * _mp_z(dx, dy, dz))
            jm = _certified_floor(lambda: N * (mpmath.mpf(0.5) + _mp_tt(dx, dy)) + 0.75 * N * _mp_z(dx, dy, dz))
        k = N + 1 + jp - jm
        s = 1 if k % 2 == 0 else 0
        q = ((jp + jm - N + s + 1) // 2) % (4 * N)
        return 2 * N * (N - 1) + 4 * N * (k - 1) + q

    Zabs = abs(Z)
    if tts is not None:
        u = tts - math.floor(tts)
        jp = 0 if u == 0 else _floor_h_sigma(u, N, Zabs, r2)
        jm = _floor_h_sigma(1 - u, N, Zabs, r2)
        k = jp + jm + 1
        q = math.floor(tts * k) % (4 * k)
    else:
        ftt = _certified_floor(lambda: _mp_tt(dx, dy))

        def sig():
            za = abs(_mp_z(dx, dy, dz))
            return N * mpmath.sqrt(3 * (1 - za))

        jp = _certified_floor(lambda: (_mp_tt(dx, dy) - ftt) * sig())
        jm = _certified_floor(lambda: (1 - (_mp_tt(dx, dy) - ftt)) * sig())
        k = jp + jm + 1
        q = _certified_floor(lambda: _mp_tt(dx, dy) * k) % (4 * k)
    if Z > 0:
        return 2 * k * (k - 1) + q
    return 12 * N * N - 2 * k * (k + 1) + q


# ---------------------------------------------------------------------------
# Pixel centres (pix2ang), for round trips and the projection brute force.
# Ring i = 1 .. 4N-1 counted from the north pole:
#   i < N      : 4i pixels,  z = 1 - i^2/(3N^2),   phi = (pi/(2i)) (j + 1/2)
#   N <= i <= 3N: 4N pixels, z = 4/3 - 2i/(3N),     phi = (pi/(2N)) (j + o), o = 1/2 if i-N even else 0
#   i > 3N     : mirror of ring 4N - i.
# ---------------------------------------------------------------------------

def ring_of_pixel(nside: int, p: int):
    """(ring i, index j within the ring, number of pixels in the ring)."""
    N = nside
    ncap = 2 * N * (N - 1)
    if p < ncap:
        i = int((math.isqrt(2 * p + 1) + 1) // 2)
        while 2 * i * (i - 1) > p:
            i -= 1
        while 2 * (i + 1) * i <= p:
            i += 1
        return i, p - 2 * i * (i - 1), 4 * i
    if p < 12 * N * N - ncap:
        off = p - ncap
        return N + off // (4 * N), off % (4 * N), 4 * N
    pr = 12 * N * N - 1 - p                     # counted back from the last pixel
    ip = int((math.isqrt(2 * pr + 1) + 1) // 2)
    while 2 * ip * (ip - 1) > pr:
        ip -= 1
    while 2 * (ip + 1) * ip <= pr:
        ip += 1
    j = 4 * ip - 1 - (pr - 2 * ip * (ip - 1))
    return 4 * N - ip, j, 4 * ip


def pix2ang_ring(nside: int, p: int):
    """Centre of pixel p as (z as Fraction, phi as float)."""
    N = nside
    i, j, nr = ring_of_pixel(nside, p)
    if i < N:
        return 1 - F(i * i, 3 * N * N), math.pi / (2 * i) * (j + 0.5)
    if i <= 3 * N:
        o = 0.5 if (i - N) % 2 == 0 else 0.0
        return F(4, 3) - F(2 * i, 3 * N), math.pi / (2 * N) * (j + o)
    ii = 4 * N - i
    return -(1 - F(ii * ii, 3 * N * N)), math.pi / (2 * ii) * (j + 0.5)


def centre_vector(nside: int, p: int):
    z, phi = pix2ang_ring(nside, p)
    zf = float(z)
    st = math.sqrt(max(0.0, 1.0 - zf * zf))
    return st * math.cos(phi), st * math.sin(phi), zf


# ---------------------------------------------------------------------------
# Independent brute force via the HEALPix projection (Calabretta & Roukema 2007):
# equatorial: x = phi, y = (3 pi / 8) z;  polar: sigma = sqrt(3 (1 - |z|)),
# phi_c = (floor(2 phi / pi) + 1/2) pi / 2, x = phi_c + (phi - phi_c) sigma,
# y = +-(pi/4)(2 - sigma).  Pixels are diamonds |dx| + |dy| < pi/(4N) around the
# projected centres (x periodic in 2 pi).
# ---------------------------------------------------------------------------

def project(z: float, phi: float):
    if abs(z) <= 2.0 / 3.0:
        return phi, 3.0 * math.pi / 8.0 * z
    sigma = math.sqrt(3.0 * (1.0 - abs(z)))
    phic = (math.floor(2.0 * phi / math.pi) + 0.5) * math.pi / 2.0
    x = phic + (phi - phic) * sigma
    y = math.copysign(math.pi / 4.0 * (2.0 - sigma), z)
    return x, y


def brute_force_pixel(nside: int, z: float, phi: float, centres=None):
    """Pixel whose projected diamond contains (z, phi), by scanning every pixel."""
    if centres is None:
        centres = [project(float(zc), pc) for zc, pc in (pix2ang_ring(nside, p) for p in range(npix(nside)))]
    x, y = project(z, phi)
    half = math.pi / (4 * nside)
    best, best_d = -1, 1e300
    for p, (xc, yc) in enumerate(centres):
        ddx = abs(x - xc) % (2 * math.pi)
        ddx = min(ddx, 2 * math.pi - ddx)
        d = ddx + abs(y - yc)
        if d < best_d:
            best, best_d = p, d
    return best, best_d < half
