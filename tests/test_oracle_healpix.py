"""Pins for the oracle's HEALPix RING pixelisation (section 2.4: 12*Nside^2 pixels).

Independent checks: pixel-centre round trips, a brute force through the HEALPix
projection that never uses the floor formulas, equal-area counts, symmetries
and hand-derived boundary cases.
"""

import json
import math
import os
import random

import numpy as np
import pytest

from oracle import binning as bn
from oracle import healpix as hp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(z, phi):
    st = math.sqrt(max(0.0, 1.0 - z * z))
    return st * math.cos(phi), st * math.sin(phi), z


def test_npix_matches_paper():
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))
    for nside, n in facts["npix"]["values"].items():
        assert hp.npix(int(nside)) == n


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 5, 8, 16])
def test_ring_layout(nside):
    # rings 1..4N-1, 4i pixels in the caps and 4N in the belt, in pixel order
    seen = []
    for p in range(hp.npix(nside)):
        i, j, nr = hp.ring_of_pixel(nside, p)
        assert 0 <= j < nr
        assert nr == 4 * min(i, nside, 4 * nside - i)
        seen.append((i, j))
    assert seen == sorted(seen)
    assert len(set(seen)) == hp.npix(nside)


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 7, 8, 16])
def test_round_trip_all_pixels(nside):
    for p in range(hp.npix(nside)):
        v = hp.centre_vector(nside, p)
        assert hp.ang2pix_ring(nside, *v) == p
        f = bn.fast_ring_pixel(nside, *v)
        assert f is None or f == p


@pytest.mark.parametrize("nside", [64, 1024, 2048, 8192])
def test_round_trip_sampled(nside):
    rng = random.Random(nside)
    decided = 0
    for _ in range(300):
        p = rng.randrange(hp.npix(nside))
        v = hp.centre_vector(nside, p)
        f = bn.fast_ring_pixel(nside, *v)   # ring N and 3N centres sit on |z| = 2/3 and defer
        assert f is None or f == p
        decided += f is not None
    assert decided > 250
    for _ in range(40):
        p = rng.randrange(hp.npix(nside))
        assert hp.ang2pix_ring(nside, *hp.centre_vector(nside, p)) == p


@pytest.mark.parametrize("nside", [2, 4])
def test_projection_brute_force(nside):
    cent = [hp.project(float(zc), pc) for zc, pc in (hp.pix2ang_ring(nside, p) for p in range(hp.npix(nside)))]
    rng = random.Random(7 + nside)
    for _ in range(1500):
        z = rng.uniform(-1.0, 1.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        p, inside = hp.brute_force_pixel(nside, z, phi, cent)
        assert inside
        v = _unit(z, phi)
        assert hp.ang2pix_ring(nside, *v) == p
        f = bn.fast_ring_pixel(nside, *v)
        assert f is None or f == p


def test_equal_area():
    # uniform directions -> multinomial(1/Npix) counts; chi^2 within 5 sigma of its dof
    nside = 4
    n = 1_500_000
    rng = np.random.default_rng(3)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    v *= 10.0
    counts, st = bn.bin_shells(v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(), (0, 0, 0), 1.0, 0,
                               [5.0, 20.0], nside)
    assert st["instances"] == n
    c = counts[0].astype(np.float64)
    exp = n / hp.npix(nside)
    chi2 = float(((c - exp) ** 2 / exp).sum())
    dof = hp.npix(nside) - 1
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof), chi2


@pytest.mark.parametrize("nside", [1, 3, 4, 16])
def test_symmetries(nside):
    rng = random.Random(11)
    N = nside
    for _ in range(300):
        z = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * math.pi)
        p = hp.ang2pix_ring(N, *_unit(z, phi))
        i, j, nr = hp.ring_of_pixel(N, p)
        # z -> -z mirrors ring i to 4N - i with the same in-ring index
        pm = hp.ang2pix_ring(N, *_unit(-z, phi))
        im, jm, nrm = hp.ring_of_pixel(N, pm)
        assert im == 4 * N - i and jm == j
        # phi -> phi + pi/2 shifts the in-ring index by a quarter ring
        phi2 = phi + math.pi / 2
        if phi2 >= 2 * math.pi:
            phi2 -= 2 * math.pi
        p2 = hp.ang2pix_ring(N, *_unit(z, phi2))
        i2, j2, _ = hp.ring_of_pixel(N, p2)
        assert i2 == i and j2 == (j + nr // 4) % nr


def test_hand_derived_boundary_points():
    # d = (2,2,1): |d| = 3, z = 1/3, tt = 1/2.  Nside 4: A = 3, B = 5 exactly ->
    # jp = 3, jm = 5, k = 3, s = 0, q = floor(5/2) = 2, pix = 2*4*3 + 16*2 + 2 = 58.
    assert hp.ang2pix_ring(4, 2.0, 2.0, 1.0) == 58
    # the same direction lies on the edge of pixels 57 and 58 (centres at phi = 3pi/16, 5pi/16)
    assert {hp.ang2pix_ring(4, 2.0, 2.0 + 1e-9, 1.0), hp.ang2pix_ring(4, 2.0 + 1e-9, 2.0, 1.0)} == {57, 58}
    # poles and axes
    assert hp.ang2pix_ring(8, 0.0, 0.0, 1.0) == 0
    assert hp.ang2pix_ring(8, 0.0, 0.0, -1.0) == hp.npix(8) - 4
    assert hp.ang2pix_ring(8, 0.0, 0.0, 0.0) == 0
    # +x axis on the equator: ring 2N, tt = 0; ring 2N has offset 1/2 when N even -> A = B = N/2,
    # so for N = 8: jp = jm = 4, k = 9, s = 0, q = floor((8 - 8 + 1)/2) = 0
    assert hp.ang2pix_ring(8, 1.0, 0.0, 0.0) == 2 * 8 * 7 + 4 * 8 * 8 + 0
    # z = 2/3 exactly (d = (1, 2, 2)/... -> (sqrt5 cos, ...)): use d = (2, 1, 2): |d| = 3, z = 2/3
    # belongs to the belt: tt = 2 atan(1/2)/pi, A = N(1/2 + tt) - N/2 = N tt
    N = 4
    tt = 2 * math.atan2(1.0, 2.0) / math.pi
    jp = math.floor(N * tt)
    jm = math.floor(N * tt + N)
    k = N + 1 + jp - jm
    assert k == 1
    assert hp.ang2pix_ring(N, 2.0, 1.0, 2.0) == 2 * N * (N - 1) + ((jp + jm - N + 0 + 1) // 2) % (4 * N)


def _adversarial_vectors():
    vs = []
    for a in range(-3, 4):
        for b in range(-3, 4):
            for c in range(-3, 4):
                vs.append((float(a), float(b), float(c)))
    rng = random.Random(5)
    for _ in range(150):
        # points on pixel-boundary families perturbed by a few ulp
        z = rng.choice([2.0 / 3.0, -2.0 / 3.0, 1.0 / 3.0, 0.0, 0.5, 0.9])
        phi = rng.choice([0.0, math.pi / 4, math.pi / 2, math.pi, 3 * math.pi / 2, math.pi / 16])
        x, y, zz = _unit(z, phi)
        for k in range(-3, 4):
            vs.append((x, y, zz + k * 2.2e-16))
            vs.append((math.nextafter(x, math.inf) if k > 0 else x, y, zz))
    return vs


@pytest.mark.parametrize("nside", [1, 2, 4, 5, 16, 64])
def test_fast_path_agrees_or_defers(nside):
    deferred = 0
    for v in _adversarial_vectors():
        f = bn.fast_ring_pixel(nside, *v)
        if f is None:
            deferred += 1
            continue
        assert f == hp.ang2pix_ring(nside, *v), v
    assert deferred > 0  # the guard band does fire on boundary points
