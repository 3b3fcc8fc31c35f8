"""Pins for the oracle's distances, lensing weights, nbar, kappa and adjoint
(section 2.3 eqs. (1)-(7); the Smail n(z) is a reading)."""

import json
import math
import os

import mpmath
import numpy as np
import pytest

import synth
from oracle import binning as bn
from oracle import cosmology as co

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _D_hyp2f1(z, om):
    # int_1^{1+z} dx / sqrt(L + om x^3) with int_0^X dx/sqrt(1 + a x^3) = X 2F1(1/3,1/2;4/3;-a X^3)
    lam = 1.0 - om
    a = om / lam
    G = lambda X: X * mpmath.hyp2f1(mpmath.mpf(1) / 3, mpmath.mpf(1) / 2, mpmath.mpf(4) / 3, -a * X ** 3)
    with mpmath.workdps(30):
        return float((G(mpmath.mpf(1) + z) - G(mpmath.mpf(1))) / mpmath.sqrt(lam))


@pytest.mark.parametrize("z", [0.05, 0.3, 1.0, 1.5, 3.0])
def test_distance_closed_forms(z):
    assert co.D(z, 1.0) == pytest.approx(2.0 * (1.0 - 1.0 / math.sqrt(1.0 + z)), rel=1e-13)
    assert co.D(z, 0.0) == pytest.approx(z, rel=1e-13)
    assert co.D(z, 0.3) == pytest.approx(_D_hyp2f1(z, 0.3), rel=1e-12)
    assert co.z_of_D(co.D(z, 0.3), 0.3) == pytest.approx(z, rel=1e-13)


def _W_eds_closed(D_lo, D_hi, Ds):
    # Om = 1: 1 + z = v^-2 with v = 1 - D/2; integrand v^-2 D (Ds - D)/Ds in D has primitive
    # F(D) = -4 [ -(Ds - 2)/v + (4 - Ds) ln v - 2 v ],  W = (3/2) [F(D_hi) - F(D_lo)] / Ds
    def F(u):
        v = 1.0 - u / 2.0
        return -4.0 * (-(Ds - 2.0) / v + (4.0 - Ds) * math.log(v) - 2.0 * v)
    return 1.5 * (F(D_hi) - F(D_lo)) / Ds


def test_delta_weight_eds_closed_form():
    zs = 1.2
    Ds = co.D(zs, 1.0)
    edges_z = [0.1, 0.25, 0.4, 0.8, 1.2]
    chi = [co.chi(z, 1.0) for z in edges_z]
    W = co.lensing_weights(chi, 1.0, co.DeltaSource(zs))
    for b in range(len(edges_z) - 1):
        want = _W_eds_closed(co.D(edges_z[b], 1.0), co.D(edges_z[b + 1], 1.0), Ds)
        assert W[b] == pytest.approx(want, rel=1e-11)


def test_delta_weight_zero_behind_source_and_clipped():
    chi = [co.chi(z, 0.3) for z in (0.1, 0.2, 0.3, 0.4)]
    W = co.lensing_weights(chi, 0.3, co.DeltaSource(0.25))
    assert W[0] > 0 and W[1] > 0 and W[2] == 0.0
    # shell [0.2, 0.3) is clipped at the source: equals the weight of [0.2, 0.25)
    assert W[1] == pytest.approx(co.weight_delta(0.2, 0.25, 0.25, 0.3), rel=1e-13)


def test_delta_weight_derivative_eds_zs():
    # d/dzs of the closed form by complex step of the analytic expression in Ds(zs)
    import cmath
    e_z = [0.2, 0.5, 0.9]
    D_lo = [co.D(z, 1.0) for z in e_z]

    def Wc(zs):
        Ds = 2.0 * (1.0 - 1.0 / cmath.sqrt(1.0 + zs))

        def F(u):
            v = 1.0 - u / 2.0
            return -4.0 * (-(Ds - 2.0) / v + (4.0 - Ds) * cmath.log(v) - 2.0 * v)
        return [1.5 * (F(D_lo[b + 1]) - F(D_lo[b])) / Ds for b in range(2)]

    h = 1e-30
    want = [w.imag / h for w in Wc(1.3 + 1j * h)]
    chi = [co.chi(z, 1.0) for z in e_z]
    got = co.weight_derivative(chi, 1.0, co.DeltaSource(1.3), "zs")
    assert np.allclose(got, want, rtol=1e-7)


def test_smail_normalisation_closed_form():
    a, b, z0 = 2.0, 1.5, 0.3
    src = co.SmailSource(a, b, z0, 50.0)
    want = z0 ** (a + 1) * math.gamma((a + 1) / b) / b
    assert src.norm() == pytest.approx(want, rel=1e-12)


def test_nz_weight_linear_in_the_distribution():
    om = 0.3
    chi = [co.chi(z, om) for z in (0.1, 0.3, 0.5, 0.7)]
    n1 = lambda z: math.exp(-((z - 0.45) / 0.1) ** 2)
    n2 = lambda z: z * z * math.exp(-z / 0.2)
    s1, s2 = co.FunctionSource(n1, 1.0), co.FunctionSource(n2, 1.0)
    s12 = co.FunctionSource(lambda z: n1(z) + n2(z), 1.0)
    N1, N2 = s1.norm(), s2.norm()
    W1, W2, W12 = (co.lensing_weights(chi, om, s) for s in (s1, s2, s12))
    assert np.allclose(W12, (N1 * W1 + N2 * W2) / (N1 + N2), rtol=1e-10)


def test_narrow_nz_tends_to_delta():
    om = 0.3
    # shells in front of the source: the smoothed kernel differs at O(width^2)
    chi = [co.chi(z, om) for z in (0.1, 0.3, 0.5, 0.58)]
    zc, w = 0.6, 2e-3
    src = co.FunctionSource(lambda z: math.exp(-0.5 * ((z - zc) / w) ** 2), 1.0)
    Wn = co.lensing_weights(chi, om, src)
    Wd = co.lensing_weights(chi, om, co.DeltaSource(zc))
    assert np.allclose(Wn, Wd, rtol=1e-4)


def test_delta_sum_rule_matches_continuous_born_kernel():
    # the shell weights of a source at zs add up to the continuous integral of eq. (1) for delta = 1
    om, zs = 0.3, 0.8
    chi = [co.chi(z, om) for z in np.linspace(0.0, 0.8, 9)]
    W = co.lensing_weights(chi, om, co.DeltaSource(zs))
    Ds = co.D(zs, om)
    full = 1.5 * om * mpmath.quad(lambda z: (1 + z) * co.D(float(z), om) * (Ds - co.D(float(z), om))
                                  / (Ds * co.E(float(z), om)), [0, 0.4, 0.8])
    assert W.sum() == pytest.approx(float(full), rel=1e-10)


def test_table1_particle_mass_reading():
    # mean density rho = m_p N / V (eq. (5)) with N = 1024^3 reproduces Table 1's mass resolution
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["simulation_setup"]
    rho_crit = 2.775e11  # h^2 M_sun / Mpc^3 -> h^-1 M_sun / (h^-1 Mpc)^3
    for box in facts["boxes"]:
        mp = facts["omega_m"] * rho_crit * box["L"] ** 3 / box["n_part_1d"] ** 3
        assert mp == pytest.approx(box["mass_resolution"], rel=0.03)


def test_nbar_unbiased_for_uniform_particles():
    # exact-volume nbar: mean over pixels of (n_b/nbar_b - 1) is 0 within Poisson noise;
    # the lower-edge form of eq. (6) is biased by O(Delta chi / chi)
    L, N, nside = 200.0, 400000, 4
    x, y, z = synth.uniform_box(N, L, seed=9)
    edges = [20.0, 40.0, 60.0, 90.0]
    counts, _ = bn.bin_shells(x, y, z, (100.0, 100.0, 100.0), L, 0, edges, nside)
    nb = co.nbar(N, L, edges, nside)
    ratio = counts.mean(axis=1) / nb
    tot = counts.sum(axis=1)
    assert np.all(np.abs(ratio - 1.0) < 5.0 / np.sqrt(tot))
    nb_low = co.nbar(N, L, edges, nside, mode="lower_edge")
    assert np.all(counts.mean(axis=1) / nb_low - 1.0 > 0.2)


def test_kappa_single_particle_and_linearity():
    B, npx = 3, 12
    W = np.array([[1e-4, 2e-4, 3e-4], [5e-5, 0.0, 7e-5]])
    nb = np.array([0.5, 2.0, 4.0])
    counts = np.zeros((B, npx), dtype=np.int64)
    counts[1, 5] = 1
    k = co.kappa(counts, W, nb)
    for t in range(2):
        assert k[t, 5] == pytest.approx(W[t, 1] / nb[1] - W[t].sum(), rel=1e-15)
        assert np.allclose(np.delete(k[t], 5), -W[t].sum(), rtol=1e-15)
    c2 = np.random.default_rng(0).integers(0, 9, size=(B, npx))
    lin = co.kappa(counts + c2, W, nb) + W.sum(axis=1)[:, None]
    parts = co.kappa(counts, W, nb) + co.kappa(c2, W, nb) + 2 * W.sum(axis=1)[:, None]
    assert np.allclose(lin, parts, rtol=1e-13, atol=1e-18)
    assert np.allclose(co.kappa(c2, W[1:], nb), co.kappa(c2, W, nb)[1:], rtol=0, atol=0)


def test_adjoint_is_gradient_of_quadratic_loss():
    rng = np.random.default_rng(1)
    B, npx = 4, 48
    counts = rng.integers(0, 20, size=(B, npx))
    nb = rng.uniform(3, 8, size=B)
    W = rng.uniform(1e-4, 5e-4, size=(2, B))
    kap = co.kappa(counts, W, nb)
    g = co.grad_W(counts, nb, 2.0 * kap)
    L = lambda Wm: float((co.kappa(counts, Wm, nb) ** 2).sum())
    h = 1e-7
    for t in range(2):
        for b in range(B):
            Wp, Wm = W.copy(), W.copy()
            Wp[t, b] += h
            Wm[t, b] -= h
            # L is quadratic in W: the central difference is exact up to rounding
            assert (L(Wp) - L(Wm)) / (2 * h) == pytest.approx(g[t, b], rel=1e-6)
    # dot-product test <J v, g> = <v, J^T g> for the linear map W -> kappa + sum W
    v = rng.normal(size=W.shape)
    gk = rng.normal(size=kap.shape)
    Jv = co.kappa(counts, v, nb)
    assert float((Jv * gk).sum()) == pytest.approx(float((v * co.grad_W(counts, nb, gk)).sum()), rel=1e-12)


def _dW_domega_delta_mp(chi_edges, om, zs, dps=25):
    """dW_b/dOmega_m of a delta source with frozen comoving edges, by forward
    sensitivities at 25 digits (independent of the oracle's differences).

    In the dimensionless distance D the edges D_b = chi_b H0/c do not move, so
        W_b = (3/2) Om int_{D_b}^{min(D_{b+1}, D_s)} (1 + z(D)) D (D_s - D)/D_s dD
    with dz/dD = E(z; Om).  Differentiating: y = dz/dOm at fixed D obeys
    dy/dD = (dE/dz) y + dE/dOm, y(0) = 0, and dD_s/dOm = -int_0^zs (dE/dOm)/E^2 dz;
    the moving upper limit D_s adds nothing (the integrand vanishes there)."""
    C = co.C_OVER_H0
    with mpmath.workdps(dps):
        Om = mpmath.mpf(om)
        E = lambda z: mpmath.sqrt(Om * (1 + z) ** 3 + 1 - Om)
        dEdz = lambda z: 3 * Om * (1 + z) ** 2 / (2 * E(z))
        dEdO = lambda z: ((1 + z) ** 3 - 1) / (2 * E(z))
        Ds = mpmath.quad(lambda z: 1 / E(z), [0, zs])
        dDs = -mpmath.quad(lambda z: dEdO(z) / E(z) ** 2, [0, zs])
        sol = mpmath.odefun(lambda D, v: [E(v[0]), dEdz(v[0]) * v[1] + dEdO(v[0])], 0,
                            [mpmath.mpf(0), mpmath.mpf(0)])
        W, dW = [], []
        for b in range(len(chi_edges) - 1):
            lo = mpmath.mpf(chi_edges[b]) / C
            hi = min(mpmath.mpf(chi_edges[b + 1]) / C, Ds)
            if lo >= Ds:
                W.append(0.0)
                dW.append(0.0)
                continue
            f = lambda D: (1 + sol(D)[0]) * D * (Ds - D) / Ds
            g = lambda D: sol(D)[1] * D * (Ds - D) / Ds + (1 + sol(D)[0]) * D * D / Ds ** 2 * dDs
            Wb = mpmath.fraction(3, 2) * Om * mpmath.quad(f, [lo, hi])
            W.append(float(Wb))
            dW.append(float(Wb / Om + mpmath.fraction(3, 2) * Om * mpmath.quad(g, [lo, hi])))
    return np.array(W), np.array(dW)


def test_weight_derivative_omega_m_frozen_chi_edges():
    # the Omega_m derivative with comoving edges fixed (their redshifts move):
    # against the sensitivity-equation value above, including a shell cut by the source
    chi = [co.chi(z, 0.3) for z in (0.1, 0.3, 0.5, 0.7)]
    W_mp, dW_mp = _dW_domega_delta_mp(chi, 0.3, 0.6)
    assert np.allclose(co.lensing_weights(chi, 0.3, co.DeltaSource(0.6)), W_mp, rtol=1e-12)
    got = co.weight_derivative(chi, 0.3, co.DeltaSource(0.6), "omega_m")
    assert np.allclose(got, dW_mp, rtol=1e-8)
    # the pin tells the readings apart: with the redshift edges held fixed instead,
    # the derivative is off by 8 % to 200 %
    ze = co.shell_z_edges(chi, 0.3)
    h = 1e-4
    Wz = lambda om: np.array([co.weight_delta(ze[b], ze[b + 1], 0.6, om) for b in range(3)])
    frozen_z = (Wz(0.3 + h) - Wz(0.3 - h)) / (2 * h)
    assert np.all(np.abs(frozen_z - dW_mp) > 0.05 * np.abs(dW_mp))


def test_weight_derivative_smail_z0_analytic():
    # d/dz0 of a Smail source: the z0 derivative of the normalised n(z) written out,
    # (dn nrm - n dnrm)/nrm^2 with dn/dz0 = n beta (z/z0)^beta / z0, integrated at 20
    # digits with D(z) from an ODE solution (no differences involved)
    chi = [co.chi(z, 0.3) for z in (0.1, 0.3, 0.5, 0.7)]
    C = co.C_OVER_H0
    with mpmath.workdps(20):
        Om = mpmath.mpf("0.3")
        E = lambda z: mpmath.sqrt(Om * (1 + z) ** 3 + 1 - Om)
        Dz = mpmath.odefun(lambda z, D: 1 / E(z), 0, mpmath.mpf(0))
        a, b, s, zmax = mpmath.mpf(2), mpmath.mpf("1.5"), mpmath.mpf("0.3"), mpmath.mpf(1)
        n = lambda z: z ** a * mpmath.exp(-(z / s) ** b) if z > 0 else mpmath.mpf(0)
        dn = lambda z: n(z) * b * (z / s) ** b / s
        nrm, dnrm = mpmath.quad(n, [0, zmax]), mpmath.quad(dn, [0, zmax])
        ze = [mpmath.findroot(lambda z: Dz(z) - mpmath.mpf(c) / C, 0.3) for c in chi]
        want = []
        for k in range(3):
            def dq(z):
                Dzz = Dz(z)
                return mpmath.quad(lambda zp: (dn(zp) * nrm - n(zp) * dnrm) / nrm ** 2 * (1 - Dzz / Dz(zp)),
                                   [z, zmax])
            want.append(float(mpmath.fraction(3, 2) * Om *
                              mpmath.quad(lambda z: (1 + z) * Dz(z) / E(z) * dq(z), [ze[k], ze[k + 1]])))
    got = co.weight_derivative(chi, 0.3, co.SmailSource(2.0, 1.5, 0.3, 1.0), "z0")
    assert np.allclose(got, want, rtol=1e-8)


def _eq7_literal(counts, z_edges, om, n_part, L, nside):
    """Eq. (7) evaluated as printed, term by term:
    delta = sum_b [ N_pix/(4 pi) (V/N) (H0/c)^2 n_p / D^2(z_b) - (c/H0) Delta D_b ] / sum_b (c/H0) Delta D_b,
    with D(z) by 30-digit quadrature and z_b the lower edge of shell b."""
    C = mpmath.mpf(co.C_OVER_H0)
    npx = 12 * nside * nside
    with mpmath.workdps(30):
        D = [mpmath.quad(lambda t: 1 / mpmath.sqrt(om * (1 + t) ** 3 + 1 - om), [0, z]) for z in z_edges]
        dD = [D[b + 1] - D[b] for b in range(len(D) - 1)]
        den = sum(C * d for d in dD)
        pre = [npx / (4 * mpmath.pi) * (mpmath.mpf(L) ** 3 / n_part) / C ** 2 / D[b] ** 2 for b in range(len(dD))]
        out = np.empty(counts.shape[1])
        for p in range(counts.shape[1]):
            out[p] = float(sum(pre[b] * int(counts[b, p]) - C * dD[b] for b in range(len(dD))) / den)
    return out, [float(C * d) for d in D]


def test_overdensity_is_printed_eq7():
    # the oracle's overdensity with the lower-edge nbar equals eq. (7) as printed
    om, L, N, nside = 0.3, 700.0, 250000, 4
    z_edges = [0.04, 0.07, 0.1, 0.14]
    rng = np.random.default_rng(7)
    counts = rng.integers(0, 40, size=(3, 12 * nside * nside))
    want, chi = _eq7_literal(counts, z_edges, om, N, L, nside)
    got = co.overdensity(counts, chi, co.nbar(N, L, chi, nside, mode="lower_edge"))
    tol = 1e-12 * np.abs(want).max()
    assert np.abs(got - want).max() <= tol
    # what the pin rejects: shells weighted by Delta z instead of Delta chi, or the
    # sum left without its normalisation
    dz = np.diff(z_edges)
    nb = co.nbar(N, L, chi, nside, mode="lower_edge")
    by_dz = co.kappa(counts, dz[None, :] / dz.sum(), nb)[0]
    unnormalised = co.kappa(counts, np.diff(chi)[None, :], nb)[0]
    assert np.abs(by_dz - want).max() > 1e6 * tol
    assert np.abs(unnormalised - want).max() > 1e6 * tol


def test_overdensity_single_particle_closed_form():
    # one particle in shell 1 at pixel 5 (Nside 1, 12 pixels): eq. (7) reduces to
    #   delta[5] = 3 L^3 / (pi N chi_1^2 (chi_3 - chi_0)) - 1,  delta = -1 elsewhere
    chi = [100.0, 200.0, 400.0, 450.0]
    L, N = 1000.0, 1000
    counts = np.zeros((3, 12), dtype=np.int64)
    counts[1, 5] = 1
    got = co.overdensity(counts, chi, co.nbar(N, L, chi, 1, mode="lower_edge"))
    want5 = 3.0 * L ** 3 / (math.pi * N * chi[1] ** 2 * (chi[3] - chi[0])) - 1.0
    assert got[5] == pytest.approx(want5, rel=1e-14)
    assert np.all(np.delete(got, 5) == -1.0)


def test_adjoint_pairwise_summation_matches_exact():
    rng = np.random.default_rng(3)
    counts = rng.integers(0, 50, size=(3, 200000))
    nb = np.array([4.0, 11.0, 23.0])
    g = rng.normal(size=(2, 200000))
    ex = co.grad_W(counts, nb, g)
    pw = co.grad_W(counts, nb, g, summation="pairwise")
    scale = np.abs(g).sum() * 50.0 / nb.min()
    assert np.abs(pw - ex).max() <= 1e-13 * scale
