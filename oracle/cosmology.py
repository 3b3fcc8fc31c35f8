"""Oracle (test infrastructure only): distances, Born lensing weights, nbar, kappa and gradients.

Paper passages followed (section 2.3):
  * eq. (1): continuous Born convergence with prefactor (3/2) Omega_m, 1/E(z),
    D(z) D(z, z_s) / D(z_s) and 1/a = 1 + z;
  * dimensionless comoving distance D(z) = (H0/c) chi(z);
  * eq. (3): delta-source weight of a shell; eqs. (4)-(6): the shell sum in
    terms of counts n_p, pixel area 4 pi chi^2 / N_pix and mean density
    N_part / V_sim; eq. (7) is the overdensity analogue.

Readings (the paper is silent or loose; listed in the design notes):
  * flat LambdaCDM without radiation: E(z) = sqrt(Om (1+z)^3 + 1 - Om),
    D(z, z_s) = D(z_s) - D(z);
  * eq. (6) equals sum_b W_b (n_b/nbar_b - 1) with
        W_b = (3/2) Om * int_{z_b}^{min(z_{b+1}, z_s)} dz (1+z) D (D_s - D) / (D_s E)
    (the numerator of eq. (3) times (3/2) Om; lenses behind the source give 0);
  * a source distribution n(z) on [0, z_max] replaces (D_s - D)/D_s by
    int_z^{z_max} dz' nhat(z') (1 - D(z)/D(z')), nhat = n / int_0^{z_max} n;
    the Smail form n ~ z^alpha exp(-(z/z0)^beta);
  * nbar_b = (N/L^3) (4 pi/3)(chi_{b+1}^3 - chi_b^3) / N_pix (exact shell volume;
    eq. (6) literally uses chi_b^2 Delta chi_b at the lower edge, kept as
    mode "lower_edge").
Everything is FP64 with adaptive quadrature (scipy.integrate.quad) at
relative tolerance ~1e-13.  Derivatives use Richardson-extrapolated central
differences of these functions, independent of any forward-mode code.
"""

from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy import integrate, optimize

C_OVER_H0 = 2997.92458  # c/H0 in Mpc/h  (c = 299792.458 km/s, H0 = 100 h km/s/Mpc)

_QK = dict(epsabs=0.0, epsrel=1e-13, limit=200)


def E(z, om):
    return math.sqrt(om * (1.0 + z) ** 3 + 1.0 - om)


@lru_cache(maxsize=1 << 18)
def D(z, om):
    """Dimensionless comoving distance int_0^z dz'/E(z')."""
    if z == 0.0:
        return 0.0
    return integrate.quad(lambda t: 1.0 / E(t, om), 0.0, z, **_QK)[0]


def chi(z, om):
    return C_OVER_H0 * D(z, om)


def z_of_D(Dt, om):
    if Dt == 0.0:
        return 0.0
    return optimize.brentq(lambda z: D(z, om) - Dt, 0.0, 50.0, xtol=1e-15, rtol=8.9e-16, maxiter=200)


def z_of_chi(c, om):
    return z_of_D(c / C_OVER_H0, om)


# ---------------------------------------------------------------- source models

class DeltaSource:
    def __init__(self, zs):
        self.zs = float(zs)


class FunctionSource:
    """A source distribution given by an unnormalised density n(z) on [0, z_max]."""

    def __init__(self, n, z_max):
        self._n = n
        self.z_max = float(z_max)

    def n(self, z):
        return self._n(z)

    def norm(self):
        return integrate.quad(self.n, 0.0, self.z_max, **_QK)[0]


class SmailSource(FunctionSource):
    """n(z) ~ z^alpha exp(-(z/z0)^beta) on [0, z_max]."""

    def __init__(self, alpha, beta, z0, z_max):
        self.alpha, self.beta, self.z0, self.z_max = float(alpha), float(beta), float(z0), float(z_max)

    def n(self, z):
        if z <= 0.0:
            return 0.0
        return z ** self.alpha * math.exp(-((z / self.z0) ** self.beta))


# ---------------------------------------------------------------- weights

def weight_delta(z_lo, z_hi, zs, om):
    """W_b for a single source plane at zs (section 2.3 eqs. (3), (6))."""
    if z_lo >= zs:
        return 0.0
    Ds = D(zs, om)
    hi = min(z_hi, zs)
    f = lambda z: (1.0 + z) * D(z, om) * (Ds - D(z, om)) / (Ds * E(z, om))
    return 1.5 * om * integrate.quad(f, z_lo, hi, **_QK)[0]


def weight_nz(z_lo, z_hi, src: FunctionSource, om):
    """W_b for a source distribution (section 2.4 names n(z); the form is a reading)."""
    norm = src.norm()
    zmax = src.z_max

    def inner(z):
        if z >= zmax:
            return 0.0
        Dz = D(z, om)
        g = lambda zp: src.n(zp) * (1.0 - Dz / D(zp, om))
        return integrate.quad(g, z, zmax, **_QK)[0] / norm

    f = lambda z: (1.0 + z) * D(z, om) / E(z, om) * inner(z)
    hi = min(z_hi, zmax)
    if z_lo >= hi:
        return 0.0
    return 1.5 * om * integrate.quad(f, z_lo, hi, **_QK)[0]


def shell_z_edges(chi_edges, om):
    """Redshifts of frozen comoving edges at cosmology om (chi = (c/H0) D(z))."""
    return [z_of_chi(float(c), om) for c in chi_edges]


def lensing_weights(chi_edges, om, source):
    """W_b for every shell [chi_b, chi_{b+1}); chi edges stay fixed when om changes."""
    ze = shell_z_edges(chi_edges, om)
    out = []
    for b in range(len(ze) - 1):
        if isinstance(source, DeltaSource):
            out.append(weight_delta(ze[b], ze[b + 1], source.zs, om))
        else:
            out.append(weight_nz(ze[b], ze[b + 1], source, om))
    return np.array(out)


def weight_derivative(chi_edges, om, source, param, h=None):
    """dW_b/dparam by Richardson-extrapolated central differences.

    param in {"omega_m", "zs", "alpha", "beta", "z0"}.
    """
    base = {"omega_m": om}
    if isinstance(source, DeltaSource):
        base["zs"] = source.zs
    else:
        base.update(alpha=source.alpha, beta=source.beta, z0=source.z0)
    x0 = base[param]
    if h is None:
        h = 1e-3 * max(1.0, abs(x0))

    def W_at(v):
        p = dict(base)
        p[param] = v
        if isinstance(source, DeltaSource):
            s = DeltaSource(p["zs"])
        else:
            s = SmailSource(p["alpha"], p["beta"], p["z0"], source.z_max)
        return lensing_weights(chi_edges, p["omega_m"], s)

    d1 = (W_at(x0 + h) - W_at(x0 - h)) / (2 * h)
    d2 = (W_at(x0 + h / 2) - W_at(x0 - h / 2)) / h
    return (4.0 * d2 - d1) / 3.0


# ---------------------------------------------------------------- nbar, kappa, adjoint

def nbar(n_src, box_L, chi_edges, nside, mode="exact_volume"):
    """Mean count per pixel of each shell: (N / L^3) * shell volume / N_pix."""
    e = np.asarray(chi_edges, dtype=np.float64)
    npx = 12 * nside * nside
    dens = n_src / float(box_L) ** 3
    if mode == "exact_volume":
        vol = 4.0 * math.pi / 3.0 * (e[1:] ** 3 - e[:-1] ** 3)
    elif mode == "lower_edge":
        vol = 4.0 * math.pi * e[:-1] ** 2 * (e[1:] - e[:-1])
    else:
        raise ValueError(mode)
    return dens * vol / npx


def kappa(counts, W, nb):
    """kappa_t[p] = sum_b W[t,b] (n_b[p]/nbar_b - 1), FP64, shells summed in order (eq. (6))."""
    counts = np.asarray(counts)
    W = np.atleast_2d(np.asarray(W, dtype=np.float64))
    out = np.zeros((W.shape[0], counts.shape[1]), dtype=np.float64)
    for t in range(W.shape[0]):
        for b in range(counts.shape[0]):
            out[t] += W[t, b] * (counts[b].astype(np.float64) / nb[b] - 1.0)
    return out


def overdensity(counts, chi_edges, nb):
    """delta[p] = sum_b Delta chi_b (n_b/nbar_b - 1) / sum_b Delta chi_b (eq. (7))."""
    e = np.asarray(chi_edges, dtype=np.float64)
    dchi = e[1:] - e[:-1]
    return kappa(counts, dchi[None, :] / dchi.sum(), nb)[0]


def grad_W(counts, nb, grad_kappa, summation="exact"):
    """dL/dW[t,b] = sum_p g_t[p] (n_b[p]/nbar_b - 1) for a loss L with dL/dkappa = g.

    summation="exact": math.fsum (correctly rounded); "pairwise": numpy's pairwise
    sum, relative error of order log2(N_pix) ulp of sum |terms| -- for maps too
    large for fsum to finish in seconds."""
    counts = np.asarray(counts)
    g = np.atleast_2d(np.asarray(grad_kappa, dtype=np.float64))
    out = np.zeros((g.shape[0], counts.shape[0]))
    for t in range(g.shape[0]):
        for b in range(counts.shape[0]):
            terms = g[t] * (counts[b].astype(np.float64) / nb[b] - 1.0)
            if summation == "exact":
                out[t, b] = math.fsum(terms)
            elif summation == "pairwise":
                out[t, b] = float(np.sum(terms))
            else:
                raise ValueError(summation)
    return out
