"""GPU parity: Born convergence, overdensity, adjoint, lensing weights, distances and
gradients (section 2.3 eqs. (1)-(7)) against the oracle."""

import numpy as np
import pytest
import torch

import paper_1801_05745_amd as uf
import synth
from oracle import binning as obin
from oracle import cosmology as ocos

from workloads import OMEGA_M, chi_edges_from_z, config1

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(*ts):
    return [t.to(DEV) for t in ts]


@pytest.fixture(scope="module")
def c1():
    c = config1()
    counts, _ = obin.bin_shells(c["x"], c["y"], c["z"], (250.0,) * 3, c["L"], 0, c["edges"], c["nside"])
    c["ref_counts"] = counts
    return c


def test_comoving_distance(ufalcon):
    z = torch.tensor([0.0, 0.01, 0.1, 0.3, 0.5, 1.0, 1.5, 3.0], dtype=torch.float64, device=DEV)
    chi = uf.comoving_distance(z, OMEGA_M).cpu().numpy()
    want = np.array([ocos.chi(float(v), OMEGA_M) for v in z.cpu()])
    assert np.allclose(chi, want, rtol=1e-13, atol=1e-12)


def test_weights_delta_config1(ufalcon, c1):
    W, dW = uf.lensing_weights(OMEGA_M, [uf.SourceSpec("delta", z_s=0.3)], c1["edges"], with_derivatives=True)
    W = W.cpu().numpy()[0]
    want = ocos.lensing_weights(c1["edges"], OMEGA_M, ocos.DeltaSource(0.3))
    assert np.allclose(W, want, rtol=1e-12, atol=0)
    d_om = ocos.weight_derivative(c1["edges"], OMEGA_M, ocos.DeltaSource(0.3), "omega_m")
    d_zs = ocos.weight_derivative(c1["edges"], OMEGA_M, ocos.DeltaSource(0.3), "zs")
    dW = dW.cpu().numpy()[0]
    assert np.allclose(dW[:, 0], d_om, rtol=1e-7, atol=1e-14)
    assert np.allclose(dW[:, 1], d_zs, rtol=1e-7, atol=1e-14)


def test_weights_delta_behind_source():
    edges = chi_edges_from_z(0.1, 0.9, 8)
    W = uf.lensing_weights(OMEGA_M, [uf.SourceSpec("delta", z_s=0.45)], edges).cpu().numpy()[0]
    want = ocos.lensing_weights(edges, OMEGA_M, ocos.DeltaSource(0.45))
    assert np.allclose(W, want, rtol=1e-12, atol=1e-20)
    assert np.all(W[4:] == 0.0)


@pytest.mark.parametrize("zlo,zhi,B,z0", [(0.1, 0.5, 30, 0.3), (0.1, 1.5, 47, 0.7)])
def test_weights_smail(ufalcon, zlo, zhi, B, z0):
    edges = chi_edges_from_z(zlo, zhi, B)
    src = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=z0, z_max=zhi)
    W, dW = uf.lensing_weights(OMEGA_M, [src], edges, with_derivatives=True)
    osrc = ocos.SmailSource(2.0, 1.5, z0, zhi)
    want = ocos.lensing_weights(edges, OMEGA_M, osrc)
    W = W.cpu().numpy()[0]
    assert np.allclose(W, want, rtol=1e-11, atol=0)
    dW = dW.cpu().numpy()[0]
    for slot, name in ((0, "omega_m"), (3, "z0")):
        d = ocos.weight_derivative(edges, OMEGA_M, osrc, name)
        assert np.allclose(dW[:, slot], d, rtol=1e-6, atol=1e-9 * np.abs(d).max()), name


def test_inv_nbar_modes(ufalcon, c1):
    e = c1["edges"][1:]  # lower edge > 0 for the literal mode
    for mode, name in ((uf.NBAR_EXACT_VOLUME, "exact_volume"), (uf.NBAR_LOWER_EDGE, "lower_edge")):
        got = uf.inv_nbar(c1["n"], c1["L"], e, 64, mode=mode).cpu().numpy()
        want = 1.0 / ocos.nbar(c1["n"], c1["L"], e, 64, mode=name)
        assert np.allclose(got, want, rtol=1e-14)


def test_config1_kappa_fp64(ufalcon, c1):
    counts = torch.from_numpy(c1["ref_counts"].astype(np.uint32)).to(DEV)
    W = uf.lensing_weights(OMEGA_M, [uf.SourceSpec("delta", z_s=0.3)], c1["edges"])
    inb = uf.inv_nbar(c1["n"], c1["L"], c1["edges"], 64)
    kap = uf.born_kappa(counts, W, inb, out_dtype=torch.float64).cpu().numpy()
    Wr = ocos.lensing_weights(c1["edges"], OMEGA_M, ocos.DeltaSource(0.3))
    ref = ocos.kappa(c1["ref_counts"], Wr[None, :], ocos.nbar(c1["n"], c1["L"], c1["edges"], 64))
    rms = np.sqrt((ref ** 2).mean())
    assert np.abs(kap - ref).max() <= 1e-10 * rms


def test_kappa_fp32_tomographic_rows_and_tail(ufalcon):
    # Nside 13: npix = 2028 (two 1024-pixel blocks, ragged tail); T = 3 rows equal T = 1 runs
    rng = np.random.default_rng(2)
    B, nside = 7, 13
    counts = rng.poisson(5.0, size=(B, 12 * nside * nside)).astype(np.uint32)
    W = rng.uniform(1e-5, 3e-4, size=(3, B))
    nb = rng.uniform(4.0, 6.0, size=B)
    cd = torch.from_numpy(counts).to(DEV)
    Wd = torch.from_numpy(W).to(DEV)
    inb = torch.from_numpy(1.0 / nb).to(DEV)
    k3 = uf.born_kappa(cd, Wd, inb).cpu().numpy()
    ref = ocos.kappa(counts, W, nb)
    for t in range(3):
        rms = np.sqrt((ref[t] ** 2).mean())
        assert np.abs(k3[t] - ref[t]).max() <= 1e-5 * rms
        k1 = uf.born_kappa(cd, Wd[t], inb).cpu().numpy()[0]
        assert np.array_equal(k1, k3[t])


def test_overdensity(ufalcon, c1):
    e = c1["edges"][1:]
    counts = c1["ref_counts"][1:]
    cd = torch.from_numpy(counts.astype(np.uint32)).to(DEV)
    inb = uf.inv_nbar(c1["n"], c1["L"], e, 64)
    got = uf.overdensity(cd, e, inb, out_dtype=torch.float64).cpu().numpy()
    want = ocos.overdensity(counts, e, ocos.nbar(c1["n"], c1["L"], e, 64))
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_adjoint_matches_oracle_and_is_deterministic(ufalcon):
    rng = np.random.default_rng(4)
    B, nside, T = 11, 40, 2     # npix = 19200: two stage-1 blocks, ragged
    counts = rng.poisson(3.0, size=(B, 12 * nside * nside)).astype(np.uint32)
    nb = rng.uniform(2.0, 4.0, size=B)
    g = rng.normal(size=(T, 12 * nside * nside)).astype(np.float32)
    cd = torch.from_numpy(counts).to(DEV)
    inb = torch.from_numpy(1.0 / nb).to(DEV)
    gd = torch.from_numpy(g).to(DEV)
    a = uf.born_kappa_adjoint(cd, inb, gd)
    b = uf.born_kappa_adjoint(cd, inb, gd)
    assert torch.equal(a, b)
    ref = ocos.grad_W(counts, nb, g.astype(np.float64))
    assert np.allclose(a.cpu().numpy(), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_gradients_through_autograd(ufalcon):
    # L = sum_p kappa^2 on a small lognormal lightcone, Smail source:
    # dL/dW, dL/dOmega_m, dL/dz0 vs the oracle gradient and central FD (step 1e-4, FP64 forward)
    L = 300.0
    x, y, z = synth.lognormal_box(200000, L, seed=7, ngrid=32, dtype=torch.float32)
    edges = chi_edges_from_z(0.02, 0.12, 6)
    R = obin.default_n_rep(edges, L)
    nside = 16
    counts_ref, _ = obin.bin_shells(x, y, z, (L / 2,) * 3, L, R, edges, nside, threads=8)
    xd, yd, zd = _dev(x, y, z)
    counts = uf.bin_shells(xd, yd, zd, edges, nside, box_L=L, n_rep=R)
    assert np.array_equal(counts.cpu().numpy().astype(np.int64), counts_ref)
    inb = uf.inv_nbar(x.numel(), L, edges, nside)
    base = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=0.05, z_max=0.12)

    def loss(om, params, out_dtype):
        W = uf.LensingWeights.apply(om, params, [base], edges, DEV)
        kap = uf.BornKappa.apply(W, counts, inb, out_dtype)
        return (kap.to(torch.float64) ** 2).sum(), W

    om = torch.tensor(OMEGA_M, dtype=torch.float64, requires_grad=True)
    params = torch.tensor([base.params()], dtype=torch.float64, requires_grad=True)
    Lv, W = loss(om, params, torch.float32)
    W.retain_grad()
    Lv.backward()
    g_om, g_z0 = om.grad.item(), params.grad[0, 2].item()

    # oracle gradient from oracle counts: dL/dW = sum_p 2 kappa (n/nbar - 1); dW/dtheta by Richardson
    osrc = ocos.SmailSource(2.0, 1.5, 0.05, 0.12)
    Wr = ocos.lensing_weights(edges, OMEGA_M, osrc)
    nb = ocos.nbar(x.numel(), L, edges, nside)
    kr = ocos.kappa(counts_ref, Wr[None, :], nb)
    gW_ref = ocos.grad_W(counts_ref, nb, 2.0 * kr)[0]
    assert np.linalg.norm(W.grad.cpu().numpy()[0] - gW_ref) <= 1e-4 * np.linalg.norm(gW_ref)
    ref_om = float(gW_ref @ ocos.weight_derivative(edges, OMEGA_M, osrc, "omega_m"))
    ref_z0 = float(gW_ref @ ocos.weight_derivative(edges, OMEGA_M, osrc, "z0"))
    assert g_om == pytest.approx(ref_om, rel=1e-4)
    assert g_z0 == pytest.approx(ref_z0, rel=1e-4)

    # central differences of the FP64 forward, step 1e-4
    h = 1e-4
    with torch.no_grad():
        def L64(o, p):
            return loss(torch.tensor(o, dtype=torch.float64), torch.tensor([p], dtype=torch.float64),
                        torch.float64)[0].item()
        p0 = base.params()
        fd_om = (L64(OMEGA_M + h, p0) - L64(OMEGA_M - h, p0)) / (2 * h)
        fd_z0 = (L64(OMEGA_M, [p0[0], p0[1], p0[2] + h]) - L64(OMEGA_M, [p0[0], p0[1], p0[2] - h])) / (2 * h)
    assert g_om == pytest.approx(fd_om, rel=1e-4)
    assert g_z0 == pytest.approx(fd_z0, rel=1e-4)
