"""GPU parity: spherical-harmonic coefficients, power spectra (section 3.1
eq. (9)) and their covariance over realisations (section 3.2 eqs. (10), (11))
against the oracle.

Tolerance (FP64 on both sides, different summation orders): the GPU's ring
sums advance their twiddles by complex multiplication for up to 63 pixels
between exact re-seeds (a relative error of ~1e-14) and both sides run an
l-step recurrence of a few ulp per step, so coefficients agree to ~1e-13 of
the largest |a_lm|; the bound is 1e-10 of it.
"""

import numpy as np
import pytest
import torch

import paper_1801_05745_amd as uf
import synth
from oracle import spectra as S

pytestmark = pytest.mark.gpu
DEV = "cuda"
ALM_TOL = 1e-10


def _map(nside, seed, dtype=torch.float64, n_maps=1):
    npx = S.npix(nside)
    v = synth.normal64(n_maps * npx, seed=seed, stream=41).reshape(n_maps, npx)
    return v.to(dtype)


def _packed_to_full(v, lmax):
    a = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    for m in range(lmax + 1):
        off = m * (2 * lmax + 1 - m) // 2
        a[m, m:] = v[off + m:off + lmax + 1]
    return a


def _check_alm(got_full, want_full, where):
    scale = np.abs(want_full).max()
    err = np.abs(got_full - want_full).max()
    assert err <= ALM_TOL * scale, (where, err, scale)


@pytest.mark.parametrize("nside,lmax,dtype", [
    (1, None, torch.float64), (2, None, torch.float64), (4, None, torch.float32), (4, 20, torch.float64),
    (5, 9, torch.float64), (16, None, torch.float64), (16, None, torch.float32), (32, None, torch.float64),
    (64, None, torch.float32),
])
def test_map2alm_full_parity(ufalcon, nside, lmax, dtype):
    mp = _map(nside, seed=nside, dtype=dtype)
    L = 3 * nside - 1 if lmax is None else lmax
    got = uf.map2alm(mp[0].to(DEV), L).cpu().numpy()
    want = S.map2alm(mp[0].double().numpy(), nside, L)
    _check_alm(_packed_to_full(got, L), want, (nside, L, dtype))
    # C_l of the same coefficients
    cl = uf.alm2cl(torch.from_numpy(got).to(DEV), L).cpu().numpy()
    cl_want = S.alm2cl(_packed_to_full(got, L))
    np.testing.assert_allclose(cl, cl_want, rtol=1e-12, atol=0)
    cl_ref = S.alm2cl(want)
    np.testing.assert_allclose(cl, cl_ref, rtol=1e-8, atol=1e-10 * cl_ref.max())


def test_map2alm_batch_and_determinism(ufalcon):
    nside = 16
    maps = _map(nside, seed=5, n_maps=3).to(DEV)
    a = uf.map2alm(maps)
    for t in range(3):
        one = uf.map2alm(maps[t])
        assert torch.equal(one, a[t])
    assert torch.equal(uf.map2alm(maps), a)


@pytest.mark.parametrize("nside,lmax,ms", [
    (1024, None, [0, 1, 2, 3, 4, 17, 100, 1024, 2047, 2048, 3000, 3071]),
    (513, None, [0, 1, 5, 512, 1000, 1538]),
    (1100, 100, [0, 1, 33, 99, 100]),        # more ring pairs than one workgroup covers
    (2048, None, [0, 7, 3000, 6143]),        # four ring-pair blocks, lmax 6143
])
def test_map2alm_sampled_large(ufalcon, nside, lmax, ms):
    mp = _map(nside, seed=nside, dtype=torch.float32)
    L = 3 * nside - 1 if lmax is None else lmax
    got = uf.map2alm(mp[0].to(DEV), L).cpu().numpy()
    want = S.map2alm(mp[0].double().numpy(), nside, L, ms=ms)
    full = _packed_to_full(got, L)
    scale = np.abs(want).max()
    worst = 0.0
    for k, m in enumerate(ms):
        err = np.abs(full[m] - want[k]).max()
        worst = max(worst, err / scale)
        assert err <= ALM_TOL * scale, (nside, m, err, scale)
    print(f"nside {nside}: max |a_gpu - a_oracle| / max |a| = {worst:.2e}")


def test_map2alm_edge_cases(ufalcon):
    # lmax 0: a_00 only; no maps: nothing to do; lmax beyond 3 Nside - 1 (aliased, still the quadrature)
    nside = 4
    mp = _map(nside, seed=3)[0]
    a0 = uf.map2alm(mp.to(DEV), 0).cpu().numpy()
    assert a0.shape == (1,)
    ref0 = S.map2alm(mp.numpy(), nside, 0)
    assert abs(a0[0] - ref0[0, 0]) <= 1e-14 * abs(ref0[0, 0])
    empty = uf.map2alm(torch.zeros((0, S.npix(nside)), dtype=torch.float64, device=DEV), 5)
    assert empty.shape == (0, 21)
    big = uf.map2alm(mp.to(DEV), 40).cpu().numpy()
    _check_alm(_packed_to_full(big, 40), S.map2alm(mp.numpy(), nside, 40), "lmax 40 at Nside 4")
    with pytest.raises(ValueError):
        uf.map2alm(torch.zeros(100, dtype=torch.float64, device=DEV))


def test_anafast_of_constant_map(ufalcon):
    # C_0 = 4 pi c^2 exactly; the pixel quadrature leaks ~1e-8 of it into higher l
    nside = 32
    npx = S.npix(nside)
    c = uf.anafast(torch.full((npx,), 2.0, dtype=torch.float64, device=DEV)).cpu().numpy()
    assert abs(c[0] - 4 * np.pi * 4.0) <= 1e-13 * c[0]
    ref = S.alm2cl(S.map2alm(np.full(npx, 2.0), nside))
    np.testing.assert_allclose(c, ref, rtol=1e-8, atol=1e-10 * c[0])
    assert c[1:].max() <= 1e-7 * c[0]


@pytest.mark.parametrize("ell_min,delta_ell,n_bands,ddof", [(0, 1, None, 1), (2, 10, 9, 1), (5, 4, 20, 0),
                                                            (0, 96, 1, 0), (95, 1, 1, 1)])
def test_cl_covariance_parity(ufalcon, ell_min, delta_ell, n_bands, ddof):
    R, n_ell = 150, 96
    u = synth.uniform64(R * n_ell, seed=9, stream=43).reshape(R, n_ell).numpy()
    cl = (1.0 + u) / (1.0 + np.arange(n_ell))[None, :] ** 2
    mean, cov, corr = uf.cl_covariance(torch.from_numpy(cl).to(DEV), ell_min, delta_ell, n_bands, ddof)
    m_ref, c_ref, r_ref = S.cl_covariance(cl, ell_min, delta_ell, n_bands, ddof)
    np.testing.assert_allclose(mean.cpu().numpy(), m_ref, rtol=1e-13)
    np.testing.assert_allclose(cov.cpu().numpy(), c_ref, rtol=1e-11, atol=1e-14 * np.abs(c_ref).max())
    np.testing.assert_allclose(corr.cpu().numpy(), r_ref, rtol=1e-10, atol=1e-12)


def test_cl_covariance_two_realisations(ufalcon):
    cl = np.array([[1.0, 2.0, 4.0], [3.0, 2.0, 0.0]])
    mean, cov, corr = uf.cl_covariance(torch.from_numpy(cl).to(DEV), ddof=1)
    np.testing.assert_allclose(mean.cpu().numpy(), [2.0, 2.0, 2.0])
    np.testing.assert_allclose(cov.cpu().numpy(), np.cov(cl, rowvar=False, ddof=1), rtol=1e-15, atol=1e-15)
    c = corr.cpu().numpy()
    assert c[0, 2] == pytest.approx(-1.0) and c[0, 0] == pytest.approx(1.0)
    assert np.isnan(c[1]).all()   # zero variance at l = 1


def test_power_spectrum_of_many_maps_then_covariance(ufalcon):
    # the section 3.2 pipeline at small size: R maps -> C_l -> band covariance
    nside, R = 8, 12
    maps = _map(nside, seed=21, n_maps=R)
    cl = uf.anafast(maps.to(DEV)).cpu().numpy()
    cl_ref = np.stack([S.alm2cl(S.map2alm(maps[r].numpy(), nside)) for r in range(R)])
    np.testing.assert_allclose(cl, cl_ref, rtol=1e-8, atol=1e-10 * cl_ref.max())
    mean, cov, _ = uf.cl_covariance(torch.from_numpy(cl).to(DEV), 2, 4, 5, 1)
    m_ref, c_ref, _ = S.cl_covariance(cl, 2, 4, 5, 1)
    np.testing.assert_allclose(cov.cpu().numpy(), c_ref, rtol=1e-11, atol=1e-14 * np.abs(c_ref).max())
