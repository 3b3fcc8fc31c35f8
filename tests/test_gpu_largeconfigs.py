"""GPU parity at the larger workloads' full sizes (the batched draw's largest
realisation, the nested Nside-2048 lightcone, the covariance batch), where the
oracle cannot pixelise every instance inside a test: count maps are checked
bit for bit against the oracle on the first 2^20-2^21 particles (same geometry,
same launch path), and at full size through properties that hold at any size:
two independent accumulations agree, streamed chunks compose, the Born sum of
the full maps equals the oracle's Born sum of the same maps, and gradients match
the oracle gradient and central differences.
"""

import os

import numpy as np
import pytest
import torch

import paper_1801_05745_amd as uf
from oracle import binning as obin
from oracle import cosmology as ocos

from workloads import OMEGA_M, config3_draw, config3_realisation, config4, config5_realisation

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _subset_bit_exact(x, y, z, L, R, edges, nside, m, b0=0, b1=None):
    xs, ys, zs = (t[:m].contiguous() for t in (x, y, z))
    got = uf.bin_shells(xs, ys, zs, edges, nside, box_L=L, n_rep=R, shell_begin=b0, shell_end=b1)
    torch.cuda.synchronize()
    ref, _ = obin.bin_shells(*(t.cpu().numpy() for t in (xs, ys, zs)), (L / 2,) * 3, L, R, edges, nside,
                             shell_begin=b0, shell_end=b1, threads=_threads())
    g = got.cpu().numpy().astype(np.int64)
    if b1 is not None or b0:
        g = g[b0:(b1 if b1 is not None else len(edges) - 1)]
    assert np.array_equal(g, ref)


@pytest.mark.timeout(1200)
def test_batched_draw_largest_realisation(ufalcon):
    sizes, shells = config3_draw()
    r = int(np.argmax(sizes))
    c = config3_realisation(r, device=DEV)
    x, y, z, L, R, edges, nside = c["x"], c["y"], c["z"], c["L"], c["n_rep"], c["edges"], c["nside"]
    assert R == obin.default_n_rep(edges, L)
    st_p, st_a = uf.new_status(DEV), uf.new_status(DEV)
    part = uf.bin_shells(x, y, z, edges, nside, box_L=L, n_rep=R, status=st_p, method="partition")
    atom = uf.bin_shells(x, y, z, edges, nside, box_L=L, n_rep=R, status=st_a, method="atomic")
    torch.cuda.synchronize()
    # two accumulations (keys + radix partition + LDS histograms; one atomic per instance)
    assert torch.equal(part, atom)
    sp, sa = uf.status_dict(st_p), uf.status_dict(st_a)
    assert sp["n_instances"] == sa["n_instances"] == int(part.sum(dtype=torch.int64))
    assert sp["n_unresolved"] == 0 and sp["n_invalid"] == 0
    del part, atom
    _subset_bit_exact(x, y, z, L, R, edges, nside, 1 << 21)


@pytest.mark.timeout(1200)
def test_nested_lightcone_streamed(ufalcon):
    c = config4(device=DEV)
    edges, nside, chunk = c["edges"], c["nside"], c["chunk"]
    B = len(edges) - 1
    streamed = uf.new_counts(B, nside, DEV)
    whole = uf.new_counts(B, nside, DEV)
    for box in c["boxes"]:
        L, b0, b1 = box["L"], box["shell_begin"], box["shell_end"]
        R = obin.default_n_rep(edges[b0:b1 + 1], L)
        for k in range(0, box["n"], chunk):
            sl = slice(k, min(k + chunk, box["n"]))
            uf.bin_shells(box["x"][sl], box["y"][sl], box["z"][sl], edges, nside, box_L=L, n_rep=R,
                          shell_begin=b0, shell_end=b1, counts=streamed)
        uf.bin_shells(box["x"], box["y"], box["z"], edges, nside, box_L=L, n_rep=R, shell_begin=b0,
                      shell_end=b1, counts=whole)
        box["R"] = R
    torch.cuda.synchronize()
    # counts accumulate: chunks of the stream compose into the one-call map
    assert torch.equal(streamed, whole)
    del whole
    for box in c["boxes"]:
        _subset_bit_exact(box["x"], box["y"], box["z"], box["L"], box["R"], edges, nside, 1 << 20,
                          box["shell_begin"], box["shell_end"])

    # the four tomographic bins' FP32 kappa of the full maps against the oracle's
    # Born sum of the same maps (each box's density in its shells)
    srcs = [uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=z0, z_max=1.5) for z0 in c["z0s"]]
    W = uf.lensing_weights(OMEGA_M, srcs, edges, device=DEV)
    inb = torch.cat([uf.inv_nbar(box["n"], box["L"], edges[box["shell_begin"]:box["shell_end"] + 1], nside,
                                 device=DEV) for box in c["boxes"]])
    kap = uf.born_kappa(streamed, W, inb, out_dtype=torch.float32)
    torch.cuda.synchronize()
    Wr = np.array([ocos.lensing_weights(edges, OMEGA_M, ocos.SmailSource(2.0, 1.5, z0, 1.5)) for z0 in c["z0s"]])
    assert np.allclose(W.cpu().numpy(), Wr, rtol=1e-11, atol=0.0)
    nb = np.concatenate([ocos.nbar(box["n"], box["L"], edges[box["shell_begin"]:box["shell_end"] + 1], nside)
                         for box in c["boxes"]])
    counts_h = streamed.cpu().numpy()
    del streamed
    kr = ocos.kappa(counts_h, Wr, nb)
    rms = np.sqrt((kr ** 2).mean(axis=1))
    err = np.abs(kap.cpu().numpy().astype(np.float64) - kr).max(axis=1)
    assert (err <= 1e-5 * rms).all(), (err, rms)


@pytest.mark.timeout(1200)
def test_covariance_batch_gradients(ufalcon):
    # two realisations of the covariance batch at full size: counts through the batched
    # plan, realisation 0 bit-exact against the oracle; L = sum_r sum_p kappa_r^2 back to
    # W, Omega_m and z0 against the oracle gradient (on the verified counts) and central
    # differences of the FP64 forward (step 1e-4)
    reals = [config5_realisation(r, device=DEV) for r in (0, 1)]
    edges, nside, L, R = reals[0]["edges"], reals[0]["nside"], reals[0]["L"], reals[0]["n_rep"]
    assert R == obin.default_n_rep(edges, L)
    B = len(edges) - 1
    items = [dict(x=c["x"], y=c["y"], z=c["z"], chi_edges=edges, box_L=L, n_rep=R,
                  counts=uf.new_counts(B, nside, DEV)) for c in reals]
    plan = uf.BatchPlan(items, nside, T=0)
    plan.clear()
    plan.bin()
    torch.cuda.synchronize()
    plan.close()
    ref0, _ = obin.bin_shells(*(reals[0][k].cpu().numpy() for k in ("x", "y", "z")), (L / 2,) * 3, L, R, edges,
                              nside, threads=_threads())
    assert np.array_equal(items[0]["counts"].cpu().numpy().astype(np.int64), ref0)

    n = reals[0]["n"]
    inb = uf.inv_nbar(n, L, edges, nside, device=DEV)
    base = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=0.3, z_max=1.5)

    def loss(om, params, out_dtype):
        W = uf.LensingWeights.apply(om, params, [base], edges, DEV)
        tot = 0.0
        for it in items:
            kap = uf.BornKappa.apply(W, it["counts"], inb, out_dtype)
            tot = tot + (kap.to(torch.float64) ** 2).sum()
        return tot, W

    om = torch.tensor(OMEGA_M, dtype=torch.float64, requires_grad=True)
    params = torch.tensor([base.params()], dtype=torch.float64, requires_grad=True)
    Lv, W = loss(om, params, torch.float32)
    W.retain_grad()
    Lv.backward()
    g_om, g_z0 = om.grad.item(), params.grad[0, 2].item()

    osrc = ocos.SmailSource(2.0, 1.5, 0.3, 1.5)
    Wr = ocos.lensing_weights(edges, OMEGA_M, osrc)
    nb = ocos.nbar(n, L, edges, nside)
    gW_ref = np.zeros(B)
    for it in items:
        ch = it["counts"].cpu().numpy().astype(np.int64)
        kr = ocos.kappa(ch, Wr[None, :], nb)
        gW_ref += ocos.grad_W(ch, nb, 2.0 * kr)[0]
    assert np.linalg.norm(W.grad.cpu().numpy()[0] - gW_ref) <= 1e-4 * np.linalg.norm(gW_ref)
    ref_om = float(gW_ref @ ocos.weight_derivative(edges, OMEGA_M, osrc, "omega_m"))
    ref_z0 = float(gW_ref @ ocos.weight_derivative(edges, OMEGA_M, osrc, "z0"))
    assert g_om == pytest.approx(ref_om, rel=1e-4)
    assert g_z0 == pytest.approx(ref_z0, rel=1e-4)

    h = 1e-4
    with torch.no_grad():
        def L64(o, p):
            return loss(torch.tensor(o, dtype=torch.float64), torch.tensor([p], dtype=torch.float64),
                        torch.float64)[0].item()
        p0 = list(base.params())
        fd_om = (L64(OMEGA_M + h, p0) - L64(OMEGA_M - h, p0)) / (2 * h)
        pp, pm = list(p0), list(p0)
        pp[2] += h
        pm[2] -= h
        fd_z0 = (L64(OMEGA_M, pp) - L64(OMEGA_M, pm)) / (2 * h)
    assert g_om == pytest.approx(fd_om, rel=1e-4)
    assert g_z0 == pytest.approx(fd_z0, rel=1e-4)
