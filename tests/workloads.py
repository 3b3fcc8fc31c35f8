"""Synthetic workloads of the paper's kind, shared by the GPU tests.

Shell edges given in redshift are converted to comoving distance with the
oracle's distance (the edges are inputs to both sides; the library's own
distance is checked separately).  Catalogues come from `synth` and are
generated once and handed to both sides.
"""

from __future__ import annotations

import numpy as np
import torch

import synth
from oracle import cosmology as ocos

OMEGA_M = 0.3


def chi_edges_from_z(z_lo, z_hi, n_shells, om=OMEGA_M):
    return [ocos.chi(float(z), om) for z in np.linspace(z_lo, z_hi, n_shells + 1)]


def config1(device="cpu"):
    """2^18 FP64 particles uniform in a 500 Mpc/h cube, observer at the centre,
    10 equal shells to 250 Mpc/h, Nside 64, single source plane at z = 0.3."""
    L = 500.0
    x, y, z = synth.uniform_box(1 << 18, L, seed=0, dtype=torch.float64, device=device)
    return dict(x=x, y=y, z=z, L=L, n=1 << 18, edges=list(np.linspace(0.0, 250.0, 11)), nside=64, n_rep=0,
                source=("delta", 0.3))


def config2(device="cpu", n=1 << 27, seed=0):
    """512^3 FP32 particles from a seeded lognormal field (sigma_ln = 1, 256^3 grid) in a
    1 Gpc/h box, replicated to reach z = 0.5, 30 shells over z = 0.1..0.5, Nside 1024,
    Smail n(z) (alpha 2, beta 1.5, z0 0.3)."""
    L = 1000.0
    x, y, z = synth.lognormal_box(n, L, seed=seed, ngrid=256, dtype=torch.float32, device=device)
    edges = chi_edges_from_z(0.1, 0.5, 30)
    return dict(x=x, y=y, z=z, L=L, n=n, edges=edges, nside=1024, n_rep=1,
                source=("smail", 2.0, 1.5, 0.3, 0.5))


M = 1 << 20


def config3_draw():
    """The 16 realisations of the batched workload: particle counts ~ U[64M, 256M] and
    shell counts ~ U{20..60} drawn from meta-seed 0 (realisation r is seeded r)."""
    return (synth.randint(16, 64 * M, 256 * M, seed=0, stream=900),
            synth.randint(16, 20, 60, seed=0, stream=901))


def config3_realisation(r, device="cpu"):
    """Realisation r: lognormal FP32 particles in a 1 Gpc/h box, shells over z = 0.1..1.0,
    Nside 1024, images {-2..2}^3."""
    sizes, shells = config3_draw()
    L = 1000.0
    x, y, z = synth.lognormal_box(sizes[r], L, seed=r, ngrid=256, dtype=torch.float32, device=device)
    return dict(x=x, y=y, z=z, L=L, n=sizes[r], edges=chi_edges_from_z(0.1, 1.0, shells[r]), nside=1024, n_rep=2)


def config4(device="cpu"):
    """Nested full-sky lightcone, z = 0.1..1.5 in 47 shells, Nside 2048: an inner 1 Gpc/h box of
    768^3 particles (seed 0) for the shells below the first edge at z >= 0.6, an outer
    3 Gpc/h box of 768^3 particles (seed 1) beyond; particles streamed in 2^28 chunks;
    four Smail bins (alpha 2, beta 1.5, z0 = 0.3, 0.5, 0.7, 0.9)."""
    n = 768 ** 3
    zs = np.linspace(0.1, 1.5, 48)
    split = int(np.nonzero(zs >= 0.6)[0][0])
    edges = [ocos.chi(float(v), OMEGA_M) for v in zs]
    boxes = []
    for seed, L, b0, b1 in ((0, 1000.0, 0, split), (1, 3000.0, split, 47)):
        x, y, z = synth.lognormal_box(n, L, seed=seed, ngrid=256, dtype=torch.float32, device=device)
        boxes.append(dict(x=x, y=y, z=z, L=L, n=n, shell_begin=b0, shell_end=b1))
    return dict(boxes=boxes, edges=edges, nside=2048, split=split, chunk=1 << 28,
                z0s=(0.3, 0.5, 0.7, 0.9))


def config5_realisation(r, device="cpu"):
    """Realisation r of the differentiable covariance batch: 256^3 lognormal FP32 particles
    (seed r) in a 1 Gpc/h box, 40 shells over z = 0.1..1.5, Nside 512, Smail n(z)
    (alpha 2, beta 1.5, z0 0.3) on [0, 1.5]."""
    n = 256 ** 3
    L = 1000.0
    x, y, z = synth.lognormal_box(n, L, seed=r, ngrid=256, dtype=torch.float32, device=device)
    return dict(x=x, y=y, z=z, L=L, n=n, edges=chi_edges_from_z(0.1, 1.5, 40), nside=512, n_rep=3,
                source=("smail", 2.0, 1.5, 0.3, 1.5))
