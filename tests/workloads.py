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
