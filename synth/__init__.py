"""Seeded synthetic particle catalogues shared by the oracle tests, the GPU tests and the bench.

This module holds only input generation: counter-based random numbers, a
lognormal density field and the placement of particles in a periodic box.
It contains none of the binning or lensing arithmetic.  The paper's own inputs
(L-PICOLA light-cone catalogues, section 2.2 and Table 1) are not available, so
these catalogues stand in for them with the same kind of structure: comoving
positions in a periodic cube, clustered like a non-linear matter field.

Random numbers come from SplitMix64 used as a counter-based hash
(Steele, Lea & Flood 2014): value(seed, stream, i) = mix(seed_key(seed, stream) + (i + 1) * GOLDEN).
The hash is written with torch int64 arithmetic (wrapping multiply, logical
shifts emulated with masks), so the same seed gives the same uniforms on the
CPU and on the GPU.  The lognormal field goes through an FFT, whose rounding
differs between devices; a test therefore generates a catalogue once and hands
the same arrays to both sides.
"""

from __future__ import annotations

import math

import torch

# SplitMix64 constants, written as signed int64 (two's complement).
_GOLDEN = 0x9E3779B97F4A7C15 - (1 << 64)
_MIX1 = 0xBF58476D1CE4E5B9 - (1 << 64)
_MIX2 = 0x94D049BB133111EB - (1 << 64)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 values (torch's >> is arithmetic)."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _MIX1
    z = (z ^ _srl(z, 27)) * _MIX2
    return z ^ _srl(z, 31)


def _seed_key(seed: int, stream: int) -> int:
    """Scalar SplitMix64 of (seed, stream) computed with Python integers."""
    m = (1 << 64) - 1
    z = ((seed & m) * 0x9E3779B97F4A7C15 + (stream & m) * 0xD1B54A32D192ED03 + 0x632BE59BD9B4E019) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    z ^= z >> 31
    return z - (1 << 64) if z >= (1 << 63) else z


def uniform64(n: int, seed: int, stream: int, device="cpu", offset: int = 0) -> torch.Tensor:
    """n uniforms in [0, 1) as float64, 53 random bits each, counter-based."""
    key = _seed_key(seed, stream)
    i = torch.arange(offset + 1, offset + n + 1, dtype=torch.int64, device=device)
    z = _mix(i * _GOLDEN + key)
    return _srl(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def normal64(n: int, seed: int, stream: int, device="cpu") -> torch.Tensor:
    """n standard normals by Box-Muller on two counter streams."""
    u1 = uniform64(n, seed, stream, device)
    u2 = uniform64(n, seed, stream + 0x10000, device)
    u1 = 1.0 - u1  # (0, 1]
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def _below(L: float, dtype: torch.dtype) -> float:
    """Largest value of `dtype` strictly below L."""
    t = torch.tensor(L, dtype=dtype)
    return float(torch.nextafter(t, torch.tensor(-math.inf, dtype=dtype)))


def uniform_box(n: int, L: float, seed: int, dtype=torch.float64, device="cpu"):
    """n positions uniform in [0, L)^3, as three SoA tensors of `dtype`."""
    out = []
    for axis in range(3):
        u = uniform64(n, seed, 100 + axis, device) * L
        v = u.to(dtype)
        v = torch.clamp(v, max=_below(L, dtype))
        out.append(v.contiguous())
    return tuple(out)


def lognormal_field(ngrid: int, seed: int, sigma_ln: float = 1.0, spectral_index: float = -2.0,
                    device="cpu") -> torch.Tensor:
    """Lognormal density rho = exp(G - var/2) on an ngrid^3 periodic grid.

    G is Gaussian with power spectrum P(k) ~ k^spectral_index (zero mean mode),
    rescaled so that its grid variance is sigma_ln^2.  Returns float64 [ngrid]*3.
    """
    white = normal64(ngrid ** 3, seed, 1, device).reshape(ngrid, ngrid, ngrid)
    fk = torch.fft.rfftn(white)
    kx = torch.fft.fftfreq(ngrid, device=device, dtype=torch.float64)
    kz = torch.fft.rfftfreq(ngrid, device=device, dtype=torch.float64)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (spectral_index / 4.0), torch.zeros_like(k2))
    g = torch.fft.irfftn(fk * amp, s=(ngrid, ngrid, ngrid))
    g = g - g.mean()
    g = g * (sigma_ln / g.std())
    return torch.exp(g - 0.5 * sigma_ln ** 2)


def lognormal_box(n: int, L: float, seed: int, ngrid: int = 256, sigma_ln: float = 1.0,
                  dtype=torch.float32, device="cpu", order: str = "shuffled", chunk: int = 1 << 26):
    """Exactly n particles in [0, L)^3 drawn from a seeded lognormal field.

    Cells are chosen multinomially with probability proportional to rho (Poisson
    sampling conditioned on the total), positions are uniform inside the cell.
    order="shuffled" keeps the random draw order; order="cell" sorts by cell.
    """
    rho = lognormal_field(ngrid, seed, sigma_ln, device=device).reshape(-1)
    # the CDF is summed on the host: a device scan may combine its partial sums
    # in a timing-dependent order, and a last-bit change of the CDF moves a
    # particle to another cell now and then
    cdf = torch.cumsum(rho.cpu(), 0)
    cdf = (cdf / cdf[-1]).to(device)
    xs = torch.empty(n, dtype=dtype, device=device)
    ys = torch.empty(n, dtype=dtype, device=device)
    zs = torch.empty(n, dtype=dtype, device=device)
    cell_size = L / ngrid
    top = _below(L, dtype)
    cells_all = []
    for start in range(0, n, chunk):
        m = min(chunk, n - start)
        u = uniform64(m, seed, 2, device, offset=start)
        cell = torch.searchsorted(cdf, u, right=True).clamp_(max=ngrid ** 3 - 1)
        if order == "cell":
            cells_all.append(cell)
            continue
        _place(cell, start, m, seed, ngrid, cell_size, top, dtype, device, xs, ys, zs)
    if order == "cell":
        cell = torch.sort(torch.cat(cells_all)).values
        del cells_all
        for start in range(0, n, chunk):
            m = min(chunk, n - start)
            _place(cell[start:start + m], start, m, seed, ngrid, cell_size, top, dtype, device, xs, ys, zs)
    return xs, ys, zs


def _place(cell, start, m, seed, ngrid, cell_size, top, dtype, device, xs, ys, zs):
    ci = cell // (ngrid * ngrid)
    cj = (cell // ngrid) % ngrid
    ck = cell % ngrid
    for idx, (c, out) in enumerate(((ci, xs), (cj, ys), (ck, zs))):
        u = uniform64(m, seed, 10 + idx, device, offset=start)
        v = ((c.to(torch.float64) + u) * cell_size).to(dtype)
        out[start:start + m] = torch.clamp(v, max=top)


def randint(n: int, lo: int, hi: int, seed: int, stream: int) -> list:
    """n integers uniform in [lo, hi] (inclusive) from the counter generator."""
    u = uniform64(n, seed, stream)
    return [lo + min(int(x * (hi - lo + 1)), hi - lo) for x in u.tolist()]
