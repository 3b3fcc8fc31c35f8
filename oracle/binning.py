"""Oracle (test infrastructure only): particle -> (shell, RING pixel) count maps.

Section 2.3 eq. (5) defines n_p(pix, Delta chi_b), the number of particles of
shell b in pixel pix; section 2.4 eq. (8) defines shell membership by comoving
radius, with the observer at the box centre, and builds the map from
independently processed subvolumes whose maps are summed.

Definition implemented here (readings listed in the design notes):
  * instance (i, s): d = fl64(fl64(x_i - o) + fl64(s L)) per axis, for every
    periodic image s in {-R..R}^3 (R = 0: no replication);
  * shell b in [b0, b1) with e_b <= |d| < e_{b+1} (half-open; eq. (8) prints <= on
    both ends, which would count edge particles twice);
  * pixel = exact RING pixel of d (oracle.healpix.ang2pix_ring);
  * particles with a non-finite coordinate are skipped and counted as invalid.

The C loop (bin_oracle.c) takes the FP64 decisions that are clear; the
instances it flags near a boundary are decided here exactly.
"""

from __future__ import annotations

import ctypes
import os
import threading
from fractions import Fraction as F

import numpy as np

from . import build as _build
from .healpix import ang2pix_ring, npix

_lib = None
_lock = threading.Lock()


def _load():
    global _lib
    with _lock:
        if _lib is None:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
            lib = ctypes.CDLL(path)
            lib.oracle_bin_fast.restype = ctypes.c_int64
            lib.oracle_bin_fast.argtypes = [
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                ctypes.c_int64, ctypes.c_int64,
                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
            lib.oracle_shell_totals.restype = ctypes.c_int64
            lib.oracle_shell_totals.argtypes = [
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                ctypes.c_int64, ctypes.c_int64,
                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
            lib.oracle_fast_ring_pixel.restype = ctypes.c_int
            lib.oracle_fast_ring_pixel.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
            _lib = lib
    return _lib


def fast_ring_pixel(nside: int, dx: float, dy: float, dz: float):
    """The C loop's FP64 pixel decision: pixel, or None when it defers to the exact path."""
    out = ctypes.c_int64(-1)
    ok = _load().oracle_fast_ring_pixel(nside, dx, dy, dz, ctypes.byref(out))
    return int(out.value) if ok else None


def instance_vector(x: float, y: float, z: float, observer, L: float, s):
    """d = fl64(fl64(x - o) + fl64(s L)) per axis (Python floats are IEEE binary64)."""
    return ((x - observer[0]) + float(s[0]) * L,
            (y - observer[1]) + float(s[1]) * L,
            (z - observer[2]) + float(s[2]) * L)


def exact_shell(d, edges, b0: int, b1: int):
    """Shell b in [b0, b1) with e_b^2 <= |d|^2 < e_{b+1}^2, exactly; None if outside."""
    r2 = F(d[0]) ** 2 + F(d[1]) ** 2 + F(d[2]) ** 2
    if r2 < F(edges[b0]) ** 2 or r2 >= F(edges[b1]) ** 2:
        return None
    for b in range(b0, b1):
        if F(edges[b]) ** 2 <= r2 < F(edges[b + 1]) ** 2:
            return b
    raise AssertionError("unreachable")


def exact_instance(d, edges, b0, b1, nside):
    """(shell, pixel) of one instance, decided exactly, or None if outside the shells."""
    b = exact_shell(d, edges, b0, b1)
    if b is None:
        return None
    return b, ang2pix_ring(nside, d[0], d[1], d[2])


def _as_np(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.float32, np.float64):
        raise TypeError("positions must be float32 or float64")
    return a


def check_edges(edges):
    e = [float(v) for v in edges]
    if len(e) < 2 or len(e) > 1025:
        raise ValueError("need 1..1024 shells")
    if any(not np.isfinite(v) or v < 0 for v in e) or any(e[j] >= e[j + 1] for j in range(len(e) - 1)):
        raise ValueError("edges must be finite, >= 0 and strictly ascending")
    return e


def bin_shells(x, y, z, observer, box_L: float, n_rep: int, edges, nside: int,
               shell_begin: int = 0, shell_end: int | None = None, threads: int = 1,
               flag_cap: int = 1 << 20):
    """Count maps int64 [shell_end - shell_begin][12 nside^2] for shells [shell_begin, shell_end).

    threads > 1 splits the particles into contiguous subvolumes of the input
    order processed concurrently into one map (the subvolume decomposition of
    section 2.4); integer counts make the result independent of the split.
    Returns (counts, stats) with stats = dict(instances, invalid, flagged).
    """
    xs, ys, zs = _as_np(x), _as_np(y), _as_np(z)
    if not (xs.dtype == ys.dtype == zs.dtype) or not (xs.shape == ys.shape == zs.shape):
        raise ValueError("x, y, z must share dtype and length")
    e = check_edges(edges)
    nshell = len(e) - 1
    b0 = int(shell_begin)
    b1 = nshell if shell_end is None else int(shell_end)
    if not (0 <= b0 <= b1 <= nshell):
        raise ValueError("bad shell range")
    n = xs.shape[0]
    N = int(nside)
    if N < 1:
        raise ValueError("nside >= 1")
    counts = np.zeros((b1 - b0, npix(N)), dtype=np.int64)
    stats = {"instances": 0, "invalid": 0, "flagged": 0}
    if n == 0 or b0 == b1:
        return counts, stats
    lib = _load()
    is_f64 = 1 if xs.dtype == np.float64 else 0
    e_arr = np.asarray(e, dtype=np.float64)
    ox, oy, oz = (float(v) for v in observer)
    R = int(n_rep)
    W = 2 * R + 1
    threads = max(1, min(int(threads), n))
    bounds = [n * k // threads for k in range(threads + 1)]
    st = np.zeros(2, dtype=np.int64)
    results = [None] * threads

    def work(k, cap):
        fl = np.zeros((cap, 2), dtype=np.int64)
        nf = lib.oracle_bin_fast(xs.ctypes.data, ys.ctypes.data, zs.ctypes.data, is_f64,
                                 bounds[k], bounds[k + 1], ox, oy, oz, float(box_L), R,
                                 e_arr.ctypes.data, b0, b1, N, counts.ctypes.data,
                                 fl.ctypes.data, cap, st.ctypes.data, 1 if threads > 1 else 0)
        results[k] = (nf, fl)

    def run_all(cap):
        if threads == 1:
            work(0, cap)
        else:
            ts = [threading.Thread(target=work, args=(k, cap)) for k in range(threads)]
            for t in ts:
                t.start()
            for t in ts:
                t.join()

    run_all(flag_cap)
    if any(r[0] > flag_cap for r in results):
        # Too many near-boundary instances for the buffer: redo with room for all.
        need = max(r[0] for r in results)
        counts[:] = 0
        st[:] = 0
        run_all(need)
    stats["instances"] = int(st[0])
    stats["invalid"] = int(st[1])
    for nf, fl in results:
        for i, code in fl[:nf]:
            sz = code % W - R
            sy = (code // W) % W - R
            sx = code // (W * W) - R
            d = instance_vector(float(xs[i]), float(ys[i]), float(zs[i]), (ox, oy, oz), float(box_L),
                                (sx, sy, sz))
            res = exact_instance(d, e, b0, b1, N)
            stats["flagged"] += 1
            if res is not None:
                counts[res[0] - b0, res[1]] += 1
                stats["instances"] += 1
    return counts, stats


def shell_totals(x, y, z, observer, box_L: float, n_rep: int, edges, shell_begin: int = 0,
                 shell_end: int | None = None, threads: int = 1, flag_cap: int = 1 << 20):
    """Instances per shell, int64 [shell_end - shell_begin] (section 2.4 eq. (8) alone):
    the row sums of bin_shells' count maps, without the pixelisation.  Guarded
    radii are decided exactly.  Returns (totals, stats) like bin_shells."""
    xs, ys, zs = _as_np(x), _as_np(y), _as_np(z)
    e = check_edges(edges)
    nshell = len(e) - 1
    b0 = int(shell_begin)
    b1 = nshell if shell_end is None else int(shell_end)
    if not (0 <= b0 <= b1 <= nshell):
        raise ValueError("bad shell range")
    n = xs.shape[0]
    totals = np.zeros(b1 - b0, dtype=np.int64)
    stats = {"instances": 0, "invalid": 0, "flagged": 0}
    if n == 0 or b0 == b1:
        return totals, stats
    lib = _load()
    is_f64 = 1 if xs.dtype == np.float64 else 0
    e_arr = np.asarray(e, dtype=np.float64)
    ox, oy, oz = (float(v) for v in observer)
    R = int(n_rep)
    W = 2 * R + 1
    threads = max(1, min(int(threads), n))
    bounds = [n * k // threads for k in range(threads + 1)]
    st = np.zeros(2, dtype=np.int64)
    results = [None] * threads

    def work(k, cap):
        fl = np.zeros((cap, 2), dtype=np.int64)
        nf = lib.oracle_shell_totals(xs.ctypes.data, ys.ctypes.data, zs.ctypes.data, is_f64,
                                     bounds[k], bounds[k + 1], ox, oy, oz, float(box_L), R,
                                     e_arr.ctypes.data, b0, b1, totals.ctypes.data,
                                     fl.ctypes.data, cap, st.ctypes.data, 1 if threads > 1 else 0)
        results[k] = (nf, fl)

    def run_all(cap):
        ts = [threading.Thread(target=work, args=(k, cap)) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()

    run_all(flag_cap)
    if any(r[0] > flag_cap for r in results):
        need = max(r[0] for r in results)
        totals[:] = 0
        st[:] = 0
        run_all(need)
    stats["invalid"] = int(st[1])
    for nf, fl in results:
        for i, code in fl[:nf]:
            sz = code % W - R
            sy = (code // W) % W - R
            sx = code // (W * W) - R
            d = instance_vector(float(xs[i]), float(ys[i]), float(zs[i]), (ox, oy, oz), float(box_L),
                                (sx, sy, sz))
            b = exact_shell(d, e, b0, b1)
            stats["flagged"] += 1
            if b is not None:
                totals[b - b0] += 1
    stats["instances"] = int(totals.sum())
    return totals, stats


def bin_shells_bruteforce(x, y, z, observer, box_L, n_rep, edges, nside, shell_begin=0, shell_end=None):
    """Every instance decided by the exact path (no FP64 shortcut).  Tiny inputs only."""
    xs, ys, zs = _as_np(x), _as_np(y), _as_np(z)
    e = check_edges(edges)
    b0 = int(shell_begin)
    b1 = len(e) - 1 if shell_end is None else int(shell_end)
    counts = np.zeros((b1 - b0, npix(nside)), dtype=np.int64)
    R = int(n_rep)
    for i in range(xs.shape[0]):
        px, py, pz = float(xs[i]), float(ys[i]), float(zs[i])
        if not (np.isfinite(px) and np.isfinite(py) and np.isfinite(pz)):
            continue
        for sx in range(-R, R + 1):
            for sy in range(-R, R + 1):
                for sz in range(-R, R + 1):
                    d = instance_vector(px, py, pz, observer, float(box_L), (sx, sy, sz))
                    res = exact_instance(d, e, b0, b1, nside)
                    if res is not None:
                        counts[res[0] - b0, res[1]] += 1
    return counts


def default_n_rep(edges, box_L: float, observer=None) -> int:
    """Smallest R such that images {-R..R}^3 of [0, L)^3 cover the ball of radius e_B around o."""
    L = float(box_L)
    o = observer if observer is not None else (L / 2, L / 2, L / 2)
    emax = float(edges[-1])
    R = 0
    for oj in o:
        # need s with s L <= oj - emax and (s + 1) L >= oj + emax covered
        lo = int(np.floor((oj - emax) / L))
        hi = int(np.floor((oj + emax) / L))
        R = max(R, -lo, hi)
    return R
