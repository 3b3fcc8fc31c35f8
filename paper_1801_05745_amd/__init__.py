"""Python binding of libufalcon (MI355X / gfx950): shell binning onto HEALPix RING
count maps and the Born convergence sum with its adjoint (UFalcon, arXiv:1801.05745,
sections 2.3-2.4).

The functions mirror the C entry points in include/ufalcon.h one to one; they
only marshal torch tensors (device memory) and the current HIP stream into the
C-ABI.  Every step of the computation runs in the library's HIP kernels.  There
is no CPU fallback: without the built library every call raises.
"""

from __future__ import annotations

import ctypes
import json
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; UFALCON_LIB selects another build of the same library
LIB_PATH = os.environ.get("UFALCON_LIB") or os.path.join(_HERE, "libufalcon.so")

F32, F64 = 0, 1
SOURCE_DELTA, SOURCE_SMAIL = 0, 1
NBAR_EXACT_VOLUME, NBAR_LOWER_EDGE = 0, 1
NPARAM = 4
MAX_SHELLS = 256
MAX_BINS = 8
C_OVER_H0 = 2997.92458

_lib = None


class UfalconError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.ufalcon_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")


class Status(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_ulonglong), ("n_invalid", ctypes.c_ulonglong),
                ("n_guarded", ctypes.c_ulonglong), ("n_unresolved", ctypes.c_ulonglong),
                ("n_fallback", ctypes.c_ulonglong)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("z_s", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("z0", ctypes.c_double), ("z_max", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("observer", ctypes.c_double * 3), ("box_L", ctypes.c_double), ("n_rep", ctypes.c_int32),
                ("n_shells", ctypes.c_int32), ("shell_begin", ctypes.c_int32), ("shell_end", ctypes.c_int32),
                ("chi_edges", ctypes.POINTER(ctypes.c_double)), ("counts", ctypes.c_void_p),
                ("W", ctypes.c_void_p), ("inv_nbar", ctypes.c_void_p), ("kappa", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("accumulation", ctypes.c_int32), ("persistent_wgs", ctypes.c_int32), ("tile", ctypes.c_int64),
                ("n_tried", ctypes.c_int32), ("best", ctypes.c_int32), ("ms", ctypes.c_double * 16),
                ("cand_accumulation", ctypes.c_int32 * 16), ("cand_wgs", ctypes.c_int32 * 16),
                ("cand_tile", ctypes.c_int64 * 16)]


_P = ctypes.c_void_p
_I32, _I64, _D, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "ufalcon_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ufalcon_version": (ctypes.c_int, []),
    "ufalcon_fill_u32": (ctypes.c_int, [_P, _I64, ctypes.c_uint32, _P]),
    "ufalcon_counts_to_i64": (ctypes.c_int, [_P, _I64, _P, ctypes.c_int, _P]),
    "ufalcon_bin_shells_workspace_size": (_SZ, [_I64]),
    "ufalcon_bin_shells_workspace_size_partitioned": (_SZ, [_I64, _I32, _I32, _I64, _I64]),
    "ufalcon_bin_shells_partition_capacity": (_I64, [_I64, _I32, _I32, _I64, _SZ]),
    "ufalcon_bin_shells": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, ctypes.POINTER(_D), _D, _I32,
                                          ctypes.POINTER(_D), _I32, _I32, _I32, _I64, _P, _P, _P, _SZ, _P]),
    "ufalcon_bin_shells_timed": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, ctypes.POINTER(_D), _D, _I32,
                                                ctypes.POINTER(_D), _I32, _I32, _I32, _I64, _P, _P, _P, _SZ, _P,
                                                _P]),
    "ufalcon_bin_shells_noalloc": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, ctypes.POINTER(_D), _D, _I32,
                                                  ctypes.POINTER(_D), _I32, _I32, _I32, _I64, _P, _P, _P]),
    "ufalcon_phase_timer_create": (ctypes.c_int, [ctypes.POINTER(_P)]),
    "ufalcon_phase_timer_destroy": (ctypes.c_int, [_P]),
    "ufalcon_phase_timer_read": (ctypes.c_int, [_P, ctypes.POINTER(_D)]),
    "ufalcon_phase_timer_intervals": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "ufalcon_comoving_distance": (ctypes.c_int, [_P, _I64, _D, _P, _P]),
    "ufalcon_lensing_weights": (ctypes.c_int, [_D, ctypes.POINTER(Source), _I32, ctypes.POINTER(_D), _I32,
                                               _P, _P, _P]),
    "ufalcon_lensing_weights_vjp": (ctypes.c_int, [_P, _P, _I32, _I32, _P, _P]),
    "ufalcon_inv_nbar": (ctypes.c_int, [_I64, _D, ctypes.POINTER(_D), _I32, _I32, _I32, _I64, _I32, _P, _P]),
    "ufalcon_born_kappa": (ctypes.c_int, [_P, _I32, _I64, _P, _P, _I32, _P, ctypes.c_int, _P]),
    "ufalcon_overdensity": (ctypes.c_int, [_P, _I32, _I64, ctypes.POINTER(_D), _P, _P, ctypes.c_int, _P]),
    "ufalcon_born_kappa_adjoint_workspace_size": (_SZ, [_I32, _I64, _I32]),
    "ufalcon_born_kappa_adjoint": (ctypes.c_int, [_P, _I32, _I64, _P, _P, ctypes.c_int, _I32, _P, _P, _SZ, _P]),
    "ufalcon_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(BatchItem), _I32, ctypes.c_int, _I64, _I32,
                                                 ctypes.c_int, _I64, _I32, _I32, ctypes.POINTER(_P)]),
    "ufalcon_batch_plan_destroy": (ctypes.c_int, [_P]),
    "ufalcon_batch_clear": (ctypes.c_int, [_P, _P]),
    "ufalcon_bin_shells_batched": (ctypes.c_int, [_P, _P, _P]),
    "ufalcon_born_kappa_batched": (ctypes.c_int, [_P, _P]),
    "ufalcon_batch_run_graph": (ctypes.c_int, [_P, _P, _P]),
    "ufalcon_batch_autotune": (ctypes.c_int, [ctypes.POINTER(BatchItem), _I32, ctypes.c_int, _I64, _I32, ctypes.c_int,
                                              _I32, _P, _P]),
    "ufalcon_batch_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
    "ufalcon_batch_tuning_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_I32)]),
    "ufalcon_map2alm_workspace_size": (_SZ, [_I64, _I32]),
    "ufalcon_map2alm": (ctypes.c_int, [_P, ctypes.c_int, _I32, _I64, _I32, _P, _P, _SZ, _P]),
    "ufalcon_alm2cl": (ctypes.c_int, [_P, _I32, _I32, _P, _P]),
    "ufalcon_cl_covariance_workspace_size": (_SZ, [_I32, _I32]),
    "ufalcon_cl_covariance": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "ufalcon_alm2map_workspace_size": (_SZ, [_I64, _I32]),
    "ufalcon_alm2map": (ctypes.c_int, [_P, _I32, _I64, _I32, _P, _P, ctypes.c_int, _P, _SZ, _P]),
    "ufalcon_gaussian_beam": (ctypes.c_int, [_D, _I32, _P, _P]),
    "ufalcon_map_moments_workspace_size": (_SZ, [_I32]),
    "ufalcon_map_moments": (ctypes.c_int, [_P, ctypes.c_int, _I32, _I64, _P, _P, _SZ, _P]),
}


def exported_symbols():
    """Names of the C entry points this binding expects (one per declaration in ufalcon.h)."""
    return sorted(_SIGS)


def load():
    """Load libufalcon.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != 0:
        raise UfalconError(rc, where)


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype_code(dt):
    if dt == torch.float32:
        return F32
    if dt == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {dt} (float32 or float64)")


def _host_doubles(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * len(vals))(*vals), len(vals)


def npix(nside: int) -> int:
    return 12 * int(nside) * int(nside)


# ---------------------------------------------------------------- workspaces

_ws_cache = {}


def release_workspaces():
    """Drop the cached workspaces (their memory returns to torch's allocator)."""
    _ws_cache.clear()


def _workspace(nbytes: int, device, key: str):
    """A cached device byte buffer of at least nbytes (256-byte aligned by the caching allocator)."""
    k = (key, str(device))
    buf = _ws_cache.get(k)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[k] = buf
    return buf


def bin_shells_workspace(max_listed: int = 1 << 20, device="cuda"):
    """Workspace for the atomic accumulation path (guard list of max_listed entries)."""
    lib = load()
    return _workspace(int(lib.ufalcon_bin_shells_workspace_size(max_listed)), device, "bin")


MAX_PARTITION_KEYS = 0xFFF00000 - (1 << 25)


def expected_keys(n, chi_edges, box_L, n_rep, shell_begin=0, shell_end=None, headroom=1.25):
    """Keys a binning call of n particles is expected to emit: a particle uniform in
    [0, L)^3 has on average V / L^3 images in the shell range (section 2.4), V the
    volume between the range's radii, fewer when the range leaves the replicated
    boxes; here with 25 % headroom, at most n (2 n_rep + 1)^3, and n without a box.
    A partitioned workspace sized for it takes most calls in one chunk; a set with
    more keys (strong clustering near the range's edges) runs in further chunks,
    with the same counts."""
    side = 2 * int(n_rep) + 1
    if box_L <= 0.0:
        return int(n)
    e = [float(v) for v in chi_edges]
    hi = e[len(e) - 1 if shell_end is None else int(shell_end)]
    lo = e[int(shell_begin)]
    per = min(4.0 / 3.0 * math.pi * (hi ** 3 - lo ** 3) / box_L ** 3 * headroom, float(side ** 3))
    return int(min(n * side ** 3, math.ceil(n * per) + (1 << 20)))


def partition_capacity(n, n_rep, shells_in_range, nside, nbytes):
    """Keys one chunk of the partitioned accumulation takes at least with a workspace of
    nbytes (0: that workspace selects the atomic path); a host computation."""
    return int(load().ufalcon_bin_shells_partition_capacity(int(n), int(n_rep), int(shells_in_range), int(nside),
                                                            int(nbytes)))


def partition_workspace(n, n_rep, shells_in_range, nside, max_keys=None, device="cuda", cached=True):
    """Workspace that selects the partitioned accumulation path (keys per chunk: max_keys,
    default n (2 n_rep + 1)^3, capped below 2^32)."""
    lib = load()
    if max_keys is None:
        max_keys = n * (2 * n_rep + 1) ** 3
    max_keys = int(min(max_keys, MAX_PARTITION_KEYS))
    nbytes = int(lib.ufalcon_bin_shells_workspace_size_partitioned(int(n), int(n_rep), int(shells_in_range),
                                                                  int(nside), max_keys))
    if nbytes == 0:
        raise ValueError("no partitioned layout for these sizes")
    if not cached:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    return _workspace(nbytes, device, "partition")


STATUS_FIELDS = ("n_instances", "n_invalid", "n_guarded", "n_unresolved", "n_fallback")


def new_status(device="cuda"):
    """A zeroed device ufalcon_status (one uint64 per field of STATUS_FIELDS)."""
    return torch.zeros(len(STATUS_FIELDS), dtype=torch.int64, device=device)


def status_dict(st: torch.Tensor):
    return dict(zip(STATUS_FIELDS, st.cpu().tolist()))


# ---------------------------------------------------------------- entry points

def fill_u32(t: torch.Tensor, value: int = 0):
    lib = load()
    assert t.dtype == torch.uint32 and t.is_contiguous() and t.is_cuda
    _check(lib.ufalcon_fill_u32(_ptr(t), t.numel(), value, _stream(t.device)), "ufalcon_fill_u32")
    return t


def counts_to_i64(counts: torch.Tensor, out: torch.Tensor = None, accumulate: bool = False):
    """int64 copy of a uint32 count map (or, with accumulate, out += counts)."""
    lib = load()
    if counts.dtype != torch.uint32 or not counts.is_contiguous() or not counts.is_cuda:
        raise ValueError("counts must be a contiguous uint32 device tensor")
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an out tensor")
        out = torch.empty(counts.shape, dtype=torch.int64, device=counts.device)
    if out.dtype != torch.int64 or not out.is_contiguous() or out.numel() != counts.numel() or out.device != counts.device:
        raise ValueError("out must be a contiguous int64 tensor of the counts' size on their device")
    _check(lib.ufalcon_counts_to_i64(_ptr(counts), counts.numel(), _ptr(out), 1 if accumulate else 0,
                                     _stream(counts.device)), "ufalcon_counts_to_i64")
    return out


def new_counts(n_shells: int, nside: int, device="cuda"):
    t = torch.empty((n_shells, npix(nside)), dtype=torch.uint32, device=device)
    return fill_u32(t, 0)


PHASES = ("setup", "decide", "partition", "accumulate", "exact")


class PhaseTimer:
    """HIP events that a timed binning call records between its phases
    (setup, decide, partition, accumulate, exact); read() waits for the last
    one and returns the milliseconds of each phase, summed over chunks."""

    def __init__(self, device="cuda"):
        lib = load()
        with torch.cuda.device(torch.device(device)):
            h = ctypes.c_void_p()
            _check(lib.ufalcon_phase_timer_create(ctypes.byref(h)), "ufalcon_phase_timer_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def read(self):
        ms = (ctypes.c_double * len(PHASES))()
        _check(load().ufalcon_phase_timer_read(self._h, ms), "ufalcon_phase_timer_read")
        return dict(zip(PHASES, list(ms)))

    def intervals(self):
        """How many intervals each phase's sum covers (decide: key-pass launches)."""
        c = (ctypes.c_int32 * len(PHASES))()
        _check(load().ufalcon_phase_timer_intervals(self._h, c), "ufalcon_phase_timer_intervals")
        return dict(zip(PHASES, list(c)))

    def close(self):
        if self._h is not None and self._h.value:
            load().ufalcon_phase_timer_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bin_shells(x, y, z, chi_edges, nside, observer=None, box_L=0.0, n_rep=0, shell_begin=0, shell_end=None,
               counts=None, status=None, workspace=None, method="partition", timer=None):
    """Add the particles' (shell, RING pixel) counts to `counts` (uint32 [n_shells][npix]).

    x, y, z: contiguous float32 or float64 device tensors of equal length.
    chi_edges: shell edges in Mpc/h (host sequence, n_shells + 1 values).
    method: "partition" (keys + radix partition + LDS histograms) or "atomic"
    (one global atomic per instance); it only chooses the default workspace.
    timer: optional PhaseTimer that records the phases of this call.
    """
    lib = load()
    if not (x.dtype == y.dtype == z.dtype) or not (x.numel() == y.numel() == z.numel()):
        raise ValueError("x, y, z must share dtype and length")
    for t in (x, y, z):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("positions must be contiguous device tensors")
    e, ne = _host_doubles(chi_edges)
    n_shells = ne - 1
    if shell_end is None:
        shell_end = n_shells
    if observer is None:
        observer = (0.5 * box_L,) * 3
    obs, _ = _host_doubles(observer)
    if counts is None:
        counts = new_counts(n_shells, nside, x.device)
    if counts.dtype != torch.uint32 or not counts.is_contiguous() or counts.numel() != n_shells * npix(nside):
        raise ValueError("counts must be contiguous uint32 [n_shells][12 nside^2]")
    if workspace is None:
        if method == "partition":
            workspace = partition_workspace(x.numel(), n_rep, int(shell_end) - int(shell_begin), nside,
                                            max_keys=expected_keys(x.numel(), chi_edges, box_L, n_rep, shell_begin,
                                                                   shell_end),
                                            device=x.device)
        elif method == "atomic":
            workspace = bin_shells_workspace(device=x.device)
        else:
            raise ValueError(method)
    args = (_ptr(x), _ptr(y), _ptr(z), x.numel(), _dtype_code(x.dtype), obs, float(box_L), int(n_rep), e, n_shells,
            int(shell_begin), int(shell_end), int(nside), _ptr(counts), _ptr(status), _ptr(workspace),
            workspace.numel(), _stream(x.device))
    if timer is None:
        _check(lib.ufalcon_bin_shells(*args), "ufalcon_bin_shells")
    else:
        _check(lib.ufalcon_bin_shells_timed(*args, timer.handle), "ufalcon_bin_shells_timed")
    return counts


def bin_shells_noalloc(x, y, z, chi_edges, nside, observer=None, box_L=0.0, n_rep=0, shell_begin=0,
                       shell_end=None, counts=None, status=None):
    """bin_shells through the allocation-free entry point (atomic accumulation, library-held
    scratch).  `counts` must be given (the call itself allocates nothing)."""
    lib = load()
    if counts is None:
        raise ValueError("bin_shells_noalloc needs a caller-allocated counts tensor")
    if not (x.dtype == y.dtype == z.dtype) or not (x.numel() == y.numel() == z.numel()):
        raise ValueError("x, y, z must share dtype and length")
    for t in (x, y, z):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("positions must be contiguous device tensors")
    e, ne = _host_doubles(chi_edges)
    n_shells = ne - 1
    if shell_end is None:
        shell_end = n_shells
    if observer is None:
        observer = (0.5 * box_L,) * 3
    obs, _ = _host_doubles(observer)
    if counts.dtype != torch.uint32 or not counts.is_contiguous() or counts.numel() != n_shells * npix(nside):
        raise ValueError("counts must be contiguous uint32 [n_shells][12 nside^2]")
    _check(lib.ufalcon_bin_shells_noalloc(_ptr(x), _ptr(y), _ptr(z), x.numel(), _dtype_code(x.dtype), obs,
                                          float(box_L), int(n_rep), e, n_shells, int(shell_begin), int(shell_end),
                                          int(nside), _ptr(counts), _ptr(status), _stream(x.device)),
           "ufalcon_bin_shells_noalloc")
    return counts


def save_stream_checkpoint(prefix, cursor, counts, status=None):
    """Write a resumable state of a chunked binning run: the count map (host copy
    of `counts`), the status counters and `cursor` (a dict: the next chunk and the
    run's shape).  The map goes to a file named after the chunks done and the
    JSON file <prefix>.json, replaced atomically, commits the state; the previous
    map file is removed afterwards, so a crash at any point leaves one whole state."""
    import numpy as np

    prefix = os.fspath(prefix)
    state = dict(cursor)
    old = load_stream_checkpoint(prefix, counts_too=False)
    name = f"{os.path.basename(prefix)}.{int(state['chunks_done'])}.npy"
    path = os.path.join(os.path.dirname(prefix) or ".", name)
    host = counts.detach().view(torch.int32).cpu().numpy().view(np.uint32)
    with open(path + ".tmp", "wb") as f:
        np.save(f, host, allow_pickle=False)
        f.flush()
        os.fsync(f.fileno())
    os.replace(path + ".tmp", path)
    state["counts_file"] = name
    state["status"] = None if status is None else [int(v) for v in status.cpu().tolist()]
    with open(prefix + ".json.tmp", "w") as f:
        json.dump(state, f)
        f.flush()
        os.fsync(f.fileno())
    os.replace(prefix + ".json.tmp", prefix + ".json")
    if old is not None and old["counts_file"] != name:
        try:
            os.remove(os.path.join(os.path.dirname(prefix) or ".", old["counts_file"]))
        except FileNotFoundError:
            pass


def load_stream_checkpoint(prefix, counts_too=True):
    """The state written by save_stream_checkpoint (with the map as a numpy uint32
    array under "counts" when counts_too), or None if there is none."""
    import numpy as np

    prefix = os.fspath(prefix)
    if not os.path.exists(prefix + ".json"):
        return None
    with open(prefix + ".json") as f:
        state = json.load(f)
    if counts_too:
        state["counts"] = np.load(os.path.join(os.path.dirname(prefix) or ".", state["counts_file"]),
                                  allow_pickle=False)
    return state


class HostStream:
    """Bins particles held in pinned host memory: chunks of `chunk` particles are
    copied to two device staging slots on a copy stream, and each chunk is binned
    on the caller's stream as soon as its copy lands, so the copy of chunk k+1
    overlaps the binning of chunk k (the subvolume decomposition of section 2.4:
    chunk maps add up in the count map).  The slots and the binning workspace are
    allocated once, at construction.  copy_ms() reads the copy engine's busy time
    (HIP events on the copy stream) of the last run.

    A run can be made resumable: with `checkpoint` (a path prefix) and
    checkpoint_every = k > 0 the count map, the status and the cursor of the next
    chunk are saved every k chunks and when the run stops; run(..., resume=True)
    loads them and continues at the cursor.  Integer counts add associatively, so
    a resumed run gives the same map, bit for bit, as an uninterrupted one.
    max_chunks stops a run after that many chunks (self.cursor then names the
    next one; None when every chunk is done)."""

    def __init__(self, chunk, n_rep_max, shells_max, nside, device="cuda", dtype=torch.float32):
        self.chunk = int(chunk)
        self.device = torch.device(device)
        self.slots = [[torch.empty(self.chunk, dtype=dtype, device=self.device) for _ in range(3)]
                      for _ in range(2)]
        self.ws = partition_workspace(self.chunk, n_rep_max, shells_max, nside, device=self.device, cached=False)
        self.copy = torch.cuda.Stream(self.device)
        self._events = []
        self.cursor = None

    def run(self, boxes, chi_edges, nside, counts, status=None, checkpoint=None, checkpoint_every=0, resume=False,
            max_chunks=None):
        """boxes: dicts with host (pinned) x, y, z, box_L, n_rep, shell_begin, shell_end
        (and optionally observer); every chunk is added to `counts`."""
        compute = torch.cuda.current_stream(self.device)
        free = [None, None]
        self._events = []
        shape = {"chunk": self.chunk, "nside": int(nside), "cells": int(counts.numel()),
                 "boxes": [int(b["x"].numel()) for b in boxes]}
        start_box, start_off, done = 0, 0, 0
        if resume:
            if checkpoint is None:
                raise ValueError("resume needs the checkpoint prefix")
            st = load_stream_checkpoint(checkpoint)
            if st is None:
                raise FileNotFoundError(f"no checkpoint at {checkpoint}.json")
            if st["shape"] != shape:
                raise ValueError(f"checkpoint of another run: {st['shape']} != {shape}")
            if st["counts"].size != counts.numel():
                raise ValueError("checkpoint map size differs")
            counts.view(torch.int32).view(-1).copy_(torch.from_numpy(st["counts"].view("int32")).view(-1))
            if status is not None and st["status"] is not None:
                status.copy_(torch.tensor(st["status"], dtype=status.dtype))
            if st["next"] is None:
                self.cursor = None
                return counts
            start_box, start_off = st["next"]
            done = int(st["chunks_done"])

        def save(nxt):
            save_stream_checkpoint(checkpoint, {"shape": shape, "next": nxt, "chunks_done": done}, counts, status)

        j = 0
        self.cursor = None
        for bi, b in enumerate(boxes):
            if bi < start_box:
                continue
            hx, hy, hz = b["x"], b["y"], b["z"]
            for t in (hx, hy, hz):
                if t.is_cuda or not t.is_pinned():
                    raise ValueError("HostStream needs pinned host tensors")
            n = hx.numel()
            for k in range(start_off if bi == start_box else 0, n, self.chunk):
                if max_chunks is not None and j >= max_chunks:
                    self.cursor = (bi, k)
                    if checkpoint is not None:
                        save(list(self.cursor))
                    return counts
                m = min(self.chunk, n - k)
                s = j & 1
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                with torch.cuda.stream(self.copy):
                    if free[s] is not None:
                        self.copy.wait_event(free[s])
                    ev[0].record(self.copy)
                    for a, h in enumerate((hx, hy, hz)):
                        self.slots[s][a][:m].copy_(h[k:k + m], non_blocking=True)
                    ev[1].record(self.copy)
                compute.wait_event(ev[1])
                bin_shells(self.slots[s][0][:m], self.slots[s][1][:m], self.slots[s][2][:m], chi_edges, nside,
                           observer=b.get("observer"), box_L=b["box_L"], n_rep=b["n_rep"],
                           shell_begin=b.get("shell_begin", 0), shell_end=b.get("shell_end"), counts=counts,
                           status=status, workspace=self.ws)
                done_ev = torch.cuda.Event()
                done_ev.record(compute)
                free[s] = done_ev
                self._events.append(ev)
                j += 1
                done += 1
                if checkpoint is not None and checkpoint_every > 0 and done % checkpoint_every == 0:
                    nxt = [bi, k + self.chunk] if k + self.chunk < n else [bi + 1, 0]
                    save(nxt if nxt[0] < len(boxes) else None)
        if checkpoint is not None:
            save(None)
        return counts

    def copy_ms(self):
        """Milliseconds the copy stream spent in the last run's copies (waits for them)."""
        for _, b in self._events:
            b.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._events)


def comoving_distance(z: torch.Tensor, omega_m: float):
    lib = load()
    z = z.to(torch.float64).contiguous()
    chi = torch.empty_like(z)
    _check(lib.ufalcon_comoving_distance(_ptr(z), z.numel(), float(omega_m), _ptr(chi), _stream(z.device)),
           "ufalcon_comoving_distance")
    return chi


@dataclass
class SourceSpec:
    """One source bin: kind "delta" (z_s) or "smail" (alpha, beta, z0, z_max)."""
    kind: str
    z_s: float = 0.0
    alpha: float = 0.0
    beta: float = 0.0
    z0: float = 0.0
    z_max: float = 0.0

    def params(self):
        """Differentiable parameters in derivative slots 1..3."""
        if self.kind == "delta":
            return [self.z_s, 0.0, 0.0]
        return [self.alpha, self.beta, self.z0]

    def with_params(self, p):
        if self.kind == "delta":
            return SourceSpec("delta", z_s=float(p[0]))
        return SourceSpec("smail", alpha=float(p[0]), beta=float(p[1]), z0=float(p[2]), z_max=self.z_max)

    def c_struct(self):
        if self.kind == "delta":
            return Source(SOURCE_DELTA, self.z_s, 0.0, 0.0, 0.0, 0.0)
        if self.kind == "smail":
            return Source(SOURCE_SMAIL, 0.0, self.alpha, self.beta, self.z0, self.z_max)
        raise ValueError(self.kind)


def lensing_weights(omega_m, sources, chi_edges, with_derivatives=False, device="cuda"):
    """W [T][B] (float64, device) and optionally dW [T][B][4] (d/dOmega_m, d/d source parameters)."""
    lib = load()
    srcs = (Source * len(sources))(*[s.c_struct() for s in sources])
    e, ne = _host_doubles(chi_edges)
    T, B = len(sources), ne - 1
    W = torch.empty((T, B), dtype=torch.float64, device=device)
    dW = torch.empty((T, B, NPARAM), dtype=torch.float64, device=device) if with_derivatives else None
    _check(lib.ufalcon_lensing_weights(float(omega_m), srcs, T, e, B, _ptr(W), _ptr(dW), _stream(W.device)),
           "ufalcon_lensing_weights")
    return (W, dW) if with_derivatives else W


def lensing_weights_vjp(dW, grad_W):
    lib = load()
    T, B, _ = dW.shape
    out = torch.empty((T, NPARAM), dtype=torch.float64, device=dW.device)
    gW = grad_W.to(torch.float64).contiguous()
    _check(lib.ufalcon_lensing_weights_vjp(_ptr(dW), _ptr(gW), T, B, _ptr(out), _stream(dW.device)),
           "ufalcon_lensing_weights_vjp")
    return out


def inv_nbar(n_src, box_L, chi_edges, nside, mode=NBAR_EXACT_VOLUME, shell_begin=0, shell_end=None, out=None,
             device="cuda"):
    """1 / nbar_b (float64 device [n_shells]) for shells [shell_begin, shell_end)."""
    lib = load()
    e, ne = _host_doubles(chi_edges)
    B = ne - 1
    if shell_end is None:
        shell_end = B
    if out is None:
        out = torch.zeros(B, dtype=torch.float64, device=device)
    _check(lib.ufalcon_inv_nbar(int(n_src), float(box_L), e, B, int(shell_begin), int(shell_end), int(nside),
                                int(mode), _ptr(out), _stream(out.device)), "ufalcon_inv_nbar")
    return out


def _nside_of(npx: int) -> int:
    nside = int(round((npx / 12) ** 0.5))
    if nside < 1 or npix(nside) != npx:
        raise ValueError(f"{npx} is not a HEALPix pixel count 12 nside^2")
    return nside


def _check_counts(counts):
    """(B, npix, nside) of a count map; raises ValueError unless it is a contiguous
    uint32 device tensor [B][12 nside^2].  Shapes and dtypes are checked before the
    device, so every defect is reported on any machine."""
    if not isinstance(counts, torch.Tensor) or counts.dim() != 2:
        raise ValueError("counts must be a 2-d tensor [n_shells][12 nside^2]")
    if counts.dtype != torch.uint32:
        raise ValueError(f"counts must be uint32 (got {counts.dtype}); the kernels read 32-bit counts")
    B, npx = counts.shape
    if B < 1 or B > MAX_SHELLS:
        raise ValueError(f"counts has {B} shells; 1..{MAX_SHELLS} are supported")
    return B, npx, _nside_of(npx)


def _check_device(where, ref, *tensors):
    """Every tensor contiguous and on ref's CUDA device."""
    for t in (ref,) + tensors:
        if not t.is_contiguous():
            raise ValueError(f"{where}: tensors must be contiguous")
        if not t.is_cuda or t.device != ref.device:
            raise ValueError(f"{where}: tensors must live on one CUDA device (got {t.device} and {ref.device})")


def _check_inv_nbar(inv_nbar_, B):
    if not isinstance(inv_nbar_, torch.Tensor) or inv_nbar_.dtype != torch.float64 or inv_nbar_.numel() != B:
        raise ValueError(f"inv_nbar must be a float64 tensor of {B} values (one per shell)")


def born_kappa(counts, W, inv_nbar_, out_dtype=torch.float32):
    """kappa [T][npix] = sum_b W[t][b] (counts[b] * inv_nbar[b] - 1).

    counts: uint32 [B][12 nside^2]; W: float64 [T][B] or [B]; inv_nbar: float64 [B];
    all contiguous on one device (ValueError otherwise)."""
    lib = load()
    B, npx, nside = _check_counts(counts)
    if not isinstance(W, torch.Tensor) or W.dim() not in (1, 2) or W.shape[-1] != B:
        raise ValueError(f"W must be [T][{B}] or [{B}] (one weight per shell)")
    if not W.dtype.is_floating_point:
        raise ValueError("W must be floating point")
    _check_inv_nbar(inv_nbar_, B)
    W = W.to(torch.float64).contiguous()
    if W.dim() == 1:
        W = W[None, :]
    T = W.shape[0]
    if T < 1 or T > MAX_BINS:
        raise ValueError(f"{T} source bins; 1..{MAX_BINS} are supported")
    _dtype_code(out_dtype)
    _check_device("born_kappa", counts, W, inv_nbar_)
    out = torch.empty((T, npx), dtype=out_dtype, device=counts.device)
    _check(lib.ufalcon_born_kappa(_ptr(counts), B, nside, _ptr(W), _ptr(inv_nbar_), T, _ptr(out),
                                  _dtype_code(out_dtype), _stream(counts.device)), "ufalcon_born_kappa")
    return out


def overdensity(counts, chi_edges, inv_nbar_, out_dtype=torch.float32):
    """Projected overdensity [npix]: the Born sum with weights Delta chi_b / sum Delta chi_b."""
    lib = load()
    B, npx, nside = _check_counts(counts)
    e, ne = _host_doubles(chi_edges)
    if ne != B + 1:
        raise ValueError(f"chi_edges must hold {B + 1} values for {B} shells (got {ne})")
    _check_inv_nbar(inv_nbar_, B)
    _dtype_code(out_dtype)
    _check_device("overdensity", counts, inv_nbar_)
    out = torch.empty(npx, dtype=out_dtype, device=counts.device)
    _check(lib.ufalcon_overdensity(_ptr(counts), B, nside, e, _ptr(inv_nbar_), _ptr(out), _dtype_code(out_dtype),
                                   _stream(counts.device)), "ufalcon_overdensity")
    return out


def born_kappa_adjoint(counts, inv_nbar_, grad_kappa):
    """grad_W [T][B] = sum_p grad_kappa[t][p] (counts[b][p] inv_nbar[b] - 1), deterministic.

    grad_kappa: float32 or float64 [T][npix] or [npix], on the counts' device."""
    lib = load()
    B, npx, nside = _check_counts(counts)
    _check_inv_nbar(inv_nbar_, B)
    if not isinstance(grad_kappa, torch.Tensor) or grad_kappa.dim() not in (1, 2) or grad_kappa.shape[-1] != npx:
        raise ValueError(f"grad_kappa must be [T][{npx}] or [{npx}]")
    g = grad_kappa.contiguous()
    if g.dim() == 1:
        g = g[None, :]
    T = g.shape[0]
    if T < 1 or T > MAX_BINS:
        raise ValueError(f"{T} source bins; 1..{MAX_BINS} are supported")
    code = _dtype_code(g.dtype)
    _check_device("born_kappa_adjoint", counts, inv_nbar_, g)
    nbytes = int(lib.ufalcon_born_kappa_adjoint_workspace_size(B, nside, T))
    ws = _workspace(nbytes, counts.device, "adjoint")
    out = torch.empty((T, B), dtype=torch.float64, device=counts.device)
    _check(lib.ufalcon_born_kappa_adjoint(_ptr(counts), B, nside, _ptr(inv_nbar_), _ptr(g), code, T,
                                          _ptr(out), _ptr(ws), ws.numel(), _stream(counts.device)),
           "ufalcon_born_kappa_adjoint")
    return out


# ---------------------------------------------------------------- power spectra

def n_alm(lmax: int) -> int:
    return (int(lmax) + 1) * (int(lmax) + 2) // 2


def map2alm(maps, lmax=None):
    """a_lm of HEALPix RING maps [n_maps][npix] (or one map [npix]), complex128
    [n_maps][n_alm] in m-major order (index m (2 lmax + 1 - m)/2 + l);
    lmax defaults to 3 Nside - 1."""
    lib = load()
    m = maps.contiguous()
    single = m.dim() == 1
    if single:
        m = m[None, :]
    nmaps, npx = m.shape
    nside = int(round((npx / 12) ** 0.5))
    if npix(nside) != npx:
        raise ValueError(f"{npx} is not a HEALPix pixel count")
    if lmax is None:
        lmax = 3 * nside - 1
    nbytes = int(lib.ufalcon_map2alm_workspace_size(nside, int(lmax)))
    if nbytes == 0:
        raise ValueError("invalid nside or lmax")
    ws = _workspace(nbytes, m.device, "map2alm")
    out = torch.empty((nmaps, n_alm(lmax), 2), dtype=torch.float64, device=m.device)
    _check(lib.ufalcon_map2alm(_ptr(m), _dtype_code(m.dtype), nmaps, nside, int(lmax), _ptr(out), _ptr(ws),
                               ws.numel(), _stream(m.device)), "ufalcon_map2alm")
    out = torch.view_as_complex(out)
    return out[0] if single else out


def alm2cl(alm, lmax):
    """C_l [n_maps][lmax+1] from complex128 coefficients [n_maps][n_alm] (or [n_alm])."""
    lib = load()
    a = alm.contiguous()
    single = a.dim() == 1
    if single:
        a = a[None, :]
    if a.shape[1] != n_alm(lmax) or a.dtype != torch.complex128:
        raise ValueError("alm must be complex128 [n_maps][(lmax+1)(lmax+2)/2]")
    out = torch.empty((a.shape[0], int(lmax) + 1), dtype=torch.float64, device=a.device)
    _check(lib.ufalcon_alm2cl(_ptr(torch.view_as_real(a)), a.shape[0], int(lmax), _ptr(out), _stream(a.device)),
           "ufalcon_alm2cl")
    return out[0] if single else out


def anafast(maps, lmax=None):
    """Power spectra C_l of maps [n_maps][npix] (or [npix]); lmax defaults to 3 Nside - 1."""
    npx = maps.shape[-1]
    nside = int(round((npx / 12) ** 0.5))
    if lmax is None:
        lmax = 3 * nside - 1
    return alm2cl(map2alm(maps, lmax), lmax)


def cl_covariance(cl, ell_min=0, delta_ell=1, n_bands=None, ddof=1, with_corr=True):
    """(band means [n_bands], covariance [n_bands][n_bands], correlation or None) of
    power spectra cl [n_real][n_ell] over the realisations."""
    lib = load()
    c = cl.to(torch.float64).contiguous()
    R, n_ell = c.shape
    if n_bands is None:
        n_bands = (n_ell - ell_min) // delta_ell
    nbytes = int(lib.ufalcon_cl_covariance_workspace_size(R, int(n_bands)))
    ws = _workspace(max(nbytes, 1), c.device, "cl_covariance")
    mean = torch.empty(n_bands, dtype=torch.float64, device=c.device)
    cov = torch.empty((n_bands, n_bands), dtype=torch.float64, device=c.device)
    corr = torch.empty_like(cov) if with_corr else None
    _check(lib.ufalcon_cl_covariance(_ptr(c), R, n_ell, int(ell_min), int(delta_ell), int(n_bands), int(ddof),
                                     _ptr(mean), _ptr(cov), _ptr(corr), _ptr(ws), ws.numel(), _stream(c.device)),
           "ufalcon_cl_covariance")
    return mean, cov, corr


def gaussian_beam(sigma, lmax, device="cuda"):
    """b_l = exp(-l(l+1) sigma^2 / 2) for l = 0..lmax (sigma: r.m.s. radius in radians)."""
    lib = load()
    out = torch.empty(int(lmax) + 1, dtype=torch.float64, device=device)
    _check(lib.ufalcon_gaussian_beam(float(sigma), int(lmax), _ptr(out), _stream(out.device)), "ufalcon_gaussian_beam")
    return out


def alm2map(alm, nside, lmax, beam=None, out_dtype=torch.float64):
    """Real maps [n_maps][npix] (or [npix]) from complex128 coefficients
    [n_maps][n_alm] (or [n_alm]), optionally multiplied by a beam b_l."""
    lib = load()
    a = alm.contiguous()
    single = a.dim() == 1
    if single:
        a = a[None, :]
    if a.shape[1] != n_alm(lmax) or a.dtype != torch.complex128:
        raise ValueError("alm must be complex128 [n_maps][(lmax+1)(lmax+2)/2]")
    b = None
    if beam is not None:
        b = beam.to(device=a.device, dtype=torch.float64).contiguous()
        if b.numel() != int(lmax) + 1:
            raise ValueError("beam must hold lmax + 1 values")
    nbytes = int(lib.ufalcon_alm2map_workspace_size(int(nside), int(lmax)))
    if nbytes == 0:
        raise ValueError("invalid nside or lmax")
    ws = _workspace(nbytes, a.device, "map2alm")
    out = torch.empty((a.shape[0], npix(nside)), dtype=out_dtype, device=a.device)
    _check(lib.ufalcon_alm2map(_ptr(torch.view_as_real(a)), a.shape[0], int(nside), int(lmax), _ptr(b), _ptr(out),
                               _dtype_code(out_dtype), _ptr(ws), ws.numel(), _stream(a.device)), "ufalcon_alm2map")
    return out[0] if single else out


def smooth(maps, sigma, lmax=None, out_dtype=None):
    """Maps smoothed with a Gaussian beam of r.m.s. radius sigma (radians):
    analysis to lmax (default 3 Nside - 1), beam, synthesis."""
    npx = maps.shape[-1]
    nside = int(round((npx / 12) ** 0.5))
    if lmax is None:
        lmax = 3 * nside - 1
    a = map2alm(maps, lmax)
    return alm2map(a, nside, lmax, gaussian_beam(sigma, lmax, maps.device),
                   out_dtype=maps.dtype if out_dtype is None else out_dtype)


MOMENT_NAMES = ("mean", "m2", "m4", "s2", "var_s2")


def map_moments(maps):
    """[n_maps][5] (or [5]) FP64: mean, m2, m4, s^2 and sigma_{s^2}^2 of each map."""
    lib = load()
    m = maps.contiguous()
    single = m.dim() == 1
    if single:
        m = m[None, :]
    nbytes = int(lib.ufalcon_map_moments_workspace_size(m.shape[0]))
    ws = _workspace(max(nbytes, 8), m.device, "moments")
    out = torch.empty((m.shape[0], len(MOMENT_NAMES)), dtype=torch.float64, device=m.device)
    _check(lib.ufalcon_map_moments(_ptr(m), _dtype_code(m.dtype), m.shape[0], m.shape[1], _ptr(out), _ptr(ws),
                                   ws.numel(), _stream(m.device)), "ufalcon_map_moments")
    return out[0] if single else out


# ---------------------------------------------------------------- autograd

class BornKappa(torch.autograd.Function):
    """kappa = Born sum of fixed counts with differentiable weights W [T][B]."""

    @staticmethod
    def forward(ctx, W, counts, inv_nbar_, out_dtype=torch.float32):
        ctx.save_for_backward(counts, inv_nbar_)
        return born_kappa(counts, W, inv_nbar_, out_dtype)

    @staticmethod
    def backward(ctx, grad_kappa):
        counts, inv_nbar_ = ctx.saved_tensors
        return born_kappa_adjoint(counts, inv_nbar_, grad_kappa), None, None, None


class LensingWeights(torch.autograd.Function):
    """W [T][B] from Omega_m (0-d float64) and source parameters [T][3] (float64, host)."""

    @staticmethod
    def forward(ctx, omega_m, params, sources, chi_edges, device):
        srcs = [s.with_params(params[t].tolist()) for t, s in enumerate(sources)]
        W, dW = lensing_weights(float(omega_m), srcs, chi_edges, with_derivatives=True, device=device)
        ctx.save_for_backward(dW)
        ctx.host_device = omega_m.device
        return W

    @staticmethod
    def backward(ctx, grad_W):
        (dW,) = ctx.saved_tensors
        gt = lensing_weights_vjp(dW, grad_W).to(ctx.host_device)
        return gt[:, 0].sum(), gt[:, 1:], None, None, None


# ---------------------------------------------------------------- batched

def _batch_items(items):
    """ctypes array of ufalcon_batch_item for the binding's item dicts (plus the host
    buffers that must outlive the call)."""
    keep = []
    arr = (BatchItem * len(items))()
    dtype = None
    for k, it in enumerate(items):
        e, ne = _host_doubles(it["chi_edges"])
        keep.append(e)
        obs = it.get("observer") or (0.5 * it["box_L"],) * 3
        x, y, z = it["x"], it["y"], it["z"]
        dtype = _dtype_code(x.dtype)
        arr[k].x, arr[k].y, arr[k].z = x.data_ptr(), y.data_ptr(), z.data_ptr()
        arr[k].n = x.numel()
        for j in range(3):
            arr[k].observer[j] = float(obs[j])
        arr[k].box_L = float(it["box_L"])
        arr[k].n_rep = int(it.get("n_rep", 0))
        arr[k].n_shells = ne - 1
        arr[k].shell_begin = int(it.get("shell_begin", 0))
        arr[k].shell_end = int(it.get("shell_end", ne - 1))
        arr[k].chi_edges = e
        arr[k].counts = it["counts"].data_ptr()
        arr[k].W = it["W"].data_ptr() if it.get("W") is not None else None
        arr[k].inv_nbar = it["inv_nbar"].data_ptr() if it.get("inv_nbar") is not None else None
        arr[k].kappa = it["kappa"].data_ptr() if it.get("kappa") is not None else None
    return arr, dtype, keep


ACCUMULATION_NAMES = {0: "partition", 1: "atomic", 3: "partition-one-stream"}
_ACCUMULATION_CODES = {"partition": 0, "atomic": 1, "auto": 2, "partition-one-stream": 3}


def save_tuning(path):
    """Write the autotuner's cached choices to `path` (one JSON object per line)."""
    _check(load().ufalcon_batch_tuning_save(os.fsencode(path)), "ufalcon_batch_tuning_save")


def load_tuning(path):
    """Add the choices saved in `path` to the autotuner's cache; returns how many were read."""
    n = ctypes.c_int32(0)
    _check(load().ufalcon_batch_tuning_load(os.fsencode(path), ctypes.byref(n)), "ufalcon_batch_tuning_load")
    return n.value


def autotune_batch(items, nside, T=1, out_dtype=torch.float32, sample_items=0):
    """Time the batched form's candidate configurations on (the first sample_items of)
    these realisations and record the fastest for BatchPlan(method="auto").  Overwrites
    the sampled realisations' counts and kappa.  Returns the tuning record as a dict."""
    lib = load()
    arr, dtype, keep = _batch_items(items)
    tun = Tuning()
    _check(lib.ufalcon_batch_autotune(arr, len(items), dtype, int(nside), int(T), _dtype_code(out_dtype),
                                      int(sample_items), ctypes.byref(tun), _stream()), "ufalcon_batch_autotune")
    names = ACCUMULATION_NAMES
    cands = [{"method": names[tun.cand_accumulation[i]], "tile": int(tun.cand_tile[i]),
              "persistent_wgs": int(tun.cand_wgs[i]), "ms": float(tun.ms[i])} for i in range(tun.n_tried)]
    return {"method": names[tun.accumulation], "tile": int(tun.tile), "persistent_wgs": int(tun.persistent_wgs),
            "best": int(tun.best), "candidates": cands}


class BatchPlan:
    """Many realisations binned by one persistent launch and reduced by one batched Born launch.

    items: list of dicts with keys x, y, z (device), chi_edges (host), box_L, n_rep,
    observer (optional), shell_begin/shell_end (optional), counts (uint32 device),
    and for the Born pass W, inv_nbar, kappa (device).
    """

    def __init__(self, items, nside, T=1, out_dtype=torch.float32, tile=0, persistent_wgs=0, method="partition"):
        lib = load()
        arr, dtype, self._keep = _batch_items(items)
        self.items = items
        handle = ctypes.c_void_p()
        acc = _ACCUMULATION_CODES[method]
        _check(lib.ufalcon_batch_plan_create(arr, len(items), dtype, int(nside), int(T), _dtype_code(out_dtype),
                                             int(tile), int(persistent_wgs), acc, ctypes.byref(handle)),
               "ufalcon_batch_plan_create")
        self.handle = handle

    def clear(self):
        _check(load().ufalcon_batch_clear(self.handle, _stream()), "ufalcon_batch_clear")

    def bin(self, status=None):
        _check(load().ufalcon_bin_shells_batched(self.handle, _ptr(status), _stream()), "ufalcon_bin_shells_batched")

    def born(self):
        _check(load().ufalcon_born_kappa_batched(self.handle, _stream()), "ufalcon_born_kappa_batched")

    def run_graph(self, status=None):
        _check(load().ufalcon_batch_run_graph(self.handle, _ptr(status), _stream()), "ufalcon_batch_run_graph")

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.ufalcon_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
