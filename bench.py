"""Throughput of the shell-binning + Born-convergence hot path on one MI355X.

Headline workload (the largest single-GPU configuration, timed for --steps):
  16 realisations with uneven particle counts N_r ~ U[2^26, 2^28] (seeded
  lognormal fields, sigma_ln = 1 on a 256^3 grid, multinomial placement, FP32,
  1 Gpc/h box replicated to z = 1.0, images {-2..2}^3) and per-realisation
  shell sets B_r ~ U{20..60} over z = 0.1 .. 1.0, HEALPix Nside 1024, delta
  source at z = 1.0, flat LCDM Omega_m = 0.3.
  step = per realisation: lensing weights (+ derivatives) and 1/nbar, then one
         replay of the batch plan's HIP graph (clear + bin every realisation +
         batched Born kappa, FP32), then per realisation dL/dkappa for
         L = sum kappa^2, the adjoint and the weights VJP (dL/dOmega_m, dL/dz_s).
  value = input particles binned per second over the whole step.
  The same step as 16 sequences of plain calls gives the plain maps/s.

Also measured (each after the headline, with its own repetitions):
  config1  2^18 FP64 uniform particles, 10 shells to 250 Mpc/h, Nside 64, no
           replication, source z = 0.3; int64 count maps (widened on the device)
           and FP64 kappa: absolute time per step;
  config2  2^27 lognormal particles, 30 shells z = 0.1-0.5, Nside 1024, Smail
           n(z): one plain step, particle order shuffled and cell-ordered, with
           the phases of the binning call;
  config4  nested full-sky lightcone z = 0.1-1.5, 47 shells, Nside 2048: inner
           1 Gpc/h box (768^3) for z < 0.6, outer 3 Gpc/h box (768^3) beyond,
           positions streamed from pinned host memory in 2^28-particle chunks
           (copies on a second stream overlapped with binning), four Smail
           tomographic bins;
  config5  150 realisations of 256^3 particles, 40 shells z = 0.1-1.5, Nside 512:
           forward (one batch-plan graph) and backward of L = sum_r sum_p kappa_r^2
           to the weights, Omega_m and z0;
  spectra  map2alm / C_l of a kappa map, covariance of 150 spectra, smoothing
           and moments (the consumers of the maps).

roofline: the dominant kernel of the headline, the FP64 decision pass
(keys_kernel: shell and RING pixel of every image), timed with HIP events that
the library records on the stream the kernel runs on (one phase-timed plain
pass over the 16 realisations).  cpu_baseline: the oracle on one host core on
a bounded sample of the headline workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s binned to HEALPix shells; kappa maps/s batched vs plain, Δ≤1e-5·RMS"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # vector FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions per second (4 cycles each per SIMD)

# Algorithmic FP64 operations of the decision pass, counted from the operations
# the fast path performs (add, multiply, divide, square root, floor: 1; FMA: 2):
#   per image tested:   d_z = (x_z - o_z) + s_z L and r^2 against the range -> 4
#   per decided instance: radius and shell guards, then the RING pixel
#   (rho^2, z, |z| = 2/3 test, sqrt, azimuth with one division and a degree-9
#   polynomial, the shared division, floors with their guards)      -> 80
FLOPS_PER_IMAGE = 4
FLOPS_PER_INSTANCE = 80

# The files keys_kernel is compiled from: partition.hip and what it includes.
KEYS_KERNEL_SOURCES = ("paper_1801_05745_amd/csrc/partition.hip", "paper_1801_05745_amd/csrc/binning_core.hpp",
                       "paper_1801_05745_amd/csrc/common.hpp", "paper_1801_05745_amd/csrc/exact.hpp",
                       "paper_1801_05745_amd/csrc/internal.hpp", "paper_1801_05745_amd/csrc/ring.hpp",
                       "include/ufalcon.h")

# HBM bytes of keys_kernel on the headline workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB summed over the dispatches of one pass over
# the 16 realisations) scaled by what the same counters read for a 1 GiB device
# copy (FETCH_SIZE x fetch_scale, WRITE_SIZE x write_scale).  Reported only while
# the kernel's sources hash to the value the counters were taken on.
PMC_TRAFFIC = {
    "kernel": "keys_kernel<float>",
    "fetch_kib": 15471282.25,
    "write_kib": 549916290.16,
    "fetch_scale": 1.99995,
    "write_scale": 1.0,
    "sources_sha1": "fd858db964fa5452729b193aa187fa45afc6f4e3",
    "profile": "profiles/keys_kernel_batched16_nside1024_pmc.md",
}


def sources_sha1():
    """sha1 over the sources of keys_kernel (KEYS_KERNEL_SOURCES)."""
    import hashlib

    h = hashlib.sha1()
    for f in sorted(os.path.join(ROOT, f) for f in KEYS_KERNEL_SOURCES):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    t = PMC_TRAFFIC
    if t["fetch_kib"] is None or t["sources_sha1"] != sources_sha1():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


ALL_PARTS = ("batched_cell", "config1", "config2", "config4", "config5", "spectra")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", choices=["shuffled", "cell"], default="shuffled",
                    help="particle order of the headline catalogues")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of the secondary parts to run after the headline "
                         f"({', '.join(ALL_PARTS)}; 'none' for the headline alone)")
    ap.add_argument("--no-plain", action="store_true", help="skip the 16 plain call sequences")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 21)
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the secondary parts named by --only (for profiling them); no metric line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only the 1 GiB device copy (the reference kernel that scales the HBM counters)")
    return ap.parse_args()


def sht_flops(nside, lmax):
    """Algorithmic FP64 flops of one spherical-harmonic analysis or synthesis at
    Nside, lmax, fixed by the transform (not by a kernel variant): every ring of
    n = 4 n4 pixels as four direct length-n4 DFTs (4 flops per real-by-complex
    multiply-add: 16 n4^2 per ring), and the Legendre step, 7 flops per (l, m,
    ring pair): the three-term recurrence (3) and the complex multiply-add with
    the folded ring sums (4)."""
    N = nside
    n_alm = (lmax + 1) * (lmax + 2) // 2
    legendre = 7 * n_alm * 2 * N
    dft = (2 * N + 1) * 16 * N * N + 2 * sum(16 * i * i for i in range(1, N))
    return float(legendre + dft)


def sht_flops_executed(nside, lmax, inverse=False):
    """The flops the kernels execute: the ring DFTs divided by their number K of
    output classes (equatorial rings: K = 4 when 4 | Nside, 2 when Nside is even,
    and for the inverse 8 when 8 | Nside, with complex sums from K = 4 on; polar
    rings: K = 2 on even rings), plus the same Legendre step."""
    N = nside
    n_alm = (lmax + 1) * (lmax + 2) // 2
    legendre = 7 * n_alm * 2 * N
    if inverse:
        k_eq = 8 if N % 8 == 0 else (4 if N % 4 == 0 else (2 if N % 2 == 0 else 1))
        dft_eq = (2 * N + 1) * 16 * N * N // k_eq * (2 if k_eq >= 4 else 1)
    else:
        k_eq = 4 if N % 4 == 0 else (2 if N % 2 == 0 else 1)
        dft_eq = (2 * N + 1) * 16 * N * N // k_eq
    dft_polar = sum(2 * 16 * i * i // (2 if i % 2 == 0 else 1) for i in range(1, N))
    return float(legendre + dft_eq + dft_polar)


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "nproc": avail, "cpu_count": os.cpu_count()}


def copy_bandwidth(dev):
    """Measured device-to-device copy of 1 GiB (read + write bytes / time)."""
    import torch

    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return {"bytes": 8 * n, "ms": ms, "GBs": 8 * n / (ms / 1e3) / 1e9}


def radius_reps(edges, L):
    """Smallest R with images {-R..R}^3 of [0, L)^3 covering the ball of the outer edge around the centre."""
    R = 0
    for oj in (L / 2,) * 3:
        R = max(R, -math.floor((oj - edges[-1]) / L), math.floor((oj + edges[-1]) / L))
    return R


def free_device():
    import torch

    import paper_1801_05745_amd as uf

    uf.release_workspaces()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- headline (batched, 16 realisations)

TUNE_SAMPLE = 4  # realisations the headline's autotuner times each candidate on


def batched16(dev, args, order=None, steps=None, warmup=None, plain_reps=2, roofline=True):
    import torch

    import paper_1801_05745_amd as uf
    import synth

    L, nside, om, zs = 1000.0, 1024, 0.3, 1.0
    M = 1 << 20
    sizes = synth.randint(16, 64 * M, 256 * M, seed=0, stream=900)
    shells = synth.randint(16, 20, 60, seed=0, stream=901)
    t0 = time.time()
    items = []
    for r in range(16):
        x, y, z = synth.lognormal_box(sizes[r], L, seed=r, ngrid=256, dtype=torch.float32, device=dev,
                                      order=order or args.order)
        zg = torch.linspace(0.1, 1.0, shells[r] + 1, dtype=torch.float64, device=dev)
        edges = uf.comoving_distance(zg, om).cpu().tolist()
        R = radius_reps(edges, L)
        items.append(dict(x=x, y=y, z=z, n=sizes[r], chi_edges=edges, box_L=L, n_rep=R,
                          counts=torch.empty((shells[r], uf.npix(nside)), dtype=torch.uint32, device=dev),
                          W=torch.empty((1, shells[r]), dtype=torch.float64, device=dev),
                          inv_nbar=torch.empty(shells[r], dtype=torch.float64, device=dev),
                          kappa=torch.empty((1, uf.npix(nside)), dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"headline: 16 realisations generated in {gen_s:.1f} s ({sum(sizes)} particles)")
    src = uf.SourceSpec("delta", z_s=zs)
    outs = {}

    def scalars():
        for it in items:
            W, dW = uf.lensing_weights(om, [src], it["chi_edges"], with_derivatives=True, device=dev)
            it["W"].copy_(W)
            it["dW"] = dW
            uf.inv_nbar(it["n"], L, it["chi_edges"], nside, out=it["inv_nbar"])

    scalars()
    t0 = time.time()
    # four realisations: the persistent atomic kernel gains on longer batches, and a
    # two-item sample under-rates it against the per-item partitioned pipeline
    tuning = uf.autotune_batch(items, nside, T=1, sample_items=TUNE_SAMPLE)
    tune_s = time.time() - t0
    log(f"headline: autotuned in {tune_s:.1f} s -> {tuning['method']}")
    plan = uf.BatchPlan(items, nside, T=1, method="auto")
    status = uf.new_status(dev)

    def backward(kappas):
        gth = []
        for it, kap in zip(items, kappas):
            gW = uf.born_kappa_adjoint(it["counts"], it["inv_nbar"], kap * 2.0)  # dL/dkappa of L = sum kappa^2
            gth.append(uf.lensing_weights_vjp(it["dW"], gW))
        outs["gth"] = gth

    def step():
        scalars()
        plan.run_graph(status)
        backward([it["kappa"] for it in items])

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    status.zero_()
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms_per_step = 1e3 * wall / steps
    st = uf.status_dict(status)
    log(f"batched16 ({order or args.order}): {ms_per_step:.1f} ms per step")
    n_total = sum(sizes)
    inst = st["n_instances"] / steps
    kap = torch.cat([it["kappa"].double() for it in items], 0)
    rms = kap.pow(2).mean(dim=1).sqrt()
    max_over_rms = float((kap.abs().max(dim=1).values / rms).max())
    del kap

    # the batched step's outputs, compared below with the plain calls' (same inputs, same kernels)
    batched_kappa = [it["kappa"].clone() for it in items]
    batched_grad = [g.clone() for g in outs["gth"]]

    # plain: the same step as 16 sequences of single-map calls (one shared workspace)
    plain = None
    match = None
    ws = None
    if not args.no_plain and (plain_reps > 0 or roofline):
        ws = uf.partition_workspace(max(sizes), max(it["n_rep"] for it in items), max(shells), nside, device=dev)
    if ws is not None and plain_reps > 0:

        def plain_step():
            kappas = []
            for it in items:
                uf.fill_u32(it["counts"], 0)
                uf.bin_shells(it["x"], it["y"], it["z"], it["chi_edges"], nside, box_L=L, n_rep=it["n_rep"],
                              counts=it["counts"], workspace=ws)
                W, dW = uf.lensing_weights(om, [src], it["chi_edges"], with_derivatives=True, device=dev)
                it["dW"] = dW
                inb = uf.inv_nbar(it["n"], L, it["chi_edges"], nside, device=dev)
                kappas.append(uf.born_kappa(it["counts"], W, inb))
            backward(kappas)
            outs["plain_kappa"] = kappas

        plain_step()
        torch.cuda.synchronize()
        reps = plain_reps
        t1 = time.perf_counter()
        for _ in range(reps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - t1) / reps
        log(f"headline: plain {plain_ms:.1f} ms per batch")
        plain = {"ms_per_batch": plain_ms, "maps_per_s": 16e3 / plain_ms, "reps": reps}
        match = {"kappa": all(torch.equal(a, b) for a, b in zip(batched_kappa, outs["plain_kappa"])),
                 "grad": all(torch.equal(a, b) for a, b in zip(batched_grad, outs["gth"]))}
        if not (match["kappa"] and match["grad"]):
            log(f"headline: batched and plain outputs differ: {match}")
        del outs["plain_kappa"]
    del batched_kappa, batched_grad

    if roofline and ws is not None:
        # the dominant kernel, timed on its own stream by the library's phase events:
        # one phase-timed plain binning pass over the 16 realisations
        phases = {name: 0.0 for name in uf.PHASES}
        launches = 0
        timer = uf.PhaseTimer(dev)
        for it in items:
            uf.fill_u32(it["counts"], 0)
            uf.bin_shells(it["x"], it["y"], it["z"], it["chi_edges"], nside, box_L=L, n_rep=it["n_rep"],
                          counts=it["counts"], workspace=ws, timer=timer)
            for k, v in timer.read().items():
                phases[k] += v
            launches += timer.intervals()["decide"]
        timer.close()
    del ws
    plan.close()
    images = sum(it["n"] * (2 * it["n_rep"] + 1) ** 3 for it in items)
    flops = FLOPS_PER_IMAGE * images + FLOPS_PER_INSTANCE * inst
    bin_bytes = sum(12 * it["n"] + 4 * it["counts"].numel() for it in items)
    res = {
        "ms_per_step": ms_per_step, "particles": n_total, "instances_per_step": inst, "images": images,
        "order": order or args.order, "steps": steps,
        "guarded_per_step": st["n_guarded"] / steps, "unresolved": st["n_unresolved"],
        "fallback": st["n_fallback"], "kappa_max_over_rms": max_over_rms, "shells": shells,
        "maps_per_s_batched": 16e3 / ms_per_step, "plain": plain,
        "batched_equals_plain": match,
        "tuning": {"method": tuning["method"], "tile": tuning["tile"], "persistent_wgs": tuning["persistent_wgs"],
                   "candidates": tuning["candidates"], "tune_s": tune_s, "sample_items": TUNE_SAMPLE},
        "input_generation_s": gen_s,
    }
    if roofline and not args.no_plain:
        res["phases_ms"] = phases
        res["decide_ms"] = phases["decide"]
        res["decide_launches"] = launches
        res["algorithmic_flops"] = flops
        res["bin_bytes"] = bin_bytes
    cpu_sample = None
    if roofline and not args.no_cpu_baseline:
        it = items[0]
        m = min(args.cpu_sample, it["n"])
        cpu_sample = dict(x=it["x"][:m].cpu().numpy(), y=it["y"][:m].cpu().numpy(), z=it["z"][:m].cpu().numpy(),
                          edges=it["chi_edges"], L=L, R=it["n_rep"], nside=nside, m=m, n_rep=it["n_rep"])
    items.clear()
    free_device()
    return res, cpu_sample


def cpu_baseline(sample):
    """The oracle (plain single-threaded FP64 C loop + exact resolver) on the first
    `m` particles of the headline's realisation 0, one host core."""
    from oracle import binning as obin

    s = sample
    L = s["L"]
    t0 = time.perf_counter()
    counts, st = obin.bin_shells(s["x"], s["y"], s["z"], (L / 2,) * 3, L, s["R"], s["edges"], s["nside"], threads=1)
    dt = time.perf_counter() - t0
    return {"value": s["m"] / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {s['m']} particles of the headline's realisation 0 ({len(s['edges']) - 1} shells "
                      f"z = 0.1-1.0, Nside {s['nside']}, images {{-{s['R']}..{s['R']}}}^3); "
                      f"{st['instances']} instances in {dt:.1f} s on one core",
            "instances_per_s": st["instances"] / dt, "host": cpu_info()}


# ---------------------------------------------------------------- config 1

def config1(dev):
    """2^18 FP64 uniform particles in a 500 Mpc/h cube, 10 shells to 250 Mpc/h, Nside 64, R = 0,
    delta source z = 0.3: bin + int64 widening + weights + FP64 kappa + adjoint, absolute time."""
    import torch

    import paper_1801_05745_amd as uf
    import synth

    L, nside, n = 500.0, 64, 1 << 18
    x, y, z = synth.uniform_box(n, L, seed=0, dtype=torch.float64, device=dev)
    edges = [25.0 * k for k in range(11)]
    src = uf.SourceSpec("delta", z_s=0.3)
    counts = uf.new_counts(10, nside, dev)
    c64 = torch.empty((10, uf.npix(nside)), dtype=torch.int64, device=dev)
    ws = uf.partition_workspace(n, 0, 10, nside, device=dev)
    out = {}

    def step():
        uf.fill_u32(counts, 0)
        uf.bin_shells(x, y, z, edges, nside, box_L=L, n_rep=0, counts=counts, workspace=ws)
        uf.counts_to_i64(counts, out=c64)
        W = uf.lensing_weights(0.3, [src], edges, device=dev)
        # exact-volume nbar is finite for the first shell (chi_0 = 0)
        inb = uf.inv_nbar(n, L, edges, nside, device=dev)
        kap = uf.born_kappa(counts, W, inb, out_dtype=torch.float64)
        out["gW"] = uf.born_kappa_adjoint(counts, inb, 2.0 * kap)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    times = []
    for _ in range(20):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    times.sort()
    med = times[len(times) // 2]
    res = {"workload": "2^18 FP64 uniform particles, 500 Mpc/h cube, 10 shells to 250 Mpc/h, Nside 64, no "
                       "replication, delta source z = 0.3; int64 counts + FP64 kappa + adjoint",
           "ms_per_step_median": med, "ms_min": times[0], "reps": len(times),
           "particles_per_s": n / (med / 1e3), "instances": int(c64.sum())}
    del x, y, z, counts, c64, ws, out
    free_device()
    return res


# ---------------------------------------------------------------- config 2

def config2(dev, order, steps=8, warmup=2):
    import torch

    import paper_1801_05745_amd as uf
    import synth

    L, nside, om, n = 1000.0, 1024, 0.3, 1 << 27
    t0 = time.time()
    x, y, z = synth.lognormal_box(n, L, seed=0, ngrid=256, dtype=torch.float32, device=dev, order=order)
    zg = torch.linspace(0.1, 0.5, 31, dtype=torch.float64, device=dev)
    edges = uf.comoving_distance(zg, om).cpu().tolist()
    B = len(edges) - 1
    R = radius_reps(edges, L)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    src = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=0.3, z_max=0.5)
    counts = torch.empty((B, uf.npix(nside)), dtype=torch.uint32, device=dev)
    status = uf.new_status(dev)
    ws = uf.partition_workspace(n, R, B, nside, device=dev)
    stream = torch.cuda.current_stream(dev)
    timers = [uf.PhaseTimer(dev) for _ in range(steps)]
    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
          for k in ("b0", "b1")}
    outs = {}

    def step(k=None):
        rec = (lambda name: ev[name][k].record(stream)) if k is not None else (lambda name: None)
        uf.fill_u32(counts, 0)
        rec("b0")
        uf.bin_shells(x, y, z, edges, nside, box_L=L, n_rep=R, counts=counts, status=status, workspace=ws,
                      timer=timers[k] if k is not None else None)
        rec("b1")
        W, dW = uf.lensing_weights(om, [src], edges, with_derivatives=True, device=dev)
        inb = uf.inv_nbar(n, L, edges, nside, device=dev)
        kap = uf.born_kappa(counts, W, inb, out_dtype=torch.float32)
        g = kap * 2.0
        gW = uf.born_kappa_adjoint(counts, inb, g)
        outs.update(kappa=kap, gth=uf.lensing_weights_vjp(dW, gW), inb=inb)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    status.zero_()
    t1 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / steps
    avg = lambda a, b: sum(p.elapsed_time(q) for p, q in zip(ev[a], ev[b])) / steps
    bin_ms = avg("b0", "b1")
    # the streaming kernels timed as back-to-back calls, so that the host's
    # argument checks between the events never leave the GPU idle
    g = outs["kappa"] * 2.0
    W = uf.lensing_weights(om, [src], edges, device=dev)

    def b2b(fn, reps=20):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    born_ms = b2b(lambda: uf.born_kappa(counts, W, outs["inb"], out_dtype=torch.float32))
    adj_ms = b2b(lambda: uf.born_kappa_adjoint(counts, outs["inb"], g))
    st = uf.status_dict(status)
    inst = st["n_instances"] / steps
    ph = [t.read() for t in timers]
    phases = {name: sum(p[name] for p in ph) / len(ph) for name in uf.PHASES}
    for t in timers:
        t.close()
    # projected overdensity (eq. (7)) of the last map: the same streaming pass with chi weights
    uf.overdensity(counts, edges, outs["inb"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        uf.overdensity(counts, edges, outs["inb"])
    e1.record(stream)
    torch.cuda.synchronize()
    od_ms = e0.elapsed_time(e1) / 3
    images = n * (2 * R + 1) ** 3
    flops = FLOPS_PER_IMAGE * images + FLOPS_PER_INSTANCE * inst
    bin_bytes = 3 * 4 * n + 4 * B * uf.npix(nside)
    born_bytes = 4 * B * uf.npix(nside) + 4 * uf.npix(nside)
    kap = outs["kappa"].double()
    rms = float(kap.pow(2).mean().sqrt())
    res = {
        "workload": f"2^27 lognormal FP32 particles, 1 Gpc/h box replicated to z=0.5 (images {{-{R}..{R}}}^3), "
                    "30 shells z=0.1-0.5, Nside 1024, Smail n(z); bin + weights + Born + adjoint per step",
        "order": order, "ms_per_step": ms, "particles_per_s": n / (ms / 1e3),
        "instances_per_step": inst, "instances_per_s": inst / (ms / 1e3),
        "binning": {"ms": bin_ms, "phases_ms": phases, "algorithmic_bytes": bin_bytes,
                    "frac_hbm": bin_bytes / (bin_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "decide": {"ms": phases["decide"], "achieved_TFLOPs": flops / (phases["decide"] / 1e3) / 1e12,
                   "frac_fp64": flops / (phases["decide"] / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                   "algorithmic_flops": flops},
        "born": {"ms": born_ms, "GBs": born_bytes / (born_ms / 1e3) / 1e9,
                 "frac_hbm": born_bytes / (born_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "adjoint": {"ms": adj_ms, "GBs": born_bytes / (adj_ms / 1e3) / 1e9,
                    "frac_hbm": born_bytes / (adj_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "overdensity": {"ms": od_ms, "GBs": born_bytes / (od_ms / 1e3) / 1e9,
                        "frac_hbm": born_bytes / (od_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "guarded_per_step": st["n_guarded"] / steps, "unresolved": st["n_unresolved"],
        "fallback": st["n_fallback"], "kappa_max_over_rms": float(kap.abs().max()) / rms,
        "input_generation_s": gen_s, "steps": steps,
    }
    kappa_map = outs["kappa"][0].clone() if order == "shuffled" else None
    del x, y, z, counts, ws, outs, kap
    free_device()
    return res, kappa_map


# ---------------------------------------------------------------- config 4

def config4(dev, reps=2):
    """Nested lightcone streamed from pinned host memory in 2^28-particle chunks."""
    import numpy as np
    import torch

    import paper_1801_05745_amd as uf
    import synth

    om, nside, n, chunk = 0.3, 2048, 768 ** 3, 1 << 28
    zs = np.linspace(0.1, 1.5, 48)
    split = int(np.nonzero(zs >= 0.6)[0][0])
    edges = uf.comoving_distance(torch.tensor(zs, dtype=torch.float64, device=dev), om).cpu().tolist()
    B = len(edges) - 1
    t0 = time.time()
    boxes = []
    for seed, L, b0, b1 in ((0, 1000.0, 0, split), (1, 3000.0, split, B)):
        host = []
        for t in synth.lognormal_box(n, L, seed=seed, ngrid=256, dtype=torch.float32, device=dev):
            h = torch.empty(n, dtype=torch.float32, pin_memory=True)
            h.copy_(t)
            host.append(h)
            del t
        R = radius_reps(edges[:b1 + 1], L)
        boxes.append(dict(host=host, L=L, b0=b0, b1=b1, R=R))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    gen_s = time.time() - t0
    log(f"config4: catalogues in pinned host memory ({gen_s:.1f} s)")
    z0s = (0.3, 0.5, 0.7, 0.9)
    srcs = [uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=z0, z_max=1.5) for z0 in z0s]
    counts = torch.empty((B, uf.npix(nside)), dtype=torch.uint32, device=dev)
    status = uf.new_status(dev)
    streamer = uf.HostStream(chunk, max(b["R"] for b in boxes), B, nside, device=dev)
    feed = [dict(x=b["host"][0], y=b["host"][1], z=b["host"][2], box_L=b["L"], n_rep=b["R"], shell_begin=b["b0"],
                 shell_end=b["b1"]) for b in boxes]
    out = {}
    copy_ms = []

    def step(record=False):
        uf.fill_u32(counts, 0)
        streamer.run(feed, edges, nside, counts, status=status)
        W, dW = uf.lensing_weights(om, srcs, edges, with_derivatives=True, device=dev)
        inb = torch.cat([uf.inv_nbar(n, b["L"], edges[b["b0"]:b["b1"] + 1], nside, device=dev) for b in boxes])
        kap = uf.born_kappa(counts, W, inb, out_dtype=torch.float32)
        gW = uf.born_kappa_adjoint(counts, inb, 2.0 * kap)
        out.update(kappa=kap, gth=uf.lensing_weights_vjp(dW, gW))
        if record:
            copy_ms.append(streamer.copy_ms())

    step()
    torch.cuda.synchronize()
    status.zero_()
    t1 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / reps
    st = uf.status_dict(status)
    step(record=True)
    h2d_ms = copy_ms[-1]
    h2d_bytes = 12 * 2 * n
    kap = out["kappa"].double()
    rms = kap.pow(2).mean(dim=1).sqrt()
    res = {"workload": "nested lightcone z=0.1-1.5, 47 shells, Nside 2048: 768^3 in 1 Gpc/h (z<0.6) + 768^3 in "
                       "3 Gpc/h, streamed from pinned host memory in 2^28-particle chunks, 4 Smail bins; "
                       "bin + weights + Born (T=4) + adjoint per step",
           "ms_per_step": ms, "particles": 2 * n, "particles_per_s": 2 * n / (ms / 1e3),
           "instances_per_step": st["n_instances"] / reps, "instances_per_s": st["n_instances"] / reps / (ms / 1e3),
           "h2d": {"bytes": h2d_bytes, "ms_copy_stream": h2d_ms, "GBs": h2d_bytes / (h2d_ms / 1e3) / 1e9,
                   "overlapped": "copies of chunk k+1 on a second stream while chunk k is binned"},
           "chunks": sum((n + chunk - 1) // chunk for _ in boxes), "unresolved": st["n_unresolved"],
           "fallback": st["n_fallback"],
           "kappa_max_over_rms": float((kap.abs().max(dim=1).values / rms).max()),
           "input_generation_s": gen_s, "reps": reps}
    del boxes, feed, streamer, counts, out, kap
    free_device()
    return res


# ---------------------------------------------------------------- config 5

def config5(dev, reps=2):
    """150 realisations of 256^3 particles: forward (one graph) and backward of L = sum kappa^2."""
    import torch

    import paper_1801_05745_amd as uf
    import synth

    L, nside, om, n, R_real = 1000.0, 512, 0.3, 256 ** 3, 150
    zg = torch.linspace(0.1, 1.5, 41, dtype=torch.float64, device=dev)
    edges = uf.comoving_distance(zg, om).cpu().tolist()
    B = len(edges) - 1
    R = radius_reps(edges, L)
    t0 = time.time()
    base = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=0.3, z_max=1.5)
    W = torch.empty((1, B), dtype=torch.float64, device=dev)
    inb = uf.inv_nbar(n, L, edges, nside, device=dev)
    items = []
    for r in range(R_real):
        x, y, z = synth.lognormal_box(n, L, seed=r, ngrid=256, dtype=torch.float32, device=dev)
        items.append(dict(x=x, y=y, z=z, chi_edges=edges, box_L=L, n_rep=R,
                          counts=torch.empty((B, uf.npix(nside)), dtype=torch.uint32, device=dev),
                          W=W, inv_nbar=inb, kappa=torch.empty((1, uf.npix(nside)), dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"config5: 150 realisations generated in {gen_s:.1f} s")
    W.copy_(uf.lensing_weights(om, [base], edges, device=dev))
    tuning = uf.autotune_batch(items, nside, T=1, sample_items=4)
    plan = uf.BatchPlan(items, nside, T=1, method="auto")
    status = uf.new_status(dev)
    out = {}

    def step():
        om_t = torch.tensor(om, dtype=torch.float64, requires_grad=True)
        params = torch.tensor([base.params()], dtype=torch.float64, requires_grad=True)
        Wt = uf.LensingWeights.apply(om_t, params, [base], edges, dev)
        with torch.no_grad():
            W.copy_(Wt)
        plan.run_graph(status)                       # forward: bin + Born for all realisations
        gW = torch.zeros_like(Wt)
        for it in items:                             # backward of L = sum_r sum_p kappa_r^2
            gW += uf.born_kappa_adjoint(it["counts"], inb, 2.0 * it["kappa"])
        Wt.backward(gW)
        out.update(g_om=om_t.grad, g_z0=params.grad[0, 2])

    step()
    torch.cuda.synchronize()
    status.zero_()
    t1 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / reps
    st = uf.status_dict(status)
    t1 = time.perf_counter()
    plan.run_graph(status)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t1)
    plan.close()
    check = [0, R_real // 2, R_real - 1]
    batched_kappa = [items[r]["kappa"].clone() for r in check]
    # the same forward pass as 150 plain calls (one shared workspace)
    ws = uf.partition_workspace(n, R, B, nside, device=dev)

    def plain_forward():
        for it in items:
            uf.fill_u32(it["counts"], 0)
            uf.bin_shells(it["x"], it["y"], it["z"], edges, nside, box_L=L, n_rep=R, counts=it["counts"],
                          workspace=ws)
            it["kappa"].copy_(uf.born_kappa(it["counts"], W, inb))

    plain_forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain_forward()
    torch.cuda.synchronize()
    plain_fwd_ms = 1e3 * (time.perf_counter() - t1)
    batched_equals_plain = all(torch.equal(a, items[r]["kappa"]) for a, r in zip(batched_kappa, check))
    del ws, batched_kappa
    res = {"workload": "150 realisations x 256^3 lognormal FP32 particles, 1 Gpc/h box, 40 shells z=0.1-1.5, "
                       "Nside 512, images {-3..3}^3, Smail n(z); forward (batch-plan graph: bin + Born) + backward "
                       "(adjoint of L = sum kappa^2 to W, Omega_m, z0)",
           "ms_per_step": ms, "maps_per_s": R_real * 1e3 / ms, "particles_per_s": R_real * n / (ms / 1e3),
           "instances_per_step": st["n_instances"] / reps,
           "instances_per_s": st["n_instances"] / reps / (ms / 1e3),
           "unresolved": st["n_unresolved"], "fallback": st["n_fallback"],
           "dL_dOmega_m": float(out["g_om"]), "dL_dz0": float(out["g_z0"]),
           "tuning": {"method": tuning["method"], "candidates_ms": [round(c["ms"], 2) for c in tuning["candidates"]],
                      "sample_items": 4},
           "forward_batched_ms": fwd_ms,
           "batched_equals_plain": {"kappa_realisations": check, "equal": batched_equals_plain}, "forward_batched_maps_per_s": R_real * 1e3 / fwd_ms,
           "forward_plain_ms": plain_fwd_ms, "forward_plain_maps_per_s": R_real * 1e3 / plain_fwd_ms,
           "input_generation_s": gen_s, "reps": reps}
    del items, plan, out
    free_device()
    return res


# ---------------------------------------------------------------- spectra

def spectra(dev, kmap):
    """Power spectrum of a kappa map (section 3.1), covariance of 150 spectra (3.2),
    smoothing and moments (3.3), each timed on its own."""
    import torch

    import paper_1801_05745_amd as uf
    import synth

    nside = 1024
    lmax = 3 * nside - 1
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    alm = uf.map2alm(kmap, lmax)
    cl = uf.alm2cl(alm, lmax)
    ev[0].record(stream)
    for _ in range(3):
        alm = uf.map2alm(kmap, lmax)
    ev[1].record(stream)
    for _ in range(3):
        cl = uf.alm2cl(alm, lmax)
    ev[2].record(stream)
    torch.cuda.synchronize()
    sht_ms = ev[0].elapsed_time(ev[1]) / 3
    cl_ms = ev[1].elapsed_time(ev[2]) / 3
    fl = sht_flops(nside, lmax)
    jitter = synth.uniform64(150 * (lmax + 1), seed=5, stream=7, device=dev).reshape(150, lmax + 1)
    cls = cl[None, :] * (0.5 + jitter)
    uf.cl_covariance(cls)
    ev[0].record(stream)
    for _ in range(3):
        uf.cl_covariance(cls)
    ev[1].record(stream)
    torch.cuda.synchronize()
    cov_ms = ev[0].elapsed_time(ev[1]) / 3
    sigma = math.radians(10.8 / 60.0)
    beam = uf.gaussian_beam(sigma, lmax, device=dev)
    sm = uf.alm2map(alm, nside, lmax, beam, out_dtype=torch.float32)
    mom = uf.map_moments(sm)
    ev[0].record(stream)
    for _ in range(3):
        sm = uf.alm2map(alm, nside, lmax, beam, out_dtype=torch.float32)
    ev[1].record(stream)
    for _ in range(3):
        mom = uf.map_moments(sm)
    ev[2].record(stream)
    torch.cuda.synchronize()
    a2m_ms = ev[0].elapsed_time(ev[1]) / 3
    mom_ms = ev[1].elapsed_time(ev[2]) / 3
    mom = mom.cpu().tolist()
    res = {
        "nside": nside, "lmax": lmax, "algorithmic_flops_per_transform": fl,
        "executed_flops": {"map2alm": sht_flops_executed(nside, lmax),
                           "alm2map": sht_flops_executed(nside, lmax, inverse=True)},
        "map2alm": {"ms": sht_ms, "TFLOPs": fl / (sht_ms / 1e3) / 1e12,
                    "frac_fp64": fl / (sht_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS},
        "alm2cl_ms": cl_ms, "power_spectra_per_s": 1e3 / (sht_ms + cl_ms),
        "cl_covariance": {"realisations": 150, "multipoles": lmax + 1, "ms": cov_ms},
        "smoothing": {"sigma_arcmin": 10.8, "alm2map_ms": a2m_ms, "TFLOPs": fl / (a2m_ms / 1e3) / 1e12,
                      "frac_fp64": fl / (a2m_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                      "moments_ms": mom_ms, "s2": mom[3], "sigma_s2": math.sqrt(max(mom[4], 0.0))},
    }
    del alm, cls, sm, beam
    free_device()
    return res


# ---------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs the path on "
              f"a single GPU and has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1801_05745_amd as uf

    uf.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only is None:
        parts = set(ALL_PARTS)
    elif args.only == "none":
        parts = set()
    else:
        parts = set(p.strip() for p in args.only.split(","))
        unknown = parts - set(ALL_PARTS)
        if unknown:
            print(f"unknown parts {sorted(unknown)}", file=sys.stderr)
            sys.exit(2)

    copy = copy_bandwidth(dev)
    if args.copy_calibration:
        print(json.dumps({"hbm_copy": copy}), flush=True)
        return
    if args.skip_headline:
        print(json.dumps(secondary(dev, args, parts, {"hbm_copy": copy})), flush=True)
        return
    head, cpu_sample = batched16(dev, args)
    value = head["particles"] / (head["ms_per_step"] / 1e3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batched lightcones: 16 realisations, N_r ~ U[2^26, 2^28] seeded lognormal FP32 particles "
                        "(2.63e9 in total), 1 Gpc/h box replicated to z=1.0 (images {-2..2}^3), B_r ~ U{20..60} "
                        "shells z=0.1-1.0, Nside 1024 RING, delta source z=1.0; per step: weights + 1/nbar, one "
                        "batch-plan graph replay (clear + bin + Born kappa), adjoint + weights VJP",
            "realisations": 16, "particles": head["particles"], "nside": 1024, "order": args.order,
            "accumulation": head["tuning"]["method"], "instances_per_step": head["instances_per_step"],
        },
        "maps_per_s_batched": head["maps_per_s_batched"],
        "maps_per_s_plain": head["plain"]["maps_per_s"] if head["plain"] else None,
        "batched_over_plain": (head["maps_per_s_batched"] / head["plain"]["maps_per_s"]) if head["plain"] else None,
        "instances_per_s": head["instances_per_step"] / (head["ms_per_step"] / 1e3),
    }
    if head["plain"] is not None:
        dec = head["decide_ms"]
        line["roofline"] = {
            "bound": "alu",
            "kernel": "keys_kernel (FP64 shell + RING pixel decision of every image): one launch per key chunk of "
                      "each of the 16 plain calls (launches that find no work left exit at once); achieved = "
                      "algorithmic FLOP of the batch / summed launch time",
            "achieved": head["algorithmic_flops"] / (dec / 1e3) / 1e12,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": head["algorithmic_flops"] / (dec / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(),
            "launch_ms_per_batch": dec,
            "launches_per_batch": head["decide_launches"],
            "avg_launch_ms": dec / head["decide_launches"],
            "algorithmic_flops": head["algorithmic_flops"],
            "flops_per_image": FLOPS_PER_IMAGE, "flops_per_instance": FLOPS_PER_INSTANCE,
            "images": head["images"],
        }
        line["roofline_hbm"] = {
            "bound": "hbm", "kernel": "ufalcon_bin_shells (all kernels of the 16 plain calls)",
            "achieved": head["bin_bytes"] / (sum(head["phases_ms"].values()) / 1e3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["bin_bytes"] / (sum(head["phases_ms"].values()) / 1e3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": head["bin_bytes"], "phases_ms": head["phases_ms"],
        }
    line["headline_detail"] = head
    line["hbm_copy"] = copy
    if not args.no_cpu_baseline and cpu_sample is not None:
        line["cpu_baseline"] = cpu_baseline(cpu_sample)
        log(f"cpu baseline: {line['cpu_baseline']['value']:.3g} particles/s")
    print(json.dumps(secondary(dev, args, parts, line)), flush=True)


def secondary(dev, args, parts, line):
    """The parts after the headline, added to `line`."""
    if "batched_cell" in parts:
        cell, _ = batched16(dev, args, order="cell", steps=3, warmup=1, plain_reps=1, roofline=False)
        line["batched_cell_order"] = {k: cell[k] for k in ("ms_per_step", "maps_per_s_batched", "plain",
                                                           "batched_equals_plain", "tuning",
                                                           "instances_per_step", "fallback", "unresolved")}
    kmap = None
    if "config2" in parts:
        line["config2"], kmap = config2(dev, "shuffled")
        log(f"config2 shuffled: {line['config2']['ms_per_step']:.2f} ms")
        line["config2_cell_order"], _ = config2(dev, "cell")
        log(f"config2 cell: {line['config2_cell_order']['ms_per_step']:.2f} ms")
    if "config1" in parts:
        line["config1"] = config1(dev)
        log(f"config1: {line['config1']['ms_per_step_median']:.2f} ms")
    if "config4" in parts:
        line["config4"] = config4(dev)
        log(f"config4: {line['config4']['ms_per_step']:.1f} ms")
    if "config5" in parts:
        line["config5"] = config5(dev)
        log(f"config5: {line['config5']['ms_per_step']:.1f} ms")
    if "spectra" in parts and kmap is not None:
        line["spectra"] = spectra(dev, kmap)
    return line


if __name__ == "__main__":
    main()
