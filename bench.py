"""Throughput of the shell-binning + Born-convergence hot path on one MI355X.

Workload (one step = the whole path over one catalogue resident in HBM):
  512^3 = 2^27 FP32 particles from a seeded lognormal field (sigma_ln = 1 on a
  256^3 grid, multinomial placement) in a 1 Gpc/h box, replicated to reach z = 0.5;
  30 shells over z = 0.1 .. 0.5 (flat LCDM, Omega_m = 0.3); HEALPix Nside 1024;
  Smail n(z) (alpha 2, beta 1.5, z0 0.3).
  step = clear counts -> bin shells -> lensing weights (+ derivatives) -> 1/nbar
         -> Born kappa (FP32 out) -> dL/dkappa for L = sum kappa^2 -> adjoint
         -> weights VJP (dL/dOmega_m, dL/dz0).

Prints one JSON line.  value = input particles binned per second (whole step).
The roofline object describes the dominant kernel, the FP64 decision pass of
the binning call (keys_kernel: shell and RING pixel of every image), timed with
HIP events that the library records on the stream the kernel runs on; it is
bound by FP64 vector arithmetic (valu_issue: its measured VALU instruction rate
against the issue ceiling).  roofline_hbm gives the whole binning call against
HBM bandwidth, born / overdensity / adjoint the streaming passes.  After the
timed steps the bench also times, each on its own, the power spectrum of the
last kappa map, the covariance of 150 spectra, Gaussian smoothing and the
moments of the smoothed map, and (unless --no-batched) the batched workload of
16 realisations.  cpu_baseline times the oracle on one host core on a bounded
sample of the same catalogue.
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

# Algorithmic FP64 operations of the decision pass, counted from the operations
# the fast path performs (add, multiply, divide, square root, floor: 1; FMA: 2):
#   per image tested:   d_z = (x_z - o_z) + s_z L and r^2 against the range -> 4
#   per decided instance: radius and shell guards, then the RING pixel
#   (rho^2, z, |z| = 2/3 test, sqrt, azimuth with one division and a degree-9
#   polynomial, the shared division, floors with their guards)      -> 80
FLOPS_PER_IMAGE = 4
FLOPS_PER_INSTANCE = 80

# HBM bytes of one keys_kernel launch on this workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same
# counters read for a 1 GiB device copy (FETCH_SIZE reads half: x2.0;
# WRITE_SIZE exact: x1.0).  Valid only for the kernel sources they were taken
# on: the sha1 of the kernel's sources at that time is kept, and a mismatch
# reports traffic null.
PMC_TRAFFIC = {
    "kernel": "keys_kernel<float>",
    "fetch_kib": 786738.0,
    "write_kib": 5073815.0,
    "fetch_scale": 2.0,
    "write_scale": 1.0,
    "sources_sha1": "15ff6b11cc7a090242447e20a2329fbdc9dc3d13",
    "profile": "profiles/keys_kernel_lognormal512_z05_nside1024_pmc.md",
}

# VALU wave instructions of one keys_kernel launch (PMC SQ_INSTS_VALU, same
# workload), against the issue ceiling: one 64-lane VALU instruction occupies a
# SIMD for 4 cycles, so 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 6.14e11 per second.
PMC_VALU = {
    "instructions": 5.065e+09,
    "fp64_instructions": 1.638e+09,
    "sources_sha1": "15ff6b11cc7a090242447e20a2329fbdc9dc3d13",
    "profile": "profiles/keys_kernel_lognormal512_z05_nside1024_instmix.md",
}
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


# The files keys_kernel is compiled from: partition.hip and what it includes.
KEYS_KERNEL_SOURCES = ("paper_1801_05745_amd/csrc/partition.hip", "paper_1801_05745_amd/csrc/binning_core.hpp",
                       "paper_1801_05745_amd/csrc/common.hpp", "paper_1801_05745_amd/csrc/exact.hpp",
                       "paper_1801_05745_amd/csrc/internal.hpp", "paper_1801_05745_amd/csrc/ring.hpp",
                       "include/ufalcon.h")


def sources_sha1():
    """sha1 over the sources of keys_kernel (KEYS_KERNEL_SOURCES)."""
    import hashlib

    h = hashlib.sha1()
    files = sorted(os.path.join(ROOT, f) for f in KEYS_KERNEL_SOURCES)
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    t = PMC_TRAFFIC
    if t["fetch_kib"] is None or t["sources_sha1"] != sources_sha1():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def valu_issue(launch_ms):
    """Measured VALU instruction issue rate of the decision pass against its ceiling
    (null once the library sources differ from those the counters were taken on)."""
    v = PMC_VALU
    if v["sources_sha1"] != sources_sha1():
        return None
    rate = v["instructions"] / (launch_ms / 1e3)
    return {"instructions": v["instructions"], "fp64_share": v["fp64_instructions"] / v["instructions"],
            "achieved_per_s": rate, "peak_per_s": VALU_ISSUE_PEAK, "frac": rate / VALU_ISSUE_PEAK}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", choices=["shuffled", "cell"], default="shuffled")
    ap.add_argument("--method", choices=["partition", "atomic"], default="partition",
                    help="count accumulation: keyed partition + LDS histograms, or one atomic per instance")
    ap.add_argument("--particles", type=int, default=1 << 27)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched form against plain calls (16 realisations, 2.6e9 particles)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of known size (for PMC byte-counter scaling)")
    return ap.parse_args()


def sht_flops(nside, lmax, inverse=False):
    """Algorithmic FP64 flops of one map2alm (inverse=False) or alm2map: the ring
    transforms as four direct length-n/4 DFTs per ring (4 flops per
    real-by-complex multiply-add), divided by the number K of output classes the
    kernels use (equatorial rings: K = 4 when 4 | Nside, 2 when Nside is even;
    polar rings: K = 2 on even rings; the inverse uses K = 8 when 8 | Nside and
    keeps complex sums from K = 4 on, which doubles the flops per class), and the
    Legendre step, 7 flops per (l, m, ring pair): the three-term recurrence (3)
    and the complex multiply-add with the folded ring sum (4)."""
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build runs the path on "
              f"a single GPU and has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1801_05745_amd as uf
    import synth

    uf.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return

    L, nside, om = 1000.0, 1024, 0.3
    n = int(args.particles)
    t0 = time.time()
    x, y, z = synth.lognormal_box(n, L, seed=0, ngrid=256, dtype=torch.float32, device=dev, order=args.order)
    zg = torch.linspace(0.1, 0.5, 31, dtype=torch.float64, device=dev)
    edges = uf.comoving_distance(zg, om).cpu().tolist()
    B = len(edges) - 1
    R = 0
    for oj in (L / 2,) * 3:
        R = max(R, -math.floor((oj - edges[-1]) / L), math.floor((oj + edges[-1]) / L))
    torch.cuda.synchronize()
    gen_s = time.time() - t0

    src = uf.SourceSpec("smail", alpha=2.0, beta=1.5, z0=0.3, z_max=0.5)
    counts = torch.empty((B, uf.npix(nside)), dtype=torch.uint32, device=dev)
    status = uf.new_status(dev)
    if args.method == "partition":
        ws = uf.partition_workspace(n, R, B, nside, device=dev)
    else:
        ws = uf.bin_shells_workspace(device=dev)
    stream = torch.cuda.current_stream(dev)
    timers = [uf.PhaseTimer(dev) for _ in range(args.steps)]
    ev_bin0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_bin1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_born0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_born1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_adj0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_adj1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    outs = {}

    def step(k=None):
        uf.fill_u32(counts, 0)
        if k is not None:
            ev_bin0[k].record(stream)
        uf.bin_shells(x, y, z, edges, nside, box_L=L, n_rep=R, counts=counts, status=status, workspace=ws,
                      timer=timers[k] if k is not None else None)
        if k is not None:
            ev_bin1[k].record(stream)
        W, dW = uf.lensing_weights(om, [src], edges, with_derivatives=True, device=dev)
        inb = uf.inv_nbar(n, L, edges, nside, device=dev)
        if k is not None:
            ev_born0[k].record(stream)
        kap = uf.born_kappa(counts, W, inb, out_dtype=torch.float32)
        if k is not None:
            ev_born1[k].record(stream)
        g = kap * 2.0  # dL/dkappa of L = sum kappa^2
        if k is not None:
            ev_adj0[k].record(stream)
        gW = uf.born_kappa_adjoint(counts, inb, g)
        if k is not None:
            ev_adj1[k].record(stream)
        gth = uf.lensing_weights_vjp(dW, gW)
        outs.update(kappa=kap, W=W, gW=gW, gth=gth, inb=inb)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    status.zero_()
    t1 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms_per_step = 1e3 * wall / args.steps
    bin_ms = sum(a.elapsed_time(b) for a, b in zip(ev_bin0, ev_bin1)) / args.steps
    born_ms = sum(a.elapsed_time(b) for a, b in zip(ev_born0, ev_born1)) / args.steps
    adj_ms = sum(a.elapsed_time(b) for a, b in zip(ev_adj0, ev_adj1)) / args.steps
    st = uf.status_dict(status)
    inst_per_step = st["n_instances"] / args.steps

    # projected overdensity (eq. (7)) on the last step's map: the same streaming
    # pass with weights Delta chi_b / sum Delta chi_b, timed on its own
    ev_od = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    uf.overdensity(counts, edges, outs["inb"])
    ev_od[0].record(stream)
    for _ in range(3):
        delta = uf.overdensity(counts, edges, outs["inb"])
    ev_od[1].record(stream)
    torch.cuda.synchronize()
    od_ms = ev_od[0].elapsed_time(ev_od[1]) / 3
    del delta

    # angular power spectrum of the last step's kappa map (section 3.1: ANAFAST
    # to lmax = 3 Nside - 1) and the covariance of 150 spectra (section 3.2),
    # each timed on its own
    lmax = 3 * nside - 1
    kmap = outs["kappa"][0]
    ev_sh = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    alm = uf.map2alm(kmap, lmax)
    cl = uf.alm2cl(alm, lmax)
    ev_sh[0].record(stream)
    for _ in range(3):
        alm = uf.map2alm(kmap, lmax)
    ev_sh[1].record(stream)
    for _ in range(3):
        cl = uf.alm2cl(alm, lmax)
    ev_sh[2].record(stream)
    torch.cuda.synchronize()
    sht_ms = ev_sh[0].elapsed_time(ev_sh[1]) / 3
    cl_ms = ev_sh[1].elapsed_time(ev_sh[2]) / 3
    sht_fl = sht_flops(nside, lmax)
    a2m_fl = sht_flops(nside, lmax, inverse=True)
    n_real = 150
    jitter = synth.uniform64(n_real * (lmax + 1), seed=5, stream=7, device=dev).reshape(n_real, lmax + 1)
    cls = cl[None, :] * (0.5 + jitter)
    ev_cv = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    uf.cl_covariance(cls)
    ev_cv[0].record(stream)
    for _ in range(3):
        _, cov, corr = uf.cl_covariance(cls)
    ev_cv[1].record(stream)
    torch.cuda.synchronize()
    cov_ms = ev_cv[0].elapsed_time(ev_cv[1]) / 3
    # smoothing with a Gaussian beam of r.m.s. 10.8 arcmin and the one-point
    # moments of the smoothed map (section 3.3, eqs. (12), (13))
    sigma = math.radians(10.8 / 60.0)
    beam = uf.gaussian_beam(sigma, lmax, device=dev)
    sm = uf.alm2map(alm, nside, lmax, beam, out_dtype=torch.float32)
    mom = uf.map_moments(sm)
    ev_sm = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev_sm[0].record(stream)
    for _ in range(3):
        sm = uf.alm2map(alm, nside, lmax, beam, out_dtype=torch.float32)
    ev_sm[1].record(stream)
    for _ in range(3):
        mom = uf.map_moments(sm)
    ev_sm[2].record(stream)
    torch.cuda.synchronize()
    a2m_ms = ev_sm[0].elapsed_time(ev_sm[1]) / 3
    mom_ms = ev_sm[1].elapsed_time(ev_sm[2]) / 3
    mom = mom.cpu().tolist()
    del alm, cls, cov, corr, sm, beam
    uf.release_workspaces()

    kap = outs["kappa"].double()
    rms = float(kap.pow(2).mean().sqrt())
    max_over_rms = float(kap.abs().max()) / rms

    # per-phase milliseconds of the binning call, from the events the library
    # recorded on the stream its kernels ran on
    ph = [t.read() for t in timers]
    phases = {name: sum(p[name] for p in ph) / len(ph) for name in uf.PHASES}
    decide_ms = phases["decide"]
    images = n * (2 * R + 1) ** 3
    flops = FLOPS_PER_IMAGE * images + FLOPS_PER_INSTANCE * inst_per_step
    traffic = measured_traffic()

    # algorithmic bytes of one binning launch: positions once + the count map written once
    bin_bytes = 3 * 4 * n + 4 * B * uf.npix(nside)
    born_bytes = 4 * B * uf.npix(nside) + 4 * uf.npix(nside)
    value = n / (ms_per_step / 1e3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "lognormal lightcone: 2^27 FP32 particles, 1 Gpc/h box replicated to z=0.5 "
                        f"(images {{-{R}..{R}}}^3), 30 shells z=0.1-0.5, Nside 1024 RING, Smail n(z); "
                        "bin + weights + Born kappa + adjoint per step",
            "particles": n, "shells": B, "nside": nside, "order": args.order, "accumulation": args.method,
            "instances_per_step": inst_per_step,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "keys_kernel (FP64 shell + RING pixel decision of every image)",
            "achieved": flops / (decide_ms / 1e3) / 1e12,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops / (decide_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "launch_ms": decide_ms,
            "algorithmic_flops": flops,
            "flops_per_image": FLOPS_PER_IMAGE,
            "flops_per_instance": FLOPS_PER_INSTANCE,
            "images": images,
            "valu_issue": valu_issue(decide_ms),
        },
        "roofline_hbm": {
            "bound": "hbm",
            "kernel": "ufalcon_bin_shells (all kernels of the call)",
            "achieved": bin_bytes / (bin_ms / 1e3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": bin_bytes / (bin_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "launch_ms": bin_ms,
            "algorithmic_bytes": bin_bytes,
            "phases_ms": phases,
        },
        "born": {
            "launch_ms": born_ms,
            "achieved_GBs": born_bytes / (born_ms / 1e3) / 1e9,
            "frac_hbm": born_bytes / (born_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "maps_per_s": 1e3 / born_ms,
        },
        "overdensity": {
            "launch_ms": od_ms,
            "achieved_GBs": born_bytes / (od_ms / 1e3) / 1e9,
            "frac_hbm": born_bytes / (od_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        },
        "adjoint": {
            "launch_ms": adj_ms,
            "achieved_GBs": born_bytes / (adj_ms / 1e3) / 1e9,  # counts + dL/dkappa (FP32) read once
            "frac_hbm": born_bytes / (adj_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        },
        "power_spectrum": {
            "kernel": "ufalcon_map2alm (ring DFTs + Legendre contraction, FP64) + ufalcon_alm2cl",
            "nside": nside, "lmax": lmax,
            "map2alm_ms": sht_ms, "alm2cl_ms": cl_ms,
            "maps_per_s": 1e3 / (sht_ms + cl_ms),
            "algorithmic_flops": sht_fl,
            "achieved": sht_fl / (sht_ms / 1e3) / 1e12,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": sht_fl / (sht_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
        },
        "cl_covariance": {"realisations": n_real, "bands": lmax + 1, "launch_ms": cov_ms},
        "smoothing": {
            "kernel": "ufalcon_alm2map (Legendre synthesis + inverse ring DFTs, FP64), Gaussian beam",
            "sigma_arcmin": 10.8, "lmax": lmax,
            "alm2map_ms": a2m_ms,
            "algorithmic_flops": a2m_fl,
            "achieved": a2m_fl / (a2m_ms / 1e3) / 1e12,
            "frac": a2m_fl / (a2m_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "moments_ms": mom_ms,
            "moments_GBs": 2 * 4 * uf.npix(nside) / (mom_ms / 1e3) / 1e9,
            "s2": mom[3],
            "sigma_s2": math.sqrt(max(mom[4], 0.0)),
        },
        "instances_per_s": inst_per_step / (ms_per_step / 1e3),
        "guarded_per_step": st["n_guarded"] / args.steps,
        "unresolved": st["n_unresolved"],
        "kappa_max_over_rms": max_over_rms,
        "input_generation_s": gen_s,
    }

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, y, z, edges, nside, L, R, args.cpu_sample, n)

    if not args.no_batched:
        # release the step's buffers first: the batched workload holds ~100 GB
        del x, y, z, counts, ws, outs, kap
        uf.release_workspaces()
        torch.cuda.empty_cache()
        line["batched"] = batched_vs_plain(dev)

    print(json.dumps(line), flush=True)


def cpu_baseline(x, y, z, edges, nside, L, R, sample, n):
    """The oracle (plain single-threaded FP64 C loop + exact resolver) on the first
    `sample` particles of the same catalogue, one host core."""
    from oracle import binning as obin

    m = min(sample, n)
    xs, ys, zs = (t[:m].cpu().numpy() for t in (x, y, z))
    t0 = time.perf_counter()
    counts, st = obin.bin_shells(xs, ys, zs, (L / 2,) * 3, L, R, edges, nside, threads=1)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} particles of the bench catalogue (all {len(edges) - 1} shells, "
                      f"Nside {nside}, images {{-{R}..{R}}}^3); {st['instances']} instances in {dt:.1f} s",
            "instances_per_s": st["instances"] / dt}


def batched_vs_plain(dev):
    """Maps/s of 16 realisations (uneven 64M-256M particles, 20-60 shells over z = 0.1-1.0,
    Nside 1024, delta source z = 1.0): one graph replay of the autotuned batch plan against
    16 sequences of plain calls (partitioned accumulation, one shared workspace)."""
    import torch

    import paper_1801_05745_amd as uf
    import synth

    L, nside, om = 1000.0, 1024, 0.3
    M = 1 << 20
    sizes = synth.randint(16, 64 * M, 256 * M, seed=0, stream=900)
    shells = synth.randint(16, 20, 60, seed=0, stream=901)
    items = []
    t0 = time.time()
    for r in range(16):
        x, y, z = synth.lognormal_box(sizes[r], L, seed=r, ngrid=256, dtype=torch.float32, device=dev)
        zg = torch.linspace(0.1, 1.0, shells[r] + 1, dtype=torch.float64, device=dev)
        edges = uf.comoving_distance(zg, om).cpu().tolist()
        W = uf.lensing_weights(om, [uf.SourceSpec("delta", z_s=1.0)], edges, device=dev)
        inb = uf.inv_nbar(sizes[r], L, edges, nside, device=dev)
        items.append(dict(x=x, y=y, z=z, chi_edges=edges, box_L=L, n_rep=2,
                          counts=torch.empty((shells[r], uf.npix(nside)), dtype=torch.uint32, device=dev),
                          W=W, inv_nbar=inb,
                          kappa=torch.empty((1, uf.npix(nside)), dtype=torch.float32, device=dev)))
        print(f"batched: realisation {r} generated ({sizes[r]} particles, {shells[r]} shells)", file=sys.stderr,
              flush=True)
    gen_s = time.time() - t0
    t0 = time.time()
    tuning = uf.autotune_batch(items, nside, T=1, sample_items=2)
    tune_s = time.time() - t0
    print(f"batched: autotuned in {tune_s:.1f} s -> {tuning['method']}", file=sys.stderr, flush=True)
    plan = uf.BatchPlan(items, nside, T=1, method="auto")
    ws = uf.partition_workspace(max(sizes), 2, max(shells), nside, device=dev)

    def plain():
        for it in items:
            uf.fill_u32(it["counts"], 0)
            uf.bin_shells(it["x"], it["y"], it["z"], it["chi_edges"], nside, box_L=L, n_rep=2, counts=it["counts"],
                          workspace=ws)
            it["kappa"].copy_(uf.born_kappa(it["counts"], it["W"], it["inv_nbar"]))

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_plain = timed(plain)
    print(f"batched: plain {t_plain:.3f} s per batch", file=sys.stderr, flush=True)
    t_graph = timed(plan.run_graph)
    print(f"batched: graph {t_graph:.3f} s per batch", file=sys.stderr, flush=True)
    plan.close()
    return {"maps_per_s_batched": 16 / t_graph, "maps_per_s_plain": 16 / t_plain,
            "speedup": t_plain / t_graph, "particles": int(sum(sizes)), "shells": shells,
            "tuning": {"method": tuning["method"], "tile": tuning["tile"],
                       "persistent_wgs": tuning["persistent_wgs"],
                       "candidates_ms": [round(c["ms"], 2) for c in tuning["candidates"]],
                       "tune_s": tune_s, "sample_items": 2},
            "input_generation_s": gen_s}


if __name__ == "__main__":
    main()
