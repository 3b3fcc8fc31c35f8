"""GPU parity: ufalcon_bin_shells (HIP, through the C-ABI) against the oracle.

Count maps must match bit for bit (section 2.3 eq. (5), section 2.4 eq. (8)).
"""

import math

import numpy as np
import pytest
import torch

import paper_1801_05745_amd as uf
import synth
from oracle import binning as obin

from workloads import config1

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu_counts(x, y, z, edges, nside, L, R, observer=None, **kw):
    st = uf.new_status(DEV)
    c = uf.bin_shells(x.to(DEV), y.to(DEV), z.to(DEV), edges, nside, observer=observer, box_L=L, n_rep=R,
                      status=st, **kw)
    torch.cuda.synchronize()
    return c.cpu().numpy().astype(np.int64), uf.status_dict(st)


def test_config1_counts_bit_exact(ufalcon):
    c = config1()
    got, st = _gpu_counts(c["x"], c["y"], c["z"], c["edges"], c["nside"], c["L"], 0)
    ref, rst = obin.bin_shells(c["x"], c["y"], c["z"], (250.0,) * 3, c["L"], 0, c["edges"], c["nside"])
    assert np.array_equal(got, ref)
    assert st["n_instances"] == rst["instances"] == int(ref.sum())
    assert st["n_unresolved"] == 0 and st["n_invalid"] == 0


@pytest.mark.parametrize("nside,R,dtype", [(1, 1, torch.float32), (8, 1, torch.float64), (32, 2, torch.float32)])
def test_replicated_lognormal_several_tiles(ufalcon, nside, R, dtype):
    # 300001 particles: many 256-particle blocks and a ragged tail
    L = 100.0
    x, y, z = synth.lognormal_box(300001, L, seed=3, ngrid=32, dtype=dtype)
    edges = [5.0, 20.0, 40.0, 61.0, 90.0, 130.0][: 3 + R]
    got, st = _gpu_counts(x, y, z, edges, nside, L, R)
    ref, rst = obin.bin_shells(x, y, z, (50.0,) * 3, L, R, edges, nside, threads=8)
    assert np.array_equal(got, ref)
    assert st["n_instances"] == int(ref.sum())


def _lattice_particles():
    pts = []
    for a in range(-3, 4):
        for b in range(-3, 4):
            for c in range(-3, 4):
                pts.append((float(a), float(b), float(c)))
    rng = np.random.default_rng(0)
    for _ in range(400):
        z = rng.choice([2 / 3, -2 / 3, 1 / 3, 0.0, 0.5])
        phi = rng.choice([0.0, math.pi / 4, math.pi / 2, math.pi, math.pi / 16])
        st = math.sqrt(1 - z * z)
        r = rng.choice([1.0, 2.0, math.sqrt(2.0), 2.5])
        pts.append((r * st * math.cos(phi), r * st * math.sin(phi), r * z))
    xs, ys, zs = (torch.tensor(v, dtype=torch.float64) for v in zip(*pts))
    return xs, ys, zs


@pytest.mark.parametrize("nside", [1, 2, 4, 5, 64])
def test_boundary_particles_exact(ufalcon, nside):
    xs, ys, zs = _lattice_particles()
    edges = [0.0, 1.0, math.sqrt(2.0), 2.0, 3.0, 3.5, 6.0]
    obs = (0.0, 0.0, 0.0)
    got, st = _gpu_counts(xs, ys, zs, edges, nside, 1000.0, 0, observer=obs)
    ref, _ = obin.bin_shells(xs, ys, zs, obs, 1000.0, 0, edges, nside)
    assert np.array_equal(got, ref)
    assert st["n_guarded"] > 0 and st["n_unresolved"] == 0


def test_guard_list_overflow_takes_rescue_pass(ufalcon):
    xs, ys, zs = _lattice_particles()
    edges = [0.0, 1.0, math.sqrt(2.0), 2.0, 3.0, 3.5, 6.0]
    obs = (0.0, 0.0, 0.0)
    ws = torch.empty(int(uf.load().ufalcon_bin_shells_workspace_size(3)), dtype=torch.uint8, device=DEV)
    got, st = _gpu_counts(xs, ys, zs, edges, 4, 1000.0, 0, observer=obs, workspace=ws)
    ref, _ = obin.bin_shells(xs, ys, zs, obs, 1000.0, 0, edges, 4)
    assert st["n_guarded"] > 3
    assert np.array_equal(got, ref)


def test_edge_cases(ufalcon):
    e = torch.zeros(0, dtype=torch.float64)
    got, st = _gpu_counts(e, e, e, [0.0, 1.0], 1, 1.0, 0)
    assert got.sum() == 0 and got.shape == (1, 12)
    # invalid coordinates are skipped and counted once per particle
    xs = torch.tensor([5.0, float("nan"), 5.0, float("inf"), 5.0], dtype=torch.float64)
    ys = torch.tensor([5.0, 5.0, 5.0, 5.0, 5.0], dtype=torch.float64)
    zs = torch.tensor([5.0, 5.0, 5.5, 5.0, 4.0], dtype=torch.float64)
    got, st = _gpu_counts(xs, ys, zs, [0.0, 1.0, 2.0], 4, 10.0, 1)
    ref, rst = obin.bin_shells(xs, ys, zs, (5.0, 5.0, 5.0), 10.0, 1, [0.0, 1.0, 2.0], 4)
    assert np.array_equal(got, ref)
    assert st["n_invalid"] == 2 == rst["invalid"]
    assert got[0, 0] == 2  # at the observer -> pixel 0; straight up -> pixel 0


def test_shell_range_and_accumulation(ufalcon):
    L = 50.0
    x, y, z = synth.uniform_box(40000, L, seed=5, dtype=torch.float32)
    edges = [5.0, 15.0, 25.0, 40.0, 55.0]
    xd, yd, zd = x.to(DEV), y.to(DEV), z.to(DEV)
    full = uf.bin_shells(xd, yd, zd, edges, 8, box_L=L, n_rep=1)
    part = uf.new_counts(4, 8, DEV)
    uf.bin_shells(xd, yd, zd, edges, 8, box_L=L, n_rep=1, shell_begin=0, shell_end=2, counts=part)
    uf.bin_shells(xd, yd, zd, edges, 8, box_L=L, n_rep=1, shell_begin=2, shell_end=4, counts=part)
    assert torch.equal(full, part)
    # chunks add up (subvolume decomposition, section 2.4)
    chunked = uf.new_counts(4, 8, DEV)
    for k in range(0, 40000, 7001):
        uf.bin_shells(xd[k:k + 7001].contiguous(), yd[k:k + 7001].contiguous(), zd[k:k + 7001].contiguous(), edges,
                      8, box_L=L, n_rep=1, counts=chunked)
    assert torch.equal(full, chunked)
    # determinism: a second run gives the identical map
    again = uf.bin_shells(xd, yd, zd, edges, 8, box_L=L, n_rep=1)
    assert torch.equal(full, again)


def _both_paths(x, y, z, edges, nside, L, R, **kw):
    xd, yd, zd = x.to(DEV), y.to(DEV), z.to(DEV)
    out = {}
    for method in ("atomic", "partition"):
        st = uf.new_status(DEV)
        c = uf.bin_shells(xd, yd, zd, edges, nside, box_L=L, n_rep=R, status=st, method=method, **kw)
        torch.cuda.synchronize()
        out[method] = (c.cpu().numpy().astype(np.int64), uf.status_dict(st))
    return out


@pytest.mark.parametrize("nside,R", [(4, 1), (64, 1), (16, 2)])
def test_partitioned_path_matches_atomic_and_oracle(ufalcon, nside, R):
    L = 100.0
    x, y, z = synth.lognormal_box(250001, L, seed=11, ngrid=32, dtype=torch.float32)
    edges = [7.0, 25.0, 50.0, 80.0, 110.0, 150.0][: 3 + R]
    res = _both_paths(x, y, z, edges, nside, L, R)
    ref, rst = obin.bin_shells(x, y, z, (50.0,) * 3, L, R, edges, nside, threads=8)
    for method, (got, st) in res.items():
        assert np.array_equal(got, ref), method
        assert st["n_instances"] == int(ref.sum()), method


def test_partitioned_path_several_chunks(ufalcon):
    # keys per chunk far below the instances: the device plan splits the particles
    L = 100.0
    n = 1_500_000
    x, y, z = synth.lognormal_box(n, L, seed=12, ngrid=32, dtype=torch.float32)
    edges = [10.0, 30.0, 60.0, 99.0, 140.0]
    R = 2
    ws = uf.partition_workspace(n, R, len(edges) - 1, 32, max_keys=3_000_000, device=DEV, cached=False)
    st = uf.new_status(DEV)
    got = uf.bin_shells(x.to(DEV), y.to(DEV), z.to(DEV), edges, 32, box_L=L, n_rep=R, status=st, workspace=ws)
    torch.cuda.synchronize()
    ref, _ = obin.bin_shells(x, y, z, (50.0,) * 3, L, R, edges, 32, threads=8)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), ref)
    assert uf.status_dict(st)["n_instances"] == int(ref.sum())


@pytest.mark.parametrize("nside,R,max_keys", [(64, 1, 2_000_000), (256, 2, None)])
def test_partitioned_path_cell_ordered(ufalcon, nside, R, max_keys):
    # particles sorted by grid cell: neighbouring keys share buckets and cell
    # blocks, so the partition's LDS ranks contend on few counters and the
    # second level's runs are long and uneven (a super-tile leaves most blocks
    # no key and a few thousands); with max_keys the particles run in chunks
    L = 100.0
    n = 400_003
    x, y, z = synth.lognormal_box(n, L, seed=5, ngrid=64, dtype=torch.float32, order="cell")
    edges = [5.0, 20.0, 40.0, 61.0, 90.0, 130.0, 180.0, 240.0][: 3 + 2 * R]
    ws = uf.partition_workspace(n, R, len(edges) - 1, nside, max_keys=max_keys, device=DEV, cached=False)
    got, st = _gpu_counts(x, y, z, edges, nside, L, R, workspace=ws, method="partition")
    ref, _ = obin.bin_shells(x, y, z, (50.0,) * 3, L, R, edges, nside, threads=8)
    assert np.array_equal(got, ref)
    assert st["n_instances"] == int(ref.sum()) and st["n_fallback"] == 0


@pytest.mark.parametrize("method", ["partition", "atomic"])
def test_phase_timer_records_phases_without_changing_counts(ufalcon, method):
    L = 100.0
    x, y, z = synth.lognormal_box(200003, L, seed=5, ngrid=32, dtype=torch.float32)
    edges = [5.0, 20.0, 40.0, 61.0, 90.0]
    plain, _ = _gpu_counts(x, y, z, edges, 16, L, 1, method=method)
    timer = uf.PhaseTimer(DEV)
    timed, st = _gpu_counts(x, y, z, edges, 16, L, 1, method=method, timer=timer)
    ms = timer.read()
    assert np.array_equal(plain, timed)
    assert set(ms) == set(uf.PHASES)
    assert all(v >= 0.0 for v in ms.values())
    assert ms["decide"] > 0.0
    iv = timer.intervals()
    assert set(iv) == set(uf.PHASES) and iv["setup"] == 1 and iv["exact"] == 1
    if method == "atomic":
        assert ms["partition"] == 0.0 and ms["accumulate"] == 0.0
        assert iv["decide"] == 1 and iv["partition"] == 0
    else:
        assert ms["partition"] > 0.0 and ms["accumulate"] > 0.0
        # one key pass, partition and accumulation per chunk
        assert iv["decide"] >= 1 and iv["partition"] == iv["decide"] == iv["accumulate"]
    timer.close()
