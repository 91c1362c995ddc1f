"""Batched persistent launch: many uneven RTT chains in one captured graph give
bit-identical results to stepping each RTT on its own through the C ABI
(which is itself parity-tested against the oracle), on every graph replay."""
import json
import math
import os

import numpy as np
import pytest
import torch

from helpers import case, device_cores
from oracle import rtt as orc, tfim
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu

RUNS = [  # Lx, Ly, R, chi, dtype, W
    (3, 3, 2, 16, "f32", 40),
    (4, 4, 3, 32, "bf16", 70),
    (4, 3, 2, 64, "bf16", 33),
    (4, 4, 2, 32, "bf16", 100),
    (5, 4, 2, 32, "fp8", 17),
    (4, 4, 2, 8, "f32", 64),
    (5, 5, 2, 128, "bf16", 40),     # the widest class of the benchmark batch
    (4, 4, 3, 128, "fp8", 24),      # FP8 cores: a class of their own
    (10, 10, 2, 32, "bf16", 50),    # the largest lattice of the benchmark batch
]


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def build(R):
    """The runs, created without column checkpoints: the persistent batch
    kernels contract every proposal's columns from the right boundary, and
    the eager reference must do the same to agree bit for bit (the eager
    sampler runs 16 walkers per block at these sizes, whatever tile the
    batch uses)."""
    rtts, hams, spins, meta = [], [], [], []
    for i, (Lx, Ly, Rr, chi, dtype, W) in enumerate(RUNS):
        N = Lx * Ly
        pi, bond, cores = case(N, Rr, chi, "perm", seed=40 + i)
        os.environ["RTT_CHAIN_CHECKPOINTS"] = "0"
        try:
            rtts.append(R.RTT.create(N, pi, cores, dtype))
        finally:
            del os.environ["RTT_CHAIN_CHECKPOINTS"]
        hams.append(R.TFIM(Lx, Ly, 1.0, 2.0 + 0.3 * i))
        spins.append(R.spins_to_device(wl.pack_spins(wl.random_spins(W, N, 50 + i))))
        meta.append((pi, bond, N, Lx, Ly, 2.0 + 0.3 * i))
    return rtts, hams, spins, meta


@pytest.mark.parametrize("tile", ["16", "32"])
def test_batch_equals_individual_runs(R, tile):
    rtts, hams, spins, meta = build(R)
    ref_spins = [s.clone() for s in spins]
    os.environ["RTT_BATCH_TILE"] = tile      # sampler walkers per block (bonds 32, 128)
    try:
        batch = R.Batch(rtts, hams, spins, seed=777)
    finally:
        del os.environ["RTT_BATCH_TILE"]
    for rep in range(3):
        batch.step(n_sweeps=2)
        torch.cuda.synchronize()
        # eager reference between replays: each run on its own
        for i, r in enumerate(rtts):
            r.sweep(ref_spins[i], seed=777, rng_stream=i, sweep0=2 * rep, n_sweeps=2)
            e = r.local_energy(ref_spins[i], hams[i])
            torch.cuda.synchronize()
            assert torch.equal(batch.spins[i], ref_spins[i]), (rep, i)
            assert torch.equal(batch.eloc[i], e), (rep, i)
            es = batch.esum[i].cpu().numpy()
            ev = e.cpu().numpy()
            assert es[2] == len(ev)
            assert abs(es[0] - math.fsum(ev)) <= 1e-12 * max(1.0, abs(math.fsum(np.abs(ev))))
    batch.close()


def test_batch_energies_match_oracle_on_a_sample(R):
    rtts, hams, spins, meta = build(R)
    batch = R.Batch(rtts, hams, spins, seed=5)
    batch.step(n_sweeps=1)
    torch.cuda.synchronize()
    for i in (0, 3, 4, 6, 7):
        pi, bond, N, Lx, Ly, h = meta[i]
        qc = device_cores(rtts[i], bond)
        bits = wl.unpack_spins(R.spins_to_host(batch.spins[i]), N)[:6]
        el = orc.local_energy(qc, pi, bits, tfim.bonds(Lx, Ly), 1.0, h)
        kap = orc.flip_condition_numbers(qc, pi, bits).max(axis=1)
        tol = 1e-5 if RUNS[i][4] == "f32" else 2e-2
        got = batch.eloc[i].cpu().numpy()[:6]
        assert np.all(np.abs(got - el) / np.maximum(1, np.abs(el)) <= tol * np.maximum(1, kap / 10))
    batch.close()


def test_autotune_picks_a_shape_and_keeps_results_exact(R, tmp_path):
    rtts, hams, spins, meta = build(R)
    ref_spins = [s.clone() for s in spins]
    batch = R.Batch(rtts, hams, spins, seed=11)
    conc, occ = batch.autotune(n_sweeps=1, reps=1, cache_path=str(tmp_path / "tune.jsonl"))
    assert conc in (0, 1) and 1 <= occ <= 4
    lines = (tmp_path / "tune.jsonl").read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    tiles = {(c["dtype"], c["bond"]): c["sampler_walkers_per_block"] for c in rec["classes"]}
    print(f"  autotuned: {rec}", flush=True)
    assert set(tiles.values()) <= {16, 32} and tiles[(2, 64)] == 16
    # 8 launch shapes, then one trial per class with a second tile (BF16 and
    # FP8 at bonds 32 and 128), each 1 warm-up + 1 timed step of 1 sweep
    assert rec["trials"] == 8 + 4
    n_done = 2 * rec["trials"]
    batch.step(n_sweeps=1)
    torch.cuda.synchronize()
    for i, r in enumerate(rtts):
        r.sweep(ref_spins[i], seed=11, rng_stream=i, sweep0=0, n_sweeps=n_done + 1)
    torch.cuda.synchronize()
    for i in range(len(rtts)):
        assert torch.equal(batch.spins[i], ref_spins[i]), i
    batch.close()


def test_benchmark_batch_sampled_runs(R):
    """The benchmark's batch in its launch configuration: 256 uneven BF16 RTTs
    (side 4-10, R 2-3, chi 16-128, 256-4096 walkers), autotuned, one step of
    1 sweep + local energies.  The oracle recomputes the local energies of
    three walkers of six runs: the two largest chi = 128 runs, the largest
    R = 3 run, and the smallest runs of chi 16, 32 and 64."""
    ws = wl.batched_workloads(256)
    rtts = [R.RTT.create(w.N, w.pi(), w.cores(), "bf16") for w in ws]
    hams = [R.TFIM(w.Lx, w.Ly, w.J, w.h) for w in ws]
    spins = [R.spins_to_device(wl.pack_spins(w.spins())) for w in ws]
    batch = R.Batch(rtts, hams, spins, seed=3100)
    conc, occ = batch.autotune(n_sweeps=1, reps=1)
    batch.step(n_sweeps=1)
    torch.cuda.synchronize()
    work = [w.W * w.N * w.N * w.R * w.chi ** 2 for w in ws]
    c128 = sorted((i for i, w in enumerate(ws) if w.chi == 128), key=lambda i: -work[i])[:2]
    r3 = max((i for i, w in enumerate(ws) if w.R == 3), key=lambda i: work[i])
    small = [min((i for i, w in enumerate(ws) if w.chi == c), key=lambda i: work[i]) for c in (16, 32, 64)]
    picks = list(dict.fromkeys(c128 + [r3] + small))
    print(f"  autotuned shape: concurrent {conc}, blocks per CU {occ}; runs {picks}", flush=True)
    for i in picks:
        w = ws[i]
        qc = device_cores(rtts[i], w.bond())
        sub = [0, w.W // 2, w.W - 1]
        bits = wl.unpack_spins(R.spins_to_host(batch.spins[i]), w.N)[sub]
        el = orc.local_energy(qc, w.pi(), bits, tfim.bonds(w.Lx, w.Ly), w.J, w.h)
        got = batch.eloc[i].cpu().numpy()[sub]
        rel = np.abs(got - el) / np.maximum(1.0, np.abs(el))
        print(f"  run {i}: {w.Lx}x{w.Ly} R={w.R} chi={w.chi} W={w.W}: E_loc rel err {rel.max():.2e}", flush=True)
        assert np.all(rel <= 2e-2)
        es = batch.esum[i].cpu().numpy()
        assert es[2] == w.W
    batch.close()
