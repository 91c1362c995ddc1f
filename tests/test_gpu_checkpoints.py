"""Sweeps that keep column checkpoints (the right environments of a few bonds
of the current configuration, reused by later proposals and replaced when a
walker accepts) make the oracle's decisions: same Philox words, every walker
whose decisions stay clear of near-ties.  The cases cover R = 1 (a proposal
can meet its checkpoint with no column step left), R = 2 and 3 on both path
kinds, several sweeps in one call (checkpoints carried across sweeps), a
two-term combination, the two-column-group launch at bond 128 and the 8x8
benchmark workload at full size."""
import os

import numpy as np
import pytest
import torch

from helpers import case, device_cores
from oracle import mcmc, rtt as orc
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def run_and_compare(R, psi, amp, pi, bits, seed, stream, n_sweeps, margin, calls=1, walker_ids=None,
                    min_clean=0.75):
    N = bits.shape[1]
    spins = R.spins_to_device(wl.pack_spins(bits))
    la = torch.empty(bits.shape[0], dtype=torch.float64, device="cuda")
    sg = torch.empty(bits.shape[0], dtype=torch.int8, device="cuda")
    per = n_sweeps // calls
    for c in range(calls):
        psi.sweep(spins, seed=seed, rng_stream=stream, sweep0=c * per, n_sweeps=per, logabs=la, sign=sg)
    torch.cuda.synchronize()
    got = wl.unpack_spins(R.spins_to_host(spins), N)
    idx = np.arange(bits.shape[0]) if walker_ids is None else np.asarray(walker_ids)
    ref, _, margins = mcmc.metropolis(None, pi, bits[idx], seed=seed, stream=stream, sweep0=0,
                                      n_sweeps=n_sweeps, walker_ids=idx, record=True, amp_fn=amp)
    clean = np.min(np.abs(margins), axis=(0, 1)) > margin
    assert clean.sum() >= max(1, int(min_clean * len(idx))), clean.sum()
    assert np.array_equal(got[idx][clean], ref[clean])
    lref, sref = orc.log_sign(amp(ref))
    la = la.cpu().numpy()[idx]
    sg = sg.cpu().numpy()[idx]
    assert np.all(sg[clean] == sref[clean])
    return np.max(np.abs(la[clean] - lref[clean]))


@pytest.mark.parametrize("N,Rr,chi,path,W", [
    (16, 1, 16, "repeat", 48),
    (24, 2, 32, "perm", 64),
    (12, 3, 64, "perm", 40),
    (12, 3, 64, "repeat", 40),
])
def test_checkpointed_sweeps_match_oracle(R, N, Rr, chi, path, W):
    pi, bond, cores = case(N, Rr, chi, path, seed=700 + N + chi)
    psi = R.RTT.create(N, pi, cores, "f32")
    qc = device_cores(psi, bond)
    amp = lambda S: orc.amplitudes(qc, pi, S)
    bits = wl.random_spins(W, N, 701 + chi)
    err = run_and_compare(R, psi, amp, pi, bits, seed=702, stream=3, n_sweeps=4, margin=1e-4)
    assert err < 1e-4


def test_checkpoints_carried_across_calls_and_sweeps(R):
    """Four sweeps as one call and as four calls follow the same oracle chain."""
    N, Rr, chi, W = 20, 2, 32, 64
    pi, bond, cores = case(N, Rr, chi, "perm", seed=710)
    psi = R.RTT.create(N, pi, cores, "f32")
    qc = device_cores(psi, bond)
    amp = lambda S: orc.amplitudes(qc, pi, S)
    bits = wl.random_spins(W, N, 711)
    for calls in (1, 4):
        err = run_and_compare(R, psi, amp, pi, bits, seed=712, stream=1, n_sweeps=4, margin=1e-4, calls=calls)
        assert err < 1e-4


def test_checkpointed_lincomb_sweep_matches_oracle(R):
    N, Rr, chi, W = 16, 2, 32, 48
    pi = wl.path_site_plus_perms(N, Rr, 720)
    bond = wl.open_bonds(N * Rr, chi)
    c = np.array([0.9, -0.5])
    hs = [R.RTT.create(N, pi, wl.gaussian_cores(bond, 721 + t), "f32") for t in range(2)]
    comb = R.RTT.lincomb(hs, c)
    qts = device_cores(comb, bond, n_terms=2)
    amp = lambda S: orc.lincomb_amplitudes(qts, c, pi, S)
    bits = wl.random_spins(W, N, 722)
    err = run_and_compare(R, comb, amp, pi, bits, seed=723, stream=0, n_sweeps=3, margin=1e-4)
    assert err < 1e-4


def test_checkpoints_off_matches_oracle(R):
    """RTT_CHAIN_CHECKPOINTS=0: every proposal contracts its columns from the
    right boundary, with the same decisions."""
    N, Rr, chi, W = 16, 2, 32, 48
    pi, bond, cores = case(N, Rr, chi, "perm", seed=730)
    os.environ["RTT_CHAIN_CHECKPOINTS"] = "0"
    try:
        psi = R.RTT.create(N, pi, cores, "f32")
    finally:
        del os.environ["RTT_CHAIN_CHECKPOINTS"]
    qc = device_cores(psi, bond)
    amp = lambda S: orc.amplitudes(qc, pi, S)
    bits = wl.random_spins(W, N, 731)
    err = run_and_compare(R, psi, amp, pi, bits, seed=732, stream=2, n_sweeps=3, margin=1e-4)
    assert err < 1e-4


def test_checkpointed_two_group_launch_sampled(R):
    """Bond 128, BF16, 8192 walkers (two column groups of 16 per block on a
    256-CU device): a sample of walkers follows the oracle's chain."""
    N, Rr, chi, W = 10, 2, 128, 8192
    pi, bond, cores = case(N, Rr, chi, "perm", seed=740)
    psi = R.RTT.create(N, pi, cores, "bf16")
    qc = device_cores(psi, bond)
    amp = lambda S: orc.amplitudes(qc, pi, S)
    bits = wl.random_spins(W, N, 741)
    ids = [0, 1, 17, 31, 4000, 8191]
    err = run_and_compare(R, psi, amp, pi, bits, seed=742, stream=0, n_sweeps=2, margin=1e-2,
                          walker_ids=ids)
    assert err < 2e-2


@pytest.mark.parametrize("dtype,margin,sweeps", [("f32", 1e-4, 2), ("bf16", 2e-3, 1)])
def test_full_size_8x8_sweeps_sampled(R, dtype, margin, sweeps):
    """8x8, R=2, chi=64, 4096 walkers: the benchmark's launch (one block of 16
    walkers per CU, 13 checkpoints); a sample of walkers follows the oracle's
    chain.  BF16 cores with hi+lo activations give log-ratio errors of order
    1e-4, so its decisions are compared where every margin exceeds 2e-3 (one
    sweep: over 64 decisions most walkers stay that clear of ties)."""
    w = wl.MEDIUM_8x8
    pi, bond = w.pi(), w.bond()
    psi = R.RTT.create(w.N, pi, w.cores(), dtype)
    qc = device_cores(psi, bond)
    amp = lambda S: orc.amplitudes(qc, pi, S)
    bits = w.spins()
    ids = [0, 5, 17, 300, 1234, 2047, 2048, 3000, 3333, 3999, 4090, 4095]
    err = run_and_compare(R, psi, amp, pi, bits, seed=w.chain_seed, stream=7, n_sweeps=sweeps, margin=margin,
                          walker_ids=ids, min_clean=0.5)
    assert err < (1e-4 if dtype == "f32" else 2e-2)


@pytest.mark.parametrize("checkpoints", ["1", "0"])
def test_sequential_fp8_bond256_checkpoints(R, checkpoints):
    """A four-term FP8 combination at bond 256 samples with the terms taking
    turns (their rows do not fit on chip together); its column checkpoints
    then live in global memory.  Three sweeps in one call and in three calls
    (checkpoints carried across sweeps, then rebuilt) make the oracle's
    decisions on the summed amplitudes away from near-ties, with and
    without checkpoints (RTT_CHAIN_CHECKPOINTS=0)."""
    N, Rr, chi, T, W = 16, 2, 256, 4, 48
    pi = wl.path_site_plus_perms(N, Rr, 81)
    bond = wl.open_bonds(N * Rr, chi)
    terms = [wl.gaussian_cores(bond, 82 + t) for t in range(T)]
    c = np.array([0.9, -1.2, 0.5, 0.7])
    os.environ["RTT_CHAIN_CHECKPOINTS"] = checkpoints
    try:
        hs = [R.RTT.create(N, pi, t, "fp8") for t in terms]
        comb = R.RTT.lincomb(hs, c)
    finally:
        del os.environ["RTT_CHAIN_CHECKPOINTS"]
    for h in hs:
        h.close()
    qts = device_cores(comb, bond, n_terms=T)
    amp = lambda S: orc.lincomb_amplitudes(qts, c, pi, S)
    bits = wl.random_spins(W, N, 83)
    for calls in (1, 3):
        print(f"[case] checkpoints={checkpoints} calls={calls}", flush=True)
        err = run_and_compare(R, comb, amp, pi, bits, seed=84, stream=1, n_sweeps=3, margin=1e-3,
                              calls=calls, min_clean=0.5)
        assert err < 2e-2
    comb.close()
