"""Shapes that do not fit on chip in one piece: row groups in the flip-ratio
passes, and the term-sequential sweep of a large linear combination; the
sampler's two-column-group blocks (bond 128, at least 32 walkers per compute
unit); the largest spin count.  (The 16x16, chi = 256, 4-term FP8 workload
is tested at full size in test_gpu_fullsize.py.)"""
import numpy as np
import pytest
import torch

from helpers import HILO_TOL, case, check_ratios, device_cores
from oracle import mcmc, rtt as orc, tt
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def test_row_groups_match_oracle(R):
    N, Rr, chi, W = 100, 2, 256, 2
    pi, bond, cores = case(N, Rr, chi, "perm", seed=60)
    psi = R.RTT.create(N, pi, cores, "bf16")
    assert psi.info["groups"] >= 2
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, 61)
    out = psi.evaluate(R.spins_to_device(wl.pack_spins(bits)))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    r_ref = orc.flip_ratios(qc, pi, bits)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], r_ref, kap, 2e-2)
    print(psi.info, st)
    assert st["n_bad"] == 0 and st["n_sign_bad"] == 0
    assert check_ratios(out["logratio"], out["rsign"], r_ref, kap, HILO_TOL)["n_bad"] == 0
    la, sg = orc.log_sign(orc.amplitudes(qc, pi, bits))
    assert np.all(out["sign"] == sg) and np.max(np.abs(out["logabs"] - la)) < 2e-2


@pytest.mark.parametrize("N,W,seed,chi,dtype", [(16, 8, 70, 256, "fp8"), (100, 4, 60, 256, "fp8"),
                                                (160, 1, 64, 256, "fp8"), (101, 4, 61, 128, "bf16"),
                                                (102, 4, 62, 128, "fp8")])
def test_k_outer_pass_row_tiles_match_oracle(R, N, W, seed, chi, dtype):
    """The K-outer flip-ratio pass with rows updated in place (FP8 at bond
    256, BF16 and FP8 at bond 128): a second row tile that first appears on
    the last two steps (N = 16), row groups (N = 100), six row tiles per
    group, more rows than two buffers would hold (N = 160), and bond 128
    with up to seven row tiles in one group."""
    print(f"[case] {dtype} bond {chi} N={N} W={W}", flush=True)
    pi, bond, cores = case(N, 2, chi, "perm", seed=seed)
    psi = R.RTT.create(N, pi, cores, dtype)
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, seed + 1)
    out = psi.evaluate(R.spins_to_device(wl.pack_spins(bits)))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    r_ref = orc.flip_ratios(qc, pi, bits)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], r_ref, kap, HILO_TOL, min_well=0)
    print(psi.info, st)
    if N == 160:
        assert psi.info["nslot"] > 64
    assert st["n_bad"] == 0 and st["n_sign_bad"] == 0
    la, sg = orc.log_sign(orc.amplitudes(qc, pi, bits))
    assert np.all(out["sign"] == sg) and np.max(np.abs(out["logabs"] - la)) < 1e-3


def test_row_groups_fp32_many_spins(R):
    """FP32, chi = 128, N = 144: groups also in the FP32 path."""
    N, Rr, chi, W = 144, 2, 128, 2
    pi, bond, cores = case(N, Rr, chi, "perm", seed=62)
    psi = R.RTT.create(N, pi, cores, "f32")
    assert psi.info["groups"] >= 2
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, 63)
    out = psi.evaluate(R.spins_to_device(wl.pack_spins(bits)))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    r_ref = orc.flip_ratios(qc, pi, bits)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], r_ref, kap, 1e-5)
    print(psi.info, st)
    assert st["n_bad"] == 0 and st["n_sign_bad"] == 0


def test_sequential_terms_sweep_matches_oracle(R):
    """4 terms at chi = 256 exceed on-chip memory together, so the sweep runs
    term by term; decisions equal the oracle's Metropolis on the direct-sum
    train's amplitudes (the summed terms) away from near-ties."""
    N, Rr, chi, T, W = 9, 2, 256, 4, 16
    pi = wl.path_site_plus_perms(N, Rr, 64)
    bond = wl.open_bonds(N * Rr, chi)
    bond[1:-1] = 256
    terms = [wl.gaussian_cores(bond, 65 + t) for t in range(T)]
    c = np.array([1.0, -0.6, 0.8, 0.3])
    hs = [R.RTT.create(N, pi, t, "bf16") for t in terms]
    comb = R.RTT.lincomb(hs, c)
    qts = device_cores(comb, bond, n_terms=T)
    amp = lambda S: orc.lincomb_amplitudes(qts, c, pi, S)
    bits = wl.random_spins(W, N, 66)
    spins = R.spins_to_device(wl.pack_spins(bits))
    la = torch.empty(W, dtype=torch.float64, device="cuda")
    sg = torch.empty(W, dtype=torch.int8, device="cuda")
    comb.sweep(spins, seed=17, rng_stream=2, sweep0=0, n_sweeps=2, logabs=la, sign=sg)
    torch.cuda.synchronize()
    ref, _, margins = mcmc.metropolis(None, pi, bits, seed=17, stream=2, sweep0=0, n_sweeps=2,
                                      record=True, amp_fn=amp)
    clean = np.min(np.abs(margins), axis=(0, 1)) > 1e-2   # BF16 ratios: 2e-2-level agreement
    got = wl.unpack_spins(R.spins_to_host(spins), N)
    assert clean.sum() >= W // 2
    assert np.array_equal(got[clean], ref[clean])
    lref, sref = orc.log_sign(amp(ref))
    ok = clean
    assert np.all(sg.cpu().numpy()[ok] == sref[ok])
    assert np.max(np.abs(la.cpu().numpy()[ok] - lref[ok])) < 2e-2


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_two_column_groups_many_walkers(R, dtype):
    """Bond 128 with 32 * 256 + 24 walkers: the sampler runs 32 walkers per
    block (two MFMA column groups sharing each core fragment), the last
    block ragged.  Amplitudes of walkers in both groups, in the first and the
    last block, match the oracle; one FP32 sweep makes the oracle's decisions
    for the same walkers (Philox counters follow the walker index)."""
    N, Rr, chi = 16, 2, 128
    W = 32 * 256 + 24
    pi, bond, cores = case(N, Rr, chi, "perm", seed=70)
    psi = R.RTT.create(N, pi, cores, dtype)
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, 71)
    spins = R.spins_to_device(wl.pack_spins(bits))
    la, sg = psi.amplitudes(spins)
    torch.cuda.synchronize()
    idx = np.r_[0:40, W - 40:W]
    la_ref, sg_ref = orc.log_sign(orc.amplitudes(qc, pi, bits[idx]))
    k0 = orc.condition_numbers(qc, pi, bits[idx])
    tol = {"f32": 1e-5, "bf16": 2e-2}[dtype]
    assert np.all(sg.cpu().numpy()[idx] == sg_ref)
    assert np.all(np.abs(la.cpu().numpy()[idx] - la_ref) <= tol * np.maximum(1.0, k0 / 10.0))
    if dtype != "f32":
        return
    psi.sweep(spins, seed=77, rng_stream=2, sweep0=0, n_sweeps=1)
    torch.cuda.synchronize()
    got = wl.unpack_spins(R.spins_to_host(spins), N)[idx]
    ref, _, margins = mcmc.metropolis(qc, pi, bits[idx], seed=77, stream=2, sweep0=0, n_sweeps=1,
                                      walker_ids=idx, record=True)
    clean = np.min(np.abs(margins), axis=(0, 1)) > 1e-4
    assert clean.sum() >= len(idx) - 3
    assert np.array_equal(got[clean], ref[clean])


def test_maximum_spin_count_matrix_cores(R):
    """N = 1024 (the largest the library takes), one replica, bond 16 on the
    matrix-core kernels: 16 spin words per walker, long flip-ratio rows.
    Ratios, amplitudes and one sweep of the sampled walkers against the
    oracle."""
    N, chi, W = 1024, 16, 3
    pi = np.arange(N, dtype=np.int32)
    bond = wl.open_bonds(N, chi)
    cores = wl.gaussian_cores(bond, 64)
    psi = R.RTT.create(N, pi, cores, "f32")
    assert psi.info["narrow"] == 0 and psi.info["nw"] == 16
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, 65)
    sp = R.spins_to_device(wl.pack_spins(bits))
    out = psi.evaluate(sp)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.all(out["status"] == 0)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], orc.flip_ratios(qc, pi, bits), kap, 1e-5)
    print(psi.info, st)
    assert st["n_bad"] == 0 and st["n_sign_bad"] == 0
    la, sg = orc.log_sign(orc.amplitudes(qc, pi, bits))
    k0 = orc.condition_numbers(qc, pi, bits)
    assert np.all(out["sign"] == sg) and np.all(np.abs(out["logabs"] - la) <= 1e-5 * np.maximum(1.0, k0 / 10.0))
    psi.sweep(sp, seed=66, n_sweeps=1)
    torch.cuda.synchronize()
    got = wl.unpack_spins(R.spins_to_host(sp), N)
    ref, _, margins = mcmc.metropolis(qc, pi, bits, seed=66, n_sweeps=1, record=True)
    clean = np.min(np.abs(margins), axis=(0, 1)) > 1e-4
    assert np.array_equal(got[clean], ref[clean])
