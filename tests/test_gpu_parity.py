"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs and the library's own quantised cores.

Tolerances on log-ratios (the relative errors of r_j): 1e-5 for FP32 cores
on FP32 matrix cores, 2e-2 for BF16 and FP8 cores (hi+lo BF16 activations,
FP32 accumulation), for ratios whose oracle condition number kappa is <= 10;
beyond that the bound grows as tol * kappa / 10 (any floating-point
evaluation of psi has relative error ~ gamma * kappa).  log|psi| uses the
same rule with kappa(s).
"""
import math

import numpy as np
import pytest
import torch

from helpers import HILO_TOL, assert_ratio_summary, case, check_ratios, device_cores
from oracle import mcmc, rtt as orc, stats, tfim
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2, "fp8": 2e-2}


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def run_eval(R, pi, bond, cores, N, bits, dtype, ham=None):
    psi = R.RTT.create(N, pi, cores, dtype)
    qc = device_cores(psi, bond)
    spins = R.spins_to_device(wl.pack_spins(bits))
    out = psi.evaluate(spins, ham)
    torch.cuda.synchronize()
    return psi, qc, {k: v.cpu().numpy() for k, v in out.items()}


EVAL_CASES = [
    # name, N, R, chi, path, dtype, W
    ("4x4_repeat_chi8", 16, 2, 8, "repeat", "f32", 37),
    ("n40_perm_chi32_ragged", 40, 2, 32, "perm", "f32", 21),
    ("n20_R3_chi16", 20, 3, 16, "perm", "f32", 9),
    ("n30_R1_chi64", 30, 1, 64, "perm", "f32", 6),
    ("n24_perm_chi64_bf16", 24, 2, 64, "perm", "bf16", 7),
    ("n24_perm_chi64_fp8", 24, 2, 64, "perm", "fp8", 7),
    ("n20_perm_chi32_fp8_ragged", 20, 2, 32, "perm", "fp8", 13),
    ("n16_R3_chi128_fp8", 16, 3, 128, "perm", "fp8", 5),
    ("n12_perm_chi256_fp8", 12, 2, 256, "perm", "fp8", 3),
    ("n20_perm_chi128_f32", 20, 2, 128, "perm", "f32", 3),
    ("n12_perm_chi256_bf16", 12, 2, 256, "perm", "bf16", 3),
]


def assert_parity(out, qc, pi, bits, dtype, label="", min_well=1):
    psi_ref = orc.amplitudes(qc, pi, bits)
    la_ref, sg_ref = orc.log_sign(psi_ref)
    k0 = orc.condition_numbers(qc, pi, bits)
    tol = TOL[dtype]
    assert np.all(out["status"] == 0)
    assert np.all(out["sign"] == sg_ref)
    assert np.all(np.abs(out["logabs"] - la_ref) <= tol * np.maximum(1.0, k0 / 10.0))
    r_ref = orc.flip_ratios(qc, pi, bits)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], r_ref, kap, tol, min_well=min_well)
    print(f"  {label} {st}", flush=True)
    assert_ratio_summary(st)
    if tol > 1e-3:   # reduced precision: the accuracy of hi + lo activations
        sh = check_ratios(out["logratio"], out["rsign"], r_ref, kap, HILO_TOL, min_well=0)
        print(f"  {label} at {HILO_TOL}: {sh}", flush=True)
        assert sh["n_bad"] == 0, sh
        if label == "sampled":   # configurations the chain visits: the stated bound, unscaled
            assert st["frac_within_tol"] >= 0.99, st
    return st


def sampled(qc, pi, W, N, seed, sweeps=6):
    """Configurations from the oracle's own Metropolis chain (|psi|^2)."""
    s0 = wl.random_spins(W, N, seed)
    s, _, _ = mcmc.metropolis(qc, pi, s0, seed=seed, stream=9, n_sweeps=sweeps)
    return s


@pytest.mark.parametrize("name,N,Rr,chi,path,dtype,W", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_evaluate_matches_oracle(R, name, N, Rr, chi, path, dtype, W):
    print(f"[case] {name}", flush=True)
    pi, bond, cores = case(N, Rr, chi, path, seed=len(name))
    bits = wl.random_spins(W, N, 7 + N)
    psi, qc, out = run_eval(R, pi, bond, cores, N, bits, dtype)
    # uniform spins of the wide-bond cases have no well-conditioned ratio
    assert_parity(out, qc, pi, bits, dtype, "uniform", min_well=0)
    # configurations the chain samples
    bits2 = sampled(qc, pi, min(W, 12), N, 100 + N)
    out2 = psi.evaluate(R.spins_to_device(wl.pack_spins(bits2)))
    torch.cuda.synchronize()
    out2 = {k: v.cpu().numpy() for k, v in out2.items()}
    assert_parity(out2, qc, pi, bits2, dtype, "sampled", min_well=1 if dtype == "f32" else 0)


def test_general_path_with_unread_spins_and_uneven_bonds(R):
    """pi with spins read once, twice, three times and never; adjacent repeats;
    bond dimensions that vary along the train."""
    N = 12
    pi = np.array([3, 0, 0, 5, 1, 7, 3, 2, 9, 1, 4, 3, 6, 0, 8, 2, 5, 9], dtype=np.int32)  # 10, 11 unread
    L = len(pi)
    bond = np.array([1, 2, 5, 9, 16, 13, 7, 16, 11, 3, 8, 16, 16, 4, 9, 12, 6, 2, 1])
    assert len(bond) == L + 1
    cores = wl.gaussian_cores(bond, 77, std=0.4)
    bits = wl.random_spins(19, N, 78)
    _, qc, out = run_eval(R, pi, bond, cores, N, bits, "f32")
    assert np.all(out["logratio"][:, 10:] == 0.0) and np.all(out["rsign"][:, 10:] == 1)
    assert_parity(out, qc, pi, bits, "f32")


def test_worked_path_flip_indexing(R):
    """The paper's 6-spin HV path: flipping spin 3 switches tensors 3 and 8.
    Cores that differ between slices only at those two positions give r != 1
    only for spin 3; the ratio equals the oracle's."""
    pi = wl.path_hv_2x3()
    bond = wl.open_bonds(12, 3)
    cores = wl.gaussian_cores(bond, 91)
    for k in range(12):
        if k not in (2, 7):
            cores[k][1] = cores[k][0]
    bits = orc.all_configs(6)
    _, qc, out = run_eval(R, pi, bond, cores, 6, bits, "f32")
    r = out["rsign"] * np.exp(out["logratio"])
    others = [0, 1, 3, 4, 5]
    assert np.allclose(r[:, others], 1.0, rtol=1e-6)
    assert np.allclose(r[:, 2], orc.flip_ratios(qc, pi, bits)[:, 2], rtol=1e-5)


def test_local_energy_matches_oracle(R):
    N, Rr, chi = 16, 2, 8
    pi, bond, cores = case(N, Rr, chi, "repeat", seed=3)
    bits = wl.random_spins(64, N, 2001)
    ham = R.TFIM(4, 4, 1.0, 3.04)
    _, qc, out = run_eval(R, pi, bond, cores, N, bits, "f32", ham)
    el_ref = orc.local_energy(qc, pi, bits, tfim.bonds(4, 4), 1.0, 3.04)
    rel = np.abs(out["eloc"] - el_ref) / np.maximum(1.0, np.abs(el_ref))
    kap = orc.flip_condition_numbers(qc, pi, bits).max(axis=1)
    assert np.all(rel <= 1e-5 * np.maximum(1.0, kap / 10.0))
    assert np.median(rel) < 1e-6


def test_lincomb_matches_oracle(R):
    N, Rr, chi, T = 20, 2, 32, 3
    pi = wl.path_site_plus_perms(N, Rr, 55)
    bond = wl.open_bonds(N * Rr, chi)
    terms = [wl.gaussian_cores(bond, 300 + t) for t in range(T)]
    c = np.array([0.8, -1.1, 0.5])
    hs = [R.RTT.create(N, pi, t, "f32") for t in terms]
    comb = R.RTT.lincomb(hs, c)
    for h in hs:
        h.close()
    qts = device_cores(comb, bond, n_terms=T)
    bits = wl.random_spins(11, N, 56)
    ham = R.TFIM(5, 4, 1.0, 3.04)
    out = comb.evaluate(R.spins_to_device(wl.pack_spins(bits)), ham)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    psi_ref = orc.lincomb_amplitudes(qts, c, pi, bits)
    la, sg = orc.log_sign(psi_ref)
    assert np.all(out["sign"] == sg)
    assert np.max(np.abs(out["logabs"] - la)) < 1e-4
    r_ref = orc.lincomb_flip_ratios(qts, c, pi, bits)
    # conditioning of the sum: the direct-sum train is one RTT with the same psi
    from oracle import tt
    ds = tt.direct_sum(qts, c)
    kap = orc.flip_condition_numbers(ds, pi, bits)
    st = check_ratios(out["logratio"], out["rsign"], r_ref, kap, 1e-5)
    print(st)
    assert st["n_bad"] == 0 and st["n_sign_bad"] == 0
    el = orc.lincomb_local_energy(qts, c, pi, bits, tfim.bonds(5, 4), 1.0, 3.04)
    scale = np.maximum(1.0, kap.max(axis=1) / 10.0)
    assert np.all(np.abs(out["eloc"] - el) / np.maximum(1, np.abs(el)) <= 1e-5 * scale)
    # chain amplitudes agree with the evaluation path
    la2, sg2 = comb.amplitudes(R.spins_to_device(wl.pack_spins(bits)))
    assert np.max(np.abs(la2.cpu().numpy() - la)) < 1e-4


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_chain_amplitudes_match_oracle(R, dtype):
    N, Rr, chi = 64, 2, 64
    pi, bond, cores = case(N, Rr, chi, "perm", seed=9)
    bits = wl.random_spins(40, N, 10)
    psi = R.RTT.create(N, pi, cores, dtype)
    qc = device_cores(psi, bond)
    la, sg = psi.amplitudes(R.spins_to_device(wl.pack_spins(bits)))
    torch.cuda.synchronize()
    la_ref, sg_ref = orc.log_sign(orc.amplitudes(qc, pi, bits))
    k0 = orc.condition_numbers(qc, pi, bits)
    assert np.all(sg.cpu().numpy() == sg_ref)
    assert np.all(np.abs(la.cpu().numpy() - la_ref) <= TOL[dtype] * np.maximum(1.0, k0 / 10.0))


def test_quantisation_matches_torch_casts(R):
    from oracle import quant
    pi, bond, cores = case(10, 2, 32, "perm", seed=4)
    big = [c * 300.0 for c in cores]          # exercise the e4m3 scale and clamp
    for dtype, src in (("bf16", cores), ("fp8", big), ("f32", cores)):
        psi = R.RTT.create(10, pi, src, dtype)
        got = device_cores(psi, bond)
        want = quant.quantise_cores(src, dtype)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), dtype


def test_sweep_trajectory_parity(R):
    """Identical Philox words: GPU and oracle chains make the same decisions
    for every walker up to its first near-tie |u - r^2| < 1e-4."""
    N, Rr, chi, W = 16, 2, 8, 64
    pi, bond, cores = case(N, Rr, chi, "repeat", seed=21)
    bits = wl.random_spins(W, N, 22)
    psi = R.RTT.create(N, pi, cores, "f32")
    qc = device_cores(psi, bond)
    spins = R.spins_to_device(wl.pack_spins(bits))
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    S = 6
    ref_states, s = [], bits.copy()
    tie_free = np.ones(W, dtype=bool)
    for t in range(S):
        psi.sweep(spins, seed=123, rng_stream=4, sweep0=t, n_sweeps=1, accepts=acc)
        torch.cuda.synchronize()
        s, _, margins = mcmc.metropolis(qc, pi, s, seed=123, stream=4, sweep0=t, n_sweeps=1, record=True)
        tie_free &= np.min(np.abs(margins), axis=(0, 1)) > 1e-4
        got = wl.unpack_spins(R.spins_to_host(spins), N)
        assert np.array_equal(got[tie_free], s[tie_free]), f"sweep {t}"
    assert tie_free.sum() >= W - 3


def test_multi_sweep_call_equals_single_sweeps(R):
    N, Rr, chi, W = 24, 2, 32, 33
    pi, bond, cores = case(N, Rr, chi, "perm", seed=31)
    bits = wl.random_spins(W, N, 32)
    psi = R.RTT.create(N, pi, cores, "f32")
    a = R.spins_to_device(wl.pack_spins(bits))
    b = a.clone()
    psi.sweep(a, seed=5, sweep0=10, n_sweeps=3)
    for t in range(3):
        psi.sweep(b, seed=5, sweep0=10 + t, n_sweeps=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_energy_reduce_matches_fsum(R):
    g = np.random.default_rng(3)
    x = g.standard_normal(5000) * 1e3 + 1e8
    x[17] = np.nan
    out = R.energy_reduce(torch.from_numpy(x).cuda()).cpu().numpy()
    fin = x[np.isfinite(x)]
    assert out[2] == len(fin)
    assert abs(out[0] - math.fsum(fin)) <= 1e-15 * abs(math.fsum(fin)) * 4
    assert abs(out[1] - math.fsum(fin * fin)) <= 1e-13 * math.fsum(fin * fin)


def test_pair_sums_match_fsum(R):
    """rtt_pair_sums: compensated sums of row products (and of rows alone)
    against math.fsum of the same FP64 products; non-finite terms skipped
    and not counted."""
    g = np.random.default_rng(4)
    A, B, W = 3, 4, 3001
    x = g.standard_normal((A, W)) * 1e3 + 1e6
    y = g.standard_normal((B, W))
    x[1, 17] = np.nan
    y[2, 5] = np.inf
    out = R.pair_sums(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
    for a in range(A):
        for b in range(B):
            p = x[a] * y[b]
            fin = p[np.isfinite(p)]
            assert out[a, b, 1] == len(fin)
            assert abs(out[a, b, 0] - math.fsum(fin)) <= 4e-16 * math.fsum(np.abs(fin))
    rows = R.pair_sums(torch.from_numpy(x).cuda()).cpu().numpy()
    for a in range(A):
        fin = x[a][np.isfinite(x[a])]
        assert rows[a, 0, 1] == len(fin) and abs(rows[a, 0, 0] - math.fsum(fin)) <= 4e-16 * math.fsum(np.abs(fin))


def test_zero_amplitude_walkers_are_flagged(R):
    N = 8
    pi = wl.path_repeat(N, 2)
    bond = wl.open_bonds(16, 4)
    cores = wl.gaussian_cores(bond, 5)
    cores[3][1][:] = 0.0                      # psi = 0 whenever s_3 = 1
    bits = wl.random_spins(16, N, 6)
    _, qc, out = run_eval(R, pi, bond, cores, N, bits, "f32")
    zero = bits[:, 3] == 1
    assert zero.any() and (~zero).any()
    assert np.all(out["status"][zero] == -5) and np.all(out["status"][~zero] == 0)
    assert np.all(np.isnan(out["logratio"][zero]))
    # the sampler never advances a zero-amplitude walker and flags it
    psi = R.RTT.create(N, pi, cores, "f32")
    spins = R.spins_to_device(wl.pack_spins(bits))
    st = torch.zeros(16, dtype=torch.int32, device="cuda")
    before = spins.clone()
    psi.sweep(spins, seed=1, n_sweeps=2, status=st)
    torch.cuda.synchronize()
    z = torch.from_numpy(zero).cuda()
    assert torch.equal(spins[z], before[z])
    assert torch.all(st[z] == -5) and torch.all(st[~z] == 0)


def test_determinism(R):
    pi, bond, cores = case(32, 2, 64, "perm", seed=41)
    bits = wl.random_spins(50, 32, 42)
    psi = R.RTT.create(32, pi, cores, "bf16")
    sp = R.spins_to_device(wl.pack_spins(bits))
    o1 = psi.evaluate(sp)
    o2 = psi.evaluate(sp)
    torch.cuda.synchronize()
    assert torch.equal(o1["logratio"], o2["logratio"])
    a, b = sp.clone(), sp.clone()
    psi.sweep(a, seed=9, n_sweeps=2)
    psi.sweep(b, seed=9, n_sweeps=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_tiny_and_degenerate_shapes(R):
    # one spin, one core; W = 1
    for pi, bond in [([0], [1, 1]), ([0, 0, 0], [1, 3, 2, 1])]:
        cores = wl.gaussian_cores(np.array(bond), 8)
        bits = np.array([[0], [1]], dtype=np.uint8)
        _, qc, out = run_eval(R, np.array(pi), np.array(bond), cores, 1, bits, "f32")
        r_ref = orc.flip_ratios(qc, np.array(pi), bits)
        assert np.allclose(out["rsign"] * np.exp(out["logratio"]), r_ref, rtol=1e-5)


def test_chain_energy_matches_exact_enumeration(R):
    """4x4, R=2 (site order twice), chi=8, 64 walkers, 20 burn-in + 200 sweeps
    with a local-energy measurement after every sweep: the GPU mean is within
    3 sigma (tau_int error bar) of the exact <H> from all 2^16 amplitudes."""
    w = wl.SMALL_4x4
    pi, bond, cores = w.pi(), w.bond(), w.cores()
    psi = R.RTT.create(w.N, pi, cores, "f32")
    qc = device_cores(psi, bond)
    exact = orc.exact_energy(qc, pi, w.N, tfim.bonds(4, 4), w.J, w.h)
    ham = R.TFIM(4, 4, w.J, w.h)
    spins = R.spins_to_device(wl.pack_spins(w.spins()))
    psi.sweep(spins, seed=w.chain_seed, sweep0=0, n_sweeps=w.burn_in)
    series = []
    for t in range(w.sweeps):
        psi.sweep(spins, seed=w.chain_seed, sweep0=w.burn_in + t, n_sweeps=1)
        series.append(psi.local_energy(spins, ham))
    E = torch.stack(series).cpu().numpy()
    mean, sigma, tau, var = stats.energy_estimate(E)
    print(f"GPU <E> {mean:.6f} +- {sigma:.6f} (tau {tau:.2f}) exact {exact:.6f}")
    assert abs(mean - exact) < 3 * sigma


@pytest.mark.parametrize("dtype,chi", [("bf16", 32), ("fp8", 32), ("fp8", 64), ("bf16", 128), ("fp8", 128),
                                       ("bf16", 256), ("fp8", 256)])
def test_sweep_decisions_reduced_precision(R, dtype, chi):
    """BF16 / FP8 cores (hi+lo BF16 activations): one GPU sweep makes the
    oracle's decisions (same Philox words, oracle on the library's quantised
    cores) for every walker whose margins |u - r^2| all exceed 1e-2, widened
    by the condition number.  The stated tolerance (2e-2 on log-ratios)
    would allow flips up to ~4e-2; the hi+lo path is far more accurate, and
    this pins that its decisions follow the exact ones away from ties."""
    N, Rr, W = 12, 2, 24
    pi, bond, cores = case(N, Rr, chi, "perm", seed=340 + chi)
    psi = R.RTT.create(N, pi, cores, dtype)
    qc = device_cores(psi, bond)
    bits = wl.random_spins(W, N, 341)
    spins = R.spins_to_device(wl.pack_spins(bits))
    psi.sweep(spins, seed=342, rng_stream=1, sweep0=0, n_sweeps=1)
    torch.cuda.synchronize()
    got = wl.unpack_spins(R.spins_to_host(spins), N)
    ref, _, margins = mcmc.metropolis(qc, pi, bits, seed=342, stream=1, sweep0=0, n_sweeps=1, record=True)
    kap = orc.condition_numbers(qc, pi, bits)
    allow = 1e-2 * np.maximum(1.0, kap / 10.0)
    clean = np.all(np.abs(margins[0]) > allow[None, :], axis=0)
    assert clean.sum() >= W // 2, clean.sum()
    assert np.array_equal(got[clean], ref[clean])
