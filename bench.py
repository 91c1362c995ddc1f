#!/usr/bin/env python3
"""Throughput of the RTT Monte Carlo hot path on one MI355X.

Headline workload: the 16x16 periodic TFIM (N = 256, h = 3.04), R = 2
(L = 512, site order + a seeded permutation), bond 256, a linear combination
of 4 RTTs with Gaussian real weights, FP8 e4m3 cores with a power-of-two
scale per position, 16384 walkers, learned multi-spin proposal enabled.
Synthetic Gaussian cores N(0, 1/chi).

Before the timed region: burn-in sweeps, each followed by learned moves and
one online training step of the proposal network (trained on the chain's
own states), then the network is frozen.  One timed step = one
single-spin-flip Metropolis sweep of every walker + the learned
Metropolis-Hastings moves + local energies (all N flip ratios + diagonal)
of every walker + the compensated FP64 energy reduction, all on the GPU.

Prints one JSON line.  value = local-energy evaluations per second over the
whole timed region (walkers x steps / wall time), inputs resident in HBM.
effective_samples_per_s divides by the integrated autocorrelation time of
the walkers' local-energy series.  Energy errors against FP64 come from the
oracle's stored values (tests/golden, written by oracle-only scripts): per
sample on configurations the oracle's chain visited, and for the 8x8 lines
as chain means against the oracle's FP64 chain.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA peaks (FLOP/s); FP8 cores are decoded to BF16 and run on the BF16 matrix ops
PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "fp8": 2.5e15}
HBM_PEAK = 8.0e12
METRIC = "local-energy evals/s & effective samples/s at fixed energy error vs FP64"
HEADLINE = "tfim16x16_R2_chi256_W16384_T4"


def schedule_rowsteps(pi, N, L, cut):
    """Useful row-vector x core products of the flip-ratio passes per walker:
    forward over positions [0, cut) and backward over [cut, L), each step
    advancing the base vector and every spawned flipped vector."""
    fwd, seen = 0, set()
    for k in range(cut):
        seen.add(int(pi[k]))
        fwd += 1 + len(seen)
    bwd, seen = 0, set()
    for k in range(L - 1, cut - 1, -1):
        seen.add(int(pi[k]))
        bwd += 1 + len(seen)
    return fwd, bwd


def sweep_rowsteps(pi, N, L):
    """Row-vector x core products a sweep needs per walker: the amplitude (L)
    plus, for each proposal, the positions from the spin's first replica to
    its last one (with the prefix and the right environment of the current
    configuration at hand, the rest of the train is the current amplitude's).
    The sampler performs somewhat more: its right environments are kept only
    at checkpoint bonds, and the batched kernels contract every proposal's
    columns from the right boundary."""
    first, last = {}, {}
    for k, j in enumerate(pi):
        first.setdefault(int(j), k)
        last[int(j)] = k
    return L + sum(last[j] - first[j] + 1 for j in first)


def baseline_sweep_rowsteps(pi, N, L):
    """Row-vector x core products per walker of a sweep whose flipped row
    runs from the spin's first position to the end of the train, with the
    prefix kept current by one step per proposal: sum_j (L - first(j)) + the
    number of spins read.  This is the per-walker algorithmic work the
    roofline fraction is quoted on; sweep_rowsteps gives the stricter
    minimum beside it."""
    first = {}
    for k, j in enumerate(pi):
        first.setdefault(int(j), k)
    return len(first) + sum(L - f for f in first.values())


# Sources that define or launch the matrix-core kernels, and the build flags:
# counter figures taken on other versions of these are stale.  (The host
# tensor-train algebra, the narrow-bond and the learned-proposal kernels
# cannot change what the matrix-core kernels read and write.)
KERNEL_SOURCES = ("csrc/rtt_device.hpp", "csrc/rtt_kernels.hpp", "csrc/rtt_lib.hip", "build.py")


def src_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2604_22718_amd", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("src_hash") != src_hash():
        return None
    return d.get("bytes_per_launch")



def run_batched(steps, n_rtt=256):
    """256 uneven RTTs (side 4..10, R 2..3, chi 16..128, 256..4096 walkers,
    BF16) stepped together: each step = 1 sweep + local energies of every
    walker of every RTT, one captured graph of persistent kernels whose
    launch shape and per-class sampler tiles the autotuner picks."""
    import tempfile

    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    t0 = time.perf_counter()
    ws = wl.batched_workloads(n_rtt)
    rtts, hams, spins = [], [], []
    flops_le = flops_sw = 0.0
    per_class = {}
    for w in ws:
        pi = w.pi()
        rtts.append(R.RTT.create(w.N, pi, w.cores(), "bf16"))
        hams.append(R.TFIM(w.Lx, w.Ly, w.J, w.h))
        spins.append(R.spins_to_device(wl.pack_spins(w.spins())))
        info = R.rtt_info(rtts[-1].handle)
        f, b = schedule_rowsteps(pi, w.N, w.L, info["cut"])
        le = w.W * (f + b) * 2.0 * info["chi"] ** 2
        sw = w.W * baseline_sweep_rowsteps(pi, w.N, w.L) * 2.0 * info["chi"] ** 2
        flops_le += le
        flops_sw += sw
        c = per_class.setdefault(info["chi"], {"runs": 0, "walkers": 0, "algorithmic_flops": 0.0})
        c["runs"] += 1
        c["walkers"] += w.W
        c["algorithmic_flops"] += le + sw
    batch = R.Batch(rtts, hams, spins, seed=3100)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    cache = os.path.join(tempfile.mkdtemp(), "tune.jsonl")
    choice = batch.autotune(n_sweeps=1, reps=1, cache_path=cache)
    tune = time.perf_counter() - t1
    rec = json.loads(open(cache).read().splitlines()[-1])
    for c in rec["classes"]:
        if c["bond"] in per_class:
            per_class[c["bond"]]["sampler_walkers_per_block"] = c["sampler_walkers_per_block"]
    batch.step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        batch.step(1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    walkers = sum(w.W for w in ws)
    tot = flops_le + flops_sw
    for c in per_class.values():
        c["share_of_work"] = c["algorithmic_flops"] / tot
    res = {"workload": f"{n_rtt} uneven RTTs (side 4-10, R 2-3, chi 16-128, 256-4096 walkers), bf16",
           "walkers": walkers, "steps": steps, "ms_per_step": ms,
           "local_energy_evals_per_s": walkers / (ms * 1e-3),
           "algorithmic_tflops": tot / (ms * 1e-3) / 1e12,
           "frac_of_bf16_peak": tot / (ms * 1e-3) / PEAK["bf16"],
           "autotuned": {"concurrent_classes": choice[0], "blocks_per_cu": choice[1], "trials": rec["trials"]},
           "classes_by_bond": {str(k): v for k, v in sorted(per_class.items())},
           "setup_s": setup, "autotune_s": tune}
    batch.close()
    return res


def compare_learned(psi, ham, net, spins0, N, seed, n_meas, train_steps, learned_per_sweep, burn, lr,
                    sigma_target):
    """Single-flip sweeps against sweeps + learned MH moves on the same state
    and walkers: burn-in, online training of the network on the chain's own
    states (then frozen), and n_meas measurements of every walker's E_loc per
    chain.  Both chains sample |psi|^2 exactly; the wall time to bring the
    error of the mean energy to sigma_target (per site) is
    (sigma_E / sigma_target)^2 / ESS-rate, so ESS/s orders them at equal
    energy error."""
    import torch

    from paper_2604_22718_amd import rtt as R
    W = spins0.shape[0]
    out = {"walkers": W, "burn_in_sweeps": burn, "measurements": n_meas}
    ch = R.LearnedChain(psi, net, spins0.clone(), seed=seed)
    t0 = time.perf_counter()
    ch.sweep(burn)
    for it in range(train_steps):
        ch.learned_step()
        ch.train(lr=lr)
        if it % 4 == 3:
            ch.sweep(1)
    torch.cuda.synchronize()
    out["burn_in_and_training_s"] = time.perf_counter() - t0
    out["train_steps"] = train_steps
    eloc = torch.empty(W, dtype=torch.float64, device="cuda")

    def measure(learned):
        c = R.LearnedChain(psi, net, ch.spins.clone(), seed=seed + 1, rng_stream=1 + int(learned))
        c.sweep(5)
        torch.cuda.synchronize()
        series = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        for t in range(n_meas):
            c.sweep(1)
            if learned:
                for _ in range(learned_per_sweep):
                    c.learned_step()
            R.rtt_evaluate(psi.handle, ham.handle, c.spins, eloc=eloc)
            series.append(eloc.clone())
        ev[1].record()
        torch.cuda.synchronize()
        secs = ev[0].elapsed_time(ev[1]) * 1e-3
        ev[2].record()
        c.sweep(1)
        ev[3].record()
        torch.cuda.synchronize()
        E = torch.stack(series).cpu().numpy()
        st = energy_stats(E, N)
        ess = W * n_meas / st["tau_int"] / secs
        sig = float(E.std()) / N
        res = {"seconds": secs, "tau_int": st["tau_int"], "E_per_site": st["E_per_site"],
               "sigma_of_mean_per_site": st["sigma_per_site"], "sigma_E_per_sample_per_site": sig,
               "effective_samples_per_s": ess,
               "seconds_to_sigma_target": (sig / sigma_target) ** 2 / ess,
               "sweep_ms": ev[2].elapsed_time(ev[3]),
               "single_flip_acceptance": c.acc_flip.sum().item() / (W * N * (n_meas + 6))}
        if learned:
            ev[2].record()
            c.learned_step()
            ev[3].record()
            torch.cuda.synchronize()
            res["learned_move_ms"] = ev[2].elapsed_time(ev[3])
            res["learned_acceptance"] = c.acc_learn.sum().item() / (W * learned_per_sweep * n_meas + W)
        return res

    out["sigma_target_per_site"] = sigma_target
    out["single_flip"] = measure(False)
    out["single_flip_plus_learned"] = measure(True)
    # the network's forward pass alone over every walker (head outputs to HBM)
    net.forward(ch.spins)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(10):
        net.forward(ch.spins)
    ev[1].record()
    torch.cuda.synchronize()
    out["network_forward_ms"] = ev[0].elapsed_time(ev[1]) / 10
    out["network_forward_over_sweep"] = out["network_forward_ms"] / out["single_flip"]["sweep_ms"]
    out["learned_moves_per_sweep"] = learned_per_sweep
    out["ess_gain"] = (out["single_flip_plus_learned"]["effective_samples_per_s"]
                       / out["single_flip"]["effective_samples_per_s"])
    out["tau_ratio"] = out["single_flip"]["tau_int"] / out["single_flip_plus_learned"]["tau_int"]
    return out


def run_learned(n_meas=200, train_steps=150, learned_per_sweep=4):
    """10x10 periodic TFIM, R = 3, chi = 128, 8192 walkers, BF16 cores (the
    learned-proposal workload): single-flip sweeps against sweeps + learned
    moves, network trained online on the chain and then frozen."""
    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.LARGE_10x10
    psi = R.RTT.create(w.N, w.pi(), w.cores(), "bf16")
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    net = R.Net(w.Lx, w.Ly, wl.net_init_params(4004))
    spins0 = R.spins_to_device(wl.pack_spins(w.spins()))
    out = {"workload": w.name}
    out.update(compare_learned(psi, ham, net, spins0, w.N, w.chain_seed, n_meas, train_steps,
                               learned_per_sweep, w.burn_in, 2e-3, sigma_target=1e-4))
    net.close()
    psi.close()
    ham.close()
    return out


def run_learned_chi2(n_meas=300, train_steps=300, learned_per_sweep=2, burn=50, W=4096, power_steps=120):
    """The bond-2 state of the paper's pipeline (10x10 open lattice, h = 3,
    H+V+D+D' path, replica-space power method with H-bar_HV from the
    constant train), where single-flip sweeps decorrelate more slowly than
    on random cores: single-flip sweeps against sweeps + learned moves."""
    from paper_2604_22718_amd import pipeline
    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    L, hx = 10, 3.0
    N = L * L
    t0 = time.perf_counter()
    pi, phi = pipeline.power_method(L, L, "HV", hx, 0.1, power_steps, chi=2, chi_sum=8, periodic=False)
    out = {"workload": f"tfim{L}x{L}_open_h3_path_HVDDp_chi2_HV", "power_steps": power_steps,
           "power_method_s": time.perf_counter() - t0}
    psi = R.RTT.create(N, pi, phi, "f32")
    ham = R.TFIM(L, L, 1.0, hx, periodic=False)
    net = R.Net(L, L, wl.net_init_params(4006))
    out["narrow_kernels"] = bool(psi.info.get("narrow", 0))
    spins0 = R.spins_to_device(wl.pack_spins(wl.random_spins(W, N, 4007)))
    out.update(compare_learned(psi, ham, net, spins0, N, 4008, n_meas, train_steps, learned_per_sweep, burn,
                               2e-3, sigma_target=1e-5))
    net.close()
    psi.close()
    ham.close()
    return out


def run_wide(name, n_eval=3, with_sweep=True):
    """Local energies (and one sweep) of a wide-bond workload: 10x10, R=3,
    chi=128, 8192 walkers, BF16 (or 16x16, R=2, chi=256, 16384 walkers,
    4-term FP8 combination).  Reports algorithmic TFLOP/s against the BF16
    MFMA peak; with hi+lo BF16 activations the matrix cores execute twice
    the algorithmic flops, which mfma_frac_hilo counts."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.WORKLOADS[name]
    dtype = "bf16" if w.chi <= 128 else "fp8"
    pi = w.pi()
    if w.n_terms > 1:
        terms = [R.RTT.create(w.N, pi, w.cores(t), dtype) for t in range(w.n_terms)]
        psi = R.RTT.lincomb(terms, w.coeffs())
        del terms
    else:
        psi = R.RTT.create(w.N, pi, w.cores(), dtype)
    info = R.rtt_info(psi.handle)
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    bits = w.spins()
    spins = R.spins_to_device(wl.pack_spins(bits))
    eloc = torch.empty(w.W, dtype=torch.float64, device="cuda")
    R.rtt_evaluate(psi.handle, ham.handle, spins, eloc=eloc)
    err = sampled_energy_error(R, psi, ham, w.name, dtype)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(n_eval):
        R.rtt_evaluate(psi.handle, ham.handle, spins, eloc=eloc)
    e[1].record()
    if with_sweep:
        psi.sweep(spins, seed=w.chain_seed, sweep0=0, n_sweeps=1)
    e[2].record()
    torch.cuda.synchronize()
    le_ms = e[0].elapsed_time(e[1]) / n_eval
    T = w.n_terms
    fwd, bwd = schedule_rowsteps(pi, w.N, w.L, info["cut"])
    le_flops = w.W * T * (fwd + bwd) * 2.0 * w.chi * w.chi
    out = {"workload": w.name, "dtype": dtype, "walkers": w.W, "row_groups": info["groups"],
           "le_evals_per_s": w.W / (le_ms * 1e-3), "le_ms": le_ms,
           "le_algorithmic_tflops": le_flops / (le_ms * 1e-3) / 1e12,
           "le_frac_bf16_peak": le_flops / (le_ms * 1e-3) / PEAK["bf16"],
           "le_mfma_frac_hilo": 2 * le_flops / (le_ms * 1e-3) / PEAK["bf16"]}
    if with_sweep:
        sw_ms = e[1].elapsed_time(e[2])
        sw_flops = w.W * T * baseline_sweep_rowsteps(pi, w.N, w.L) * 2.0 * w.chi * w.chi
        sw_min = w.W * T * sweep_rowsteps(pi, w.N, w.L) * 2.0 * w.chi * w.chi
        out.update({"sweep_ms": sw_ms, "sweep_algorithmic_tflops": sw_flops / (sw_ms * 1e-3) / 1e12,
                    "sweep_frac_bf16_peak": sw_flops / (sw_ms * 1e-3) / PEAK["bf16"],
                    "sweep_frac_bf16_peak_method_minimum": sw_min / (sw_ms * 1e-3) / PEAK["bf16"]})
    out["energy_error"] = err
    psi.close()
    ham.close()
    torch.cuda.empty_cache()
    return out



def run_dual(steps=5, warmup=1):
    """Dual Monte Carlo step on the 8x8 workload (chi=64, FP32, 4096 walkers
    per chain): three states (the workload's RTT, a second seeded RTT and
    their combination 0.8 a - 1.1 b); for each state one sweep of its own
    chain, then overlap and mixed-energy estimators of its walkers against
    all three states (rows of H~ and S~)."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.MEDIUM_8x8
    pi = w.pi()
    a = R.RTT.create(w.N, pi, w.cores(), "f32")
    b = R.RTT.create(w.N, pi, wl.gaussian_cores(w.bond(), w.core_seed + 5), "f32")
    c = R.RTT.lincomb([a, b], np.array([0.8, -1.1]))
    states = [a, b, c]
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    W, M = w.W, len(states)
    chains = []
    for i in range(M):
        spins = R.spins_to_device(wl.pack_spins(wl.random_spins(W, w.N, w.chain_seed + 10 + i)))
        la = torch.empty(W, dtype=torch.float64, device="cuda")
        sg = torch.empty(W, dtype=torch.int8, device="cuda")
        chains.append((spins, la, sg))
    # per step and sampled state: the library's compensated row sums of both estimators
    sums = torch.zeros((steps + warmup, M, 2, M, 1, 2), dtype=torch.float64, device="cuda")

    def step(t):
        for i, (spins, la, sg) in enumerate(chains):
            states[i].sweep(spins, seed=w.chain_seed, rng_stream=100 + i, sweep0=t, n_sweeps=1, logabs=la, sign=sg)
            ratio, mixed, _ = R.mixed_estimators(states, ham, spins, la, sg)
            R.rtt_pair_sums(ratio, None, sums[t, i, 0])
            R.rtt_pair_sums(mixed, None, sums[t, i, 1])

    for t in range(warmup):
        step(t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(steps):
        step(warmup + t)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    X = sums.cpu().numpy()
    S = (X[:, :, 0, :, 0, 0] / X[:, :, 0, :, 0, 1]).mean(axis=0)
    H = (X[:, :, 1, :, 0, 0] / X[:, :, 1, :, 0, 1]).mean(axis=0)
    out = {"workload": w.name + "_dual3", "states": M, "walkers_per_chain": W, "ms_per_step": ms,
           "mixed_estimator_evals_per_s": W * M * M / (ms * 1e-3),
           "step": "per state: 1 sweep + overlap and mixed-energy estimators against all 3 states",
           "S_tilde_diag": np.diag(S).tolist(), "H_tilde_diag_per_site": (np.diag(H) / w.N).tolist()}
    for x in states[::-1]:
        x.close()
    ham.close()
    return out



def time_narrow(N, pi, cores, ham, W=4096, reps=20):
    """Sweep and local-energy times of a narrow-bond train (every bond <= 4)
    with HIP events, and their algorithmic FP32 rates: an amplitude costs
    sum_k 2 chi_k chi_{k+1} flops (row vector times the selected slice); a
    local energy needs N + 1 of them, a sweep proposal for spin j the part
    of the train from its first position on (the prefix is shared)."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    psi = R.RTT.create(N, pi, cores, "f32")
    assert psi.info["narrow"] in (2, 4), "narrow-bond path not taken"
    bond = [1] + [c.shape[2] for c in cores]
    per_pos = np.array([2.0 * bond[k] * bond[k + 1] for k in range(len(cores))])
    tail = np.concatenate([np.cumsum(per_pos[::-1])[::-1], [0.0]])
    first = {}
    for k, j in enumerate(pi):
        first.setdefault(int(j), k)
    sweep_flops = W * sum(tail[f] for f in first.values())
    le_flops = W * (len(first) + 1) * tail[0]
    sp = R.spins_to_device(wl.pack_spins(wl.random_spins(W, N, 77)))
    psi.sweep(sp, seed=3, n_sweeps=2)
    psi.local_energy(sp, ham)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for t in range(reps):
        psi.sweep(sp, seed=3, sweep0=2 + t, n_sweeps=1)
    ev[1].record()
    for t in range(reps):
        psi.local_energy(sp, ham)
    ev[2].record()
    torch.cuda.synchronize()
    sweep_ms, le_ms = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    psi.close()
    peak = 157.3
    return {"walkers": W, "sweep_ms": sweep_ms, "local_energy_ms": le_ms,
            "sweep": {"bound": "alu", "achieved": sweep_flops / (sweep_ms * 1e9), "peak": peak,
                      "unit": "TFLOP/s", "frac": sweep_flops / (sweep_ms * 1e9) / peak},
            "local_energy": {"bound": "alu", "achieved": le_flops / (le_ms * 1e9), "peak": peak,
                             "unit": "TFLOP/s", "frac": le_flops / (le_ms * 1e9) / peak}}



# Operator sets of the paper's physical-space table (rows in its order) and
# the energies per site and V-scores it reports for them at 10x10, h = 3.
PAPER_TABLE = [
    (("ZZ_HV", "ZZ_DD'"), -3.1682, 0.0013),
    (("ZZ_HV", "ZZ_DD'", "X"), -3.1682, 0.0013),
    (("ZZ_HV", "X"), -3.163, 0.005),
    (("ZZ_DD'", "X"), -3.1682, 0.0013),
    ((), -3.163, 0.005),
]


def run_paper_pipeline(L=10, steps=120, phys_steps=2, table=False):
    """The paper's chi = 2 pipeline on an L x L open lattice, h = 3 (the
    setting of its physical-space table): H+V+D+D' path, replica-space power
    method with H-bar_HV (tau = 0.1, host rounding, partial sums at rank 8)
    from the constant train, then physical-space steps with I, O_X,
    O_ZZ,HV, O_ZZ,DD'.  Energies from GPU chains (FP32, 4096 walkers)."""
    import time

    import torch

    from paper_2604_22718_amd import pipeline
    from paper_2604_22718_amd import rtt as R
    N, hx = L * L, 3.0
    ham = R.TFIM(L, L, 1.0, hx, periodic=False)
    def progress(p, _):
        if (p + 1) % 20 == 0:
            print(f"[paper pipeline] power step {p + 1}/{steps}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    pi, phi = pipeline.power_method(L, L, "HV", hx, 0.1, steps, chi=2, chi_sum=8, periodic=False,
                                    callback=progress)
    host_ms = (time.perf_counter() - t0) * 1e3 / steps

    def energy(cores, seed):
        psi = R.RTT.create(N, pi, cores, "f32")
        r = pipeline.vmc_energy(psi, ham, 4096, 50, 200, seed=seed)
        psi.close()
        return {"E_per_site": r["mean"] / N, "sigma_per_site": r["sigma"] / N, "v_score": r["v_score"]}

    phi0 = phi
    out = {"workload": f"tfim{L}x{L}_open_h3_path_HVDDp_chi2", "power_steps": steps,
           "power_step_host_ms": host_ms, "replica_HV": energy(phi, 1200), "physical": []}
    for it in range(phys_steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        phi, info = pipeline.physical_space_step(pi, phi, L, L, ["I", "X", "ZZ_HV", "ZZ_DD'"], 2, ham, 4096, 300,
                                                 200, seed=1300 + 10 * it, chi_sum=8, periodic=False)
        torch.cuda.synchronize()
        out["physical"].append({"lambda_per_site": info["lambda"] / N, "coeffs": info["coeffs"],
                                "step_s": time.perf_counter() - t, **energy(phi, 1400 + it)})
    if L == 10:
        out["paper_table_context"] = {"replica_HV_only": {"E_per_site": -3.163, "v_score": 0.005},
                                      "with_ZZ_DDp": {"E_per_site": -3.1682, "v_score": 0.0013}}
    if table:   # every operator set of the table, each from the same replica-space state
        rows = []
        # Z-only sets run twice: dual Monte Carlo, and one chain on the first state
        cases = [(ops, e, v, "dual") for ops, e, v in PAPER_TABLE]
        cases += [(ops, e, v, "single") for ops, e, v in PAPER_TABLE if ops and "X" not in ops]
        for ops, e_paper, v_paper, sampling in cases:
            cur = phi0
            row = {"operators": ["I", *ops], "sampling": sampling, "paper_E_per_site": e_paper,
                   "paper_v_score": v_paper}
            t_row = time.perf_counter()
            for it in range(phys_steps if ops else 0):
                cur, info = pipeline.physical_space_step(pi, cur, L, L, ["I", *ops], 2, ham, 4096, 300, 200,
                                                         seed=1500 + 10 * it + len(rows), chi_sum=8,
                                                         periodic=False, sampling=sampling)
                row["lambda_per_site"] = info["lambda"] / N
            row["steps_s"] = time.perf_counter() - t_row
            row.update(energy(cur, 1600 + len(rows)))
            rows.append(row)
            print(f"[paper pipeline] table row {len(rows)}: {row['operators']} E/N {row['E_per_site']:.5f}",
                  file=sys.stderr, flush=True)
        out["table"] = rows
    if L == 20:   # reference energy quoted by the paper for its replica-space runs at this size
        out["paper_reference_E_per_site"] = -3.18185
    out["narrow_kernels"] = time_narrow(N, pi, phi, ham)
    ham.close()
    return out




# ------------------------------------------------------------------ statistics
def tau_int(E, c=5.0):
    """Integrated autocorrelation time tau = 1 + 2 sum_t rho(t) of a (T,) or
    (T, W) series (Sokal's window, c = 5).  With many walkers the
    autocovariance is averaged over walkers around the global mean, so a
    short series of many walkers still resolves rho(t) at small t.  A series
    without fluctuations has tau = 1."""
    x = np.asarray(E, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    if T < 2:
        return 1.0
    d = x - x.mean()
    c0 = np.mean(d * d)
    if not c0 > 0:
        return 1.0
    tau = 1.0
    for M in range(1, T):
        tau += 2.0 * np.mean(d[: T - M] * d[M:]) / c0
        if M >= c * tau:
            break
    return max(tau, 1.0)


def energy_stats(E, N):
    """Mean (exactly rounded), variance, tau_int, sigma of the mean and the
    V-score N var / E^2 of a (T, W) local-energy series."""
    x = np.asarray(E, dtype=np.float64)
    mean = math.fsum(x.ravel()) / x.size
    var = float(np.mean((x - mean) ** 2))
    tau = tau_int(x)
    sigma = math.sqrt(var * tau / x.size)
    return {"E_per_site": mean / N, "sigma_per_site": sigma / N, "tau_int": tau, "var_eloc": var,
            "v_score": N * var / (mean * mean) if mean != 0 else None, "samples": int(x.size)}


# ------------------------------------------------------------------ stored FP64 references
def golden(name, dtype):
    """Configurations the oracle's chain visited and its FP64 values there,
    stored by tests/golden/make_sampled_refs.py (None if absent)."""
    p = os.path.join(ROOT, "tests", "golden", "sampled_refs.json")
    if not os.path.exists(p):
        return None
    for c in json.load(open(p))["cases"]:
        if c["workload"] == name and c["dtype"] == dtype:
            out = dict(c)
            for k in ("start", "sampled", "after", "final"):
                out[k] = np.array([[int(x, 16) for x in row] for row in c[k]], dtype=np.uint64)
            return out
    return None


def sampled_energy_error(R, psi, ham, name, dtype):
    """GPU local energies on the oracle-sampled configurations against the
    oracle's FP64 values on the same quantised cores (arithmetic error) and
    on the unquantised FP64 cores (arithmetic + state quantisation)."""
    import torch
    g = golden(name, dtype)
    if g is None:
        return None
    spins = R.spins_to_device(g["sampled"])
    out = psi.evaluate(spins, ham)
    torch.cuda.synchronize()
    e = out["eloc"].cpu().numpy()
    q, u = np.array(g["eloc_quantised_cores"]), np.array(g["eloc_fp64_cores"])
    rq = np.abs(e - q) / np.maximum(1.0, np.abs(q))
    ru = np.abs(e - u) / np.maximum(1.0, np.abs(u))
    # every flip ratio of those configurations against the oracle's FP64
    # ratios: the stated bar unscaled, and how far each ratio is inside
    # its condition-number-scaled bound tol * max(1, kappa / 10)
    r_ref = np.asarray(g["flip_ratios"], dtype=np.float64)
    kap = np.asarray(g["flip_kappa"], dtype=np.float64)
    lr = out["logratio"].cpu().numpy()
    nz = r_ref != 0
    dlog = np.abs(lr[nz] - np.log(np.abs(r_ref[nz])))
    tol = 1e-5 if dtype == "f32" else 2e-2
    allow = tol * np.maximum(1.0, kap[nz] / 10.0)
    ratios = {"n": int(nz.sum()), "tol": tol, "frac_within_tol": float(np.mean(dlog <= tol)),
              "p999": float(np.quantile(dlog, 0.999)), "max": float(dlog.max()),
              "n_well_conditioned": int(np.sum(kap[nz] <= 10.0)),
              "n_held_to_scaled_bound_only": int(np.sum(kap[nz] > 10.0)),
              "worst_ratio_to_scaled_bound": float(np.max(dlog / allow)),
              "sign_errors": int(np.sum(np.sign(r_ref[nz]) != out["rsign"].cpu().numpy()[nz]))}
    return {"walkers": len(e), "configurations": f"oracle Metropolis chain, {g['burn']} sweeps from the seeded walkers",
            "max_rel_vs_fp64_same_cores": float(rq.max()), "median_rel_vs_fp64_same_cores": float(np.median(rq)),
            "mean_diff_vs_fp64_same_cores": float(np.mean(e - q)),
            "max_rel_vs_fp64_unquantised_cores": float(ru.max()),
            "mean_diff_vs_fp64_unquantised_cores": float(np.mean(e - u)),
            "flip_ratios_vs_fp64_same_cores": ratios,
            "reference": "tests/golden/sampled_refs.json"}


def build_state(R, w, dtype):
    pi = w.pi()
    if w.n_terms == 1:
        return R.RTT.create(w.N, pi, w.cores(), dtype)
    terms = [R.RTT.create(w.N, pi, w.cores(t), dtype) for t in range(w.n_terms)]
    psi = R.RTT.lincomb(terms, w.coeffs())
    for t in terms:
        t.close()
    return psi


def core_bytes(w, chi_pad, dtype):
    """Device bytes of the packed cores: both fragment layouts, every term."""
    eb = {"f32": 4, "bf16": 2, "fp8": 1}[dtype]
    return 2 * w.n_terms * w.L * 2 * chi_pad * chi_pad * eb


# ------------------------------------------------------------------ headline
def headline(steps, warmup, burn, learned_per_step=2, lr=1e-3):
    """The 16x16 chi=256 four-term FP8 workload with the learned proposal
    (see the module docstring).  Returns the bench record."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.WORKLOADS[HEADLINE]
    dtype = w.dtype
    t_setup = time.perf_counter()
    psi = build_state(R, w, dtype)
    info = psi.info
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    net = R.Net(w.Lx, w.Ly, wl.net_init_params(4005))
    spins = R.spins_to_device(wl.pack_spins(w.spins()))
    ch = R.LearnedChain(psi, net, spins, seed=w.chain_seed)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    err = sampled_energy_error(R, psi, ham, w.name, dtype)

    # burn-in with online training of the proposal network on the chain's states
    t_burn = time.perf_counter()
    burn_means = []
    for t in range(burn):
        ch.sweep(1)
        for _ in range(learned_per_step):
            ch.learned_step()
            ch.train(lr=lr)
        if t % 5 == 4 or t == burn - 1:
            burn_means.append(float(psi.local_energy(ch.spins, ham).mean().item()) / w.N)
        print(f"[bench] burn-in sweep {t + 1}/{burn}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    burn_s = time.perf_counter() - t_burn
    acc_flip0, acc_learn0 = ch.acc_flip.sum().item(), ch.acc_learn.sum().item()
    sweeps0, steps0 = ch.sweeps, ch.steps

    W = w.W
    eloc = torch.empty(W, dtype=torch.float64, device="cuda")
    red = torch.empty(3, dtype=torch.float64, device="cuda")
    series, sums = [], []

    def step(ev=None):
        if ev: ev[0].record()
        ch.sweep(1)
        if ev: ev[1].record()
        for _ in range(learned_per_step):
            ch.learned_step()
        if ev: ev[2].record()
        R.rtt_evaluate(psi.handle, ham.handle, ch.spins, eloc=eloc)
        if ev: ev[3].record()
        R.rtt_energy_reduce(eloc, red)
        if ev: ev[4].record()
        series.append(eloc.clone())
        sums.append(red.clone())

    for t in range(warmup):
        step()
        print(f"[bench] warm-up step {t + 1}/{warmup}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    series.clear()
    sums.clear()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        step(evs[t])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {steps} timed steps in {dt:.1f} s", file=sys.stderr, flush=True)
    ms = lambda a, b: np.array([e[a].elapsed_time(e[b]) for e in evs])
    sweep_ms, learn_ms, eval_ms, red_ms = ms(0, 1), ms(1, 2), ms(2, 3), ms(3, 4)

    E = torch.stack(series).cpu().numpy()            # (steps, W)
    S = torch.stack(sums).cpu().numpy()              # (steps, 3): library's compensated sums
    st = energy_stats(E, w.N)
    st["E_per_site_library_reduce"] = float(S[:, 0].sum() / S[:, 2].sum()) / w.N
    st["finite_fraction"] = float(S[:, 2].sum() / (W * steps))

    pi, T, chi = w.pi(), w.n_terms, info["chi"]
    fwd, bwd = schedule_rowsteps(pi, w.N, w.L, info["cut"])
    row = 2.0 * chi * chi
    le_flops = W * T * (fwd + bwd) * row
    sw_flops = W * T * baseline_sweep_rowsteps(pi, w.N, w.L) * row
    sw_min = W * T * sweep_rowsteps(pi, w.N, w.L) * row
    am_flops = W * T * w.L * row                      # one amplitude per learned move
    kernels = {
        "chain_kernel (1 sweep)": {"ms": float(sweep_ms.mean()), "algorithmic_flops": sw_flops,
                                   "tflops": sw_flops / (sweep_ms.mean() * 1e-3) / 1e12,
                                   "algorithmic_flops_method_minimum": sw_min},
        f"learned moves x{learned_per_step} (network kernels + chain_kernel amplitudes)":
            {"ms": float(learn_ms.mean()), "algorithmic_flops_amplitudes": learned_per_step * am_flops},
        "pass_kernel x2 + combine (local energies)": {"ms": float(eval_ms.mean()), "algorithmic_flops": le_flops,
                                                      "tflops": le_flops / (eval_ms.mean() * 1e-3) / 1e12,
                                                      "frac_bf16_peak": le_flops / (eval_ms.mean() * 1e-3) / PEAK["bf16"]},
        "reduce_kernel": {"ms": float(red_ms.mean())},
    }
    ach = sw_flops / (sweep_ms.mean() * 1e-3)
    ach_min = sw_min / (sweep_ms.mean() * 1e-3)
    nm = "chain_kernel"
    if eval_ms.mean() > sweep_ms.mean():
        ach, nm = le_flops / (eval_ms.mean() * 1e-3), "pass_kernel+combine"
        ach_min = ach
    roof = {"kernel": nm, "bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[dtype] / 1e12,
            "unit": "TFLOP/s", "frac": ach / PEAK[dtype],
            "achieved_method_minimum": ach_min / 1e12, "frac_method_minimum": ach_min / PEAK[dtype],
            "traffic": traffic_from_profile(nm, w.name),
            "traffic_note": "bytes fetched past L2 (MALL hits included) and written, per launch, from the committed "
                            "counter summary of the same kernel sources",
            "flop_count": "per walker-sweep and term, sum_j (L - first_j) + N row-steps of 2 chi^2 flops (a "
                          "sweep whose flipped rows run from the spin's first position to the end of the train); "
                          "*_method_minimum: L + sum_j (last_j - first_j + 1) row-steps, what a sweep needs with "
                          "both environments of every bond at hand.  Neither counts the hi+lo activation split "
                          "or the second core slice, which the matrix ops also execute"}
    if roof["traffic"] is not None:   # the rate those bytes imply at the measured launch time
        t_ms = sweep_ms.mean() if nm == "chain_kernel" else eval_ms.mean()
        roof["traffic_TB_per_s"] = roof["traffic"] / (t_ms * 1e-3) / 1e12
    ess = W * steps / st["tau_int"]
    n_fl = (ch.sweeps - sweeps0) * W * w.N
    n_le = (ch.steps - steps0) * W
    res = {
        "metric": METRIC, "value": W * steps / dt, "unit": "local-energy evals/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (seeded Gaussian cores, seeded walkers)",
        "config": {"workload": w.name, "lattice": f"{w.Lx}x{w.Ly} periodic TFIM", "J": w.J, "h": w.h,
                   "R": w.R, "L": w.L, "chi": w.chi, "terms": T, "walkers": W, "core_dtype": "fp8_e4m3",
                   "core_bytes_on_device": core_bytes(w, chi, "fp8"),
                   "learned_proposal": {"enabled": True, "moves_per_step": learned_per_step,
                                        "trained_steps": burn * learned_per_step, "frozen_when_timed": True},
                   "burn_in_sweeps": burn,
                   "step": "1 Metropolis sweep + learned MH moves + local energies of all walkers + FP64 reduction"},
        "effective_samples_per_s": ess / dt,
        "energy": st,
        "energy_error": err,
        "acceptance": {"single_flip": (ch.acc_flip.sum().item() - acc_flip0) / max(1, n_fl),
                       "learned": (ch.acc_learn.sum().item() - acc_learn0) / max(1, n_le)},
        "burn_in": {"seconds": burn_s, "E_per_site_every_5_sweeps": burn_means},
        "setup_s": setup_s,
        "kernels": kernels,
        "roofline": roof,
    }
    net.close()
    psi.close()
    ham.close()
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------ 8x8 chains
def chain_line(dtype, burn=None, meas=None):
    """8x8, chi = 64, 4096 walkers: burn-in, then measured steps of one sweep +
    local energies + FP64 reduction.  Energy against the oracle's FP64 chain
    (16 of the same walkers, same Philox words, stored) and, where the
    trajectories coincide (FP32), sample by sample."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.MEDIUM_8x8
    burn = w.burn_in if burn is None else burn
    meas = w.sweeps if meas is None else meas
    psi = build_state(R, w, dtype)
    info = psi.info
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    spins = R.spins_to_device(wl.pack_spins(w.spins()))
    W = w.W
    eloc = torch.empty(W, dtype=torch.float64, device="cuda")
    red = torch.empty(3, dtype=torch.float64, device="cuda")
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    # burn-in and the oracle's decision sweep: sweeps 0 .. burn
    psi.sweep(spins, seed=w.chain_seed, sweep0=0, n_sweeps=burn + 1)
    series = []
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(meas)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(meas):
        e = evs[t]
        e[0].record()
        psi.sweep(spins, seed=w.chain_seed, sweep0=burn + 1 + t, n_sweeps=1, accepts=acc)
        e[1].record()
        R.rtt_evaluate(psi.handle, ham.handle, spins, eloc=eloc)
        e[2].record()
        R.rtt_energy_reduce(eloc, red)
        e[3].record()
        series.append(eloc.clone())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweep_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    eval_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    E = torch.stack(series).cpu().numpy()
    st = energy_stats(E, w.N)
    out = {"workload": w.name, "dtype": dtype, "walkers": W, "burn_in_sweeps": burn + 1, "measured_steps": meas,
           "ms_per_step": dt / meas * 1e3, "le_evals_per_s": W * meas / dt,
           "effective_samples_per_s": W * meas / st["tau_int"] / dt, "energy": st,
           "acceptance": float(acc.sum().item()) / (W * w.N * meas)}
    pi, chi = w.pi(), info["chi"]
    fwd, bwd = schedule_rowsteps(pi, w.N, w.L, info["cut"])
    row = 2.0 * chi * chi
    le_flops, sw_flops = W * (fwd + bwd) * row, W * baseline_sweep_rowsteps(pi, w.N, w.L) * row
    sw_min = W * sweep_rowsteps(pi, w.N, w.L) * row
    out["kernels"] = {"chain_kernel (1 sweep)": {"ms": float(sweep_ms.mean()),
                                                 "tflops": sw_flops / (sweep_ms.mean() * 1e-3) / 1e12},
                      "pass_kernel x2 + combine": {"ms": float(eval_ms.mean()),
                                                   "tflops": le_flops / (eval_ms.mean() * 1e-3) / 1e12}}
    dom = ("chain_kernel", sw_flops, sweep_ms) if sweep_ms.mean() >= eval_ms.mean() else \
        ("pass_kernel+combine", le_flops, eval_ms)
    ach = dom[1] / (dom[2].mean() * 1e-3)
    out["roofline"] = {"kernel": dom[0], "bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[dtype] / 1e12,
                       "unit": "TFLOP/s", "frac": ach / PEAK[dtype], "traffic": traffic_from_profile(dom[0], w.name)}
    if dom[0] == "chain_kernel":
        out["roofline"]["frac_method_minimum"] = sw_min / (sweep_ms.mean() * 1e-3) / PEAK[dtype]
    g = golden(w.name, dtype)
    if g is not None:
        eo = np.array(g["eloc_series"])                  # (meas, 16): oracle FP64 chain energies
        so = energy_stats(eo, w.N)
        z = abs(st["E_per_site"] - so["E_per_site"]) / math.hypot(st["sigma_per_site"], so["sigma_per_site"])
        ee = {"oracle_chain": {"walkers": eo.shape[1], "measured_sweeps": eo.shape[0],
                               "E_per_site": so["E_per_site"], "sigma_per_site": so["sigma_per_site"]},
              "abs_diff_per_site": abs(st["E_per_site"] - so["E_per_site"]), "z": z}
        ids = np.array(g["walkers"])
        same = np.all(R.spins_to_host(spins)[ids] == g["final"], axis=1)
        ee["oracle_walkers_on_same_trajectory"] = int(same.sum())
        if same.any() and eo.shape[0] == meas:
            rel = np.abs(E[:, ids[same]] - eo[:, same]) / np.maximum(1.0, np.abs(eo[:, same]))
            ee["per_sample_on_same_trajectory"] = {"samples": int(rel.size), "max_rel": float(rel.max()),
                                                   "median_rel": float(np.median(rel)),
                                                   "mean_diff_per_site": float(np.mean(E[:, ids[same]] - eo[:, same])) / w.N}
        out["energy_error_vs_fp64"] = ee
    out["energy_error_sampled"] = sampled_energy_error(R, psi, ham, w.name, dtype)
    psi.close()
    ham.close()
    return out


# ------------------------------------------------------------------ CPU oracle
def cpu_baseline(n_props=16, n_ratios=64):
    """The FP64 oracle on the host, one BLAS thread, on a bounded sample of the
    headline workload (one walker at the first oracle-sampled configuration):
    its Metropolis sweep costs two full amplitudes (4 terms x 512 positions)
    per proposal, timed on n_props proposals and scaled to the 256 of a sweep;
    its local energy costs the N flipped amplitudes, timed on n_ratios spins
    and scaled to 256.  The two give the oracle's time for one walker-step
    (sweep + local energy), i.e. its local-energy evals/s at the step the GPU
    times (learned moves excluded: they add two network passes and one
    amplitude)."""
    from threadpoolctl import threadpool_limits

    from oracle import quant, rtt as orc
    from paper_2604_22718_amd import workloads as wl
    w = wl.WORKLOADS[HEADLINE]
    pi, c = w.pi(), w.coeffs()
    terms = [quant.quantise_cores(w.cores(t), w.dtype) for t in range(w.n_terms)]
    g = golden(w.name, w.dtype)
    s = wl.unpack_spins(g["sampled"][:1], w.N) if g is not None else w.spins(1)
    def timed(threads, n_p, n_r):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            for j in range(n_p):
                orc.lincomb_amplitudes(terms, c, pi, s)
                orc.lincomb_amplitudes(terms, c, pi, orc.flip(s, j))
            t_p = time.perf_counter() - t0
            t0 = time.perf_counter()
            orc.lincomb_flip_ratios(terms, c, pi, s, which=list(range(n_r)))
            t_r = time.perf_counter() - t0
        return t_p, t_r, t_p * w.N / n_p + t_r * w.N / n_r

    t_props, t_ratios, step_s = timed(1, n_props, n_ratios)
    ncpu = len(os.sched_getaffinity(0))
    # the same with BLAS threads on every host core, on a quarter of the sample
    a_p, a_r, a_step = timed(ncpu, max(1, n_props // 4), max(1, n_ratios // 4))
    return {"value": 1.0 / step_s, "unit": "local-energy evals/s", "cores": 1, "kind": "oracle",
            "sample": f"1 walker of the {w.name} workload (FP8-quantised cores, FP64 numpy): {n_props} Metropolis "
                      f"proposals ({t_props:.1f} s) and {n_ratios} of the {w.N} flip ratios of a local energy "
                      f"({t_ratios:.1f} s), scaled to one sweep + local energy = {step_s:.0f} s per walker-step",
            "host_cpus_available": ncpu,
            "all_cores": {"value": 1.0 / a_step, "unit": "local-energy evals/s", "cores": ncpu, "kind": "oracle",
                          "sample": f"{max(1, n_props // 4)} proposals ({a_p:.1f} s) and {max(1, n_ratios // 4)} "
                                    f"ratios ({a_r:.1f} s) of the same walker, BLAS threads = {ncpu}"}}


def cpu_baseline_8x8(n_walkers=64, n_steps=6):
    """The oracle's step (sweep + local energies) on a sample of the 8x8
    workload's walkers, one BLAS thread (beside the 8x8 lines)."""
    from threadpoolctl import threadpool_limits

    from oracle import mcmc, quant, rtt as orc, tfim
    from paper_2604_22718_amd import workloads as wl
    w = wl.MEDIUM_8x8
    pi, cores = w.pi(), quant.quantise_cores(w.cores(), "f32")
    s = w.spins(n_walkers)
    bonds = tfim.bonds(w.Lx, w.Ly)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for t in range(n_steps):
            s, _, _ = mcmc.metropolis(cores, pi, s, seed=w.chain_seed, stream=0, sweep0=t, n_sweeps=1)
            orc.local_energy(cores, pi, s, bonds, w.J, w.h)
        dt = time.perf_counter() - t0
    return {"value": n_walkers * n_steps / dt, "unit": "local-energy evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_walkers} walkers x {n_steps} steps (sweep + local energies) of {w.name}, FP64 numpy, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--burn", type=int, default=None, help="burn-in sweeps (default: the workload's, 20)")
    ap.add_argument("--learned-per-step", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-8x8", action="store_true", help="skip the 8x8 FP32 / BF16 chain lines")
    ap.add_argument("--no-wide", action="store_true", help="skip the 10x10 chi=128 BF16 wide-bond line")
    ap.add_argument("--only-8x8", action="store_true", help="only the 8x8 lines (no headline)")
    ap.add_argument("--batched", type=int, default=3, help="time the 256-RTT batch for this many steps (0: skip)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal ESS/s comparison on the 10x10, chi=128 workload")
    ap.add_argument("--no-learned-chi2", action="store_true",
                    help="skip the learned-proposal ESS/s comparison on the bond-2 H-bar_HV state (10x10 open)")
    ap.add_argument("--dual", action="store_true", help="also the dual Monte Carlo line")
    ap.add_argument("--paper-pipeline", type=int, default=0, metavar="STEPS",
                    help="also run the chi=2 power method for STEPS steps plus two physical-space steps")
    ap.add_argument("--paper-side", type=int, default=10, help="lattice side of the chi=2 pipeline (10 or 20)")
    ap.add_argument("--paper-table", action="store_true",
                    help="with --paper-pipeline: also every operator set of the physical-space table")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many MiB device-to-device 3 times (counter calibration) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for {a.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes_per_launch": n * 4}))
        return
    from paper_2604_22718_amd import workloads as wl
    if a.only_8x8:
        res = {"lines_8x8": [chain_line("f32"), chain_line("bf16")]}
        print(json.dumps(res), flush=True)
        return
    burn = wl.WORKLOADS[HEADLINE].burn_in if a.burn is None else a.burn
    res = headline(a.steps, a.warmup, burn, a.learned_per_step)
    if not a.no_8x8:
        res["lines_8x8"] = [chain_line("f32"), chain_line("bf16")]
        print("[bench] 8x8 lines done", file=sys.stderr, flush=True)
    if not a.no_wide:
        res["wide_bond"] = [run_wide("tfim10x10_R3_chi128_W8192")]
    if a.dual:
        res["dual_mc"] = run_dual()
    if a.paper_pipeline:
        res["paper_pipeline"] = run_paper_pipeline(L=a.paper_side, steps=a.paper_pipeline, table=a.paper_table)
    if a.batched:
        res["batched"] = run_batched(a.batched)
    if not a.no_learned:
        res["learned"] = run_learned()
        print("[bench] learned-proposal comparison (10x10, chi=128) done", file=sys.stderr, flush=True)
    if not a.no_learned_chi2:
        res["learned_chi2"] = run_learned_chi2()
        print("[bench] learned-proposal comparison done", file=sys.stderr, flush=True)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline()
        res["cpu_baseline"]["beside_8x8"] = cpu_baseline_8x8()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
