#!/usr/bin/env python3
"""Throughput of the RTT Monte Carlo hot path on one MI355X.

One step = one single-spin-flip Metropolis sweep of every walker + local
energies (all N flip ratios + diagonal) of every walker + the compensated
FP64 energy reduction, on the 8x8 periodic TFIM workload (N = 64, R = 2,
L = 128, chi = 64, 4096 walkers, h = 3.04; synthetic Gaussian cores).

Prints one JSON line.  value = local-energy evaluations per second over the
whole timed region (walkers x steps / time), inputs resident in HBM.
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

PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "fp8": 2.5e15}  # dense MFMA FLOP/s (fp8 cores run as bf16)
HBM_PEAK = 8.0e12
METRIC = "local-energy evals/s & effective samples/s at fixed energy error vs FP64"


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


def eloc_error(workload, dtype, e_gpu):
    """Relative error of GPU local energies of the seeded initial walkers
    against FP64 values stored by tests/golden/make_eloc_refs.py (computed by
    the oracle on the same quantised cores, and on the unquantised cores)."""
    p = os.path.join(ROOT, "tests", "golden", "eloc_fp64_refs.json")
    if not os.path.exists(p):
        return None
    for c in json.load(open(p))["cases"]:
        if c["workload"] == workload and c["dtype"] == dtype:
            idx = np.array(c["walkers"])
            got = np.asarray(e_gpu)[idx]
            q, u = np.array(c["eloc_quantised_cores"]), np.array(c["eloc_fp64_cores"])
            return {"eloc_max_rel_vs_fp64_same_cores": float(np.max(np.abs(got - q) / np.abs(q))),
                    "eloc_median_rel_vs_fp64_same_cores": float(np.median(np.abs(got - q) / np.abs(q))),
                    "eloc_max_rel_vs_fp64_unquantised_cores": float(np.max(np.abs(got - u) / np.abs(u))),
                    "sample_walkers": idx.tolist(), "reference": "tests/golden/eloc_fp64_refs.json"}
    return None


def cpu_baseline(w, n_walkers, n_steps):
    """The FP64 oracle on the host, single-threaded BLAS: the same step on a
    sample of the workload's walkers."""
    from threadpoolctl import threadpool_limits

    from oracle import mcmc, rtt as orc, tfim
    pi, cores = w.pi(), w.cores()
    bits = w.spins(n_walkers)
    bonds = tfim.bonds(w.Lx, w.Ly)
    def steps(n):
        t0 = time.perf_counter()
        s = bits
        for t in range(n):
            s, _, _ = mcmc.metropolis(cores, pi, s, seed=w.chain_seed, stream=0, sweep0=t, n_sweeps=1)
            orc.local_energy(cores, pi, s, bonds, w.J, w.h)
        return time.perf_counter() - t0

    with threadpool_limits(limits=1):
        dt = steps(n_steps)
    ncpu = len(os.sched_getaffinity(0))
    n_all = max(1, n_steps // 3)
    with threadpool_limits(limits=ncpu):
        dt_all = steps(n_all)
    return {"value": n_walkers * n_steps / dt, "unit": "local-energy evals/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_walkers} walkers x {n_steps} steps (sweep + local energies) of the same "
                      f"8x8 chi=64 workload, FP64 numpy, 1 BLAS thread, {dt:.1f} s",
            "host_cpus_available": ncpu,
            "all_cores": {"value": n_walkers * n_all / dt_all, "unit": "local-energy evals/s", "cores": ncpu,
                          "sample": f"{n_walkers} walkers x {n_all} steps, BLAS threads = {ncpu}, "
                                    f"{dt_all:.1f} s"}}


def cpu_baseline_rows(n_dual=48, n_narrow=1024, n_wide=8):
    """The FP64 oracle beside three more GPU lines, on samples of their
    workloads, single-threaded BLAS: a dual Monte Carlo step (one sweep per
    state, then overlap and mixed-energy estimators against all three
    states; 8x8 chi=64), a sweep plus local energies of a chi = 2 train on
    the 10x10 H+V+D+D' path (400 positions, the narrow-kernel shape), and
    local energies of the 10x10 R=3 chi=128 workload (the wide-bond line)."""
    from threadpoolctl import threadpool_limits

    from oracle import dual, mcmc, rtt as orc, tfim
    from paper_2604_22718_amd import lattice
    from paper_2604_22718_amd import workloads as wl
    out = {}
    w = wl.MEDIUM_8x8
    pi = w.pi()
    a, b = w.cores(), wl.gaussian_cores(w.bond(), w.core_seed + 5)
    states = [a, b, ([a, b], np.array([0.8, -1.1]))]
    bonds = tfim.bonds(w.Lx, w.Ly)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for i, st in enumerate(states):
            amp = (lambda S, st=st: dual.state_amplitudes(st, pi, S))
            s, _, _ = mcmc.metropolis(None, pi, w.spins(n_dual), seed=w.chain_seed, stream=100 + i, n_sweeps=1,
                                      amp_fn=amp)
            for st_b in states:
                dual.mixed_estimators(st, st_b, pi, s, bonds, w.J, w.h)
        dt = time.perf_counter() - t0
    out["dual_mc"] = {"value": n_dual * 9 / dt, "unit": "mixed estimators/s", "cores": 1, "kind": "oracle",
                      "sample": f"{n_dual} walkers per state, 3 states: one sweep each and 9 estimator "
                                f"rows, 8x8 chi=64, FP64 numpy, {dt:.1f} s"}
    L = 10
    pi2 = lattice.path(L, L)
    c2 = wl.gaussian_cores(wl.open_bonds(len(pi2), 2), 5)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        s, _, _ = mcmc.metropolis(c2, pi2, wl.random_spins(n_narrow, L * L, 6), seed=3, n_sweeps=1)
        orc.local_energy(c2, pi2, s, tfim.bonds(L, L, periodic=False), 1.0, 3.0)
        dt = time.perf_counter() - t0
    out["narrow_chi2"] = {"value": n_narrow / dt, "unit": "local-energy evals/s (sweep + local energies)",
                          "cores": 1, "kind": "oracle",
                          "sample": f"{n_narrow} walkers x 1 step on the 10x10 open H+V+D+D' chi=2 train, "
                                    f"FP64 numpy, {dt:.1f} s"}
    ww = wl.WORKLOADS["tfim10x10_R3_chi128_W8192"]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orc.local_energy(ww.cores(), ww.pi(), ww.spins(n_wide), tfim.bonds(ww.Lx, ww.Ly), ww.J, ww.h)
        dt = time.perf_counter() - t0
    out["wide_chi128"] = {"value": n_wide / dt, "unit": "local-energy evals/s", "cores": 1, "kind": "oracle",
                          "sample": f"{n_wide} walkers x 1 local-energy evaluation of the 10x10 R=3 chi=128 "
                                    f"workload, FP64 cores, FP64 numpy, {dt:.1f} s"}
    return out


def run(dtype, steps, warmup, with_cpu):
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl

    w = wl.MEDIUM_8x8
    pi, bond, cores = w.pi(), w.bond(), w.cores()
    psi = R.RTT.create(w.N, pi, cores, dtype)
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    bits = w.spins()
    spins = R.spins_to_device(wl.pack_spins(bits))
    W, N, L, chi = w.W, w.N, w.L, w.chi

    # energy error vs FP64 on the seeded configurations (sample of walkers)
    err = eloc_error(w.name, dtype, psi.local_energy(spins, ham).cpu().numpy())

    eloc = torch.empty(W, dtype=torch.float64, device="cuda")
    red = torch.empty(3, dtype=torch.float64, device="cuda")
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    series = []

    def step(t, ev=None):
        if ev: ev[0].record()
        psi.sweep(spins, seed=w.chain_seed, sweep0=t, n_sweeps=1, accepts=acc)
        if ev: ev[1].record()
        R.rtt_evaluate(psi.handle, ham.handle, spins, eloc=eloc)
        if ev: ev[2].record()
        R.rtt_energy_reduce(eloc, red)
        if ev: ev[3].record()
        series.append(red.clone())

    for t in range(warmup):
        step(t)
    torch.cuda.synchronize()
    series.clear()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        step(warmup + t, evs[t])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweep_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    eval_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    red_ms = np.array([e[2].elapsed_time(e[3]) for e in evs])

    sums = torch.stack(series).cpu().numpy()          # (steps, 3)
    means = sums[:, 0] / sums[:, 2]
    var = float(np.mean(sums[:, 1] / sums[:, 2] - means ** 2))
    tau = stats_tau(means)
    energy = float(np.mean(means))
    ess = W * steps / tau

    info = R.rtt_info(psi.handle)
    fwd, bwd = schedule_rowsteps(pi, N, L, info["cut"])
    flops_row = 2.0 * chi * chi
    le_flops = W * (fwd + bwd) * flops_row
    sw_flops = W * sweep_rowsteps(pi, N, L) * flops_row
    kernels = {
        "chain_kernel (1 sweep)": {"ms": float(sweep_ms.mean()), "algorithmic_flops": sw_flops,
                                   "tflops": sw_flops / (sweep_ms.mean() * 1e-3) / 1e12},
        "pass_kernel x2 + combine (local energies)": {"ms": float(eval_ms.mean()),
                                                      "algorithmic_flops": le_flops,
                                                      "tflops": le_flops / (eval_ms.mean() * 1e-3) / 1e12},
        "reduce_kernel": {"ms": float(red_ms.mean())},
    }
    dom = "chain_kernel" if sweep_ms.mean() >= eval_ms.mean() else "evaluate"
    if dom == "chain_kernel":
        ach, nm = sw_flops / (sweep_ms.mean() * 1e-3), "chain_kernel"
    else:
        ach, nm = le_flops / (eval_ms.mean() * 1e-3), "pass_kernel+combine"
    roof = {"kernel": nm, "bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[dtype] / 1e12,
            "unit": "TFLOP/s", "frac": ach / PEAK[dtype],
            "traffic": traffic_from_profile(nm, w.name)}
    res = {
        "metric": METRIC, "value": W * steps / dt, "unit": "local-energy evals/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": f"{w.Lx}x{w.Ly} periodic TFIM", "J": w.J, "h": w.h,
                   "R": w.R, "L": L, "chi": chi, "walkers": W,
                   "step": "1 Metropolis sweep + local energies of all walkers + FP64 reduction"},
        "effective_samples_per_s": ess / dt, "tau_int_steps": tau,
        "energy_per_site": energy / N, "var_eloc": var,
        "acceptance": float(acc.sum().item()) / (W * N * (steps + warmup)),
        "energy_error": err,
        "kernels": kernels,
        "roofline": roof,
    }
    psi.close()
    ham.close()
    return res


def run_batched(steps, n_rtt=256):
    """256 uneven RTTs (side 4..10, R 2..3, chi 16..128, 256..4096 walkers,
    BF16) stepped together: each step = 1 sweep + local energies of every
    walker of every RTT, one captured graph of persistent kernels whose
    launch shape the autotuner picks."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    t0 = time.perf_counter()
    ws = wl.batched_workloads(n_rtt)
    rtts, hams, spins = [], [], []
    flops_le = flops_sw = 0.0
    for w in ws:
        pi = w.pi()
        rtts.append(R.RTT.create(w.N, pi, w.cores(), "bf16"))
        hams.append(R.TFIM(w.Lx, w.Ly, w.J, w.h))
        spins.append(R.spins_to_device(wl.pack_spins(w.spins())))
        info = R.rtt_info(rtts[-1].handle)
        f, b = schedule_rowsteps(pi, w.N, w.L, info["cut"])
        flops_le += w.W * (f + b) * 2.0 * w.chi * w.chi
        flops_sw += w.W * sweep_rowsteps(pi, w.N, w.L) * 2.0 * w.chi * w.chi
    batch = R.Batch(rtts, hams, spins, seed=3100)
    setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    choice = batch.autotune(n_sweeps=1, reps=1, cache_path=os.environ.get("RTT_TUNE_CACHE"))
    tune = time.perf_counter() - t1
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
    res = {"workload": f"{n_rtt} uneven RTTs (side 4-10, R 2-3, chi 16-128, 256-4096 walkers), bf16",
           "walkers": walkers, "steps": steps, "ms_per_step": ms,
           "local_energy_evals_per_s": walkers / (ms * 1e-3),
           "algorithmic_tflops": (flops_le + flops_sw) / (ms * 1e-3) / 1e12,
           "frac_of_bf16_peak": (flops_le + flops_sw) / (ms * 1e-3) / PEAK["bf16"],
           "autotuned_shape": {"concurrent_classes": choice[0], "blocks_per_cu": choice[1]},
           "setup_s": setup, "autotune_s": tune}
    batch.close()
    return res


def run_learned(n_meas=30, train_steps=150, learned_per_sweep=4):
    """10x10, R=3, chi=128, 8192 walkers, BF16: effective samples/s of
    single-flip sweeps alone vs single-flip sweeps + learned multi-spin moves
    (network trained online on the chain, then frozen), same GPU."""
    import torch

    from paper_2604_22718_amd import rtt as R
    from paper_2604_22718_amd import workloads as wl
    w = wl.LARGE_10x10
    psi = R.RTT.create(w.N, w.pi(), w.cores(), "bf16")
    ham = R.TFIM(w.Lx, w.Ly, w.J, w.h)
    net = R.Net(w.Lx, w.Ly, wl.net_init_params(4004))
    out = {"workload": w.name, "walkers": w.W}
    spins0 = R.spins_to_device(wl.pack_spins(w.spins()))
    # burn-in and online training
    ch = R.LearnedChain(psi, net, spins0.clone(), seed=w.chain_seed)
    t0 = time.perf_counter()
    ch.sweep(5)
    for it in range(train_steps):
        ch.learned_step()
        ch.train(lr=2e-3)
        if it % 10 == 9:
            ch.sweep(1)
    torch.cuda.synchronize()
    out["train_s"] = time.perf_counter() - t0
    out["train_steps"] = train_steps

    def measure(learned):
        c = R.LearnedChain(psi, net, ch.spins.clone(), seed=w.chain_seed + 17, rng_stream=1 + int(learned))
        c.sweep(2)
        torch.cuda.synchronize()
        series = []
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(n_meas):
            c.sweep(1)
            if learned:
                for _ in range(learned_per_sweep):
                    c.learned_step()
            series.append(psi.local_energy(c.spins, ham).mean())
        ev1.record()
        torch.cuda.synchronize()
        secs = ev0.elapsed_time(ev1) * 1e-3
        e = torch.stack(series).cpu().numpy()
        tau = stats_tau(e)
        res = {"seconds": secs, "tau_int_measurements": tau, "energy_per_site": float(e.mean()) / w.N,
               "effective_samples_per_s": w.W * n_meas / tau / secs,
               "single_flip_acceptance": c.acc_flip.sum().item() / (w.W * w.N * (n_meas + 2))}
        if learned:
            res["learned_acceptance"] = c.acc_learn.sum().item() / (w.W * learned_per_sweep * n_meas)
        return res

    out["single_flip"] = measure(False)
    out["single_flip_plus_learned"] = measure(True)
    out["learned_moves_per_sweep"] = learned_per_sweep
    out["ess_gain"] = (out["single_flip_plus_learned"]["effective_samples_per_s"]
                       / out["single_flip"]["effective_samples_per_s"])
    return out


def stats_tau(x):
    """Integrated autocorrelation time of a 1-D series (Sokal window, c = 5)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 4:
        return 1.0
    d = x - x.mean()
    c0 = np.mean(d * d)
    if c0 == 0:
        return 1.0
    tau = 1.0
    for M in range(1, n):
        tau += 2.0 * np.mean(d[: n - M] * d[M:]) / c0
        if M >= 5 * tau:
            break
    return max(tau, 1.0)


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
    err = eloc_error(w.name, dtype, eloc.cpu().numpy())
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
        sw_flops = w.W * T * sweep_rowsteps(pi, w.N, w.L) * 2.0 * w.chi * w.chi
        out.update({"sweep_ms": sw_ms, "sweep_algorithmic_tflops": sw_flops / (sw_ms * 1e-3) / 1e12,
                    "sweep_frac_bf16_peak": sw_flops / (sw_ms * 1e-3) / PEAK["bf16"]})
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
    sums = torch.zeros((M, 2, M), dtype=torch.float64, device="cuda")

    def step(t):
        for i, (spins, la, sg) in enumerate(chains):
            states[i].sweep(spins, seed=w.chain_seed, rng_stream=100 + i, sweep0=t, n_sweeps=1, logabs=la, sign=sg)
            ratio, mixed, _ = R.mixed_estimators(states, ham, spins, la, sg)
            sums[i, 0] += ratio.mean(dim=1)
            sums[i, 1] += mixed.mean(dim=1)

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
    S = (sums[:, 0] / (steps + warmup)).cpu().numpy()
    H = (sums[:, 1] / (steps + warmup)).cpu().numpy()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "fp8"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--also", default="bf16", help="second precision reported alongside ('' for none)")
    ap.add_argument("--batched", type=int, default=0, help="also time the 256-RTT batch for this many steps")
    ap.add_argument("--learned", action="store_true", help="also compare learned-proposal ESS/s (10x10, chi=128)")
    ap.add_argument("--no-wide", action="store_true", help="skip the 10x10 chi=128 BF16 wide-bond line")
    ap.add_argument("--huge", action="store_true", help="also time the 16x16 chi=256 4-term FP8 workload (slow)")
    ap.add_argument("--no-dual", action="store_true", help="skip the dual Monte Carlo line")
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
    res = run(a.dtype, a.steps, a.warmup, not a.no_cpu)
    if a.also and a.also != a.dtype:
        other = run(a.also, a.steps, a.warmup, False)
        res["also"] = {k: other[k] for k in ("dtype", "value", "ms_per_step", "effective_samples_per_s",
                                             "energy_error", "kernels", "roofline")}
    if not a.no_wide:
        res["wide_bond"] = [run_wide("tfim10x10_R3_chi128_W8192")]
        if a.huge:
            res["wide_bond"].append(run_wide("tfim16x16_R2_chi256_W16384_T4", n_eval=1))
    if not a.no_dual:
        res["dual_mc"] = run_dual()
    if a.paper_pipeline:
        res["paper_pipeline"] = run_paper_pipeline(L=a.paper_side, steps=a.paper_pipeline, table=a.paper_table)
    if a.batched:
        res["batched"] = run_batched(a.batched)
    if a.learned:
        res["learned"] = run_learned()
    if not a.no_cpu:
        from paper_2604_22718_amd import workloads as wl
        res["cpu_baseline"] = cpu_baseline(wl.MEDIUM_8x8, 64, 12)
        res["cpu_baseline"]["rows"] = cpu_baseline_rows()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
