"""Write sampled_refs.json: configurations the oracle's own Metropolis chain
visits on the benchmark workloads, and FP64 reference values on them.
Test infrastructure: only ``oracle/`` computes, ``workloads`` supplies the
seeded inputs.

For every case a set of walker indices starts from the workload's seeded
spins (the rows the GPU chain starts from) and runs the oracle's Metropolis
chain (Philox key (seed, 0), counter (walker index, sweep, spin, 0)) on the
cores exactly as the device holds them (quantised to the precision):

  * ``burn`` sweeps; the configurations reached are ``sampled``;
  * on them: every flip ratio (FP64), its condition number
    max(kappa(s), kappa(s^j)), E_loc on the quantised cores and on the
    unquantised FP64 cores;
  * ``decide`` more sweeps with the decision margins u - r^2 recorded: the
    configurations after them are ``after``, the smallest |margin| of each
    walker is ``min_margin`` (a GPU chain from ``sampled`` with the same
    Philox words must reach ``after`` wherever its ratios' errors stay below
    that margin);
  * ``meas`` further sweeps with E_loc measured after each (the FP64 chain
    energies of these walkers; the series is ``eloc_series``).

The cases are independent and run in parallel processes (one BLAS thread
each).  Run from the repository root:
    python tests/golden/make_sampled_refs.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# name, dtype, walker indices, burn-in sweeps, decision sweeps, measured sweeps
CASES = [
    ("tfim8x8_R2_chi64_W4096", "f32", [0, 1, 255, 256, 1023, 1024, 1500, 2047, 2048, 2500, 3000, 3001,
                                       3500, 4000, 4094, 4095], 50, 1, 200),
    ("tfim8x8_R2_chi64_W4096", "bf16", [0, 1, 255, 256, 1023, 1024, 1500, 2047, 2048, 2500, 3000, 3001,
                                        3500, 4000, 4094, 4095], 50, 1, 200),
    ("tfim10x10_R3_chi128_W8192", "bf16", [0, 31, 32, 4095, 4096, 8160, 8191, 6000], 20, 1, 0),
    ("tfim16x16_R2_chi256_W16384_T4", "fp8", [0], 3, 1, 0),
    ("tfim16x16_R2_chi256_W16384_T4", "fp8", [5461], 3, 1, 0),
    ("tfim16x16_R2_chi256_W16384_T4", "fp8", [10922], 3, 1, 0),
    ("tfim16x16_R2_chi256_W16384_T4", "fp8", [16383], 3, 1, 0),
]


def words(bits):
    from paper_2604_22718_amd import workloads as wl
    return [[format(int(x), "016x") for x in row] for row in wl.pack_spins(bits)]


def run_case(case):
    from threadpoolctl import threadpool_limits

    from oracle import mcmc, quant, rtt as orc, tfim
    from paper_2604_22718_amd import workloads as wl
    name, dtype, ids, burn, decide, meas = case
    t0 = time.time()
    w = wl.WORKLOADS[name]
    pi, bonds = w.pi(), tfim.bonds(w.Lx, w.Ly)
    ids = np.asarray(ids)
    start = w.spins()[ids]
    with threadpool_limits(limits=1):
        if w.n_terms == 1:
            qc = quant.quantise_cores(w.cores(), dtype)
            uc = w.cores()
            amp = lambda S: orc.amplitudes(qc, pi, S)
            ratios = lambda S: orc.flip_ratios(qc, pi, S)
            kappa = lambda S: orc.flip_condition_numbers(qc, pi, S)
            eloc_q = lambda S: orc.local_energy(qc, pi, S, bonds, w.J, w.h)
            eloc_u = lambda S: orc.local_energy(uc, pi, S, bonds, w.J, w.h)
        else:
            c = w.coeffs()
            qts = [quant.quantise_cores(w.cores(t), dtype) for t in range(w.n_terms)]
            uts = [w.cores(t) for t in range(w.n_terms)]
            amp = lambda S: orc.lincomb_amplitudes(qts, c, pi, S)
            ratios = lambda S: orc.lincomb_flip_ratios(qts, c, pi, S)
            kappa = lambda S: orc.lincomb_flip_condition_numbers(qts, c, pi, S)
            eloc_q = lambda S: orc.lincomb_local_energy(qts, c, pi, S, bonds, w.J, w.h)
            eloc_u = lambda S: orc.lincomb_local_energy(uts, c, pi, S, bonds, w.J, w.h)
        seed = w.chain_seed
        s, _, _ = mcmc.metropolis(None, pi, start, seed, 0, 0, burn, walker_ids=ids, amp_fn=amp)
        r = ratios(s)
        kap = kappa(s)
        diag = orc.diagonal_energy(s, bonds, w.J)
        el_q = diag - w.h * r.sum(axis=1)
        el_u = eloc_u(s)
        after, _, margins = mcmc.metropolis(None, pi, s, seed, 0, burn, decide, walker_ids=ids,
                                            record=True, amp_fn=amp)
        series = []
        cur = after
        for t in range(meas):
            cur, _, _ = mcmc.metropolis(None, pi, cur, seed, 0, burn + decide + t, 1, walker_ids=ids,
                                        amp_fn=amp)
            series.append(eloc_q(cur).tolist())
    out = {"workload": name, "dtype": dtype, "walkers": ids.tolist(), "seed": int(seed), "stream": 0,
           "burn": burn, "decide": decide, "meas": meas,
           "start": words(start), "sampled": words(s), "after": words(after),
           "min_margin": np.min(np.abs(margins), axis=(0, 1)).tolist(),
           "flip_ratios": r.tolist(), "flip_kappa": kap.tolist(),
           "eloc_quantised_cores": el_q.tolist(), "eloc_fp64_cores": el_u.tolist(),
           "eloc_series": series, "final": words(cur), "seconds": time.time() - t0}
    print(f"{name} {dtype} {ids.tolist()} done in {time.time() - t0:.0f} s", flush=True)
    return out


def merge(cases):
    """Cases of one (workload, dtype) computed walker by walker, merged."""
    out = []
    for c in cases:
        prev = next((o for o in out if o["workload"] == c["workload"] and o["dtype"] == c["dtype"]), None)
        if prev is None:
            out.append(c)
            continue
        for k in ("walkers", "start", "sampled", "after", "min_margin", "flip_ratios", "flip_kappa",
                  "eloc_quantised_cores", "eloc_fp64_cores", "final"):
            prev[k] = prev[k] + c[k]
        prev["seconds"] = max(prev["seconds"], c["seconds"])
    return out


def main():
    with ProcessPoolExecutor(max_workers=min(len(CASES), os.cpu_count() or 1)) as ex:
        res = list(ex.map(run_case, CASES))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sampled_refs.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_sampled_refs.py", "cases": merge(res)}, f)


if __name__ == "__main__":
    main()
