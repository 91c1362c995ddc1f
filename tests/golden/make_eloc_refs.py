"""Write eloc_fp64_refs.json: FP64 local energies of seeded benchmark
walkers, computed by the oracle only (test infrastructure).

For each workload and precision, the walkers' initial configurations are the
workload's seeded spins; energies are given on the cores exactly as the
device holds them (quantised to the precision) and on the unquantised FP64
cores.  The benchmark compares its GPU energies against these numbers.

Run from the repository root:  python tests/golden/make_eloc_refs.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import quant, rtt as orc, tfim  # noqa: E402
from paper_2604_22718_amd import workloads as wl  # noqa: E402

CASES = [
    ("tfim8x8_R2_chi64_W4096", "f32", [0, 1, 2, 3, 1000, 2000, 3000, 4095]),
    ("tfim8x8_R2_chi64_W4096", "bf16", [0, 1, 2, 3, 1000, 2000, 3000, 4095]),
    ("tfim10x10_R3_chi128_W8192", "bf16", [0, 1, 2, 3]),
    ("tfim16x16_R2_chi256_W16384_T4", "fp8", [0]),
]


def energies(w, cores_of_term, idx):
    bits = w.spins()[idx]
    bonds = tfim.bonds(w.Lx, w.Ly)
    pi = w.pi()
    if w.n_terms == 1:
        return orc.local_energy(cores_of_term(0), pi, bits, bonds, w.J, w.h)
    terms = [cores_of_term(t) for t in range(w.n_terms)]
    return orc.lincomb_local_energy(terms, w.coeffs(), pi, bits, bonds, w.J, w.h)


def main():
    out = []
    for name, dtype, idx in CASES:
        w = wl.WORKLOADS[name]
        q = energies(w, lambda t: quant.quantise_cores(w.cores(t), dtype), idx)
        u = energies(w, lambda t: w.cores(t), idx)
        out.append({"workload": name, "dtype": dtype, "walkers": idx,
                    "eloc_quantised_cores": [float(x) for x in q],
                    "eloc_fp64_cores": [float(x) for x in u]})
        print(name, dtype, np.round(q, 6), flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "eloc_fp64_refs.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_eloc_refs.py", "cases": out}, f, indent=1)


if __name__ == "__main__":
    main()
