"""The stored FP64 energy references that the benchmark compares against
were written by tests/golden/make_eloc_refs.py from the oracle alone; spot
check two of them against a fresh oracle evaluation."""
import json
import os

import numpy as np

from oracle import quant, rtt as orc, tfim
from paper_2604_22718_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def test_stored_energies_reproduce():
    refs = json.load(open(os.path.join(HERE, "golden", "eloc_fp64_refs.json")))
    case = next(c for c in refs["cases"] if c["workload"] == "tfim8x8_R2_chi64_W4096" and c["dtype"] == "f32")
    w = wl.WORKLOADS[case["workload"]]
    idx = case["walkers"][:2]
    bits = w.spins()[idx]
    bonds = tfim.bonds(w.Lx, w.Ly)
    q = orc.local_energy(quant.quantise_cores(w.cores(), "f32"), w.pi(), bits, bonds, w.J, w.h)
    u = orc.local_energy(w.cores(), w.pi(), bits, bonds, w.J, w.h)
    assert np.allclose(q, case["eloc_quantised_cores"][:2], rtol=1e-12, atol=0)
    assert np.allclose(u, case["eloc_fp64_cores"][:2], rtol=1e-12, atol=0)
    names = {(c["workload"], c["dtype"]) for c in refs["cases"]}
    assert ("tfim10x10_R3_chi128_W8192", "bf16") in names
