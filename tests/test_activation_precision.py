"""Why BF16 and FP8 cores take their activations as a hi + lo BF16 pair.

A contraction in which every activation row is renormalised by a power of
two and rounded once per core product to FP16 (one matrix op per product,
twice the rate of hi + lo) is emulated in numpy on configurations the
oracle's own chain samples on the 10x10, R = 3, bond-128 BF16 workload
(tests/golden/sampled_refs.json).  Its log-amplitude and log-ratio errors
against FP64 on the same quantised cores reach the 2e-2 bound the parity
tests hold BF16 ratios to, while the hi + lo rounding the kernels use stays
two orders of magnitude below it.  CPU only; no kernel is run."""
import numpy as np

from helpers import sampled_refs
from oracle import quant
from paper_2604_22718_amd import workloads as wl

NAME = "tfim10x10_R3_chi128_W8192"


def _bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def hilo(x):
    h = _bf16(x)
    return h + _bf16(x - h)


def fp16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def exact(x):
    return x


def log_amplitude(cores, pi, s, rnd):
    """log|psi(s)| with the activation row rounded by rnd before every
    product (after a power-of-two renormalisation, as the kernels do)."""
    v, lg = np.ones(1), 0.0
    for k, c in enumerate(cores):
        e = np.frexp(np.max(np.abs(v)))[1]
        v, lg = v * 2.0 ** -e, lg + e * np.log(2.0)
        v = rnd(v) @ c[s[pi[k]]]
    return lg + np.log(abs(v[0]))


def test_fp16_activations_miss_the_bf16_bound_hilo_meets_it():
    w = wl.WORKLOADS[NAME]
    pi = w.pi()
    cores = quant.quantise_cores(w.cores(), "bf16")
    # the kernels hold each core divided by a power of two (largest entry in [0.5, 1))
    cores = [c * 2.0 ** -np.frexp(np.max(np.abs(c)))[1] for c in cores]
    S = wl.unpack_spins(sampled_refs(NAME, "bf16")["sampled"], w.N)[:2]
    err = {"hilo": [], "fp16": []}
    for s in S:
        base = {r: log_amplitude(cores, pi, s, f) for r, f in (("exact", exact), ("hilo", hilo), ("fp16", fp16))}
        for j in (7, 55):
            sj = s.copy()
            sj[j] ^= 1
            for r, f in (("hilo", hilo), ("fp16", fp16)):
                d = (log_amplitude(cores, pi, sj, f) - base[r]) - (log_amplitude(cores, pi, sj, exact) - base["exact"])
                err[r].append(abs(d))
    print({r: float(np.max(v)) for r, v in err.items()})
    assert np.max(err["hilo"]) < 2e-3
    assert np.max(err["fp16"]) > 1e-2
