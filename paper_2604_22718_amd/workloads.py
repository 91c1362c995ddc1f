"""Seeded synthetic inputs for replica-tensor-train (RTT) workloads.

This module only draws random numbers and lays data out; it holds none of the
method's arithmetic.  It is the one module shared by the GPU path and by the
CPU reference used in tests, so both consume bit-identical inputs.

Conventions (paper, Sec. 2.1 and Sec. 2.2.1):
  * N physical spins, a train of L cores, and a path ``pi[k]`` (0-based) that
    names the spin read by train position k.
  * ``bond[k]`` is the bond dimension to the left of core k; open boundary
    bonds ``bond[0] = bond[L] = 1``.
  * core k is an array of shape ``(2, bond[k], bond[k+1])``; slice ``[s]`` is
    the matrix used when the spin read at position k has value s.
  * spins: bool/uint8 arrays ``(W, N)``; the packed device form is
    ``uint64 (W, ceil(N/64))`` with bit ``j % 64`` of word ``j // 64`` = s_j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def generator(seed: int) -> np.random.Generator:
    """numpy Generator on the Philox bit generator, keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(int(seed)))


# --------------------------------------------------------------------------
# paths
# --------------------------------------------------------------------------
def path_repeat(N: int, R: int) -> np.ndarray:
    """Site order repeated R times (the path sum of R identical orderings)."""
    return np.tile(np.arange(N, dtype=np.int32), R)


def path_site_plus_perms(N: int, R: int, seed: int) -> np.ndarray:
    """Site order followed by R-1 seeded random orderings (path sum)."""
    g = generator(seed)
    parts = [np.arange(N, dtype=np.int32)]
    for _ in range(R - 1):
        parts.append(g.permutation(N).astype(np.int32))
    return np.concatenate(parts)


def path_hv_2x3() -> np.ndarray:
    """The 6-spin horizontal+vertical path of Sec. 2.2.1 (0-based)."""
    one_based = [1, 2, 3, 4, 5, 6, 4, 3, 2, 5, 6, 1]
    return np.asarray(one_based, dtype=np.int32) - 1


# --------------------------------------------------------------------------
# cores
# --------------------------------------------------------------------------
def open_bonds(L: int, chi: int) -> np.ndarray:
    b = np.full(L + 1, chi, dtype=np.int32)
    b[0] = 1
    b[L] = 1
    return b


def gaussian_cores(bond, seed: int, std: float | None = None) -> list[np.ndarray]:
    """Cores with i.i.d. N(0, std^2) entries; std defaults to 1/sqrt(max bond)."""
    bond = np.asarray(bond)
    L = len(bond) - 1
    chi = int(bond.max())
    if std is None:
        std = 1.0 / math.sqrt(chi)
    g = generator(seed)
    return [g.standard_normal((2, int(bond[k]), int(bond[k + 1]))) * std
            for k in range(L)]


def flatten_cores(cores) -> np.ndarray:
    """Concatenate cores, each row-major (2, bond[k], bond[k+1]), as float64."""
    return np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel()
                           for c in cores])


def bonds_of(cores) -> np.ndarray:
    b = [cores[0].shape[1]] + [c.shape[2] for c in cores]
    return np.asarray(b, dtype=np.int32)


# --------------------------------------------------------------------------
# spins
# --------------------------------------------------------------------------
def random_spins(W: int, N: int, seed: int) -> np.ndarray:
    g = generator(seed)
    return g.integers(0, 2, size=(W, N), dtype=np.uint8)


def pack_spins(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint64)
    W, N = bits.shape
    nw = (N + 63) // 64
    out = np.zeros((W, nw), dtype=np.uint64)
    for j in range(N):
        out[:, j // 64] |= bits[:, j] << np.uint64(j % 64)
    return out


def unpack_spins(words: np.ndarray, N: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    W = words.shape[0]
    out = np.zeros((W, N), dtype=np.uint8)
    for j in range(N):
        out[:, j] = ((words[:, j // 64] >> np.uint64(j % 64)) & np.uint64(1)).astype(np.uint8)
    return out


# --------------------------------------------------------------------------
# learned-proposal network: seeded initial weights
# --------------------------------------------------------------------------
# Parameter blocks in storage order: three 3x3 convolutions with 32 channels
# (weights [out][in][3][3], then biases) and a 1x1 head with 9 outputs per
# site.  Only the shapes are needed here, to draw the initial weights.
NET_BLOCKS = [(32, 1, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (9, 32), (9,)]


def net_init_params(seed: int) -> np.ndarray:
    """Flat initial network weights: uniform in +-sqrt(3 / fan_in) for the
    weight blocks (fan_in = product of all but the first dimension), zero
    biases, drawn from Philox(seed) block by block."""
    g = generator(seed)
    parts = []
    for shp in NET_BLOCKS:
        if len(shp) > 1:
            lim = math.sqrt(3.0 / int(np.prod(shp[1:])))
            parts.append(g.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# workload configurations (synthetic stand-ins for the paper's 2D TFIM runs)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    Lx: int
    Ly: int
    R: int
    chi: int
    W: int
    h: float
    J: float = 1.0
    periodic: bool = True
    path: str = "site+perm"          # or "repeat"
    dtype: str = "f32"
    core_seed: int = 0
    chain_seed: int = 0
    perm_seed: int = 0
    n_terms: int = 1
    coeff_seed: int = 0
    burn_in: int = 0
    sweeps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.Lx * self.Ly

    @property
    def L(self) -> int:
        return self.R * self.N

    def pi(self) -> np.ndarray:
        if self.path == "repeat":
            return path_repeat(self.N, self.R)
        return path_site_plus_perms(self.N, self.R, self.perm_seed)

    def bond(self) -> np.ndarray:
        return open_bonds(self.L, self.chi)

    def cores(self, term: int = 0) -> list[np.ndarray]:
        return gaussian_cores(self.bond(), self.core_seed + 7919 * term)

    def coeffs(self) -> np.ndarray:
        if self.n_terms == 1:
            return np.ones(1)
        return generator(self.coeff_seed).standard_normal(self.n_terms)

    def spins(self, W: int | None = None) -> np.ndarray:
        return random_spins(self.W if W is None else W, self.N, self.chain_seed)


# 4x4, R=2 (site order twice), chi=8, 64 walkers: the small exact-enumeration case.
SMALL_4x4 = Workload("tfim4x4_R2_chi8_W64", 4, 4, 2, 8, 64, 3.04, path="repeat",
                     dtype="f32", core_seed=1001, chain_seed=2001, burn_in=20, sweeps=200)
# 8x8, R=2 (site order + seeded permutation), chi=64, 4096 walkers.
MEDIUM_8x8 = Workload("tfim8x8_R2_chi64_W4096", 8, 8, 2, 64, 4096, 3.04,
                      dtype="f32", core_seed=1002, chain_seed=2002, perm_seed=3002,
                      burn_in=50, sweeps=200)
# 10x10, R=3, chi=128, 8192 walkers, BF16 cores.
LARGE_10x10 = Workload("tfim10x10_R3_chi128_W8192", 10, 10, 3, 128, 8192, 3.04,
                       dtype="bf16", core_seed=1004, chain_seed=2004, perm_seed=3004,
                       burn_in=100, sweeps=400)
# 16x16, R=2, chi=256, 16384 walkers, 4-term linear combination, FP8 cores.
HUGE_16x16 = Workload("tfim16x16_R2_chi256_W16384_T4", 16, 16, 2, 256, 16384, 3.04,
                      dtype="fp8", core_seed=1005, chain_seed=2005, perm_seed=3005,
                      n_terms=4, coeff_seed=4005, burn_in=20, sweeps=100)

WORKLOADS = {w.name: w for w in (SMALL_4x4, MEDIUM_8x8, LARGE_10x10, HUGE_16x16)}


def batched_workloads(n_rtt: int = 256, seed: int = 3100):
    """Uneven batch: side U{4..10}, R U{2,3}, chi U{16,32,64,128},
    walkers log-uniform in [256, 4096], h U[2,4]; BF16 cores."""
    out = []
    for b in range(n_rtt):
        g = generator(seed + b)
        side = int(g.integers(4, 11))
        R = int(g.integers(2, 4))
        chi = int([16, 32, 64, 128][g.integers(0, 4)])
        W = int(round(math.exp(g.uniform(math.log(256), math.log(4096)))))
        h = float(g.uniform(2.0, 4.0))
        out.append(Workload(f"batch{b}", side, side, R, chi, W, h, dtype="bf16",
                            core_seed=seed + 10000 + b, chain_seed=seed + 20000 + b,
                            perm_seed=seed + 30000 + b))
    return out
