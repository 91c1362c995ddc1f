"""RTT amplitudes, single-spin-flip ratios and local energies in plain FP64.

Test infrastructure only (see ``oracle/__init__``).

Definitions followed:
  * Tensor train: phi_{i_1..i_Omega} = Tr A_1^{i_1} ... A_Omega^{i_Omega},
    chi_1 = chi_{Omega+1} = 1 (paper Sec. 2.1).
  * RTT amplitude: psi_s = Tr A_1^{s_sigma(1)} ... A_Omega^{s_sigma(Omega)}
    (Sec. 2.2.1); here sigma is the 0-based array ``pi``.
  * Replica sets R_j = sigma^{-1}(j) (Sec. 2.2.1).
  * An X on spin j commutes through the constraint into X on every replica
    of j (Sec. 2.2.3, the X rule and the worked operator example), so the
    flipped amplitude uses slice 1-s_j at every position of R_j.
  * Local energy of H = J sum_<ij> Z_i Z_j - h sum_i X_i (Sec. 4, Ising model
    equation; the local-energy form is the psi^1 = psi^2 case of the mixed
    local energy of Sec. 3.3).  Z|s> = (-1)^s |s>, so z = 1 - 2 s.
  * Linear combination psi = sum_a c_a psi^a (Sec. 3.2, lin_comb equation).
"""
from __future__ import annotations

import math

import numpy as np


def replica_sets(pi, N: int) -> list[list[int]]:
    """R_j = sigma^{-1}(j), the train positions that read spin j (Sec. 2.2.1)."""
    out = [[] for _ in range(N)]
    for k, j in enumerate(np.asarray(pi)):
        out[int(j)].append(k)
    return out


def amplitude(cores, pi, s) -> float:
    """psi(s) for one configuration: direct product of the selected slices."""
    v = np.ones((1, 1))
    for k, A in enumerate(cores):
        v = v @ A[int(s[int(pi[k])])]
    return float(v[0, 0])


def amplitudes(cores, pi, spins) -> np.ndarray:
    """psi(s) for a batch ``spins`` (W, N): the same product, walkers batched
    with numpy matmul position by position."""
    spins = np.asarray(spins)
    W = spins.shape[0]
    v = np.ones((W, 1, 1))
    for k, A in enumerate(cores):
        sel = A[spins[:, int(pi[k])].astype(np.int64)]        # (W, a, b)
        v = np.matmul(v, sel)
    return v[:, 0, 0].copy()


def log_sign(psi):
    psi = np.asarray(psi, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.log(np.abs(psi)), np.sign(psi).astype(np.int8)


def flip(spins, j: int) -> np.ndarray:
    out = np.array(spins, copy=True)
    out[..., j] ^= 1
    return out


def flip_ratios(cores, pi, spins) -> np.ndarray:
    """r_j(s) = psi(s with s_j flipped) / psi(s), for every spin j.

    Each flipped amplitude is recomputed from scratch (no environments), so
    the result depends only on the amplitude definition.  Returns (W, N).
    """
    spins = np.asarray(spins)
    W, N = spins.shape
    base = amplitudes(cores, pi, spins)
    out = np.empty((W, N))
    for j in range(N):
        out[:, j] = amplitudes(cores, pi, flip(spins, j)) / base
    return out


def diagonal_energy(spins, bonds, J: float) -> np.ndarray:
    """J * sum over bonds of z_i z_j with z = 1 - 2 s."""
    spins = np.asarray(spins, dtype=np.int64)
    z = 1 - 2 * spins
    b = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
    if len(b) == 0:
        return np.zeros(spins.shape[0])
    return J * np.sum(z[:, b[:, 0]] * z[:, b[:, 1]], axis=1).astype(np.float64)


def local_energy(cores, pi, spins, bonds, J: float, h: float) -> np.ndarray:
    """E_loc(s) = sum_s' H_{s s'} psi(s') / psi(s).

    The diagonal part gives J sum z_i z_j; each X_j connects s to the
    configuration with s_j flipped with matrix element -h, giving -h r_j.
    """
    r = flip_ratios(cores, pi, spins)
    return diagonal_energy(spins, bonds, J) - h * r.sum(axis=1)


# --------------------------------------------------------------------------
# linear combinations (Sec. 3.2)
# --------------------------------------------------------------------------
def lincomb_amplitudes(terms, coeffs, pi, spins) -> np.ndarray:
    """psi = sum_a c_a psi^a evaluated by summing the per-term amplitudes."""
    tot = np.zeros(np.asarray(spins).shape[0])
    for c, cores in zip(coeffs, terms):
        tot = tot + c * amplitudes(cores, pi, spins)
    return tot


def lincomb_flip_ratios(terms, coeffs, pi, spins, which=None) -> np.ndarray:
    """Ratios of the summed amplitudes; ``which`` restricts to a subset of spins."""
    spins = np.asarray(spins)
    W, N = spins.shape
    js = range(N) if which is None else which
    base = lincomb_amplitudes(terms, coeffs, pi, spins)
    out = np.empty((W, len(js)))
    for col, j in enumerate(js):
        out[:, col] = lincomb_amplitudes(terms, coeffs, pi, flip(spins, j)) / base
    return out


def lincomb_local_energy(terms, coeffs, pi, spins, bonds, J, h) -> np.ndarray:
    r = lincomb_flip_ratios(terms, coeffs, pi, spins)
    return diagonal_energy(spins, bonds, J) - h * r.sum(axis=1)


# --------------------------------------------------------------------------
# exhaustive enumeration (small N)
# --------------------------------------------------------------------------
def all_configs(N: int) -> np.ndarray:
    """All 2^N configurations; row index = sum_j s_j 2^j."""
    idx = np.arange(2 ** N, dtype=np.int64)
    return ((idx[:, None] >> np.arange(N)) & 1).astype(np.uint8)


def exact_energy(cores, pi, N, bonds, J, h) -> float:
    """<psi|H|psi>/<psi|psi> = sum |psi|^2 E_loc / sum |psi|^2 by enumeration."""
    S = all_configs(N)
    psi = amplitudes(cores, pi, S)
    p = psi * psi
    el = local_energy(cores, pi, S, bonds, J, h)
    return math.fsum(p * el) / math.fsum(p)


# --------------------------------------------------------------------------
# conditioning of an amplitude (used to scale floating-point tolerances)
# --------------------------------------------------------------------------
def condition_numbers(cores, pi, spins) -> np.ndarray:
    """kappa(s) = max over bonds c of ||l_c(s)|| ||r_c(s)|| / |psi(s)|, where
    l_c is the product of the first c selected slices (a row vector) and r_c
    the product of the remaining ones (a column vector), so psi = l_c . r_c
    at every c.  kappa >= 1 (Cauchy-Schwarz); it measures the cancellation in
    psi that any floating-point evaluation must resolve."""
    spins = np.asarray(spins)
    W = spins.shape[0]
    L = len(cores)
    left = [np.ones((W, 1))]
    for k in range(L):
        left.append(np.einsum("wa,wab->wb", left[-1], cores[k][spins[:, int(pi[k])].astype(np.int64)]))
    right = [np.ones((W, 1))]
    for k in reversed(range(L)):
        right.append(np.einsum("wab,wb->wa", cores[k][spins[:, int(pi[k])].astype(np.int64)], right[-1]))
    right = right[::-1]
    psi = np.abs(left[-1][:, 0])
    prod = np.stack([np.linalg.norm(left[c], axis=1) * np.linalg.norm(right[c], axis=1)
                     for c in range(L + 1)])
    with np.errstate(divide="ignore"):
        return prod.max(axis=0) / psi


def flip_condition_numbers(cores, pi, spins) -> np.ndarray:
    """max(kappa(s), kappa(s with s_j flipped)) for every spin j, shape (W, N)."""
    spins = np.asarray(spins)
    k0 = condition_numbers(cores, pi, spins)
    return np.stack([np.maximum(k0, condition_numbers(cores, pi, flip(spins, j)))
                     for j in range(spins.shape[1])], axis=1)


def lincomb_condition_numbers(terms, coeffs, pi, spins) -> np.ndarray:
    """kappa(s) of psi = sum_a c_a psi^a evaluated term by term:
    max over bonds c of sum_a |c_a| ||l^a_c(s)|| ||r^a_c(s)|| / |psi(s)|, with
    l^a_c, r^a_c the row and column products of term a split at bond c (as in
    condition_numbers).  Each term's product at bond c carries rounding error
    ~ gamma ||l^a_c|| ||r^a_c||, so this measures the cancellation an
    evaluation that sums the terms' amplitudes must resolve.  It is >= 1
    (triangle and Cauchy-Schwarz inequalities), equals condition_numbers for
    one term with coefficient 1, and is at most the kappa of the direct-sum
    train (Cauchy-Schwarz over the terms)."""
    spins = np.asarray(spins)
    W = spins.shape[0]
    L = len(terms[0])
    num = np.zeros((L + 1, W))
    psi = np.zeros(W)
    for ca, cores in zip(coeffs, terms):
        left = [np.ones((W, 1))]
        for k in range(L):
            left.append(np.einsum("wa,wab->wb", left[-1], cores[k][spins[:, int(pi[k])].astype(np.int64)]))
        right = [np.ones((W, 1))]
        for k in reversed(range(L)):
            right.append(np.einsum("wab,wb->wa", cores[k][spins[:, int(pi[k])].astype(np.int64)], right[-1]))
        right = right[::-1]
        psi = psi + ca * left[-1][:, 0]
        num += abs(ca) * np.stack([np.linalg.norm(left[c], axis=1) * np.linalg.norm(right[c], axis=1)
                                   for c in range(L + 1)])
    with np.errstate(divide="ignore"):
        return num.max(axis=0) / np.abs(psi)


def lincomb_flip_condition_numbers(terms, coeffs, pi, spins) -> np.ndarray:
    """max(kappa(s), kappa(s with s_j flipped)) of a linear combination, (W, N)."""
    spins = np.asarray(spins)
    k0 = lincomb_condition_numbers(terms, coeffs, pi, spins)
    return np.stack([np.maximum(k0, lincomb_condition_numbers(terms, coeffs, pi, flip(spins, j)))
                     for j in range(spins.shape[1])], axis=1)
