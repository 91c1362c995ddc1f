"""Dual Monte Carlo matrix elements (paper Sec. 3.3, "Dual Monte Carlo" and
the generalised eigenproblem of the physical-space optimisation).  Test
infrastructure only.

A state is an RTT (list of cores) or a linear combination ``(terms, coeffs)``
of RTTs sharing one path (Sec. 3.2).  For a sampled state a and a target
state b, with P^a(s) = |psi^a(s)|^2 / Z_a and Z_a = sum_s |psi^a(s)|^2:

  overlap estimator    o_ab(s) = psi^b(s) / psi^a(s),          S~_ab = <o_ab>_{P^a}
  mixed local energy   e_ab(s) = sum_t H_{s,t} psi^b(t) / psi^a(s),  H~_ab = <e_ab>_{P^a}

For the TFIM, H_{s,s} = J sum_<ij> z_i z_j and H_{s,s^j} = -h (s^j: s with
s_j flipped, every replica position of j switching slice).  The paper's
un-symmetrised matrices satisfy Z_a H~_ab = psi^a . H psi^b = Z_b H~_ba and
Z_a S~_ab = psi^a . psi^b; the generalised problem H~ c = lambda S~ c has
the eigenvalues of the symmetric one H c = lambda S c.  Stochastic
Gram-Schmidt replaces psi^m by psi^m - sum_{a<m} S~_am psi^a.
"""
from __future__ import annotations

import numpy as np

from .rtt import all_configs, amplitudes, diagonal_energy, flip, lincomb_amplitudes
from .tfim import sparse_hamiltonian


def state_amplitudes(state, pi, spins) -> np.ndarray:
    """Amplitudes of an RTT (list of cores) or of a (terms, coeffs) combination."""
    if isinstance(state, tuple):
        terms, coeffs = state
        return lincomb_amplitudes(terms, coeffs, pi, spins)
    return amplitudes(state, pi, spins)


def mixed_estimators(state_a, state_b, pi, spins, bonds, J: float, h: float):
    """Per configuration: o_ab(s) and e_ab(s), each amplitude recomputed in
    full (no environments), H applied term by term."""
    spins = np.asarray(spins)
    N = spins.shape[1]
    pa = state_amplitudes(state_a, pi, spins)
    pb = state_amplitudes(state_b, pi, spins)
    off = np.zeros(spins.shape[0])
    for j in range(N):
        off += state_amplitudes(state_b, pi, flip(spins, j))
    hpsi_b = diagonal_energy(spins, bonds, J) * pb - h * off
    return pb / pa, hpsi_b / pa


def exact_matrices(states, pi, Lx: int, Ly: int, J: float, h: float, periodic=True):
    """H~ and S~ of a list of states by enumeration of all 2^N configurations
    with the sparse Hamiltonian (another route than mixed_estimators), plus
    the norms Z_a."""
    N = Lx * Ly
    S = all_configs(N)
    psi = [state_amplitudes(st, pi, S) for st in states]
    H = sparse_hamiltonian(Lx, Ly, J, h, periodic)
    M = len(states)
    Z = np.array([p @ p for p in psi])
    Ht = np.empty((M, M))
    St = np.empty((M, M))
    for a in range(M):
        for b in range(M):
            Ht[a, b] = psi[a] @ (H @ psi[b]) / Z[a]
            St[a, b] = psi[a] @ psi[b] / Z[a]
    return Ht, St, Z


def lowest_generalised_eigenvalue(Ht, St) -> float:
    """Smallest real eigenvalue of H~ c = lambda S~ c (generalised
    eigenproblem of the un-symmetrised matrices), by a library routine."""
    import scipy.linalg
    w = scipy.linalg.eig(np.asarray(Ht), np.asarray(St), right=False)
    w = w[np.isfinite(w)]
    return float(np.min(w.real))


def gram_schmidt_coefficients(St) -> np.ndarray:
    """Coefficients of the stochastic Gram-Schmidt states in the original
    basis: psi'^m = psi^m - sum_{a<m} S~_am psi^a (rows: m, columns: a)."""
    St = np.asarray(St)
    M = St.shape[0]
    C = np.eye(M)
    for m in range(1, M):
        for a in range(m):
            C[m, a] = -St[a, m]
    return C


def apply_z(cores, pi, i: int):
    """The RTT of Z_i psi: Z on a spin acts on one of its replicas (Sec. 2.2.3
    commutation rules), here the first position k of spin i, whose slice 1
    changes sign, since Z|s> = (-1)^s |s>."""
    k = int(np.flatnonzero(np.asarray(pi) == i)[0])
    out = [np.array(c, copy=True) for c in cores]
    out[k][1] = -out[k][1]
    return out


def z_only_matrices(ratio_rows, mixed_rows):
    """Z-only shortcut: when every state is psi^a = d_a psi with d_a(s) = +-1
    (diagonal operators made of Z's), all P^a equal P = |psi|^2/Z and one
    chain on psi gives every element.  Inputs are per-walker arrays over
    walkers sampled from P: ratio_rows[b] = psi^b/psi and mixed_rows[b] =
    sum_t H_st psi^b(t)/psi(s).  Returns per-walker H~ and S~ estimators of
    shape (M, M, W): S~_ab = psi^b/psi^a = r_b / r_a and
    H~_ab = mixed_b / r_a (r_a = +-1)."""
    r = np.asarray(ratio_rows)
    e = np.asarray(mixed_rows)
    return e[None, :, :] / r[:, None, :], r[None, :, :] / r[:, None, :]
