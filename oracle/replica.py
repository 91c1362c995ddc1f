"""Replica-space operators, tensor-train algebra and the power method
(paper Sec. 2.2.3, commutation rules of X, Z with the copy tensor, and
Sec. 3.1, optimisation in the replica space).  Test infrastructure only.

A replica-space state phi is a train of L = R N cores; the physical state is
psi = C phi, psi(s) = prod_k A_k[s_pi(k)].
  * X_j C = C prod_{k in R_j} X_k : X acts on every replica of j (slices of
    all those cores swapped);
  * Z_j C = C Z_k for one k in R_j (here the first position of j): slice 1 of
    that core changes sign.
TFIM in replica space: H-bar = J sum_<ij> Zbar_i Zbar_j - h sum_j Xbar_j.
A power step phi' = phi - tau H-bar phi: every term eta_t H-bar_t phi is a
rank-1 operator applied to phi (bond dimensions unchanged); the terms are
summed two by two, each sum compressed to at most chi_max; the result is
multiplied by tau, subtracted from phi and compressed once more.
Compression is tensor-train rounding: right-to-left orthogonalisation by
QR, then left-to-right truncated SVDs keeping at most chi_max singular
values and none below rel_tol times the largest of that bond.
"""
from __future__ import annotations

import numpy as np


def apply_x(cores, pi, j: int):
    out = [np.array(c, copy=True) for c in cores]
    for k in np.flatnonzero(np.asarray(pi) == j):
        out[k] = out[k][::-1].copy()
    return out


def apply_z(cores, pi, i: int):
    out = [np.array(c, copy=True) for c in cores]
    k = int(np.flatnonzero(np.asarray(pi) == i)[0])
    out[k][1] = -out[k][1]
    return out


def scale(cores, c: float):
    out = [np.array(x, copy=True) for x in cores]
    out[0] = out[0] * c
    return out


def add(a, b):
    """The train of phi_a + phi_b: block-diagonal interior cores, the first
    cores side by side, the last ones stacked."""
    L = len(a)
    out = []
    for k in range(L):
        A, B = a[k], b[k]
        if L == 1:
            out.append(A + B)
        elif k == 0:
            out.append(np.concatenate([A, B], axis=2))
        elif k == L - 1:
            out.append(np.concatenate([A, B], axis=1))
        else:
            C = np.zeros((2, A.shape[1] + B.shape[1], A.shape[2] + B.shape[2]))
            C[:, :A.shape[1], :A.shape[2]] = A
            C[:, A.shape[1]:, A.shape[2]:] = B
            out.append(C)
    return out


def round_tt(cores, chi_max: int, rel_tol: float = 1e-14):
    """Tensor-train rounding; returns the cores (2, a, b)."""
    c = [np.array(x, dtype=np.float64, copy=True) for x in cores]
    L = len(c)
    for k in range(L - 1, 0, -1):              # right-to-left: right-orthonormal cores
        a, b = c[k].shape[1], c[k].shape[2]
        M = c[k].transpose(1, 0, 2).reshape(a, 2 * b)
        Q, R = np.linalg.qr(M.T)                 # M = R^T Q^T
        r = Q.shape[1]
        c[k] = Q.T.reshape(r, 2, b).transpose(1, 0, 2)
        c[k - 1] = np.einsum("sxa,ya->sxy", c[k - 1], R)
    for k in range(L - 1):                     # left-to-right: truncated SVD
        a, b = c[k].shape[1], c[k].shape[2]
        M = c[k].transpose(1, 0, 2).reshape(a * 2, b)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        keep = 1 if S[0] == 0 else max(1, min(chi_max, int(np.sum(S > rel_tol * S[0]))))
        c[k] = U[:, :keep].reshape(a, 2, keep).transpose(1, 0, 2)
        c[k + 1] = np.einsum("xy,syb->sxb", S[:keep, None] * Vt[:keep], c[k + 1])
    return c


def hbar_terms(cores, pi, bonds, J: float, h: float):
    """eta_t H-bar_t phi for every Pauli string of the replica-space TFIM:
    bonds first (J Zbar_i Zbar_j), then fields (-h Xbar_j)."""
    N = int(np.max(pi)) + 1
    terms = [scale(apply_z(apply_z(cores, pi, int(i)), pi, int(j)), J) for i, j in np.asarray(bonds).reshape(-1, 2)]
    terms += [scale(apply_x(cores, pi, j), -h) for j in range(N)]
    return terms


def power_step(cores, pi, bonds, J: float, h: float, tau: float, chi_max: int, rel_tol: float = 1e-14):
    terms = hbar_terms(cores, pi, bonds, J, h)
    while len(terms) > 1:
        nxt = []
        for t in range(0, len(terms), 2):
            nxt.append(round_tt(add(terms[t], terms[t + 1]), chi_max, rel_tol) if t + 1 < len(terms) else terms[t])
        terms = nxt
    return round_tt(add(cores, scale(terms[0], -tau)), chi_max, rel_tol)


def apply_string(cores, ops):
    """A Pauli string on the replica indices (Sec. 2.2.3): per position
    0 I, 1 X (phi_i -> phi_{1-i}), 2 Z (phi_i -> (-1)^i phi_i),
    3 X Z (Z first, then X)."""
    out = [np.array(c, copy=True) for c in cores]
    for k, o in enumerate(np.asarray(ops)):
        if o & 2:
            out[k][1] = -out[k][1]
        if o & 1:
            out[k] = out[k][::-1].copy()
    return out


def pairwise_sum(terms, chi_max, rel_tol=1e-14):
    """Trains summed two by two in order, each sum compressed."""
    terms = list(terms)
    while len(terms) > 1:
        nxt = []
        for t in range(0, len(terms), 2):
            nxt.append(round_tt(add(terms[t], terms[t + 1]), chi_max, rel_tol) if t + 1 < len(terms) else terms[t])
        terms = nxt
    return terms[0]


def pauli_apply(cores, coeffs, ops, alpha, beta, chi_max, rel_tol=1e-14, chi_sum=None):
    """alpha phi + beta sum_t c_t O_t phi, compressed: the terms c_t O_t phi
    summed two by two (each partial sum compressed to chi_sum, by default
    chi_max), scaled by beta, alpha phi added when alpha != 0, and the whole
    compressed to chi_max.  alpha = 1, beta = -tau is a power step of
    Sec. 3.1 for any replica Hamiltonian.  Sec. 3.1 names one target rank;
    the partial sums of H-bar phi are read as allowed a larger one, since
    cutting them to the final rank loses most of the step (on a 4x4 open
    lattice with H-bar_HV at chi = 2 the error after 40 steps is 2e-2 with
    chi_sum = 2 and 1.2e-3 with chi_sum = 8 or unbounded)."""
    terms = [scale(apply_string(cores, o), float(c)) for c, o in zip(coeffs, ops)]
    s = scale(pairwise_sum(terms, chi_max if chi_sum is None else chi_sum, rel_tol), beta)
    if alpha != 0.0:
        s = add(scale(cores, alpha), s)
    return round_tt(s, chi_max, rel_tol)


def combine(trains, coeffs, chi_max, rel_tol=1e-14):
    """sum_m c_m phi_m compressed (the final compression of a linear
    combination, Sec. 4.3): terms summed two by two, then compressed."""
    return round_tt(pairwise_sum([scale(t, float(c)) for t, c in zip(trains, coeffs)], chi_max, rel_tol),
                    chi_max, rel_tol)


def constant_train(L):
    """phi^(0)_i = 1 for every replica index (bond dimension 1)."""
    return [np.ones((2, 1, 1)) for _ in range(L)]
