"""Tensor-train utilities used to build exact test states.
Test infrastructure only.

  * tt_svd: exact tensor-train (MPS) decomposition of a state vector by
    successive SVDs (Sec. 2.1 defines the MPS as a TT with Omega = N).
  * direct_sum: the sum of tensor trains as one train with block-diagonal
    cores (adding two TTs yields a TT, Sec. 2.2.3).
  * mps_energy: <psi|H|psi>/<psi|psi> of an R = 1 train by transfer matrices.
"""
from __future__ import annotations

import numpy as np


def tt_svd(vec, N: int, tol: float = 1e-14):
    """Cores (2, a, b) with psi(s) = prod_k A_k[s_k]; vector index = sum s_j 2^j."""
    T = np.asarray(vec, dtype=np.float64).reshape((2,) * N)   # axes s_{N-1}..s_0
    T = np.transpose(T, list(reversed(range(N))))               # axes s_0..s_{N-1}
    cores = []
    a = 1
    M = T.reshape(a * 2, -1)
    for k in range(N - 1):
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        keep = max(1, int(np.sum(S > tol * S[0])))
        U, S, Vt = U[:, :keep], S[:keep], Vt[:keep]
        cores.append(U.reshape(a, 2, keep).transpose(1, 0, 2).copy())
        M = (S[:, None] * Vt)
        a = keep
        M = M.reshape(a * 2, -1)
    cores.append(M.reshape(a, 2, 1).transpose(1, 0, 2).copy())
    return cores


def direct_sum(terms, coeffs):
    """One train whose amplitude is sum_a c_a psi^a (all terms share the path)."""
    L = len(terms[0])
    out = []
    for k in range(L):
        blocks = [t[k] for t in terms]
        if k == 0:
            blocks = [c * b for c, b in zip(coeffs, blocks)]
        rows = [b.shape[1] for b in blocks]
        cols = [b.shape[2] for b in blocks]
        if k == 0:
            C = np.concatenate(blocks, axis=2)                  # (2, 1, sum b)
        elif k == L - 1:
            C = np.concatenate(blocks, axis=1)                  # (2, sum a, 1)
        else:
            C = np.zeros((2, sum(rows), sum(cols)))
            r0 = c0 = 0
            for b in blocks:
                C[:, r0:r0 + b.shape[1], c0:c0 + b.shape[2]] = b
                r0 += b.shape[1]
                c0 += b.shape[2]
        out.append(C)
    return out


def _transfer(E, A, op):
    """E (a, a) -> sum_{s,s'} op[s, s'] A[s]^T E A[s'] (bra slice s, ket s')."""
    out = 0.0
    for s in range(2):
        for t in range(2):
            if op[s, t] != 0.0:
                out = out + op[s, t] * (A[s].T @ E @ A[t])
    return out


def mps_energy(cores, bonds, J: float, h: float) -> float:
    """<H>/<1> for psi(s) = prod_k A_k[s_k] (R = 1, site order)."""
    N = len(cores)
    I = np.eye(2)
    Z = np.diag([1.0, -1.0])
    X = np.array([[0.0, 1.0], [1.0, 0.0]])

    def expect(ops):
        E = np.ones((1, 1))
        for k in range(N):
            E = _transfer(E, cores[k], ops.get(k, I))
        return float(E[0, 0])

    norm = expect({})
    tot = 0.0
    for i, j in np.asarray(bonds).reshape(-1, 2):
        tot += J * expect({int(i): Z, int(j): Z})
    for i in range(N):
        tot -= h * expect({i: X})
    return tot / norm
