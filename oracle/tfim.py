"""Transverse-field Ising model on an Lx x Ly square lattice (paper Sec. 4,
Ising model equation).  Test infrastructure only.

Site numbering is raster order i = y*Lx + x.  Bonds are nearest-neighbour
pairs; with ``periodic`` the wrap-around bonds are added along every side of
length >= 3 (a side of length 2 already has its only bond).  The Hamiltonian
is H = J sum_<ij> Z_i Z_j - h sum_i X_i with Z|s> = (-1)^s |s>.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def bonds(Lx: int, Ly: int, periodic: bool = True) -> np.ndarray:
    out = []
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            if x + 1 < Lx:
                out.append((i, y * Lx + x + 1))
            elif periodic and Lx >= 3:
                out.append((i, y * Lx))
            if y + 1 < Ly:
                out.append((i, (y + 1) * Lx + x))
            elif periodic and Ly >= 3:
                out.append((i, x))
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def _pauli_chain(N: int, site_ops: dict):
    """Kronecker product of single-site operators; basis index sum_j s_j 2^j,
    so site j is the j-th least significant factor."""
    I = sp.identity(2, format="csr")
    M = sp.identity(1, format="csr")
    for j in reversed(range(N)):
        M = sp.kron(M, site_ops.get(j, I), format="csr")
    return M


def sparse_hamiltonian(Lx: int, Ly: int, J: float, h: float, periodic=True):
    """H built from Pauli matrices and Kronecker products (independent of the
    local-energy formula)."""
    N = Lx * Ly
    X = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
    Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
    H = sp.csr_matrix((2 ** N, 2 ** N))
    for i, j in bonds(Lx, Ly, periodic):
        H = H + J * _pauli_chain(N, {int(i): Z, int(j): Z})
    for i in range(N):
        H = H - h * _pauli_chain(N, {i: X})
    return H.tocsr()


def ground_state(Lx: int, Ly: int, J: float, h: float, periodic=True):
    """Lowest eigenpair by scipy eigsh (exact diagonalisation)."""
    H = sparse_hamiltonian(Lx, Ly, J, h, periodic)
    vals, vecs = spla.eigsh(H, k=1, which="SA", tol=1e-12)
    v = vecs[:, 0]
    if v[np.argmax(np.abs(v))] < 0:
        v = -v
    return float(vals[0]), v
