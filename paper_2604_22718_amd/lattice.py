"""The four-part path H + V + D + D' of the paper's Ising study (Sec. 4.1.1)
and the replica-space Pauli strings of its operators (Sec. 4.1.2-4.1.3),
as tables for rtt_create and rtt_pauli_apply.

Sites are numbered in raster order i = y*Lx + x.  H visits the rows as a
snake (even rows left to right), V the columns from the last one as a snake
(the first column bottom to top), D the diagonals x + y = const and D' the
anti-diagonals x - y = const, each as a snake (even diagonals with x rising).
The train is H, V, D, D' in that order, so R_{i,c} = c*N + (index of site i
in part c).  A ZZ operator of one bond direction is sent to one part ("-> C"):
both Z's act on the two sites' positions in that part; X acts on all four.
Bond directions: H (x,y)-(x+1,y), V (x,y)-(x,y+1), D (x,y)-(x+1,y+1),
D' (x,y)-(x+1,y-1); periodic boundaries wrap along sides of length >= 3.
Strings are listed bond by bond in raster order of the bond's first site.
"""
from __future__ import annotations

import numpy as np

PARTS = ("H", "V", "D", "D'")
OP_I, OP_X, OP_Z = 0, 1, 2
_STEP = {"H": (1, 0), "V": (0, 1), "D": (1, 1), "D'": (1, -1)}


def _grid(Lx, Ly):
    return np.arange(Lx * Ly, dtype=np.int64).reshape(Ly, Lx)


def _diagonal_snake(Lx, Ly, anti):
    y, x = np.divmod(np.arange(Lx * Ly), Lx)
    d = (x - y + Ly - 1) if anti else (x + y)
    along = np.where(d % 2 == 0, x, -x)
    return np.lexsort((along, d))


def part_orders(Lx, Ly):
    """Site order of each part, as int arrays of length N."""
    g = _grid(Lx, Ly)
    h = g.copy()
    h[1::2] = h[1::2, ::-1]
    v = g.T[::-1].copy()            # row n: column x = Lx-1-n, y rising
    v[0::2] = v[0::2, ::-1]
    return {"H": h.ravel(), "V": v.ravel(), "D": _diagonal_snake(Lx, Ly, False),
            "D'": _diagonal_snake(Lx, Ly, True)}


def path(Lx, Ly):
    """pi of the train: position k reads spin pi[k] (length 4N)."""
    o = part_orders(Lx, Ly)
    return np.concatenate([o[p] for p in PARTS]).astype(np.int32)


def replica_positions(Lx, Ly):
    """pos[c, i] = R_{i,c}: the train position of site i in part c."""
    N = Lx * Ly
    o = part_orders(Lx, Ly)
    pos = np.empty((4, N), dtype=np.int64)
    for c, p in enumerate(PARTS):
        pos[c, o[p]] = c * N + np.arange(N)
    return pos


def bond_pairs(Lx, Ly, direction, periodic=True):
    """(n, 2) site pairs of one bond direction."""
    dx, dy = _STEP[direction]
    y, x = np.divmod(np.arange(Lx * Ly), Lx)
    x2, y2 = x + dx, y + dy
    ok = np.ones(Lx * Ly, dtype=bool)
    outx = (x2 < 0) | (x2 >= Lx)
    outy = (y2 < 0) | (y2 >= Ly)
    ok &= ~outx | (periodic and Lx >= 3)
    ok &= ~outy | (periodic and Ly >= 3)
    j = (y2 % Ly) * Lx + (x2 % Lx)
    return np.stack([np.arange(Lx * Ly)[ok], j[ok]], axis=1)


def zz_ops(Lx, Ly, direction, to_part, periodic=True):
    """Strings of O-bar_{ZZ, direction -> to_part}: (n_bonds, 4N) uint8."""
    N = Lx * Ly
    pos = replica_positions(Lx, Ly)[PARTS.index(to_part)]
    b = bond_pairs(Lx, Ly, direction, periodic)
    ops = np.zeros((len(b), 4 * N), dtype=np.uint8)
    rows = np.arange(len(b))
    ops[rows, pos[b[:, 0]]] ^= OP_Z
    ops[rows, pos[b[:, 1]]] ^= OP_Z
    return ops


def x_ops(Lx, Ly):
    """Strings of O-bar_X: X on the four replicas of each site, (N, 4N)."""
    N = Lx * Ly
    ops = np.zeros((N, 4 * N), dtype=np.uint8)
    pos = replica_positions(Lx, Ly)
    for c in range(4):
        ops[np.arange(N), pos[c]] = OP_X
    return ops


def replica_hamiltonian(Lx, Ly, kind, h, alpha=0.0, J=1.0, periodic=True):
    """(coeffs, ops) of H-bar_H (both bond directions sent to H), H-bar_HV
    (each direction to its own part) or H-bar_HVDD' (H-bar_HV plus alpha
    times the diagonal bonds, each sent to its own part); Sec. 4.2."""
    if kind == "H":
        zz = [zz_ops(Lx, Ly, "H", "H", periodic), zz_ops(Lx, Ly, "V", "H", periodic)]
    elif kind in ("HV", "HVDD'"):
        zz = [zz_ops(Lx, Ly, "H", "H", periodic), zz_ops(Lx, Ly, "V", "V", periodic)]
    else:
        raise ValueError(f"unknown replica Hamiltonian {kind!r}")
    blocks = [(J, z) for z in zz] + [(-h, x_ops(Lx, Ly))]
    if kind == "HVDD'":
        blocks += [(alpha, zz_ops(Lx, Ly, "D", "D", periodic)), (alpha, zz_ops(Lx, Ly, "D'", "D'", periodic))]
    coeffs = np.concatenate([np.full(len(o), c, dtype=np.float64) for c, o in blocks])
    return coeffs, np.concatenate([o for _, o in blocks])


def operator(Lx, Ly, name, periodic=True):
    """(coeffs, ops) of the physical-space operators of Sec. 4.3: 'I', 'X',
    'ZZ_HV' (H -> H plus V -> V) and 'ZZ_DD'' (D -> D plus D' -> D')."""
    N = Lx * Ly
    if name == "I":
        ops = np.zeros((1, 4 * N), dtype=np.uint8)
    elif name == "X":
        ops = x_ops(Lx, Ly)
    elif name == "ZZ_HV":
        ops = np.concatenate([zz_ops(Lx, Ly, "H", "H", periodic), zz_ops(Lx, Ly, "V", "V", periodic)])
    elif name == "ZZ_DD'":
        ops = np.concatenate([zz_ops(Lx, Ly, "D", "D", periodic), zz_ops(Lx, Ly, "D'", "D'", periodic)])
    else:
        raise ValueError(f"unknown operator {name!r}")
    return np.ones(len(ops)), ops
