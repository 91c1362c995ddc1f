"""The paper's four-part path and its replica-space operators (Sec. 4.1:
the V, H, D, D' orderings, the bond operators O_{ZZ,B} and O_X, and their
replica images routed to one part of the path, "-> C").  Test
infrastructure only.

Readings (the drawings of the orderings are missing from the text):
  * sites are numbered in raster order i = y*Lx + x;
  * H visits the rows y = 0, 1, ... as a snake (even rows with x rising,
    odd rows with x falling); V visits the columns x = Lx-1, Lx-2, ... as a
    snake, the first column with y falling.  With the sites relabelled
    along the H snake, H is the identity and, on 2 rows of 3 sites, V is
    the ordering (4,3,2,5,6,1) of the worked example of Sec. 2.2.1;
  * D visits the diagonals x + y = 0, 1, ... and D' the anti-diagonals
    x - y = -(Ly-1), ..., Lx-1, each as a snake (even diagonals with x
    rising, odd ones with x falling);
  * the whole path is H + V + D + D' in that order: the name HVDD' of the
    path and the statement that R_{i1} is the H position agree on it, while
    the displayed concatenation lists V first;
  * the bond directions: H (x,y)-(x+1,y), V (x,y)-(x,y+1), D (x,y)-(x+1,y+1),
    D' (x,y)-(x+1,y-1); with periodic boundaries a bond wraps only along
    sides of length >= 3 (as for the TFIM bonds).
Operator strings are per-position codes 0 I, 1 X, 2 Z, 3 X Z.
"""
from __future__ import annotations

import numpy as np

PARTS = ("H", "V", "D", "D'")


def path_h(Lx, Ly):
    out = []
    for y in range(Ly):
        xs = range(Lx) if y % 2 == 0 else range(Lx - 1, -1, -1)
        out += [y * Lx + x for x in xs]
    return out


def path_v(Lx, Ly):
    out = []
    for n, x in enumerate(range(Lx - 1, -1, -1)):
        ys = range(Ly - 1, -1, -1) if n % 2 == 0 else range(Ly)
        out += [y * Lx + x for y in ys]
    return out


def path_d(Lx, Ly):
    out = []
    for d in range(Lx + Ly - 1):
        cells = [(x, d - x) for x in range(Lx) if 0 <= d - x < Ly]
        if d % 2 == 1:
            cells = cells[::-1]
        out += [y * Lx + x for x, y in cells]
    return out


def path_dp(Lx, Ly):
    out = []
    for n, e in enumerate(range(-(Ly - 1), Lx)):
        cells = [(x, x - e) for x in range(Lx) if 0 <= x - e < Ly]
        if n % 2 == 1:
            cells = cells[::-1]
        out += [y * Lx + x for x, y in cells]
    return out


def path_parts(Lx, Ly):
    return {"H": path_h(Lx, Ly), "V": path_v(Lx, Ly), "D": path_d(Lx, Ly), "D'": path_dp(Lx, Ly)}


def path_hvddp(Lx, Ly):
    """pi of the four-part path: position k reads spin pi[k]."""
    p = path_parts(Lx, Ly)
    return np.array(p["H"] + p["V"] + p["D"] + p["D'"], dtype=np.int32)


def position(Lx, Ly, site, part, parts=PARTS):
    """Train position of ``site`` inside part ``part`` (R_{site, part})."""
    p = path_parts(Lx, Ly)
    c = parts.index(part)
    return c * Lx * Ly + p[part].index(site)


def direction_bonds(Lx, Ly, direction, periodic=True):
    """Pairs (i, j) of the bonds of one direction."""
    dx, dy = {"H": (1, 0), "V": (0, 1), "D": (1, 1), "D'": (1, -1)}[direction]
    out = []
    for y in range(Ly):
        for x in range(Lx):
            x2, y2 = x + dx, y + dy
            if not (0 <= x2 < Lx):
                if not (periodic and Lx >= 3):
                    continue
                x2 %= Lx
            if not (0 <= y2 < Ly):
                if not (periodic and Ly >= 3):
                    continue
                y2 %= Ly
            out.append((y * Lx + x, y2 * Lx + x2))
    return out


def string(L, x_positions=(), z_positions=()):
    ops = np.zeros(L, dtype=np.uint8)
    for k in x_positions:
        ops[k] |= 1
    for k in z_positions:
        ops[k] ^= 2      # Z Z on one position is the identity
    return ops


def zz_strings(Lx, Ly, direction, to_part, periodic=True):
    """Strings of O-bar_{ZZ, direction -> to_part}: Z_{R_{i,c}} Z_{R_{j,c}}."""
    L = 4 * Lx * Ly
    return [string(L, z_positions=(position(Lx, Ly, i, to_part), position(Lx, Ly, j, to_part)))
            for i, j in direction_bonds(Lx, Ly, direction, periodic)]


def x_strings(Lx, Ly):
    """Strings of O-bar_X: X on every replica of a site."""
    L = 4 * Lx * Ly
    return [string(L, x_positions=[position(Lx, Ly, i, c) for c in PARTS]) for i in range(Lx * Ly)]


def hamiltonian(Lx, Ly, kind, h, alpha=0.0, J=1.0, periodic=True):
    """(coeffs, ops) of the replica Hamiltonians of Sec. 4.2: 'H' (both bond
    directions sent to H), 'HV' (each to its own part) and 'HVDD'' (HV plus
    alpha times the diagonal bonds, each sent to its own part)."""
    terms = []
    if kind == "H":
        terms += [(J, s) for s in zz_strings(Lx, Ly, "H", "H", periodic)]
        terms += [(J, s) for s in zz_strings(Lx, Ly, "V", "H", periodic)]
    elif kind in ("HV", "HVDD'"):
        terms += [(J, s) for s in zz_strings(Lx, Ly, "H", "H", periodic)]
        terms += [(J, s) for s in zz_strings(Lx, Ly, "V", "V", periodic)]
    else:
        raise ValueError(kind)
    terms += [(-h, s) for s in x_strings(Lx, Ly)]
    if kind == "HVDD'":
        terms += [(alpha, s) for s in zz_strings(Lx, Ly, "D", "D", periodic)]
        terms += [(alpha, s) for s in zz_strings(Lx, Ly, "D'", "D'", periodic)]
    return np.array([c for c, _ in terms]), np.array([s for _, s in terms], dtype=np.uint8)


def operator(Lx, Ly, name, periodic=True):
    """(coeffs, ops) of the physical-space operators of Sec. 4.3: 'I', 'X',
    'ZZ_HV' (H -> H plus V -> V) and 'ZZ_DD'' (D -> D plus D' -> D')."""
    L = 4 * Lx * Ly
    if name == "I":
        strs = [string(L)]
    elif name == "X":
        strs = x_strings(Lx, Ly)
    elif name == "ZZ_HV":
        strs = zz_strings(Lx, Ly, "H", "H", periodic) + zz_strings(Lx, Ly, "V", "V", periodic)
    elif name == "ZZ_DD'":
        strs = zz_strings(Lx, Ly, "D", "D", periodic) + zz_strings(Lx, Ly, "D'", "D'", periodic)
    else:
        raise ValueError(name)
    return np.ones(len(strs)), np.array(strs, dtype=np.uint8)
