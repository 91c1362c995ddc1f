"""Pins of the oracle's four-part path, its replica-space operators and the
general Pauli-string power step (Sec. 2.2.1 worked paths, Sec. 2.2.3
operator example and commutation rules, Sec. 4.1 orderings and operators)
against the paper's printed example, lattice geometry, dense Kronecker
products and the physical operators applied to enumerated amplitudes."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import paths, replica, rtt, tfim
from paper_2604_22718_amd import workloads as wl

I2 = np.eye(2)
X2 = np.array([[0.0, 1.0], [1.0, 0.0]])
Z2 = np.diag([1.0, -1.0])
MATS = {0: I2, 1: X2, 2: Z2, 3: X2 @ Z2}


def labels_along_h(Lx, Ly):
    """1-based labels that number the sites along the H snake."""
    lab = np.zeros(Lx * Ly, dtype=int)
    for n, s in enumerate(paths.path_h(Lx, Ly)):
        lab[s] = n + 1
    return lab


def test_h_and_v_reproduce_the_worked_path():
    g = read_golden("path_hv_2x3.txt")
    lab = labels_along_h(3, 2)
    assert [lab[s] for s in paths.path_h(3, 2)] == [1, 2, 3, 4, 5, 6]
    assert [lab[s] for s in paths.path_v(3, 2)] == g["path_v"]
    assert [lab[s] for s in paths.path_h(3, 2) + paths.path_v(3, 2)] == g["path_hv"]


def test_operator_example_routes_as_printed():
    """A = Z1Z2 + Z1Z6 + X3 + X1X2 with Z1Z2 sent to H and Z1Z6 to V gives
    A-bar = Z1Z2 + Z11Z12 + X3X8 + X1X2X9X12 on the 12-position HV path."""
    lab = labels_along_h(3, 2)
    site = {lab[s]: s for s in range(6)}
    hv = ("H", "V")
    pos = lambda label, part: paths.position(3, 2, site[label], part, parts=hv)
    got = [
        paths.string(12, z_positions=(pos(1, "H"), pos(2, "H"))),
        paths.string(12, z_positions=(pos(1, "V"), pos(6, "V"))),
        paths.string(12, x_positions=[pos(3, c) for c in hv]),
        paths.string(12, x_positions=[pos(1, c) for c in hv] + [pos(2, c) for c in hv]),
    ]
    printed = [((), (1, 2)), ((), (11, 12)), ((3, 8), ()), ((1, 2, 9, 12), ())]
    for s, (xs, zs) in zip(got, printed):
        want = np.zeros(12, dtype=np.uint8)
        want[[x - 1 for x in xs]] |= 1
        want[[z - 1 for z in zs]] |= 2
        assert np.array_equal(s, want)


@pytest.mark.parametrize("Lx,Ly", [(4, 4), (5, 3), (2, 6), (1, 4)])
def test_parts_are_connected_orderings(Lx, Ly):
    for name, p in paths.path_parts(Lx, Ly).items():
        assert sorted(p) == list(range(Lx * Ly)), name
        xy = [(s % Lx, s // Lx) for s in p]
        for (x0, y0), (x1, y1) in zip(xy, xy[1:]):
            d = (abs(x1 - x0), abs(y1 - y0))
            if name in ("H", "V"):
                assert d in ((1, 0), (0, 1)), (name, d)
            else:
                assert max(d) == 1, (name, d)
    pi = paths.path_hvddp(Lx, Ly)
    assert len(pi) == 4 * Lx * Ly
    for c, part in enumerate(paths.PARTS):
        for s in range(Lx * Ly):
            assert pi[paths.position(Lx, Ly, s, part)] == s


@pytest.mark.parametrize("periodic", [True, False])
def test_direction_bonds(periodic):
    for Lx, Ly in ((4, 4), (3, 5), (2, 3)):
        h = paths.direction_bonds(Lx, Ly, "H", periodic)
        v = paths.direction_bonds(Lx, Ly, "V", periodic)
        assert sorted(map(tuple, tfim.bonds(Lx, Ly, periodic).tolist())) == sorted(h + v)
        for d in ("D", "D'"):
            b = paths.direction_bonds(Lx, Ly, d, periodic)
            for i, j in b:
                dx = (j % Lx - i % Lx) % Lx
                dy = (j // Lx - i // Lx) % Ly
                assert dx == 1 % Lx and dy == (1 if d == "D" else Ly - 1) % Ly
            if periodic and Lx >= 3 and Ly >= 3:
                assert len(b) == Lx * Ly
            if not periodic:
                assert len(b) == (Lx - 1) * (Ly - 1)


def dense_train(cores):
    v = np.ones((1, 1))
    for A in cores:
        v = np.einsum("pa,sab->psb", v, A).reshape(-1, A.shape[2])
    return v.ravel()


def test_pauli_apply_is_the_kronecker_product():
    L = 8
    phi = wl.gaussian_cores(wl.open_bonds(L, 3), 700)
    rng = np.random.default_rng(701)
    ops = rng.integers(0, 4, size=(4, L)).astype(np.uint8)
    coeffs = rng.normal(size=4)
    got = dense_train(replica.pauli_apply(phi, coeffs, ops, 0.7, -0.3, 4096))
    v = dense_train(phi)
    want = 0.7 * v
    for c, o in zip(coeffs, ops):
        M = np.ones((1, 1))
        for k in range(L):
            M = np.kron(M, MATS[int(o[k])])
        want = want - 0.3 * c * (M @ v)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # combine: sum_m c_m phi_m
    other = wl.gaussian_cores(wl.open_bonds(L, 2), 702)
    got = dense_train(replica.combine([phi, other], [0.4, -1.5], 4096))
    want = 0.4 * v - 1.5 * dense_train(other)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def physical(op, Lx, Ly, psi, periodic):
    """The physical operator of Sec. 4.1.2 applied to the amplitude vector
    psi (index sum_j s_j 2^j) by enumeration."""
    N = Lx * Ly
    S = rtt.all_configs(N)
    z = 1 - 2 * S.astype(float)
    idx = np.arange(2 ** N)
    if op == "X":
        return sum(psi[idx ^ (1 << j)] for j in range(N))
    dirs = {"ZZ_HV": ("H", "V"), "ZZ_DD'": ("D", "D'"), "ZZ_H": ("H",), "ZZ_V": ("V",)}[op]
    diag = np.zeros(2 ** N)
    for d in dirs:
        for i, j in paths.direction_bonds(Lx, Ly, d, periodic):
            diag += z[:, i] * z[:, j]
    return diag * psi


@pytest.mark.parametrize("periodic", [True, False])
def test_replica_operators_commute_with_the_copy_tensor(periodic):
    """C O-bar phi = O C phi for O_X, O_{ZZ,HV}, O_{ZZ,DD'}, whichever part
    the Z's are sent to, and the replica Hamiltonians H and HV give C phi' =
    (1 - tau H) C phi for an uncompressed power step."""
    Lx, Ly = 3, 3
    N = Lx * Ly
    pi = paths.path_hvddp(Lx, Ly)
    phi = wl.gaussian_cores(wl.open_bonds(len(pi), 2), 710)
    S = rtt.all_configs(N)
    psi = rtt.amplitudes(phi, pi, S)
    big = 4096
    for name in ("X", "ZZ_HV", "ZZ_DD'"):
        c, o = paths.operator(Lx, Ly, name, periodic)
        got = rtt.amplitudes(replica.pauli_apply(phi, c, o, 0.0, 1.0, big), pi, S)
        want = physical(name, Lx, Ly, psi, periodic)
        assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max()), name
    for d in ("H", "V"):
        for part in paths.PARTS:
            strs = paths.zz_strings(Lx, Ly, d, part, periodic)
            got = rtt.amplitudes(replica.pauli_apply(phi, np.ones(len(strs)), strs, 0.0, 1.0, big), pi, S)
            want = physical("ZZ_" + d, Lx, Ly, psi, periodic)
            assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max()), (d, part)
    hx, tau = 3.0, 0.05
    Hpsi = physical("ZZ_HV", Lx, Ly, psi, periodic) - hx * physical("X", Lx, Ly, psi, periodic)
    for kind in ("H", "HV"):
        c, o = paths.hamiltonian(Lx, Ly, kind, hx, periodic=periodic)
        got = rtt.amplitudes(replica.pauli_apply(phi, c, o, 1.0, -tau, big), pi, S)
        want = psi - tau * Hpsi
        assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max()), kind
    c, o = paths.hamiltonian(Lx, Ly, "HVDD'", hx, alpha=0.08, periodic=periodic)
    got = rtt.amplitudes(replica.pauli_apply(phi, c, o, 1.0, -tau, big), pi, S)
    want = psi - tau * (Hpsi + 0.08 * physical("ZZ_DD'", Lx, Ly, psi, periodic))
    assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_power_method_from_the_constant_train():
    """phi^(0) = 1 is the uniform superposition (energy -h N: every
    <Z_i Z_j> vanishes in it); chi = 2 power steps with H-bar_HV lower the exact energy
    towards, and never below, E0 (3x3 periodic, h = 3, tau = 0.1)."""
    Lx, Ly, hx = 3, 3, 3.0
    N = Lx * Ly
    pi = paths.path_hvddp(Lx, Ly)
    phi = replica.constant_train(len(pi))
    bonds = tfim.bonds(Lx, Ly)
    e = [rtt.exact_energy(phi, pi, N, bonds, 1.0, hx)]
    assert math.isclose(e[0], -hx * N, rel_tol=1e-12)
    c, o = paths.hamiltonian(Lx, Ly, "HV", hx)
    for _ in range(12):
        phi = replica.pauli_apply(phi, c, o, 1.0, -0.1, 2)
        phi = replica.scale(phi, 1.0 / np.linalg.norm(phi[-1]))
        e.append(rtt.exact_energy(phi, pi, N, bonds, 1.0, hx))
    e0, _ = tfim.ground_state(Lx, Ly, 1.0, hx)
    assert max(x.shape[2] for x in phi) == 2
    assert e0 - 1e-9 <= e[-1] < e[0]
