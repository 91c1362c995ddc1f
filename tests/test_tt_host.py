"""The library's host tensor-train algebra (rtt_tt_round, rtt_tfim_power_step;
paper Sec. 3.1) against the oracle: physical amplitudes on every
configuration (gauge-invariant), energies after several truncated power
steps, and host-side argument errors.  Runs without a GPU."""
import ctypes as C

import numpy as np
import pytest

from oracle import replica, rtt as orc, tfim
from paper_2604_22718_amd import workloads as wl

J, HF = 1.0, 3.04


@pytest.fixture(scope="module")
def R():
    from paper_2604_22718_amd import rtt
    return rtt


def amps(cores, pi, N):
    return orc.amplitudes(cores, pi, orc.all_configs(N))


@pytest.mark.parametrize("chi_max", [64, 5, 3])
def test_round_matches_oracle(R, chi_max):
    N = 7
    pi = wl.path_site_plus_perms(N, 2, 400)
    a = wl.gaussian_cores(wl.open_bonds(2 * N, 3), 401)
    b = wl.gaussian_cores(wl.open_bonds(2 * N, 3), 402)
    s = replica.add(a, replica.scale(b, 0.6))
    got = R.rtt_tt_round(s, chi_max)
    ref = replica.round_tt(s, chi_max)
    assert [c.shape for c in got] == [c.shape for c in ref]
    x, y = amps(got, pi, N), amps(ref, pi, N)
    assert np.allclose(x, y, rtol=0, atol=1e-10 * np.abs(y).max())
    if chi_max >= 6:  # untruncated: the same state
        assert np.allclose(x, amps(s, pi, N), rtol=0, atol=1e-10 * np.abs(y).max())


def test_power_step_matches_oracle(R):
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi = wl.path_site_plus_perms(N, 2, 410)
    c = wl.gaussian_cores(wl.open_bonds(2 * N, 2), 411)
    for chi_max in (4096, 4):
        got = R.rtt_tfim_power_step(N, pi, c, Lx, Ly, J, HF, 0.05, chi_max)
        ref = replica.power_step(c, pi, tfim.bonds(Lx, Ly), J, HF, 0.05, chi_max)
        x, y = amps(got, pi, N), amps(ref, pi, N)
        assert np.allclose(x, y, rtol=0, atol=1e-9 * np.abs(y).max()), chi_max


def test_power_method_energies_track_the_oracle(R):
    """3x3, R = 2, bond 6, 25 truncated steps on both sides: the exact
    energies of the two trains agree and fall towards E0."""
    Lx, Ly = 3, 3
    N = Lx * Ly
    pi = wl.path_site_plus_perms(N, 2, 420)
    c0 = wl.gaussian_cores(wl.open_bonds(2 * N, 2), 421)
    bonds = tfim.bonds(Lx, Ly)
    a, b = c0, c0
    for step in range(25):
        a = R.rtt_tfim_power_step(N, pi, a, Lx, Ly, J, HF, 0.04, 6)
        b = replica.power_step(b, pi, bonds, J, HF, 0.04, 6)
        na, nb = np.abs(amps(a, pi, N)).max(), np.abs(amps(b, pi, N)).max()
        a, b = replica.scale(a, 1 / na), replica.scale(b, 1 / nb)
    ea = orc.exact_energy(a, pi, N, bonds, J, HF)
    eb = orc.exact_energy(b, pi, N, bonds, J, HF)
    e_start = orc.exact_energy(c0, pi, N, bonds, J, HF)
    e0, _ = tfim.ground_state(Lx, Ly, J, HF)
    assert abs(ea - eb) < 1e-6 * abs(eb)
    assert e0 - 1e-9 <= ea < e_start


def test_host_argument_errors(R):
    from paper_2604_22718_amd._lib import lib
    L = lib()
    bond = np.array([1, 2, 1], dtype=np.int32)
    cores = np.zeros(8)
    out_b = np.zeros(3, dtype=np.int32)
    out = np.zeros(1)
    n = C.c_int64()
    st = L.rtt_tt_round(2, bond.ctypes.data, cores.ctypes.data, 2, 1e-14, out_b.ctypes.data, out.ctypes.data, 1,
                        C.byref(n))
    assert st == -1 and n.value >= 4 and b"capacity" in L.rtt_last_error()
    bad = np.array([2, 2, 1], dtype=np.int32)
    assert L.rtt_tt_round(2, bad.ctypes.data, cores.ctypes.data, 2, 1e-14, out_b.ctypes.data, out.ctypes.data,
                          8, C.byref(n)) == -1
    nanc = cores.copy()
    nanc[1] = np.nan
    assert L.rtt_tt_round(2, bond.ctypes.data, nanc.ctypes.data, 2, 1e-14, out_b.ctypes.data, out.ctypes.data,
                          8, C.byref(n)) == -1
    pi = np.array([0, 0], dtype=np.int32)   # spin 1 of a 2-site lattice read by no position
    assert L.rtt_tfim_power_step(2, 2, pi.ctypes.data, bond.ctypes.data, cores.ctypes.data, 2, 1, 0, 1.0, 1.0, 0.1,
                                 4, 1e-14, out_b.ctypes.data, out.ctypes.data, 8, C.byref(n)) == -1
    assert b"read by no position" in L.rtt_last_error()


def test_long_constant_train_stays_finite(R):
    """The constant train on 1600 positions (a 20x20 lattice, four parts) has
    norm 2^800: rounding squares no entry of that size, a power step with
    the full replica Hamiltonian stays finite, and normalisation works."""
    from paper_2604_22718_amd import lattice, pipeline
    L = 20
    pi = lattice.path(L, L)
    phi = pipeline.constant_train(len(pi))
    r = R.rtt_tt_round(phi, 2)
    assert all(np.all(np.isfinite(c)) for c in r)
    assert np.isclose(np.abs(r[-1]).max() * np.sqrt(2), 2.0 ** 800, rtol=1e-12)
    c, o = lattice.replica_hamiltonian(L, L, "HV", 3.0, periodic=False)
    sel = np.r_[0:40, 760:800]                      # ZZ and X strings
    out = R.rtt_pauli_apply(phi, c[sel], o[sel], 1.0, -0.1, 2, 4)
    assert all(np.all(np.isfinite(x)) for x in out)
    n = pipeline.normalise(out)
    assert np.isclose(np.linalg.norm(n[-1]), 1.0) and all(np.all(np.isfinite(x)) for x in n)


def test_degenerate_trains(R):
    """One core; a train that is exactly zero; beta = 0 (rounding alone);
    a single Pauli string."""
    from oracle import replica as orep
    one = [np.array([[[0.7]], [[-1.3]]])]
    x = R.rtt_pauli_apply(one, [2.0], np.array([[1]], dtype=np.uint8), 0.5, 1.0, 4)
    assert np.allclose(x[0].ravel(), 0.5 * np.array([0.7, -1.3]) + 2.0 * np.array([-1.3, 0.7]))
    assert np.allclose(R.rtt_tt_combine([one, one], [1.0, -3.0], 2)[0].ravel(), -2.0 * one[0].ravel())
    c = wl.gaussian_cores(wl.open_bonds(6, 3), 950)
    pi = np.arange(6, dtype=np.int32)
    S = orc.all_configs(6)
    z = R.rtt_tt_combine([c, c], [1.0, -1.0], 3)            # zero up to rounding
    assert all(np.all(np.isfinite(k)) for k in z)
    assert np.abs(orc.amplitudes(z, pi, S)).max() < 1e-13 * np.abs(orc.amplitudes(c, pi, S)).max()
    zero = [np.zeros((2, a, b)) for a, b in zip(wl.open_bonds(6, 3)[:-1], wl.open_bonds(6, 3)[1:])]
    z = R.rtt_tt_round(zero, 3)                              # exactly zero: one bond kept, psi = 0
    assert max(k.shape[2] for k in z) == 1 and np.all(orc.amplitudes(z, pi, S) == 0.0)
    r = R.rtt_pauli_apply(c, [1.0], np.zeros((1, 6), dtype=np.uint8), 1.0, 0.0, 2)
    ref = orep.round_tt(c, 2)
    assert np.allclose(orc.amplitudes(r, pi, S), orc.amplitudes(ref, pi, S), rtol=0, atol=1e-12)
    ops = np.array([[3, 0, 2, 1, 0, 3]], dtype=np.uint8)
    got = R.rtt_pauli_apply(c, [-0.4], ops, 0.0, 1.0, 64)
    want = orep.pauli_apply(c, [-0.4], ops, 0.0, 1.0, 64)
    assert np.allclose(orc.amplitudes(got, pi, S), orc.amplitudes(want, pi, S), rtol=0, atol=1e-12)
