"""Pins of the replica-space oracle (paper Sec. 2.2.3 and Sec. 3.1) against
facts outside it: the physical Pauli operators on enumerated amplitudes,
the Kronecker-product Hamiltonian, exactness of untruncated rounding, exact
low-rank sums, and the ground energy from exact diagonalisation."""
import numpy as np
import pytest

from oracle import replica, rtt, tfim
from paper_2604_22718_amd import workloads as wl


def state(N, R, chi, seed):
    pi = wl.path_site_plus_perms(N, R, seed)
    return pi, wl.gaussian_cores(wl.open_bonds(N * R, chi), seed + 1)


def test_x_on_all_replicas_and_z_on_one():
    N = 6
    pi, c = state(N, 2, 3, 200)
    S = rtt.all_configs(N)
    psi = rtt.amplitudes(c, pi, S)
    for j in (0, 2, 5):
        x = rtt.amplitudes(replica.apply_x(c, pi, j), pi, S)
        assert np.allclose(x, rtt.amplitudes(c, pi, rtt.flip(S, j)), rtol=1e-12, atol=0)
        z = rtt.amplitudes(replica.apply_z(c, pi, j), pi, S)
        assert np.allclose(z, (1 - 2 * S[:, j].astype(np.int64)) * psi, rtol=1e-12, atol=0)


def test_rounding_without_truncation_is_exact_and_sums_compress_to_their_rank():
    N = 6
    pi, a = state(N, 2, 3, 210)
    _, b = state(N, 2, 3, 220)
    b = [x for x in b]
    S = rtt.all_configs(N)
    s = replica.add(a, replica.scale(b, -0.7))
    ref = rtt.amplitudes(a, pi, S) - 0.7 * rtt.amplitudes(b, pi, S)
    full = replica.round_tt(s, 64)
    assert np.allclose(rtt.amplitudes(full, pi, S), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # the sum of two bond-3 trains has bond <= 6: rounding to 6 is exact
    six = replica.round_tt(s, 6)
    assert max(c.shape[2] for c in six) <= 6
    assert np.allclose(rtt.amplitudes(six, pi, S), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # and a sum of a train with itself has the train's rank
    twice = replica.round_tt(replica.add(a, a), 3)
    assert np.allclose(rtt.amplitudes(twice, pi, S), 2 * rtt.amplitudes(a, pi, S), rtol=1e-10)


def test_untruncated_power_step_is_one_minus_tau_h():
    """C phi' = (1 - tau H) C phi with H from Pauli Kronecker products."""
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi, c = state(N, 2, 2, 230)
    J, h, tau = 1.0, 3.04, 0.05
    new = replica.power_step(c, pi, tfim.bonds(Lx, Ly), J, h, tau, chi_max=4096)
    S = rtt.all_configs(N)
    psi = rtt.amplitudes(c, pi, S)
    H = tfim.sparse_hamiltonian(Lx, Ly, J, h)
    want = psi - tau * (H @ psi)
    got = rtt.amplitudes(new, pi, S)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-11 * np.abs(want).max())


def test_power_method_approaches_the_ground_energy():
    """3x3 lattice, R = 2, bond 6 kept by compression: 80 steps of
    (1 - tau H-bar) lower the energy monotonically towards E0."""
    Lx, Ly = 3, 3
    N = Lx * Ly
    pi, c = state(N, 2, 2, 240)
    J, h, tau = 1.0, 3.04, 0.04
    bonds = tfim.bonds(Lx, Ly)
    e0, _ = tfim.ground_state(Lx, Ly, J, h)
    es = []
    for step in range(80):
        c = replica.power_step(c, pi, bonds, J, h, tau, chi_max=6)
        c = replica.scale(c, 1.0 / np.abs(rtt.amplitudes(c, pi, rtt.all_configs(N))).max())  # keep O(1)
        if step % 20 == 19:
            es.append(rtt.exact_energy(c, pi, N, bonds, J, h))
    assert all(es[i + 1] <= es[i] + 1e-9 for i in range(len(es) - 1))
    assert es[-1] >= e0 - 1e-9
    assert (es[-1] - e0) < 0.05 * abs(e0), (es, e0)
