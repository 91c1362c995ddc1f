"""Pins of the dual Monte Carlo oracle (paper Sec. 3.3) against facts that do
not come from it: exact enumeration with the Kronecker-product Hamiltonian,
the symmetry of H and S, the eigenvalues of the symmetric problem by a
library routine, the exact ground state, and the Gram-Schmidt identity."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dual, mcmc, rtt, tfim, tt
from paper_2604_22718_amd import workloads as wl

J, H_FIELD = 1.0, 3.04


def three_states(N, R, chi, seed):
    pi = wl.path_site_plus_perms(N, R, seed)
    bond = wl.open_bonds(N * R, chi)
    a = wl.gaussian_cores(bond, seed + 1)
    b = wl.gaussian_cores(bond, seed + 2)
    c = wl.gaussian_cores(bond, seed + 3)
    return pi, [a, (([a, b], np.array([0.7, -1.3]))), c]


def test_same_state_reduces_to_local_energy():
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi, st = three_states(N, 2, 3, 40)
    S = wl.random_spins(30, N, 41)
    o, e = dual.mixed_estimators(st[0], st[0], pi, S, tfim.bonds(Lx, Ly), J, H_FIELD)
    assert np.allclose(o, 1.0, rtol=0, atol=1e-14)
    ref = rtt.local_energy(st[0], pi, S, tfim.bonds(Lx, Ly), J, H_FIELD)
    assert np.allclose(e, ref, rtol=1e-11)


@pytest.mark.parametrize("Lx,Ly", [(3, 2), (3, 3)])
def test_mixed_estimators_average_to_enumerated_matrices(Lx, Ly):
    """<o_ab>_{P^a} and <e_ab>_{P^a}, averaged exactly over all 2^N
    configurations, equal psi^a.psi^b / Z_a and psi^a.H psi^b / Z_a with H
    from Pauli Kronecker products (two independent routes)."""
    N = Lx * Ly
    pi, st = three_states(N, 2, 3, 50 + N)
    S = rtt.all_configs(N)
    bonds = tfim.bonds(Lx, Ly)
    Ht, St, Z = dual.exact_matrices(st, pi, Lx, Ly, J, H_FIELD)
    for a in range(3):
        pa = dual.state_amplitudes(st[a], pi, S)
        P = pa * pa / (pa @ pa)
        for b in range(3):
            o, e = dual.mixed_estimators(st[a], st[b], pi, S, bonds, J, H_FIELD)
            assert P @ o == pytest.approx(St[a, b], rel=1e-10, abs=1e-12)
            assert P @ e == pytest.approx(Ht[a, b], rel=1e-10, abs=1e-10)


def test_symmetry_and_generalised_eigenvalues():
    """Z_a H~_ab = Z_b H~_ba and Z_a S~_ab = Z_b S~_ba (H and S symmetric);
    H~ c = lambda S~ c has the eigenvalues of the symmetric-definite problem
    H c = lambda S c (scipy eigh), bounded below by the exact ground energy."""
    Lx, Ly = 3, 3
    N = Lx * Ly
    pi, st = three_states(N, 2, 4, 60)
    Ht, St, Z = dual.exact_matrices(st, pi, Lx, Ly, J, H_FIELD)
    Hs, Ss = Z[:, None] * Ht, Z[:, None] * St
    assert np.allclose(Hs, Hs.T, rtol=1e-10)
    assert np.allclose(Ss, Ss.T, rtol=1e-10)
    lam_sym = scipy.linalg.eigh(Hs, Ss, eigvals_only=True)[0]
    lam = dual.lowest_generalised_eigenvalue(Ht, St)
    assert lam == pytest.approx(lam_sym, rel=1e-9)
    e0, _ = tfim.ground_state(Lx, Ly, J, H_FIELD)
    assert lam >= e0 - 1e-9
    # the combination is no worse than any single state
    assert lam <= min(Ht[a, a] for a in range(3)) + 1e-9


def test_span_containing_the_ground_state_gives_e0():
    """psi^1 = exact ground state (TT-SVD, R = 1), psi^2 random: the lowest
    generalised eigenvalue is E0."""
    Lx, Ly = 3, 3
    N = Lx * Ly
    e0, v = tfim.ground_state(Lx, Ly, J, H_FIELD)
    gs = tt.tt_svd(v, N)
    rnd = wl.gaussian_cores(wl.bonds_of(gs), 71)
    pi = np.arange(N, dtype=np.int32)
    Ht, St, _ = dual.exact_matrices([rnd, gs], pi, Lx, Ly, J, H_FIELD)
    assert dual.lowest_generalised_eigenvalue(Ht, St) == pytest.approx(e0, rel=1e-9)
    assert Ht[1, 1] == pytest.approx(e0, rel=1e-9)


def test_gram_schmidt_removes_the_overlap():
    """psi'^2 = psi^2 - S~_12 psi^1 has S~'_12 = 0, and psi'^3 (against both
    predecessors, exact S~) has zero overlap estimator with psi^1."""
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi, st = three_states(N, 2, 3, 80)
    st = [st[0], st[2], wl.gaussian_cores(wl.open_bonds(2 * N, 3), 83)]
    Ht, St, _ = dual.exact_matrices(st, pi, Lx, Ly, J, H_FIELD)
    C = dual.gram_schmidt_coefficients(St)
    new2 = ([st[1], st[0]], np.array([C[1, 1], C[1, 0]]))
    _, St2, _ = dual.exact_matrices([st[0], new2], pi, Lx, Ly, J, H_FIELD)
    assert abs(St2[0, 1]) < 1e-12
    assert C[2, 0] == -St[0, 2] and C[2, 1] == -St[1, 2]


def test_sampled_estimates_within_three_sigma():
    """Metropolis chains on P^a (the oracle's own sampler) give H~_ab and
    S~_ab within 3 sigma of enumeration."""
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi, st = three_states(N, 2, 3, 90)
    Ht, St, _ = dual.exact_matrices(st[:2], pi, Lx, Ly, J, H_FIELD)
    bonds = tfim.bonds(Lx, Ly)
    a, b = 0, 1
    s = wl.random_spins(200, N, 91)
    s, _, _ = mcmc.metropolis(st[a], pi, s, seed=92, n_sweeps=20)
    os_, es = [], []
    for t in range(60):
        s, _, _ = mcmc.metropolis(st[a], pi, s, seed=92, sweep0=20 + t, n_sweeps=1)
        o, e = dual.mixed_estimators(st[a], st[b], pi, s, bonds, J, H_FIELD)
        os_.append(o.mean())
        es.append(e.mean())
    for series, exact in ((np.array(os_), St[a, b]), (np.array(es), Ht[a, b])):
        sig = series.std(ddof=1) / np.sqrt(len(series)) * 2.0   # generous tau
        assert abs(series.mean() - exact) < 3 * sig + 1e-12


def test_z_operator_on_one_replica():
    """Negating slice 1 of one replica core of spin i gives (-1)^{s_i} psi
    (closed form over every configuration), whichever replica is used."""
    N, R = 6, 2
    pi = wl.path_site_plus_perms(N, R, 95)
    cores = wl.gaussian_cores(wl.open_bonds(N * R, 3), 96)
    S = rtt.all_configs(N)
    psi = rtt.amplitudes(cores, pi, S)
    for i in (0, 3, 5):
        z = rtt.amplitudes(dual.apply_z(cores, pi, i), pi, S)
        assert np.allclose(z, (1 - 2 * S[:, i].astype(np.int64)) * psi, rtol=1e-12, atol=0)


def test_z_only_shortcut_equals_enumeration():
    """States Z_i Z_j psi: every row of H~ and S~ is the average over
    P = |psi|^2 / Z of the single chain's estimators, mapped by
    z_only_matrices (exact enumeration on both sides)."""
    Lx, Ly = 3, 2
    N = Lx * Ly
    pi = wl.path_site_plus_perms(N, 2, 97)
    psi = wl.gaussian_cores(wl.open_bonds(2 * N, 3), 98)
    states = [psi, dual.apply_z(dual.apply_z(psi, pi, 0), pi, 1), dual.apply_z(psi, pi, 4)]
    Ht, St, _ = dual.exact_matrices(states, pi, Lx, Ly, J, H_FIELD)
    S = rtt.all_configs(N)
    p = rtt.amplitudes(psi, pi, S)
    P = p * p / (p @ p)
    rows = [dual.mixed_estimators(psi, st, pi, S, tfim.bonds(Lx, Ly), J, H_FIELD) for st in states]
    h, s = dual.z_only_matrices([r[0] for r in rows], [r[1] for r in rows])
    assert np.allclose(h @ P, Ht, rtol=1e-10, atol=1e-10)
    assert np.allclose(s @ P, St, rtol=1e-10, atol=1e-12)
