"""Host logic of the optimisation drivers (no GPU): the generalised
eigenpair against scipy's, the block-average error bar against the known
error of the mean of independent samples, train normalisation, and the
replica-space power method against the oracle's
(physical amplitudes, every step compressed the same way)."""
import numpy as np
import scipy.linalg

from oracle import paths, replica, rtt as orc
from paper_2604_22718_amd import pipeline


def test_lowest_eigenpair_matches_scipy():
    rng = np.random.default_rng(900)
    for M in (1, 2, 4, 5):
        B = rng.normal(size=(M, M))
        S = B @ B.T + M * np.eye(M)
        Hs = rng.normal(size=(M, M))
        H = Hs + Hs.T
        D = np.diag(rng.uniform(0.5, 2.0, size=M))     # un-symmetrised rows: H~ = D H, S~ = D S
        lam, c = pipeline.lowest_eigenpair(D @ H, D @ S)
        ref = scipy.linalg.eigh(H, S, eigvals_only=True)[0]
        assert abs(lam - ref) < 1e-10 * max(1.0, abs(ref))
        assert np.allclose(D @ H @ c, lam * (D @ S @ c), atol=1e-9)
        assert abs(c @ (D @ S) @ c - 1.0) < 1e-9 and c[0] >= 0


def test_blocked_sigma_of_independent_samples():
    rng = np.random.default_rng(901)
    x = rng.normal(2.0, 3.0, size=20000)
    s = pipeline._blocked_sigma(x, 20)
    assert abs(s - 3.0 / np.sqrt(len(x))) < 0.35 * 3.0 / np.sqrt(len(x))
    assert np.isnan(pipeline._blocked_sigma(x[:1], 20))


def test_normalise_keeps_the_state_direction():
    from paper_2604_22718_amd import workloads as wl
    pi = np.array([0, 1, 2, 0, 1, 2], dtype=np.int32)
    c = wl.gaussian_cores(wl.open_bonds(6, 3), 902)
    n = pipeline.normalise(c)
    S = orc.all_configs(3)
    a, b = orc.amplitudes(c, pi, S), orc.amplitudes(n, pi, S)
    assert np.isclose(np.linalg.norm(n[-1]), 1.0)
    assert np.allclose(b * (a @ b) / (b @ b), a, rtol=1e-12, atol=1e-14)


def test_power_method_matches_oracle():
    """A random start: from the constant train the singular values at the
    cut come in symmetric (degenerate) pairs, and which of two equal values
    a rounding keeps is decided by rounding error on either side."""
    from paper_2604_22718_amd import workloads as wl
    Lx, Ly, h = 3, 3, 3.0
    phi0 = wl.gaussian_cores(wl.open_bonds(4 * Lx * Ly, 2), 903)
    pi, phi = pipeline.power_method(Lx, Ly, "HVDD'", h, 0.1, 6, chi=2, chi_sum=4, alpha=0.08, periodic=False,
                                    phi=phi0)
    ref = phi0
    c, o = paths.hamiltonian(Lx, Ly, "HVDD'", h, alpha=0.08, periodic=False)
    for _ in range(6):
        ref = replica.pauli_apply(ref, c, o, 1.0, -0.1, 2, chi_sum=4)
        ref = replica.scale(ref, 1.0 / np.linalg.norm(ref[-1]))
    S = orc.all_configs(Lx * Ly)
    a, b = orc.amplitudes(phi, pi, S), orc.amplitudes(ref, pi, S)
    assert np.allclose(a, b, rtol=0, atol=1e-8 * np.abs(b).max())
