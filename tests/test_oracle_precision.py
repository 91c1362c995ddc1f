"""The oracle's own floating-point error, bounded by a 50-digit evaluation
of the same products (mpmath), and the constant replica train giving
psi = 1 on every configuration (the power method's starting state)."""
import mpmath
import numpy as np

from oracle import replica, rtt as orc
from paper_2604_22718_amd import workloads as wl


def mp_amplitude(cores, pi, s):
    v = [mpmath.mpf(1)]
    for k, A in enumerate(cores):
        sl = A[int(s[pi[k]])]
        v = [mpmath.fsum(v[i] * mpmath.mpf(float(sl[i, j])) for i in range(len(v))) for j in range(sl.shape[1])]
    return v[0]


def test_fp64_oracle_error_is_bounded_by_its_condition_number():
    mpmath.mp.dps = 50
    N = 6
    pi = wl.path_site_plus_perms(N, 2, 960)
    cores = wl.gaussian_cores(wl.open_bonds(2 * N, 4), 961)
    bits = wl.random_spins(12, N, 962)
    psi = orc.amplitudes(cores, pi, bits)
    kap = orc.condition_numbers(cores, pi, bits)
    r = orc.flip_ratios(cores, pi, bits)
    for w in range(len(bits)):
        exact = mp_amplitude(cores, pi, bits[w])
        rel = abs((mpmath.mpf(float(psi[w])) - exact) / exact)
        assert rel <= 64 * 2.0 ** -52 * kap[w] * len(pi), (w, float(rel), kap[w])
        for j in (0, 3, 5):
            s2 = bits[w].copy()
            s2[j] ^= 1
            exact_r = mp_amplitude(cores, pi, s2) / exact
            assert abs(float(r[w, j]) - float(exact_r)) <= 1e-10 * max(1.0, abs(float(exact_r)))


def test_constant_train_is_one_everywhere():
    pi = wl.path_site_plus_perms(5, 3, 963)
    S = orc.all_configs(5)
    assert np.all(orc.amplitudes(replica.constant_train(len(pi)), pi, S) == 1.0)
