"""Imaginary-time power method in replica space (paper Sec. 3.1 with the
operators of Sec. 2.2.3) feeding the GPU sampler: the library's host step
phi <- phi - tau H phi with TT rounding produces an uneven-bond train that
is loaded on the GPU; its amplitudes and flip ratios match the oracle on
the library's quantised cores, and its MCMC energy agrees with exact
enumeration within 3 sigma and lies below the starting state's."""
import numpy as np
import pytest
import torch

from helpers import check_ratios, device_cores
from oracle import replica, rtt as orc, stats, tfim
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu
J, HF = 1.0, 3.04


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def project(R, N, Lx, Ly, pi, c, steps, tau, chi_max):
    for _ in range(steps):
        c = R.rtt_tfim_power_step(N, pi, c, Lx, Ly, J, HF, tau, chi_max)
        c = replica.scale(c, 1.0 / np.linalg.norm(c[-1]))   # left-orthonormal: norm in the last core
    return c


def test_power_method_then_gpu_sampling(R):
    Lx, Ly = 4, 4
    N = Lx * Ly
    pi = wl.path_site_plus_perms(N, 2, 500)
    c0 = wl.gaussian_cores(wl.open_bonds(2 * N, 4), 501)
    c = project(R, N, Lx, Ly, pi, c0, 30, 0.03, 8)
    bond = np.array([1] + [x.shape[2] for x in c])
    assert bond.max() <= 8 and len(set(bond[1:-1].tolist())) > 1   # uneven bonds after rounding
    psi = R.RTT.create(N, pi, c, "f32")
    qc = device_cores(psi, bond)
    bonds = tfim.bonds(Lx, Ly)
    # parity of the evaluation on the projected train
    bits = wl.random_spins(257, N, 502)
    out = psi.evaluate(R.spins_to_device(wl.pack_spins(bits)), R.TFIM(Lx, Ly, J, HF))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.all(out["status"] == 0)
    kap = orc.flip_condition_numbers(qc, pi, bits)
    rep = check_ratios(out["logratio"], out["rsign"], orc.flip_ratios(qc, pi, bits), kap, 1e-5)
    assert rep["n_bad"] == 0 and rep["n_sign_bad"] == 0, rep
    # energy from the GPU chain against enumeration
    exact = orc.exact_energy(qc, pi, N, bonds, J, HF)
    e_start = orc.exact_energy(c0, pi, N, bonds, J, HF)
    e0, _ = tfim.ground_state(Lx, Ly, J, HF)
    assert exact < e_start and exact >= e0 - 1e-9
    ham = R.TFIM(Lx, Ly, J, HF)
    spins = R.spins_to_device(wl.pack_spins(wl.random_spins(1024, N, 503)))
    psi.sweep(spins, seed=504, sweep0=0, n_sweeps=20)
    series = []
    for t in range(100):
        psi.sweep(spins, seed=504, sweep0=20 + t, n_sweeps=1)
        series.append(psi.local_energy(spins, ham))
    E = torch.stack(series).cpu().numpy()
    mean, sigma, tau, _ = stats.energy_estimate(E)
    print(f"power method: E_start {e_start:.5f}  exact {exact:.5f}  GPU {mean:.5f} +- {sigma:.5f}  E0 {e0:.5f}")
    assert abs(mean - exact) < 3 * sigma
