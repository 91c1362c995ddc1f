"""The paper's optimisation routes on the H+V+D+D' path (Sec. 4) with GPU
sampling: the replica-space power method with H-bar_HV (host rounding,
rtt_pauli_apply) gives a train whose GPU VMC energy agrees with exact
enumeration within 3 sigma; one physical-space step with the operators
I, O_X, O_ZZ,HV, O_ZZ,DD' (Sec. 4.3) gives a lowest generalised eigenvalue
from GPU-sampled H~, S~ that agrees with the one from enumerated matrices
of the same states, and a compressed combination no worse than the start."""
import numpy as np
import pytest
import torch

from helpers import split_cores
from oracle import dual, rtt as orc, tfim
from paper_2604_22718_amd import lattice

pytestmark = pytest.mark.gpu
J, HX = 1.0, 3.0
Lx = Ly = 4


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def quantised(R, pi, cores):
    """The cores exactly as the FP32 library holds them."""
    psi = R.RTT.create(Lx * Ly, pi, cores, "f32")
    bond = np.array([1] + [c.shape[2] for c in cores])
    q = split_cores(psi.core_values(bond, 0), bond)
    psi.close()
    return q


@pytest.fixture(scope="module")
def projected(R):
    from paper_2604_22718_amd import pipeline
    pi, phi = pipeline.power_method(Lx, Ly, "HV", HX, 0.1, 30, chi=2, chi_sum=8, periodic=False)
    return pi, phi


def test_power_method_energy_on_the_gpu(R, projected):
    from paper_2604_22718_amd import pipeline
    pi, phi = projected
    N = Lx * Ly
    bonds = tfim.bonds(Lx, Ly, periodic=False)
    exact = orc.exact_energy(quantised(R, pi, phi), pi, N, bonds, J, HX)
    e0, _ = tfim.ground_state(Lx, Ly, J, HX, periodic=False)
    assert e0 - 1e-9 <= exact < -HX * N        # below the constant start
    assert (exact - e0) / abs(e0) < 5e-3
    psi = R.RTT.create(N, pi, phi, "f32")
    ham = R.TFIM(Lx, Ly, J, HX, periodic=False)
    r = pipeline.vmc_energy(psi, ham, walkers=2048, burn=20, sweeps=200, seed=810)
    print(f"HV power method: GPU {r['mean'] / N:.5f} +- {r['sigma'] / N:.5f}  exact {exact / N:.5f}  "
          f"E0 {e0 / N:.5f}  V-score {r['v_score']:.4f}")
    assert abs(r["mean"] - exact) < 3 * r["sigma"]


def test_physical_space_step(R, projected):
    from paper_2604_22718_amd import pipeline
    pi, phi = projected
    N = Lx * Ly
    ham = R.TFIM(Lx, Ly, J, HX, periodic=False)
    ops = ["I", "X", "ZZ_HV", "ZZ_DD'"]
    # the Z-operator states need a long burn-in (separated modes of |psi^a|^2)
    new, info = pipeline.physical_space_step(pi, phi, Lx, Ly, ops, 2, ham, walkers=2048, burn=400, sweeps=200,
                                             seed=820, chi_sum=8, periodic=False)
    q = [quantised(R, pi, t) for t in info["trains"]]
    Ht_ex, St_ex, _ = dual.exact_matrices(q, pi, Lx, Ly, J, HX, periodic=False)
    lam_ex = dual.lowest_generalised_eigenvalue(Ht_ex, St_ex)
    Ht, St = np.array(info["H_tilde"]), np.array(info["S_tilde"])
    sH, sS = np.array(info["sigma_H"]), np.array(info["sigma_S"])
    print(np.round(Ht - Ht_ex, 4), np.round(sH, 4), np.round(St - St_ex, 5), np.round(sS, 5), sep='\n')
    # every matrix element within 4 sigma (16 elements each) plus the FP32 evaluation tolerance
    assert np.all(np.abs(Ht - Ht_ex) < 4 * sH + 1e-5 * (1 + np.abs(Ht_ex)))
    assert np.all(np.abs(St - St_ex) < 4 * sS + 1e-5 * (1 + np.abs(St_ex)))
    bonds = tfim.bonds(Lx, Ly, periodic=False)
    e_start = orc.exact_energy(quantised(R, pi, phi), pi, N, bonds, J, HX)
    e_new = orc.exact_energy(quantised(R, pi, new), pi, N, bonds, J, HX)
    print(f"physical step: lambda GPU {info['lambda'] / N:.5f} exact {lam_ex / N:.5f}; "
          f"E start {e_start / N:.5f} after {e_new / N:.5f}")
    assert lam_ex <= e_start + 1e-9                  # the span contains the start
    assert abs(info["lambda"] - lam_ex) < 2e-3 * abs(lam_ex)
    assert e_new < e_start + 1e-3 * abs(e_start)
    assert max(c.shape[2] for c in new) <= 2


def test_single_chain_matrices_for_z_operators(R, projected):
    """Operators made of Z's (I, O_ZZ,HV, O_ZZ,DD'): H and S from one chain
    on the first state agree with enumeration (up to the common factor
    <psi^0|psi^0>) within 4 sigma, and the lowest eigenvalue with the one
    of the enumerated matrices."""
    from paper_2604_22718_amd import pipeline
    pi, phi = projected
    N = Lx * Ly
    ham = R.TFIM(Lx, Ly, J, HX, periodic=False)
    new, info = pipeline.physical_space_step(pi, phi, Lx, Ly, ["I", "ZZ_HV", "ZZ_DD'"], 2, ham, walkers=2048,
                                             burn=50, sweeps=200, seed=830, chi_sum=8, periodic=False,
                                             sampling="single")
    q = [quantised(R, pi, t) for t in info["trains"]]
    S_all = orc.all_configs(N)
    amps = [orc.amplitudes(t, pi, S_all) for t in q]
    H = tfim.sparse_hamiltonian(Lx, Ly, J, HX, periodic=False)
    z0 = amps[0] @ amps[0]
    S_ex = np.array([[a @ b for b in amps] for a in amps]) / z0
    H_ex = np.array([[a @ (H @ b) for b in amps] for a in amps]) / z0
    Hs, Ss = np.array(info["H_tilde"]), np.array(info["S_tilde"])
    sH, sS = np.array(info["sigma_H"]), np.array(info["sigma_S"])
    assert np.all(np.abs(Ss - S_ex) < 4 * sS + 1e-5 * (1 + np.abs(S_ex)))
    assert np.all(np.abs(Hs - H_ex) < 4 * sH + 1e-5 * (1 + np.abs(H_ex)))
    lam_ex = dual.lowest_generalised_eigenvalue(H_ex, S_ex)
    print(f"single chain: lambda {info['lambda'] / N:.5f} exact {lam_ex / N:.5f}")
    assert abs(info["lambda"] - lam_ex) < 2e-3 * abs(lam_ex)
