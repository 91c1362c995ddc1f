"""The paper's two optimisation routes on the four-part path, driven through
the library: the replica-space power method (Sec. 3.1 with the replica
Hamiltonians of Sec. 4.2) run by rtt_pauli_apply on the host, energies by
GPU Markov chains (Sec. 3.3), and one physical-space step (Sec. 3.3 dual
Monte Carlo with the operators of Sec. 4.3): states O-bar_a phi compressed,
re-orthogonalised against the first, the matrices H~ and S~ from one GPU
chain per state, the lowest generalised eigenpair, and the combination
compressed back into one train.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice
from . import rtt as R
from . import workloads as wl


def normalise(cores):
    """Scale a train so that its last core has unit Frobenius norm (after a
    left-to-right rounding the norm of the whole train sits there).  The
    norm is taken of the core divided by its largest entry: the constant
    train on 1600 positions has norm 2^800, whose square overflows."""
    out = [np.array(c, copy=True) for c in cores]
    m = np.abs(out[-1]).max()
    out[-1] /= m * np.linalg.norm(out[-1] / m)
    return out


def constant_train(L):
    """phi^(0) = 1: every replica index has amplitude one (bond 1)."""
    return [np.ones((2, 1, 1)) for _ in range(L)]


def power_method(Lx, Ly, kind, h, tau, steps, chi, chi_sum=None, alpha=0.0, J=1.0, periodic=False, phi=None,
                 callback=None):
    """phi^(P) = (1 - tau H-bar)^P phi^(0) with a compression after every
    step; H-bar is H-bar_H, H-bar_HV or H-bar_HVDD' on the H+V+D+D' path.
    Returns (pi, cores)."""
    pi = lattice.path(Lx, Ly)
    coeffs, ops = lattice.replica_hamiltonian(Lx, Ly, kind, h, alpha=alpha, J=J, periodic=periodic)
    phi = constant_train(len(pi)) if phi is None else phi
    for p in range(steps):
        phi = normalise(R.rtt_pauli_apply(phi, coeffs, ops, 1.0, -tau, chi, chi_sum))
        if callback is not None:
            callback(p, phi)
    return pi, phi


def _walkers(W, N, seed):
    return R.spins_to_device(wl.pack_spins(wl.random_spins(W, N, seed)))


def _blocked_sigma(series, blocks=20):
    """Error bar of the mean of a correlated series by block averages."""
    x = np.asarray(series, dtype=np.float64)
    nb = min(blocks, len(x))
    if nb < 2:
        return float("nan")
    m = np.array([b.mean() for b in np.array_split(x, nb)])
    return float(m.std(ddof=1) / np.sqrt(nb))


def vmc_energy(psi, ham, walkers, burn, sweeps, seed, rng_stream=0):
    """<H> under |psi|^2 from one GPU chain of ``walkers`` walkers: burn-in,
    then E_loc after every sweep.  Returns mean, sigma (block averages over
    sweeps), variance of E_loc and the V-score N var / E^2."""
    N = psi.N
    spins = _walkers(walkers, N, seed)
    psi.sweep(spins, seed=seed, rng_stream=rng_stream, sweep0=0, n_sweeps=burn)
    # per sweep the library's compensated sums: sum E_loc, sum E_loc^2, count
    sums = torch.empty((sweeps, 3), dtype=torch.float64, device=spins.device)
    for t in range(sweeps):
        psi.sweep(spins, seed=seed, rng_stream=rng_stream, sweep0=burn + t, n_sweeps=1)
        R.rtt_energy_reduce(psi.local_energy(spins, ham), sums[t])
    S = sums.cpu().numpy()
    means, squares = S[:, 0] / S[:, 2], S[:, 1] / S[:, 2]
    mean = float(means.mean())
    var = float(squares.mean() - mean * mean)
    return {"mean": mean, "sigma": _blocked_sigma(means), "var": var, "v_score": N * var / (mean * mean)}


def dual_matrices(states, ham, walkers, burn, sweeps, seed, blocks=10, rows=None):
    """H~_ab and S~_ab (Sec. 3.3): for each a, one GPU chain on |psi^a|^2 and
    the overlap and mixed-energy estimators against every state after each
    sweep.  Returns H~, S~ and their block-average error bars (only the
    listed ``rows`` are sampled when given; the others stay zero).

    States made by Z operators (O_ZZ phi) change sign across a surface of
    configurations, and |psi^a|^2 then has separated modes that single-spin
    Metropolis crosses slowly: such chains need a burn-in of hundreds of
    sweeps (on a 4x4 lattice, 20 sweeps leave a bias of 0.6% in H~_aa)."""
    M, N = len(states), states[0].N
    Ht, St = np.zeros((M, M)), np.zeros((M, M))
    sH, sS = np.zeros((M, M)), np.zeros((M, M))
    for a in (range(M) if rows is None else rows):
        spins = _walkers(walkers, N, seed + a)
        la = torch.empty(walkers, dtype=torch.float64, device=spins.device)
        sg = torch.empty(walkers, dtype=torch.int8, device=spins.device)
        states[a].sweep(spins, seed=seed, rng_stream=a, sweep0=0, n_sweeps=burn, logabs=la, sign=sg)
        # per sweep the library's compensated row sums of both estimators
        rows = torch.empty((sweeps, 2, M, 1, 2), dtype=torch.float64, device=spins.device)
        for t in range(sweeps):
            states[a].sweep(spins, seed=seed, rng_stream=a, sweep0=burn + t, n_sweeps=1, logabs=la, sign=sg)
            ratio, mixed, st = R.mixed_estimators(states, ham, spins, la, sg)
            R.rtt_pair_sums(ratio, None, rows[t, 0])
            R.rtt_pair_sums(mixed, None, rows[t, 1])
        X = rows.cpu().numpy()
        O = X[:, 0, :, 0, 0] / X[:, 0, :, 0, 1]
        E = X[:, 1, :, 0, 0] / X[:, 1, :, 0, 1]
        St[a], Ht[a] = O.mean(axis=0), E.mean(axis=0)
        sS[a] = [_blocked_sigma(O[:, b], blocks) for b in range(M)]
        sH[a] = [_blocked_sigma(E[:, b], blocks) for b in range(M)]
    return Ht, St, sH, sS


def single_chain_matrices(states, ham, walkers, burn, sweeps, seed, blocks=10):
    """H and S of a list of states up to one common factor from a single
    chain on |psi^0|^2 (importance sampling): S_ab = <r_a r_b>, H_ab =
    <r_a m_b>, with r_b = psi^b/psi^0 and m_b = sum_t H_st psi^b(t)/psi^0(s).
    This is the single-simulation route the paper notes for operators made
    of Z's (Sec. 4.1.3): psi^a = d_a psi^0 with d_a diagonal, so no chain
    has to sample |psi^a|^2; it holds for any states whose support lies in
    that of psi^0.  Returns H, S and their block-average error bars."""
    M, N = len(states), states[0].N
    spins = _walkers(walkers, N, seed)
    la = torch.empty(walkers, dtype=torch.float64, device=spins.device)
    sg = torch.empty(walkers, dtype=torch.int8, device=spins.device)
    states[0].sweep(spins, seed=seed, rng_stream=0, sweep0=0, n_sweeps=burn, logabs=la, sign=sg)
    # per sweep the library's compensated sums of r_a r_b and r_a m_b
    sums = torch.empty((sweeps, 2, M, M, 2), dtype=torch.float64, device=spins.device)
    for t in range(sweeps):
        states[0].sweep(spins, seed=seed, rng_stream=0, sweep0=burn + t, n_sweeps=1, logabs=la, sign=sg)
        ratio, mixed, st = R.mixed_estimators(states, ham, spins, la, sg)
        R.rtt_pair_sums(ratio, ratio, sums[t, 0])
        R.rtt_pair_sums(ratio, mixed, sums[t, 1])
    X = sums.cpu().numpy()
    Sx = X[:, 0, :, :, 0] / X[:, 0, :, :, 1]   # (sweeps, M, M)
    Hx = X[:, 1, :, :, 0] / X[:, 1, :, :, 1]
    S, H = Sx.mean(axis=0), Hx.mean(axis=0)
    sS = np.array([[_blocked_sigma(Sx[:, a, b], blocks) for b in range(M)] for a in range(M)])
    sH = np.array([[_blocked_sigma(Hx[:, a, b], blocks) for b in range(M)] for a in range(M)])
    return H, S, sH, sS


def lowest_eigenpair(Ht, St):
    """Lowest real eigenvalue of H~ c = lambda S~ c and its vector, scaled so
    that c^T S~ c = 1 (with c[0] >= 0)."""
    w, v = np.linalg.eig(np.linalg.solve(St, Ht))
    ok = np.isfinite(w) & (np.abs(w.imag) <= 1e-9 * np.maximum(1.0, np.abs(w.real)))
    if not ok.any():
        raise RuntimeError("no real eigenvalue in the generalised problem")
    i = np.flatnonzero(ok)[np.argmin(w.real[ok])]
    c = v[:, i].real
    n = c @ St @ c
    c = c / np.sqrt(abs(n)) if n != 0 else c
    return float(w.real[i]), (c if c[0] >= 0 else -c)


def physical_space_step(pi, phi, Lx, Ly, operators, chi, ham, walkers, burn, sweeps, seed, chi_sum=None,
                        periodic=False, orthogonalise=True, dtype="f32", sampling="dual", chi_state=None):
    """One physical-space optimisation step (Sec. 3.3, Sec. 4.3): states
    psi^a = C O-bar_a phi for the named operators (each compressed to
    chi_state, by default chi),
    re-orthogonalised against psi^1 with a GPU overlap estimate, dual Monte
    Carlo H~ and S~ (or, with sampling="single", H and S from one chain on
    the first state), the lowest generalised eigenpair, and the combination
    sum_a c_a psi^a compressed to chi.  Returns (new cores, info)."""
    if sampling not in ("dual", "single"):
        raise ValueError(f"sampling must be 'dual' or 'single', not {sampling!r}")
    N = Lx * Ly
    trains = []
    for name in operators:
        if name == "I":
            trains.append(normalise(phi))
            continue
        c, o = lattice.operator(Lx, Ly, name, periodic)
        cs = chi if chi_state is None else chi_state
        trains.append(normalise(R.rtt_pauli_apply(phi, c, o, 0.0, 1.0, cs, max(cs, chi_sum or cs))))
    gs = np.zeros(len(trains))
    if orthogonalise and len(trains) > 1:
        first = R.RTT.create(N, pi, trains[0], dtype)
        others = [R.RTT.create(N, pi, t, dtype) for t in trains[1:]]
        _, St, _, _ = dual_matrices([first] + others, ham, walkers, burn, sweeps, seed + 1000, rows=[0])
        for m in range(1, len(trains)):
            gs[m] = St[0, m]
            trains[m] = normalise(R.rtt_tt_combine([trains[m], trains[0]], [1.0, -gs[m]],
                                                   chi if chi_state is None else chi_state))
        for x in [first] + others:
            x.close()
    states = [R.RTT.create(N, pi, t, dtype) for t in trains]
    if sampling == "single":
        Ht, St, sH, sS = single_chain_matrices(states, ham, walkers, burn, sweeps, seed)
    else:
        Ht, St, sH, sS = dual_matrices(states, ham, walkers, burn, sweeps, seed)
    lam, c = lowest_eigenpair(Ht, St)
    new = normalise(R.rtt_tt_combine(trains, c, chi))
    for x in states:
        x.close()
    return new, {"lambda": lam, "coeffs": c.tolist(), "sampling": sampling,
                 "H_tilde": Ht.tolist(), "S_tilde": St.tolist(), "sigma_H": sH.tolist(), "sigma_S": sS.tolist(),
                 "gram_schmidt": gs.tolist(), "trains": trains}
