"""Single-spin-flip Metropolis sampling of P_s = |psi_s|^2 / Z (paper Sec. 3.3,
where the observables are averages over P sampled by Markov-chain Monte Carlo,
"e.g. the Metropolis algorithm").  Test infrastructure only.

The paper does not fix the proposal scheme; the reading used here:
  * one sweep proposes every spin once, in order of the spin's first train
    position (spins read by no position come last, in index order);
  * the proposal for spin j flips s_j; the Metropolis ratio is
    |psi(s')|^2 / |psi(s)|^2 = r_j^2 with r_j the flip ratio;
  * the uniform u for walker w, absolute sweep t and spin j is word 0 of
    Philox4x64-10 with key (seed, stream) and counter (w, t, j, 0), top 53
    bits; the move is accepted iff u < r_j^2.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .rtt import amplitudes, flip


def proposal_order(pi, N: int) -> list[int]:
    first = {}
    for k, j in enumerate(np.asarray(pi)):
        first.setdefault(int(j), k)
    seen = sorted(first, key=lambda j: first[j])
    rest = [j for j in range(N) if j not in first]
    return seen + rest


def uniforms(seed, stream, walker_ids, sweep, spin) -> np.ndarray:
    return np.array([philox.uniform(seed, stream, int(w), int(sweep), int(spin))
                     for w in walker_ids])


def metropolis(cores, pi, spins, seed: int, stream: int = 0, sweep0: int = 0,
               n_sweeps: int = 1, walker_ids=None, record: bool = False, amp_fn=None):
    """Run ``n_sweeps`` sweeps from ``spins`` (W, N).  Returns the final spins,
    per-walker accept counts and, with ``record``, per-decision margins
    u - r^2 (shape (n_sweeps, N, W)) for near-tie detection.  ``amp_fn``
    replaces the single-train amplitude (e.g. a linear combination)."""
    s = np.array(spins, dtype=np.uint8, copy=True)
    W, N = s.shape
    wid = np.arange(W) if walker_ids is None else np.asarray(walker_ids)
    order = proposal_order(pi, N)
    amp = amp_fn or (lambda S: amplitudes(cores, pi, S))
    accepts = np.zeros(W, dtype=np.int64)
    margins = np.zeros((n_sweeps, N, W)) if record else None
    for t in range(n_sweeps):
        sweep = sweep0 + t
        for qi, j in enumerate(order):
            psi = amp(s)
            psi_new = amp(flip(s, j))
            r = psi_new / psi
            u = uniforms(seed, stream, wid, sweep, j)
            acc = u < r * r
            s[acc, j] ^= 1
            accepts += acc
            if record:
                margins[t, qi] = u - r * r
    return s, accepts, margins


def energy_series(cores, pi, spins, seed, stream, n_burn, n_meas, bonds, J, h,
                  walker_ids=None, local_energy_fn=None):
    """Burn-in, then one local-energy measurement after every sweep.
    Returns the final spins and the (n_meas, W) series of E_loc."""
    from .rtt import local_energy
    le = local_energy_fn or (lambda S: local_energy(cores, pi, S, bonds, J, h))
    s, _, _ = metropolis(cores, pi, spins, seed, stream, 0, n_burn, walker_ids)
    series = []
    for t in range(n_meas):
        s, _, _ = metropolis(cores, pi, s, seed, stream, n_burn + t, 1, walker_ids)
        series.append(le(s))
    return s, np.array(series)


def transition_matrix(cores, pi, N: int) -> np.ndarray:
    """Full one-sweep transition matrix over all 2^N states (tiny N), for the
    stationarity check.  Each single-spin step is the Metropolis kernel
    T_j(s -> s^j) = min(1, r_j^2); a sweep is their product in proposal order."""
    from .rtt import all_configs
    S = all_configs(N)
    n = 2 ** N
    psi = amplitudes(cores, pi, S)
    T = np.eye(n)
    for j in proposal_order(pi, N):
        Tj = np.zeros((n, n))
        psi_f = amplitudes(cores, pi, flip(S, j))
        a = np.minimum(1.0, (psi_f / psi) ** 2)
        idx = np.arange(n)
        jdx = idx ^ (1 << j)
        Tj[idx, jdx] = a
        Tj[idx, idx] = 1.0 - a
        T = T @ Tj
    return T
