"""Pins of the learned-proposal oracle: torch's conv2d (circular padding) and
autograd, central finite differences, normalisation of q, and brute-force
stationarity of the learned-proposal Metropolis-Hastings kernel."""
import math

import numpy as np
import pytest
import torch

from oracle import net, rtt
from paper_2604_22718_amd import workloads as wl


def torch_forward(params, spins, Lx, Ly):
    P = {k: torch.tensor(v) for k, v in net.unflatten(params).items()}
    z = torch.tensor(1.0 - 2.0 * np.asarray(spins, dtype=np.float64)).reshape(-1, 1, Ly, Lx)
    F = torch.nn.functional

    def conv(x, W, b):
        return F.conv2d(F.pad(x, (1, 1, 1, 1), mode="circular"), W, b)

    h = F.silu(conv(z, P["W1"], P["b1"]))
    h = F.silu(conv(h, P["W2"], P["b2"]))
    h = F.silu(conv(h, P["W3"], P["b3"]))
    o = F.conv2d(h, P["Wh"][:, :, None, None], P["bh"])
    return o.reshape(o.shape[0], 9, Ly * Lx)


def test_param_count():
    assert net.N_PARAMS == 19113


def test_forward_matches_torch_conv2d():
    Lx, Ly = 5, 4
    p = net.init_params(3) + 0.05 * np.random.default_rng(1).standard_normal(net.N_PARAMS)
    s = wl.random_spins(6, Lx * Ly, 4)
    o = net.forward(p, s, Lx, Ly)
    ref = torch_forward(p, s, Lx, Ly).numpy()
    assert np.allclose(o, ref, rtol=1e-12, atol=1e-12)


def test_reinforce_gradient_matches_autograd_and_differences():
    Lx, Ly = 4, 3
    p = net.init_params(5) + 0.1 * np.random.default_rng(2).standard_normal(net.N_PARAMS)
    s = wl.random_spins(3, Lx * Ly, 6)
    moves = [(1, 3), (7, 1), (11, 8)]
    coef = np.array([0.7, -1.2, 0.4])
    g = net.reinforce_grad(p, s, moves, coef, Lx, Ly)
    # autograd through the torch forward
    pt = torch.tensor(p, requires_grad=True)
    parts, off = {}, 0
    for name, shp in net.SHAPES:
        n = int(np.prod(shp))
        parts[name] = pt[off:off + n].reshape(shp)
        off += n
    F = torch.nn.functional
    z = torch.tensor(1.0 - 2.0 * s.astype(np.float64)).reshape(-1, 1, Ly, Lx)
    conv = lambda x, W, b: F.conv2d(F.pad(x, (1, 1, 1, 1), mode="circular"), W, b)
    h = F.silu(conv(z, parts["W1"], parts["b1"]))
    h = F.silu(conv(h, parts["W2"], parts["b2"]))
    h = F.silu(conv(h, parts["W3"], parts["b3"]))
    o = F.conv2d(h, parts["Wh"][:, :, None, None], parts["bh"]).reshape(3, 9, Lx * Ly)
    loss = 0
    for b, (c, k) in enumerate(moves):
        loss = loss + coef[b] * (torch.log_softmax(o[b, 0], 0)[c] + torch.log_softmax(o[b, 1:9, c], 0)[k - 1])
    loss.backward()
    assert np.allclose(g, pt.grad.numpy(), rtol=1e-9, atol=1e-12)
    # central differences on a few coordinates
    for i in [0, 5, 320, 400, 9568 + 12, 18900, 19112]:
        e = np.zeros_like(p); e[i] = 1e-6
        f = lambda q: float(np.sum(coef * net.log_q(q, s, moves, Lx, Ly)))
        fd = (f(p + e) - f(p - e)) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_proposal_probabilities_normalise():
    Lx, Ly = 3, 4
    p = net.init_params(7) + 0.3 * np.random.default_rng(3).standard_normal(net.N_PARAMS)
    s = wl.random_spins(1, 12, 8)
    o = net.forward(p, s, Lx, Ly)[0]
    masks = {net.flip_mask(c, k, Lx, Ly) for c in range(12) for k in range(1, 9)}
    tot = sum(net.set_prob(o, m, Lx, Ly) for m in masks)
    assert tot == pytest.approx(1.0, rel=1e-12)
    assert len(net.flip_sites(4, 8, Lx, Ly)) == len(set(net.flip_sites(4, 8, Lx, Ly))) == 8


def test_learned_mh_kernel_is_stationary():
    """3x3 lattice, R = 2 RTT: |psi|^2 is left-invariant under the full
    transition matrix of the learned-proposal MH kernel."""
    Lx = Ly = 3
    pi = wl.path_site_plus_perms(9, 2, 9)
    cores = wl.gaussian_cores(wl.open_bonds(18, 2), 10)
    p = net.init_params(11) + 0.3 * np.random.default_rng(4).standard_normal(net.N_PARAMS)
    amp = lambda S: rtt.amplitudes(cores, pi, S)
    T = net.transition_matrix(p, amp, Lx, Ly)
    pr = amp(rtt.all_configs(9)) ** 2
    pr /= pr.sum()
    assert np.allclose(T.sum(axis=1), 1.0)
    assert np.allclose(pr @ T, pr, atol=1e-13)


def test_adam_closed_form_first_step():
    p = np.array([1.0, -2.0]); g = np.array([0.5, -4.0])
    q, m, v = net.adam(p, np.zeros(2), np.zeros(2), g, 1, lr=0.1)
    # first bias-corrected step moves each coordinate by lr * sign(g)
    assert np.allclose(q, p - 0.1 * np.sign(g), atol=1e-7)


def test_shared_initial_weights_match_the_oracle_draw():
    """The benchmark draws its initial network weights from the shared input
    module; they are the same numbers the oracle's initialiser draws."""
    from paper_2604_22718_amd import workloads as wl
    for seed in (3, 33, 4004):
        assert np.array_equal(wl.net_init_params(seed), net.init_params(seed))


def test_sample_move_is_the_inverse_cdf():
    """sample_move draws the centre c and then the size k by inverse CDF: the
    first index whose cumulative probability exceeds the uniform.  Pinned on
    both sides of every cell boundary (a relative 1e-12 below a cumulative
    value stays in the cell, as far above moves to the next one) and by the
    frequencies of (c, k) under many seeded uniforms, which must follow
    p(c) p(k | c) (binomial bounds per cell and a chi-square over all cells).
    An off-by-one in c or k, the size drawn from the wrong axis or from
    unnormalised weights each fail one of these."""
    N = 6
    o = np.random.default_rng(11).standard_normal((9, N)) * 1.3
    pc = np.exp(o[0] - o[0].max()); pc /= pc.sum()
    pk = np.exp(o[1:9] - o[1:9].max(axis=0)); pk /= pk.sum(axis=0)   # (8, N)
    cum_c = np.cumsum(pc)
    lo, hi = 1.0 - 1e-12, 1.0 + 1e-12
    for i in range(N - 1):      # centre cells (size uniform 0: k = 1)
        assert net.sample_move(o, cum_c[i] * lo, 0.0) == (i, 1)
        assert net.sample_move(o, cum_c[i] * hi, 0.0) == (i + 1, 1)
    assert net.sample_move(o, 0.0, 0.0) == (0, 1)
    assert net.sample_move(o, 1.0 - 1e-12, 0.0)[0] == N - 1
    for c in range(N):          # size cells at every centre
        uc = 0.5 * (cum_c[c] + (0.0 if c == 0 else cum_c[c - 1]))
        cum_k = np.cumsum(pk[:, c])
        for k in range(1, 8):
            assert net.sample_move(o, uc, cum_k[k - 1] * lo) == (c, k)
            assert net.sample_move(o, uc, cum_k[k - 1] * hi) == (c, k + 1)
        assert net.sample_move(o, uc, 1.0 - 1e-12) == (c, 8)
    n = 60000                   # frequencies
    u = wl.generator(12).random((n, 2))
    counts = np.zeros((N, 8))
    for uc, uk in u:
        c, k = net.sample_move(o, uc, uk)
        counts[c, k - 1] += 1
    p = pc[:, None] * pk.T                                # (N, 8)
    assert np.all(np.abs(counts - n * p) <= 5 * np.sqrt(n * p * (1 - p)) + 1)
    chi2 = float(np.sum((counts - n * p) ** 2 / (n * p)))
    assert chi2 < 47 + 5 * math.sqrt(2 * 47)               # 47 degrees of freedom
