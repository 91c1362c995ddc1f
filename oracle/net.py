"""Learned multi-spin proposal: FP64 reference.  Test infrastructure only.

The paper leaves the sampler open (Sec. 3.3 samples P = |psi|^2 / Z "by
Markov chain Monte Carlo, e.g. the Metropolis algorithm"); any proposal is
valid as long as the Metropolis-Hastings ratio includes the proposal
probabilities in both directions.  Readings used here (architecture and move
from the workload definition, details chosen and pinned):

Network (19,113 parameters), input z = 1 - 2 s on the periodic Lx x Ly
lattice, one channel:
  h1 = SiLU(conv3x3(z;  W1[32,1,3,3],  b1[32]))
  h2 = SiLU(conv3x3(h1; W2[32,32,3,3], b2[32]))
  h3 = SiLU(conv3x3(h2; W3[32,32,3,3], b3[32]))
  o  = conv1x1(h3; Wh[9,32], bh[9])              (9 outputs per site)
conv3x3 is the circular cross-correlation
  out[co,y,x] = b[co] + sum_{ci,ky,kx} W[co,ci,ky,kx] in[ci,(y+ky-1)%Ly,(x+kx-1)%Lx];
SiLU(x) = x / (1 + exp(-x)).  Parameters are flattened in the order
W1, b1, W2, b2, W3, b3, Wh, bh (each row-major).

Move: centre c ~ softmax_i(o[0, i]) over sites; size k ~ softmax_k(o[k, c]),
k = 1..8; flip the first k sites of the spiral SPIRAL around c.  The proposal
probability of the flip set S is q(S|s) = sum over all (c', k') whose flip
set equals S of p(c'|s) p(k'|c', s).  Uniforms: word 0 of Philox4x64-10 under
key (seed, stream), counter (walker, step, 2^32 + i, 0), i = 0 centre,
1 size, 2 acceptance; sampling by inverse CDF (first index whose cumulative
probability exceeds u).  Accept iff u < r^2 q(S|s') / q(S|s).

Training (REINFORCE): per state s with sampled (c, k), acceptance a and
coefficient w = -(a k - baseline) / B, the loss is sum_b w_b log q(c_b,k_b|s_b)
with log q(c,k|s) = log softmax(o0)[c] + log softmax(o[1:9, c])[k-1].
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

C = 32
SPIRAL = [(0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1)]   # (dx, dy)
SHAPES = [("W1", (C, 1, 3, 3)), ("b1", (C,)), ("W2", (C, C, 3, 3)), ("b2", (C,)),
          ("W3", (C, C, 3, 3)), ("b3", (C,)), ("Wh", (9, C)), ("bh", (9,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 19113


def unflatten(p):
    out, off = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[off:off + n], dtype=np.float64).reshape(shp)
        off += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-style uniform init, seeded (numpy Philox)."""
    g = np.random.Generator(np.random.Philox(seed))
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            fan_in = int(np.prod(shp[1:]))
            lim = math.sqrt(3.0 / fan_in)
            d[name] = g.uniform(-lim, lim, size=shp)
        else:
            d[name] = np.zeros(shp)
    return flatten(d)


def silu(x):
    return x / (1.0 + np.exp(-x))


def conv3x3(x, W, b):
    """x (B, ci, Ly, Lx) -> (B, co, Ly, Lx), circular cross-correlation."""
    out = np.zeros((x.shape[0], W.shape[0], x.shape[2], x.shape[3])) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            # in[(y+ky-1) % Ly, (x+kx-1) % Lx]: roll by -(ky-1), -(kx-1)
            sh = np.roll(x, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))
            out += np.einsum("oc,bcyx->boyx", W[:, :, ky, kx], sh)
    return out


def forward(params, spins, Lx, Ly, keep=False):
    """spins (B, N) -> outputs o (B, 9, N) (and the activations with keep)."""
    P = unflatten(params)
    B = spins.shape[0]
    z = (1.0 - 2.0 * np.asarray(spins, dtype=np.float64)).reshape(B, 1, Ly, Lx)
    a1 = conv3x3(z, P["W1"], P["b1"]); h1 = silu(a1)
    a2 = conv3x3(h1, P["W2"], P["b2"]); h2 = silu(a2)
    a3 = conv3x3(h2, P["W3"], P["b3"]); h3 = silu(a3)
    o = np.einsum("kc,bcyx->bkyx", P["Wh"], h3) + P["bh"][None, :, None, None]
    o = o.reshape(B, 9, Ly * Lx)
    if keep:
        return o, (z, a1, h1, a2, h2, a3, h3)
    return o


def log_softmax(x, axis):
    m = np.max(x, axis=axis, keepdims=True)
    return x - m - np.log(np.sum(np.exp(x - m), axis=axis, keepdims=True))


def flip_sites(c, k, Lx, Ly):
    x, y = c % Lx, c // Lx
    return [((y + dy) % Ly) * Lx + (x + dx) % Lx for dx, dy in SPIRAL[:k]]


def flip_mask(c, k, Lx, Ly):
    return frozenset(flip_sites(c, k, Lx, Ly))


def set_prob(o_b, mask, Lx, Ly):
    """q(S|s) for one state's outputs o_b (9, N): sum over (c', k') with the same set."""
    N = Lx * Ly
    lc = log_softmax(o_b[0], 0)
    lk = log_softmax(o_b[1:9], 0)                 # (8, N)
    tot = 0.0
    for c in range(N):
        for k in range(1, 9):
            if flip_mask(c, k, Lx, Ly) == mask:
                tot += math.exp(lc[c] + lk[k - 1, c])
    return tot


def sample_move(o_b, u_c, u_k):
    """Inverse-CDF sampling of the centre and the size."""
    pc = np.exp(log_softmax(o_b[0], 0))
    c = int(np.searchsorted(np.cumsum(pc), u_c, side="right"))
    c = min(c, len(pc) - 1)
    pk = np.exp(log_softmax(o_b[1:9, c], 0))
    k = int(np.searchsorted(np.cumsum(pk), u_k, side="right")) + 1
    return c, min(k, 8)


def uniform(seed, stream, walker, step, i):
    x = philox.philox4x64_10((walker, step, (1 << 32) + i, 0), (seed, stream))[0]
    return (x >> 11) * (1.0 / 9007199254740992.0)


def mh_step(params, amp_fn, spins, Lx, Ly, seed, stream, step, walker_ids=None):
    """One learned-proposal MH step for every walker.  amp_fn(spins) returns
    psi for a batch.  Returns new spins, moves (c, k), acceptance probability
    a, accepted flags and the margins u - A of the decisions."""
    s = np.array(spins, dtype=np.uint8, copy=True)
    W, N = s.shape
    wid = np.arange(W) if walker_ids is None else np.asarray(walker_ids)
    o = forward(params, s, Lx, Ly)
    moves, masks = [], []
    sp = s.copy()
    for b in range(W):
        c, k = sample_move(o[b], uniform(seed, stream, wid[b], step, 0), uniform(seed, stream, wid[b], step, 1))
        moves.append((c, k))
        m = flip_mask(c, k, Lx, Ly)
        masks.append(m)
        for i in m:
            sp[b, i] ^= 1
    o2 = forward(params, sp, Lx, Ly)
    psi, psi2 = amp_fn(s), amp_fn(sp)
    acc = np.zeros(W, dtype=bool)
    a = np.zeros(W)
    margin = np.zeros(W)
    for b in range(W):
        qf = set_prob(o[b], masks[b], Lx, Ly)
        qr = set_prob(o2[b], masks[b], Lx, Ly)
        A = (psi2[b] / psi[b]) ** 2 * qr / qf
        a[b] = min(1.0, A)
        u = uniform(seed, stream, wid[b], step, 2)
        acc[b] = u < A
        margin[b] = u - A
    s[acc] = sp[acc]
    return s, moves, a, acc, margin


def transition_matrix(params, amp_fn, Lx, Ly):
    """Full transition matrix of the learned-proposal MH kernel (tiny N)."""
    from .rtt import all_configs
    N = Lx * Ly
    S = all_configs(N)
    n = 2 ** N
    psi = amp_fn(S)
    o = forward(params, S, Lx, Ly)
    lc = log_softmax(o[:, 0], 1)
    lk = log_softmax(o[:, 1:9], 1)
    T = np.zeros((n, n))
    for a in range(n):
        for c in range(N):
            for k in range(1, 9):
                m = flip_mask(c, k, Lx, Ly)
                bidx = a
                for i in m:
                    bidx ^= (1 << i)
                p = math.exp(lc[a, c] + lk[a, k - 1, c])
                qf = set_prob(o[a], m, Lx, Ly)
                qr = set_prob(o[bidx], m, Lx, Ly)
                A = min(1.0, (psi[bidx] / psi[a]) ** 2 * qr / qf)
                T[a, bidx] += p * A
                T[a, a] += p * (1 - A)
    return T


def reinforce_grad(params, spins, moves, coef, Lx, Ly):
    """Gradient of sum_b coef_b log q(c_b, k_b | s_b) with respect to the
    flattened parameters (hand-written backward pass)."""
    P = unflatten(params)
    B = spins.shape[0]
    N = Lx * Ly
    o, (z, a1, h1, a2, h2, a3, h3) = forward(params, spins, Lx, Ly, keep=True)
    do = np.zeros_like(o)                           # (B, 9, N)
    for b, (c, k) in enumerate(moves):
        pc = np.exp(log_softmax(o[b, 0], 0))
        do[b, 0] = -pc
        do[b, 0, c] += 1.0
        pk = np.exp(log_softmax(o[b, 1:9, c], 0))
        do[b, 1:9, c] = -pk
        do[b, k, c] += 1.0
        do[b] *= coef[b]
    do = do.reshape(B, 9, Ly, Lx)
    g = {}
    g["Wh"] = np.einsum("bkyx,bcyx->kc", do, h3)
    g["bh"] = do.sum(axis=(0, 2, 3))
    dh3 = np.einsum("kc,bkyx->bcyx", P["Wh"], do)

    def silu_back(dh, a):
        sg = 1.0 / (1.0 + np.exp(-a))
        return dh * (sg * (1.0 + a * (1.0 - sg)))

    def conv_back(da, x, W):
        """da (B,co,Ly,Lx), x input (B,ci,Ly,Lx) -> dW, db, dx."""
        dW = np.zeros_like(W)
        dx = np.zeros_like(x)
        for ky in range(3):
            for kx in range(3):
                sh = np.roll(x, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))
                dW[:, :, ky, kx] = np.einsum("boyx,bcyx->oc", da, sh)
                dsh = np.einsum("oc,boyx->bcyx", W[:, :, ky, kx], da)
                dx += np.roll(dsh, shift=(ky - 1, kx - 1), axis=(2, 3))
        return dW, da.sum(axis=(0, 2, 3)), dx

    da3 = silu_back(dh3, a3)
    g["W3"], g["b3"], dh2 = conv_back(da3, h2, P["W3"])
    da2 = silu_back(dh2, a2)
    g["W2"], g["b2"], dh1 = conv_back(da2, h1, P["W2"])
    da1 = silu_back(dh1, a1)
    g["W1"], g["b1"], _ = conv_back(da1, z, P["W1"])
    return flatten(g)


def log_q(params, spins, moves, Lx, Ly):
    o = forward(params, spins, Lx, Ly)
    out = []
    for b, (c, k) in enumerate(moves):
        out.append(log_softmax(o[b, 0], 0)[c] + log_softmax(o[b, 1:9, c], 0)[k - 1])
    return np.array(out)


def adam(params, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
