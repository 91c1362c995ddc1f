"""The algorithmic work counts behind bench.py's roofline figures, checked
against closed forms.  For R = 2 with the first replica in site order and
the second a permutation, both the flip-ratio passes (cut after the first
replica) and a sweep with both environments at hand need N^2 + 3N row-steps
per walker: the passes advance 1 + k rows at forward step k < N and
1 + (L - k) at backward step k >= N; a proposal for spin j contracts its
positions j .. p2(j), and the p2 sum to N(N-1)/2 + N^2."""
import numpy as np

import bench
from paper_2604_22718_amd import workloads as wl


def test_pass_and_sweep_counts_closed_form():
    for N, seed in ((8, 1), (17, 2), (64, 3)):
        pi = wl.path_site_plus_perms(N, 2, seed)
        L = len(pi)
        fwd, bwd = bench.schedule_rowsteps(pi, N, L, N)
        assert fwd == N + N * (N + 1) // 2
        assert bwd == N + N * (N + 1) // 2
        assert bench.sweep_rowsteps(pi, N, L) == N * N + 3 * N


def test_sweep_count_is_the_span_sum():
    """Any path: L plus, per spin read somewhere, the positions from its first
    replica to its last; spins read by no position cost nothing."""
    rng = np.random.default_rng(5)
    N = 10
    pi = rng.integers(0, N - 2, size=37)          # spins N-2, N-1 unread
    L = len(pi)
    want = L
    for j in range(N):
        pos = np.flatnonzero(pi == j)
        if len(pos):
            want += pos[-1] - pos[0] + 1
    assert bench.sweep_rowsteps(pi, N, L) == want


def test_eight_by_eight_workload_count():
    w = wl.MEDIUM_8x8
    pi = w.pi()
    assert bench.sweep_rowsteps(pi, w.N, len(pi)) == 4288


def test_bench_statistics_on_known_series():
    """tau_int of an AR(1) series of many walkers against (1 + rho)/(1 - rho),
    a constant series (tau 1, sigma 0), and the V-score / sigma formulas of
    energy_stats on a white-noise series."""
    import math
    g = np.random.default_rng(3)
    for rho in (0.0, 0.6):
        T, W = 400, 512
        e = g.standard_normal((T, W))
        y = np.empty_like(e)
        y[0] = e[0] / math.sqrt(1 - rho * rho)
        for t in range(1, T):
            y[t] = rho * y[t - 1] + e[t]
        assert abs(bench.tau_int(y) - (1 + rho) / (1 - rho)) < 0.1 * (1 + rho) / (1 - rho)
    assert bench.tau_int(np.full((10, 3), 2.5)) == 1.0
    x = 5.0 + g.standard_normal((50, 200))
    st = bench.energy_stats(x, 4)
    assert abs(st["E_per_site"] * 4 - x.mean()) < 1e-12
    assert abs(st["v_score"] - 4 * x.var() / x.mean() ** 2) < 1e-12
    assert abs(st["sigma_per_site"] * 4 - math.sqrt(x.var() * st["tau_int"] / x.size)) < 1e-12
