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


def test_baseline_sweep_count_closed_form():
    """A sweep whose flipped rows run from each spin's first position to the
    end of the train, one prefix step per proposal: with the first replica
    in site order, first(j) = j, so sum_j (L - j) + N = N L - N(N-1)/2 + N
    whatever the later replicas (6240, 25150 and 98688 row-steps per walker
    and term on the 8x8, 10x10 R = 3 and 16x16 workloads)."""
    for name, want in (("tfim8x8_R2_chi64_W4096", 6240), ("tfim10x10_R3_chi128_W8192", 25150),
                       ("tfim16x16_R2_chi256_W16384_T4", 98688)):
        w = wl.WORKLOADS[name]
        pi = w.pi()
        N, L = w.N, len(pi)
        assert bench.baseline_sweep_rowsteps(pi, N, L) == N * L - N * (N - 1) // 2 + N == want
    pi = np.array([2, 0, 2, 1, 0])                   # spin 3 unread: first = {2: 0, 0: 1, 1: 3}
    assert bench.baseline_sweep_rowsteps(pi, 4, 5) == (5 - 0) + (5 - 1) + (5 - 3) + 3


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
