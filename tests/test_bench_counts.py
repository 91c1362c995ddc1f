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
