"""Chain checkpoints: the archive round-trips every array bit for bit (CPU),
and a chain saved after some sweeps and resumed in fresh tensors makes the
uninterrupted chain's decisions (GPU; matrix-core and narrow-bond kernels),
since the Philox uniforms depend only on (walker, sweep, spin)."""
import numpy as np
import pytest
import torch

from paper_2604_22718_amd import checkpoint
from paper_2604_22718_amd import workloads as wl


def test_archive_round_trip(tmp_path):
    spins = torch.from_numpy(wl.pack_spins(wl.random_spins(7, 100, 1)).view(np.int64))
    logabs = torch.randn(7, dtype=torch.float64)
    sign = torch.tensor([1, -1, 1, 1, -1, 0, 1], dtype=torch.int8)
    p = tmp_path / "chain.npz"
    checkpoint.save(p, spins, seed=2**63 + 5, rng_stream=3, next_sweep=120, logabs=logabs, sign=sign,
                    energies=np.arange(4.0))
    d = checkpoint.load(p, device="cpu")
    assert d["seed"] == 2**63 + 5 and d["rng_stream"] == 3 and d["next_sweep"] == 120
    assert torch.equal(d["spins"], spins) and torch.equal(d["logabs"], logabs) and torch.equal(d["sign"], sign)
    assert "accepts" not in d and np.array_equal(d["energies"], np.arange(4.0))


@pytest.mark.gpu
@pytest.mark.parametrize("chi", [2, 16])
def test_resume_is_exact(tmp_path, chi):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import lattice
    from paper_2604_22718_amd import rtt as R
    pi = lattice.path(4, 4)
    bond = wl.open_bonds(len(pi), chi)
    psi = R.RTT.create(16, pi, wl.gaussian_cores(bond, 700 + chi), "f32")
    assert (psi.info["narrow"] > 0) == (chi <= 4)
    W = 300
    start = R.spins_to_device(wl.pack_spins(wl.random_spins(W, 16, 701)))

    def fresh():
        return (start.clone(), torch.empty(W, dtype=torch.float64, device="cuda"),
                torch.empty(W, dtype=torch.int8, device="cuda"), torch.zeros(W, dtype=torch.int32, device="cuda"))

    a, la, sa, acc_a = fresh()
    psi.sweep(a, seed=11, rng_stream=2, sweep0=0, n_sweeps=6, logabs=la, sign=sa, accepts=acc_a)
    b, lb, sb, acc_b = fresh()
    psi.sweep(b, seed=11, rng_stream=2, sweep0=0, n_sweeps=3, logabs=lb, sign=sb, accepts=acc_b)
    p = tmp_path / "chain.npz"
    checkpoint.save(p, b, seed=11, rng_stream=2, next_sweep=3, logabs=lb, sign=sb, accepts=acc_b)
    del b, lb, sb, acc_b
    d = checkpoint.load(p)
    psi.sweep(d["spins"], seed=d["seed"], rng_stream=d["rng_stream"], sweep0=d["next_sweep"], n_sweeps=3,
              logabs=d["logabs"], sign=d["sign"], accepts=d["accepts"])
    torch.cuda.synchronize()
    # same decisions; the carried log-amplitude is recomputed at the start of
    # each call, so it agrees to FP32 evaluation accuracy rather than bitwise
    assert torch.equal(d["spins"], a) and torch.equal(d["accepts"], acc_a) and torch.equal(d["sign"], sa)
    assert torch.max(torch.abs(d["logabs"] - la)).item() < 1e-5
