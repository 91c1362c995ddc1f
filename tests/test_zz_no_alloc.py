"""rtt_evaluate_noalloc (the evaluation entry point that allocates nothing:
its workspace is a fixed device array inside the library) against
rtt_evaluate through the C ABI: bit-identical outputs on two calls in a row,
the second with fewer walkers (the array keeps the first call's contents),
on an FP32 and a BF16 train and a narrow-bond train; a walker count beyond
the array is refused on the host before any launch."""
import numpy as np
import pytest
import torch

from helpers import case
from paper_2604_22718_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_22718_amd import rtt
    return rtt


def outputs(R, W, N):
    f = lambda dt: torch.empty(W, dtype=dt, device="cuda")
    return {"logabs": f(torch.float64), "sign": f(torch.int8),
            "logratio": torch.empty(W, N, dtype=torch.float64, device="cuda"),
            "rsign": torch.empty(W, N, dtype=torch.int8, device="cuda"),
            "eloc": f(torch.float64), "status": f(torch.int32)}


def both(R, psi, ham, bits):
    W, N = bits.shape
    spins = R.spins_to_device(wl.pack_spins(bits))
    a, b = outputs(R, W, N), outputs(R, W, N)
    R.rtt_evaluate(psi.handle, ham.handle, spins, **a)
    R.rtt_evaluate_noalloc(psi.handle, ham.handle, spins, **b)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("dtype,chi,W1,W2", [("f32", 64, 1200, 301), ("bf16", 128, 90, 7)])
def test_noalloc_matches_evaluate(R, dtype, chi, W1, W2):
    Lx, Ly = 6, 6
    N = Lx * Ly
    pi, bond, cores = case(N, 2, chi, "perm", seed=91)
    psi = R.RTT.create(N, pi, cores, dtype)
    ham = R.TFIM(Lx, Ly, 1.0, 3.04)
    for W, seed in ((W1, 92), (W2, 93)):      # second call smaller: stale contents beyond it
        print(f"[case] {dtype} chi={chi} W={W}", flush=True)
        a, b = both(R, psi, ham, wl.random_spins(W, N, seed))
        for k in a:
            assert torch.equal(a[k], b[k]), (W, k)
        assert torch.all(b["status"] == 0)
    psi.close()
    ham.close()


def test_noalloc_narrow_bond_train(R):
    N, chi = 12, 2
    pi, bond, cores = case(N, 2, chi, "perm", seed=94)
    psi = R.RTT.create(N, pi, cores, "f32")
    assert psi.info["narrow"] == 2
    ham = R.TFIM(4, 3, 1.0, 2.0)
    for W in (50, 9):
        a, b = both(R, psi, ham, wl.random_spins(W, N, 95 + W))
        for k in a:
            assert torch.equal(a[k], b[k]), (W, k)
    psi.close()
    ham.close()


def test_noalloc_refuses_more_walkers_than_its_workspace(R):
    N, chi = 64, 64
    pi, bond, cores = case(N, 2, chi, "perm", seed=96)
    psi = R.RTT.create(N, pi, cores, "f32")
    info = psi.info
    per = 2 * info["terms"] * info["groups"] * info["nslot"] * (4 * info["chi"] + 4)
    W = (64 << 20) // per + 1
    spins = R.spins_to_device(wl.pack_spins(wl.random_spins(W, N, 97)))
    out = outputs(R, W, N)
    with pytest.raises(R.RTTError) as e:
        R.rtt_evaluate_noalloc(psi.handle, None, spins, logratio=out["logratio"], rsign=out["rsign"])
    assert e.value.status == -1 and "at most" in str(e.value)
    # one walker fewer fits and matches
    sp = spins[: W - 1]
    o1, o2 = outputs(R, W - 1, N), outputs(R, W - 1, N)
    R.rtt_evaluate(psi.handle, None, sp, logratio=o1["logratio"], rsign=o1["rsign"])
    R.rtt_evaluate_noalloc(psi.handle, None, sp, logratio=o2["logratio"], rsign=o2["rsign"])
    torch.cuda.synchronize()
    assert torch.equal(o1["logratio"], o2["logratio"]) and torch.equal(o1["rsign"], o2["rsign"])
    psi.close()
