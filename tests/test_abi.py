"""CPU-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid arguments on the host before any launch."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rtt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_22718_amd._lib import lib as L
    return L()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2604_22718_amd._lib import SIGNATURES
    assert set(SIGNATURES) == set(syms)


def test_abi_version(lib):
    assert lib.rtt_abi_version() == 3


def _create(lib, N, pi, bond, cores, dtype=1):
    h = C.c_void_p()
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    bond = np.ascontiguousarray(bond, dtype=np.int32)
    cores = np.ascontiguousarray(cores, dtype=np.float64)
    st = lib.rtt_create(N, len(pi), pi.ctypes.data, bond.ctypes.data, cores.ctypes.data, dtype,
                        C.byref(h))
    return st, h


def test_create_rejects_bad_arguments(lib):
    pi = np.array([0, 1, 2, 0], dtype=np.int32)
    bond = np.array([1, 2, 2, 2, 1], dtype=np.int32)
    cores = np.zeros(2 * (2 + 4 + 4 + 2))
    st, h = _create(lib, 3, np.array([0, 1, 3, 0]), bond, cores)
    assert st == -1 and h.value is None
    assert b"pi[2]" in lib.rtt_last_error()
    st, _ = _create(lib, 3, pi, np.array([2, 2, 2, 2, 1]), cores)
    assert st == -1 and b"boundary" in lib.rtt_last_error()
    st, _ = _create(lib, 3, pi, bond, cores, dtype=9)
    assert st == -1 and b"dtype" in lib.rtt_last_error()
    bad = cores.copy()
    bad[3] = np.nan
    st, _ = _create(lib, 3, pi, bond, bad)
    assert st == -1 and b"non-finite" in lib.rtt_last_error()
    st, _ = _create(lib, 0, pi, bond, cores)
    assert st == -1
    big = np.array([1, 200, 200, 200, 1], dtype=np.int32)
    st, _ = _create(lib, 3, pi, big, np.zeros(2 * (200 * 3 * 200 + 2 * 200)))
    assert st == -4 and b"FP32" in lib.rtt_last_error()


def test_other_entry_points_reject_null_handles(lib):
    assert lib.rtt_evaluate(None, None, 4, None, None, None, None, None, None, None, None) == -1
    assert lib.rtt_mcmc_sweep(None, 4, None, None, None, 0, 0, 0, 1, None, None, None) == -1
    assert lib.rtt_amplitudes(None, 4, None, None, None, None) == -1
    assert lib.rtt_energy_reduce(-1, None, None, None) == -1
    H = C.c_void_p()
    assert lib.rtt_tfim_create(0, 4, 1, 1.0, 3.0, C.byref(H)) == -1
    assert lib.rtt_tfim_create(4, 4, 1, float("nan"), 3.0, C.byref(H)) == -1
    assert lib.rtt_lincomb(0, None, None, C.byref(C.c_void_p())) == -1
    assert lib.rtt_destroy(None) == 0


def test_binding_rejects_wrong_buffers_before_any_launch():
    """The binding refuses device buffers of the wrong dtype, element count
    or spin-word count instead of passing their pointers on: the kernels
    would read or write past their ends.  Checked on the host (CPU tensors
    that pass the dtype and size checks are refused as not on the device)."""
    import torch

    from paper_2604_22718_amd import rtt as R
    nw = 2
    with pytest.raises(ValueError):
        R._spins_ptr(torch.zeros(5, nw + 1, dtype=torch.int64), nw)         # wrong word count
    with pytest.raises(ValueError):
        R._spins_ptr(torch.zeros(5 * nw, dtype=torch.int64), nw)            # not [W][nw]
    with pytest.raises(ValueError):
        R._spins_ptr(torch.zeros(0, nw, dtype=torch.int64), nw)             # no walkers
    with pytest.raises(TypeError):
        R._spins_ptr(torch.zeros(5, nw, dtype=torch.int32), nw)             # not 64-bit words
    with pytest.raises(ValueError, match="CUDA"):
        R._spins_ptr(torch.zeros(5, nw, dtype=torch.int64), nw)             # right, but host memory
    with pytest.raises(TypeError):
        R._ptr(torch.zeros(5, dtype=torch.float32), "eloc", R.F64, 5)       # float32 energies
    with pytest.raises(ValueError):
        R._ptr(torch.zeros(4, dtype=torch.float64), "eloc", R.F64, 5)       # too short
    with pytest.raises(TypeError):
        R._ptr(torch.zeros(5, 3, dtype=torch.int32), "rsign", R.I8, 15)     # int32 signs
    with pytest.raises(ValueError):
        R._ptr(torch.zeros(3, dtype=torch.float64), "out", R.F64, 3)        # host memory
    with pytest.raises(TypeError):
        R._ptr(np.zeros(3), "out", R.F64, 3)                                # not a tensor
    with pytest.raises(ValueError):
        R._net_sites(C.c_void_p(12345))                                     # unknown network
    assert R._ptr(None) is None


def test_pair_sums_argument_errors(lib):
    """rtt_pair_sums checks its arguments on the host, before any launch."""
    p = C.c_void_p(16)   # never dereferenced: every call below is refused first
    assert lib.rtt_pair_sums(0, 1, 5, p, p, p, None) == -1
    assert lib.rtt_pair_sums(2, 1, 0, p, p, p, None) == -1
    assert lib.rtt_pair_sums(2, 1, 5, None, p, p, None) == -1
    assert lib.rtt_pair_sums(2, 1, 5, p, p, None, None) == -1
    assert lib.rtt_pair_sums(2, 3, 5, p, None, p, None) == -1     # row sums take B = 1
    assert b"B = 1" in lib.rtt_last_error()
