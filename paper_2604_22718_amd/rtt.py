"""Python binding of librtt: argument marshalling only.

Functions carry the names of the C entry points (include/rtt.h) and take
torch tensors for device memory; the current torch stream is passed as the
HIP stream.  Every computation runs in the library's HIP kernels.  Spin
configurations are int64 tensors [W, ceil(N/64)] holding the uint64 words.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import RTTError, check, lib  # noqa: F401  (RTTError: raised by check)

DTYPES = {"f32": 1, "bf16": 2, "fp8": 3}


def _ptr(t, name="tensor", dtypes=None, numel=None):
    """Device pointer of a contiguous CUDA tensor of one of ``dtypes`` with
    ``numel`` elements (None: no such check); None passes through.  The
    kernels read and write exactly that many elements, so anything else is
    refused here instead of becoming an out-of-bounds access on the GPU."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError(f"{name}: dtype {t.dtype}, expected one of {[str(d) for d in dtypes]}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: device tensors must be contiguous CUDA tensors")
    return C.c_void_p(t.data_ptr())


F64, F32, I32, I8, I64 = (torch.float64,), (torch.float32,), (torch.int32,), (torch.int8,), (torch.int64,)
U32 = (torch.int32, torch.uint32)   # accept counts: the library adds uint32 values


def _spins_ptr(spins, nw, name="spins"):
    """spins: int64 [W][nw] holding the uint64 spin words; returns (W, ptr)."""
    if not isinstance(spins, torch.Tensor) or spins.dim() != 2 or spins.shape[1] != nw:
        shape = tuple(spins.shape) if isinstance(spins, torch.Tensor) else type(spins).__name__
        raise ValueError(f"{name}: expected an int64 tensor [W][{nw}], got {shape}")
    W = int(spins.shape[0])
    if W < 1:
        raise ValueError(f"{name}: no walkers")
    return W, _ptr(spins, name, I64)


def _words(h):
    """Spin count and words per walker of an RTT handle."""
    info = np.zeros(10, dtype=np.int32)
    check(lib().rtt_info(h, info.ctypes.data))
    return int(info[0]), int(info[5])


# spin counts of the network handles created here (the C ABI keeps them opaque)
_NET_SITES = {}
# run counts of the batch handles created here
_BATCH_RUNS = {}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- C entry points
def rtt_create(n_spins, pi, bond, cores_flat, dtype="f32"):
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    bond = np.ascontiguousarray(bond, dtype=np.int32)
    cores_flat = np.ascontiguousarray(cores_flat, dtype=np.float64)
    h = C.c_void_p()
    check(lib().rtt_create(int(n_spins), len(pi), pi.ctypes.data, bond.ctypes.data,
                           cores_flat.ctypes.data, DTYPES[dtype], C.byref(h)))
    return h


def rtt_lincomb(handles, coeffs):
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    co = np.ascontiguousarray(coeffs, dtype=np.float64)
    h = C.c_void_p()
    check(lib().rtt_lincomb(len(handles), C.cast(arr, C.c_void_p), co.ctypes.data, C.byref(h)))
    return h


def rtt_destroy(h):
    check(lib().rtt_destroy(h))


def rtt_info(h):
    info = np.zeros(10, dtype=np.int32)
    check(lib().rtt_info(h, info.ctypes.data))
    return dict(zip(["N", "L", "chi", "dtype", "terms", "nw", "cut", "nslot", "groups", "narrow"], info.tolist()))


def rtt_get_cores(h, term, size):
    out = np.zeros(size, dtype=np.float64)
    check(lib().rtt_get_cores(h, int(term), out.ctypes.data))
    return out


def rtt_tfim_create(Lx, Ly, periodic, J, h):
    H = C.c_void_p()
    check(lib().rtt_tfim_create(int(Lx), int(Ly), int(bool(periodic)), float(J), float(h), C.byref(H)))
    return H


def rtt_tfim_destroy(H):
    check(lib().rtt_tfim_destroy(H))


def rtt_evaluate(h, ham, spins, logabs=None, sign=None, logratio=None, rsign=None, eloc=None,
                 status=None):
    N, nw = _words(h)
    W, sp = _spins_ptr(spins, nw)
    check(lib().rtt_evaluate(h, ham, W, sp, _ptr(logabs, "logabs", F64, W), _ptr(sign, "sign", I8, W),
                             _ptr(logratio, "logratio", F64, W * N), _ptr(rsign, "rsign", I8, W * N),
                             _ptr(eloc, "eloc", F64, W), _ptr(status, "status", I32, W), _stream()))


def rtt_evaluate_noalloc(h, ham, spins, logabs=None, sign=None, logratio=None, rsign=None, eloc=None,
                         status=None):
    N, nw = _words(h)
    W, sp = _spins_ptr(spins, nw)
    check(lib().rtt_evaluate_noalloc(h, ham, W, sp, _ptr(logabs, "logabs", F64, W), _ptr(sign, "sign", I8, W),
                                     _ptr(logratio, "logratio", F64, W * N), _ptr(rsign, "rsign", I8, W * N),
                                     _ptr(eloc, "eloc", F64, W), _ptr(status, "status", I32, W), _stream()))


def rtt_amplitudes(h, spins, logabs, sign):
    W, sp = _spins_ptr(spins, _words(h)[1])
    check(lib().rtt_amplitudes(h, W, sp, _ptr(logabs, "logabs", F64, W), _ptr(sign, "sign", I8, W),
                               _stream()))


def rtt_flip_ratios(h, spins, logratio, rsign):
    N, nw = _words(h)
    W, sp = _spins_ptr(spins, nw)
    check(lib().rtt_flip_ratios(h, W, sp, _ptr(logratio, "logratio", F64, W * N),
                                _ptr(rsign, "rsign", I8, W * N), _stream()))


def rtt_local_energy(h, ham, spins, eloc):
    W, sp = _spins_ptr(spins, _words(h)[1])
    check(lib().rtt_local_energy(h, ham, W, sp, _ptr(eloc, "eloc", F64, W), _stream()))


def rtt_mcmc_sweep(h, spins, seed, rng_stream, sweep0, n_sweeps, logabs=None, sign=None,
                   accepts=None, status=None):
    W, sp = _spins_ptr(spins, _words(h)[1])
    check(lib().rtt_mcmc_sweep(h, W, sp, _ptr(logabs, "logabs", F64, W), _ptr(sign, "sign", I8, W),
                               int(seed), int(rng_stream), int(sweep0), int(n_sweeps),
                               _ptr(accepts, "accepts", U32, W), _ptr(status, "status", I32, W), _stream()))


def rtt_energy_reduce(x, out):
    check(lib().rtt_energy_reduce(x.numel(), _ptr(x, "x", F64), _ptr(out, "out", F64, 3), _stream()))


def rtt_pair_sums(x, y, out):
    """x: float64 [A][W], y: float64 [B][W] or None; out: float64 [A][B][2]
    (compensated sums of x[a] * y[b], and their finite-term counts)."""
    if x.dim() != 2 or (y is not None and (y.dim() != 2 or y.shape[1] != x.shape[1])):
        raise ValueError("rtt_pair_sums: x [A][W] and y [B][W] with the same W")
    A, W = int(x.shape[0]), int(x.shape[1])
    B = 1 if y is None else int(y.shape[0])
    check(lib().rtt_pair_sums(A, B, W, _ptr(x, "x", F64), _ptr(y, "y", F64), _ptr(out, "out", F64, 2 * A * B),
                              _stream()))


def _flat_cores(cores):
    bond = np.asarray([cores[0].shape[1]] + [c.shape[2] for c in cores], dtype=np.int32)
    flat = np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cores])
    return bond, flat


def _split_flat(bond, flat):
    out, off = [], 0
    for k in range(len(bond) - 1):
        a, b = int(bond[k]), int(bond[k + 1])
        out.append(flat[off:off + 2 * a * b].reshape(2, a, b).copy())
        off += 2 * a * b
    return out


def _out_cap(bond, chi_max, mult):
    """Doubles that bound the output train: bond k is at most chi_max, at most
    mult times the input bond, and at most 2^min(k, L-k)."""
    L = len(bond) - 1
    b = [min(int(chi_max), int(mult) * int(bond[k]), 1 << min(k, L - k, 40)) for k in range(L + 1)]
    return 2 * sum(b[k] * b[k + 1] for k in range(L))


def rtt_tt_round(cores, chi_max, rel_tol=1e-14):
    """Host FP64 tensor-train rounding; cores: list of (2, a, b) arrays."""
    bond, flat = _flat_cores(cores)
    L = len(cores)
    bout = np.zeros(L + 1, dtype=np.int32)
    cap = 2 * sum(int(min(bond[k], chi_max)) * int(min(bond[k + 1], chi_max)) for k in range(L)) + 2 * L
    out = np.zeros(cap)
    n = C.c_int64()
    check(lib().rtt_tt_round(L, bond.ctypes.data, flat.ctypes.data, chi_max, rel_tol, bout.ctypes.data,
                             out.ctypes.data, cap, C.byref(n)))
    return _split_flat(bout, out[:n.value])


def rtt_tfim_power_step(n_spins, pi, cores, Lx, Ly, J, h, tau, chi_max, rel_tol=1e-14, periodic=1):
    """One replica-space TFIM power step on the host; returns the new cores."""
    bond, flat = _flat_cores(cores)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    L = len(cores)
    bout = np.zeros(L + 1, dtype=np.int32)
    cap = _out_cap(bond, chi_max, Lx * Ly * 3 + 1)
    out = np.zeros(cap)
    n = C.c_int64()
    check(lib().rtt_tfim_power_step(n_spins, L, pi.ctypes.data, bond.ctypes.data, flat.ctypes.data, Lx, Ly,
                                    periodic, J, h, tau, chi_max, rel_tol, bout.ctypes.data, out.ctypes.data,
                                    cap, C.byref(n)))
    return _split_flat(bout, out[:n.value])


def rtt_pauli_apply(cores, coeffs, ops, alpha, beta, chi_max, chi_sum=None, rel_tol=1e-14):
    """round(alpha phi + beta sum_t coeffs[t] O_t phi) on the host; ops is a
    (n_terms, L) uint8 table (0 I, 1 X, 2 Z, 3 XZ); partial sums rounded to
    chi_sum (default chi_max).  Returns the new cores."""
    chi_sum = chi_max if chi_sum is None else chi_sum
    bond, flat = _flat_cores(cores)
    L = len(cores)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    ops = np.ascontiguousarray(ops, dtype=np.uint8)
    if ops.ndim != 2 or ops.shape != (len(coeffs), L):
        raise ValueError(f"ops must be ({len(coeffs)}, {L}), got {ops.shape}")
    bout = np.zeros(L + 1, dtype=np.int32)
    cap = _out_cap(bond, chi_max, len(coeffs) + 1)
    out = np.zeros(cap)
    n = C.c_int64()
    check(lib().rtt_pauli_apply(L, bond.ctypes.data, flat.ctypes.data, len(coeffs), coeffs.ctypes.data,
                                ops.ctypes.data, alpha, beta, chi_max, chi_sum, rel_tol, bout.ctypes.data,
                                out.ctypes.data, cap, C.byref(n)))
    return _split_flat(bout, out[:n.value])


def rtt_tt_combine(trains, coeffs, chi_max, rel_tol=1e-14):
    """round(sum_m coeffs[m] phi_m) on the host for trains on one path."""
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    L = len(trains[0])
    if len(coeffs) != len(trains) or any(len(t) != L for t in trains):
        raise ValueError("one coefficient per train, all trains of the same length")
    flats = [_flat_cores(t) for t in trains]
    bonds = np.ascontiguousarray(np.stack([b for b, _ in flats]), dtype=np.int32)
    ptrs = (C.c_void_p * len(trains))(*[f.ctypes.data for _, f in flats])
    bmax = bonds.max(axis=0)
    bout = np.zeros(L + 1, dtype=np.int32)
    cap = _out_cap(bmax, chi_max, len(trains))
    out = np.zeros(cap)
    n = C.c_int64()
    check(lib().rtt_tt_combine(len(trains), L, bonds.ctypes.data, C.cast(ptrs, C.c_void_p), coeffs.ctypes.data,
                               chi_max, rel_tol, bout.ctypes.data, out.ctypes.data, cap, C.byref(n)))
    return _split_flat(bout, out[:n.value])


def rtt_mixed_estimators(targets, ham, spins, logabs_a, sign_a, ratio, mixed, status=None):
    """targets: list of RTT handles; ratio, mixed: float64 [M][W] device tensors."""
    M = len(targets)
    if M < 1:
        raise ValueError("rtt_mixed_estimators: no targets")
    arr = (C.c_void_p * M)(*[t.value for t in targets])
    W, sp = _spins_ptr(spins, _words(targets[0])[1])
    check(lib().rtt_mixed_estimators(M, C.cast(arr, C.c_void_p), ham, W, sp, _ptr(logabs_a, "logabs_a", F64, W),
                                      _ptr(sign_a, "sign_a", I8, W), _ptr(ratio, "ratio", F64, M * W),
                                      _ptr(mixed, "mixed", F64, M * W), _ptr(status, "status", I32, W),
                                      _stream()))


def rtt_batch_create(rtts, hams, walkers, spins, eloc, seed):
    n = len(rtts)
    if not (len(hams) == len(walkers) == len(spins) == len(eloc) == n) or n < 1:
        raise ValueError("rtt_batch_create: one Hamiltonian, walker count, spin and energy buffer per run")
    for i in range(n):
        Wi, _ = _spins_ptr(spins[i], _words(rtts[i])[1], f"spins[{i}]")
        if Wi != int(walkers[i]):
            raise ValueError(f"rtt_batch_create: run {i} has {Wi} spin rows for {walkers[i]} walkers")
        _ptr(eloc[i], f"eloc[{i}]", F64, Wi)
    arr = lambda xs: (C.c_void_p * n)(*xs)
    w = np.ascontiguousarray(walkers, dtype=np.int32)
    b = C.c_void_p()
    check(lib().rtt_batch_create(n, C.cast(arr([r.value for r in rtts]), C.c_void_p),
                                 C.cast(arr([h.value for h in hams]), C.c_void_p), w.ctypes.data,
                                 C.cast(arr([t.data_ptr() for t in spins]), C.c_void_p),
                                 C.cast(arr([t.data_ptr() for t in eloc]), C.c_void_p),
                                 int(seed), C.byref(b)))
    _BATCH_RUNS[b.value] = n
    return b


def rtt_batch_step(b, n_sweeps, esum=None):
    n = _BATCH_RUNS.get(b.value)
    check(lib().rtt_batch_step(b, int(n_sweeps), _ptr(esum, "esum", F64, None if n is None else 3 * n),
                               _stream()))


def rtt_batch_autotune(b, n_sweeps, reps, cache_path=None):
    choice = np.zeros(2, dtype=np.int32)
    check(lib().rtt_batch_autotune(b, int(n_sweeps), int(reps),
                                   cache_path.encode() if cache_path else None,
                                   choice.ctypes.data, _stream()))
    return int(choice[0]), int(choice[1])


def rtt_batch_destroy(b):
    check(lib().rtt_batch_destroy(b))
    _BATCH_RUNS.pop(b.value, None)


N_NET_PARAMS = 19113


def rtt_net_create(Lx, Ly, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.size != N_NET_PARAMS:
        raise ValueError(f"rtt_net_create: {p.size} parameters, expected {N_NET_PARAMS}")
    h = C.c_void_p()
    check(lib().rtt_net_create(int(Lx), int(Ly), p.ctypes.data, C.byref(h)))
    _NET_SITES[h.value] = int(Lx) * int(Ly)
    return h


def rtt_net_destroy(h):
    check(lib().rtt_net_destroy(h))
    _NET_SITES.pop(h.value, None)


def _net_sites(h):
    if h is None or h.value not in _NET_SITES:
        raise ValueError("unknown network handle")
    return _NET_SITES[h.value]


def rtt_net_get_params(h, which=0):
    out = np.zeros(N_NET_PARAMS, dtype=np.float64)
    check(lib().rtt_net_get_params(h, int(which), out.ctypes.data))
    return out


def rtt_net_forward(h, spins, out):
    N = _net_sites(h)
    W, sp = _spins_ptr(spins, (N + 63) // 64)
    check(lib().rtt_net_forward(h, W, sp, _ptr(out, "out", F32, W * 9 * N), _stream()))


def rtt_mh_learned_step(rtt_h, net_h, spins, logabs, sign, seed, rng_stream, step, moves=None,
                        accept_prob=None, before=None, accepts=None, status=None):
    N, nw = _words(rtt_h)
    W, sp = _spins_ptr(spins, nw)
    if before is not None and tuple(before.shape) != tuple(spins.shape):
        raise ValueError(f"before: shape {tuple(before.shape)}, expected {tuple(spins.shape)}")
    check(lib().rtt_mh_learned_step(rtt_h, net_h, W, sp, _ptr(logabs, "logabs", F64, W),
                                    _ptr(sign, "sign", I8, W), int(seed), int(rng_stream), int(step),
                                    _ptr(moves, "moves", I32, W), _ptr(accept_prob, "accept_prob", F32, W),
                                    _ptr(before, "before", I64, W * nw), _ptr(accepts, "accepts", U32, W),
                                    _ptr(status, "status", I32, W), _stream()))


def _train_args(h, spins, moves, accept_prob):
    B, sp = _spins_ptr(spins, (_net_sites(h) + 63) // 64)
    return B, sp, _ptr(moves, "moves", I32, B), _ptr(accept_prob, "accept_prob", F32, B)


def rtt_net_grad(h, spins, moves, accept_prob, grad):
    B, sp, mv, ap = _train_args(h, spins, moves, accept_prob)
    check(lib().rtt_net_grad(h, B, sp, mv, ap, _ptr(grad, "grad", F32, N_NET_PARAMS), _stream()))


def rtt_net_train(h, spins, moves, accept_prob, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    B, sp, mv, ap = _train_args(h, spins, moves, accept_prob)
    check(lib().rtt_net_train(h, B, sp, mv, ap, float(lr), float(beta1), float(beta2), float(eps), _stream()))


# ---------------------------------------------------------------- convenience
class TFIM:
    """H = J sum_<ij> Z_i Z_j - h sum_i X_i on an Lx x Ly lattice."""

    def __init__(self, Lx, Ly, J=1.0, h=3.04, periodic=True):
        self.Lx, self.Ly, self.J, self.h, self.periodic = Lx, Ly, J, h, periodic
        self.handle = rtt_tfim_create(Lx, Ly, periodic, J, h)

    def close(self):
        if self.handle is not None:
            rtt_tfim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RTT:
    """An RTT (or a linear combination of RTTs) resident on the GPU."""

    def __init__(self, pi, cores=None, dtype="f32", _handle=None, _n_spins=None):
        self.pi = np.asarray(pi, dtype=np.int32)
        if _handle is not None:
            self.handle = _handle
        else:
            bond = [cores[0].shape[1]] + [c.shape[2] for c in cores]
            flat = np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cores])
            n = int(self.pi.max()) + 1 if _n_spins is None else _n_spins
            self.handle = rtt_create(n, self.pi, bond, flat, dtype)
        self.info = rtt_info(self.handle)
        self.N = self.info["N"]
        self.nw = self.info["nw"]
        self.dtype = dtype

    @classmethod
    def create(cls, n_spins, pi, cores, dtype="f32"):
        return cls(pi, cores, dtype, _n_spins=n_spins)

    @classmethod
    def lincomb(cls, terms, coeffs):
        h = rtt_lincomb([t.handle for t in terms], coeffs)
        return cls(terms[0].pi, _handle=h, dtype=terms[0].dtype)

    def close(self):
        if self.handle is not None:
            rtt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def core_values(self, bond, term=0):
        size = int(sum(2 * bond[k] * bond[k + 1] for k in range(len(bond) - 1)))
        return rtt_get_cores(self.handle, term, size)

    # ---- evaluation
    def evaluate(self, spins, ham=None, ratios=True, energy=True):
        W, dev = spins.shape[0], spins.device
        out = {
            "logabs": torch.empty(W, dtype=torch.float64, device=dev),
            "sign": torch.empty(W, dtype=torch.int8, device=dev),
            "status": torch.empty(W, dtype=torch.int32, device=dev),
        }
        if ratios:
            out["logratio"] = torch.empty(W, self.N, dtype=torch.float64, device=dev)
            out["rsign"] = torch.empty(W, self.N, dtype=torch.int8, device=dev)
        if energy and ham is not None:
            out["eloc"] = torch.empty(W, dtype=torch.float64, device=dev)
        rtt_evaluate(self.handle, ham.handle if ham is not None else None, spins,
                     out["logabs"], out["sign"], out.get("logratio"), out.get("rsign"),
                     out.get("eloc"), out["status"])
        return out

    def amplitudes(self, spins):
        W, dev = spins.shape[0], spins.device
        la = torch.empty(W, dtype=torch.float64, device=dev)
        sg = torch.empty(W, dtype=torch.int8, device=dev)
        rtt_amplitudes(self.handle, spins, la, sg)
        return la, sg

    def local_energy(self, spins, ham):
        e = torch.empty(spins.shape[0], dtype=torch.float64, device=spins.device)
        rtt_local_energy(self.handle, ham.handle, spins, e)
        return e

    def sweep(self, spins, seed, rng_stream=0, sweep0=0, n_sweeps=1, accepts=None, status=None,
              logabs=None, sign=None):
        rtt_mcmc_sweep(self.handle, spins, seed, rng_stream, sweep0, n_sweeps, logabs, sign,
                       accepts, status)


class Net:
    """Learned multi-spin proposal network resident on the GPU."""

    def __init__(self, Lx, Ly, params):
        self.Lx, self.Ly, self.N = Lx, Ly, Lx * Ly
        self.handle = rtt_net_create(Lx, Ly, params)

    def params(self, which=0):
        return rtt_net_get_params(self.handle, which)

    def forward(self, spins):
        out = torch.empty(spins.shape[0], 9, self.N, dtype=torch.float32, device=spins.device)
        rtt_net_forward(self.handle, spins, out)
        return out

    def close(self):
        if self.handle is not None:
            rtt_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LearnedChain:
    """Walkers sampled by single-flip sweeps and learned multi-spin moves;
    all arithmetic in the library's kernels, this class only sequences calls
    and owns the buffers."""

    def __init__(self, psi, net, spins, seed, rng_stream=0):
        self.psi, self.net, self.seed, self.rs = psi, net, seed, rng_stream
        self.spins = spins
        W, dev = spins.shape[0], spins.device
        self.logabs = torch.empty(W, dtype=torch.float64, device=dev)
        self.sign = torch.empty(W, dtype=torch.int8, device=dev)
        self.moves = torch.empty(W, dtype=torch.int32, device=dev)
        self.aprob = torch.empty(W, dtype=torch.float32, device=dev)
        self.before = torch.empty_like(spins)
        self.acc_flip = torch.zeros(W, dtype=torch.int32, device=dev)
        self.acc_learn = torch.zeros(W, dtype=torch.int32, device=dev)
        self.sweeps = 0
        self.steps = 0
        rtt_amplitudes(psi.handle, spins, self.logabs, self.sign)

    def sweep(self, n=1):
        rtt_mcmc_sweep(self.psi.handle, self.spins, self.seed, self.rs, self.sweeps, n,
                       self.logabs, self.sign, self.acc_flip)
        self.sweeps += n

    def learned_step(self):
        rtt_mh_learned_step(self.psi.handle, self.net.handle, self.spins, self.logabs, self.sign,
                            self.seed, self.rs, self.steps, self.moves, self.aprob, self.before,
                            self.acc_learn)
        self.steps += 1

    def train(self, lr=1e-3):
        rtt_net_train(self.net.handle, self.before, self.moves, self.aprob, lr)


class Batch:
    """Many independent RTT chains stepped together in one captured graph.
    Owns the spin and local-energy buffers of every run."""

    def __init__(self, rtts, hams, spins, seed):
        self.rtts, self.hams = rtts, hams
        self.spins = [s.contiguous() for s in spins]
        self.eloc = [torch.empty(s.shape[0], dtype=torch.float64, device=s.device) for s in self.spins]
        self.esum = torch.zeros(len(rtts), 3, dtype=torch.float64, device=self.spins[0].device)
        self.handle = rtt_batch_create([r.handle for r in rtts], [h.handle for h in hams],
                                       [s.shape[0] for s in self.spins], self.spins, self.eloc, seed)

    def step(self, n_sweeps=1, esum=True):
        rtt_batch_step(self.handle, n_sweeps, self.esum if esum else None)

    def autotune(self, n_sweeps=1, reps=2, cache_path=None):
        return rtt_batch_autotune(self.handle, n_sweeps, reps, cache_path)

    def close(self):
        if self.handle is not None:
            rtt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mixed_estimators(targets, ham, spins, logabs_a, sign_a):
    """Dual Monte Carlo estimators of walkers sampled from psi^a against the
    RTT objects ``targets``: (ratio, mixed, status), ratio and mixed [M][W]."""
    M, W = len(targets), spins.shape[0]
    ratio = torch.empty((M, W), dtype=torch.float64, device=spins.device)
    mixed = torch.empty((M, W), dtype=torch.float64, device=spins.device)
    status = torch.empty(W, dtype=torch.int32, device=spins.device)
    rtt_mixed_estimators([t.handle for t in targets], ham.handle, spins, logabs_a, sign_a, ratio, mixed,
                         status)
    return ratio, mixed, status


def energy_reduce(x):
    out = torch.empty(3, dtype=torch.float64, device=x.device)
    rtt_energy_reduce(x, out)
    return out


def pair_sums(x, y=None):
    """[A][B][2] device tensor: compensated sums of x[a] * y[b] (or of x[a]
    alone) and the number of finite terms."""
    A, B = x.shape[0], (1 if y is None else y.shape[0])
    out = torch.empty((A, B, 2), dtype=torch.float64, device=x.device)
    rtt_pair_sums(x, y, out)
    return out


def spins_to_device(bits_uint64: np.ndarray, device="cuda"):
    """uint64 numpy words -> int64 device tensor with the same bits."""
    return torch.from_numpy(np.ascontiguousarray(bits_uint64).view(np.int64)).to(device)


def spins_to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)
