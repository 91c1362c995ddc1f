"""Chain checkpoints.  A Metropolis chain of the library is fully described
by its spins, the log-amplitude and sign carried with them, the Philox key
(seed, stream) and the index of its next sweep: every uniform is a function
of (walker, sweep, spin) alone, so a chain resumed from these makes the
same decisions as one never interrupted (the log-amplitude is recomputed at
the start of each sampling call, to FP32 evaluation accuracy).  Files are
plain .npz archives (no pickled objects)."""
from __future__ import annotations

import numpy as np
import torch

_KEYS = ("spins", "logabs", "sign", "accepts")


def save(path, spins, seed, rng_stream, next_sweep, logabs=None, sign=None, accepts=None, **extra):
    """Write the chain state; device tensors are copied to the host."""
    arrays = {"seed": np.uint64(seed), "rng_stream": np.uint64(rng_stream), "next_sweep": np.uint64(next_sweep)}
    for k, v in zip(_KEYS, (spins, logabs, sign, accepts)):
        if v is not None:
            arrays[k] = v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else np.asarray(v)
    for k, v in extra.items():
        arrays["extra_" + k] = np.asarray(v)
    np.savez(path, **arrays)


def load(path, device="cuda"):
    """Read a chain state: tensors on ``device`` for the per-walker arrays,
    Python ints for the key and the sweep index, numpy arrays for extras."""
    with np.load(path, allow_pickle=False) as z:
        out = {"seed": int(z["seed"]), "rng_stream": int(z["rng_stream"]), "next_sweep": int(z["next_sweep"])}
        for k in _KEYS:
            if k in z:
                out[k] = torch.from_numpy(z[k].copy()).to(device)
        for k in z.files:
            if k.startswith("extra_"):
                out[k[6:]] = z[k].copy()
    return out
