"""Core quantisation for the reduced-precision forms.  Test infrastructure only.

The paper fixes no precision.  Readings used:
  * BF16: each FP64 entry is rounded to FP32, then to BF16, both
    round-to-nearest-even (torch CPU casts).
  * FP8 e4m3 ("fn": finite, max 448): one power-of-two scale per train
    position, s_k = 2^ceil(log2(amax_k / 448)) with amax_k over both slices;
    codes = RNE(FP32(x / s_k)) after an explicit clamp to [-448, 448] (torch's cast
    maps out-of-range values to NaN); value = code * s_k exactly.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def bf16_round(x) -> np.ndarray:
    t = torch.from_numpy(np.asarray(x, dtype=np.float64)).to(torch.float32)
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def fp32_round(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def fp8_scale_exponent(core) -> int:
    amax = float(np.max(np.abs(core)))
    if amax == 0.0:
        return 0
    return int(math.ceil(math.log2(amax / 448.0)))


def fp8_quantise(core):
    """Returns (dequantised FP64 values, scale exponent e, e4m3 codes as uint8)."""
    e = fp8_scale_exponent(core)
    scaled = np.clip(np.asarray(core, dtype=np.float64) * 2.0 ** (-e), -448.0, 448.0)
    t = torch.from_numpy(scaled).to(torch.float32).to(torch.float8_e4m3fn)
    codes = t.view(torch.uint8).numpy().copy()
    deq = t.to(torch.float64).numpy() * 2.0 ** e
    return deq, e, codes


def quantise_cores(cores, dtype: str):
    """Cores as the arithmetic on the device sees them, in FP64."""
    if dtype in ("f64",):
        return [np.asarray(c, dtype=np.float64) for c in cores]
    if dtype == "f32":
        return [fp32_round(c) for c in cores]
    if dtype == "bf16":
        return [bf16_round(c) for c in cores]
    if dtype == "fp8":
        return [fp8_quantise(c)[0] for c in cores]
    raise ValueError(dtype)
