"""Dequantised factor sets for the low-precision storage forms -- TEST INFRASTRUCTURE ONLY.

Written independently of the GPU library's quantiser, from the storage rules:
  fp16  one power-of-two scale per stored array (each D_ts, U_ts, V_ts):
        s = 2^(ceil(log2 amax) - 15), q = round-to-nearest-even(v / s) to IEEE
        half (numpy's float16 cast), dequantised value q * s (exact in FP32);
  bf16  q = round-to-nearest-even(v) to bfloat16 (torch's CPU cast).
"""
from __future__ import annotations

import copy
import math

import numpy as np


def fp16_scale(amax: float) -> float:
    if not amax > 0.0:
        return 1.0
    c = math.ceil(math.log2(amax))
    # guard against log2 rounding at exact powers of two
    if 2.0 ** (c - 1) >= amax:
        c -= 1
    elif 2.0 ** c < amax:
        c += 1
    return 2.0 ** max(c - 15, -126)


def _dequant_fp16(a: np.ndarray) -> np.ndarray:
    s = fp16_scale(float(np.max(np.abs(a))) if a.size else 0.0)
    q = (a.astype(np.float64) / s).astype(np.float32).astype(np.float16)
    return (q.astype(np.float64) * s).astype(np.float32)


def _dequant_bf16(pool: np.ndarray) -> np.ndarray:
    import torch

    t = torch.from_numpy(np.ascontiguousarray(pool, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def dequantised(data, form: str):
    """A copy of ``data`` (HMatrixData) whose pool holds the dequantised factors."""
    if form == "fp32":
        return data
    if form == "bf16":
        out = copy.copy(data)
        out.pool = _dequant_bf16(data.pool)
        return out
    if form != "fp16":
        raise ValueError(form)
    out = copy.copy(data)
    pool = data.pool.copy()
    sz = data.tree.end - data.tree.begin
    for b in range(len(data.blocks)):
        t, s, r = int(data.blocks.target[b]), int(data.blocks.source[b]), int(data.blocks.rank[b])
        m, n = int(sz[t]), int(sz[s])
        oa = int(data.off_a[b])
        if r == 0:
            pool[oa:oa + m * n] = _dequant_fp16(pool[oa:oa + m * n])
        else:
            pool[oa:oa + m * r] = _dequant_fp16(pool[oa:oa + m * r])
            ob = int(data.off_b[b])
            pool[ob:ob + n * r] = _dequant_fp16(pool[ob:ob + n * r])
    out.pool = pool
    return out
