"""Dequantised factor sets for the low-precision storage forms -- TEST INFRASTRUCTURE ONLY.

Written independently of the GPU library's quantiser, from the storage rules:
  fp16  one power-of-two scale per stored array of a low-rank block (each
        U_ts, V_ts), and per group of dense blocks (the D_ts whose target leaves
        t have one parent and whose source leaves s have one parent; amax over
        the group):
        s = 2^(ceil(log2 amax) - 15), q = round-to-nearest-even(v / s) to IEEE
        half (numpy's float16 cast), dequantised value q * s (exact in FP32);
  bf16  q = round-to-nearest-even(v) to bfloat16 (torch's CPU cast);
  fp8   low-rank factors U and V column by column: s = the smallest power of
        two with amax / s <= 448, hi = E4M3 of v / s, r = v / s - hi,
        s' = the same power of two for amax(r), lo = E4M3 of r / s', and the
        value s * RNE_f16(hi + s' lo) (E4M3 = OCP E4M3FN, torch's
        float8_e4m3fn cast); dense blocks D as s * RNE_f16(BF16(v / s)) with
        the fp16 form's power of two s for the block's group;
  fp8_f16d  U and V as in fp8, D as in fp16.
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


def _amax(a: np.ndarray) -> float:
    return float(np.max(np.abs(a))) if a.size else 0.0


def _dequant_fp16(a: np.ndarray, amax: float | None = None) -> np.ndarray:
    """FP16 values of a with the scale of amax (a's own largest |entry| by default)."""
    s = fp16_scale(_amax(a) if amax is None else amax)
    q = (a.astype(np.float64) / s).astype(np.float32).astype(np.float16)
    return (q.astype(np.float64) * s).astype(np.float32)


def _dequant_bf16(pool: np.ndarray) -> np.ndarray:
    import torch

    t = torch.from_numpy(np.ascontiguousarray(pool, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def fp8_scale(amax: float) -> float:
    """Smallest power of two s with amax / s <= 448 (1 for amax == 0)."""
    if not amax > 0.0:
        return 1.0
    k = math.ceil(math.log2(amax / 448.0))
    while amax > 448.0 * 2.0 ** k:
        k += 1
    while amax <= 448.0 * 2.0 ** (k - 1):
        k -= 1
    return 2.0 ** k


def _e4m3(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even to E4M3FN values (inputs exact in FP32, |x| <= 448)."""
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()


def _fp8_scales(amax: np.ndarray) -> np.ndarray:
    """fp8_scale of every entry of amax."""
    out = np.ones_like(amax, dtype=np.float64)
    pos = amax > 0
    k = np.ceil(np.log2(amax[pos] / 448.0))
    k += amax[pos] > 448.0 * np.exp2(k)          # guards against log2 rounding at powers of two
    k -= amax[pos] <= 448.0 * np.exp2(k - 1)
    out[pos] = np.exp2(k)
    return out


def _dequant_fp8_columns(a: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """FP8 hi + lo values of a column-major rows x cols factor (flat in, flat out)."""
    m = a.reshape(cols, rows).astype(np.float64)   # row j of m = column j of the factor
    if rows == 0:
        return a.copy()
    s = _fp8_scales(np.max(np.abs(m), axis=1))[:, None]
    u = m / s
    hi = _e4m3(u)
    r = u - hi
    s2 = _fp8_scales(np.max(np.abs(r), axis=1))[:, None]
    lo = _e4m3(r / s2)
    return (s * (hi + s2 * lo).astype(np.float16).astype(np.float64)).reshape(-1).astype(np.float32)


def _dequant_dense_bf16_scaled(a: np.ndarray, amax: float | None = None) -> np.ndarray:
    import torch

    s = fp16_scale(_amax(a) if amax is None else amax)
    q = torch.from_numpy((a.astype(np.float64) / s).astype(np.float32)).to(torch.bfloat16).to(torch.float32)
    return (q.numpy().astype(np.float16).astype(np.float64) * s).astype(np.float32)


def dequantised(data, form: str):
    """A copy of ``data`` (HMatrixData) whose pool holds the dequantised factors."""
    if form == "fp32":
        return data
    if form == "bf16":
        out = copy.copy(data)
        out.pool = _dequant_bf16(data.pool)
        return out
    if form not in ("fp16", "fp8", "fp8_f16d"):
        raise ValueError(form)
    out = copy.copy(data)
    pool = data.pool.copy()
    sz = data.tree.end - data.tree.begin
    parent = data.tree.parent
    # a dense block's scale is that of its group: the dense blocks whose target
    # and source leaves have the same parents as its own
    group = {}
    for b in range(len(data.blocks)):
        if int(data.blocks.rank[b]) == 0:
            t, s = int(data.blocks.target[b]), int(data.blocks.source[b])
            oa = int(data.off_a[b])
            key = (int(parent[t]), int(parent[s]))
            group[key] = max(group.get(key, 0.0), _amax(data.pool[oa:oa + int(sz[t]) * int(sz[s])]))
    for b in range(len(data.blocks)):
        t, s, r = int(data.blocks.target[b]), int(data.blocks.source[b]), int(data.blocks.rank[b])
        m, n = int(sz[t]), int(sz[s])
        oa = int(data.off_a[b])
        if r == 0:
            dq = _dequant_dense_bf16_scaled if form == "fp8" else _dequant_fp16
            pool[oa:oa + m * n] = dq(pool[oa:oa + m * n], group[(int(parent[t]), int(parent[s]))])
        else:
            ob = int(data.off_b[b])
            if form == "fp16":
                pool[oa:oa + m * r] = _dequant_fp16(pool[oa:oa + m * r])
                pool[ob:ob + n * r] = _dequant_fp16(pool[ob:ob + n * r])
            else:
                pool[oa:oa + m * r] = _dequant_fp8_columns(pool[oa:oa + m * r], m, r)
                pool[ob:ob + n * r] = _dequant_fp8_columns(pool[ob:ob + n * r], n, r)
    out.pool = pool
    return out
