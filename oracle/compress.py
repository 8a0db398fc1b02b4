"""Oracle for the construction of the block factors -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module. The GPU library shares no code with it.

The paper takes the blocks of Def. 2.3 as given and leaves their construction
to the literature (end of Sec. 2). The library's construction call fills a
block structure from points and a kernel function; this module computes the
same thing plainly in FP64:

  * kernel entries K(p_i, p_j) of Eq. (2.1) without quadrature weights:
    -log|p_i - p_j| / (2 pi) (``log``) or 1 / (4 pi |p_i - p_j|) (``inv``), and
    a given value where the global indices coincide;
  * dense blocks: the entries themselves;
  * low-rank blocks: the randomized SVD of Halko, Martinsson and Tropp (SIAM
    Review 53, 2011): the range finder of their Algorithm 4.1 with
    l = min(r + p, |t|, |s|) sample columns, then the direct SVD of their
    Algorithm 5.1 (Householder QR of the sample, SVD of the projected block),
    truncated to rank r, singular values split evenly between the factors;
  * the test matrix is Rademacher (+-1): entry (j, c) is +1 when bit c mod 64 of
    word c div 64 of Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011) at
    counter (j, 0, 0, 0) and key (seed, 0) is clear, -1 when it is set, j being
    the global (tree order) index of the source point.

The factors themselves are not unique (signs, rotations among equal singular
values); what the tests compare is the product U V^T of each block.
"""
from __future__ import annotations

import math

import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a: int, x: np.ndarray):
    """High and low 64-bit words of the 128-bit products a * x (x uint64 array)."""
    a_lo, a_hi = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    x_lo, x_hi = x & _MASK32, x >> np.uint64(32)
    ll = a_lo * x_lo
    lh = a_lo * x_hi
    hl = a_hi * x_lo
    hh = a_hi * x_hi
    mid = (ll >> np.uint64(32)) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = (ll & _MASK32) | ((mid & _MASK32) << np.uint64(32))
    return hi, lo


def philox4x64_10(counters: np.ndarray, key) -> np.ndarray:
    """Philox4x64 with 10 rounds over an (n, 4) uint64 counter array and a key of two words."""
    c = [np.asarray(counters[:, i], dtype=np.uint64).copy() for i in range(4)]
    k0, k1 = int(key[0]) & ((1 << 64) - 1), int(key[1]) & ((1 << 64) - 1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = (k0 + _W0) & ((1 << 64) - 1)
                k1 = (k1 + _W1) & ((1 << 64) - 1)
            hi0, lo0 = _mulhilo(_M0, c[0])
            hi1, lo1 = _mulhilo(_M1, c[2])
            c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return np.stack(c, axis=1)


def rademacher(rows: np.ndarray, ell: int, seed: int) -> np.ndarray:
    """The test matrix rows for global source indices ``rows``: (len(rows), ell) of +-1."""
    ctr = np.zeros((len(rows), 4), dtype=np.uint64)
    ctr[:, 0] = np.asarray(rows, dtype=np.uint64)
    words = philox4x64_10(ctr, (seed, 0))
    cols = np.arange(ell)
    bits = (words[:, cols // 64] >> (cols % 64).astype(np.uint64)) & np.uint64(1)
    return np.where(bits == 1, -1.0, 1.0)


def kernel_entries(pt: np.ndarray, ps: np.ndarray, kind: str) -> np.ndarray:
    """FP64 entries between target points pt (m x d) and source points ps (n x d), off the diagonal."""
    pt = np.asarray(pt, dtype=np.float64)
    ps = np.asarray(ps, dtype=np.float64)
    d2 = np.zeros((len(pt), len(ps)))
    for a in range(pt.shape[1]):
        diff = pt[:, a][:, None] - ps[:, a][None, :]
        d2 += diff * diff
    dist = np.sqrt(d2)
    with np.errstate(divide="ignore"):
        if kind == "log":
            return -np.log(dist) / (2.0 * math.pi)
        if kind == "inv":
            return 1.0 / (4.0 * math.pi * dist)
    raise ValueError(f"unknown kernel {kind!r}")


def block_entries(points: np.ndarray, t0: int, t1: int, s0: int, s1: int, kind: str, diag: float) -> np.ndarray:
    """K over rows [t0, t1) and columns [s0, s1) of the tree-ordered points, diagonal set to ``diag``."""
    k = kernel_entries(points[t0:t1], points[s0:s1], kind)
    i = np.arange(t0, t1)[:, None]
    j = np.arange(s0, s1)[None, :]
    k[i == j] = diag
    return k


def rsvd(k: np.ndarray, omega: np.ndarray, r: int):
    """Randomized SVD of k with test matrix omega (|s| x l), truncated to rank r.

    Range finder (Y = K Omega, Q from the Householder QR of Y), then the SVD of
    B = Q^T K; U = Q U_B[:, :r] S^(1/2), V = V_B[:, :r] S^(1/2).
    """
    y = k @ omega
    q, _ = np.linalg.qr(y)
    b = q.T @ k
    ub, sv, vt = np.linalg.svd(b, full_matrices=False)
    root = np.sqrt(sv[:r])
    return (q @ ub[:, :r]) * root[None, :], vt[:r].T * root[None, :]


def compress(points: np.ndarray, begin, end, blocks, kind: str, diag: float, oversample: int, seed: int):
    """Every block of ``blocks`` ((target, source, rank) triples over the tree's begin/end arrays).

    Returns a list of ("dense", D) or ("lowrank", U, V), FP64.
    """
    out = []
    for t, s, r in blocks:
        t0, t1, s0, s1 = int(begin[t]), int(end[t]), int(begin[s]), int(end[s])
        k = block_entries(points, t0, t1, s0, s1, kind, diag)
        if r == 0:
            out.append(("dense", k))
            continue
        ell = min(r + oversample, t1 - t0, s1 - s0)
        omega = rademacher(np.arange(s0, s1), ell, seed)
        u, v = rsvd(k, omega, r)
        out.append(("lowrank", u, v))
    return out
