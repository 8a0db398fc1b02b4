"""Seeded factor sets for the weak-admissibility H-matrix (setup only).

The H-matrix-vector product takes its blocks as given: dense blocks D and
low-rank blocks U V^T (Def. 2.3, Sec. 2). How they are computed is outside the
paper's scope (end of Sec. 2), so this module supplies them as inputs:

  * kernel entries K(p_i, p_j) = -log|p_i - p_j| / (2 pi) in 2D and
    1 / (4 pi |p_i - p_j|) in 3D, with the diagonal set to 1, evaluated in FP64
    (the Nystrom matrix of Eq. (2.1) without quadrature weights);
  * low-rank factors by exact truncated SVD, by randomized SVD (Gaussian test
    matrix with r + p columns, QR of the sample, SVD of the projected block;
    Halko, Martinsson and Tropp, SIAM Review 2011), by the exact full-rank
    split U = K_ts, V = I, or filled with random numbers as in the paper's own
    experiments (Sec. 5);
  * the singular values are split evenly: U = U_r S_r^(1/2), V = V_r S_r^(1/2).

All factors are rounded to FP32 (round to nearest even) and packed into one
pool. This FP32 pool is the canonical factor set: the oracle and the GPU
library both read exactly these values.

Layout in the pool: a dense block is |t| x |s| column-major (ld = |t|); a
low-rank block stores U (|t| x r, ld = |t|) and then V (|s| x r, ld = |s|).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .tree import BlockList, ClusterTree, enumerate_blocks

KERNELS = ("log", "inv")


def kernel_matrix(pt: np.ndarray, ps: np.ndarray, kind: str, diag_mask=None) -> np.ndarray:
    """FP64 kernel entries between target points pt (m x d) and source points ps (n x d).

    ``diag_mask`` (m x n bool) marks the entries whose global indices coincide;
    they are set to 1.
    """
    diff = pt[:, None, :] - ps[None, :, :]
    dist = np.sqrt(np.sum(diff * diff, axis=2))
    with np.errstate(divide="ignore"):
        if kind == "log":
            k = -np.log(dist) / (2.0 * math.pi)
        elif kind == "inv":
            k = 1.0 / (4.0 * math.pi * dist)
        else:
            raise ValueError(f"unknown kernel {kind!r}")
    if diag_mask is not None:
        k[diag_mask] = 1.0
    return k


def block_kernel(tree: ClusterTree, t: int, s: int, kind: str) -> np.ndarray:
    """FP64 entries K[t rows, s cols] with K_ii = 1 on the global diagonal."""
    bt, et, bs, es = int(tree.begin[t]), int(tree.end[t]), int(tree.begin[s]), int(tree.end[s])
    gi = np.arange(bt, et)[:, None]
    gj = np.arange(bs, es)[None, :]
    mask = gi == gj
    return kernel_matrix(tree.points[bt:et], tree.points[bs:es], kind, mask if mask.any() else None)


def dense_kernel(tree: ClusterTree, kind: str) -> np.ndarray:
    """The full N x N kernel matrix in tree order (small N only)."""
    return block_kernel(tree, 0, 0, kind)


def _balanced(uu: np.ndarray, sv: np.ndarray, vv: np.ndarray, r: int):
    root = np.sqrt(sv[:r])
    return uu[:, :r] * root[None, :], vv[:, :r] * root[None, :]


def truncated_svd(k: np.ndarray, r: int):
    """Exact rank-r truncated SVD in FP64, singular values split evenly."""
    uu, sv, vt = np.linalg.svd(k, full_matrices=False)
    return _balanced(uu, sv, vt.T, r)


def _rsvd_numpy(kfun, m: int, n: int, r: int, p: int, rng: np.random.Generator):
    l = min(r + p, m, n)
    omega = rng.standard_normal((n, l))
    k = kfun()
    y = k @ omega
    q, _ = np.linalg.qr(y)
    b = q.T @ k
    ub, sv, vt = np.linalg.svd(b, full_matrices=False)
    return _balanced(q @ ub, sv, vt.T, r)


def _rsvd_torch(pt: np.ndarray, ps: np.ndarray, kind: str, r: int, p: int,
                rng: np.random.Generator, device):
    """Randomized SVD with the two kernel-block sweeps done on a GPU in FP32.

    Only the products K Omega and K^T Q touch the (never stored) block; the QR
    and the small SVD run on the host in FP64.
    """
    import torch

    m, n = len(pt), len(ps)
    l = min(r + p, m, n)
    omega = rng.standard_normal((n, l))
    tpts = torch.as_tensor(pt, dtype=torch.float32, device=device)
    spts = torch.as_tensor(ps, dtype=torch.float32, device=device)
    chunk = max(1, min(n, (1 << 30) // max(m, 1)))

    def kblock(c0, c1):
        acc = None
        for a in range(pt.shape[1]):
            diff = tpts[:, a:a + 1] - spts[None, c0:c1, a]
            diff.mul_(diff)
            acc = diff if acc is None else acc.add_(diff)
        if kind == "log":
            acc.log_().mul_(-1.0 / (4.0 * math.pi))
        else:
            acc.rsqrt_().mul_(1.0 / (4.0 * math.pi))
        return acc

    om = torch.as_tensor(omega, dtype=torch.float32, device=device)
    y = torch.zeros((m, l), dtype=torch.float32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        y.addmm_(kblock(c0, c1), om[c0:c1])
    q, _ = np.linalg.qr(y.double().cpu().numpy())
    qd = torch.as_tensor(q, dtype=torch.float32, device=device)
    bt = torch.empty((n, l), dtype=torch.float32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        torch.mm(kblock(c0, c1).t(), qd, out=bt[c0:c1])
    b = bt.double().cpu().numpy().T
    ub, sv, vt = np.linalg.svd(b, full_matrices=False)
    return _balanced(q @ ub, sv, vt.T, r)


@dataclasses.dataclass
class HMatrixData:
    """A canonical FP32 factor set: tree, blocks and one packed pool."""

    tree: ClusterTree
    blocks: BlockList
    pool: np.ndarray          # float32
    off_a: np.ndarray         # int64: D (dense) or U (low-rank) offset into pool
    off_b: np.ndarray         # int64: V offset (low-rank) or -1
    kind: str
    method: str

    @property
    def n(self) -> int:
        return self.tree.n

    def rows(self, b: int):
        t = int(self.blocks.target[b])
        return int(self.tree.begin[t]), int(self.tree.end[t])

    def cols(self, b: int):
        s = int(self.blocks.source[b])
        return int(self.tree.begin[s]), int(self.tree.end[s])

    def dense(self, b: int) -> np.ndarray:
        m = self.rows(b)[1] - self.rows(b)[0]
        n = self.cols(b)[1] - self.cols(b)[0]
        o = int(self.off_a[b])
        return self.pool[o:o + m * n].reshape(n, m).T

    def u(self, b: int) -> np.ndarray:
        m = self.rows(b)[1] - self.rows(b)[0]
        r = int(self.blocks.rank[b])
        o = int(self.off_a[b])
        return self.pool[o:o + m * r].reshape(r, m).T

    def v(self, b: int) -> np.ndarray:
        n = self.cols(b)[1] - self.cols(b)[0]
        r = int(self.blocks.rank[b])
        o = int(self.off_b[b])
        return self.pool[o:o + n * r].reshape(r, n).T

    def stored_bytes(self) -> int:
        return int(self.pool.nbytes)


def _layout(tree: ClusterTree, blocks: BlockList):
    sz = tree.end - tree.begin
    m = sz[blocks.target].astype(np.int64)
    n = sz[blocks.source].astype(np.int64)
    r = blocks.rank.astype(np.int64)
    count = np.where(r == 0, m * n, (m + n) * r)
    off_a = np.zeros(len(blocks), np.int64)
    if len(blocks) > 1:
        off_a[1:] = np.cumsum(count)[:-1]
    off_b = np.where(r == 0, -1, off_a + m * r)
    return off_a, off_b, int(count.sum())


def _put(pool, off, mat):
    """Store an m x n matrix column-major at pool[off:]."""
    m, n = mat.shape
    pool[off:off + m * n] = np.asarray(mat, dtype=np.float64).T.reshape(-1).astype(np.float32)


def _random_fill_torch(pool, blocks, off_a, off_b, sz, seed, device):
    """The ``random`` fill drawn on a torch device: N(0,1) numbers times a
    per-block factor (U: r^-1/2; V and D: |s|^-1/2), copied into ``pool``."""
    import torch

    starts, lens, scales = [], [], []
    for b in range(len(blocks)):
        t, s, r = int(blocks.target[b]), int(blocks.source[b]), int(blocks.rank[b])
        m, n = int(sz[t]), int(sz[s])
        if r == 0:
            starts.append(int(off_a[b])); lens.append(m * n); scales.append(1.0 / math.sqrt(n))
        else:
            starts.append(int(off_a[b])); lens.append(m * r); scales.append(1.0 / math.sqrt(r))
            starts.append(int(off_b[b])); lens.append(n * r); scales.append(1.0 / math.sqrt(n))
    order = np.argsort(np.asarray(starts, np.int64), kind="stable")
    starts = np.asarray(starts, np.int64)[order]
    lens = np.asarray(lens, np.int64)[order]
    scales = np.asarray(scales, np.float32)[order]
    if len(starts) and (starts[0] != 0 or np.any(starts[1:] != starts[:-1] + lens[:-1])
                        or starts[-1] + lens[-1] != pool.size):
        raise AssertionError("factor pool is not tiled by the blocks")
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 0xD0)
    chunk = 1 << 26
    seg = np.concatenate([[0], np.cumsum(lens)])
    i = 0
    while i < len(lens):   # groups of whole blocks of at most `chunk` entries (or one larger block)
        j = int(np.searchsorted(seg, seg[i] + chunk, side="right")) - 1
        j = max(j, i + 1)
        n_el = int(seg[j] - seg[i])
        vals = torch.randn(n_el, generator=g, device=device, dtype=torch.float32)
        fac = torch.repeat_interleave(torch.from_numpy(scales[i:j]).to(device),
                                      torch.from_numpy(lens[i:j]).to(device))
        pool[seg[i]:seg[j]] = (vals * fac).cpu().numpy()
        i = j


def make_hmatrix(tree: ClusterTree, rank: int, *, kind: str = "log", method: str = "svd",
                 seed: int = 0, oversample: int = 10, device=None, dedupe: bool = True,
                 gpu_min_entries: int = 1 << 24, admissibility: str = "weak") -> HMatrixData:
    """Build the canonical FP32 factor set for the H-matrix of ``tree``.

    ``admissibility`` ("weak" or "standard") selects the block structure.

    method:
      ``svd``      exact truncated SVD of every low-rank block;
      ``rsvd``     randomized SVD with ``oversample`` extra columns (blocks with at
                   least ``gpu_min_entries`` entries are sampled on ``device`` when
                   it is given);
      ``fullrank`` U = K_ts, V = I (or U = I, V = K_ts^T when |t| < |s|):
                   an exact split, so the H-matrix equals the kernel matrix;
      ``random``   U, V, D filled with N(0,1) numbers scaled per block
                   (U by r^-1/2, V and D by |s|^-1/2), as in the paper's
                   experiments, which use random fills. With ``device`` the
                   normal numbers are drawn there by torch's generator (seeded
                   from ``seed``), a different but equally seeded stream.

    For the kernel methods, blocks whose target and source boxes have the same
    shapes and the same relative offset hold the same entries (the kernels are
    translation invariant and every box of a given shape has the same internal
    point order); with ``dedupe`` such blocks are factorised once, and a block
    whose transpose was already factorised reuses it with U and V swapped
    (both kernels are symmetric). Every block still receives its own copy in
    the pool.
    """
    if method == "fullrank":
        rank = 1 << 30
    blocks = enumerate_blocks(tree, rank, admissibility)
    off_a, off_b, total = _layout(tree, blocks)
    pool = np.empty(total, dtype=np.float32)
    sz = tree.end - tree.begin

    if method == "random" and device is not None:
        _random_fill_torch(pool, blocks, off_a, off_b, sz, seed, device)
        return HMatrixData(tree, blocks, pool, off_a, off_b, kind, method)
    if method == "random":
        rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xD0]))
        rng.standard_normal(size=total, dtype=np.float32, out=pool)
        # per-block factors as FP32 scalars, applied segment by segment (U, then V, of a block)
        m = sz[blocks.target].astype(np.int64)
        n = sz[blocks.source].astype(np.int64)
        r = blocks.rank.astype(np.int64)
        lr = r > 0
        starts = np.concatenate([off_a, off_b[lr]])
        lens = np.concatenate([np.where(lr, m * r, m * n), n[lr] * r[lr]])
        fac = np.concatenate([np.where(lr, 1.0 / np.sqrt(np.maximum(r, 1)), 1.0 / np.sqrt(n)),
                              1.0 / np.sqrt(n[lr])]).astype(np.float32)
        order = np.argsort(starts, kind="stable")
        starts, lens, fac = starts[order], lens[order], fac[order]
        step = 1 << 24
        i = 0
        while i < len(starts):  # runs of whole segments, about `step` entries at a time
            j = max(int(np.searchsorted(starts, starts[i] + step, side="right")), i + 1)
            o0, o1 = int(starts[i]), int(starts[j - 1] + lens[j - 1])
            pool[o0:o1] *= np.repeat(fac[i:j], lens[i:j])
            i = j
        return HMatrixData(tree, blocks, pool, off_a, off_b, kind, method)

    if method not in ("svd", "rsvd", "fullrank"):
        raise ValueError(f"unknown method {method!r}")

    cache: dict = {}

    def key_of(t, s):
        return (tuple(tree.shape[t]), tuple(tree.shape[s]), tuple(tree.lo[s] - tree.lo[t]),
                t == s)

    for b in range(len(blocks)):
        t, s, r = int(blocks.target[b]), int(blocks.source[b]), int(blocks.rank[b])
        key = key_of(t, s)
        if r == 0:
            dk = ("D",) + key
            if dedupe and dk in cache:
                pool[int(off_a[b]):int(off_a[b]) + cache[dk].size] = cache[dk]
                continue
            kts = block_kernel(tree, t, s, kind)
            _put(pool, int(off_a[b]), kts)
            if dedupe:
                cache[dk] = pool[int(off_a[b]):int(off_a[b]) + kts.size].copy()
            continue

        uk = ("UV", r) + key
        tk = ("UV", r) + key_of(s, t)
        if dedupe and uk in cache:
            uf, vf = cache[uk]
        elif dedupe and tk in cache:
            vf, uf = cache[tk]
        else:
            m, n = int(sz[t]), int(sz[s])
            if method == "fullrank":
                kts = block_kernel(tree, t, s, kind)
                if m >= n:
                    u, v = kts, np.eye(n)
                else:
                    u, v = np.eye(m), kts.T
            elif method == "svd":
                u, v = truncated_svd(block_kernel(tree, t, s, kind), r)
            else:
                rng = np.random.default_rng(
                    np.random.SeedSequence([int(seed), int(tree.depth[t]), t, s]))
                if device is not None and m * n >= gpu_min_entries:
                    bt, et, bs, es = tree.begin[t], tree.end[t], tree.begin[s], tree.end[s]
                    u, v = _rsvd_torch(tree.points[bt:et], tree.points[bs:es], kind, r,
                                       oversample, rng, device)
                else:
                    u, v = _rsvd_numpy(lambda: block_kernel(tree, t, s, kind), m, n, r,
                                       oversample, rng)
            uf = np.asarray(u, dtype=np.float64).T.reshape(-1).astype(np.float32)
            vf = np.asarray(v, dtype=np.float64).T.reshape(-1).astype(np.float32)
            if dedupe:
                cache[uk] = (uf, vf)
        oa, ob = int(off_a[b]), int(off_b[b])
        pool[oa:oa + uf.size] = uf
        pool[ob:ob + vf.size] = vf
    return HMatrixData(tree, blocks, pool, off_a, off_b, kind, method)


def make_rhs(n: int, k: int, seed: int) -> np.ndarray:
    """Right-hand sides x ~ N(0,1): FP64 draws rounded to FP32, n x k column-major."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((k, n)).astype(np.float32)
    return np.asfortranarray(x.T)
