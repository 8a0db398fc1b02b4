"""Seeded inputs for the H^2-matrix variant (setup only).

An H^2-matrix (Hackbusch's nested-basis format, which Sec. 1 introduces next
to the H-matrix and which a remark of Sec. 3.2 extends the data distribution
to) keeps the block structure of Def. 2.3 but stores every low-rank block
(t, s) as U_t S_ts V_s^T: one row basis U_t and one column basis V_s per box,
shared by all blocks of that box, and a small coupling matrix S_ts (k_t x k_s)
per block. The bases are nested: only the leaves store U_t and V_t
(|t| x k_t) explicitly; every other box t with a basis is given through
transfer matrices of its children c,

    U_t = [U_c1 E_c1; U_c2 E_c2; ...],   V_t = [V_c1 F_c1; V_c2 F_c2; ...],

E_c and F_c of size k_c x k_t. Dense blocks are as in the H-matrix. Every
non-root box carries a basis (k_t >= 1) once the tree has low-rank blocks
(leaf depth L >= 2); the root never does.

This module builds such factor sets in one FP32 pool (the canonical values
both the oracle and the library read):

  * ``random``: U, V of the leaves, E, F, S and D filled with N(0, 1) numbers
    scaled so that every expanded basis and block stays of unit size
    (leaf bases by k^-1/2, transfers by k_c^-1/2, couplings by k_s^-1/2, dense
    blocks by |s|^-1/2), as in the paper's experiments with random factors;
  * ``cheb``: tensor Chebyshev interpolation of a kernel function with q
    points per axis in each box (k = q^d): U_t = V_t holds the Lagrange
    polynomials of box t at its points, E_c = F_c the parent's Lagrange
    polynomials at the child's interpolation points (which makes the bases
    exactly nested), S_ts the kernel between the interpolation points of t
    and s, D the kernel entries. Boxes are the closed grid-cell regions they
    own, points the cell centres.

Layout in the pool (all column-major): per leaf U_t then V_t (|t| x k_t); per
box below a box with a basis E_t then F_t (k_t x k_parent); per block either
S_ts (k_t x k_s) or D_ts (|t| x |s|).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .factors import block_kernel
from .tree import BlockList, ClusterTree, enumerate_blocks

H2_KINDS = ("log", "inv", "poly2")


@dataclasses.dataclass
class H2Data:
    """A canonical FP32 H^2 factor set: tree, blocks, per-node bases and one pool."""

    tree: ClusterTree
    blocks: BlockList         # rank[b] > 0 marks a coupling block (its value is k_t, informational)
    rank: np.ndarray          # int32 [num_nodes]: basis rank k_t (0: no basis)
    pool: np.ndarray          # float32
    u_off: np.ndarray         # int64 [num_nodes]: U_t of a leaf, -1 otherwise
    v_off: np.ndarray         # int64 [num_nodes]: V_t of a leaf, -1 otherwise
    e_off: np.ndarray         # int64 [num_nodes]: E_t (k_t x k_parent), -1 when the parent has no basis
    f_off: np.ndarray         # int64 [num_nodes]: F_t (k_t x k_parent), -1 when the parent has no basis
    blk_off: np.ndarray       # int64 [num_blocks]: S_ts or D_ts
    kind: str
    method: str

    @property
    def n(self) -> int:
        return self.tree.n

    def _mat(self, off, rows, cols) -> np.ndarray:
        o = int(off)
        return self.pool[o:o + rows * cols].reshape(cols, rows).T

    def leaf_u(self, t: int) -> np.ndarray:
        return self._mat(self.u_off[t], self.tree.size(t), int(self.rank[t]))

    def leaf_v(self, t: int) -> np.ndarray:
        return self._mat(self.v_off[t], self.tree.size(t), int(self.rank[t]))

    def transfer_e(self, t: int) -> np.ndarray:
        return self._mat(self.e_off[t], int(self.rank[t]), int(self.rank[self.tree.parent[t]]))

    def transfer_f(self, t: int) -> np.ndarray:
        return self._mat(self.f_off[t], int(self.rank[t]), int(self.rank[self.tree.parent[t]]))

    def coupling(self, b: int) -> np.ndarray:
        t, s = int(self.blocks.target[b]), int(self.blocks.source[b])
        return self._mat(self.blk_off[b], int(self.rank[t]), int(self.rank[s]))

    def dense(self, b: int) -> np.ndarray:
        t, s = int(self.blocks.target[b]), int(self.blocks.source[b])
        return self._mat(self.blk_off[b], self.tree.size(t), self.tree.size(s))


def h2_stored_elements(tree: ClusterTree, blocks: BlockList, rank: np.ndarray) -> int:
    """Elements of an H^2 factor set: leaf bases, transfers, couplings, dense blocks."""
    sz = (tree.end - tree.begin).astype(np.int64)
    k = rank.astype(np.int64)
    total = 0
    for t in range(tree.num_nodes):
        if k[t] == 0:
            continue
        if tree.is_leaf(t):
            total += 2 * sz[t] * k[t]
        p = tree.parent[t]
        if p >= 0 and k[p] > 0:
            total += 2 * k[t] * k[p]
    lr = blocks.rank > 0
    total += int(np.sum(k[blocks.target[lr]] * k[blocks.source[lr]]))
    total += int(np.sum(sz[blocks.target[~lr]] * sz[blocks.source[~lr]]))
    return int(total)


def _node_ranks(tree: ClusterTree, k: int) -> np.ndarray:
    rank = np.zeros(tree.num_nodes, np.int32)
    if tree.leaf_depth >= 2:
        rank[1:] = k
    return rank


def _layout(tree: ClusterTree, blocks: BlockList, rank: np.ndarray):
    n = tree.num_nodes
    u_off = np.full(n, -1, np.int64)
    v_off = np.full(n, -1, np.int64)
    e_off = np.full(n, -1, np.int64)
    f_off = np.full(n, -1, np.int64)
    cur = 0
    for t in range(n):
        k = int(rank[t])
        if k == 0:
            continue
        if tree.is_leaf(t):
            u_off[t] = cur
            v_off[t] = cur + tree.size(t) * k
            cur += 2 * tree.size(t) * k
        p = int(tree.parent[t])
        if p >= 0 and rank[p] > 0:
            e_off[t] = cur
            f_off[t] = cur + k * int(rank[p])
            cur += 2 * k * int(rank[p])
    blk_off = np.zeros(len(blocks), np.int64)
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        blk_off[b] = cur
        cur += int(rank[t] * rank[s]) if blocks.rank[b] > 0 else tree.size(t) * tree.size(s)
    return u_off, v_off, e_off, f_off, blk_off, cur


def _put(pool, off, mat):
    m = np.asarray(mat, dtype=np.float64)
    pool[int(off):int(off) + m.size] = m.T.reshape(-1).astype(np.float32)


def _cheb_nodes(a: float, b: float, q: int) -> np.ndarray:
    """Chebyshev points of the first kind on [a, b] (strictly inside)."""
    j = np.arange(q)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * j + 1) * math.pi / (2 * q))


def _lagrange(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """len(x) x len(nodes): the Lagrange polynomials of `nodes` evaluated at x."""
    out = np.ones((len(x), len(nodes)))
    for j in range(len(nodes)):
        for m in range(len(nodes)):
            if m != j:
                out[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def _box_nodes(tree: ClusterTree, t: int, q: int):
    """Per axis: the interpolation points of box t (a closed region of grid cells)."""
    n_full = np.asarray(tree.n_full, dtype=np.float64)
    lo = tree.lo[t] / n_full
    hi = (tree.lo[t] + tree.shape[t]) / n_full
    return [_cheb_nodes(lo[a], hi[a], q) for a in range(tree.d)]


def _tensor_lagrange(axes_nodes, pts: np.ndarray) -> np.ndarray:
    """len(pts) x q^d tensor Lagrange basis, multi-index with axis 0 fastest."""
    cols = None
    for a, nodes in enumerate(axes_nodes):
        la = _lagrange(nodes, pts[:, a])                       # n x q
        cols = la if cols is None else (la[:, :, None] * cols[:, None, :]).reshape(len(pts), -1)
    return cols


def _tensor_points(axes_nodes) -> np.ndarray:
    """q^d x d interpolation points, multi-index with axis 0 fastest."""
    grids = np.meshgrid(*axes_nodes[::-1], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)


def _kernel_points(kind: str, pt: np.ndarray, ps: np.ndarray) -> np.ndarray:
    diff = pt[:, None, :] - ps[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    if kind == "log":
        return -np.log(r) / (2 * math.pi)
    if kind == "inv":
        return 1.0 / (4 * math.pi * r)
    if kind == "poly2":
        return (1.0 + pt @ ps.T) ** 2
    raise ValueError(kind)


def make_h2(tree: ClusterTree, *, method: str = "random", rank: int = 16, q: int = 4, kind: str = "log",
            seed: int = 0, admissibility: str = "weak", device=None) -> H2Data:
    """Canonical FP32 H^2 factor set for ``tree`` (see the module docstring).

    ``method``: "random" (basis rank ``rank``) or "cheb" (q points per axis,
    k = q^d). ``kind`` picks the kernel of the "cheb" couplings and of the
    dense blocks: "log" (-log|x-y| / (2 pi)), "inv" (1 / (4 pi |x-y|)), both
    with unit diagonal, or "poly2" ((1 + x.y)^2, a polynomial of degree 2 in
    each variable, which interpolation with q >= 3 reproduces exactly).
    With ``device`` the random numbers are drawn there by torch's generator.
    """
    k = q ** tree.d if method == "cheb" else int(rank)
    blocks = enumerate_blocks(tree, 1, admissibility)
    rank_arr = _node_ranks(tree, k)
    blocks = BlockList(blocks.target, blocks.source,
                       np.where(blocks.rank > 0, rank_arr[blocks.target], 0).astype(np.int32))
    u_off, v_off, e_off, f_off, blk_off, total = _layout(tree, blocks, rank_arr)
    pool = np.empty(total, dtype=np.float32)
    if method == "random":
        _random_fill(pool, tree, blocks, rank_arr, u_off, v_off, e_off, f_off, blk_off, seed, device)
    elif method == "cheb":
        _cheb_fill(pool, tree, blocks, rank_arr, q, kind, u_off, v_off, e_off, f_off, blk_off)
    else:
        raise ValueError(f"unknown method {method!r}")
    return H2Data(tree, blocks, rank_arr, pool, u_off, v_off, e_off, f_off, blk_off, kind, method)


def _random_fill(pool, tree, blocks, rank, u_off, v_off, e_off, f_off, blk_off, seed, device):
    if device is not None:
        import torch

        g = torch.Generator(device=device)
        g.manual_seed(int(seed) * 7919 + 17)
        step = 1 << 26
        for o in range(0, pool.size, step):
            m = min(step, pool.size - o)
            pool[o:o + m] = torch.randn(m, generator=g, device=device, dtype=torch.float32).cpu().numpy()
    else:
        rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x42]))
        rng.standard_normal(size=pool.size, dtype=np.float32, out=pool)
    sz = tree.end - tree.begin
    segs = []   # (offset, length, factor)
    for t in range(tree.num_nodes):
        k = int(rank[t])
        if k == 0:
            continue
        if u_off[t] >= 0:
            segs.append((u_off[t], 2 * int(sz[t]) * k, 1.0 / math.sqrt(k)))
        if e_off[t] >= 0:
            segs.append((e_off[t], 2 * k * int(rank[tree.parent[t]]), 1.0 / math.sqrt(k)))
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        if blocks.rank[b] > 0:
            segs.append((blk_off[b], int(rank[t] * rank[s]), 1.0 / math.sqrt(int(rank[s]))))
        else:
            segs.append((blk_off[b], int(sz[t] * sz[s]), 1.0 / math.sqrt(int(sz[s]))))
    for o, m, f in segs:
        pool[int(o):int(o) + m] *= np.float32(f)


def _cheb_fill(pool, tree, blocks, rank, q, kind, u_off, v_off, e_off, f_off, blk_off):
    nodes = {}
    for t in range(1, tree.num_nodes):
        if rank[t] > 0:
            nodes[t] = _box_nodes(tree, t, q)
    for t, ax in nodes.items():
        if tree.is_leaf(t):
            pts = tree.points[tree.begin[t]:tree.end[t]]
            lu = _tensor_lagrange(ax, pts)                     # |t| x k
            _put(pool, u_off[t], lu)
            _put(pool, v_off[t], lu)
        p = int(tree.parent[t])
        if p in nodes:
            tr = _tensor_lagrange(nodes[p], _tensor_points(ax))  # k_t x k_p: parent's polynomials at t's points
            _put(pool, e_off[t], tr)
            _put(pool, f_off[t], tr)
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        if blocks.rank[b] > 0:
            _put(pool, blk_off[b], _kernel_points(kind, _tensor_points(nodes[t]), _tensor_points(nodes[s])))
        elif kind == "poly2":
            pt = tree.points[tree.begin[t]:tree.end[t]]
            ps = tree.points[tree.begin[s]:tree.end[s]]
            _put(pool, blk_off[b], _kernel_points(kind, pt, ps))
        else:
            _put(pool, blk_off[b], block_kernel(tree, t, s, kind))
