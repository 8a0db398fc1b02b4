"""Geometry, cluster tree and block structure of an H-matrix (weak or standard admissibility).

This module only builds *inputs*: point sets on a grid, the domain tree
(Sec. 2, Def. "Domain tree"), and the list of dense and low-rank blocks that
Def. 2.3 ("H-matrix", Sec. 2) produces under the weak admissibility condition
(Sec. 2, Def. "Weak admissibility condition"). It performs none of the
matrix-vector arithmetic.

Conventions (readings of points the paper leaves open):
  * points are cell centres (i + 1/2) / n_full on each axis of the full grid;
  * a box is split on every axis whose extent is at least 2, at lo + ceil(size/2);
    on an ideal domain this is the 2^d uniform partition of Sec. 2;
  * children are ordered by the Morton index sum_a b_a 2^a (axis 0 = x);
  * nodes are numbered level by level (root = 0), left to right;
  * points are stored in tree order: leaves in depth-first order, and inside a
    leaf in lexicographic order with axis 0 fastest. Every node therefore owns
    one contiguous index range [begin, end).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class ClusterTree:
    """A domain tree over grid points, level ordered.

    Attributes
    ----------
    d : spatial dimension.
    n_full : per-axis size of the full grid that fixes the cell-centre coordinates.
    parent, begin, end, depth : per-node arrays (root = node 0, parent[0] = -1).
    lo, shape : per-node integer grid corner and extent (num_nodes x d).
    children : list of child-id lists, in Morton order.
    points : (N x d) float64 coordinates in tree order.
    leaf_depth : depth L of every leaf (the trees built here are of uniform depth).
    """

    d: int
    n_full: tuple
    parent: np.ndarray
    begin: np.ndarray
    end: np.ndarray
    depth: np.ndarray
    lo: np.ndarray
    shape: np.ndarray
    children: list
    points: np.ndarray
    leaf_depth: int

    @property
    def num_nodes(self) -> int:
        return len(self.parent)

    @property
    def n(self) -> int:
        return int(self.end[0] - self.begin[0])

    def size(self, node: int) -> int:
        return int(self.end[node] - self.begin[node])

    def is_leaf(self, node: int) -> bool:
        return len(self.children[node]) == 0

    def nodes_at_depth(self, level: int) -> np.ndarray:
        return np.nonzero(self.depth == level)[0]


def _split_depth(shape, leaf_max: int) -> int:
    """Smallest depth at which every box of an axis-aligned grid holds <= leaf_max points.

    Splitting an extent s at ceil(s/2) repeatedly leaves at most ceil(s / 2^l)
    cells per axis after l splits.
    """
    level = 0
    while True:
        worst = 1
        for s in shape:
            worst *= -(-int(s) // (1 << level))
        if worst <= leaf_max:
            return level
        level += 1


def build_tree(shape, *, n_full=None, offset=None, leaf_max: int = 64) -> ClusterTree:
    """Build the domain tree of the sub-grid ``offset + [0, shape)`` of a full grid.

    Every branch is split to the same depth L, the smallest depth at which all
    leaves hold at most ``leaf_max`` points. For an ideal domain
    (shape = (n,)*d with n a power of two times the leaf side) this is the
    recursive 2^d uniform partition.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    if d not in (1, 2, 3):
        raise ValueError("dimension must be 1, 2 or 3")
    n_full = tuple(int(s) for s in (n_full if n_full is not None else shape))
    offset = tuple(int(o) for o in (offset if offset is not None else (0,) * d))
    for a in range(d):
        if shape[a] < 1 or offset[a] < 0 or offset[a] + shape[a] > n_full[a]:
            raise ValueError("sub-grid does not fit the full grid")
    leaf_depth = _split_depth(shape, leaf_max)

    parent = [-1]
    depth = [0]
    lo = [offset]
    shp = [shape]
    children: list[list[int]] = [[]]
    frontier = [0]
    for level in range(leaf_depth):
        nxt = []
        for node in frontier:
            nlo, nsh = lo[node], shp[node]
            halves = []
            for a in range(d):
                s = nsh[a]
                if s >= 2:
                    h = -(-s // 2)
                    halves.append([(nlo[a], h), (nlo[a] + h, s - h)])
                else:
                    halves.append([(nlo[a], s)])
            # Morton order: child index sum_a b_a 2^a, axis 0 is the lowest bit.
            combos = []
            for code in range(1 << d):
                bits = [(code >> a) & 1 for a in range(d)]
                if any(b >= len(halves[a]) for a, b in enumerate(bits)):
                    continue
                combos.append(bits)
            for bits in combos:
                clo = tuple(halves[a][bits[a]][0] for a in range(d))
                csh = tuple(halves[a][bits[a]][1] for a in range(d))
                cid = len(parent)
                parent.append(node)
                depth.append(level + 1)
                lo.append(clo)
                shp.append(csh)
                children.append([])
                children[node].append(cid)
                nxt.append(cid)
        frontier = nxt

    num_nodes = len(parent)
    parent_a = np.asarray(parent, dtype=np.int32)
    depth_a = np.asarray(depth, dtype=np.int32)
    lo_a = np.asarray(lo, dtype=np.int64).reshape(num_nodes, d)
    shp_a = np.asarray(shp, dtype=np.int64).reshape(num_nodes, d)
    begin = np.zeros(num_nodes, dtype=np.int64)
    end = np.zeros(num_nodes, dtype=np.int64)

    # Depth-first traversal assigns contiguous index ranges and emits points.
    pts = []
    cursor = 0
    stack = [(0, False)]
    while stack:
        node, done = stack.pop()
        if done:
            end[node] = cursor
            continue
        begin[node] = cursor
        stack.append((node, True))
        if children[node]:
            for c in reversed(children[node]):
                stack.append((c, False))
        else:
            grids = [np.arange(lo_a[node, a], lo_a[node, a] + shp_a[node, a]) for a in range(d)]
            # lexicographic with axis 0 fastest
            mesh = np.meshgrid(*grids[::-1], indexing="ij")
            coords = np.stack([m.reshape(-1) for m in mesh[::-1]], axis=1)
            pts.append(coords)
            cursor += coords.shape[0]
    idx = np.concatenate(pts, axis=0).astype(np.float64)
    points = (idx + 0.5) / np.asarray(n_full, dtype=np.float64)
    return ClusterTree(d=d, n_full=n_full, parent=parent_a, begin=begin, end=end, depth=depth_a,
                       lo=lo_a, shape=shp_a, children=children, points=points,
                       leaf_depth=leaf_depth)


def uniform_tree(d: int, n: int, leaf_max: int = 64) -> ClusterTree:
    """Ideal d-dimensional domain [0,1]^d with n points per axis (Sec. 2)."""
    return build_tree((n,) * d, leaf_max=leaf_max)


@dataclasses.dataclass
class BlockList:
    """Blocks of the H-matrix in the order Def. 2.3 visits them.

    target[b], source[b] are node ids; rank[b] = 0 marks a dense block D,
    rank[b] > 0 a low-rank block U V^T of that rank.
    """

    target: np.ndarray
    source: np.ndarray
    rank: np.ndarray

    def __len__(self) -> int:
        return len(self.target)


def enumerate_blocks(tree: ClusterTree, rank: int, admissibility: str = "weak") -> BlockList:
    """Blocks of Def. 2.3 under the weak or the standard admissibility condition."""
    if admissibility == "weak":
        return _enumerate_weak(tree, rank)
    if admissibility == "standard":
        return enumerate_blocks_standard(tree, rank)
    raise ValueError(f"unknown admissibility condition {admissibility!r}")


def _enumerate_weak(tree: ClusterTree, rank: int) -> BlockList:
    """Blocks of Def. 2.3 under weak admissibility, checked in the definition's order.

    For every child pair (ct, cs) of a recursion pair: (1) if either child is a
    leaf the block is dense; else (2) if the two are disjoint (weakly
    admissible: distinct siblings) it is low-rank; else (3) the pair (which is
    (c, c)) is recursed into. The recursion starts at (root, root). A root that
    is itself a leaf gives a single dense block (the definition has no child
    pairs to visit then).

    The rank of a low-rank block is min(rank, |t|, |s|).
    """
    tgt, src, rk = [], [], []
    if tree.is_leaf(0):
        return BlockList(np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32))
    stack = [0]
    while stack:
        p = stack.pop(0)
        kids = tree.children[p]
        for ct in kids:
            for cs in kids:
                if tree.is_leaf(ct) or tree.is_leaf(cs):
                    tgt.append(ct); src.append(cs); rk.append(0)
                elif ct != cs:
                    tgt.append(ct); src.append(cs)
                    rk.append(min(rank, tree.size(ct), tree.size(cs)))
                else:
                    stack.append(ct)
    return BlockList(np.asarray(tgt, np.int32), np.asarray(src, np.int32), np.asarray(rk, np.int32))


def standard_admissible(tree: ClusterTree, t, s, rho2=None) -> np.ndarray:
    """Sec. 2, Def. "Standard admissibility condition": min(diam t, diam s) <= rho dist(t, s).

    A box is the closed region [lo, lo + shape] / n_full of the cells it owns
    (its points are the cell centres). rho = sqrt(d), the paper's choice, unless
    ``rho2`` (rho squared) is given. The comparison is exact: squared lengths in
    integer units of 1 / lcm(n_full).
    """
    t = np.asarray(t, np.int64)
    s = np.asarray(s, np.int64)
    d = tree.d
    rho2 = d if rho2 is None else rho2
    m = math.lcm(*[int(v) for v in tree.n_full])
    unit = np.asarray([m // int(v) for v in tree.n_full], np.int64)
    lo_t, lo_s = tree.lo[t] * unit, tree.lo[s] * unit
    hi_t, hi_s = lo_t + tree.shape[t] * unit, lo_s + tree.shape[s] * unit
    diam2_t = np.sum((hi_t - lo_t) ** 2, axis=-1)
    diam2_s = np.sum((hi_s - lo_s) ** 2, axis=-1)
    gap = np.maximum(np.maximum(lo_s - hi_t, lo_t - hi_s), 0)
    dist2 = np.sum(gap ** 2, axis=-1)
    return np.minimum(diam2_t, diam2_s) <= rho2 * dist2


def enumerate_blocks_standard(tree: ClusterTree, rank: int, rho2=None) -> BlockList:
    """Blocks of Def. 2.3 under standard admissibility, in the definition's order.

    Recursion pairs are visited level by level from (root, root); for each, its
    child pairs (ct, cs) in child order: (1) a leaf child makes the block dense;
    else (2) an admissible pair is low-rank; else (3) the pair recurses. On an
    ideal domain this gives low-rank blocks between boxes whose parents are
    neighbours but which are not neighbours themselves, and dense blocks between
    every leaf and the leaves of its parent's neighbours.
    """
    if tree.is_leaf(0):
        return BlockList(np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32))
    nn = tree.num_nodes
    width = max(len(c) for c in tree.children)
    kids = np.full((nn, width), -1, np.int64)
    for a, c in enumerate(tree.children):
        kids[a, :len(c)] = c
    size = (tree.end - tree.begin).astype(np.int64)
    leaf = np.asarray([len(c) == 0 for c in tree.children])
    tgt, src, rk = [], [], []
    pairs = np.zeros((1, 2), np.int64)
    while len(pairs):
        ct = np.repeat(kids[pairs[:, 0]], width, axis=1).reshape(-1)
        cs = np.tile(kids[pairs[:, 1]], (1, width)).reshape(-1)
        ok = (ct >= 0) & (cs >= 0)
        ct, cs = ct[ok], cs[ok]
        is_leaf = leaf[ct] | leaf[cs]
        adm = np.zeros(len(ct), bool)
        adm[~is_leaf] = standard_admissible(tree, ct[~is_leaf], cs[~is_leaf], rho2)
        block = is_leaf | adm
        tgt.append(ct[block])
        src.append(cs[block])
        rk.append(np.where(is_leaf[block], 0,
                           np.minimum(np.minimum(size[ct[block]], size[cs[block]]), rank)))
        pairs = np.stack([ct[~block], cs[~block]], axis=1)
    return BlockList(np.concatenate(tgt).astype(np.int32), np.concatenate(src).astype(np.int32),
                     np.concatenate(rk).astype(np.int32))


def stored_elements(tree: ClusterTree, blocks: BlockList) -> int:
    """Number of stored matrix entries: |t||s| per dense block, (|t|+|s|) r per low-rank block."""
    sz = (tree.end - tree.begin)
    t = sz[blocks.target]
    s = sz[blocks.source]
    r = blocks.rank.astype(np.int64)
    return int(np.sum(np.where(r == 0, t * s, (t + s) * r)))
