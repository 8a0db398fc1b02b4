"""Tree and block structure of the H-matrix (Def. 2.3, Sec. 2): weak and standard admissibility."""
import os

import numpy as np
import pytest

from hmat_inputs import (batch_problems, build_tree, enumerate_blocks, stored_elements,
                         uniform_tree)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = int(v)
    return out


def test_walkthrough_2d_root_counts():
    """The 2D worked example after Def. 2.3: 16 pairs, 12 low-rank, 4 recursed."""
    g = _read_golden("walkthrough_2d.txt")
    tree = uniform_tree(2, 64)
    root_kids = set(tree.children[0])
    blocks = enumerate_blocks(tree, 16)
    at_root = [(t, s, r) for t, s, r in zip(blocks.target, blocks.source, blocks.rank)
               if t in root_kids and s in root_kids]
    assert len(root_kids) ** 2 == g["root_child_pairs"]
    assert sum(1 for *_, r in at_root if r > 0) == g["root_low_rank"]
    assert sum(1 for *_, r in at_root if r == 0) == g["root_dense"]
    # the recursed pairs are exactly the (c, c) pairs
    assert g["root_child_pairs"] - len(at_root) == g["root_recursed"]
    assert all(t != s for t, s, _ in at_root)


@pytest.mark.parametrize("d,n,r", [(2, 64, 16), (2, 256, 8), (3, 32, 8), (3, 16, 4), (1, 1024, 4)])
def test_block_counts_closed_form(d, n, r):
    """(c-1) c^l low-rank blocks at level l = 1..L-1, c dense blocks per leaf."""
    c = 2 ** d
    tree = uniform_tree(d, n)
    L = tree.leaf_depth
    blocks = enumerate_blocks(tree, r)
    lr = blocks.rank > 0
    per_level = np.bincount(tree.depth[blocks.target[lr]], minlength=L)
    for lvl in range(1, L):
        assert per_level[lvl] == (c - 1) * c ** lvl
    n_leaves = int(np.sum([tree.is_leaf(i) for i in range(tree.num_nodes)]))
    assert int(np.sum(~lr)) == c * n_leaves
    # low-rank blocks join distinct siblings; dense blocks join leaves of one parent
    for t, s, rk in zip(blocks.target, blocks.source, blocks.rank):
        assert tree.parent[t] == tree.parent[s]
        if rk > 0:
            assert t != s and not tree.is_leaf(t) and not tree.is_leaf(s)
        else:
            assert tree.is_leaf(t) and tree.is_leaf(s)


@pytest.mark.parametrize("d,n,r,per_point", [(2, 64, 16, 448), (2, 1024, 32, 1408),
                                              (3, 64, 64, 3200), (3, 128, 32, 2304)])
def test_stored_elements(d, n, r, per_point):
    """Storage (L-1) 2 (c-1) N r + c m N: the constant of the O(r N log N) bound (Sec. 2)."""
    tree = uniform_tree(d, n)
    blocks = enumerate_blocks(tree, r)
    N = n ** d
    c, m, L = 2 ** d, 64, tree.leaf_depth
    assert stored_elements(tree, blocks) == (L - 1) * 2 * (c - 1) * N * r + c * m * N
    assert stored_elements(tree, blocks) == per_point * N


@pytest.mark.parametrize("shape", [(64, 64), (16, 16, 16), (40, 23), (9, 30, 5), (8,), (3, 3)])
def test_tree_is_a_domain_tree(shape):
    """Def. "Domain tree": root = whole set; children partition their parent."""
    tree = build_tree(shape, n_full=tuple(max(s, 64) for s in shape))
    N = int(np.prod(shape))
    assert tree.begin[0] == 0 and tree.end[0] == N
    for p in range(tree.num_nodes):
        kids = tree.children[p]
        if not kids:
            assert tree.depth[p] == tree.leaf_depth
            assert tree.size(p) <= 64
            continue
        assert tree.begin[kids[0]] == tree.begin[p] and tree.end[kids[-1]] == tree.end[p]
        for a, b in zip(kids[:-1], kids[1:]):
            assert tree.end[a] == tree.begin[b]
        assert sum(tree.size(k) for k in kids) == tree.size(p)
    # every point lies inside its leaf's box
    for p in range(tree.num_nodes):
        if tree.children[p]:
            continue
        pts = tree.points[tree.begin[p]:tree.end[p]]
        lo = (tree.lo[p] + 0.5) / np.asarray(tree.n_full)
        hi = (tree.lo[p] + tree.shape[p] - 0.5) / np.asarray(tree.n_full)
        assert np.all(pts >= lo - 1e-12) and np.all(pts <= hi + 1e-12)
    # points are distinct
    assert len(np.unique(tree.points, axis=0)) == N


def test_degenerate_trees():
    """N <= 64: the root is a leaf and the matrix is one dense block; L = 1: dense only."""
    t0 = uniform_tree(2, 8)
    assert t0.leaf_depth == 0
    b0 = enumerate_blocks(t0, 4)
    assert len(b0) == 1 and b0.rank[0] == 0 and b0.target[0] == 0 and b0.source[0] == 0
    t1 = uniform_tree(2, 16)
    assert t1.leaf_depth == 1
    b1 = enumerate_blocks(t1, 4)
    assert len(b1) == 16 and np.all(b1.rank == 0)


def test_batch_generator_shapes():
    specs = batch_problems(256, seed=4)
    assert len(specs) == 256
    ns = [int(np.prod(s["shape"])) for s in specs]
    assert min(ns) >= 1000 and max(ns) <= 70000
    assert {s["rank"] for s in specs} <= {8, 16, 32}
    assert all(s["d"] == (2 if i % 2 == 0 else 3) for i, s in enumerate(specs))
    for s in specs[:12]:
        tree = build_tree(s["shape"], n_full=s["n_full"], offset=s["offset"])
        assert all(tree.size(p) <= 64 for p in range(tree.num_nodes) if not tree.children[p])


# ---------------------------------------------------------------------------
# Standard admissibility (Sec. 2, Def. "Standard admissibility condition", with
# rho = sqrt(d) as the paper fixes it).
# ---------------------------------------------------------------------------

def _standard_bruteforce(tree, r):
    """Def. 2.3 with the standard condition, by plain recursion over one pair at a
    time and float geometry of the boxes (min(diam) <= sqrt(d) dist)."""
    d = tree.d
    nf = np.asarray(tree.n_full, float)

    def box(a):
        lo = tree.lo[a] / nf
        return lo, lo + tree.shape[a] / nf

    def admissible(t, s):
        (lt, ht), (ls, hs) = box(t), box(s)
        diam = min(np.linalg.norm(ht - lt), np.linalg.norm(hs - ls))
        gap = np.maximum(np.maximum(ls - ht, lt - hs), 0.0)
        return diam <= np.sqrt(d) * np.linalg.norm(gap) * (1 + 1e-12)

    out = {}
    todo = [(0, 0)]
    while todo:
        p, q = todo.pop()
        for ct in tree.children[p]:
            for cs in tree.children[q]:
                if tree.is_leaf(ct) or tree.is_leaf(cs):
                    out[(ct, cs)] = 0
                elif admissible(ct, cs):
                    out[(ct, cs)] = min(r, tree.size(ct), tree.size(cs))
                else:
                    todo.append((ct, cs))
    return out


@pytest.mark.parametrize("shape", [(16, 16), (32, 32), (8, 8, 8), (256,), (40, 23), (9, 13, 6)])
def test_standard_blocks_match_bruteforce(shape):
    tree = build_tree(shape, leaf_max=4 if len(shape) > 1 else 8)
    blocks = enumerate_blocks(tree, 3, "standard")
    got = {(int(t), int(s)): int(k) for t, s, k in zip(blocks.target, blocks.source, blocks.rank)}
    assert len(got) == len(blocks)
    assert got == _standard_bruteforce(tree, 3)


@pytest.mark.parametrize("d,n", [(2, 256), (2, 1024), (3, 32), (3, 64), (1, 4096)])
def test_standard_block_counts_closed_form(d, n):
    """On the ideal domain with m = 2^l boxes per axis, the ordered pairs whose
    parents are neighbours number (6m - 8)^d per level and the neighbour pairs
    (3m - 2)^d; the low-rank blocks are their difference, the dense blocks all
    (6m - 8)^d leaf pairs."""
    tree = uniform_tree(d, n)
    L = tree.leaf_depth
    blocks = enumerate_blocks(tree, 4, "standard")
    lr = blocks.rank > 0
    per_level = np.bincount(tree.depth[blocks.target[lr]], minlength=L + 1)
    for lvl in range(1, L):
        m = 2 ** lvl
        assert per_level[lvl] == (6 * m - 8) ** d - (3 * m - 2) ** d
    assert per_level[L] == 0
    assert int(np.sum(~lr)) == (6 * 2 ** L - 8) ** d
    # same depth on both sides; dense only between leaves
    assert np.all(tree.depth[blocks.target] == tree.depth[blocks.source])
    assert np.all(tree.depth[blocks.target[~lr]] == L)


def test_standard_admissibility_boundary():
    """Boxes of side h one box apart are admissible (h sqrt(d) <= sqrt(d) h, equality);
    boxes that touch, even at a corner, are not."""
    from hmat_inputs.tree import standard_admissible
    tree = uniform_tree(2, 256)   # level 2: 4 x 4 boxes of 64 x 64 cells
    lvl2 = [int(a) for a in tree.nodes_at_depth(2)]
    pos = {tuple(int(v) // 64 for v in tree.lo[a]): a for a in lvl2}
    a = pos[(0, 0)]
    assert standard_admissible(tree, [a], [pos[(2, 0)]])[0]
    assert standard_admissible(tree, [a], [pos[(2, 2)]])[0]
    assert not standard_admissible(tree, [a], [pos[(1, 1)]])[0]
    assert not standard_admissible(tree, [a], [pos[(1, 0)]])[0]
    assert not standard_admissible(tree, [a], [a])[0]


def test_standard_stored_elements():
    """Storage of the 1024^2, rank-4 workload: 2 r sum_l count_l N / 4^l + 64^2 dense count."""
    tree = uniform_tree(2, 1024)
    blocks = enumerate_blocks(tree, 4, "standard")
    N, L = tree.n, tree.leaf_depth
    lr = sum(((6 * 2 ** l - 8) ** 2 - (3 * 2 ** l - 2) ** 2) * 2 * 4 * (N // 4 ** l) for l in range(1, L))
    dense = (6 * 2 ** L - 8) ** 2 * 64 * 64
    assert stored_elements(tree, blocks) == lr + dense
