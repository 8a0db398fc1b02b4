"""Pins of the H^2 oracle (oracle/h2.py) on the CPU.

The oracle writes each box's nested bases out by stacking the children's
U_c E_c (V_c F_c) and sums U_t S_ts V_s^T x_s + D_ts x_s over the blocks.
Pinned against:

  H1  a dense assembly whose basis rows come from a different route: for
      every leaf under t, the leaf basis times the chain of transfer matrices
      along the leaf's path up to t (brute force, tiny N);
  H2  the H-matrix oracle (the pinned C oracle of Eq. (2.4)) over the H-matrix
      factors U_ts = U_t S_ts, V_ts = V_s of the same operator;
  H3  exactness of Chebyshev interpolation: for a kernel that is a
      polynomial of degree 2 in each variable, the interpolation-built H^2
      (q = 3 points per axis) is the kernel matrix itself, so the product
      equals the dense kernel product (FP32 rounding of the factors aside),
      and with q = 2 it does not;
  H4  convergence: under standard admissibility the interpolation error of
      the 1/r kernel falls geometrically with q;
  H5  storage: the stored element count has the closed form of a uniform
      tree, linear in N (Sec. 1: nested bases bring the memory cost down to
      linear), while the H-matrix's grows like N log N;
  H6  alpha / beta.

Planted mistakes in a copy of the oracle (transposed transfer, V built with
E, children stacked in reverse, transposed coupling, dense part dropped, the
target's column basis in place of the source's) must each fail H1, H2 or H3.
"""
import inspect
import math
import types

import numpy as np
import pytest

import oracle
import oracle.h2 as h2o
from hmat_inputs import HMatrixData, build_tree, dense_kernel, make_rhs, stored_elements, uniform_tree
from hmat_inputs.h2 import h2_stored_elements, make_h2
from hmat_inputs.tree import BlockList, enumerate_blocks


def _chain_basis_rows(h2, t, which):
    """Basis of box t by leaf-path products: rows of leaf l under t are
    U_l E_l E_parent(l) ... E_(child of t on the path)."""
    tree = h2.tree
    rows = []
    stack = [t]
    leaves = []
    while stack:                                   # leaves under t in tree order
        a = stack.pop()
        if tree.is_leaf(a):
            leaves.append(a)
        else:
            stack.extend(reversed(tree.children[a]))
    for leaf in leaves:
        base = (h2.leaf_u(leaf) if which == "u" else h2.leaf_v(leaf)).astype(np.float64)
        m = np.eye(int(h2.rank[leaf]))
        a = leaf
        while a != t:
            tr = h2.transfer_e(a) if which == "u" else h2.transfer_f(a)
            m = m @ tr.astype(np.float64)
            a = int(tree.parent[a])
        rows.append(base @ m)
    return np.vstack(rows)


def _assemble_h2(h2):
    tree, blocks = h2.tree, h2.blocks
    n = tree.n
    k = np.full((n, n), np.nan)
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        rt = slice(int(tree.begin[t]), int(tree.end[t]))
        rs = slice(int(tree.begin[s]), int(tree.end[s]))
        if blocks.rank[b] == 0:
            k[rt, rs] = h2.dense(b).astype(np.float64)
        else:
            k[rt, rs] = _chain_basis_rows(h2, t, "u") @ h2.coupling(b).astype(np.float64) @ \
                _chain_basis_rows(h2, s, "v").T
    assert np.isfinite(k).all(), "blocks do not cover the matrix"
    return k


def _as_h_factors(h2):
    """The H-matrix factor set of the same operator: U_ts = U_t S_ts, V_ts = V_s (FP32)."""
    tree, blocks = h2.tree, h2.blocks
    ranks = np.where(blocks.rank > 0, h2.rank[blocks.source], 0).astype(np.int32)
    sz = tree.end - tree.begin
    off_a = np.zeros(len(blocks), np.int64)
    off_b = np.full(len(blocks), -1, np.int64)
    cur = 0
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        off_a[b] = cur
        if ranks[b] == 0:
            cur += int(sz[t] * sz[s])
        else:
            cur += int(sz[t]) * int(ranks[b])
            off_b[b] = cur
            cur += int(sz[s]) * int(ranks[b])
    pool = np.empty(cur, np.float32)
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        if ranks[b] == 0:
            d = h2.dense(b)
            pool[off_a[b]:off_a[b] + d.size] = d.T.reshape(-1)
        else:
            u = _chain_basis_rows(h2, t, "u") @ h2.coupling(b).astype(np.float64)
            v = _chain_basis_rows(h2, s, "v")
            pool[off_a[b]:off_a[b] + u.size] = u.T.reshape(-1).astype(np.float32)
            pool[off_b[b]:off_b[b] + v.size] = v.T.reshape(-1).astype(np.float32)
    return HMatrixData(tree, BlockList(blocks.target, blocks.source, ranks), pool, off_a, off_b, h2.kind, "h2")


def _poly2_dense(tree):
    p = tree.points
    return (1.0 + p @ p.T) ** 2


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TREES = {
    "2d-32x32-leaf4": lambda: uniform_tree(2, 32, leaf_max=4),         # L = 4
    "2d-ragged-23x17-leaf4": lambda: build_tree((23, 17), n_full=(32, 32), leaf_max=4),
    "1d-256-leaf8": lambda: uniform_tree(1, 256, leaf_max=8),
}


def _pins(mod, name="2d-32x32-leaf4", rank=6, admissibility="weak"):
    """H1, H2 and H3 for the oracle module `mod`; returns the three errors."""
    tree = TREES[name]()
    h2 = make_h2(tree, method="random", rank=rank, seed=5, admissibility=admissibility)
    x = make_rhs(tree.n, 2, 9)
    y = mod.h2_oracle_matvec(h2, x)
    e1 = _rel(y, _assemble_h2(h2) @ x.astype(np.float64))
    e2 = _rel(y, oracle.oracle_matvec(_as_h_factors(h2), x))
    t3 = uniform_tree(2, 16, leaf_max=4)
    p3 = make_h2(t3, method="cheb", q=3, kind="poly2")
    x3 = make_rhs(t3.n, 1, 2)
    e3 = _rel(mod.h2_oracle_matvec(p3, x3), _poly2_dense(t3) @ x3.astype(np.float64))
    return e1, e2, e3


@pytest.mark.parametrize("name", ["2d-32x32-leaf4", "2d-ragged-23x17-leaf4", "1d-256-leaf8"])
@pytest.mark.parametrize("admissibility", ["weak", "standard"])
def test_h1_h2_against_path_products_and_h_oracle(name, admissibility):
    if name.startswith("1d") and admissibility == "standard":
        pytest.skip("the standard-admissibility generator covers 2D and 3D grids")
    e1, e2, _ = _pins(h2o, name, admissibility=admissibility)
    assert e1 <= 1e-12, e1
    assert e2 <= 1e-6, e2      # the H factors U_t S_ts are rounded to FP32


def test_h1_3d():
    tree = uniform_tree(3, 16, leaf_max=8)
    h2 = make_h2(tree, method="random", rank=5, seed=2)
    assert tree.leaf_depth >= 3
    x = make_rhs(tree.n, 1, 3)
    assert _rel(h2o.h2_oracle_matvec(h2, x), _assemble_h2(h2) @ x.astype(np.float64)) <= 1e-12


@pytest.mark.parametrize("d,n,q", [(2, 16, 3), (2, 16, 4), (3, 8, 3)])
def test_h3_interpolation_reproduces_a_polynomial_kernel(d, n, q):
    tree = uniform_tree(d, n, leaf_max=4)
    assert tree.leaf_depth >= 2
    h2 = make_h2(tree, method="cheb", q=q, kind="poly2")
    x = make_rhs(tree.n, 2, 4)
    err = _rel(h2o.h2_oracle_matvec(h2, x), _poly2_dense(tree) @ x.astype(np.float64))
    assert err <= 1e-5, err


def test_h3_has_teeth_with_too_few_points():
    tree = uniform_tree(2, 16, leaf_max=4)
    h2 = make_h2(tree, method="cheb", q=2, kind="poly2")
    x = make_rhs(tree.n, 1, 4)
    assert _rel(h2o.h2_oracle_matvec(h2, x), _poly2_dense(tree) @ x.astype(np.float64)) > 1e-3


def test_h4_interpolation_error_decays_with_q():
    tree = uniform_tree(3, 16, leaf_max=8)
    k = dense_kernel(tree, "inv")
    x = make_rhs(tree.n, 1, 6)
    ref = k @ x.astype(np.float64)
    errs = [_rel(h2o.h2_oracle_matvec(make_h2(tree, method="cheb", q=q, kind="inv", admissibility="standard"), x),
                 ref) for q in (2, 3, 4)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.25 * errs[0], errs


@pytest.mark.parametrize("k", [8, 32])
def test_h5_storage_closed_form_and_linear_growth(k):
    per_n_h2, per_n_h = [], []
    for n in (128, 256, 512):
        tree = uniform_tree(2, n)
        L = tree.leaf_depth
        blocks = enumerate_blocks(tree, 1)
        rank = np.zeros(tree.num_nodes, np.int32)
        rank[1:] = k
        got = h2_stored_elements(tree, blocks, rank)
        nn = tree.n
        closed = (2 * nn * k + 2 * k * k * sum(4 ** l for l in range(2, L + 1))
                  + 3 * k * k * sum(4 ** l for l in range(1, L)) + 4 * 64 * nn)
        assert got == closed
        per_n_h2.append(got / nn)
        per_n_h.append(stored_elements(tree, enumerate_blocks(tree, k)) / nn)
    # per point, the H^2 storage converges (geometric tail) while the H storage grows by a level each time
    assert per_n_h2[2] - per_n_h2[1] < 0.3 * (per_n_h2[1] - per_n_h2[0]) + 1e-9
    assert per_n_h[2] - per_n_h[1] == pytest.approx(per_n_h[1] - per_n_h[0])
    assert per_n_h[2] - per_n_h[1] > 0


def test_h5_pool_matches_count():
    tree = uniform_tree(2, 64)
    h2 = make_h2(tree, method="random", rank=16, seed=1)
    assert h2.pool.size == h2_stored_elements(tree, h2.blocks, h2.rank)


def test_h6_alpha_beta():
    tree = uniform_tree(2, 32, leaf_max=4)
    h2 = make_h2(tree, method="random", rank=4, seed=8)
    x = make_rhs(tree.n, 3, 1)
    y0 = np.random.default_rng(0).standard_normal((tree.n, 3))
    y = h2o.h2_oracle_matvec(h2, x)
    got = h2o.h2_oracle_matvec(h2, x, alpha=-0.75, beta=1.5, y_in=y0)
    assert _rel(got, -0.75 * y + 1.5 * y0) <= 1e-15


def test_degenerate_trees_have_no_bases():
    for tree in (uniform_tree(2, 8), uniform_tree(2, 16)):    # root a leaf; L = 1
        h2 = make_h2(tree, method="random", rank=4, seed=3)
        assert (h2.rank == 0).all() and (h2.blocks.rank == 0).all()
        x = make_rhs(tree.n, 1, 2)
        assert _rel(h2o.h2_oracle_matvec(h2, x), _assemble_h2(h2) @ x.astype(np.float64)) <= 1e-12


# ---------------------------------------------------------------------------
# Planted mistakes
# ---------------------------------------------------------------------------
MUTANTS = {
    "transfer_transposed": [("uc @ h2.transfer_e(c).astype(np.float64)", "uc @ h2.transfer_e(c).astype(np.float64).T")],
    "v_built_with_e": [("vc @ h2.transfer_f(c).astype(np.float64)", "vc @ h2.transfer_e(c).astype(np.float64)")],
    "children_reversed": [("for c in tree.children[t]:", "for c in reversed(tree.children[t]):")],
    "coupling_transposed": [("h2.coupling(b).astype(np.float64) @", "h2.coupling(b).astype(np.float64).T @")],
    "dense_dropped": [("y[rt] += h2.dense(b).astype(np.float64) @ xd[rs]", "pass")],
    "source_basis_of_target": [("v_s = bases[s][1]", "v_s = bases[t][1]")],
}


def _mutant(name):
    src = inspect.getsource(h2o)
    for old, new in MUTANTS[name]:
        assert old in src, f"mutation anchor missing for {name}: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType(f"h2_mutant_{name}")
    exec(compile(src, f"<h2 mutant {name}>", "exec"), mod.__dict__)
    return mod


def test_unmutated_oracle_passes_pins():
    e1, e2, e3 = _pins(h2o)
    assert e1 <= 1e-12 and e2 <= 1e-6 and e3 <= 1e-5


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_h2_mutant_is_caught(name):
    mod = _mutant(name)
    try:
        e1, e2, e3 = _pins(mod)
    except (ValueError, IndexError, KeyError):
        return                                     # a shape mismatch is caught too
    assert not (e1 <= 1e-12 and e2 <= 1e-6 and e3 <= 1e-5), f"pins missed mutant {name}: {e1}, {e2}, {e3}"
