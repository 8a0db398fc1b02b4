"""Pins of the FP64 oracle to results fixed by the paper and by the mathematics.

P1  assembled dense H-matrix: placing every block of Def. 2.3 in an N x N array
    and multiplying with numpy gives the oracle's y (and shows the blocks tile
    N x N exactly once), under weak and standard admissibility;
P2  full-rank special case: with U = K_ts, V = I every block is exact, so the
    H-matvec equals the plain kernel matvec fl32(K) x;
P3  Eckart-Young: with exact truncated-SVD factors the error against K x obeys
    |K_H x - K x| <= sum over low-rank blocks of sigma_{r+1}(K_ts) |x_s|, and
    each block's error is non-increasing in r;
P5  algebra of the GEMV form (remark closing Sec. 4.1): linearity, columns of a
    multi-RHS product, alpha/beta;
P8  symmetry: both kernels are symmetric and transposed blocks share their
    factors with U and V swapped, so <a, K_H b> = <K_H a, b>;
P9  transpose: the factor set of K^T (blocks (s, t), U and V swapped, dense
    blocks transposed) assembles to the transpose of K, and <a, K b> = <K^T a, b>
    holds for random (non-symmetric) factors.
"""
import numpy as np
import pytest

import oracle
from hmat_inputs import (block_kernel, dense_kernel, make_hmatrix, make_rhs, truncated_svd,
                         uniform_tree)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c1():
    tree = uniform_tree(2, 64)
    return make_hmatrix(tree, 16, kind="log", method="svd")


@pytest.mark.parametrize("d,n,r,method,kind,adm", [
    (2, 64, 16, "svd", "log", "weak"), (2, 32, 8, "random", "log", "weak"),
    (3, 16, 8, "random", "inv", "weak"), (3, 16, 8, "svd", "inv", "weak"),
    (1, 512, 4, "random", "log", "weak"), (2, 8, 4, "random", "log", "weak"),
    (2, 16, 4, "random", "log", "weak"), (2, 64, 8, "random", "log", "standard"),
    (2, 64, 4, "svd", "log", "standard"), (3, 16, 4, "random", "inv", "standard"),
    (1, 2048, 4, "random", "log", "standard")])
def test_p1_assembled_dense(d, n, r, method, kind, adm):
    tree = uniform_tree(d, n)
    data = make_hmatrix(tree, r, kind=kind, method=method, seed=7, admissibility=adm)
    kh = oracle.assemble_dense(data)
    assert not np.isnan(kh).any(), "blocks do not cover N x N"
    x = make_rhs(tree.n, 3, 11)
    y = oracle.oracle_matvec(data, x)
    ref = kh @ x.astype(np.float64)
    assert rel(y, ref) <= 1e-13


@pytest.mark.parametrize("d,n,kind,adm", [(2, 64, "log", "weak"), (3, 16, "inv", "weak"),
                                          (2, 32, "inv", "weak"), (2, 64, "log", "standard"),
                                          (1, 2048, "inv", "standard")])
def test_p2_full_rank_equals_kernel_matvec(d, n, kind, adm):
    tree = uniform_tree(d, n)
    data = make_hmatrix(tree, 0, kind=kind, method="fullrank", admissibility=adm)
    k32 = dense_kernel(tree, kind).astype(np.float32).astype(np.float64)
    x = make_rhs(tree.n, 2, 5)
    y = oracle.oracle_matvec(data, x)
    assert rel(y, k32 @ x.astype(np.float64)) <= 1e-12


def test_p3_eckart_young_and_rank_decay():
    tree = uniform_tree(2, 32)
    kind = "log"
    kfull = dense_kernel(tree, kind)
    x = make_rhs(tree.n, 1, 3)[:, 0].astype(np.float64)
    yk = kfull @ x
    # FP32 storage of the factors and dense blocks perturbs each product by a few
    # units of 2^-24 relative to |K| |x|
    slack = 8 * 2.0 ** -24 * np.linalg.norm(np.abs(kfull) @ np.abs(x))
    errs = []
    for r in (1, 2, 4, 8, 16, 32):
        data = make_hmatrix(tree, r, kind=kind, method="svd")
        y = oracle.oracle_matvec(data, x)[:, 0]
        bound = 0.0
        for b in range(len(data.blocks)):
            rk = int(data.blocks.rank[b])
            if rk == 0:
                continue
            t, s = int(data.blocks.target[b]), int(data.blocks.source[b])
            kts = block_kernel(tree, t, s, kind)
            sv = np.linalg.svd(kts, compute_uv=False)
            c0, c1 = data.cols(b)
            if rk < len(sv):
                bound += sv[rk] * np.linalg.norm(x[c0:c1])
        err = np.linalg.norm(y - yk)
        assert err <= bound + slack, (r, err, bound)
        errs.append(err)
    # the total error falls with the rank (allowing 1 % wiggle between blocks of one row)
    for a, b in zip(errs[:-1], errs[1:]):
        assert b <= a * 1.01
    assert errs[-1] < errs[0] * 1e-3


def test_p3_per_block_error_monotone():
    tree = uniform_tree(2, 64)
    kts = block_kernel(tree, 1, 2, "log")
    xs = np.random.default_rng(0).standard_normal(kts.shape[1])
    prev = np.inf
    for r in range(1, 40, 3):
        u, v = truncated_svd(kts, r)
        e = np.linalg.norm(kts @ xs - u @ (v.T @ xs))
        assert e <= prev * (1 + 1e-12) + 1e-13
        prev = e


def test_p5_linearity_and_multi_rhs(c1):
    x = make_rhs(c1.n, 4, 21).astype(np.float64)
    y = oracle.oracle_matvec(c1, x)
    for j in range(4):
        yj = oracle.oracle_matvec(c1, x[:, j])
        assert np.array_equal(yj[:, 0], y[:, j])
    a, b = 0.75, -2.5
    ylin = oracle.oracle_matvec(c1, a * x[:, 0] + b * x[:, 1])
    assert rel(ylin[:, 0], a * y[:, 0] + b * y[:, 1]) <= 1e-13


def test_p5_alpha_beta(c1):
    x = make_rhs(c1.n, 2, 22)
    y0 = np.random.default_rng(1).standard_normal((c1.n, 2))
    base = oracle.oracle_matvec(c1, x)
    got = oracle.oracle_matvec(c1, x, alpha=-1.5, beta=0.25, y_in=y0)
    assert rel(got, -1.5 * base + 0.25 * y0) <= 1e-14
    # beta = 0 never reads y_in (NaNs there must not leak)
    got0 = oracle.oracle_matvec(c1, x, alpha=2.0, beta=0.0)
    assert np.array_equal(got0, 2.0 * base)


def test_p5_row_restriction(c1):
    x = make_rhs(c1.n, 1, 23)
    full = oracle.oracle_matvec(c1, x)
    part = oracle.oracle_matvec(c1, x, rows=(1000, 3000))
    assert np.array_equal(part[1000:3000], full[1000:3000])
    assert np.isnan(part[:1000]).all() and np.isnan(part[3000:]).all()


def test_p8_symmetry(c1):
    rng = np.random.default_rng(9)
    a = rng.standard_normal(c1.n)
    b = rng.standard_normal(c1.n)
    ka = oracle.oracle_matvec(c1, a)[:, 0]
    kb = oracle.oracle_matvec(c1, b)[:, 0]
    lhs, rhs = a @ kb, ka @ b
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(a) * np.linalg.norm(kb) * 10


def test_threads_do_not_change_result(c1):
    x = make_rhs(c1.n, 1, 24)
    y1 = oracle.oracle_matvec(c1, x, nthreads=1)
    y4 = oracle.oracle_matvec(c1, x, nthreads=4)
    assert rel(y4, y1) <= 1e-15


@pytest.mark.parametrize("d,n,r,adm", [(2, 64, 8, "weak"), (3, 16, 4, "weak"), (2, 64, 4, "standard"),
                                       (1, 1024, 4, "standard")])
def test_p9_transpose(d, n, r, adm):
    """The factor set of K^T assembles to the transpose of K's assembled matrix,
    entry for entry, and the oracle satisfies <a, K b> = <K^T a, b>."""
    data = make_hmatrix(uniform_tree(d, n), r, kind="log", method="random", seed=13, admissibility=adm)
    dt = oracle.transposed(data)
    assert np.array_equal(oracle.assemble_dense(dt), oracle.assemble_dense(data).T)
    a = make_rhs(data.n, 2, 21).astype(np.float64)
    b = make_rhs(data.n, 2, 22).astype(np.float64)
    lhs = np.sum(a * oracle.oracle_matvec(data, b), axis=0)
    rhs = np.sum(oracle.oracle_matvec(dt, a) * b, axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=0)
