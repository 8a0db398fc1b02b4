"""GPU parity of hmat_compress (construction of the block factors) against the
construction oracle (oracle/compress.py, FP64).

Dense blocks: every entry within 4e-6 x max(1, |K|) of the FP64 entry (FP32
coordinates and distance, logf / rsqrtf within a few ulp).

Low-rank blocks: the factors are not unique, so the product U V^T is compared.
Both sides approximate the same block K from the same Rademacher sample; with
e_o = ||K - U_o V_o^T||_F the oracle's error, the GPU product must satisfy
||U V^T - U_o V_o^T||_F <= 2 e_o + 1e-5 ||K||_F and ||K - U V^T||_F <=
1.5 e_o + 1e-5 ||K||_F: FP32 entries and sample products put its floor near
1e-6 ||K||_F, and the rank-r truncation may pick a different direction where
two singular values of the sample are close (a difference of the size of the
truncation error itself). Where the block's numerical rank is below r both
errors are at the FP32 floor, so the comparison is then a tight one. The
balanced split is checked too: U^T U and V^T V have the same diagonal.

End to end: the constructed factors go through hmat_create and hmat_matvec,
checked against the FP64 product over the same factors, and the product is
as accurate (against the dense kernel matrix) as the oracle's factors.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2008_12441_amd as hm
from hmat_inputs import HMatrixData, build_tree, enumerate_blocks, make_rhs, uniform_tree
from hmat_testlib import assert_close, create, gpu_matvec
from oracle import compress as oc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tree(shape):
    if len(set(shape)) == 1 and shape[0] & (shape[0] - 1) == 0:
        return uniform_tree(len(shape), shape[0])
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    return build_tree(shape, n_full=full, offset=(1,) * len(shape))


def _blocks(tree, rank, adm):
    bl = enumerate_blocks(tree, rank, adm)
    sz = tree.end - tree.begin
    r = np.minimum(bl.rank, np.minimum(sz[bl.target], sz[bl.source])).astype(np.int32)
    return bl.target, bl.source, r


def _gpu_compress(tree, target, source, rank, kind, oversample, seed):
    return hm.compress_pool(tree.parent, tree.begin, tree.end, target, source, rank, tree.points, kernel=kind,
                            diag=1.0, oversample=oversample, seed=seed)


def _check_blocks(tree, target, source, rank, kind, oversample, seed, pool, off_a):
    sz = tree.end - tree.begin
    ref = oc.compress(tree.points, tree.begin, tree.end, zip(target, source, rank), kind, 1.0, oversample, seed)
    worst = 0.0
    for b, f in enumerate(ref):
        t, s, r = int(target[b]), int(source[b]), int(rank[b])
        m, n = int(sz[t]), int(sz[s])
        k = oc.block_entries(tree.points, tree.begin[t], tree.end[t], tree.begin[s], tree.end[s], kind, 1.0)
        o = int(off_a[b])
        if r == 0:
            d = pool[o:o + m * n].reshape(n, m).T.astype(np.float64)
            err = np.max(np.abs(d - k) / np.maximum(1.0, np.abs(k)))
            assert err <= 4e-6, f"dense block {b} ({t}, {s}): entry error {err:.2e}"
            continue
        u = pool[o:o + m * r].reshape(r, m).T.astype(np.float64)
        v = pool[o + m * r:o + (m + n) * r].reshape(r, n).T.astype(np.float64)
        a = u @ v.T
        ao = f[1] @ f[2].T
        kn = np.linalg.norm(k)
        eo = np.linalg.norm(k - ao)
        diff = np.linalg.norm(a - ao)
        eg = np.linalg.norm(k - a)
        assert diff <= 2 * eo + 1e-5 * kn, f"block {b} ({t}, {s}) r={r}: |UV'-UoVo'| {diff:.2e}, e_o {eo:.2e}"
        assert eg <= 1.5 * eo + 1e-5 * kn, f"block {b} ({t}, {s}) r={r}: error {eg:.2e} vs oracle {eo:.2e}"
        du, dv = np.diag(u.T @ u), np.diag(v.T @ v)
        assert np.allclose(du, dv, rtol=1e-3, atol=1e-5 * kn), f"block {b}: split not balanced"
        worst = max(worst, diff / kn)
    return worst


CASES = [((32, 32), 8, "weak", "log", 10), ((64, 64), 16, "weak", "log", 10), ((16, 16, 16), 8, "weak", "inv", 10),
         ((40, 23), 8, "standard", "log", 10), ((16, 16, 16), 4, "standard", "inv", 2), ((64, 64), 64, "weak", "log", 10),
         ((32, 32), 8, "weak", "log", 0), ((17, 33, 9), 8, "weak", "inv", 5), ((100, 37), 16, "weak", "log", 80)]
IDS = [f"{'x'.join(map(str, s))}-r{r}-{a}-{k}-p{p}" for s, r, a, k, p in CASES]


@pytest.mark.parametrize("shape,rank,adm,kind,p", CASES, ids=IDS)
def test_compress_blocks(shape, rank, adm, kind, p):
    _log(f"case compress {shape} rank {rank} {adm} {kind} oversample {p}")
    tree = _tree(shape)
    target, source, r = _blocks(tree, rank, adm)
    pool, off_a, _ = _gpu_compress(tree, target, source, r, kind, p, 21)
    assert np.isfinite(pool).all()
    _check_blocks(tree, target, source, r, kind, p, 21, pool, off_a)


def test_compress_deterministic_and_seeded():
    _log("case compress determinism")
    tree = _tree((32, 32))
    target, source, r = _blocks(tree, 8, "weak")
    a, _, _ = _gpu_compress(tree, target, source, r, "log", 10, 3)
    b, _, _ = _gpu_compress(tree, target, source, r, "log", 10, 3)
    c, _, _ = _gpu_compress(tree, target, source, r, "log", 10, 4)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


@pytest.mark.parametrize("shape,rank,adm,kind", [((64, 64), 16, "weak", "log"), ((16, 16, 16), 8, "standard", "inv")],
                         ids=["64x64-weak-log", "16^3-standard-inv"])
def test_compress_then_matvec(shape, rank, adm, kind):
    _log(f"case compress then matvec {shape} {adm} {kind}")
    tree = _tree(shape)
    target, source, r = _blocks(tree, rank, adm)
    pool, off_a, off_b = _gpu_compress(tree, target, source, r, kind, 10, 5)
    from hmat_inputs.tree import BlockList

    data = HMatrixData(tree, BlockList(target, source, r), pool, off_a, off_b, kind, "gpu-rsvd")
    x = make_rhs(data.n, 2, 77)
    with create(data, max_nrhs=2) as h:
        y = gpu_matvec(h, x)
    ref = oracle.oracle_matvec(data, x)
    assert_close(y, ref, 1e-5, 1e-4)
    # accuracy against the dense kernel matrix, next to the oracle's own factors
    kfull = oc.block_entries(tree.points, 0, tree.n, 0, tree.n, kind, 1.0)
    exact = kfull @ x.astype(np.float64)
    ofac = oc.compress(tree.points, tree.begin, tree.end, zip(target, source, r), kind, 1.0, 10, 5)
    y_or = np.zeros_like(exact)
    for (t, s, rr), f in zip(zip(target, source, r), ofac):
        t0, t1, s0, s1 = tree.begin[t], tree.end[t], tree.begin[s], tree.end[s]
        if rr == 0:
            y_or[t0:t1] += f[1] @ x[s0:s1]
        else:
            y_or[t0:t1] += f[1] @ (f[2].T @ x[s0:s1])
    e_gpu = np.linalg.norm(y - exact) / np.linalg.norm(exact)
    e_or = np.linalg.norm(y_or - exact) / np.linalg.norm(exact)
    assert e_gpu <= 1.5 * e_or + 1e-5, (e_gpu, e_or)


@pytest.fixture(scope="module")
def c2_gpu():
    _log("compressing the 2D 1024^2 weak-admissibility structure on the GPU (rank 32, oversample 10)")
    tree = uniform_tree(2, 1024)
    target, source, r = _blocks(tree, 32, "weak")
    t0 = time.perf_counter()
    pool, off_a, off_b = _gpu_compress(tree, target, source, r, "log", 10, 1002)
    _log(f"hmat_compress: {time.perf_counter() - t0:.2f} s including the copies to host memory")
    return tree, target, source, r, pool, off_a, off_b


def test_c2_full_size_compress(c2_gpu):
    """Full c2 size: every low-rank block the oracle can afford (up to 4096 rows) at
    the lowest three levels against the oracle, sampled dense blocks, sampled rows
    of the upper levels against exact FP64 kernel rows (a sanity bound: wrong
    points or indices give errors of order one), and the product through
    hmat_matvec against the FP64 product over the same factors."""
    tree, target, source, r, pool, off_a, off_b = c2_gpu
    assert np.isfinite(pool).all()
    sz = tree.end - tree.begin
    rng = np.random.default_rng(8)
    pick = []
    for size in (256, 1024, 4096):
        idx = np.nonzero((r > 0) & (sz[target] == size))[0]
        pick += list(rng.choice(idx, size=2, replace=False))
    pick += list(rng.choice(np.nonzero(r == 0)[0], size=8, replace=False))
    pick = np.array(pick)
    _log(f"case c2 compress: {len(pick)} blocks against the oracle")
    _check_blocks(tree, target[pick], source[pick], r[pick], "log", 10, 1002, pool, off_a[pick])
    for size in (16384, 65536, 262144):
        for b in rng.choice(np.nonzero((r > 0) & (sz[target] == size))[0], size=2, replace=False):
            t, s, rr = int(target[b]), int(source[b]), int(r[b])
            m, n = int(sz[t]), int(sz[s])
            o = int(off_a[b])
            u = pool[o:o + m * rr].reshape(rr, m).T.astype(np.float64)
            v = pool[o + m * rr:o + (m + n) * rr].reshape(rr, n).T.astype(np.float64)
            for i in rng.choice(m, size=4, replace=False):
                gi = int(tree.begin[t]) + int(i)
                k = oc.block_entries(tree.points, gi, gi + 1, tree.begin[s], tree.end[s], "log", 1.0)[0]
                e = np.linalg.norm(u[i] @ v.T - k) / np.linalg.norm(k)
                assert e <= 5e-2, f"block {b} ({t}, {s}) row {i}: relative error {e:.2e}"
    _log("case c2 compress: product through hmat_matvec")
    from hmat_inputs.tree import BlockList

    data = HMatrixData(tree, BlockList(target, source, r), pool, off_a, off_b, "log", "gpu-rsvd")
    x = make_rhs(data.n, 1, 1002)
    with create(data) as h:
        y = gpu_matvec(h, x)
    assert_close(y, oracle.oracle_matvec(data, x), 1e-5, 1e-4)


def _single_block(n, d):
    from hmat_inputs.tree import BlockList

    tree = build_tree((n,) * d if d > 1 else (n,), n_full=(max(n, 8),) * d)
    return tree, BlockList(np.array([0], np.int32), np.array([0], np.int32), np.array([0], np.int32))


def test_compress_root_leaf_and_dense_only():
    """A root that is a leaf (one dense block (0, 0) carrying the diagonal
    value), and a one-level tree (dense blocks only)."""
    _log("case compress root leaf")
    tree, bl = _single_block(7, 2)  # 49 points, one leaf
    assert tree.leaf_depth == 0
    pool, off_a, _ = hm.compress_pool(tree.parent, tree.begin, tree.end, bl.target, bl.source, bl.rank, tree.points,
                                      kernel="inv", diag=0.5, oversample=4, seed=1)
    k = oc.block_entries(tree.points, 0, tree.n, 0, tree.n, "inv", 0.5)
    d = pool.reshape(tree.n, tree.n).T.astype(np.float64)
    assert np.all(np.diag(d) == 0.5)
    assert np.max(np.abs(d - k) / np.maximum(1.0, np.abs(k))) <= 4e-6
    _log("case compress dense only (16 x 16, four leaves)")
    tree = uniform_tree(2, 16)
    target, source, r = _blocks(tree, 8, "weak")
    assert np.all(r == 0)
    pool, off_a, _ = _gpu_compress(tree, target, source, r, "log", 10, 2)
    _check_blocks(tree, target, source, r, "log", 10, 2, pool, off_a)


def test_compress_full_rank_blocks_are_exact():
    """Where rank = min(|t|, |s|) the sample spans the whole range of the block,
    so U V^T reproduces K to FP32 accuracy whatever the truncation (a tight
    check of the sample, orthonormalisation and projection kernels)."""
    _log("case compress full-rank blocks")
    tree = _tree((100, 37))  # ragged: boxes of 48 to 96 points above the leaves
    sz = tree.end - tree.begin
    target, source, r = _blocks(tree, 96, "weak")
    full = (r > 0) & (r == np.minimum(sz[target], sz[source])) & (np.minimum(sz[target], sz[source]) <= 96)
    assert full.any()
    keep = (r == 0) | full
    target, source, r = target, source, np.where(keep, r, np.minimum(r, 8)).astype(np.int32)
    pool, off_a, _ = _gpu_compress(tree, target, source, r, "log", 0, 6)
    for b in np.nonzero(full)[0]:
        t, s, rr = int(target[b]), int(source[b]), int(r[b])
        m, n = int(sz[t]), int(sz[s])
        o = int(off_a[b])
        u = pool[o:o + m * rr].reshape(rr, m).T.astype(np.float64)
        v = pool[o + m * rr:o + (m + n) * rr].reshape(rr, n).T.astype(np.float64)
        k = oc.block_entries(tree.points, tree.begin[t], tree.end[t], tree.begin[s], tree.end[s], "log", 1.0)
        e = np.linalg.norm(u @ v.T - k) / np.linalg.norm(k)
        assert e <= 2e-5, f"block {b} ({t}, {s}) |t|={m} |s|={n} r={rr}: {e:.2e}"
