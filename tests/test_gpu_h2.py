"""GPU parity of the H^2 product (hmat_h2_*) against the FP64 H^2 oracle.

Bar, as for the H-matrix product: per right-hand side the relative 2-norm
error <= 1e-5 in FP32 storage and every element within 1e-4 of the column's
RMS; the FP16 form against the oracle over its exactly dequantised factors
(same bar: the kernels' own arithmetic) and within 1e-3 of the canonical one.
"""
import sys

import numpy as np
import pytest

import oracle.h2 as h2o
import paper_2008_12441_amd as hm
from hmat_inputs import build_tree, make_rhs, uniform_tree
from hmat_inputs.h2 import make_h2
from hmat_testlib import assert_close
from oracle.quant import _dequant_fp16

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
ELEM_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(h, x, *, alpha=1.0, beta=0.0, y0=None, ld_pad=0):
    import torch

    n, k = x.shape
    ld = n + ld_pad
    xd = torch.zeros((k, ld), dtype=torch.float32, device="cuda")
    xd[:, :n] = torch.from_numpy(np.ascontiguousarray(x.T))
    yd = torch.full((k, ld), float("nan"), dtype=torch.float32, device="cuda")
    if y0 is not None:
        yd[:, :n] = torch.from_numpy(np.ascontiguousarray(y0.T.astype(np.float32)))
    stream = torch.cuda.current_stream().cuda_stream
    hm.hmat_h2_matvec(h.handle, k, alpha, xd.data_ptr(), ld, beta, yd.data_ptr(), ld, stream)
    torch.cuda.synchronize()
    if ld_pad:
        assert np.isnan(yd[:, n:].cpu().numpy()).all(), "wrote outside the rows of y"
    return yd[:, :n].cpu().numpy().T.astype(np.float64)


def dequantised_h2(h2):
    """The H^2 factor set with every stored array (leaf U and V, E, F, S, D) replaced
    by its FP16-form value: one power-of-two scale per array (the rule of the FP16
    storage form), each entry rounded to FP16 after the scaling."""
    import copy

    out = copy.copy(h2)
    pool = h2.pool.copy()
    tree = h2.tree
    segs = []
    for t in range(tree.num_nodes):
        k = int(h2.rank[t])
        if k == 0:
            continue
        if h2.u_off[t] >= 0:
            segs += [(h2.u_off[t], tree.size(t) * k), (h2.v_off[t], tree.size(t) * k)]
        if h2.e_off[t] >= 0:
            kp = int(h2.rank[tree.parent[t]])
            segs += [(h2.e_off[t], k * kp), (h2.f_off[t], k * kp)]
    for b in range(len(h2.blocks)):
        t, s = int(h2.blocks.target[b]), int(h2.blocks.source[b])
        m = int(h2.rank[t] * h2.rank[s]) if h2.blocks.rank[b] > 0 else tree.size(t) * tree.size(s)
        segs.append((h2.blk_off[b], m))
    for o, m in segs:
        pool[int(o):int(o) + m] = _dequant_fp16(pool[int(o):int(o) + m])
    out.pool = pool
    return out


CASES = [
    # name, tree, rank (random fill) or q (Chebyshev), method, kind, admissibility
    ("2d-256x256-r16-random", lambda: uniform_tree(2, 256), 16, "random", "log", "weak"),
    ("2d-128x128-r32-random-standard", lambda: uniform_tree(2, 128), 32, "random", "log", "standard"),
    ("3d-32-r8-random", lambda: uniform_tree(3, 32), 8, "random", "inv", "weak"),
    ("3d-32-q3-cheb-inv", lambda: uniform_tree(3, 32), 3, "cheb", "inv", "weak"),
    ("2d-128-q5-cheb-log", lambda: uniform_tree(2, 128), 5, "cheb", "log", "weak"),
    ("2d-ragged-255x130-r12", lambda: build_tree((255, 130), n_full=(256, 256)), 12, "random", "log", "weak"),
    ("3d-ragged-61x20x47-r7", lambda: build_tree((61, 20, 47), n_full=(64, 64, 64)), 7, "random", "inv", "weak"),
    ("3d-ragged-17x33x9-r64-standard", lambda: build_tree((17, 33, 9), n_full=(64, 64, 64)), 64, "random", "inv",
     "standard"),
    ("1d-4096-r5", lambda: uniform_tree(1, 4096), 5, "random", "log", "weak"),
    ("2d-n8-L0", lambda: uniform_tree(2, 8), 4, "random", "log", "weak"),
    ("2d-n16-L1", lambda: uniform_tree(2, 16), 4, "random", "log", "weak"),
    ("2d-n32-L2", lambda: uniform_tree(2, 32), 4, "random", "log", "weak"),
]


def _make(tree, r, method, kind, adm, seed=7):
    if method == "cheb":
        return make_h2(tree, method="cheb", q=r, kind=kind, admissibility=adm)
    return make_h2(tree, method="random", rank=r, kind=kind, seed=seed, admissibility=adm)


@pytest.mark.parametrize("name,tree,r,method,kind,adm", CASES, ids=[c[0] for c in CASES])
def test_h2_fp32(name, tree, r, method, kind, adm):
    _log(f"case h2 fp32 {name}")
    h2 = _make(tree(), r, method, kind, adm)
    x = make_rhs(h2.n, 2, 13)
    ref = h2o.h2_oracle_matvec(h2, x)
    with hm.H2Matrix(h2, storage="fp32") as h:
        y = _run(h, x, ld_pad=3)
        y2 = _run(h, x, ld_pad=3)
    assert np.array_equal(y, y2), "not deterministic"
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


@pytest.mark.parametrize("name,tree,r,method,kind,adm", CASES[:6] + CASES[7:8], ids=[c[0] for c in CASES[:6] + CASES[7:8]])
def test_h2_fp16(name, tree, r, method, kind, adm):
    _log(f"case h2 fp16 {name}")
    h2 = _make(tree(), r, method, kind, adm)
    x = make_rhs(h2.n, 1, 14)
    with hm.H2Matrix(h2, storage="fp16") as h:
        y = _run(h, x)
    assert_close(y, h2o.h2_oracle_matvec(dequantised_h2(h2), x), FP32_TOL, ELEM_TOL)
    assert_close(y, h2o.h2_oracle_matvec(h2, x), 1e-3)


def test_h2_alpha_beta():
    _log("case h2 alpha/beta")
    h2 = make_h2(uniform_tree(2, 64), method="random", rank=8, seed=3)
    x = make_rhs(h2.n, 3, 4)
    y0 = np.random.default_rng(1).standard_normal((h2.n, 3))
    ref = h2o.h2_oracle_matvec(h2, x, alpha=-0.5, beta=2.0, y_in=y0.astype(np.float32))
    with hm.H2Matrix(h2) as h:
        y = _run(h, x, alpha=-0.5, beta=2.0, y0=y0)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_h2_info_counts():
    h2 = make_h2(uniform_tree(2, 128), method="random", rank=16, seed=2)
    from hmat_inputs.h2 import h2_stored_elements

    with hm.H2Matrix(h2) as h:
        info = h.info
    assert info["stored_elements"] == h2_stored_elements(h2.tree, h2.blocks, h2.rank) == h2.pool.size
    assert info["factor_bytes"] == 4 * h2.pool.size
    assert info["num_coupling_blocks"] == int((h2.blocks.rank > 0).sum())
    assert info["leaf_depth"] == h2.tree.leaf_depth and info["max_rank"] == 16


@pytest.fixture(scope="module")
def h2_c2_random():
    _log("building the 2D N = 2^20 H^2 factor set (rank 32, random fill) and its oracle product")
    h2 = make_h2(uniform_tree(2, 1024), method="random", rank=32, seed=9, device="cuda")
    x = make_rhs(h2.n, 1, 1002)
    bases = h2o.expanded_bases(h2)
    return h2, x, h2o.h2_oracle_matvec(h2, x, bases=bases)


def test_h2_c2_full_size_fp32(h2_c2_random):
    h2, x, ref = h2_c2_random
    _log("case h2 c2 size fp32")
    with hm.H2Matrix(h2) as h:
        y = _run(h, x)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_h2_c2_full_size_fp16(h2_c2_random):
    h2, x, ref = h2_c2_random
    _log("case h2 c2 size fp16")
    with hm.H2Matrix(h2, storage="fp16") as h:
        y = _run(h, x)
    assert_close(y, h2o.h2_oracle_matvec(dequantised_h2(h2), x), FP32_TOL, ELEM_TOL)
    assert_close(y, ref, 1e-3)
