"""hmat_matvec_noalloc through the C ABI: the same y as hmat_matvec, bitwise.

The entry point keeps its workspace in the library's static scratch array,
which holds the previous call's values; two calls in a row, the second on a
smaller matrix, check that every workspace value is written before it is read.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2008_12441_amd as hm
from hmat_inputs import build_tree, make_hmatrix, make_rhs, uniform_tree
from hmat_testlib import assert_close, create

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(h, x, entry, *, alpha=1.0, beta=0.0, y0=None):
    """y of one product on cuda:0 through `entry` (hmat_matvec or hmat_matvec_noalloc)."""
    import torch

    n, k = x.shape
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    if y0 is None:
        yd = torch.full((k, n), float("nan"), dtype=torch.float32, device="cuda")
    else:
        yd = torch.from_numpy(np.ascontiguousarray(y0.T.astype(np.float32))).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    entry(h.handle, k, alpha, xd.data_ptr(), n, beta, yd.data_ptr(), n, stream)
    torch.cuda.synchronize()
    return yd.cpu().numpy().T.copy()


CASES = [
    # (name, tree, rank, storage, fp64 accumulation, right-hand sides, alpha, beta): larger first
    ("2d-256x256-r16-fp32", lambda: uniform_tree(2, 256), 16, "fp32", False, 1, 1.0, 0.0),
    ("3d-40x23x17-r8-fp16", lambda: build_tree((40, 23, 17)), 8, "fp16", False, 1, -0.5, 2.0),
    ("2d-100x37-r8-fp64acc-k2", lambda: build_tree((100, 37)), 8, "fp32", True, 2, 1.0, 0.0),
    ("2d-64x64-r8-bf16", lambda: uniform_tree(2, 64), 8, "bf16", False, 1, 1.0, 0.0),
]


@pytest.mark.parametrize("name,tree,rank,storage,fp64,k,alpha,beta", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_matvec(name, tree, rank, storage, fp64, k, alpha, beta):
    _log(f"case {name}")
    data = make_hmatrix(tree(), rank, method="random", seed=11)
    x = make_rhs(data.n, k, 23)
    y0 = np.random.default_rng(3).standard_normal((data.n, k)).astype(np.float32)
    with create(data, storage=storage, max_nrhs=k, fp64_accum=fp64) as h:
        info = hm.hmat_get_info(h.handle)
        assert info["workspace_bytes"] <= hm.HMAT_NOALLOC_SCRATCH_BYTES
        y_ref = _run(h, x, hm.hmat_matvec, alpha=alpha, beta=beta, y0=y0)
        y1 = _run(h, x, hm.hmat_matvec_noalloc, alpha=alpha, beta=beta, y0=y0)
        y2 = _run(h, x, hm.hmat_matvec_noalloc, alpha=alpha, beta=beta, y0=y0)
    assert np.array_equal(y1, y_ref), "noalloc differs from hmat_matvec"
    assert np.array_equal(y2, y_ref), "second noalloc call differs"
    if storage == "fp32":
        ref = oracle.oracle_matvec(data, x, alpha=alpha, beta=beta, y_in=y0)
        assert_close(y1.astype(np.float64), ref, 1e-5, 1e-4)


def test_noalloc_two_calls_second_smaller():
    """A large product fills the scratch with its values; a smaller one right after must not see them."""
    _log("case two calls, second smaller")
    big = make_hmatrix(uniform_tree(2, 256), 32, method="random", seed=21)
    small = make_hmatrix(build_tree((61, 20, 47)), 8, method="random", seed=22)
    xb = make_rhs(big.n, 1, 31)
    xs = make_rhs(small.n, 1, 32)
    with create(big) as hb, create(small) as hs:
        yb_ref = _run(hb, xb, hm.hmat_matvec)
        ys_ref = _run(hs, xs, hm.hmat_matvec)
        yb = _run(hb, xb, hm.hmat_matvec_noalloc)
        ys = _run(hs, xs, hm.hmat_matvec_noalloc)
    assert np.array_equal(yb, yb_ref)
    assert np.array_equal(ys, ys_ref)
    assert_close(ys.astype(np.float64), oracle.oracle_matvec(small, xs), 1e-5, 1e-4)


def test_noalloc_rejects_multi_rhs_handles():
    _log("case multi-RHS handle rejected")
    data = make_hmatrix(uniform_tree(2, 64), 8, method="random", seed=12)
    x = make_rhs(data.n, 2, 5)
    with create(data, storage="fp32", max_nrhs=2) as h:
        with pytest.raises(hm.HmatError) as e:
            _run(h, x, hm.hmat_matvec_noalloc)
    assert e.value.status == 4  # HMAT_ERR_UNSUPPORTED
