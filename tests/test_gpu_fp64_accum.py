"""GPU parity of the accuracy-check mode (HMAT_FLAG_FP64_ACCUM) against the FP64 oracle.

In this mode every product and sum of the path runs in FP64 on the device and
y is rounded to FP32 once. Products of the (dequantised) factors with FP32
vector entries are exact in FP64, so the device result must be the oracle's
FP64 value (over the same dequantised factors) rounded to FP32: every element
within one FP32 ulp of it, and nearly all of them equal to it. This bar leaves
no room for a dropped term, a wrong index or an inexact dequantisation,
which the 1e-5 bar of the FP32 mode could hide below its roundoff.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.quant import dequantised
from hmat_inputs import build_tree, make_hmatrix, make_rhs, uniform_tree
from hmat_testlib import assert_fp32_rounding_of, create, gpu_matvec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("c1-2d-n64-r16-svd", (64, 64), 16, "svd", "log"),
    ("2d-n256-r32-random", (256, 256), 32, "random", "log"),
    ("3d-n32-r8-random", (32, 32, 32), 8, "random", "inv"),
    ("ragged-100x37-r16", (100, 37), 16, "random", "log"),
    ("ragged-17x33x9-r8", (17, 33, 9), 8, "random", "inv"),
    ("2d-n8-L0", (8, 8), 4, "random", "log"),
    ("2d-n16-L1", (16, 16), 4, "random", "log"),
]


def _tree(shape):
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    return build_tree(shape, n_full=full)


@pytest.mark.parametrize("name,shape,r,method,kind", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16"])
def test_fp64_accum_is_rounded_oracle(name, shape, r, method, kind, form):
    _log(f"case fp64-accum {name} {form}")
    data = make_hmatrix(_tree(shape), r, kind=kind, method=method, seed=77)
    x = make_rhs(data.n, 1, 19)
    ref = oracle.oracle_matvec(dequantised(data, form), x)
    with create(data, storage=form, fp64_accum=True) as h:
        assert h.info["flags"] == 1
        y = gpu_matvec(h, x)
    assert_fp32_rounding_of(y, ref)


def test_fp64_accum_several_rhs_alpha_beta():
    _log("case fp64-accum nrhs=3 alpha/beta")
    data = make_hmatrix(uniform_tree(2, 128), 16, method="random", seed=3)
    x = make_rhs(data.n, 3, 4)
    y0 = np.random.default_rng(1).standard_normal((data.n, 3)).astype(np.float32)
    ref = oracle.oracle_matvec(data, x, alpha=0.75, beta=-1.5, y_in=y0)
    with create(data, max_nrhs=4, fp64_accum=True) as h:   # the mode ignores the multi-RHS layout
        y = gpu_matvec(h, x, alpha=0.75, beta=-1.5, y0=y0, ld_pad=7)
        assert_fp32_rounding_of(y, ref)
        y1 = gpu_matvec(h, x[:, 1:2], alpha=0.75, beta=-1.5, y0=y0[:, 1:2])
        assert np.array_equal(y1[:, 0], y[:, 1])


def test_fp32_mode_error_is_roundoff_of_fp64_mode():
    """The FP32 path differs from the FP64-accumulated one by FP32 roundoff only."""
    _log("case fp32 vs fp64-accum")
    data = make_hmatrix(uniform_tree(2, 256), 32, method="random", seed=8)
    x = make_rhs(data.n, 1, 6)
    with create(data) as h:
        y32 = gpu_matvec(h, x)
    with create(data, fp64_accum=True) as h:
        y64 = gpu_matvec(h, x)
    rel = np.linalg.norm(y32 - y64) / np.linalg.norm(y64)
    assert 0 < rel <= 1e-5, rel
