"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: per RHS column the relative 2-norm error is <= 1e-5 for FP32 storage,
and every element is within 1e-4 of the column's RMS (an error confined to a
few rows cannot hide in the norm). FP16 storage is compared against the
oracle over the exactly dequantised factors (same bar: the kernel's own
arithmetic) and against the canonical FP32 factors (<= 1e-3, the stated bound
of the form).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.quant import dequantised
from hmat_inputs import build_tree, make_hmatrix, make_rhs, uniform_tree
from hmat_testlib import assert_close, assert_fp32_rounding_of, create, gpu_matvec, rel_err_cols

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
ELEM_TOL = 1e-4
# The multi-RHS BF16 form feeds MFMA with activations split into two BF16
# parts (16 significant bits), so its own arithmetic error is ~2^-16 relative
# per product instead of ~2^-22 for the FP16 hi+lo split.
KERNEL_TOL = {"fp32": 1e-5, "fp16": 1e-5, "bf16": 3e-5, "fp8": 1e-5, "fp8_f16d": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


UNIFORM = [
    ("c1-2d-n64-r16-svd", 2, 64, 16, "svd", "log"),
    ("2d-n128-r8-random", 2, 128, 8, "random", "log"),
    ("2d-n256-r32-random", 2, 256, 32, "random", "log"),
    ("3d-n32-r8-random", 3, 32, 8, "random", "inv"),
    ("3d-n16-r8-svd", 3, 16, 8, "svd", "inv"),
    ("1d-n4096-r4-random", 1, 4096, 4, "random", "log"),
    ("2d-n8-L0", 2, 8, 4, "random", "log"),
    ("2d-n16-L1", 2, 16, 4, "random", "log"),
]


@pytest.mark.parametrize("name,d,n,r,method,kind", UNIFORM, ids=[u[0] for u in UNIFORM])
def test_uniform_fp32(name, d, n, r, method, kind):
    _log(f"case {name}")
    data = make_hmatrix(uniform_tree(d, n), r, kind=kind, method=method, seed=5)
    x = make_rhs(data.n, 1, 17)
    ref = oracle.oracle_matvec(data, x)
    with create(data, max_nrhs=1) as h:      # single-RHS layout and kernels
        y = gpu_matvec(h, x)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_single_rhs_alpha_beta_leading_dimension():
    _log("case single-rhs alpha/beta")
    data = make_hmatrix(uniform_tree(2, 64), 16, method="random", seed=4)
    x = make_rhs(data.n, 1, 8)
    y0 = np.random.default_rng(0).standard_normal((data.n, 1))
    ref = oracle.oracle_matvec(data, x, alpha=-0.5, beta=2.0, y_in=y0.astype(np.float32))
    with create(data, max_nrhs=1) as h:
        y = gpu_matvec(h, x, alpha=-0.5, beta=2.0, y0=y0, ld_pad=5)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


RAGGED = [((40, 23), 8), ((9, 30, 5), 4), ((100, 37), 16), ((17, 33, 9), 8), ((3, 3), 2),
          ((255, 130), 32), ((61, 20, 47), 8)]


@pytest.mark.parametrize("shape,r", RAGGED, ids=[f"{'x'.join(map(str, s))}-r{r}" for s, r in RAGGED])
def test_ragged_subgrids_fp32(shape, r):
    _log(f"case ragged {shape} r={r}")
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    tree = build_tree(shape, n_full=full, offset=(1,) * len(shape) if max(shape) < full[0] else None)
    data = make_hmatrix(tree, r, kind="log" if len(shape) == 2 else "inv", method="random", seed=9)
    x = make_rhs(data.n, 1, 3)
    ref = oracle.oracle_matvec(data, x)
    with create(data) as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_multi_rhs_leading_dimension_and_alpha_beta():
    _log("case multi-rhs/alpha-beta")
    data = make_hmatrix(uniform_tree(2, 64), 16, method="random", seed=4)
    x = make_rhs(data.n, 3, 8)
    y0 = np.random.default_rng(0).standard_normal((data.n, 3))
    ref = oracle.oracle_matvec(data, x, alpha=-0.5, beta=2.0, y_in=y0.astype(np.float32))
    with create(data, max_nrhs=3) as h:
        y = gpu_matvec(h, x, alpha=-0.5, beta=2.0, y0=y0, ld_pad=5)
        assert_close(y, ref, FP32_TOL, ELEM_TOL)
        # columns agree with single-RHS runs bit for bit
        for j in range(3):
            yj = gpu_matvec(h, x[:, j:j + 1], alpha=-0.5, beta=2.0, y0=y0[:, j:j + 1])
            assert np.array_equal(yj[:, 0], y[:, j])


def test_deterministic_bitwise():
    _log("case determinism")
    data = make_hmatrix(uniform_tree(2, 128), 8, method="random", seed=6)
    x = make_rhs(data.n, 1, 2)
    with create(data) as h:
        y1 = gpu_matvec(h, x)
        y2 = gpu_matvec(h, x)
    assert np.array_equal(y1, y2)


def test_fp16_scaled_storage():
    _log("case fp16 c1")
    data = make_hmatrix(uniform_tree(2, 64), 16, method="svd")
    x = make_rhs(data.n, 1, 1001)
    ref = oracle.oracle_matvec(data, x)
    ref_dq = oracle.oracle_matvec(dequantised(data, "fp16"), x)
    with create(data, storage="fp16") as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref_dq, FP32_TOL, ELEM_TOL)
    err = assert_close(y, ref, 1e-3)
    _log(f"fp16 error vs canonical oracle {err:.3e}")


def test_bf16_storage_single_rhs():
    _log("case bf16 c1")
    data = make_hmatrix(uniform_tree(2, 64), 16, method="svd")
    x = make_rhs(data.n, 1, 1001)
    ref_dq = oracle.oracle_matvec(dequantised(data, "bf16"), x)
    with create(data, storage="bf16") as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref_dq, FP32_TOL, ELEM_TOL)
    err = assert_close(y, oracle.oracle_matvec(data, x), 1e-2)
    _log(f"bf16 error vs canonical oracle {err:.3e}")


@pytest.mark.parametrize("shape,r", [((40, 23), 8), ((17, 33, 9), 8)])
def test_fp16_ragged(shape, r):
    _log(f"case fp16 ragged {shape}")
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    tree = build_tree(shape, n_full=full)
    data = make_hmatrix(tree, r, kind="log" if len(shape) == 2 else "inv", method="random", seed=12)
    x = make_rhs(data.n, 1, 5)
    ref_dq = oracle.oracle_matvec(dequantised(data, "fp16"), x)
    with create(data, storage="fp16") as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref_dq, FP32_TOL, ELEM_TOL)


@pytest.fixture(scope="module")
def c2_random():
    _log("building c2-size factor set (2D, N=2^20, rank 32, random fill)")
    data = make_hmatrix(uniform_tree(2, 1024), 32, method="random", seed=21)
    prep = oracle.prepare(data)
    return data, prep


def test_c2_full_size_fp32(c2_random):
    data, prep = c2_random
    _log("case c2 fp32 full size")
    x = make_rhs(data.n, 1, 1002)
    ref = oracle.oracle_matvec(prep, x)
    with create(data) as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_c2_full_size_fp64_accum(c2_random):
    data, prep = c2_random
    _log("case c2 fp32 storage, FP64 accumulation, full size")
    x = make_rhs(data.n, 1, 1002)
    ref = oracle.oracle_matvec(prep, x)
    with create(data, fp64_accum=True) as h:
        y = gpu_matvec(h, x)
    assert_fp32_rounding_of(y, ref)


def test_c2_full_size_fp16(c2_random):
    data, _ = c2_random
    _log("case c2 fp16 full size")
    x = make_rhs(data.n, 1, 1002)
    ref_dq = oracle.oracle_matvec(dequantised(data, "fp16"), x)
    with create(data, storage="fp16") as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref_dq, FP32_TOL, ELEM_TOL)


# ---------------------------------------------------------------------------
# Multi-RHS handles (max_nrhs > 1): the MFMA layout and kernels.
# ---------------------------------------------------------------------------
MR_CASES = [
    ("c1-2d-n64-r16-svd-k3", (64, 64), 16, "svd", 3),
    ("2d-n128-r8-random-k17", (128, 128), 8, "random", 17),
    ("3d-n32-r16-random-k64", (32, 32, 32), 16, "random", 64),
    ("3d-n16-r8-random-k5", (16, 16, 16), 8, "random", 5),
    ("ragged-40x23-r8-k5", (40, 23), 8, "random", 5),
    ("ragged-17x33x9-r8-k16", (17, 33, 9), 8, "random", 16),
    ("ragged-255x130-r32-k33", (255, 130), 32, "random", 33),
    ("2d-n8-L0-k2", (8, 8), 4, "random", 2),
    ("2d-n16-L1-k2", (16, 16), 4, "random", 2),
]


def _tree_for(shape):
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    return build_tree(shape, n_full=full)


@pytest.mark.parametrize("name,shape,r,method,k", MR_CASES, ids=[c[0] for c in MR_CASES])
@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16", "fp8", "fp8_f16d"])
def test_multi_rhs(name, shape, r, method, k, form):
    _log(f"case multi-rhs {name} {form}")
    kind = "log" if len(shape) == 2 else "inv"
    data = make_hmatrix(_tree_for(shape), r, kind=kind, method=method, seed=31)
    x = make_rhs(data.n, k, 41)
    ref_data = dequantised(data, form)
    ref = oracle.oracle_matvec(ref_data, x)
    with create(data, storage=form, max_nrhs=k) as h:
        y = gpu_matvec(h, x, ld_pad=3)
    assert_close(y, ref, KERNEL_TOL[form], 10 * KERNEL_TOL[form])
    if form == "fp16":
        assert_close(y, oracle.oracle_matvec(data, x), 1e-3)
    elif form.startswith("fp8"):   # the form's own quantisation error is reported, not gated
        ref0 = oracle.oracle_matvec(data, x)
        _log(f"{form} error vs canonical oracle {np.max(rel_err_cols(y, ref0)):.3e}")


@pytest.mark.parametrize("form", ["fp32", "fp16"])
def test_multi_rhs_groups_alpha_beta_and_fewer_columns(form):
    _log(f"case multi-rhs groups {form}")
    data = make_hmatrix(uniform_tree(2, 64), 16, method="random", seed=8)
    x = make_rhs(data.n, 130, 9)           # two groups: 128 + 2
    y0 = np.random.default_rng(3).standard_normal((data.n, 130))
    ref_data = dequantised(data, form)
    ref = oracle.oracle_matvec(ref_data, x, alpha=0.5, beta=-1.25, y_in=y0.astype(np.float32))
    with create(data, storage=form, max_nrhs=130) as h:
        y = gpu_matvec(h, x, alpha=0.5, beta=-1.25, y0=y0)
        assert_close(y, ref, FP32_TOL, ELEM_TOL)
        # fewer columns than max_nrhs, and a single column, on the same handle
        y7 = gpu_matvec(h, x[:, :7])
        assert_close(y7, oracle.oracle_matvec(ref_data, x[:, :7]), FP32_TOL, ELEM_TOL)
        y1 = gpu_matvec(h, x[:, :1])
        assert_close(y1, oracle.oracle_matvec(ref_data, x[:, :1]), FP32_TOL, ELEM_TOL)
        # deterministic
        y7b = gpu_matvec(h, x[:, :7])
        assert np.array_equal(y7, y7b)


@pytest.fixture(scope="module")
def c3_random():
    _log("building c3-size factor set (3D, N=64^3, rank 64, random fill)")
    data = make_hmatrix(uniform_tree(3, 64), 64, kind="inv", method="random", seed=23)
    return data


@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16", "fp8", "fp8_f16d"])
def test_c3_full_size_multi_rhs(c3_random, form):
    data = c3_random
    _log(f"case c3 {form} full size, 64 RHS")
    x = make_rhs(data.n, 64, 1003)
    ref = oracle.oracle_matvec(dequantised(data, form), x)
    with create(data, storage=form, max_nrhs=64) as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref, KERNEL_TOL[form], 10 * KERNEL_TOL[form])


@pytest.fixture(scope="module")
def c5_random():
    """The 3D 128^3 structure (N = 2^21, rank 32) with random fills drawn on the
    GPU, 128 right-hand sides, and the FP64 oracle's y over the canonical and
    over the dequantised FP16 factors (all columns)."""
    _log("building c5-size factor set (3D, N=128^3, rank 32, random fill) and its oracle products")
    data = make_hmatrix(uniform_tree(3, 128), 32, kind="inv", method="random", seed=25, device="cuda")
    x = make_rhs(data.n, 128, 1005)
    ref = oracle.oracle_matvec(data, x)
    ref16 = oracle.oracle_matvec(dequantised(data, "fp16"), x)
    return data, x, ref, ref16


@pytest.mark.parametrize("form", ["fp32", "fp16"])
def test_c5_full_size_multi_rhs(c5_random, form):
    """Every column of every 16-column n-tile at the 3D N = 2^21, 128-RHS size."""
    data, x, ref, ref16 = c5_random
    _log(f"case c5 {form} full size, 128 RHS")
    with create(data, storage=form, max_nrhs=128) as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref if form == "fp32" else ref16, KERNEL_TOL[form], 10 * KERNEL_TOL[form])
    if form == "fp16":
        assert_close(y, ref, 1e-3)
