"""GPU parity under standard admissibility (Sec. 2, Def. "Standard admissibility
condition", rho = sqrt(d)): low-rank blocks between non-neighbouring boxes whose
parents are neighbours, dense blocks between every leaf and the leaves of its
parent's neighbours. Same bar as the weak-admissibility parity tests: against
the FP64 oracle over the (dequantised) factors, per column relative 2-norm
error and per element against the column's RMS. The batched launch must give
each member bit for bit what its own hmat_matvec gives.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2008_12441_amd as hm
from oracle.quant import dequantised
from hmat_inputs import build_tree, make_hmatrix, make_rhs, uniform_tree
from hmat_testlib import assert_close, assert_fp32_rounding_of, create, gpu_matvec

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
ELEM_TOL = 1e-4
KERNEL_TOL = {"fp32": 1e-5, "fp16": 1e-5, "bf16": 3e-5, "fp8": 1e-5, "fp8_f16d": 1e-5}


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
    return build_tree(shape, n_full=full, offset=(1,) * len(shape) if max(shape) < full[0] else None)


def _data(shape, r, seed):
    kind = "inv" if len(shape) == 3 else "log"
    return make_hmatrix(_tree(shape), r, kind=kind, method="random", seed=seed, admissibility="standard")


SHAPES = [((64, 64), 8), ((128, 128), 4), ((256, 256), 8), ((16, 16, 16), 4), ((32, 32, 32), 4),
          ((4096,), 4), ((16, 16), 4), ((8, 8), 4), ((40, 23), 8), ((9, 30, 5), 4), ((100, 37), 16),
          ((17, 33, 9), 8), ((255, 130), 8), ((61, 20, 47), 4)]
IDS = [f"{'x'.join(map(str, s))}-r{r}" for s, r in SHAPES]


@pytest.mark.parametrize("shape,r", SHAPES, ids=IDS)
def test_standard_fp32(shape, r):
    _log(f"case standard fp32 {shape} r={r}")
    data = _data(shape, r, 51)
    x = make_rhs(data.n, 1, 52)
    ref = oracle.oracle_matvec(data, x)
    with create(data) as h:
        y = gpu_matvec(h, x, ld_pad=3)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


@pytest.mark.parametrize("form", ["fp16", "bf16"])
@pytest.mark.parametrize("shape,r", [((64, 64), 8), ((40, 23), 8), ((17, 33, 9), 8), ((32, 32, 32), 4)],
                         ids=["64x64", "40x23", "17x33x9", "32^3"])
def test_standard_16bit_single_rhs(shape, r, form):
    _log(f"case standard {form} {shape}")
    data = _data(shape, r, 53)
    x = make_rhs(data.n, 1, 54)
    with create(data, storage=form) as h:
        y = gpu_matvec(h, x)
    assert_close(y, oracle.oracle_matvec(dequantised(data, form), x), FP32_TOL, ELEM_TOL)


@pytest.mark.parametrize("shape,r", [((128, 128), 8), ((17, 33, 9), 8)], ids=["128x128", "17x33x9"])
def test_standard_fp64_accum(shape, r):
    _log(f"case standard fp64 accumulation {shape}")
    data = _data(shape, r, 55)
    x = make_rhs(data.n, 1, 56)
    ref = oracle.oracle_matvec(data, x, alpha=0.75, beta=-0.5, y_in=np.ones((data.n, 1), np.float32))
    with create(data, fp64_accum=True) as h:
        y = gpu_matvec(h, x, alpha=0.75, beta=-0.5, y0=np.ones((data.n, 1)))
    assert_fp32_rounding_of(y, ref)


MR = [((64, 64), 8, 5), ((16, 16, 16), 4, 17), ((40, 23), 8, 3), ((128, 128), 4, 33), ((9, 30, 5), 4, 16)]


@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16", "fp8", "fp8_f16d"])
@pytest.mark.parametrize("shape,r,k", MR, ids=[f"{'x'.join(map(str, s))}-k{k}" for s, _, k in MR])
def test_standard_multi_rhs(shape, r, k, form):
    _log(f"case standard multi-rhs {shape} k={k} {form}")
    data = _data(shape, r, 57)
    x = make_rhs(data.n, k, 58)
    with create(data, storage=form, max_nrhs=k) as h:
        y = gpu_matvec(h, x, ld_pad=2)
    assert_close(y, oracle.oracle_matvec(dequantised(data, form), x), KERNEL_TOL[form], 10 * KERNEL_TOL[form])


def test_standard_and_weak_members_in_one_batch():
    import torch

    _log("case batch with standard and weak members")
    specs = [((64, 64), 8, "standard", 1), ((40, 23), 8, "weak", 1), ((17, 33, 9), 8, "standard", 1),
             ((16, 16, 16), 4, "standard", 5), ((64, 64), 8, "standard", 16), ((100, 37), 16, "weak", 3)]
    datas, handles, ks = [], [], []
    for i, (shape, r, adm, k) in enumerate(specs):
        kind = "inv" if len(shape) == 3 else "log"
        d = make_hmatrix(_tree(shape), r, kind=kind, method="random", seed=60 + i, admissibility=adm)
        datas.append(d)
        ks.append(k)
        handles.append(create(d, storage="fp16", max_nrhs=k))
    xn, xs, ys, refs = [], [], [], []
    for j, (d, k, h) in enumerate(zip(datas, ks, handles)):
        x = make_rhs(d.n, k, 70 + j)
        xn.append(x)
        xs.append(torch.from_numpy(np.ascontiguousarray(x.T)).cuda().T)
        ys.append(torch.full((k, d.n), float("nan"), device="cuda").T)
        yr = torch.full((k, d.n), float("nan"), device="cuda").T
        h.matvec(xs[-1], yr)
        refs.append(yr)
    torch.cuda.synchronize()
    refs = [r.cpu().numpy().astype(np.float64) for r in refs]
    with hm.HBatch(handles, ks) as b:
        b.matvec(xs, ys)
        b.sync()
        torch.cuda.synchronize()
        got = [y.cpu().numpy().astype(np.float64) for y in ys]
    for g, r in zip(got, refs):
        assert np.array_equal(g, r)
    for d, x, g in zip(datas, xn, got):
        assert_close(g, oracle.oracle_matvec(dequantised(d, "fp16"), x), FP32_TOL, 10 * FP32_TOL)
    for h in handles:
        h.close()


@pytest.fixture(scope="module")
def s2_random():
    _log("building the 2D 1024^2 standard-admissibility factor set (rank 4, random fill)")
    data = make_hmatrix(uniform_tree(2, 1024), 4, method="random", seed=25, admissibility="standard")
    return data, oracle.prepare(data)


def test_s2_full_size_fp32(s2_random):
    data, prep = s2_random
    _log("case s2 fp32 full size")
    x = make_rhs(data.n, 1, 1006)
    ref = oracle.oracle_matvec(prep, x)
    with create(data) as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref, FP32_TOL, ELEM_TOL)


def test_s2_full_size_fp16(s2_random):
    data, _ = s2_random
    _log("case s2 fp16 full size")
    x = make_rhs(data.n, 1, 1006)
    ref_dq = oracle.oracle_matvec(dequantised(data, "fp16"), x)
    with create(data, storage="fp16") as h:
        y = gpu_matvec(h, x)
    assert_close(y, ref_dq, FP32_TOL, ELEM_TOL)
