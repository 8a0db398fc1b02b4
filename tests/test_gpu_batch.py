"""GPU parity of the batched persistent launch (hmat_batch_*).

The batched kernel runs the same per-item device code as the per-handle
kernels, in the same order within every item, so each member's y must equal
bit for bit what the member's own hmat_matvec gives; on top, every member is
checked against the FP64 oracle over its (dequantised) factors. Graph replays
are checked against direct launches, with other GPU work between them.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2008_12441_amd as hm
from oracle.quant import dequantised
from hmat_inputs import batch_problems, build_batch_member, build_tree, make_hmatrix, make_rhs, uniform_tree
from hmat_testlib import assert_close, create

pytestmark = pytest.mark.gpu

KERNEL_TOL = {"fp32": 1e-5, "fp16": 1e-5, "bf16": 3e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    yield


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SHAPES = [((64, 64), 16, "svd"), ((40, 23), 8, "random"), ((17, 33, 9), 8, "random"), ((16, 16, 16), 8, "random"),
          ((100, 37), 16, "random"), ((8, 8), 4, "random"), ((16, 16), 4, "random"), ((128, 96), 32, "random")]


def _member_data(i, shape, r, method):
    full = tuple(max(256 if len(shape) == 2 else 64, s) for s in shape)
    tree = build_tree(shape, n_full=full)
    return make_hmatrix(tree, r, kind="log" if len(shape) == 2 else "inv", method=method, seed=100 + i)


def _operands(datas, ks, seed):
    import torch

    xs, ys, xn = [], [], []
    for j, (d, k) in enumerate(zip(datas, ks)):
        x = make_rhs(d.n, k, seed + j)
        xn.append(x)
        xs.append(torch.from_numpy(np.ascontiguousarray(x.T)).cuda().T)   # column-major n x k
        ys.append(torch.full((k, d.n), float("nan"), device="cuda").T)
    return xn, xs, ys


def _single_runs(handles, xs, ks, alpha=1.0, beta=0.0, y0s=None):
    """Each member through its own hmat_matvec (reference for bitwise equality)."""
    import torch

    outs = []
    for j, (h, x, k) in enumerate(zip(handles, xs, ks)):
        y = (y0s[j].clone() if y0s is not None else torch.full((k, h.n), float("nan"), device="cuda").T)
        h.matvec(x, y, alpha=alpha, beta=beta)
        outs.append(y)
    torch.cuda.synchronize()
    return [o.cpu().numpy().astype(np.float64) for o in outs]


def _to_np(ys):
    import torch

    torch.cuda.synchronize()
    return [y.cpu().numpy().astype(np.float64) for y in ys]


def _check_members(datas, xn, got, form, alpha=1.0, beta=0.0, y0s=None):
    for j, (d, x, y) in enumerate(zip(datas, xn, got)):
        ref = oracle.oracle_matvec(dequantised(d, form), x, alpha=alpha, beta=beta,
                                   y_in=None if y0s is None else y0s[j])
        assert_close(y, ref, KERNEL_TOL[form], 10 * KERNEL_TOL[form])


@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16"])
def test_batch_single_vector_members(form):
    _log(f"case batch single-vector {form}")
    datas = [_member_data(i, *s) for i, s in enumerate(SHAPES)]
    ks = [1] * len(datas)
    handles = [create(d, storage=form, max_nrhs=1) for d in datas]
    xn, xs, ys = _operands(datas, ks, 50)
    ref_bits = _single_runs(handles, xs, ks)
    with hm.HBatch(handles, ks) as b:
        info = b.info()
        assert info["count"] == len(datas) and info["num_items"] > 0 and info["use_graph"] == 1
        b.matvec(xs, ys)
        b.sync()
        got = _to_np(ys)
    for g, r in zip(got, ref_bits):
        assert np.array_equal(g, r)
    _check_members(datas, xn, got, form)
    for h in handles:
        h.close()


@pytest.mark.parametrize("form", ["fp32", "fp16", "bf16"])
def test_batch_multi_rhs_members(form):
    _log(f"case batch multi-rhs {form}")
    datas = [_member_data(i, *s) for i, s in enumerate(SHAPES)]
    ks = [16, 5, 1, 16, 9, 2, 3, 16]
    handles = [create(d, storage=form, max_nrhs=m) for d, m in zip(datas, [16, 8, 4, 32, 16, 2, 3, 128])]
    xn, xs, ys = _operands(datas, ks, 60)
    ref_bits = _single_runs(handles, xs, ks)
    with hm.HBatch(handles, ks) as b:
        b.matvec(xs, ys)
        b.sync()
        got = _to_np(ys)
    for g, r in zip(got, ref_bits):
        assert np.array_equal(g, r)
    _check_members(datas, xn, got, form)
    for h in handles:
        h.close()


def test_batch_mixed_members_alpha_beta_options_and_replays():
    """Single-vector and multi-RHS members in one launch; alpha/beta; every
    option combination; graph replays interleaved with other GPU work."""
    import torch

    _log("case batch mixed")
    datas = [_member_data(i, *s) for i, s in enumerate(SHAPES)]
    maxk = [1, 8, 1, 16, 1, 4, 1, 16]
    ks = [1, 8, 1, 16, 1, 3, 1, 11]
    handles = [create(d, storage="fp16", max_nrhs=m) for d, m in zip(datas, maxk)]
    xn, xs, ys = _operands(datas, ks, 70)
    rng = np.random.default_rng(5)
    y0n = [rng.standard_normal((d.n, k)).astype(np.float32) for d, k in zip(datas, ks)]
    y0 = [torch.from_numpy(np.ascontiguousarray(y.T)).cuda().T for y in y0n]
    ref_bits = _single_runs(handles, xs, ks, alpha=0.5, beta=-2.0, y0s=y0)
    with hm.HBatch(handles, ks) as b:
        for opts in [dict(use_graph=1, wg_per_cu=0, order=0), dict(use_graph=0, wg_per_cu=1, order=0, grain_kb=1),
                     dict(use_graph=1, wg_per_cu=1, order=1, grain_kb=64), dict(use_graph=0, wg_per_cu=2, order=1),
                     dict(use_graph=1, wg_per_cu=3, order=0, grain_kb=1 << 16)]:
            b.set_options(**opts)
            for rep in range(3):
                for y, yi in zip(ys, y0):
                    y.copy_(yi)
                b.matvec(xs, ys, alpha=0.5, beta=-2.0)
                # unrelated eager work on the same stream between replays
                z = torch.randn(1 << 20, device="cuda")
                _ = (z * z).sum().item()
                b.sync()
                got = _to_np(ys)
                for g, r in zip(got, ref_bits):
                    assert np.array_equal(g, r), (opts, rep)
    _check_members(datas, xn, got, "fp16", alpha=0.5, beta=-2.0, y0s=y0n)
    for h in handles:
        h.close()


def test_batch_new_operands_each_call():
    """The operand table follows the pointers of every call."""
    _log("case batch operand swap")
    datas = [_member_data(i, *s) for i, s in enumerate(SHAPES[:4])]
    ks = [1, 1, 1, 1]
    handles = [create(d, storage="fp32") for d in datas]
    xn1, xs1, ys1 = _operands(datas, ks, 80)
    xn2, xs2, ys2 = _operands(datas, ks, 90)
    with hm.HBatch(handles, ks) as b:
        b.matvec(xs1, ys1)
        b.matvec(xs2, ys2)
        b.matvec(xs2, ys1)   # y1 now holds K x2
        b.sync()
        g1, g2 = _to_np(ys1), _to_np(ys2)
    for a, c in zip(g1, g2):
        assert np.array_equal(a, c)
    _check_members(datas, xn2, g2, "fp32")
    for h in handles:
        h.close()


def test_batch_wait_limit_reports_error_then_recovers():
    """A poll limit of one makes dependency waits give up: the call completes
    (no hang) and hmat_batch_sync reports DEVICE; with the default limit the
    next call is correct again."""
    _log("case batch wait limit")
    datas = [_member_data(i, (128, 128), 16, "random") for i in range(6)]
    ks = [1] * 6
    handles = [create(d, storage="fp32") for d in datas]
    xn, xs, ys = _operands(datas, ks, 95)
    with hm.HBatch(handles, ks, spin_limit=1) as b:
        b.matvec(xs, ys)
        with pytest.raises(hm.HmatError) as e:
            b.sync()
        assert e.value.status == hm.binding.HMAT_ERR_DEVICE
        b.set_options(spin_limit=0)
        b.matvec(xs, ys)
        b.sync()
        _check_members(datas, xn, _to_np(ys), "fp32")
    for h in handles:
        h.close()


def test_batch_autotune_and_cache(tmp_path):
    _log("case batch autotune")
    datas = [_member_data(i, *s) for i, s in enumerate(SHAPES)]
    ks = [1] * len(datas)
    handles = [create(d, storage="fp16") for d in datas]
    xn, xs, ys = _operands(datas, ks, 99)
    cache = str(tmp_path / "tune.json")
    with hm.HBatch(handles, ks) as b:
        chosen = b.autotune(xs, ys, cache_path=cache, reps=2)
        info = b.info()
        assert info["wg_per_cu"] == chosen["wg_per_cu"] and info["order"] == chosen["order"]
        assert info["grain_kb"] == chosen["grain_kb"]
        doc = json.load(open(cache))
        assert doc["format"] == "hmat-batch-tuning-1" and len(doc["entries"]) == 1
        assert doc["entries"][0]["wg_per_cu"] == chosen["wg_per_cu"]
        assert doc["entries"][0]["grain_kb"] == chosen["grain_kb"]
        again = b.autotune(xs, ys, cache_path=cache, reps=2)   # cache hit
        assert again == chosen
        b.matvec(xs, ys)
        b.sync()
        _check_members(datas, xn, _to_np(ys), "fp16")
    for h in handles:
        h.close()


def test_batch_validation_and_lifetime():
    _log("case batch validation")
    d1 = _member_data(0, (64, 64), 8, "random")
    d2 = _member_data(1, (40, 23), 8, "random")
    s1 = create(d1, storage="fp32")
    s2 = create(d2, storage="fp32")
    m1 = create(d1, storage="fp32", max_nrhs=16)
    h16 = create(d2, storage="fp16")
    f64 = create(d2, storage="fp32", fp64_accum=True)
    bad = [([s1, s1], [1, 1]), ([s1], [2]), ([m1], [17]), ([m1], [0]), ([s1, h16], [1, 1]), ([f64], [1])]
    for members, ks in bad:
        with pytest.raises(hm.HmatError) as e:
            hm.HBatch(members, ks)
        assert e.value.status == hm.binding.HMAT_ERR_INVALID_ARG, (ks, str(e.value))
    f8 = create(d1, storage="fp8", max_nrhs=4)
    with pytest.raises(hm.HmatError) as e:
        hm.HBatch([f8], [4])
    assert e.value.status == hm.binding.HMAT_ERR_UNSUPPORTED
    f8.close()
    b = hm.HBatch([s1, s2, m1], [1, 1, 16])
    with pytest.raises(hm.HmatError) as e:
        hm.hmat_destroy(s1.handle)          # still referenced by the batch
    assert e.value.status == hm.binding.HMAT_ERR_INVALID_ARG
    b.close()
    for h in (s1, s2, m1, h16, f64):
        h.close()


@pytest.fixture(scope="module")
def c4_full():
    """All 256 members of the batched workload's generator (2D and 3D sub-grids, N
    log-uniform in [4096, 65536], ranks in {8, 16, 32}), random factor fills drawn
    on the GPU, with their dequantised FP16 factor sets."""
    _log("building the 256 batched-workload members (random fills)")
    specs = batch_problems(256, seed=4)
    datas = [build_batch_member(s, method="random", seed=300 + i, device="cuda") for i, s in enumerate(specs)]
    return datas, [dequantised(d, "fp16") for d in datas]


@pytest.mark.parametrize("k", [1, 16])
def test_batch_workload_members_fp16(c4_full, k):
    """One launch over all 256 members: every member's every column, bitwise equal
    to its own hmat_matvec, within the kernel bound of the FP64 oracle over its
    dequantised factors and within the form's 1e-3 of the oracle over the
    canonical ones."""
    _log(f"case batch workload generator, 256 members, k={k}")
    datas, dqs = c4_full
    ks = [k] * len(datas)
    handles = [create(d, storage="fp16", max_nrhs=k) for d in datas]
    xn, xs, ys = _operands(datas, ks, 1004)
    ref_bits = _single_runs(handles, xs, ks)
    with hm.HBatch(handles, ks) as b:
        b.matvec(xs, ys)
        b.sync()
        got = _to_np(ys)
    for h in handles:
        h.close()
    for j, (g, r) in enumerate(zip(got, ref_bits)):
        assert np.array_equal(g, r), f"member {j}"
    worst = 0.0
    for j, (d, dq, x, y) in enumerate(zip(datas, dqs, xn, got)):
        assert_close(y, oracle.oracle_matvec(dq, x), KERNEL_TOL["fp16"], 10 * KERNEL_TOL["fp16"])
        worst = max(worst, assert_close(y, oracle.oracle_matvec(d, x), 1e-3))
    _log(f"256 members, k={k}: largest error against the canonical factors {worst:.3e}")


def test_batch_workload_layout_padding(c4_full):
    """Multi-RHS layout of the 256 batched-workload members: the bytes the
    kernels stream over the factor bytes. A chunk's rows are contiguous on
    both sides, the blocks of one target box whose ranks are not whole K-blocks
    share K-blocks, and the dense blocks between two boxes form one segment;
    what is left is each chunk's and z item's padding to whole K-blocks and row
    tiles (1.14 for FP16 and 1.07 for FP32, from 2.39 and 1.85 with per-leaf
    and per-block padding)."""
    datas, _ = c4_full
    for form, bound in (("fp16", 1.20), ("fp32", 1.12)):
        hs = [create(d, storage=form, max_nrhs=16) for d in datas]
        fb = sum(h.info["factor_bytes"] for h in hs)
        db = sum(h.info["device_factor_bytes"] for h in hs)
        for h in hs:
            h.close()
        _log(f"layout padding {form}: {db / fb:.3f}")
        assert db / fb <= bound, (form, db / fb)
