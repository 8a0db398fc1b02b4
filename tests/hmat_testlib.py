"""Glue shared by the library tests: descriptors from a factor set, GPU runs, error metrics."""
from __future__ import annotations

import numpy as np

import paper_2008_12441_amd as hm


def descriptors(data):
    t = data.tree
    return hm.make_descriptors(t.parent, t.begin, t.end, data.blocks.target, data.blocks.source,
                               data.blocks.rank, data.pool, data.off_a, data.off_b)


def create(data, storage="fp32", max_nrhs=1, fp64_accum=False, transpose=False):
    tree, blocks, keep = descriptors(data)
    return hm.HMatrix(tree, blocks, storage=storage, max_nrhs=max_nrhs, fp64_accum=fp64_accum, transpose=transpose)


def gpu_matvec(h, x, *, alpha=1.0, beta=0.0, y0=None, ld_pad=0):
    """Run h on x (n x k numpy, FP32) on cuda:0; returns y as float64 numpy."""
    import torch

    n, k = x.shape
    ld = n + ld_pad
    xd = torch.zeros((k, ld), dtype=torch.float32, device="cuda")
    xd[:, :n] = torch.from_numpy(np.ascontiguousarray(x.T))
    yd = torch.full((k, ld), float("nan"), dtype=torch.float32, device="cuda")
    if y0 is not None:
        yd[:, :n] = torch.from_numpy(np.ascontiguousarray(y0.T.astype(np.float32)))
    stream = torch.cuda.current_stream().cuda_stream
    hm.hmat_matvec(h.handle, k, alpha, xd.data_ptr(), ld, beta, yd.data_ptr(), ld, stream)
    torch.cuda.synchronize()
    out = yd[:, :n].cpu().numpy().T.astype(np.float64)
    if ld_pad:
        pad = yd[:, n:].cpu().numpy()
        assert np.isnan(pad).all(), "wrote outside the rows of y"
    return out


def rel_err_cols(y, ref):
    """Per-column relative 2-norm error."""
    num = np.linalg.norm(y - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.where(den == 0, 1.0, den)


def assert_close(y, ref, rel_tol, elem_tol=None):
    """Max over columns of the relative 2-norm error <= rel_tol, and every element
    within elem_tol x the column's RMS (catches errors confined to a few rows)."""
    assert np.isfinite(y).all(), "non-finite output"
    errs = rel_err_cols(y, ref)
    assert errs.max() <= rel_tol, f"relative error {errs.max():.3e} > {rel_tol:.1e}"
    if elem_tol is not None:
        rms = np.sqrt(np.mean(ref * ref, axis=0))
        worst = np.max(np.abs(y - ref) / rms[None, :])
        assert worst <= elem_tol, f"element error {worst:.3e} x RMS > {elem_tol:.1e}"
    return float(errs.max())


def assert_fp32_rounding_of(y, ref, min_exact=0.99):
    """y (FP32 values) is ref (FP64) rounded to FP32, up to one FP32 unit in the
    last place per element; at least ``min_exact`` of the elements round the same
    way (they differ only where ref lies within FP64 roundoff of a midpoint)."""
    assert np.isfinite(y).all(), "non-finite output"
    y32 = np.asarray(y, np.float64).astype(np.float32)
    assert np.array_equal(y32.astype(np.float64), np.asarray(y, np.float64)), "y holds non-FP32 values"
    r32 = np.asarray(ref, np.float64).astype(np.float32)
    ulp = np.maximum(np.spacing(np.abs(r32)), np.spacing(np.abs(y32))).astype(np.float64)
    diff = np.abs(y32.astype(np.float64) - r32.astype(np.float64))
    worst = float(np.max(diff / ulp)) if diff.size else 0.0
    assert worst <= 1.0, f"an element is {worst:.1f} FP32 ulp from the rounded reference"
    exact = float(np.mean(diff == 0)) if diff.size else 1.0
    assert exact >= min_exact, f"only {exact:.4f} of the elements are the rounded reference"
    return exact
