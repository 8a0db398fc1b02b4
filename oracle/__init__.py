"""Oracle for the H-matrix-vector product -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library shares no code with it.

``oracle_matvec`` evaluates Eq. (2.4) of Sec. 2 ("hmat-vec-add") in FP64 over
a canonical FP32 factor set, in the GEMV form y = alpha K x + beta y of the
remark that closes Sec. 4.1; the loops are in ``hmat_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmat_oracle.c")
_LIB = os.path.join(_HERE, "libhmat_oracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle (plain C, FP64, OpenMP)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def bind(path: str):
    """Load an oracle library from ``path`` and declare its entry points."""
    lib = ctypes.CDLL(path)
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.hmat_oracle_matvec.argtypes = [i64, i64, p, p, p, p, p, p, p, p, ctypes.c_int32,
                                       ctypes.c_double, p, i64, ctypes.c_double, p, i64,
                                       i64, i64, ctypes.c_int32]
    lib.hmat_oracle_matvec.restype = ctypes.c_int
    lib.hmat_oracle_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = bind(_LIB)
    return _lib


def max_threads() -> int:
    return int(_load().hmat_oracle_max_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class _Prepared:
    """Per-block row/column ranges of a factor set, computed once."""

    def __init__(self, data):
        tree, blocks = data.tree, data.blocks
        self.n = int(tree.n)
        self.nb = len(blocks)
        self.rb = np.ascontiguousarray(tree.begin[blocks.target], dtype=np.int64)
        self.re = np.ascontiguousarray(tree.end[blocks.target], dtype=np.int64)
        self.cb = np.ascontiguousarray(tree.begin[blocks.source], dtype=np.int64)
        self.ce = np.ascontiguousarray(tree.end[blocks.source], dtype=np.int64)
        self.rank = np.ascontiguousarray(blocks.rank, dtype=np.int32)
        self.pool = np.ascontiguousarray(data.pool, dtype=np.float32)
        self.off_a = np.ascontiguousarray(data.off_a, dtype=np.int64)
        self.off_b = np.ascontiguousarray(data.off_b, dtype=np.int64)


def prepare(data) -> _Prepared:
    return _Prepared(data)


def oracle_matvec(data, x, *, alpha: float = 1.0, beta: float = 0.0, y_in=None,
                  rows=None, nthreads: int = 0, lib=None) -> np.ndarray:
    """y = alpha * K_H x + beta * y_in in FP64.

    ``data`` is an ``hmat_inputs.HMatrixData`` (or a ``prepare``d copy), ``x`` an
    n x k array (any float dtype; promoted exactly to FP64). ``rows=(lo, hi)``
    restricts the output to those rows (the others are returned as NaN).
    """
    prep = data if isinstance(data, _Prepared) else _Prepared(data)
    lib = lib if lib is not None else _load()
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[:, None]
    n, k = x.shape
    if n != prep.n:
        raise ValueError("x has the wrong number of rows")
    xd = np.asfortranarray(x, dtype=np.float64)
    if beta != 0.0:
        if y_in is None:
            raise ValueError("beta != 0 needs y_in")
        y = np.asfortranarray(np.array(y_in, dtype=np.float64).reshape(n, k))
    else:
        y = np.full((n, k), np.nan, dtype=np.float64, order="F")
    lo, hi = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    rc = lib.hmat_oracle_matvec(prep.n, prep.nb, _ptr(prep.rb), _ptr(prep.re), _ptr(prep.cb),
                                _ptr(prep.ce), _ptr(prep.rank), _ptr(prep.pool),
                                _ptr(prep.off_a), _ptr(prep.off_b), k, float(alpha), _ptr(xd),
                                n, float(beta), _ptr(y), n, lo, hi, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"hmat_oracle_matvec failed with code {rc}")
    return y


def transposed(data):
    """The factor set of K^T: block (t, s) becomes (s, t), a low-rank block's U and
    V trade places, and a dense block's entries are stored transposed (same pool
    offsets, so every block keeps its slot)."""
    import copy

    out = copy.copy(data)
    blocks = copy.copy(data.blocks)
    blocks.target, blocks.source = data.blocks.source.copy(), data.blocks.target.copy()
    out.blocks = blocks
    lr = data.blocks.rank > 0
    out.off_a = np.where(lr, data.off_b, data.off_a)
    out.off_b = np.where(lr, data.off_a, -1)
    pool = data.pool.copy()
    for b in np.nonzero(~lr)[0]:
        o = int(data.off_a[b])
        d = data.dense(int(b))                      # |t| x |s|
        pool[o:o + d.size] = np.ascontiguousarray(d).reshape(-1)   # D^T column-major = D row-major
    out.pool = pool
    return out


def assemble_dense(data) -> np.ndarray:
    """Place every block of the H-matrix into an N x N FP64 matrix (small N only).

    Entries covered by no block stay NaN and entries covered twice raise, so the
    result also shows that the blocks tile N x N exactly once.
    """
    tree, blocks = data.tree, data.blocks
    n = tree.n
    k = np.full((n, n), np.nan)
    hit = np.zeros((n, n), dtype=np.int32)
    for b in range(len(blocks)):
        r0, r1 = data.rows(b)
        c0, c1 = data.cols(b)
        if blocks.rank[b] == 0:
            k[r0:r1, c0:c1] = data.dense(b).astype(np.float64)
        else:
            k[r0:r1, c0:c1] = data.u(b).astype(np.float64) @ data.v(b).astype(np.float64).T
        hit[r0:r1, c0:c1] += 1
    if (hit > 1).any():
        raise ValueError("blocks overlap")
    return k
