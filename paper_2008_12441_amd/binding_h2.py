"""ctypes binding of the H^2 entry points (include/hmat_h2.h): argument marshalling only.

Same conventions as ``binding``: C names, ``HmatError`` on a non-OK status,
no fallback when the library is missing.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .binding import (HMAT_NUM_PHASES, STORAGE, HmatError, _check, load_library, make_tree_desc)

HMAT_H2_MAX_RANK = 64


class hmat_h2_basis(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("u", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("v", ctypes.c_void_p), ("ldv", ctypes.c_int64),
                ("e", ctypes.c_void_p), ("lde", ctypes.c_int64), ("f", ctypes.c_void_p), ("ldf", ctypes.c_int64)]


class hmat_h2_block(ctypes.Structure):
    _fields_ = [("target", ctypes.c_int32), ("source", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("a", ctypes.c_void_p), ("lda", ctypes.c_int64)]


class hmat_h2_options(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("device", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class hmat_h2_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("leaf_depth", ctypes.c_int32), ("num_chunks", ctypes.c_int32),
                ("num_dense_blocks", ctypes.c_int64), ("num_coupling_blocks", ctypes.c_int64),
                ("stored_elements", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("device_factor_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("leaf_kernel_bytes", ctypes.c_int64), ("storage", ctypes.c_int32), ("max_rank", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


BASIS_DTYPE = np.dtype([("rank", np.int32), ("reserved", np.int32), ("u", np.uint64), ("ldu", np.int64),
                        ("v", np.uint64), ("ldv", np.int64), ("e", np.uint64), ("lde", np.int64),
                        ("f", np.uint64), ("ldf", np.int64)], align=True)
H2BLOCK_DTYPE = np.dtype([("target", np.int32), ("source", np.int32), ("kind", np.int32), ("reserved", np.int32),
                          ("a", np.uint64), ("lda", np.int64)], align=True)
assert BASIS_DTYPE.itemsize == ctypes.sizeof(hmat_h2_basis)
assert H2BLOCK_DTYPE.itemsize == ctypes.sizeof(hmat_h2_block)

_declared = False


def _lib():
    global _declared
    lib = load_library()
    if not _declared:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.hmat_h2_create.argtypes = [vp, vp, vp, i64, ctypes.POINTER(hmat_h2_options), ctypes.POINTER(vp)]
        lib.hmat_h2_matvec.argtypes = [vp, i32, ctypes.c_float, vp, i64, ctypes.c_float, vp, i64, vp]
        lib.hmat_h2_destroy.argtypes = [vp]
        lib.hmat_h2_get_info.argtypes = [vp, ctypes.POINTER(hmat_h2_info)]
        lib.hmat_h2_set_timing.argtypes = [vp, i32]
        lib.hmat_h2_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        for name in ("hmat_h2_create", "hmat_h2_matvec", "hmat_h2_destroy", "hmat_h2_get_info",
                     "hmat_h2_set_timing", "hmat_h2_get_timing"):
            getattr(lib, name).restype = ctypes.c_int
        _declared = True
    return lib


def make_h2_descriptors(tree, rank, pool, u_off, v_off, e_off, f_off, target, source, kind, blk_off):
    """Tree descriptor, basis records and block records over one FP32 pool laid out
    as ``hmat_inputs.h2`` lays it out (column-major, leading dimension = rows).
    Returns (tree_desc, bases, blocks, keepalive)."""
    pool = np.ascontiguousarray(pool, dtype=np.float32)
    base = np.uint64(pool.ctypes.data)
    begin = np.asarray(tree.begin, np.int64)
    end = np.asarray(tree.end, np.int64)
    parent = np.asarray(tree.parent, np.int32)
    size = end - begin
    rank = np.asarray(rank, np.int32)
    td = make_tree_desc(parent, begin, end)
    bases = np.zeros(len(parent), dtype=BASIS_DTYPE)
    bases["rank"] = rank

    def ptr(off):
        off = np.asarray(off, np.int64)
        return np.where(off >= 0, base + np.maximum(off, 0).astype(np.uint64) * np.uint64(4), np.uint64(0))

    bases["u"] = ptr(u_off)
    bases["v"] = ptr(v_off)
    bases["ldu"] = np.where(np.asarray(u_off) >= 0, size, 0)
    bases["ldv"] = bases["ldu"]
    bases["e"] = ptr(e_off)
    bases["f"] = ptr(f_off)
    bases["lde"] = np.where(np.asarray(e_off) >= 0, rank, 0)
    bases["ldf"] = bases["lde"]
    target = np.asarray(target, np.int32)
    blocks = np.zeros(len(target), dtype=H2BLOCK_DTYPE)
    blocks["target"] = target
    blocks["source"] = source
    blocks["kind"] = kind
    blocks["a"] = ptr(blk_off)
    blocks["lda"] = np.where(np.asarray(kind) == 1, rank[target], size[target])
    return td, bases, blocks, (td, pool, bases, blocks)


def hmat_h2_create(tree_desc, bases: np.ndarray, blocks: np.ndarray, *, storage: int = 0, device: int = 0,
                   flags: int = 0) -> int:
    opts = hmat_h2_options(int(storage), int(device), int(flags), 0)
    out = ctypes.c_void_p()
    _check(_lib().hmat_h2_create(ctypes.byref(tree_desc), bases.ctypes.data, blocks.ctypes.data, len(blocks),
                                 ctypes.byref(opts), ctypes.byref(out)))
    return out.value


def hmat_h2_matvec(h: int, nrhs: int, alpha: float, x_ptr: int, ldx: int, beta: float, y_ptr: int, ldy: int,
                   stream: int | None = None):
    _check(_lib().hmat_h2_matvec(h, int(nrhs), float(alpha), x_ptr, int(ldx), float(beta), y_ptr, int(ldy),
                                 stream))


def hmat_h2_destroy(h: int | None):
    _check(_lib().hmat_h2_destroy(h))


def hmat_h2_get_info(h: int) -> dict:
    info = hmat_h2_info()
    _check(_lib().hmat_h2_get_info(h, ctypes.byref(info)))
    return info.as_dict()


def hmat_h2_set_timing(h: int, enable: bool):
    _check(_lib().hmat_h2_set_timing(h, 1 if enable else 0))


def hmat_h2_get_timing(h: int):
    ms = (ctypes.c_double * HMAT_NUM_PHASES)()
    calls = ctypes.c_int64()
    _check(_lib().hmat_h2_get_timing(h, ms, ctypes.byref(calls)))
    return list(ms), calls.value


class H2Matrix:
    """Owner of one H^2 handle built from an ``hmat_inputs.h2.H2Data``-shaped factor set;
    matvec takes torch CUDA tensors (n x k column-major, or a vector)."""

    def __init__(self, data, *, storage="fp32", device=0):
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        td, bases, blocks, self._keep = make_h2_descriptors(
            data.tree, data.rank, data.pool, data.u_off, data.v_off, data.e_off, data.f_off,
            data.blocks.target, data.blocks.source, (data.blocks.rank > 0).astype(np.int32), data.blk_off)
        self.handle = hmat_h2_create(td, bases, blocks, storage=st, device=device)
        self._keep = None                     # the library copied everything
        self.info = hmat_h2_get_info(self.handle)
        self.n = int(self.info["n"])

    def matvec(self, x, y, *, alpha=1.0, beta=0.0, stream=None):
        import torch

        if not (x.is_cuda and y.is_cuda) or x.dtype != torch.float32 or y.dtype != torch.float32:
            raise ValueError("x and y must be float32 CUDA tensors")
        if x.shape[0] != self.n or y.shape[0] != self.n:
            raise ValueError("vector length does not match n")
        k = 1 if x.dim() == 1 else x.shape[1]
        ldx = self.n if x.dim() == 1 else x.stride(1)
        ldy = self.n if y.dim() == 1 else y.stride(1)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        hmat_h2_matvec(self.handle, k, alpha, x.data_ptr(), ldx, beta, y.data_ptr(), ldy, stream)
        return y

    def close(self):
        if self.handle:
            hmat_h2_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["HMAT_H2_MAX_RANK", "H2Matrix", "HmatError", "hmat_h2_create", "hmat_h2_destroy", "hmat_h2_get_info",
           "hmat_h2_get_timing", "hmat_h2_matvec", "hmat_h2_set_timing", "make_h2_descriptors"]
