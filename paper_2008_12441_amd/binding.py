"""ctypes binding of libhmat (include/hmat.h): argument marshalling only.

Every function keeps the C name and raises ``HmatError`` on a non-OK status.
All arithmetic runs in the library's HIP kernels; if the built library is
missing, loading fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libhmat.so")

HMAT_OK = 0
HMAT_ERR_INVALID_ARG = 1
HMAT_ERR_BAD_TREE = 2
HMAT_ERR_BAD_BLOCKS = 3
HMAT_ERR_UNSUPPORTED = 4
HMAT_ERR_NOMEM = 5
HMAT_ERR_DEVICE = 6

HMAT_STORE_FP32 = 0
HMAT_STORE_FP16_SCALED = 1
HMAT_STORE_BF16 = 2
HMAT_STORE_FP8 = 3
HMAT_STORE_FP8_F16D = 4
STORAGE = {"fp32": HMAT_STORE_FP32, "fp16": HMAT_STORE_FP16_SCALED, "bf16": HMAT_STORE_BF16,
           "fp8": HMAT_STORE_FP8, "fp8_f16d": HMAT_STORE_FP8_F16D}

HMAT_FLAG_FP64_ACCUM = 1
HMAT_FLAG_TRANSPOSE = 2

HMAT_NUM_PHASES = 3

HMAT_KERNEL_LOG = 0
HMAT_KERNEL_INV = 1
KERNEL = {"log": HMAT_KERNEL_LOG, "inv": HMAT_KERNEL_INV}


class hmat_tree_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_nodes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("parent", ctypes.c_void_p), ("begin", ctypes.c_void_p), ("end", ctypes.c_void_p)]


class hmat_block_desc(ctypes.Structure):
    _fields_ = [("target", ctypes.c_int32), ("source", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("a", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("ldb", ctypes.c_int64)]


class hmat_options(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("max_nrhs", ctypes.c_int32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_int32)]


class hmat_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("leaf_depth", ctypes.c_int32), ("num_chunks", ctypes.c_int32),
                ("num_dense_blocks", ctypes.c_int64), ("num_lowrank_blocks", ctypes.c_int64),
                ("stored_elements", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("device_factor_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("storage", ctypes.c_int32), ("max_nrhs", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# numpy twin of hmat_block_desc, so large block lists are built without Python loops
BLOCK_DTYPE = np.dtype([("target", np.int32), ("source", np.int32), ("rank", np.int32),
                        ("reserved", np.int32), ("a", np.uint64), ("lda", np.int64),
                        ("b", np.uint64), ("ldb", np.int64)], align=True)
assert BLOCK_DTYPE.itemsize == ctypes.sizeof(hmat_block_desc)

class hmat_compress_options(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("dim", ctypes.c_int32), ("diag", ctypes.c_float),
                ("oversample", ctypes.c_int32), ("seed", ctypes.c_uint64), ("device", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class hmat_batch_options(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("grain_kb", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class hmat_batch_info(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("num_items", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("max_wg_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("grain_kb", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
                ("item_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTED = ("hmat_create", "hmat_matvec", "hmat_destroy", "hmat_get_info", "hmat_set_timing",
            "hmat_get_timing", "hmat_probe_bandwidth", "hmat_last_error", "hmat_status_string",
            "hmat_batch_create", "hmat_batch_matvec", "hmat_batch_sync", "hmat_batch_set_options",
            "hmat_batch_get_info", "hmat_batch_autotune", "hmat_batch_destroy", "hmat_compress",
            "hmat_matvec_noalloc", "hmat_h2_create", "hmat_h2_matvec", "hmat_h2_destroy", "hmat_h2_get_info",
            "hmat_h2_set_timing", "hmat_h2_get_timing")


class HmatError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_status_name(status)}: {message}")


_lib = None


def _status_name(status):
    names = {0: "HMAT_OK", 1: "HMAT_ERR_INVALID_ARG", 2: "HMAT_ERR_BAD_TREE", 3: "HMAT_ERR_BAD_BLOCKS",
             4: "HMAT_ERR_UNSUPPORTED", 5: "HMAT_ERR_NOMEM", 6: "HMAT_ERR_DEVICE"}
    return names.get(status, f"status {status}")


def load_library(path: str | None = None):
    """Load libhmat.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libhmat is not built ({p} missing): run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.hmat_create.argtypes = [ctypes.POINTER(hmat_tree_desc), vp, i64, ctypes.POINTER(hmat_options),
                                ctypes.POINTER(vp)]
    lib.hmat_matvec.argtypes = [vp, i32, ctypes.c_float, vp, i64, ctypes.c_float, vp, i64, vp]
    lib.hmat_matvec_noalloc.argtypes = [vp, i32, ctypes.c_float, vp, i64, ctypes.c_float, vp, i64, vp]
    lib.hmat_destroy.argtypes = [vp]
    lib.hmat_get_info.argtypes = [vp, ctypes.POINTER(hmat_info)]
    lib.hmat_set_timing.argtypes = [vp, i32]
    lib.hmat_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.hmat_probe_bandwidth.argtypes = [vp, vp, i64, i32, vp]
    lib.hmat_last_error.restype = ctypes.c_char_p
    lib.hmat_status_string.restype = ctypes.c_char_p
    lib.hmat_status_string.argtypes = [ctypes.c_int]
    pp = ctypes.POINTER(vp)
    p64 = ctypes.POINTER(i64)
    lib.hmat_batch_create.argtypes = [pp, i32, ctypes.POINTER(i32), ctypes.POINTER(hmat_batch_options),
                                      ctypes.POINTER(vp)]
    lib.hmat_batch_matvec.argtypes = [vp, ctypes.c_float, pp, p64, ctypes.c_float, pp, p64, vp]
    lib.hmat_batch_sync.argtypes = [vp, vp]
    lib.hmat_batch_set_options.argtypes = [vp, ctypes.POINTER(hmat_batch_options)]
    lib.hmat_batch_get_info.argtypes = [vp, ctypes.POINTER(hmat_batch_info)]
    lib.hmat_batch_autotune.argtypes = [vp, ctypes.c_float, pp, p64, ctypes.c_float, pp, p64, vp,
                                        ctypes.c_char_p, i32, ctypes.POINTER(hmat_batch_options)]
    lib.hmat_batch_destroy.argtypes = [vp]
    lib.hmat_compress.argtypes = [ctypes.POINTER(hmat_tree_desc), vp, vp, i64, ctypes.POINTER(hmat_compress_options)]
    for name in ("hmat_create", "hmat_matvec", "hmat_destroy", "hmat_get_info", "hmat_set_timing",
                 "hmat_get_timing", "hmat_probe_bandwidth", "hmat_batch_create", "hmat_batch_matvec",
                 "hmat_batch_sync", "hmat_batch_set_options", "hmat_batch_get_info", "hmat_batch_autotune",
                 "hmat_batch_destroy", "hmat_compress", "hmat_matvec_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != HMAT_OK:
        raise HmatError(status, hmat_last_error())


def hmat_last_error() -> str:
    return load_library().hmat_last_error().decode()


def hmat_status_string(status: int) -> str:
    return load_library().hmat_status_string(status).decode()


def make_tree_desc(parent, begin, end):
    """hmat_tree_desc over numpy arrays (kept alive on the returned object)."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    begin = np.ascontiguousarray(begin, dtype=np.int64)
    end = np.ascontiguousarray(end, dtype=np.int64)
    d = hmat_tree_desc(int(end[0] - begin[0]), len(parent), 0, parent.ctypes.data, begin.ctypes.data,
                       end.ctypes.data)
    d._keep = (parent, begin, end)
    return d


def make_block_array(target, source, rank, pool, off_a, off_b, size_t, size_s):
    """hmat_block_desc records for factors packed in one FP32 pool.

    Block b: dense D (|t| x |s|, ld |t|) or U (|t| x r, ld |t|) at pool[off_a[b]];
    V (|s| x r, ld |s|) at pool[off_b[b]]. ``size_t``/``size_s`` are |t| and |s|.
    """
    pool = np.ascontiguousarray(pool, dtype=np.float32)
    nb = len(target)
    arr = np.zeros(nb, dtype=BLOCK_DTYPE)
    base = pool.ctypes.data
    rank = np.asarray(rank, dtype=np.int32)
    arr["target"] = target
    arr["source"] = source
    arr["rank"] = rank
    arr["a"] = base + np.asarray(off_a, np.int64).astype(np.uint64) * np.uint64(4)
    arr["lda"] = size_t
    lowrank = rank > 0
    arr["b"] = np.where(lowrank, base + np.maximum(np.asarray(off_b, np.int64), 0).astype(np.uint64) * np.uint64(4),
                        np.uint64(0))
    arr["ldb"] = np.where(lowrank, size_s, 0)
    return arr, pool


def hmat_create(tree_desc: hmat_tree_desc, blocks: np.ndarray, *, storage: int = HMAT_STORE_FP32,
                max_nrhs: int = 1, device: int = 0, flags: int = 0) -> int:
    """Create a handle; ``blocks`` is a BLOCK_DTYPE array. Returns the handle (an int)."""
    lib = load_library()
    blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
    opts = hmat_options(int(storage), int(max_nrhs), int(device), int(flags))
    out = ctypes.c_void_p()
    _check(lib.hmat_create(ctypes.byref(tree_desc), blocks.ctypes.data if len(blocks) else None,
                           len(blocks), ctypes.byref(opts), ctypes.byref(out)))
    return out.value


def hmat_matvec(h: int, nrhs: int, alpha: float, x_ptr: int, ldx: int, beta: float, y_ptr: int, ldy: int,
                stream: int | None = None):
    _check(load_library().hmat_matvec(h, int(nrhs), float(alpha), x_ptr, int(ldx), float(beta), y_ptr,
                                      int(ldy), stream))


def hmat_matvec_noalloc(h: int, nrhs: int, alpha: float, x_ptr: int, ldx: int, beta: float, y_ptr: int,
                        ldy: int, stream: int | None = None):
    """hmat_matvec with its workspace in the library's static scratch (no allocation)."""
    _check(load_library().hmat_matvec_noalloc(h, int(nrhs), float(alpha), x_ptr, int(ldx), float(beta), y_ptr,
                                              int(ldy), stream))


HMAT_NOALLOC_SCRATCH_BYTES = 64 << 20


def hmat_destroy(h: int | None):
    _check(load_library().hmat_destroy(h))


def hmat_get_info(h: int) -> dict:
    info = hmat_info()
    _check(load_library().hmat_get_info(h, ctypes.byref(info)))
    return info.as_dict()


def hmat_set_timing(h: int, enable: bool):
    _check(load_library().hmat_set_timing(h, int(bool(enable))))


def hmat_get_timing(h: int):
    ms = (ctypes.c_double * HMAT_NUM_PHASES)()
    calls = ctypes.c_int64()
    _check(load_library().hmat_get_timing(h, ms, ctypes.byref(calls)))
    return list(ms), calls.value


def hmat_probe_bandwidth(src_ptr: int, dst_ptr: int, nbytes: int, mode: int, stream: int | None = None):
    _check(load_library().hmat_probe_bandwidth(src_ptr, dst_ptr, int(nbytes), int(mode), stream))


class HMatrix:
    """Owner of one handle; matvec takes torch CUDA tensors (n x k, column-major or a vector)."""

    def __init__(self, tree_desc, blocks, *, storage="fp32", max_nrhs=1, device=0, fp64_accum=False,
                 transpose=False):
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        flags = (HMAT_FLAG_FP64_ACCUM if fp64_accum else 0) | (HMAT_FLAG_TRANSPOSE if transpose else 0)
        self.handle = hmat_create(tree_desc, blocks, storage=st, max_nrhs=max_nrhs, device=device, flags=flags)
        self.info = hmat_get_info(self.handle)
        self.n = int(self.info["n"])

    def matvec(self, x, y, *, alpha=1.0, beta=0.0, stream=None):
        import torch

        if not (x.is_cuda and y.is_cuda) or x.dtype != torch.float32 or y.dtype != torch.float32:
            raise ValueError("x and y must be float32 CUDA tensors")
        k = 1 if x.dim() == 1 else x.shape[1]
        ldx = self._ld(x)
        ldy = self._ld(y)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        hmat_matvec(self.handle, k, alpha, x.data_ptr(), ldx, beta, y.data_ptr(), ldy, stream)
        return y

    def _ld(self, t):
        if t.shape[0] != self.n:
            raise ValueError("vector length does not match n")
        if t.dim() == 1:
            if t.stride(0) != 1:
                raise ValueError("vectors must be contiguous")
            return self.n
        if t.stride(0) != 1:
            raise ValueError("multi-RHS arrays must be column-major (stride(0) == 1)")
        return t.stride(1) if t.shape[1] > 1 else max(self.n, t.stride(1))

    def close(self):
        if self.handle:
            hmat_destroy(self.handle)
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


def hmat_compress(tree_desc: hmat_tree_desc, points: np.ndarray, blocks: np.ndarray, *, kernel: str = "log",
                  diag: float = 1.0, oversample: int = 10, seed: int = 0, device: int = 0):
    """Fill the factor arrays that ``blocks`` (a BLOCK_DTYPE array) point to, on the GPU.

    ``points``: n x dim coordinates in tree order. Dense blocks receive the
    kernel entries, low-rank blocks U and V of a randomized SVD (include/hmat.h).
    """
    lib = load_library()
    pts = np.ascontiguousarray(points, dtype=np.float32)
    if pts.ndim != 2:
        raise ValueError("points must be n x dim")
    blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
    opts = hmat_compress_options(KERNEL[kernel], pts.shape[1], float(diag), int(oversample), int(seed), int(device), 0)
    _check(lib.hmat_compress(ctypes.byref(tree_desc), pts.ctypes.data, blocks.ctypes.data if len(blocks) else None,
                             len(blocks), ctypes.byref(opts)))


def compress_pool(parent, begin, end, target, source, rank, points, *, kernel: str = "log", diag: float = 1.0,
                  oversample: int = 10, seed: int = 0, device: int = 0):
    """Construct every block's factors on the GPU into one packed FP32 pool.

    Block b: dense D (|t| x |s|) or U (|t| x r) at pool[off_a[b]], V (|s| x r)
    at pool[off_b[b]] (-1 for dense), all column-major with ld |t| or |s|.
    Returns (pool, off_a, off_b).
    """
    begin = np.asarray(begin, np.int64)
    end = np.asarray(end, np.int64)
    sz = end - begin
    target = np.asarray(target, np.int32)
    source = np.asarray(source, np.int32)
    rank = np.asarray(rank, np.int32)
    m = sz[target]
    n = sz[source]
    r = rank.astype(np.int64)
    count = np.where(r == 0, m * n, (m + n) * r)
    off_a = np.zeros(len(target), np.int64)
    if len(target) > 1:
        off_a[1:] = np.cumsum(count)[:-1]
    off_b = np.where(r == 0, -1, off_a + m * r)
    pool = np.empty(int(count.sum()), np.float32)
    arr, pool = make_block_array(target, source, rank, pool, off_a, off_b, m, n)
    tree = make_tree_desc(parent, begin, end)
    hmat_compress(tree, points, arr, kernel=kernel, diag=diag, oversample=oversample, seed=seed, device=device)
    return pool, off_a, off_b


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[int(p) for p in ptrs])


def _i64_array(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def hmat_batch_create(handles, nrhs, *, use_graph=1, wg_per_cu=0, order=0, spin_limit=0, grain_kb=0,
                      null_options=False) -> int:
    """Create a batch over handle values (ints); returns the batch handle (an int)."""
    lib = load_library()
    hs = _ptr_array(handles)
    ks = (ctypes.c_int32 * len(nrhs))(*[int(k) for k in nrhs])
    opts = hmat_batch_options(int(use_graph), int(wg_per_cu), int(order), int(spin_limit), int(grain_kb))
    out = ctypes.c_void_p()
    _check(lib.hmat_batch_create(hs if len(handles) else None, len(handles), ks if len(nrhs) else None,
                                 None if null_options else ctypes.byref(opts), ctypes.byref(out)))
    return out.value


def hmat_batch_matvec(b: int, alpha: float, x_ptrs, ldx, beta: float, y_ptrs, ldy, stream: int | None = None):
    _check(load_library().hmat_batch_matvec(b, float(alpha), _ptr_array(x_ptrs), _i64_array(ldx), float(beta),
                                            _ptr_array(y_ptrs), _i64_array(ldy), stream))


def hmat_batch_sync(b: int, stream: int | None = None):
    _check(load_library().hmat_batch_sync(b, stream))


def hmat_batch_set_options(b: int, *, use_graph=1, wg_per_cu=0, order=0, spin_limit=0, grain_kb=0):
    opts = hmat_batch_options(int(use_graph), int(wg_per_cu), int(order), int(spin_limit), int(grain_kb))
    _check(load_library().hmat_batch_set_options(b, ctypes.byref(opts)))


def hmat_batch_get_info(b: int) -> dict:
    info = hmat_batch_info()
    _check(load_library().hmat_batch_get_info(b, ctypes.byref(info)))
    return info.as_dict()


def hmat_batch_autotune(b: int, alpha: float, x_ptrs, ldx, beta: float, y_ptrs, ldy, stream: int | None = None,
                        cache_path: str | None = None, reps: int = 5) -> dict:
    chosen = hmat_batch_options()
    _check(load_library().hmat_batch_autotune(b, float(alpha), _ptr_array(x_ptrs), _i64_array(ldx), float(beta),
                                              _ptr_array(y_ptrs), _i64_array(ldy), stream,
                                              cache_path.encode() if cache_path else None, int(reps),
                                              ctypes.byref(chosen)))
    return chosen.as_dict()


def hmat_batch_destroy(b: int | None):
    _check(load_library().hmat_batch_destroy(b))


class HBatch:
    """Owner of one batch over HMatrix members; operands are lists of torch CUDA tensors."""

    def __init__(self, members, nrhs, *, use_graph=True, wg_per_cu=0, order=0, spin_limit=0, grain_kb=0):
        self.members = list(members)   # kept alive: the batch references their device data
        self.nrhs = [int(k) for k in nrhs]
        self.handle = hmat_batch_create([m.handle for m in self.members], self.nrhs, use_graph=int(use_graph),
                                        wg_per_cu=wg_per_cu, order=order, spin_limit=spin_limit,
                                        grain_kb=grain_kb)

    def _operands(self, xs, ys):
        import torch

        if len(xs) != len(self.members) or len(ys) != len(self.members):
            raise ValueError("one x and one y per member")
        for t in list(xs) + list(ys):
            if not t.is_cuda or t.dtype != torch.float32:
                raise ValueError("operands must be float32 CUDA tensors")
        ldx = [m._ld(x) for m, x in zip(self.members, xs)]
        ldy = [m._ld(y) for m, y in zip(self.members, ys)]
        return [x.data_ptr() for x in xs], ldx, [y.data_ptr() for y in ys], ldy

    @staticmethod
    def _stream(stream):
        import torch

        return torch.cuda.current_stream().cuda_stream if stream is None else stream

    def matvec(self, xs, ys, *, alpha=1.0, beta=0.0, stream=None):
        xp, ldx, yp, ldy = self._operands(xs, ys)
        hmat_batch_matvec(self.handle, alpha, xp, ldx, beta, yp, ldy, self._stream(stream))
        return ys

    def sync(self, stream=None):
        hmat_batch_sync(self.handle, self._stream(stream))

    def set_options(self, **kw):
        hmat_batch_set_options(self.handle, **kw)

    def info(self):
        return hmat_batch_get_info(self.handle)

    def autotune(self, xs, ys, *, alpha=1.0, beta=0.0, cache_path=None, reps=5, stream=None):
        xp, ldx, yp, ldy = self._operands(xs, ys)
        return hmat_batch_autotune(self.handle, alpha, xp, ldx, beta, yp, ldy, self._stream(stream),
                                   cache_path=cache_path, reps=reps)

    def close(self):
        if self.handle:
            hmat_batch_destroy(self.handle)
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


def make_descriptors(parent, begin, end, target, source, rank, pool, off_a, off_b):
    """Tree descriptor and block records for a domain tree plus a packed FP32 factor pool.

    ``parent/begin/end`` describe the tree (node 0 = root), ``target/source/rank``
    the blocks, and ``off_a/off_b`` the element offsets of D or U and of V in
    ``pool`` (see ``make_block_array``). Returns (tree_desc, block_array, keepalive).
    """
    begin = np.asarray(begin, np.int64)
    end = np.asarray(end, np.int64)
    size = end - begin
    target = np.asarray(target, np.int32)
    source = np.asarray(source, np.int32)
    tree = make_tree_desc(parent, begin, end)
    blocks, pool = make_block_array(target, source, rank, pool, off_a, off_b, size[target], size[source])
    return tree, blocks, (tree, pool)
