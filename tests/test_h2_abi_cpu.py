"""The H^2 C ABI on the CPU: every malformed input is rejected before any HIP call."""
import numpy as np
import pytest

import paper_2008_12441_amd as hm
from hmat_inputs import uniform_tree
from hmat_inputs.h2 import make_h2
from paper_2008_12441_amd.binding import HMAT_ERR_BAD_BLOCKS, HMAT_ERR_INVALID_ARG, HMAT_ERR_UNSUPPORTED


@pytest.fixture(scope="module")
def small():
    return make_h2(uniform_tree(2, 64), method="random", rank=8, seed=1)   # L = 3


def _descs(h2, rank=None):
    td, bases, blocks, keep = hm.make_h2_descriptors(
        h2.tree, h2.rank if rank is None else rank, h2.pool, h2.u_off, h2.v_off, h2.e_off, h2.f_off,
        h2.blocks.target, h2.blocks.source, (h2.blocks.rank > 0).astype(np.int32), h2.blk_off)
    return td, bases, blocks, keep


def _status(td, bases, blocks, storage=0, flags=0):
    try:
        h = hm.hmat_h2_create(td, bases, blocks, storage=storage, flags=flags)
    except hm.HmatError as e:
        return e.status, str(e)
    hm.hmat_h2_destroy(h)
    return 0, ""


def test_options_and_storage(small):
    td, bases, blocks, keep = _descs(small)
    assert _status(td, bases, blocks, storage=2)[0] == HMAT_ERR_INVALID_ARG     # BF16 is not an H^2 form
    assert _status(td, bases, blocks, flags=2)[0] == HMAT_ERR_INVALID_ARG


def test_basis_errors(small):
    td, bases, blocks, keep = _descs(small)
    b = bases.copy()
    b["rank"][0] = 4                      # the root never has a basis
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    b = bases.copy()
    b["rank"][3] = 0                      # every non-root node needs one
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    b = bases.copy()
    b["rank"][3] = 65                     # above HMAT_H2_MAX_RANK
    assert _status(td, b, blocks)[0] == HMAT_ERR_UNSUPPORTED
    leaf = int(np.nonzero(small.u_off >= 0)[0][0])
    b = bases.copy()
    b["u"][leaf] = 0
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    b = bases.copy()
    b["ldv"][leaf] = 3
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    inner = int(np.nonzero(small.e_off >= 0)[0][0])
    b = bases.copy()
    b["f"][inner] = 0
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    b = bases.copy()
    b["lde"][inner] = 1
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG
    b = bases.copy()
    b["reserved"][2] = 1
    assert _status(td, b, blocks)[0] == HMAT_ERR_INVALID_ARG


def test_block_errors(small):
    td, bases, blocks, keep = _descs(small)
    cp = int(np.nonzero(blocks["kind"] == 1)[0][0])
    de = int(np.nonzero(blocks["kind"] == 0)[0][0])
    bl = blocks.copy()
    bl["kind"][cp] = 2
    assert _status(td, bases, bl)[0] == HMAT_ERR_INVALID_ARG
    bl = blocks.copy()
    bl["lda"][cp] = 1                     # < k_t
    assert _status(td, bases, bl)[0] == HMAT_ERR_INVALID_ARG
    bl = blocks.copy()
    bl["lda"][de] = 10                    # < |t|
    assert _status(td, bases, bl)[0] == HMAT_ERR_INVALID_ARG
    bl = blocks.copy()
    bl["a"][de] = 0
    assert _status(td, bases, bl)[0] == HMAT_ERR_INVALID_ARG
    assert _status(td, bases, blocks[1:])[0] == HMAT_ERR_BAD_BLOCKS            # a missing block
    dup = np.concatenate([blocks, blocks[:1]])
    assert _status(td, bases, dup)[0] == HMAT_ERR_BAD_BLOCKS                     # a duplicate
    bl = blocks.copy()
    bl["kind"][cp] = 0                    # a dense block between non-leaves
    bl["lda"][cp] = small.tree.size(int(bl["target"][cp]))
    assert _status(td, bases, bl)[0] == HMAT_ERR_UNSUPPORTED


def test_couplings_need_a_deep_tree():
    h2 = make_h2(uniform_tree(2, 16), method="random", rank=4, seed=1)          # L = 1: dense only
    td, bases, blocks, keep = _descs(h2)
    bl = blocks.copy()
    bl["kind"][0] = 1
    assert _status(td, bases, bl)[0] == HMAT_ERR_BAD_BLOCKS


def test_null_pointers(small):
    td, bases, blocks, keep = _descs(small)
    lib = hm.binding_h2._lib()
    import ctypes

    opts = hm.binding_h2.hmat_h2_options(0, 0, 0, 0)
    out = ctypes.c_void_p()
    assert lib.hmat_h2_create(ctypes.byref(td), None, blocks.ctypes.data, len(blocks), ctypes.byref(opts),
                              ctypes.byref(out)) == HMAT_ERR_INVALID_ARG
    assert lib.hmat_h2_create(ctypes.byref(td), bases.ctypes.data, None, len(blocks), ctypes.byref(opts),
                              ctypes.byref(out)) == HMAT_ERR_INVALID_ARG
    assert lib.hmat_h2_create(ctypes.byref(td), bases.ctypes.data, blocks.ctypes.data, len(blocks), None,
                              ctypes.byref(out)) == HMAT_ERR_INVALID_ARG
    assert lib.hmat_h2_destroy(None) == 0
    bogus = ctypes.c_void_p(12345)
    assert lib.hmat_h2_destroy(bogus) == HMAT_ERR_INVALID_ARG
    assert lib.hmat_h2_matvec(bogus, 1, 1.0, bogus, 10, 0.0, bogus, 10, None) == HMAT_ERR_INVALID_ARG
