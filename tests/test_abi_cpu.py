"""The C ABI on the CPU: symbols, validation before any HIP call, error paths."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2008_12441_amd as hm
from hmat_inputs import build_tree, make_hmatrix, uniform_tree
from hmat_testlib import descriptors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^(?:hmat_status|const char \*)\s*(hmat_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = hm.load_library()
    names = declared_functions()
    assert {"hmat_create", "hmat_matvec", "hmat_destroy"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", hm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (hmat_\w+)$", out, re.M))
    assert set(names) <= exported
    assert set(hm.EXPORTED) == set(names)


def test_library_has_gfx950_code():
    # the embedded offload bundle names its target triple
    blob = open(hm.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


@pytest.fixture(scope="module")
def small():
    return make_hmatrix(uniform_tree(2, 64), 8, method="random", seed=1)


def _create_status(tree, blocks, storage=0, max_nrhs=1, flags=0, device=0):
    try:
        h = hm.hmat_create(tree, blocks, storage=storage, max_nrhs=max_nrhs, flags=flags, device=device)
    except hm.HmatError as e:
        return e.status, str(e)
    hm.hmat_destroy(h)
    return 0, ""


def _expect(status, expected, text):
    assert status[0] == expected, status


def test_null_and_option_errors(small):
    lib = hm.load_library()
    tree, blocks, keep = descriptors(small)
    out = ctypes.c_void_p(123)
    opts = hm.binding.hmat_options(0, 1, 0, 0)
    assert lib.hmat_create(None, blocks.ctypes.data, len(blocks), ctypes.byref(opts), ctypes.byref(out)) == 1
    assert out.value is None
    assert lib.hmat_create(ctypes.byref(tree), None, len(blocks), ctypes.byref(opts), ctypes.byref(out)) == 1
    assert lib.hmat_create(ctypes.byref(tree), blocks.ctypes.data, len(blocks), None, ctypes.byref(out)) == 1
    assert lib.hmat_create(ctypes.byref(tree), blocks.ctypes.data, len(blocks), ctypes.byref(opts), None) == 1
    _expect(_create_status(tree, blocks, storage=7), 1, "storage")
    _expect(_create_status(tree, blocks, max_nrhs=0), 1, "max_nrhs")
    _expect(_create_status(tree, blocks, flags=4), 1, "flags")
    _expect(_create_status(tree, blocks, flags=7), 1, "flags")
    _expect(_create_status(tree, blocks, flags=-1), 1, "flags")
    # the transpose flag, alone and with the FP64 mode, passes validation (0 with a GPU, 6 without)
    for fl in (2, 3):
        st, msg = _create_status(tree, blocks, flags=fl)
        assert st in (0, 6), msg
    st, msg = _create_status(tree, blocks, storage=3, max_nrhs=8, flags=2)
    assert st in (0, 6), msg
    _expect(_create_status(tree, blocks, device=-1), 1, "device")


def test_bad_trees(small):
    t = small.tree
    _, blocks, keep = descriptors(small)
    par, beg, end = t.parent.copy(), t.begin.copy(), t.end.copy()

    def status_with(p, b, e):
        return _create_status(hm.make_tree_desc(p, b, e), blocks)

    p2 = par.copy(); p2[0] = 3
    assert status_with(p2, beg, end)[0] == 2
    b2 = beg.copy(); b2[5] += 1
    assert status_with(par, b2, end)[0] == 2
    p3 = par.copy(); p3[7] = 9   # parent id larger than the child id
    assert status_with(p3, beg, end)[0] == 2
    e3 = end.copy(); e3[1] = e3[1] + 4   # children overlap
    assert status_with(par, beg, e3)[0] == 2


def test_mixed_depth_tree_unsupported():
    # root with two children: a leaf and an internal node with two leaves
    par = np.array([-1, 0, 0, 2, 2], np.int32)
    beg = np.array([0, 0, 4, 4, 6], np.int64)
    end = np.array([8, 4, 8, 6, 8], np.int64)
    pool = np.ones(64, np.float32)
    tree, blocks, keep = hm.make_descriptors(par, beg, end, [1], [2], [1], pool, [0], [4])
    assert _create_status(tree, blocks)[0] == 4


def _mutated(data, **changes):
    tree, blocks, keep = descriptors(data)
    blocks = blocks.copy()
    for (idx, field), value in changes.items():
        blocks[field][idx] = value
    return tree, blocks, keep


def test_block_errors(small):
    d = small
    rank = d.blocks.rank
    lr = int(np.nonzero(rank > 0)[0][0])
    dn = int(np.nonzero(rank == 0)[0][0])
    tree, blocks, keep = descriptors(d)
    # duplicate (replace one block by a copy of another)
    b2 = blocks.copy(); b2[dn] = b2[dn + 1]
    assert _create_status(tree, b2)[0] == 3
    # missing block
    assert _create_status(tree, blocks[1:])[0] == 3
    # rank larger than the block
    b3 = blocks.copy(); b3["rank"][lr] = 10 ** 6
    assert _create_status(tree, b3)[0] == 1
    # NULL factor pointers
    b4 = blocks.copy(); b4["b"][lr] = 0
    assert _create_status(tree, b4)[0] == 1
    b5 = blocks.copy(); b5["a"][dn] = 0
    assert _create_status(tree, b5)[0] == 1
    # leading dimension too small
    b6 = blocks.copy(); b6["lda"][dn] = 3
    assert _create_status(tree, b6)[0] == 1
    # low-rank block between leaves (HODLR style) is unsupported
    b7 = blocks.copy(); b7["rank"][dn] = 2; b7["b"][dn] = b7["a"][dn]; b7["ldb"][dn] = 64
    assert _create_status(tree, b7)[0] == 4
    # dense block between non-leaf siblings is unsupported
    b8 = blocks.copy(); b8["rank"][lr] = 0
    assert _create_status(tree, b8)[0] == 4
    # a block moved to a cousin source: its pair is no longer a child pair of a
    # recursion pair, and the pair it leaves is missing
    t = d.tree
    lr2 = int(np.nonzero((rank > 0) & (t.depth[d.blocks.target] == 2))[0][0])
    cousin = [i for i in range(t.num_nodes) if t.depth[i] == 2
              and t.parent[i] != t.parent[int(blocks["target"][lr2])]][0]
    b9 = blocks.copy(); b9["source"][lr2] = cousin
    assert _create_status(tree, b9)[0] == 3
    # a (c, c) block above the leaves
    b10 = blocks.copy(); b10["source"][lr] = b10["target"][lr]
    assert _create_status(tree, b10)[0] == 3
    # node id out of range
    b11 = blocks.copy(); b11["target"][0] = 10 ** 6
    assert _create_status(tree, b11)[0] == 1
    b12 = blocks.copy(); b12["reserved"][0] = 1
    assert _create_status(tree, b12)[0] == 1


def test_valid_input_reaches_device_stage(small):
    tree, blocks, keep = descriptors(small)
    st, msg = _create_status(tree, blocks)
    # on a machine without a GPU the first HIP call fails; with one it succeeds
    assert st in (0, 6), msg


def test_fault_injection_alloc(small, monkeypatch):
    tree, blocks, keep = descriptors(small)
    monkeypatch.setenv("HMAT_FAULT", "alloc")
    st, msg = _create_status(tree, blocks)
    assert st == 5 and "HMAT_FAULT" in msg


def test_handle_checks():
    lib = hm.load_library()
    assert lib.hmat_destroy(None) == 0
    bogus = ctypes.c_void_p(0x1234560)
    assert lib.hmat_destroy(bogus) == 1
    info = hm.binding.hmat_info()
    assert lib.hmat_get_info(bogus, ctypes.byref(info)) == 1
    assert lib.hmat_matvec(bogus, 1, 1.0, bogus, 10, 0.0, bogus, 10, None) == 1
    assert lib.hmat_set_timing(bogus, 1) == 1
    assert hm.hmat_status_string(4) == "HMAT_ERR_UNSUPPORTED"


def test_probe_argument_checks():
    lib = hm.load_library()
    assert lib.hmat_probe_bandwidth(None, None, 16, 0, None) == 1
    p = ctypes.c_void_p(0x1000)
    assert lib.hmat_probe_bandwidth(p, p, 15, 0, None) == 1
    assert lib.hmat_probe_bandwidth(p, p, 16, 5, None) == 1


def test_degenerate_trees_validate():
    for shape in [(8, 8), (16, 16), (9, 30, 5)]:
        tree = build_tree(shape, n_full=(64,) * len(shape))
        data = make_hmatrix(tree, 4, method="random", seed=2)
        tr, bl, keep = descriptors(data)
        st, msg = _create_status(tr, bl)
        assert st in (0, 6), msg


def test_fp64_accum_lds_budget():
    """A chunk whose U-phase operand fits the LDS budget in FP32 (8500 values,
    34 KB) but not in FP64 (68 KB) is UNSUPPORTED only in the FP64 mode; the
    check runs before any device call. Factors all alias one zero buffer."""
    par = np.array([-1, 0, 0, 1, 1, 2, 2], np.int32)
    beg = np.array([0, 0, 6000, 0, 3000, 6000, 9000], np.int64)
    end = np.array([12000, 6000, 12000, 3000, 6000, 9000, 12000], np.int64)
    tree = hm.make_tree_desc(par, beg, end)
    buf = np.zeros(6000 * 2500, np.float32)
    recs = [(1, 2, 2500), (2, 1, 2500)]
    for p in (1, 2):
        kids = [3, 4] if p == 1 else [5, 6]
        recs += [(t, s_, 0) for t in kids for s_ in kids]
    blocks = np.zeros(len(recs), dtype=hm.BLOCK_DTYPE)
    for i, (t, s_, r) in enumerate(recs):
        size = 6000 if r else 3000
        blocks[i] = (t, s_, r, 0, buf.ctypes.data, size, buf.ctypes.data if r else 0, size if r else 0)
    st, msg = _create_status(tree, blocks, flags=1)
    assert st == 4 and "LDS" in msg, (st, msg)
    st, msg = _create_status(tree, blocks, flags=0)
    assert st != 4, msg


def test_batch_entry_points_validate_before_device_calls():
    lib = hm.load_library()
    out = ctypes.c_void_p(77)
    fake = (ctypes.c_void_p * 2)(0x1234, 0x5678)
    ks = (ctypes.c_int32 * 2)(1, 1)
    opts = hm.binding.hmat_batch_options(1, 0, 0, 0, 0)
    assert lib.hmat_batch_create(fake, 2, ks, ctypes.byref(opts), None) == 1
    assert lib.hmat_batch_create(fake, 0, ks, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert out.value is None
    assert lib.hmat_batch_create(None, 2, ks, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert lib.hmat_batch_create(fake, 2, None, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert lib.hmat_batch_create(fake, 2, ks, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert "not a live handle" in hm.hmat_last_error()
    for bad in [(2, 0, 0, 0, 0), (1, -1, 0, 0, 0), (1, 0, 2, 0, 0), (1, 0, 0, -5, 0), (1, 65, 0, 0, 0),
                (1, 0, 0, 0, -1), (1, 0, 0, 0, (1 << 20) + 1)]:
        o = hm.binding.hmat_batch_options(*bad)
        assert lib.hmat_batch_create(fake, 2, ks, ctypes.byref(o), ctypes.byref(out)) == 1, bad
    # NULL options take the defaults (the fake members are then rejected)
    assert lib.hmat_batch_create(fake, 2, ks, None, ctypes.byref(out)) == 1
    assert "not a live handle" in hm.hmat_last_error()
    assert lib.hmat_batch_destroy(None) == 0
    assert lib.hmat_batch_destroy(ctypes.c_void_p(0x1234)) == 1
    nb = ctypes.c_void_p(0x1234)
    p = (ctypes.c_void_p * 1)(0)
    ld = (ctypes.c_int64 * 1)(1)
    assert lib.hmat_batch_matvec(nb, 1.0, p, ld, 0.0, p, ld, None) == 1
    assert lib.hmat_batch_sync(nb, None) == 1
    assert lib.hmat_batch_set_options(nb, ctypes.byref(opts)) == 1
    info = hm.binding.hmat_batch_info()
    assert lib.hmat_batch_get_info(nb, ctypes.byref(info)) == 1
    assert lib.hmat_batch_autotune(nb, 1.0, p, ld, 0.0, p, ld, None, None, 1, None) == 1


def test_fp8_forms_need_multi_rhs_handles(small):
    tree, blocks, keep = descriptors(small)
    for form in (hm.binding.HMAT_STORE_FP8, hm.binding.HMAT_STORE_FP8_F16D):
        st, msg = _create_status(tree, blocks, storage=form, max_nrhs=1)
        assert st == 4 and "multi-RHS" in msg, (st, msg)
        st, msg = _create_status(tree, blocks, storage=form, max_nrhs=8, flags=1)
        assert st == 4, (st, msg)
        st, msg = _create_status(tree, blocks, storage=form, max_nrhs=8)
        assert st not in (1, 4), msg      # valid: fails only at the device stage on a machine without a GPU
    assert _create_status(tree, blocks, storage=5)[0] == 1


def test_standard_admissibility_structure_validation():
    """A standard-admissibility block set (Sec. 2, Eq. (2.2)) passes validation; the
    same set with a block removed, with a block split into its child pairs next to
    itself, or with a block between boxes of different depths does not."""
    d = make_hmatrix(uniform_tree(2, 256), 4, method="random", seed=2, admissibility="standard")
    tree, blocks, keep = descriptors(d)
    st, msg = _create_status(tree, blocks)
    assert st in (0, 6), msg
    t = d.tree
    rank = d.blocks.rank
    # missing block
    assert _create_status(tree, blocks[1:])[0] == 3
    # an extra block on a child pair of a low-rank block: it lies inside that block,
    # so it is no child pair of a recursion pair
    lr = int(np.nonzero((rank > 0) & (t.depth[d.blocks.target] == 2))[0][0])
    ct = t.children[int(d.blocks.target[lr])][0]
    cs = t.children[int(d.blocks.source[lr])][0]
    extra = blocks[lr:lr + 1].copy()
    extra["target"] = ct
    extra["source"] = cs
    b2 = np.concatenate([blocks, extra])
    st, msg = _create_status(tree, b2)
    assert st == 3 and "recursion pair" in msg, msg
    # a block between boxes of different depths (with a V factor of the right size)
    b3 = blocks.copy()
    par = int(t.parent[int(d.blocks.source[lr])])
    vbuf = np.zeros(t.size(par) * int(rank[lr]), np.float32)
    b3["source"][lr] = par
    b3["b"][lr] = vbuf.ctypes.data
    b3["ldb"][lr] = t.size(par)
    st, msg = _create_status(tree, b3)
    assert st == 3, msg
    # a low-rank block between two leaves (Def. 2.3 makes leaf pairs dense)
    dn = int(np.nonzero(rank == 0)[0][0])
    b4 = blocks.copy(); b4["rank"][dn] = 2; b4["b"][dn] = b4["a"][dn]; b4["ldb"][dn] = 64
    assert _create_status(tree, b4)[0] == 4
