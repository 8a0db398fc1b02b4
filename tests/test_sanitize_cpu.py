"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host sources (tree and Def. 2.3 validation, the level-ordered layouts and
their fills, the quantisers, the multi-RHS plans, the batch queue and
autotuner, hmat_compress's block sets, the H^2 layout) are compiled with
g++ -fsanitize=address,undefined and linked against host stand-ins for the
HIP runtime (tests/sanitize_stubs.cpp: device memory is host memory, launches
do nothing). tests/sanitize_driver.cpp then drives the C ABI over each
structure below -- every storage form, both plans, a batch, the construction,
and malformed variants that must be rejected -- and any sanitizer report
fails the run.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from hmat_inputs import build_tree, make_hmatrix, uniform_tree
from hmat_inputs.h2 import make_h2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_12441_amd", "csrc")
SOURCES = [os.path.join(CSRC, s) for s in ("hmat_host.cpp", "hmat_batch_host.cpp", "hmat_structure.cpp",
                                          "hmat_h2_host.cpp")] + \
          [os.path.join(ROOT, "tests", s) for s in ("sanitize_stubs.cpp", "sanitize_driver.cpp")]
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:halt_on_error=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    objs = [str(d / (os.path.basename(s) + ".o")) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=4) as pool:
        list(pool.map(lambda so: subprocess.run(["g++", *FLAGS, "-c", so[0], "-o", so[1]], check=True),
                      zip(SOURCES, objs)))
    exe = str(d / "sanitize_driver")
    subprocess.run(["g++", *FLAGS, *objs, "-o", exe, "-lpthread"], check=True)
    return exe, d


def _write(path, magic, tree, target, source, rk, off_a, off_b, pool, extra=None):
    with open(path, "wb") as f:
        n = tree.n
        np.array([magic], np.int32).tofile(f)
        np.array([n], np.int64).tofile(f)
        np.array([tree.num_nodes, len(target), tree.d], np.int32).tofile(f)
        np.asarray(tree.parent, np.int32).tofile(f)
        np.asarray(tree.begin, np.int64).tofile(f)
        np.asarray(tree.end, np.int64).tofile(f)
        for a in (target, source, rk):
            np.asarray(a, np.int32).tofile(f)
        for a in (off_a, off_b):
            np.asarray(a, np.int64).tofile(f)
        if extra is not None:
            np.asarray(extra[0], np.int32).tofile(f)
            for a in extra[1:]:
                np.asarray(a, np.int64).tofile(f)
        np.array([pool.size], np.int64).tofile(f)
        np.asarray(pool, np.float32).tofile(f)
        np.asarray(tree.points, np.float32).tofile(f)


def _run(exe, path, tmp):
    r = subprocess.run([exe, str(path)], capture_output=True, text=True, env={**ENV, "HMAT_SANITIZE_TMP": str(tmp)},
                       timeout=600)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "OK" in r.stdout, out[-4000:]


H_CASES = {
    "2d-64x64": (lambda: uniform_tree(2, 64), "weak"),
    "2d-ragged-40x23": (lambda: build_tree((40, 23), n_full=(256, 256)), "weak"),
    "3d-ragged-17x33x9": (lambda: build_tree((17, 33, 9), n_full=(64, 64, 64)), "weak"),
    "1d-1024": (lambda: uniform_tree(1, 1024), "weak"),
    "2d-L0": (lambda: uniform_tree(2, 8), "weak"),
    "2d-L1": (lambda: uniform_tree(2, 16), "weak"),
    "2d-64x64-standard": (lambda: uniform_tree(2, 64), "standard"),
    "3d-16-standard": (lambda: uniform_tree(3, 16), "standard"),
}


@pytest.mark.parametrize("name", sorted(H_CASES))
def test_host_code_sanitized_h(driver, name):
    exe, tmp = driver
    tree_fn, adm = H_CASES[name]
    data = make_hmatrix(tree_fn(), 8, method="random", seed=3, admissibility=adm)
    b = data.blocks
    path = tmp / f"h_{name}.bin"
    _write(path, 1, data.tree, b.target, b.source, b.rank, data.off_a, np.maximum(data.off_b, 0), data.pool)
    _run(exe, path, tmp)


H2_CASES = {
    "2d-64x64": (lambda: uniform_tree(2, 64), "weak", 8),
    "2d-ragged-255x130": (lambda: build_tree((255, 130), n_full=(256, 256)), "weak", 12),
    "3d-16-standard": (lambda: uniform_tree(3, 16), "standard", 6),
    "2d-L1": (lambda: uniform_tree(2, 16), "weak", 4),
}


@pytest.mark.parametrize("name", sorted(H2_CASES))
def test_host_code_sanitized_h2(driver, name):
    exe, tmp = driver
    tree_fn, adm, k = H2_CASES[name]
    h2 = make_h2(tree_fn(), method="random", rank=k, seed=4, admissibility=adm)
    b = h2.blocks
    path = tmp / f"h2_{name}.bin"
    _write(path, 2, h2.tree, b.target, b.source, (b.rank > 0).astype(np.int32), h2.blk_off,
           np.zeros(len(b), np.int64), h2.pool, extra=(h2.rank, h2.u_off, h2.v_off, h2.e_off, h2.f_off))
    _run(exe, path, tmp)


# ---------------------------------------------------------------------------
# The OpenMP oracle under ThreadSanitizer, with LLVM's OpenMP runtime and its
# Archer tool supplying the runtime's synchronisation to TSan (GCC's libgomp is
# not instrumented, so TSan would take its barrier hand-offs for races).
# ---------------------------------------------------------------------------
LLVM = "/opt/rocm/llvm"
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")


def _tsan_build(src, out):
    subprocess.run([os.path.join(LLVM, "bin", "clang"), "-std=c11", "-O1", "-g", "-fsanitize=thread", "-fopenmp",
                    f"-L{LLVM}/lib", f"-Wl,-rpath,{LLVM}/lib", src, os.path.join(ROOT, "tests", "oracle_tsan_main.c"),
                    "-o", out], check=True)


def _tsan_run(exe, path):
    env = {**os.environ, "OMP_TOOL_LIBRARIES": ARCHER, "TSAN_OPTIONS": "halt_on_error=1 ignore_noninstrumented_modules=1",
           "OMP_NUM_THREADS": "4"}
    r = subprocess.run([exe, str(path)], capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(not os.path.exists(ARCHER), reason="LLVM's Archer OpenMP tool is not installed")
def test_oracle_threads_sanitized(driver, tmp_path):
    _, tmp = driver
    exe = str(tmp_path / "oracle_tsan")
    _tsan_build(os.path.join(ROOT, "oracle", "hmat_oracle.c"), exe)
    for name in ("2d-64x64", "3d-16-standard"):
        tree_fn, adm = H_CASES[name]
        data = make_hmatrix(tree_fn(), 8, method="random", seed=3, admissibility=adm)
        b = data.blocks
        path = tmp_path / f"o_{name}.bin"
        _write(path, 1, data.tree, b.target, b.source, b.rank, data.off_a, np.maximum(data.off_b, 0), data.pool)
        rc, out = _tsan_run(exe, path)
        assert rc == 0 and "ThreadSanitizer" not in out and "rc 0" in out, out[-4000:]
    # the check has teeth: a copy of the oracle with every pass-1 thread also adding into w[0] is caught
    src = open(os.path.join(ROOT, "oracle", "hmat_oracle.c")).read()
    anchor = "w[w_off[b] + k] = s;"
    assert anchor in src
    planted = tmp_path / "oracle_race.c"
    planted.write_text(src.replace(anchor, anchor + " w[0] += 1.0;"))
    exe2 = str(tmp_path / "oracle_race")
    _tsan_build(str(planted), exe2)
    rc, out = _tsan_run(exe2, tmp_path / "o_2d-64x64.bin")
    assert "ThreadSanitizer: data race" in out and "oracle_race.c" in out, out[-2000:]
