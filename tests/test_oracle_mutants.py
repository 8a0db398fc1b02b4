"""Planted mistakes in the oracle must fail at least one pin.

Each case edits a copy of the oracle's C source (on the CPU only), compiles it
into a temporary library and runs the P1/P2/P5 pins against it. A pin set that
lets any of these plausible mistakes through would not be pinning the oracle.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from hmat_inputs import dense_kernel, make_hmatrix, make_rhs, uniform_tree

SRC = os.path.join(os.path.dirname(oracle.__file__), "hmat_oracle.c")

MUTANTS = {
    "swap_u_v": [("const float *v = pool + off_b[b];", "const float *v = pool + off_a[b];"),
                 ("const float *u = pool + off_a[b];", "const float *u = pool + off_b[b];")],
    "drop_dense": [("acc[i - row_lo] += (double)dj[i - row_begin[b]] * xj;", "(void)dj; (void)xj;")],
    "lowrank_sign": [("acc[i - row_lo] += (double)uk[i - row_begin[b]] * wk;",
                      "acc[i - row_lo] -= (double)uk[i - row_begin[b]] * wk;")],
    "dense_transposed": [("acc[i - row_lo] += (double)dj[i - row_begin[b]] * xj;",
                          "acc[i - row_lo] += (double)d[(i - row_begin[b]) * ns + j] * xj; (void)dj;")],
    "x_from_target_rows": [("s += (double)v[(int64_t)k * ns + i] * xc[col_begin[b] + i];",
                            "s += (double)v[(int64_t)k * ns + i] * xc[row_begin[b] + i];")],
    "rank_off_by_one": [("for (int32_t k = 0; k < rank[b]; ++k) {\n                double s",
                         "for (int32_t k = 0; k < rank[b] - 1; ++k) {\n                double s")],
    "beta_scaled_by_alpha": [(": alpha * acc[i - row_lo] + beta * yc[i];",
                              ": alpha * (acc[i - row_lo] + beta * yc[i]);")],
}


def _build_mutant(tmp_path, name):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert old in src, f"mutation anchor missing for {name}: {old!r}"
        src = src.replace(old, new)
    cpath = tmp_path / f"{name}.c"
    cpath.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(cpath)],
                   check=True, capture_output=True)
    return oracle.bind(str(so))


def _pins_pass(lib) -> bool:
    tree = uniform_tree(2, 32)
    ok = True
    # P1 with random factors
    data = make_hmatrix(tree, 8, method="random", seed=3)
    x = make_rhs(tree.n, 2, 4)
    kh = oracle.assemble_dense(data)
    y = oracle.oracle_matvec(data, x, lib=lib)
    ref = kh @ x.astype(np.float64)
    ok &= bool(np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref))
    # P2 full rank
    full = make_hmatrix(tree, 0, method="fullrank")
    k32 = dense_kernel(tree, "log").astype(np.float32).astype(np.float64)
    y2 = oracle.oracle_matvec(full, x, lib=lib)
    ref2 = k32 @ x.astype(np.float64)
    ok &= bool(np.linalg.norm(y2 - ref2) <= 1e-12 * np.linalg.norm(ref2))
    # P5 alpha/beta
    y0 = np.random.default_rng(2).standard_normal((tree.n, 2))
    y3 = oracle.oracle_matvec(data, x, alpha=-1.5, beta=0.25, y_in=y0, lib=lib)
    ref3 = -1.5 * ref + 0.25 * y0
    ok &= bool(np.linalg.norm(y3 - ref3) <= 1e-13 * np.linalg.norm(ref3))
    return ok


def test_unmutated_source_passes(tmp_path):
    src = open(SRC).read()
    cpath = tmp_path / "clean.c"
    cpath.write_text(src)
    so = tmp_path / "libclean.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(cpath)],
                   check=True)
    assert _pins_pass(oracle.bind(str(so)))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build_mutant(tmp_path, name)), f"pins missed mutant {name}"
