"""Pins of the dequantising oracle (oracle/quant.py) against the storage rules.

The low-precision parity tests compare the GPU with the FP64 oracle evaluated
over the *dequantised* factors of Def. 2.3 (the values D_ts, U_ts, V_ts take in
each storage form). These tests pin that dequantiser to the rules themselves,
by routes that share nothing with it:

  * rounding to p significant bits is recomputed from frexp / rint (numpy's
    rint rounds halves to even), with gradual underflow below the format's
    smallest normal, instead of numpy's float16 or torch's bfloat16 casts;
  * the power-of-two scale is recomputed from frexp (amax = m 2^e) instead of
    a logarithm: s = 2^(E - 15) for the smallest E with amax <= 2^E, at least
    2^-126, and 1 for an all-zero array;
  * the per-block dispatch of ``dequantised`` is checked array by array: one
    scale per stored U or V array in the FP16 form and one per group of dense
    blocks (those whose target leaves have one parent and whose source leaves
    have one parent, the groups found here from the tree), the dense blocks of the FP8 form
    through BF16 of v / s and those of the FP8 + FP16 D form through the FP16
    rule, and U and V per column in both FP8 forms;
  * the library's host quantiser (compiled from its source into the probe)
    reproduces the oracle's FP16 and BF16-of-scaled values bit for bit.

Planted mistakes (a wrong scale exponent, D through the wrong rule, a scale
per column instead of per array, a dense block's own scale instead of its
group's, BF16 by truncation, FP16 by truncation) are made in a copy of the
oracle's source and each must fail one of these pins.
"""
import copy
import os
import subprocess
import types

import numpy as np
import pytest

import oracle.quant as quant
from hmat_inputs import make_hmatrix, uniform_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
QUANT_SRC = os.path.join(ROOT, "oracle", "quant.py")


# ---------------------------------------------------------------------------
# Independent references of the rules
# ---------------------------------------------------------------------------
def round_sig(w, p, emin_frexp):
    """Round w (float64) to the nearest value with p significant bits, ties to
    even; below 2^(emin_frexp - 1) (the smallest normal) the quantum stays
    2^(emin_frexp - p) (gradual underflow). FP16: p = 11, emin_frexp = -13;
    BF16: p = 8, emin_frexp = -125."""
    w = np.asarray(w, dtype=np.float64)
    _, e = np.frexp(w)
    e = np.maximum(e, emin_frexp)
    return np.ldexp(np.rint(np.ldexp(w, p - e)), e - p)


def rne_f16(w):
    return round_sig(w, 11, -13)


def rne_bf16(w):
    return round_sig(w, 8, -125)


def scale_rule(amax: float) -> float:
    """s = 2^(ceil(log2 amax) - 15), at least 2^-126; 1 for amax == 0."""
    if amax == 0.0:
        return 1.0
    m, e = np.frexp(np.float64(amax))
    big_e = int(e) - 1 if m == 0.5 else int(e)      # smallest E with amax <= 2^E
    return float(np.ldexp(1.0, max(big_e - 15, -126)))


def ref_fp16_array(a, amax=None):
    """FP16 values of a with the scale of amax (a's own largest |entry| by default)."""
    a = np.asarray(a, dtype=np.float32)
    if amax is None:
        amax = float(np.max(np.abs(a))) if a.size else 0.0
    s = scale_rule(amax)
    return (rne_f16(a.astype(np.float64) / s) * s).astype(np.float32)


def ref_bf16(a):
    return rne_bf16(np.asarray(a, dtype=np.float32).astype(np.float64)).astype(np.float32)


def ref_dense_bf16_scaled(a, amax=None):
    a = np.asarray(a, dtype=np.float32)
    if amax is None:
        amax = float(np.max(np.abs(a))) if a.size else 0.0
    s = scale_rule(amax)
    return (rne_f16(rne_bf16(a.astype(np.float64) / s)) * s).astype(np.float32)


def dense_groups(data):
    """Per dense block, the largest |entry| over its group: the dense blocks whose
    target leaf is a child of the same box as its own, and whose source leaf is."""
    sz = data.tree.end - data.tree.begin
    par = data.tree.parent
    dense = [b for b in range(len(data.blocks)) if int(data.blocks.rank[b]) == 0]
    out = {}
    for b in dense:
        t, s = int(data.blocks.target[b]), int(data.blocks.source[b])
        mates = [c for c in dense if int(par[int(data.blocks.source[c])]) == int(par[s]) and
                 int(par[int(data.blocks.target[c])]) == int(par[t])]
        out[b] = max(float(np.max(np.abs(data.pool[int(data.off_a[c]):int(data.off_a[c]) +
                                                   int(sz[data.blocks.target[c]]) *
                                                   int(sz[data.blocks.source[c]])]))) for c in mates)
    return out


# ---------------------------------------------------------------------------
# Inputs
# ---------------------------------------------------------------------------
def scale_amaxes():
    rng = np.random.default_rng(11)
    vals = [np.abs(rng.standard_normal(3000)) * 10.0 ** rng.uniform(-40, 38, 3000),
            2.0 ** np.arange(-149, 128, dtype=np.float64),                  # exact powers of two
            np.nextafter(2.0 ** np.arange(-120, 120, dtype=np.float64).astype(np.float32), np.float32(np.inf)),
            np.nextafter(2.0 ** np.arange(-120, 120, dtype=np.float64).astype(np.float32), np.float32(0)),
            [1e-45, 1e-40, 2.0 ** -111, 2.0 ** -112, 3.0e38, 0.0]]          # tiny amax: the 2^-126 floor
    return np.concatenate([np.asarray(v, dtype=np.float64) for v in vals]).astype(np.float32)


def array_with_ties(rng, scale_exp: int, n: int = 4000):
    """A block-like array whose largest entry fixes s = 2^scale_exp, holding
    exact FP16 ties, exact BF16 ties, values in FP16's subnormal range, zeros
    and ordinary values."""
    s = 2.0 ** scale_exp
    f16_ties = (rng.integers(1 << 10, 1 << 11, n) + 0.5) * 2.0 ** rng.integers(-14, 5, n)   # w = v / s
    bf_ties = (rng.integers(1 << 7, 1 << 8, n) + 0.5) * 2.0 ** rng.integers(-20, 8, n)
    sub = rng.uniform(0, 2.0 ** -14, n) * rng.choice([-1, 1], n)
    ordinary = rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 4, n)
    w = np.concatenate([f16_ties * rng.choice([-1, 1], n), bf_ties * rng.choice([-1, 1], n), sub, ordinary,
                        [0.0, -0.0]])
    w = np.clip(w, -2.0 ** 14, 2.0 ** 14)
    w[0] = 2.0 ** 15 * (1 - 2.0 ** -11)          # amax in (2^14, 2^15]: s = 2^scale_exp
    a = (w * s).astype(np.float32)
    assert np.array_equal(a.astype(np.float64) / s, w.astype(np.float32).astype(np.float64))
    return a


def lowrank_test_set(seed=21):
    """Random factors on a 2D tree (N = 1024, L = 2: 12 low-rank blocks of rank 8
    and 256 dense blocks) whose U and V columns span very different magnitudes,
    so that a scale per column and a scale per array give different values."""
    data = make_hmatrix(uniform_tree(2, 32), 8, method="random", seed=seed)
    rng = np.random.default_rng(seed)
    pool = data.pool
    for b in range(len(data.blocks)):
        r = int(data.blocks.rank[b])
        m = int(data.tree.end[data.blocks.target[b]] - data.tree.begin[data.blocks.target[b]])
        n = int(data.tree.end[data.blocks.source[b]] - data.tree.begin[data.blocks.source[b]])
        oa = int(data.off_a[b])
        if r == 0:
            pool[oa:oa + m * n] *= np.float32(10.0 ** rng.uniform(-3, 3))
            continue
        ob = int(data.off_b[b])
        for off, rows in ((oa, m), (ob, n)):
            col = np.repeat(10.0 ** rng.uniform(-5, 3, r), rows).astype(np.float32)
            pool[off:off + rows * r] *= col
    return data


# ---------------------------------------------------------------------------
# The pins, written against any module with the oracle's interface, so that the
# planted mistakes below can be run through the same checks.
# ---------------------------------------------------------------------------
def pin_scale_rule(q):
    bad = []
    for amax in scale_amaxes().astype(np.float64):
        s = q.fp16_scale(float(amax))
        if s != scale_rule(float(amax)):
            bad.append((amax, s))
    assert not bad, f"fp16_scale differs from the rule at {bad[:3]}"
    # properties of the rule itself: a power of two with amax / s in (2^14, 2^15], or the floor
    for amax in scale_amaxes().astype(np.float64):
        s = scale_rule(float(amax))
        assert np.frexp(s)[0] == 0.5
        if amax > 0:
            assert amax / s <= 2.0 ** 15
            assert amax / s > 2.0 ** 14 or s == 2.0 ** -126


def pin_fp16_values(q):
    rng = np.random.default_rng(12)
    for scale_exp in (-40, -15, 0, 3, 20):
        a = array_with_ties(rng, scale_exp)
        got = q._dequant_fp16(a)
        ref = ref_fp16_array(a)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"FP16 values differ (s = 2^{scale_exp})"
        s = 2.0 ** scale_exp
        w = got.astype(np.float64) / s
        assert np.all(np.abs(w) <= 2.0 ** 15)
        assert np.array_equal(w.astype(np.float16).astype(np.float64), w), "a value is not an FP16 multiple of s"
    # an all-zero array and an empty one
    assert np.array_equal(q._dequant_fp16(np.zeros(7, np.float32)), np.zeros(7, np.float32))
    assert q._dequant_fp16(np.zeros(0, np.float32)).size == 0


def pin_bf16_values(q):
    rng = np.random.default_rng(13)
    a = np.concatenate([array_with_ties(rng, 0), array_with_ties(rng, -60), array_with_ties(rng, 40),
                        (rng.integers(1 << 7, 1 << 8, 500) + 0.5) * 2.0 ** -133]).astype(np.float32)
    got = q._dequant_bf16(a)
    ref = ref_bf16(a)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), "BF16 values differ from RNE"
    assert np.all((got.view(np.uint32) & 0xFFFF) == 0)


def pin_dense_bf16_scaled(q):
    rng = np.random.default_rng(14)
    for scale_exp in (-30, -15, 0, 6):
        a = array_with_ties(rng, scale_exp)
        got = q._dequant_dense_bf16_scaled(a)
        ref = ref_dense_bf16_scaled(a)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"BF16-of-scaled differs (s = 2^{scale_exp})"
        # above FP16's normal range the value is the BF16 value itself (8 significant bits)
        w = got.astype(np.float64) / 2.0 ** scale_exp
        big = np.abs(w) >= 2.0 ** -14
        assert np.array_equal(rne_bf16(w[big]), w[big])


def _check_block_arrays(q, form):
    data = lowrank_test_set()
    out = q.dequantised(data, form)
    assert out is not data and out.pool is not data.pool
    sz = data.tree.end - data.tree.begin
    gmax = dense_groups(data)
    for b in range(len(data.blocks)):
        r = int(data.blocks.rank[b])
        m, n = int(sz[data.blocks.target[b]]), int(sz[data.blocks.source[b]])
        oa = int(data.off_a[b])
        if r == 0:
            src = data.pool[oa:oa + m * n]
            got = out.pool[oa:oa + m * n]
            if form == "bf16":
                ref = ref_bf16(src)
            elif form == "fp8":
                ref = ref_dense_bf16_scaled(src, gmax[b])
            else:
                ref = ref_fp16_array(src, gmax[b])             # one scale for the block's group
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"{form}: dense block {b}"
            continue
        ob = int(data.off_b[b])
        for off, rows in ((oa, m), (ob, n)):
            src = data.pool[off:off + rows * r]
            got = out.pool[off:off + rows * r]
            if form == "bf16":
                ref = ref_bf16(src)
            elif form == "fp16":
                ref = ref_fp16_array(src)                       # one scale for the whole U_ts (or V_ts)
            else:
                ref = np.concatenate([_ref_fp8_column(c) for c in src.reshape(r, rows)])
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"{form}: low-rank block {b}"
    # the input is left untouched
    assert np.array_equal(data.pool, lowrank_test_set().pool)


def _ref_fp8_column(col):
    """FP8 hi + lo value of one factor column (the column split itself is pinned
    against the library's host quantiser in test_quant_cpu.py; here it is only
    applied column by column, to check the dispatch)."""
    return quant._dequant_fp8_columns(np.ascontiguousarray(col), col.size, 1)


def pin_dispatch(q):
    assert q.dequantised(lowrank_test_set(), "fp32").pool is not None
    for form in ("fp16", "bf16", "fp8", "fp8_f16d"):
        _check_block_arrays(q, form)
    with pytest.raises(ValueError):
        q.dequantised(lowrank_test_set(), "int4")


PINS = {"scale_rule": pin_scale_rule, "fp16_values": pin_fp16_values, "bf16_values": pin_bf16_values,
        "dense_bf16_scaled": pin_dense_bf16_scaled, "dispatch": pin_dispatch}


@pytest.mark.parametrize("name", sorted(PINS))
def test_pin(name):
    PINS[name](quant)


def test_scale_granularity_is_observable():
    """The test set distinguishes a scale per array from one per column: with
    per-column scales, some U entries would take a different value; and a dense
    block's own scale from its group's: some groups mix magnitudes."""
    data = lowrank_test_set()
    b = int(np.nonzero(data.blocks.rank > 0)[0][0])
    u = data.u(b)
    per_array = ref_fp16_array(np.asfortranarray(u).reshape(-1, order="F"))
    per_col = np.concatenate([ref_fp16_array(u[:, j]) for j in range(u.shape[1])])
    assert not np.array_equal(per_array, per_col)
    gmax = dense_groups(data)
    sz = data.tree.end - data.tree.begin
    differ = 0
    for d, g in gmax.items():
        oa, m, n = int(data.off_a[d]), int(sz[data.blocks.target[d]]), int(sz[data.blocks.source[d]])
        a = data.pool[oa:oa + m * n]
        differ += not np.array_equal(ref_fp16_array(a), ref_fp16_array(a, g))
    assert differ > 0


# ---------------------------------------------------------------------------
# Host quantiser against the oracle, bit for bit
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("qo") / "quant_probe")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    f"-I{ROOT}/include", f"-I{ROOT}/paper_2008_12441_amd/csrc",
                    os.path.join(ROOT, "tests", "quant_probe.cpp"), "-o", exe,
                    "-L/opt/rocm/lib", "-lamdhip64", "-lpthread"], check=True)
    return exe


def _host_block(exe, mode, a):
    payload = np.array([mode], np.int32).tobytes() + np.ascontiguousarray(a, np.float32).tobytes()
    out = subprocess.run([exe, "blk16"], input=payload, capture_output=True, check=True,
                         env={**os.environ, "LD_LIBRARY_PATH": "/opt/rocm/lib"}).stdout
    s = float(np.frombuffer(out[:4], "<f4")[0])
    codes = np.frombuffer(out[4:], "<u2")
    return s, codes


@pytest.mark.parametrize("scale_exp", [-40, -15, 0, 7])
def test_host_fp16_block_matches_oracle(probe, scale_exp):
    a = array_with_ties(np.random.default_rng(100 + scale_exp), scale_exp)
    s, codes = _host_block(probe, 0, a)
    host = (codes.view(np.float16).astype(np.float64) * s).astype(np.float32)
    assert s == quant.fp16_scale(float(np.max(np.abs(a))))
    assert np.array_equal(host.view(np.uint32), quant._dequant_fp16(a).view(np.uint32))


@pytest.mark.parametrize("scale_exp", [-40, -15, 0, 7])
def test_host_dense_bf16_block_matches_oracle(probe, scale_exp):
    a = array_with_ties(np.random.default_rng(200 + scale_exp), scale_exp)
    s, codes = _host_block(probe, 1, a)
    bvals = (codes.astype(np.uint32) << 16).view(np.float32)
    host = (bvals.astype(np.float16).astype(np.float64) * s).astype(np.float32)
    assert np.array_equal(host.view(np.uint32), quant._dequant_dense_bf16_scaled(a).view(np.uint32))


# ---------------------------------------------------------------------------
# Planted mistakes
# ---------------------------------------------------------------------------
MUTANTS = {
    "scale_exponent_14": [("return 2.0 ** max(c - 15, -126)", "return 2.0 ** max(c - 14, -126)")],
    "fp8_dense_via_fp16": [('dq = _dequant_dense_bf16_scaled if form == "fp8" else _dequant_fp16',
                            "dq = _dequant_fp16")],
    "fp8_f16d_dense_via_bf16": [('dq = _dequant_dense_bf16_scaled if form == "fp8" else _dequant_fp16',
                                 "dq = _dequant_dense_bf16_scaled")],
    "dense_scale_per_block": [("pool[oa:oa + m * n] = dq(pool[oa:oa + m * n], group[(int(parent[t]), int(parent[s]))])",
                               "pool[oa:oa + m * n] = dq(pool[oa:oa + m * n])")],
    "dense_group_per_source_leaf": [("key = (int(parent[t]), int(parent[s]))", "key = (int(parent[t]), s)"),
                                    ("group[(int(parent[t]), int(parent[s]))]", "group[(int(parent[t]), s)]")],
    "fp16_scale_per_column": [
        ("pool[oa:oa + m * r] = _dequant_fp16(pool[oa:oa + m * r])",
         "pool[oa:oa + m * r] = np.concatenate([_dequant_fp16(c) for c in np.split(pool[oa:oa + m * r], r)])")],
    "bf16_truncated": [("return t.to(torch.bfloat16).to(torch.float32).numpy()",
                        "return (t.numpy().view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)")],
    "dense_bf16_truncated": [(".to(torch.bfloat16).to(torch.float32)\n",
                              ".view(torch.int32).bitwise_and(-65536).view(torch.float32)\n")],
    "fp16_truncated": [("q = (a.astype(np.float64) / s).astype(np.float32).astype(np.float16)",
                        "q = np.trunc((a.astype(np.float64) / s) * 2.0 ** 10) / 2.0 ** 10")],
}


def _mutant(name):
    src = open(QUANT_SRC).read()
    for old, new in MUTANTS[name]:
        assert old in src, f"mutation anchor missing for {name}: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType(f"quant_{name}")
    exec(compile(src, f"<quant mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pins_pass(q) -> bool:
    for pin in PINS.values():
        try:
            pin(q)
        except AssertionError:
            return False
    return True


def test_unmutated_copy_passes():
    mod = types.ModuleType("quant_copy")
    exec(compile(open(QUANT_SRC).read(), "<quant copy>", "exec"), mod.__dict__)
    assert _pins_pass(mod)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_quant_mutant_is_caught(name):
    assert not _pins_pass(_mutant(name)), f"pins missed mutant {name}"


def test_dequantised_copies_metadata():
    data = lowrank_test_set()
    out = quant.dequantised(data, "fp16")
    assert out.blocks is data.blocks and out.tree is data.tree
    assert np.array_equal(out.off_a, data.off_a) and np.array_equal(out.off_b, data.off_b)
    assert copy.copy(out).pool is out.pool
