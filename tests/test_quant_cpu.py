"""The library's host quantisers bit-match independent library casts.

FP16 (round to nearest even) against numpy's float16 cast, BF16 against
torch's CPU bfloat16 cast, E4M3 against torch's float8_e4m3fn cast, the
power-of-two scale rules s = 2^(ceil(log2 amax) - 15) and
s = 2^ceil(log2(amax / 448)) against their definitions, and the FP8 hi + lo
column split against the oracle's independent implementation.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("q") / "quant_probe")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    f"-I{ROOT}/include", f"-I{ROOT}/paper_2008_12441_amd/csrc",
                    os.path.join(ROOT, "tests", "quant_probe.cpp"), "-o", exe,
                    "-L/opt/rocm/lib", "-lamdhip64", "-lpthread"], check=True)
    return exe


def run(exe, vals, inv=1.0):
    vals = np.ascontiguousarray(vals, dtype=np.float32)
    out = subprocess.run([exe, repr(float(inv))], input=vals.tobytes(), capture_output=True, check=True,
                         env={**os.environ, "LD_LIBRARY_PATH": "/opt/rocm/lib"}).stdout
    rec = np.frombuffer(out, dtype=np.dtype([("h", "<u2"), ("b", "<u2"), ("s", "<f4")]))
    return rec["h"], rec["b"], rec["s"]


def _values():
    rng = np.random.default_rng(0)
    v = [rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000)]
    # exact ties for FP16 (11 significant bits) and BF16 (8 bits), subnormals, edges
    base = rng.integers(1 << 10, 1 << 11, 2000).astype(np.float64)
    v.append(((base + 0.5) * 2.0 ** rng.integers(-20, 4, 2000)).astype(np.float32))
    b8 = rng.integers(1 << 7, 1 << 8, 2000).astype(np.float64)
    v.append(((b8 + 0.5) * 2.0 ** rng.integers(-60, 60, 2000)).astype(np.float32))
    v.append(np.array([0.0, -0.0, 65504.0, 65519.9, 65520.0, 7e-8, 3e-8, 6.1e-5, 5.9e-5, 1e-40,
                       np.inf, -np.inf, 3.4e38], np.float32))
    return np.concatenate(v).astype(np.float32)


def test_fp16_matches_numpy(probe):
    vals = _values()
    for inv in (1.0, 2.0 ** -7, 2.0 ** 9):
        h, _, _ = run(probe, vals, inv)
        with np.errstate(over="ignore"):
            ref = (vals * np.float32(inv)).astype(np.float16).view(np.uint16)
        assert np.array_equal(h, ref), np.nonzero(h != ref)[0][:5]


def test_bf16_matches_torch(probe):
    import torch

    vals = _values()
    _, b, _ = run(probe, vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(b, ref), np.nonzero(b != ref)[0][:5]
    # NaN stays NaN
    _, bn, _ = run(probe, np.array([np.nan], np.float32))
    assert (bn[0] & 0x7f80) == 0x7f80 and (bn[0] & 0x7f) != 0


def test_pow2_scale_rule(probe):
    rng = np.random.default_rng(1)
    a = np.concatenate([np.abs(rng.standard_normal(5000)) * 10.0 ** rng.uniform(-20, 20, 5000),
                        2.0 ** np.arange(-100, 100)]).astype(np.float32)
    _, _, s = run(probe, a)
    for amax, sc in zip(a.astype(np.float64), s.astype(np.float64)):
        c = int(np.ceil(np.log2(amax)))
        if 2.0 ** (c - 1) >= amax:
            c -= 1
        assert sc == 2.0 ** max(c - 15, -126)
        assert amax / sc <= 2.0 ** 15


def _run_mode(exe, mode, payload):
    return subprocess.run([exe, mode], input=payload, capture_output=True, check=True,
                          env={**os.environ, "LD_LIBRARY_PATH": "/opt/rocm/lib"}).stdout


def _e4m3_values():
    rng = np.random.default_rng(3)
    v = [rng.uniform(-448, 448, 20000), rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 2.6, 20000)]
    # every code's value, the midpoints between neighbours (ties), and the subnormal range
    import torch

    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    codes = np.sort(codes[np.isfinite(codes) & (codes >= 0)])
    mids = (codes[1:] + codes[:-1]) / 2
    v += [codes, -codes, mids, -mids, rng.uniform(0, 2.0 ** -6, 5000)]
    vals = np.concatenate(v)
    vals = vals[np.abs(vals) <= 448.0]
    return vals.astype(np.float32)


def test_e4m3_matches_torch(probe):
    import torch

    vals = _e4m3_values()
    out = _run_mode(probe, "e4m3", vals.tobytes())
    rec = np.frombuffer(out, dtype=np.dtype([("c", "u1"), ("s", "<f8")]))
    ref = torch.from_numpy(vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    bad = np.nonzero(rec["c"] != ref)[0]
    assert len(bad) == 0, [(float(vals[i]), int(rec["c"][i]), int(ref[i])) for i in bad[:5]]


def test_e4m3_scale_rule(probe):
    rng = np.random.default_rng(4)
    a = np.concatenate([np.abs(rng.standard_normal(5000)) * 10.0 ** rng.uniform(-30, 30, 5000),
                        448.0 * 2.0 ** np.arange(-60, 60), 448.0 * 2.0 ** np.arange(-60, 60) * 1.0000001,
                        [0.0]]).astype(np.float32)
    out = _run_mode(probe, "e4m3", a.tobytes())
    s = np.frombuffer(out, dtype=np.dtype([("c", "u1"), ("s", "<f8")]))["s"]
    for amax, sc in zip(a.astype(np.float64), s):
        if amax == 0:
            assert sc == 1.0
            continue
        assert amax / sc <= 448.0 < 2 * amax / sc, (amax, sc)
        assert sc == 2.0 ** round(np.log2(sc))


def test_fp8_column_split_matches_oracle(probe):
    """Column scales and hi/lo codes: the library's host split against the
    oracle's dequantiser, value for value."""
    import torch

    from oracle.quant import _dequant_fp8_columns

    rng = np.random.default_rng(5)
    rows, cols = 300, 24
    a = rng.standard_normal((rows, cols)) * 10.0 ** rng.uniform(-6, 3, cols)[None, :]
    a[:, 3] = 0.0                                   # an all-zero column
    a[:, 5] = 448.0 * 2.0 ** -10                    # every element exact in E4M3 (r = 0)
    a = a.astype(np.float32)
    flat = np.asfortranarray(a).reshape(-1, order="F")
    payload = np.array([rows, cols], np.int32).tobytes() + flat.astype(np.float32).tobytes()
    out = _run_mode(probe, "fp8col", payload)
    sc = np.frombuffer(out[:8 * cols], dtype="<f4").reshape(cols, 2).astype(np.float64)
    hl = np.frombuffer(out[8 * cols:], dtype="u1").reshape(cols, rows, 2)
    hi = torch.from_numpy(np.ascontiguousarray(hl[:, :, 0])).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    lo = torch.from_numpy(np.ascontiguousarray(hl[:, :, 1])).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    dev = sc[:, :1] * (hi + sc[:, 1:] * lo).astype(np.float16).astype(np.float64)   # columns x rows
    ref = _dequant_fp8_columns(flat, rows, cols).reshape(cols, rows).astype(np.float64)
    assert np.array_equal(dev.astype(np.float32), ref.astype(np.float32))
    assert sc[3, 0] == 1.0 and sc[3, 1] == 1.0 and sc[5, 1] == 1.0
