"""The library's host quantisers bit-match independent library casts.

FP16 (round to nearest even) against numpy's float16 cast, BF16 against
torch's CPU bfloat16 cast, and the power-of-two scale rule
s = 2^(ceil(log2 amax) - 15) against its definition.
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
