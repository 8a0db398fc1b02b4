"""The seeded input generators: the device-drawn random fill has the same
per-block scaling as the host one, and is reproducible."""
import math

import numpy as np

from hmat_inputs import batch_problems, build_batch_member, uniform_tree, make_hmatrix


def _block_stds(d):
    sz = d.tree.end - d.tree.begin
    out = []
    for b in range(len(d.blocks)):
        t, s, r = int(d.blocks.target[b]), int(d.blocks.source[b]), int(d.blocks.rank[b])
        m, n = int(sz[t]), int(sz[s])
        oa = int(d.off_a[b])
        if r == 0:
            out.append((d.pool[oa:oa + m * n].std(), 1.0 / math.sqrt(n)))
        else:
            out.append((d.pool[oa:oa + m * r].std(), 1.0 / math.sqrt(r)))
            ob = int(d.off_b[b])
            out.append((d.pool[ob:ob + n * r].std(), 1.0 / math.sqrt(n)))
    return out


def test_device_random_fill_scaling_and_reproducibility():
    tree = uniform_tree(2, 64)
    a = make_hmatrix(tree, 8, method="random", seed=11, device="cpu")
    b = make_hmatrix(tree, 8, method="random", seed=11, device="cpu")
    c = make_hmatrix(tree, 8, method="random", seed=12, device="cpu")
    assert np.array_equal(a.pool, b.pool)
    assert not np.array_equal(a.pool, c.pool)
    for got, want in _block_stds(a):
        assert abs(got / want - 1.0) < 0.2, (got, want)


def test_batch_member_generator_shapes():
    specs = batch_problems(8, seed=4)
    for i, s in enumerate(specs):
        assert s["d"] == (2 if i % 2 == 0 else 3) and s["rank"] in (8, 16, 32)
        assert 4096 / 4 <= math.prod(s["shape"]) <= 65536 * 4
    d = build_batch_member(specs[1], method="random", seed=5, device="cpu")
    assert d.n == math.prod(specs[1]["shape"]) and np.isfinite(d.pool).all()
