"""Named synthetic workloads (grids, kernels, ranks, right-hand sides).

Each preset fixes the geometry (uniform grid in [0,1]^d, leaf 64), the kernel,
the rank, how the low-rank factors are computed, and the number of
right-hand sides with the seed they are drawn from (x ~ N(0,1), seed 1000 +
workload number).

  c1  2D, 64 x 64 grid (N = 4096), log kernel, rank 16, exact truncated SVD, 1 RHS
  c2  2D, 1024 x 1024 grid (N = 2^20), log kernel, rank 32, randomized SVD
      (oversampling 10), 1 RHS
  c3  3D, 64^3 grid (N = 262144), 1/r kernel, rank 64, randomized SVD, 64 RHS
  c4  256 independent sub-grid H-matrices (see ``batch_problems``)
  c5  3D, 128^3 grid (N = 2^21), 1/r kernel, rank 32, randomized SVD, 128 RHS
  s2  2D, 1024 x 1024 grid (N = 2^20), standard admissibility, rank 4, random
      fills (the paper's two-dimensional experiments: random factors, r = 4), 1 RHS
  s3  3D, 64^3 grid (N = 262144), standard admissibility, rank 4, random fills, 1 RHS

Weak admissibility unless stated otherwise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .factors import HMatrixData, make_hmatrix, make_rhs
from .tree import build_tree, uniform_tree


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    d: int
    n_axis: int
    kind: str
    rank: int
    method: str
    nrhs: int
    rhs_seed: int
    admissibility: str = "weak"

    @property
    def n(self) -> int:
        return self.n_axis ** self.d

    def describe(self) -> str:
        kern = "-log|x-y|/(2pi)" if self.kind == "log" else "1/(4pi|x-y|)"
        return (f"{self.d}D uniform grid {self.n_axis}^{self.d} (N={self.n}), leaf 64, "
                f"kernel {kern} (diag 1), {self.admissibility} admissibility, rank {self.rank} "
                f"({self.method}), {self.nrhs} RHS")


WORKLOADS = {
    "c1": Workload("c1", 2, 64, "log", 16, "svd", 1, 1001),
    "c2": Workload("c2", 2, 1024, "log", 32, "rsvd", 1, 1002),
    "c3": Workload("c3", 3, 64, "inv", 64, "rsvd", 64, 1003),
    "c5": Workload("c5", 3, 128, "inv", 32, "rsvd", 128, 1005),
    "s2": Workload("s2", 2, 1024, "log", 4, "random", 1, 1006, "standard"),
    "s3": Workload("s3", 3, 64, "inv", 4, "random", 1, 1007, "standard"),
}


def build_workload(name: str, *, method: str | None = None, device=None, seed: int = 0,
                   n_axis: int | None = None, rank: int | None = None):
    """Tree, canonical factors and RHS for a named workload.

    ``n_axis``/``rank``/``method`` override the preset (scaled-down variants for tests).
    """
    w = WORKLOADS[name]
    n_axis = n_axis or w.n_axis
    tree = uniform_tree(w.d, n_axis)
    data = make_hmatrix(tree, rank or w.rank, kind=w.kind, method=method or w.method,
                        seed=seed, device=device, admissibility=w.admissibility)
    x = make_rhs(tree.n, w.nrhs, w.rhs_seed)
    return data, x


def batch_problems(count: int = 256, seed: int = 4, *, nmin: int = 4096, nmax: int = 65536):
    """Geometry of the batched workload: ``count`` random sub-grids.

    Matrix b is 2D (log kernel) when b is even and 3D (1/r kernel) when b is odd.
    Its target size N* is log-uniform in [nmin, nmax]; per-axis aspect factors
    are log-uniform in [1/2, 2], normalised to a product of 1; the axis sizes
    n_a = clamp(round(N*^(1/d) a_a), lo, full) with lo = 8 (2D) or 4 (3D) and a
    full grid of 256^2 (2D) or 64^3 (3D); the sub-grid sits at a random integer
    offset of the full grid and uses the full grid's cell centres. The rank is
    uniform on {8, 16, 32}.

    Returns a list of dicts with keys d, kind, shape, offset, n_full, rank.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        d = 2 if b % 2 == 0 else 3
        full = 256 if d == 2 else 64
        lo = 8 if d == 2 else 4
        nstar = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        a = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=d))
        a = a / np.prod(a) ** (1.0 / d)
        shape = [int(min(full, max(lo, round(nstar ** (1.0 / d) * a[i])))) for i in range(d)]
        offset = [int(rng.integers(0, full - shape[i] + 1)) for i in range(d)]
        rank = int(rng.choice([8, 16, 32]))
        out.append(dict(d=d, kind="log" if d == 2 else "inv", shape=tuple(shape),
                        offset=tuple(offset), n_full=(full,) * d, rank=rank))
    return out


def build_batch_member(spec: dict, *, method: str = "rsvd", seed: int = 0, device=None,
                       gpu_min_entries: int = 1 << 24):
    """Factor set of one member of ``batch_problems`` (see ``make_hmatrix`` for the methods)."""
    tree = build_tree(spec["shape"], n_full=spec["n_full"], offset=spec["offset"])
    return make_hmatrix(tree, spec["rank"], kind=spec["kind"], method=method, seed=seed,
                        device=device, gpu_min_entries=gpu_min_entries)
