"""Oracle for the H^2-matrix-vector product -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module; the GPU library shares no code with it.

The H^2-matrix (the nested-basis format that Sec. 1 introduces beside the
H-matrix; the Sec. 3.2 remark on distributing its bases and its small middle
matrices) has the block structure of Def. 2.3 with every low-rank block
(t, s) written U_t S_ts V_s^T. Its product is therefore Eq. (2.4) with those
blocks:

    y = sum over dense blocks of D_ts x_s + sum over low-rank blocks of U_t (S_ts (V_s^T x_s)).

This oracle evaluates exactly that sum in FP64, with each box's bases written
out from their definition: a leaf's U_t and V_t as stored, and for a box with
children c_1, c_2, ... the stacked products

    U_t = [U_c1 E_c1; U_c2 E_c2; ...],   V_t = [V_c1 F_c1; V_c2 F_c2; ...].

The factors are read from the FP32 pool and promoted exactly. No upward or
downward pass is used: the passes are the library's reordering of this sum.
"""
from __future__ import annotations

import numpy as np


def expanded_bases(h2):
    """{node: (U_t, V_t)} in FP64 for every node with a basis, written out from the
    leaves upward by the nested definition."""
    tree = h2.tree
    out = {}
    for t in sorted(range(tree.num_nodes), key=lambda a: -int(tree.depth[a])):
        if h2.rank[t] == 0:
            continue
        if tree.is_leaf(t):
            out[t] = (h2.leaf_u(t).astype(np.float64), h2.leaf_v(t).astype(np.float64))
            continue
        us, vs = [], []
        for c in tree.children[t]:                   # children in tree order tile t's rows
            uc, vc = out[c]
            us.append(uc @ h2.transfer_e(c).astype(np.float64))
            vs.append(vc @ h2.transfer_f(c).astype(np.float64))
        out[t] = (np.vstack(us), np.vstack(vs))
    return out


def h2_oracle_matvec(h2, x, *, alpha: float = 1.0, beta: float = 0.0, y_in=None, bases=None) -> np.ndarray:
    """y = alpha K x + beta y_in in FP64 for an ``hmat_inputs.h2.H2Data``; x is n x k."""
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[:, None]
    xd = x.astype(np.float64)
    tree, blocks = h2.tree, h2.blocks
    if xd.shape[0] != tree.n:
        raise ValueError("x has the wrong number of rows")
    bases = expanded_bases(h2) if bases is None else bases
    y = np.zeros_like(xd)
    for b in range(len(blocks)):
        t, s = int(blocks.target[b]), int(blocks.source[b])
        rt = slice(int(tree.begin[t]), int(tree.end[t]))
        rs = slice(int(tree.begin[s]), int(tree.end[s]))
        if blocks.rank[b] == 0:
            y[rt] += h2.dense(b).astype(np.float64) @ xd[rs]
        else:
            u_t = bases[t][0]
            v_s = bases[s][1]
            y[rt] += u_t @ (h2.coupling(b).astype(np.float64) @ (v_s.T @ xd[rs]))
    out = alpha * y
    if beta != 0.0:
        if y_in is None:
            raise ValueError("beta != 0 needs y_in")
        out = out + beta * np.asarray(y_in, dtype=np.float64).reshape(out.shape)
    return out
