// Internal interface between the host side of the H^2 product and its HIP
// kernels (hmat_h2.hip).
//
// Device layout (built by hmat_h2_create):
//
//  * Chunks are the boxes at depth max(L-1, 0), as for the H-matrix; their
//    children are the leaves ("leaf" below always means a leaf child of a
//    chunk; when the root is itself a leaf, the chunk is its own leaf).
//
//  * V panel: per leaf, its basis V_t in tiles of 64 rows; lane l owns row l
//    of the tile and reads VW consecutive basis columns per 16-byte load:
//    element (i, j) of tile i / 64 sits at
//        v_off + (i / 64) * kq * 64 * VW + ((j / VW) * 64 + i % 64) * VW + j % VW,
//    rows past the leaf hold zeros. One wave-load is a contiguous 1 KiB.
//
//  * UD panel: per chunk, rows in tiles of 64 (lane = row), columns: the U
//    basis of the row's own leaf (nq_u vectors of VW, zero beyond its rank),
//    then the dense leaf blocks grouped by source leaf (each padded to VW
//    columns), the same form as the H-matrix's target-side panel.
//
//  * Small matrices (transfers and couplings) in one array, stored by rows
//    (each row padded to a multiple of 16 bytes, every matrix 16-byte aligned),
//    so that a lane owning one output reads its row in 16-byte loads: E_t
//    (k_t x k_parent), F_t transposed (k_parent x k_t), couplings S_ts
//    (k_t x k_s).
//
//  * Workspace: x^ and y^ of every node with a basis (k_t values each).
#pragma once

#include <cstdint>

#include "hmat_internal.h"

namespace hmat {

struct H2Leaf {
    int32_t row_begin;    // global first row
    int32_t rows;
    int32_t k;            // basis rank (0 when the tree has no bases)
    int32_t kq;           // VW-vectors of a basis row: ceil(k / VW)
    int64_t v_off;        // element offset of its V tiles in the V panel
    int32_t ft_off;       // F^T of the leaf (k_chunk x k) in the small array, -1 when the chunk has no basis
    int32_t e_off;        // E of the leaf (k x k_chunk), -1 likewise
    int32_t ft_ld;        // their row strides in the small array
    int32_t e_ld;
    float sv;             // scales of its stored V, U, F and E arrays (1 in FP32)
    float su;
    float sf;
    float se;
};

struct H2Chunk {
    int32_t row_begin;
    int32_t rows;
    int32_t leaf_base;    // first of its leaves in the leaf table
    int32_t nleaf;
    int32_t nq;           // VW-vectors per row of the UD panel
    int32_t nq_u;         // of which the U basis part
    int64_t ud_off;       // element offset of its UD panel
    int32_t dseg_base;    // its dense source leaves (DSeg)
    int32_t nsrc;
    int32_t dscale_base;  // nleaf x nsrc dense-block scales (FP16 form)
    int32_t k;            // chunk basis rank (0: none)
    int32_t xh;           // offset of its x^ in the workspace
    int32_t term_base;    // terms of its y^: E_chunk y^_parent, then its couplings
    int32_t nterm;
    int32_t vec_floats;   // LDS floats of the dense vector operand
};

// One matrix-vector term of a node's y^ (downward pass: y^_t += s * M w with
// M = E_t and w = y^_parent, or M = S_ts and w = x^_s) or x^ (upward pass:
// x^_t += s * M w with M = F_c^T and w = x^_c).
struct H2Term {
    int32_t m_off;        // small-array offset of M (k_t rows, stored by rows)
    int32_t src;          // workspace offset of w: x^ entries, or y^ entries (y_from = 1)
    int32_t cols;         // length of w
    int32_t y_from;       // w comes from the y^ half of the workspace
    float scale;
    int32_t ldm;          // row stride of M
};

struct H2Node {           // a node above the chunks (depth 1 .. L-2)
    int32_t k;
    int32_t xh;           // offset of its x^ (and of its y^ in the y^ half)
    int32_t up_base;      // H2Term list of its children's F^T x^
    int32_t nup;
    int32_t term_base;    // H2Term list of its y^
    int32_t nterm;
};

struct DevPlanH2 {
    int32_t storage;
    int32_t L;
    int32_t num_chunks;
    int32_t kmax;             // largest basis rank
    int32_t lds_b_floats;     // dynamic LDS of the leaf kernel
    int32_t ws_half;          // floats in each half (x^, y^) of the workspace
    const void *V;
    const void *UD;
    const void *small;        // transfers and couplings (float or _Float16 codes)
    float *ws;                // x^ at [0, ws_half), y^ at [ws_half, 2 ws_half)
    const H2Chunk *chunks;
    const H2Leaf *leaves;
    const DSeg *dsegs;
    const float *dscale;
    const H2Node *nodes;
    const H2Term *terms;
};

// Launchers (hmat_h2.hip); each returns a hipError_t as int.
int launch_h2_upward(const DevPlanH2 &p, const float *x, void *stream);
int launch_h2_up(const DevPlanH2 &p, int32_t first, int32_t count, void *stream);
int launch_h2_down(const DevPlanH2 &p, int32_t first, int32_t count, void *stream);
int launch_h2_leaf(const DevPlanH2 &p, const float *x, float *y, float alpha, float beta, void *stream);

}  // namespace hmat
