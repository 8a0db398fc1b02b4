// Internal interface between the host side of libhmat and its HIP kernels.
//
// Device layout (built by hmat_create, streamed by the kernels):
//
//  * A "chunk" is a box at depth max(L-1, 0): the parent of a group of leaves.
//    Chunks tile [0, n) in tree order and are the unit of device work.
//
//  * V panel (source side, Sec. 4.1.1, Eq. (4.2)): for chunk p, its columns are
//    the V factors of every low-rank block whose source box contains p, level
//    by level from the root down, and inside a level ordered by target sibling.
//    The columns are cut into blocks of 64; one "vtile" = (chunk, column
//    block). A vtile stores rows in vectors of VW consecutive rows (VW = 4 for
//    FP32, 8 for FP16): element (i, 64 cb + l) sits at
//        off + ((i / VW) * 64 + l) * VW + i % VW,
//    so one 16-byte load per lane reads 64 columns x VW rows, 1 KiB per wave,
//    contiguous.
//
//  * UD panel (target side, Sec. 4.1.5, Eqs. (4.6)-(4.8)): for chunk p, its
//    columns are the U factors of every low-rank block whose target box
//    contains p (same level/sibling order, matching the z layout), then the
//    dense leaf blocks of p grouped by source leaf. Rows come in tiles of 64;
//    element (i, j) of tile i / 64 sits at
//        off + (i / 64) * nq * 64 * VW + ((j / VW) * 64 + i % 64) * VW + j % VW,
//    so each lane owns one row and reads VW columns per 16-byte load. The
//    low-rank part is padded to a multiple of VW columns, and so is each
//    source leaf of the dense part.
//
//  * part: per-chunk partial sums of V^T x (one float per V column of the
//    chunk, 64-padded). zg: per target box t, the concatenated vectors
//    z_ts = V_ts^T x_s over its siblings s, times the block's scales.
#pragma once

#include <cstddef>
#include <cstdint>

namespace hmat {

constexpr int kWave = 64;
constexpr int kMaxLdsBytes = 65536;   // U-phase vector operand budget per chunk (64 KiB)

struct ChunkMeta {
    int32_t row_begin;   // first global row
    int32_t rows;        // number of rows
    int32_t nq;          // VW-column vectors per row of the UD panel
    int32_t nq_lr;       // of which belong to the low-rank part
    int64_t ud_off;      // element offset of the chunk's UD panel
    int32_t zseg_base;   // index of its first z segment (L-1 of them)
    int32_t dseg_base;   // index of its first dense segment: nleaf source leaves, then ntleaf target leaves
    int32_t nleaf;       // number of source leaves of its dense blocks (dense segments)
    int32_t dscale_base; // index of its ntleaf x nleaf dense scales
    int32_t part_base;   // offset of its partial sums
    int32_t ntleaf;      // number of target leaves (its children)
};

struct ZSeg {            // a run of the U-phase vector taken from zg
    int32_t off;
    int32_t len;
};

struct DSeg {            // one source leaf of a chunk's dense part
    int32_t row_begin;   // global first row of the leaf (also its x offset)
    int32_t rows;        // |leaf|
    int32_t nq;          // VW-column vectors it spans (padded)
    int32_t pad_;
};

struct VTile {
    int64_t off;         // element offset of the tile in the V panel
    int32_t chunk;
    int32_t pout;        // index of its 64 partial sums in part
};

struct ZItem {           // stage 1 of the partial reduction
    int32_t chunk0;      // first chunk of the slice
    int32_t nchunks;     // chunks in the slice
    int32_t vcol;        // column of the block inside each chunk's partial vector
    int32_t rank;
    int32_t dst;         // destination offset (zg when final, else slice buffer)
    float scale;         // applied when final (1 otherwise)
};

struct ZItem2 {          // stage 2: sum of slices of a block spanning many chunks
    int32_t src;         // offset of its first slice in the slice buffer
    int32_t nslices;
    int32_t rank;
    int32_t dst;         // offset in zg
    float scale;
    int32_t pad_;
};

struct DevPlan {
    int32_t storage;          // hmat_storage
    int32_t fp64;             // HMAT_FLAG_FP64_ACCUM: part, slice, zg and all sums in double
    int32_t pad_;
    int32_t num_chunks;
    int32_t num_vtiles;
    int32_t num_z1;
    int32_t num_z2;
    int32_t num_levels;       // L - 1 (low-rank levels), >= 0
    int32_t lds_floats;       // largest U-phase vector (padded)
    int32_t max_leaf_rows;
    const void *V;            // float or _Float16
    const void *UD;
    void *part;               // float, or double in FP64 mode (offsets count elements)
    void *slice;
    void *zg;
    const ChunkMeta *chunks;
    const int32_t *pbase;     // per chunk: offset of its partial sums (= chunks[c].part_base)
    const ZSeg *zsegs;
    const DSeg *dsegs;
    const float *dscale;
    const VTile *vtiles;
    const ZItem *z1;
    const ZItem2 *z2;
};

// ---------------------------------------------------------------------------
// Multi-RHS layout (handles created with max_nrhs > 1): the products become
// matrix-matrix products on MFMA tiles of 16 x 16 outputs.
//
//  * Fragments: an A fragment is 16 rows x KB inner indices, stored as 64
//    lanes x 16 bytes (1 KiB): lane l holds row l % 16 and the VW consecutive
//    inner indices VW * (l / 16) + [0, VW) of that row (FP32: KB = 16, VW = 4,
//    fed to four 16x16x4 steps; FP16/BF16: KB = 32, VW = 8, one 16x16x32 step;
//    FP8 forms: KB = 32, VW = 8, the lane's 16 bytes are 8 hi codes then 8 lo
//    codes of U or V, or 8 BF16/FP16 codes of D, all fed as FP16).
//    A B fragment is KB inner indices x 16 columns with the mirrored lane
//    mapping (lane l: column l % 16, inner indices VW * (l / 16) + [0, VW)),
//    1 KiB for FP32, 2 KiB for FP16 (a high and a low half-precision part).
//  * Rows: a chunk's rows are taken contiguously and padded once, at the
//    chunk's end, on both sides, whatever its leaves: the target side's row
//    tiles run over the chunk's rows, and its dense part takes the rows of a
//    partner box (the source leaves of the dense blocks, whose scale the pair
//    of boxes shares) as one segment.
//  * V panel: per unit (level, source box, 64-column group, up to 4 chunks of
//    that box) the A fragments [chunk][K-block of its contiguous rows]
//    [m-subtile]; a wave computes the unit's V^T X and writes its partial sums
//    (64 x 16 NT floats).
//  * Xpack: per chunk the B fragments [K-block][n-tile] of X (FP16: hi/lo with
//    one power-of-two scale per chunk and n-tile of 16 columns).
//  * Zpack: per z item (the low-rank blocks of one target box, up to 128 rows
//    of z in all) the B fragments [K-block][n-tile] of their z stacked in the
//    box's block order, so that blocks of small rank share K-blocks (FP16:
//    hi/lo, one power-of-two scale per item and n-tile).
//  * UD panel: per row tile (<= 64 contiguous rows of one chunk) the A fragments
//    [K-block over its segments][m-subtile]; segments are the z items of every
//    ancestor (their blocks' U columns side by side, in the items' row order),
//    then x over the rows of each partner box.
// ---------------------------------------------------------------------------
struct MRChunk {
    int32_t row_begin;
    int32_t rows;
    int32_t nkb;          // K-blocks of its rows, contiguous and padded once, at the end
    int32_t leaf_base;    // first entry in the host's leaf table
    int32_t nleaf;        // its leaves (the target leaves of its rows)
    int32_t seg_base;     // first U-phase segment
    int32_t nseg;
    int32_t dscale_base;  // nsrc dense scales, one per partner box
    int64_t xoff;         // first B fragment of its Xpack (relative to xpack)
    int32_t step_base;    // first entry of its U-phase step table
    int32_t nsteps;       // K-block steps over all its segments
    int32_t ulo_base;     // FP8 forms: first of its 32 x nzsteps U lo-scales in ulo
    int32_t nzsteps;      // steps over z segments (they come first)
    int32_t nsrc;         // partner boxes of its dense blocks (one x segment each)
    int32_t pad_;
};

struct MRLeaf {           // host side: a chunk's leaf
    int32_t row_begin;    // global first row
    int32_t rows;
};

struct MRVUnit {
    int64_t aoff;         // first A fragment in the V panel
    int32_t c0;           // first chunk
    int32_t nc;           // chunks
    int32_t nm;           // m-subtiles (16 columns each), 1..4
    int32_t lo_off;       // FP8 forms: first of its 64 V lo-scales in vlo
    int64_t poff;         // offset of its partial sums (floats)
};

struct MRZMember {        // one low-rank block (t, s) of a z item
    int32_t ubase;        // unit of column group 0 of (level, s)
    int32_t nu;           // units per column group
    int32_t vcol;         // first column of the block among the columns of (level, s)
    int32_t rank;
    float scale;          // product of the U and V scales
    int32_t col_off;      // FP8 forms: first of its `rank` per-column scales in zcol
    int32_t row;          // first row of its z among the item's rows
    int32_t pad_;
};

struct MRZItem {          // low-rank blocks of one target box: their z stacked, in shared K-blocks
    int32_t m0;           // first member
    int32_t nmem;         // members
    int32_t rows;         // the members' ranks summed (at most 128)
    int32_t pad_;
    int64_t zoff;         // first B fragment of its Zpack
};

struct MRSeg {
    int64_t src;          // first B fragment (Zpack or Xpack)
    int32_t nkb;          // K-blocks
    int32_t kind;         // 0: z of a block, 1: x over a source leaf
    int32_t sidx;         // z item (z) or the partner box's chunk (x): scale row
    int32_t leaf;         // x: index of the partner box among the chunk's (its dense scale)
};

struct MRTile {
    int64_t aoff;         // first A fragment in the UD panel
    int32_t chunk;
    int32_t row0;         // global first row
    int32_t rows;         // valid rows (<= 64)
    int32_t nm;           // m-subtiles
    int32_t pad_[2];
};

struct MRTileGroup {      // up to four consecutive row tiles of one chunk, run by one workgroup
    int32_t chunk;
    int32_t tile0;
    int32_t ntiles;
    int32_t pad_;
};

struct MRUnitGroup {      // up to four consecutive V units over the same chunks, run by one workgroup
    int32_t u0;
    int32_t count;
};

struct MRStep {           // one K-block step of a chunk's target-side contraction
    int64_t bofs;         // byte offset of its B fragments from zpack (xpack follows zpack)
    int32_t srow;         // row of its n-tile scales in the scale array (z rows, then x rows)
    int32_t sleaf;        // source leaf (x steps: selects the dense-block scale), -1 for z steps
    int32_t lseg;         // index of its segment among the chunk's segments
    int32_t pad_;
};

struct DevPlanMR {
    int32_t storage;
    int32_t ntmax;            // n-tiles of 16 columns allocated (max_nrhs / 16, rounded up)
    int32_t num_chunks;
    int32_t num_vunits;
    int32_t num_zitems;
    int32_t num_tiles;
    int32_t max_nzsteps;      // most z steps of a chunk (FP8 forms: U lo-scale table size / 32)
    int32_t max_nseg;         // most target-side segments of a chunk
    int32_t num_tgroups;
    int32_t max_nsteps;       // most target-side steps of a chunk
    int32_t max_chunk_rows;
    int32_t num_ugroups;
    const void *V;            // A fragments
    const void *UD;
    void *xpack;              // B fragments of X (in the same allocation as zpack, after it)
    void *zpack;              // B fragments of z
    float *part;              // unit partial sums
    float *sx;                // per chunk x ntmax n-tile scales of Xpack
    float *sz;                // per block x ntmax n-tile scales of Zpack
    const float *dscale;
    const MRChunk *chunks;
    const MRVUnit *vunits;
    const MRZItem *zitems;
    const MRZMember *zmembers;
    const MRSeg *segs;
    const MRTile *tiles;
    const MRTileGroup *tgroups;
    const MRUnitGroup *ugroups;
    const MRStep *ustep;      // per chunk step (MRChunk::step_base)
    const float *scales;      // n-tile scales: sz rows (one per z item), then sx rows (one per chunk)
    // FP8 forms
    const uint16_t *vlo;      // FP16 lo-scales s'_j of V columns, 64 per unit column group
    const uint16_t *ulo;      // FP16 lo-scales s'_j of U columns, 32 per z step of each chunk
    const float *zcol;        // per z item and column: s_j of U times s_j of V
};

// ---------------------------------------------------------------------------
// Batched persistent launch: many handles applied by one kernel whose
// workgroups take items from a queue. An item is a piece of one member's
// product (up to four waves' worth of one stage, or one workgroup's); the
// queue holds the stages in bands (source side, reduction, target side), so an
// item only ever depends on items earlier in the queue, which keeps the queue
// free of deadlock whatever the number of resident workgroups.
// ---------------------------------------------------------------------------
enum BKind : int32_t {
    BK_SV = 0,   // single vector: vtiles (a wave each)
    BK_SZ1 = 1,  // single vector: stage-1 reduction items (a wave each)
    BK_SZ2 = 2,  // single vector: stage-2 reduction items (a wave each)
    BK_SU = 3,   // single vector: chunks (the whole workgroup each)
    BK_MX = 4,   // multi-RHS: X packing of chunks (a wave each)
    BK_MV = 5,   // multi-RHS: V units (a wave each)
    BK_MZ = 6,   // multi-RHS: z items (a wave each)
    BK_MU = 7    // multi-RHS: row tiles (a wave each)
};

struct BItem {
    int32_t member;
    int32_t kind;         // BKind
    int32_t first;        // first work index of the item's stage
    int32_t count;        // consecutive work indices in the item, >= 1
    int32_t dep;          // counter that must reach `need` before the item starts, -1 for none
    int32_t need;
    int32_t done;         // counter incremented when the item has completed, -1 for none
    int32_t lanes;        // reduction items: lanes per unit (a power of two <= 64)
};

struct BMember {
    DevPlan sp;           // single-vector plan (mr == 0)
    DevPlanMR mp;         // multi-RHS plan (mr == 1)
    int32_t mr;
    int32_t k;            // right-hand sides of this member
};

struct BArgs {            // per member, per call
    const float *x;
    float *y;
    int64_t ldx;
    int64_t ldy;
    float alpha;
    float beta;
};

struct BatchArgs {
    const BMember *members;
    const BArgs *args;
    const BItem *items;
    int32_t *ctl;         // [0] queue head, [1] error flag, [2..] stage counters
    int32_t num_items;
    int32_t num_ctl;
    int32_t spin_limit;   // polls of a dependency wait before it flags an error and goes on
    int32_t zs_rank;      // rows of the per-wave z scratch (multi-RHS members' most z rows of an item)
};

// Kernel launchers (hmat_kernels.hip). Each returns a hipError_t as int.
int launch_vphase(const DevPlan &p, const float *x, void *stream);
int launch_zfinish(const DevPlan &p, void *stream);
int launch_uphase(const DevPlan &p, const float *x, float *y, float alpha, float beta,
                  void *stream);
int launch_probe(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream);
// Device address of the library's static scratch array (HMAT_NOALLOC_SCRATCH_BYTES)
// on `device`, which must be the current device; looked up once per device.
int scratch_address(int device, void **ptr);
int launch_mr(const DevPlanMR &p, int32_t nrhs, float alpha, const float *x, int64_t ldx, float beta,
              float *y, int64_t ldy, void *stream, void (*mark)(void *ctx, int phase), void *ctx);
// hmat_batch.hip: clear the counters, then run the persistent kernel with
// `grid` workgroups and `lds` bytes of dynamic LDS.
int launch_batch(const BatchArgs &a, int32_t storage, bool has_single, bool has_multi, int grid, size_t lds,
                 void *stream);
// The persistent kernel's occupancy (workgroups per CU) for that LDS size.
int batch_max_wg_per_cu(int32_t storage, bool has_single, bool has_multi, size_t lds);

}  // namespace hmat
