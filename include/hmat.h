/*
 * hmat.h -- C ABI of the MI355X (gfx950) H-matrix-vector product library.
 *
 * The library applies an H-matrix (Li, Poulson, Ying, "Distributed-memory
 * H-matrix algebra I", Sec. 2): the matrix is defined by a domain tree
 * (Def. "Domain tree") and by the blocks that Def. 2.3 produces -- dense
 * blocks D between leaves, and low-rank blocks U V^T between admissible
 * non-leaf boxes -- under the weak or the standard admissibility condition
 * (or any other that gives a block set of Def. 2.3's shape). The product is
 * Eq. (2.4), y_t += D_ts x_s and
 * y_t += U_ts (V_ts^T x_s) over all blocks, in the GEMV form
 * y = alpha K x + beta y of the remark that closes Sec. 4.1.
 *
 * Conventions shared by every entry point:
 *  - Rows and columns are in tree order: every tree node owns one contiguous
 *    index range [begin, end). Permuting user vectors into tree order is the
 *    caller's job.
 *  - Matrices passed in are FP32, column-major, with a leading dimension.
 *  - Every call returns an hmat_status; no C++ exception crosses the ABI. On
 *    failure, hmat_last_error() returns a message for the calling thread.
 *  - Validation of arguments, tree and blocks happens before any HIP call.
 */
#ifndef HMAT_H_
#define HMAT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hmat_status {
    HMAT_OK = 0,
    HMAT_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad leading dimension, unknown handle */
    HMAT_ERR_BAD_TREE = 2,    /* the tree is not a domain tree (children do not partition the parent) */
    HMAT_ERR_BAD_BLOCKS = 3,  /* blocks overlap, are missing, or sit on a non-admissible pair */
    HMAT_ERR_UNSUPPORTED = 4, /* valid input outside what the library implements (see hmat_create) */
    HMAT_ERR_NOMEM = 5,       /* a device or host allocation failed */
    HMAT_ERR_DEVICE = 6       /* a HIP call failed (including a fault reported by a later call) */
} hmat_status;

/* How the factors are stored on the device. Quantisation happens on the host
 * inside hmat_create; the device only dequantises (exactly, up to the one
 * FP16 rounding the FP8 forms state). Accumulation is FP32 in every form. */
typedef enum hmat_storage {
    HMAT_STORE_FP32 = 0,          /* D, U, V in FP32 */
    HMAT_STORE_FP16_SCALED = 1,   /* D, U, V in FP16 with power-of-two scales
                                     s = 2^(ceil(log2 amax) - 15), q = RNE(v / s): one per stored
                                     U_ts and V_ts, and one per group of dense blocks D_ts (those
                                     whose target leaves t have one parent and whose source leaves s
                                     have one parent; amax over the group) */
    HMAT_STORE_BF16 = 2,          /* D, U, V in BF16, q = RNE(v), no scales */
    HMAT_STORE_FP8 = 3,           /* U, V in FP8 E4M3 (OCP E4M3FN) as a hi + lo pair per element with
                                     power-of-two scales per factor column j:
                                       s_j = 2^ceil(log2(amax_j / 448)), hi = RNE_e4m3(v / s_j),
                                       r = v / s_j - hi, s'_j = 2^ceil(log2(amax_j(r) / 448)),
                                       lo = RNE_e4m3(r / s'_j)  (all-zero columns: scale 1);
                                     the device multiplies with RNE_f16(hi + s'_j lo) (exact FP16
                                     conversions, one FP16 rounding) and folds s_j into z.
                                     D in BF16: q = RNE_bf16(v / s) with the power of two s of the
                                     FP16 form (the block's group), held as FP16 on the device (exact for
                                     |v / s| >= 2^-14). Multi-RHS handles (max_nrhs > 1) only. */
    HMAT_STORE_FP8_F16D = 4       /* U, V as in HMAT_STORE_FP8; D as in HMAT_STORE_FP16_SCALED */
} hmat_storage;

/* Domain tree (Def. "Domain tree", Sec. 2). Node 0 is the root with
 * parent[0] = -1 and [begin, end) = [0, n). Every other node i has
 * 0 <= parent[i] < i. The children of a node, taken in increasing node id,
 * must tile its range contiguously in that order. All leaves must sit at the
 * same depth. Arrays are host memory, read during the call that takes them
 * (hmat_create, hmat_compress) only. */
typedef struct hmat_tree_desc {
    int64_t n;              /* number of points = rows = columns, 1 <= n < 2^31 */
    int32_t num_nodes;      /* >= 1 */
    int32_t reserved;       /* must be 0 */
    const int32_t *parent;  /* [num_nodes] */
    const int64_t *begin;   /* [num_nodes] */
    const int64_t *end;     /* [num_nodes] */
} hmat_tree_desc;

/* One block of Def. 2.3. rank == 0: dense block, a = D_ts (|t| x |s|,
 * leading dimension lda >= |t|), b unused. rank > 0: low-rank block
 * K_ts = U V^T with a = U (|t| x rank, lda >= |t|) and b = V (|s| x rank,
 * ldb >= |s|). FP32 host memory, column-major, read during hmat_create only
 * (hmat_compress writes these arrays instead). */
typedef struct hmat_block_desc {
    int32_t target;         /* node id t (rows) */
    int32_t source;         /* node id s (columns) */
    int32_t rank;           /* 0 = dense; else 1 <= rank <= min(|t|, |s|) */
    int32_t reserved;       /* must be 0 */
    const float *a;
    int64_t lda;
    const float *b;
    int64_t ldb;
} hmat_block_desc;

/* Option flags (hmat_options.flags).
 *
 * HMAT_FLAG_FP64_ACCUM -- accuracy-check mode for the output accumulation of
 * the GEMV form (remark closing Sec. 4.1): every product of a stored factor
 * with a vector entry, every partial sum of V^T x, every z vector, the sum
 * over levels and the dense near field, and alpha * (...) + beta * y are
 * evaluated in FP64 on the device; y is rounded to FP32 once, at the store.
 * Products of the dequantised factors with FP32 vector entries are exact in
 * FP64, so the result differs from an exact evaluation of Eq. (2.4) over the
 * dequantised factors only by FP64 rounding and that final rounding. The mode
 * always uses the single-vector kernels (one pass per right-hand side, for
 * any max_nrhs) and is meant for checking, not for speed. */
#define HMAT_FLAG_FP64_ACCUM 1

/* HMAT_FLAG_TRANSPOSE -- the handle applies the transpose: y = alpha K^T x +
 * beta y. K^T is the H-matrix whose blocks are the given blocks transposed:
 * block (t, s) becomes (s, t), a low-rank block's U and V trade places and a
 * dense block is transposed (Eq. (2.4) with the roles of target and source
 * exchanged; the transposed block set has Def. 2.3's shape whenever the given
 * one does). Validation and error messages refer to the blocks as given; the
 * storage forms quantise the transposed factors (the same scales, since each
 * is per block or per factor column). Combines with every other option. */
#define HMAT_FLAG_TRANSPOSE 2

typedef struct hmat_options {
    int32_t storage;        /* hmat_storage */
    int32_t max_nrhs;       /* largest nrhs hmat_matvec will be called with, >= 1 */
    int32_t device;         /* HIP device ordinal the data lives on */
    int32_t flags;          /* HMAT_FLAG_FP64_ACCUM | HMAT_FLAG_TRANSPOSE; other bits give INVALID_ARG */
} hmat_options;

typedef struct hmat_info {
    int64_t n;
    int32_t leaf_depth;          /* L: depth of every leaf (root = 0) */
    int32_t num_chunks;          /* boxes at depth max(L-1, 0): the unit of device work */
    int64_t num_dense_blocks;
    int64_t num_lowrank_blocks;
    int64_t stored_elements;     /* sum |t||s| over dense + (|t|+|s|) r over low-rank blocks */
    int64_t factor_bytes;        /* bytes of those elements in the storage form, plus scales */
    int64_t device_factor_bytes; /* bytes the kernels stream, including layout padding */
    int64_t workspace_bytes;     /* partial sums and z vectors */
    int32_t storage;
    int32_t max_nrhs;
    int32_t flags;               /* the flags the handle was created with */
    int32_t reserved;
} hmat_info;

typedef struct hmat_handle *hmat_t;

/* Build a device-resident H-matrix from a domain tree and its blocks.
 *
 * The block set must have the shape of Def. 2.3 for the tree: starting from
 * the recursion pair (root, root), every ordered pair (t, s) of a child t of
 * p and a child s of q, for a recursion pair (p, q), is either a block or
 * itself a recursion pair; pairs of leaves are dense blocks, blocks between
 * non-leaf boxes are low-rank (t != s); every block is such a child pair.
 * Under weak admissibility the recursion pairs are the (c, c) pairs; under
 * standard admissibility (Eq. (2.2)) they are the pairs of neighbouring
 * boxes. A root that is itself a leaf takes one dense block (0, 0). Blocks
 * may come in any order. The library does not evaluate an admissibility
 * condition itself.
 *
 * Errors: INVALID_ARG (null pointers, sizes, leading dimensions, ranks,
 * options); BAD_TREE; BAD_BLOCKS (a block on a recursion pair (c, c) above
 * the leaves, a duplicate, a missing pair, or a block that is no child pair
 * of a recursion pair); UNSUPPORTED (leaves at mixed depths, a dense block
 * between non-leaves, a low-rank block between leaves, a chunk whose vector
 * operand exceeds the kernel's LDS budget -- 16384 FP32 values, or 8192 FP64
 * values under HMAT_FLAG_FP64_ACCUM); NOMEM; DEVICE.
 *
 * Ownership: all inputs are deep-copied and re-laid-out; the handle owns its
 * device memory until hmat_destroy. On failure *out is set to NULL and
 * nothing is leaked. The environment variable HMAT_FAULT=alloc makes the
 * first device allocation fail (NOMEM), for testing the cleanup path. */
hmat_status hmat_create(const hmat_tree_desc *tree, const hmat_block_desc *blocks,
                        int64_t num_blocks, const hmat_options *opts, hmat_t *out);

/* y = alpha * K x + beta * y for nrhs right-hand sides.
 *
 * x (n x nrhs, leading dimension ldx >= n) and y (n x nrhs, ldy >= n) are
 * FP32 device pointers on the handle's device, in tree order, owned by the
 * caller; they must not overlap. When beta == 0, y is not read (NaN in y is
 * overwritten). 1 <= nrhs <= max_nrhs. The call is asynchronous on `stream`
 * (a hipStream_t; NULL = the null stream) and does no host synchronisation.
 * One handle owns one workspace, so calls on the same handle must be ordered
 * on one stream; distinct handles are independent. The result is
 * deterministic: the same inputs give bitwise identical y.
 *
 * Errors: INVALID_ARG; DEVICE (launch failure). */
hmat_status hmat_matvec(hmat_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx,
                        float beta, float *y, int64_t ldy, void *stream);

/* For callers that cannot allocate device memory at call time: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * hmat_matvec_noalloc computes exactly what hmat_matvec computes, with the same
 * kernels in the same order (bitwise the same y), but its workspace -- the
 * partial sums of V^T x, the stage-1 slice sums and the z vectors -- lives in
 * a static array of HMAT_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends, not in the handle's workspace. The
 * call allocates nothing (no hipMalloc, no event, no host-side device-memory
 * routine); its first call on a device looks the array's address up once.
 *
 * Limits: single-vector handles only (created with max_nrhs == 1, or with
 * HMAT_FLAG_FP64_ACCUM); the handle's workspace_bytes (hmat_get_info), with
 * each of its two parts rounded up to 256 bytes, must fit in
 * HMAT_NOALLOC_SCRATCH_BYTES (the 2D N = 2^20, rank-32 matrix takes about
 * 11.5 MB, twice that under HMAT_FLAG_FP64_ACCUM). Phase timing is not
 * recorded.
 *
 * Concurrency: every call on a device shares that device's one array, and the
 * array keeps the last call's contents (each call writes every workspace
 * value before reading it). Calls that overlap in time on one device race,
 * whatever their handles and streams: order them on one stream, or join the
 * streams, as for calls on one handle.
 *
 * Arguments, ownership and the other errors as for hmat_matvec; UNSUPPORTED
 * for a multi-RHS handle or a workspace beyond the scratch size; DEVICE when
 * the scratch address cannot be obtained or a launch fails. */
#define HMAT_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
hmat_status hmat_matvec_noalloc(hmat_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx,
                                float beta, float *y, int64_t ldy, void *stream);

/* Release the handle and its device memory. NULL is a no-op; an unknown or
 * already destroyed handle gives INVALID_ARG. Work queued on a stream that
 * still uses the handle must have completed. */
hmat_status hmat_destroy(hmat_t h);

/* Sizes and counts of a handle (host only, no device call). */
hmat_status hmat_get_info(hmat_t h, hmat_info *info);

/* Per-phase timing for measurement. While enabled, hmat_matvec records HIP
 * events around each kernel on the caller's stream; hmat_get_timing waits
 * for them and returns, per phase, the summed elapsed milliseconds and the
 * number of calls since timing was enabled. Phases: 0 = V-phase (V^T x
 * partial sums), 1 = partial reduction and z routing, 2 = U-phase plus dense
 * near field and output. Enabling resets the sums. */
#define HMAT_NUM_PHASES 3
hmat_status hmat_set_timing(hmat_t h, int32_t enable);
hmat_status hmat_get_timing(hmat_t h, double ms[HMAT_NUM_PHASES], int64_t *calls);

/* HBM bandwidth probe: mode 0 reads `bytes` from src (a multiple of 16 B) and
 * writes one float per workgroup to dst (dst must hold 65536 floats);
 * mode 1 copies `bytes` from src to dst. Device pointers, asynchronous on
 * `stream`. Used to measure the achievable read bandwidth and to calibrate
 * hardware byte counters against a copy of known size. */
hmat_status hmat_probe_bandwidth(const void *src, void *dst, int64_t bytes, int32_t mode,
                                 void *stream);

/* ------------------------------------------------------------------------
 * Batched product: many independent H-matrices (each built by hmat_create)
 * applied by one persistent kernel launch, replayed as a HIP graph.
 *
 * Each member's product is split into items (pieces of the source-side
 * products, of the partial reduction and of the target-side products, Sec.
 * 4.1, Steps 1-5) held in one queue in stage order; the kernel's workgroups
 * take items from the queue, and an item waits on its own member's earlier
 * stage through a completion counter. An item's work is estimated by its
 * byte count (under weak admissibility every box of a level carries the same
 * number of blocks, Sec. 3.2), which the queue is sorted by.
 * ------------------------------------------------------------------------ */
typedef struct hmat_batch_handle *hmat_batch_t;

typedef struct hmat_batch_options {
    int32_t use_graph;      /* 1: each call replays a HIP graph of (counter clear, persistent kernel);
                               0: the two kernels are launched directly on the caller's stream */
    int32_t wg_per_cu;      /* persistent workgroups per compute unit; 0 = as many as fit */
    int32_t order;          /* queue order inside each stage band: 0 = largest item first,
                               1 = member by member (largest member first) */
    int32_t spin_limit;     /* polls before a dependency wait gives up and flags an error; 0 = 2^20 */
    int32_t grain_kb;       /* an item groups consecutive work of one stage up to this many KiB of
                               factor and operand traffic; 0 = 512 */
} hmat_batch_options;

typedef struct hmat_batch_info {
    int32_t count;          /* members */
    int32_t num_items;      /* queue length */
    int32_t grid;           /* persistent workgroups launched */
    int32_t wg_per_cu;
    int32_t max_wg_per_cu;  /* most that can be resident */
    int32_t order;
    int32_t use_graph;
    int32_t grain_kb;
    int64_t lds_bytes;      /* dynamic LDS per workgroup */
    int64_t item_bytes;     /* factor bytes the items stream per call, layout padding included */
} hmat_batch_info;

/* Build a batch over `count` live handles. nrhs[i] is the number of
 * right-hand sides member i is applied to: 1 for a handle created with
 * max_nrhs == 1 (single-vector kernels); 1 <= nrhs[i] <= min(16, max_nrhs) for
 * one created with max_nrhs > 1 (MFMA kernels, one tile of 16 columns).
 * Members must be distinct, live on one device, share one storage form and
 * not use HMAT_FLAG_FP64_ACCUM (HMAT_FLAG_TRANSPOSE members are fine). A batch uses its members' device workspaces: while it exists
 * the members cannot be destroyed (hmat_destroy gives INVALID_ARG), and a
 * member must not run hmat_matvec concurrently with the batch. opts may be
 * NULL (defaults: graph on, as many workgroups as fit, largest item first).
 *
 * Errors: INVALID_ARG; UNSUPPORTED (a member in an FP8 form, or a multi-RHS
 * member whose chunks have more than 64 target-side segments); NOMEM; DEVICE. */
hmat_status hmat_batch_create(const hmat_t *members, int32_t count, const int32_t *nrhs,
                              const hmat_batch_options *opts, hmat_batch_t *out);

/* y_i = alpha K_i x_i + beta y_i for every member i. x[i] and y[i] are device
 * pointers (n_i x nrhs[i], column-major, leading dimensions ldx[i], ldy[i] >=
 * n_i); the pointer and leading-dimension arrays are host arrays read during
 * the call. No x[i] may overlap any y[j], and the y[i] must not overlap each
 * other. Asynchronous on `stream`; when the pointers differ from the last
 * call's, they are copied to the device on `stream` first. One batch owns one
 * set of counters: calls on the same batch must be ordered on one stream.
 * Errors: INVALID_ARG; DEVICE (launch failure). */
hmat_status hmat_batch_matvec(hmat_batch_t b, float alpha, const float *const *x, const int64_t *ldx, float beta,
                              float *const *y, const int64_t *ldy, void *stream);

/* Wait for `stream` and report the last batched product's status: DEVICE
 * when one of its dependency waits hit the poll limit (its y is then not
 * valid). */
hmat_status hmat_batch_sync(hmat_batch_t b, void *stream);

/* Change the launch options (rebuilds the queue and the graph). */
hmat_status hmat_batch_set_options(hmat_batch_t b, const hmat_batch_options *opts);
hmat_status hmat_batch_get_info(hmat_batch_t b, hmat_batch_info *info);

/* Autotuner: time every candidate (wg_per_cu in {1, 2, 4, 8} up to the
 * resident maximum, order in {0, 1}, grain_kb in {128, 512, 2048}) on the
 * given operands, `reps` timed
 * calls each after two untimed ones, and keep the fastest. With a non-NULL
 * cache_path, a JSON file of earlier results keyed by a hash of the device and
 * the members' shapes is read first (a hit skips the timing) and updated
 * after. The chosen options are applied to the batch and, when `chosen` is
 * not NULL, returned there. The calls overwrite y. Synchronises `stream`.
 * Errors: INVALID_ARG; DEVICE; NOMEM. */
hmat_status hmat_batch_autotune(hmat_batch_t b, float alpha, const float *const *x, const int64_t *ldx,
                                float beta, float *const *y, const int64_t *ldy, void *stream,
                                const char *cache_path, int32_t reps, hmat_batch_options *chosen);

/* Release the batch (not its members). NULL is a no-op. Work queued on a
 * stream that still uses the batch must have completed. */
hmat_status hmat_batch_destroy(hmat_batch_t b);

/* ------------------------------------------------------------------------
 * Construction of the block factors on the GPU.
 *
 * The paper takes the blocks of Def. 2.3 as given and leaves how they are
 * computed to the literature (end of Sec. 2). hmat_compress fills a block
 * structure from the points and a kernel function of Eq. (2.1) (without
 * quadrature weights), so that the result can be passed to hmat_create:
 *   dense blocks: the entries K(p_i, p_j), and `diag` where the global
 *     indices coincide;
 *   low-rank blocks: a randomized SVD (Halko, Martinsson and Tropp, SIAM
 *     Review 53, 2011, Algorithms 4.1 and 5.1) of the block, whose entries
 *     are generated on the fly and never stored: Y = K Omega with
 *     l = min(r + oversample, |t|, |s|) columns, Q an orthonormal basis of Y,
 *     B = Q^T K, and the rank-r truncation of the SVD of B, the singular
 *     values split evenly: U = Q W S^(1/2), V = B^T W S^(-1/2) for the leading
 *     r left singular vectors W of B. Omega is Rademacher: entry (j, c) is +1
 *     when bit (c mod 64) of word (c div 64) of Philox4x64-10 (Salmon et al.,
 *     SC 2011) at counter (j, 0, 0, 0), key (seed, 0) is clear and -1 when it
 *     is set, j the global index of the source point.
 * Entries are FP32 (the sample products take them as exact three-part BF16
 * splits on the matrix cores, with FP32 accumulation); the small Gram matrices
 * and their eigen-decompositions (which give Q and W) are FP64.
 * ------------------------------------------------------------------------ */
#define HMAT_KERNEL_LOG 0  /* -log|x - y| / (2 pi) */
#define HMAT_KERNEL_INV 1  /* 1 / (4 pi |x - y|) */

typedef struct hmat_compress_options {
    int32_t kernel;      /* HMAT_KERNEL_LOG or HMAT_KERNEL_INV */
    int32_t dim;         /* coordinates per point, 1 <= dim <= 3 */
    float diag;          /* K(p_i, p_i) */
    int32_t oversample;  /* p, 0 <= p <= 96; every low-rank block needs l <= 96 */
    uint64_t seed;       /* Philox key word 0 */
    int32_t device;      /* HIP device ordinal to compute on */
    int32_t reserved;    /* must be 0 */
} hmat_compress_options;

/* Fill the factors of every block of a Def. 2.3 block structure.
 *
 * tree and blocks as for hmat_create, except that the factor pointers are
 * the destinations: a dense block's a receives the |t| x |s| entries
 * (column-major, lda); a low-rank block's a receives U (|t| x rank, lda) and
 * b receives V (|s| x rank, ldb). They are FP32 host arrays owned by the
 * caller, which the call writes (a const_cast of the descriptor's pointers).
 * points: n x dim FP32 host array, row-major, in tree order.
 * The call is synchronous; device memory it takes is released before it
 * returns.
 *
 * Errors: INVALID_ARG (null pointers, sizes, options), BAD_TREE, BAD_BLOCKS
 * and UNSUPPORTED as for hmat_create, UNSUPPORTED also for a low-rank block
 * whose l exceeds 96; NOMEM; DEVICE. Nothing is written on a validation
 * error. */
hmat_status hmat_compress(const hmat_tree_desc *tree, const float *points, const hmat_block_desc *blocks,
                          int64_t num_blocks, const hmat_compress_options *opts);

/* Message for the last failed call on this thread ("" if none). */
const char *hmat_last_error(void);

/* Name of a status code. */
const char *hmat_status_string(hmat_status s);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H_ */
