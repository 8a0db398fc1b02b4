/*
 * hmat_h2.h -- C ABI of the H^2-matrix-vector product (MI355X, gfx950).
 *
 * The H^2-matrix is the nested-basis format that Li, Poulson and Ying
 * introduce beside the H-matrix (Sec. 1) and to which their data
 * distribution extends (remark in Sec. 3.2: the nested bases are distributed
 * like the low-rank factors, the small middle matrix of each low-rank block
 * is held once). It keeps the block structure of Def. 2.3 -- dense blocks
 * between leaves, low-rank blocks between admissible non-leaf boxes -- but
 * writes every low-rank block as
 *
 *     K_ts = U_t S_ts V_s^T,
 *
 * with one row basis U_t and one column basis V_s per box (k_t columns),
 * shared by all blocks of the box, and a coupling matrix S_ts (k_t x k_s) per
 * block. The bases are nested: only leaves store U_t and V_t explicitly; for
 * a box t with children c_1, c_2, ... (in tree order)
 *
 *     U_t = [U_c1 E_c1; U_c2 E_c2; ...],   V_t = [V_c1 F_c1; V_c2 F_c2; ...]
 *
 * with transfer matrices E_c, F_c of size k_c x k_t. Storage and the product
 * are linear in N. The product is Eq. (2.4) over these blocks, in the GEMV
 * form y = alpha K x + beta y of the remark that closes Sec. 4.1; the library
 * evaluates it as an upward pass (x^_t = V_t^T x_t for leaves, then
 * x^_t = sum_c F_c^T x^_c), the couplings with a downward pass
 * (y^_t = E_t y^_parent + sum_s S_ts x^_s), and at the leaves
 * y_t = U_t y^_t + sum_s D_ts x_s.
 *
 * Conventions, status codes, the tree descriptor and the option storage enum
 * are those of hmat.h.
 */
#ifndef HMAT_H2_H_
#define HMAT_H2_H_

#include "hmat.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HMAT_H2_MAX_RANK 64

/* The basis of one node (an array of these, indexed by node id, is passed to
 * hmat_h2_create). When the tree's leaves are at depth >= 2, every non-root
 * node has a basis, 1 <= rank <= HMAT_H2_MAX_RANK; the root has rank 0. When
 * the leaves are at depth 0 or 1 there are no low-rank blocks and every rank
 * is 0 (the pointers are then ignored). FP32 host memory, column-major, read
 * during hmat_h2_create only. */
typedef struct hmat_h2_basis {
    int32_t rank;        /* k_t */
    int32_t reserved;    /* must be 0 */
    const float *u;      /* leaves: U_t, |t| x k_t, ldu >= |t|; ignored for other nodes */
    int64_t ldu;
    const float *v;      /* leaves: V_t, |t| x k_t, ldv >= |t| */
    int64_t ldv;
    const float *e;      /* nodes whose parent has a basis: E_t, k_t x k_parent, lde >= k_t */
    int64_t lde;
    const float *f;      /* likewise F_t, k_t x k_parent, ldf >= k_t */
    int64_t ldf;
} hmat_h2_basis;

/* One block of Def. 2.3. kind 0: dense, a = D_ts (|t| x |s|, lda >= |t|);
 * kind 1: low-rank, a = S_ts (k_t x k_s, lda >= k_t). */
typedef struct hmat_h2_block {
    int32_t target;
    int32_t source;
    int32_t kind;
    int32_t reserved;    /* must be 0 */
    const float *a;
    int64_t lda;
} hmat_h2_block;

typedef struct hmat_h2_options {
    int32_t storage;     /* HMAT_STORE_FP32, or HMAT_STORE_FP16_SCALED (dense blocks, leaf bases,
                            transfers and couplings in FP16 with one power-of-two scale per stored
                            array, the rule of hmat.h) */
    int32_t device;      /* HIP device ordinal */
    int32_t flags;       /* must be 0 */
    int32_t reserved;    /* must be 0 */
} hmat_h2_options;

typedef struct hmat_h2_info {
    int64_t n;
    int32_t leaf_depth;
    int32_t num_chunks;           /* boxes at depth max(L-1, 0): one workgroup of the leaf kernels each */
    int64_t num_dense_blocks;
    int64_t num_coupling_blocks;
    int64_t stored_elements;      /* leaf bases + transfers + couplings + dense entries */
    int64_t factor_bytes;         /* those elements in the storage form, plus scales */
    int64_t device_factor_bytes;  /* bytes the kernels stream, layout padding included */
    int64_t workspace_bytes;      /* x^ and y^ of every node */
    int64_t leaf_kernel_bytes;    /* algorithmic bytes of the leaf kernel per right-hand side: leaf U
                                     bases, leaf and chunk E transfers, chunk couplings, dense blocks,
                                     x read once (dense sources), y written once */
    int32_t storage;
    int32_t max_rank;
} hmat_h2_info;

typedef struct hmat_h2_handle *hmat_h2_t;

/* Build a device-resident H^2-matrix. The block set must have the shape of
 * Def. 2.3 for the tree, as for hmat_create (kind 1 in place of rank > 0).
 * Errors: INVALID_ARG (null pointers, leading dimensions, ranks, options);
 * BAD_TREE; BAD_BLOCKS; UNSUPPORTED (leaves at mixed depths, a rank above
 * HMAT_H2_MAX_RANK, a leaf of more than 64 rows in a chunk, a chunk whose
 * leaf-kernel operands exceed the LDS budget); NOMEM; DEVICE. Ownership as for
 * hmat_create; HMAT_FAULT=alloc applies. */
hmat_status hmat_h2_create(const hmat_tree_desc *tree, const hmat_h2_basis *bases, const hmat_h2_block *blocks,
                           int64_t num_blocks, const hmat_h2_options *opts, hmat_h2_t *out);

/* y = alpha K x + beta y for nrhs right-hand sides, one pass each; arguments,
 * asynchrony and determinism as for hmat_matvec. One handle owns one
 * workspace: calls on the same handle must be ordered on one stream. */
hmat_status hmat_h2_matvec(hmat_h2_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx, float beta,
                           float *y, int64_t ldy, void *stream);

/* NULL is a no-op; an unknown handle gives INVALID_ARG. */
hmat_status hmat_h2_destroy(hmat_h2_t h);

hmat_status hmat_h2_get_info(hmat_h2_t h, hmat_h2_info *info);

/* Per-phase timing on the caller's stream, as hmat_set_timing /
 * hmat_get_timing: phase 0 = upward pass (leaf x^ and the levels above),
 * phase 1 = couplings and downward pass above the chunks, phase 2 = the
 * leaf kernel (chunk couplings, leaf y^, U_t y^_t, dense near field, y). */
hmat_status hmat_h2_set_timing(hmat_h2_t h, int32_t enable);
hmat_status hmat_h2_get_timing(hmat_h2_t h, double ms[HMAT_NUM_PHASES], int64_t *calls);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H2_H_ */
