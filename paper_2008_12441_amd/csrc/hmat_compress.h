// Construction of the block factors (hmat_compress.hip; host side in
// hmat_host.cpp): the block tables of one launch set and the launchers.
// Offsets are in elements of the workspace arrays.
#pragma once

#include <cstddef>
#include <cstdint>

namespace hmat {

constexpr int kCompressMaxL = 96;  // sample columns l of a low-rank block

struct CKernel {
    const float *pts;  // n x dim, row-major
    int32_t dim;
    int32_t kind;      // HMAT_KERNEL_*
    float diag;
    int32_t pad_;
};

struct CDense {        // one dense block: |t| x |s| entries, column-major at out + off
    int64_t t0, s0;
    int32_t mt, ms;
    int64_t off;
};

struct CLowRank {      // one low-rank block
    int64_t t0, s0;    // first global row of t and of s
    int32_t mt, ms;
    int32_t ell, rank;
    int64_t yoff;      // Y, then Q: mt x ell column-major (floats)
    int64_t boff;      // B^T: ms x ell column-major (floats)
    int64_t goff;      // Gram matrix: ell x ell (doubles)
    int64_t toff;      // transform: ell x ell (orthonormalisation) or M_U, M_V: ell x rank each (floats)
    int64_t uoff, voff;  // U: mt x rank, V: ms x rank, column-major (floats)
};

struct CTile {         // 256 consecutive rows of one block (dense: entries)
    int32_t block;
    int32_t pad_;
    int64_t first;
};

struct CWork {
    const CLowRank *blocks;
    float *fws;        // float workspace (Y/Q, B^T, transforms, U, V)
    double *gram;
    uint64_t seed;
    int32_t lc;        // l rounded up to 16 over the blocks of this launch set
    int32_t max_ell;
};

// Phases of one set of low-rank blocks; each returns a hipError_t as int.
int launch_compress_dense(const CKernel &k, const CDense *blocks, const CTile *tiles, int64_t ntiles, float *out,
                          void *stream);
// mode 0: Y = K_ts Omega over the row tiles of t; mode 1: B^T = K_st Q over the row tiles of s
int launch_compress_sample(const CKernel &k, const CWork &w, const CTile *tiles, int64_t ntiles, int mode,
                           void *stream);
// Gram matrix (FP64) of Y (which 0) or of B^T (which 1), one workgroup per block
int launch_compress_gram(const CWork &w, int64_t nblocks, int which, void *stream);
// Jacobi eigen-decomposition of each Gram matrix; mode 0 writes the
// orthonormalising transform, mode 1 the factor maps M_U, M_V
int launch_compress_eig(const CWork &w, int64_t nblocks, int mode, void *stream);
// apply: 0 = Y <- Y T (row tiles of t), 1 = U = Q M_U (row tiles of t), 2 = V = B^T M_V (row tiles of s)
int launch_compress_apply(const CWork &w, const CTile *tiles, int64_t ntiles, int what, void *stream);

}  // namespace hmat
