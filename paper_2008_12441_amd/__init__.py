"""MI355X (gfx950) H-matrix-vector product (weak and standard admissibility), and the H^2 variant.

The product y = alpha K x + beta y of an H-matrix (Def. 2.3, Eq. (2.4)) runs
in hand-written HIP kernels behind the C ABI of ``include/hmat.h``, and so
does the construction of the block factors from points and a kernel function
(``hmat_compress``: dense entries, randomized SVD of the low-rank blocks); this
package is the thin Python binding of that library (``binding``) and its
build step (``_build``).
"""
from .binding import (BLOCK_DTYPE, EXPORTED, HMAT_NOALLOC_SCRATCH_BYTES, HMAT_FLAG_FP64_ACCUM, HMAT_KERNEL_INV, HMAT_KERNEL_LOG, KERNEL,
                      compress_pool, hmat_compress, HMAT_FLAG_TRANSPOSE, HMAT_STORE_BF16, HMAT_STORE_FP16_SCALED,
                      HMAT_STORE_FP32, LIB_PATH, STORAGE, HBatch, HMatrix, HmatError, hmat_batch_autotune,
                      hmat_batch_create, hmat_batch_destroy, hmat_batch_get_info, hmat_batch_matvec,
                      hmat_batch_set_options, hmat_batch_sync, hmat_create, hmat_destroy, hmat_get_info,
                      hmat_get_timing, hmat_last_error, hmat_matvec, hmat_matvec_noalloc, hmat_probe_bandwidth, hmat_set_timing,
                      hmat_status_string, load_library, make_block_array, make_descriptors, make_tree_desc)

from .binding_h2 import (HMAT_H2_MAX_RANK, H2Matrix, hmat_h2_create, hmat_h2_destroy, hmat_h2_get_info,
                         hmat_h2_get_timing, hmat_h2_matvec, hmat_h2_set_timing, make_h2_descriptors)

__all__ = [
    "HMAT_H2_MAX_RANK", "H2Matrix", "hmat_h2_create", "hmat_h2_destroy", "hmat_h2_get_info", "hmat_h2_get_timing",
    "hmat_h2_matvec", "hmat_h2_set_timing", "make_h2_descriptors",
    "BLOCK_DTYPE", "EXPORTED", "HMAT_NOALLOC_SCRATCH_BYTES", "HMAT_FLAG_FP64_ACCUM", "HMAT_KERNEL_INV", "HMAT_KERNEL_LOG", "KERNEL",
    "compress_pool", "hmat_compress", "HMAT_FLAG_TRANSPOSE", "HMAT_STORE_BF16", "HMAT_STORE_FP16_SCALED",
    "HMAT_STORE_FP32", "LIB_PATH", "STORAGE", "HBatch", "HMatrix", "HmatError", "hmat_batch_autotune",
    "hmat_batch_create", "hmat_batch_destroy", "hmat_batch_get_info", "hmat_batch_matvec",
    "hmat_batch_set_options", "hmat_batch_sync", "hmat_create", "hmat_destroy", "hmat_get_info",
    "hmat_get_timing", "hmat_last_error", "hmat_matvec", "hmat_matvec_noalloc", "hmat_probe_bandwidth", "hmat_set_timing",
    "hmat_status_string", "load_library", "make_block_array", "make_descriptors", "make_tree_desc",
]
