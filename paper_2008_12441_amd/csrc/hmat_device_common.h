// Device-side vector types and small helpers shared by the HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include "hmat.h"
#include "hmat_internal.h"

namespace hmat {
namespace dev {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Workgroups are dealt to the 8 XCDs in turn (block i runs on XCD i % 8), and
// each XCD has its own L2.
constexpr int kXcds = 8;

// Read of data that no kernel writes while it runs (layout tables, plans, the
// input vector), through the constant address space: uniform reads become
// scalar loads whatever stores the kernel makes elsewhere.
template <class T>
__device__ inline T cload(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "read as 32-bit words");
    struct Words {
        uint32_t w[sizeof(T) / 4];
    } v;
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) v.w[i] = q[i];
    return __builtin_bit_cast(T, v);
}
template <class T>
__device__ inline T cload(const T *p, int64_t i) {
    return cload(p + i);
}

// A pointer stored in memory that no kernel writes while it runs, read as a
// pointer through the constant address space: the compiler then takes it to
// point to global memory and uses global instead of flat instructions for
// the accesses through it.
template <class T>
__device__ inline T *cptr(T *const *field) {
    return *(T *const __attribute__((address_space(4))) *)field;
}

}  // namespace dev
}  // namespace hmat
