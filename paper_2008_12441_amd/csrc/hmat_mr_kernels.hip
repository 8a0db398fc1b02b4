// HIP kernels (gfx950) of the multi-RHS H-matrix-vector product on MFMA.
//
// Per group of at most 128 right-hand sides four launches run on the caller's
// stream (bodies in hmat_mr_device.h): X packing (one workgroup per chunk and
// n-tile: k_xpack_tile, or k_xpack for chunks of more than 512 rows), the
// source side (k_vmfma_group: one workgroup per group of four V units over the
// same chunks), z packing (k_zmfma: one wave per z item and n-tile)
// and the target side (k_umfma_group: one workgroup per group of four row
// tiles of a chunk; k_umfma, one wave per row tile, where a chunk's segments
// or LDS needs exceed what the group kernel holds).
#include "hmat_mr_device.h"

namespace hmat {
namespace {

using namespace hmat::dev;

__device__ inline int wave_id(int waves_per_block) {
    return __builtin_amdgcn_readfirstlane((int)blockIdx.x * waves_per_block + (int)(threadIdx.x >> 6));
}

// Renumbering the blocks so that every XCD works through one contiguous range
// of tiles keeps the B fragments that neighbouring tiles share (a chunk's X,
// its ancestors' z) in one L2.
__device__ inline int wave_id_xcd(int waves_per_block) {
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % kXcds, j = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int logical = x * per + (x < rem ? x : rem) + j;
    return __builtin_amdgcn_readfirstlane(logical * waves_per_block + (int)(threadIdx.x >> 6));
}

template <int STORE>
__global__ __launch_bounds__(256) void k_xpack(DevPlanMR p, const float *__restrict__ x, int64_t ldx, int k) {
    __shared__ float red[4];
    const int nt_used = (k + 15) / 16;
    mr_xpack<STORE>(p, blockIdx.x / nt_used, blockIdx.x % nt_used, x, ldx, k, red);
}

// chunks of at most kXpackMaxRows rows: X read coalesced through an LDS tile
template <int STORE>
__global__ __launch_bounds__(256) void k_xpack_tile(DevPlanMR p, const float *__restrict__ x, int64_t ldx, int k) {
    extern __shared__ __align__(16) float xtile[];  // 16 x (max chunk rows + 1), then 4 maxima
    const int nt_used = (k + 15) / 16;
    mr_xpack_tile<STORE>(p, blockIdx.x / nt_used, blockIdx.x % nt_used, x, ldx, k, xtile,
                         xtile + 16 * (p.max_chunk_rows + 1));
}

// waves per SIMD the group kernels are compiled for: three up to four n-tiles,
// two above (their registers fit without spilling with the prefetch depths of
// GroupDepth)
template <int STORE, int NT>
struct GroupOcc {
    static constexpr int waves = NT <= 4 ? 3 : 2;
};

// one workgroup per unit group, X fragments shared through LDS (mr_vunit_group)
template <int STORE, int NT>
__global__ __launch_bounds__(256, (GroupOcc<STORE, NT>::waves)) void k_vmfma_group(DevPlanMR p) {
    extern __shared__ __align__(16) unsigned char vring[];  // two B slots
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % kXcds, j = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    mr_vunit_group<STORE, NT>(p, x * per + (x < rem ? x : rem) + j, vring);
}

template <int STORE>
__global__ __launch_bounds__(256) void k_zmfma(DevPlanMR p, int nt_used) {
    __shared__ float zs[4][kMaxRankMR][16];
    const int w = wave_id(4);
    if (w >= p.num_zitems * nt_used) return;
    const MRZItem z = cload(p.zitems, w / nt_used);
    const MRZMember zm0 = cload(p.zmembers, z.m0);
    mr_zitem<STORE>(p, w / nt_used, z, zm0, w % nt_used, threadIdx.x & 63, zs[threadIdx.x >> 6]);
}

// LS: the chunks have at most 64 target-side segments, so a tile's step table
// and scales are held one per lane (see mfma_steps); otherwise they are read
// through the scalar cache.
template <int STORE, int NT, bool LS>
__global__ __launch_bounds__(256, Occupancy<NT>::waves) void k_umfma(DevPlanMR p, int k, float alpha, float beta,
                                                                     float *__restrict__ y, int64_t ldy) {
    extern __shared__ __align__(16) uint32_t lo_tables[];  // FP8 forms: 16 x max_nzsteps words per wave
    const int w = wave_id_xcd(4);
    if (w >= p.num_tiles) return;
    mr_tile<STORE, NT, LS>(p, w, threadIdx.x & 63, k, alpha, beta, y, ldy,
                           lo_tables + (threadIdx.x >> 6) * 16 * p.max_nzsteps);
}

// One workgroup per tile group, B shared through LDS (mr_tile_group);
// XCD-aware numbering keeps neighbouring chunks (which share their
// ancestors' z) in one L2.

template <int STORE, int NT>
__global__ __launch_bounds__(256, (GroupOcc<STORE, NT>::waves)) void k_umfma_group(DevPlanMR p, int k, float alpha, float beta,
                                                        float *__restrict__ y, int64_t ldy) {
    // two B slots, the step table (max_nsteps entries), then (FP8 forms) the lo-scale tables
    extern __shared__ __align__(16) unsigned char smem[];
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % kXcds, j = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int g = x * per + (x < rem ? x : rem) + j;
    constexpr int kRing = 2 * NT * MR<STORE>::BFRAG * 16;
    int2 *stab = reinterpret_cast<int2 *>(smem + kRing);
    mr_tile_group<STORE, NT>(p, g, k, alpha, beta, y, ldy, smem, stab,
                             reinterpret_cast<uint32_t *>(stab + p.max_nsteps) + (threadIdx.x >> 6) * 16 * p.max_nzsteps);
}

template <int STORE, int NT>
int launch_mr_nt(const DevPlanMR &p, int32_t k, float alpha, const float *x, int64_t ldx, float beta, float *y,
                 int64_t ldy, hipStream_t st, void (*mark)(void *, int), void *ctx) {
    if (mark) mark(ctx, 0);
    if (p.max_chunk_rows <= kXpackMaxRows)
        hipLaunchKernelGGL(k_xpack_tile<STORE>, dim3(p.num_chunks * NT), dim3(256),
                           (size_t)(16 * (p.max_chunk_rows + 1) + 4) * 4, st, p, x, ldx, k);
    else
        hipLaunchKernelGGL(k_xpack<STORE>, dim3(p.num_chunks * NT), dim3(256), 0, st, p, x, ldx, k);
    int e = (int)hipGetLastError();
    if (e) return e;
    if (p.num_vunits > 0) {
        hipLaunchKernelGGL((k_vmfma_group<STORE, NT>), dim3(p.num_ugroups), dim3(256),
                           (size_t)2 * NT * MR<STORE>::BFRAG * 16, st, p);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (mark) mark(ctx, 1);
    if (p.num_zitems > 0) {
        hipLaunchKernelGGL(k_zmfma<STORE>, dim3((p.num_zitems * NT + 3) / 4), dim3(256), 0, st, p, NT);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (mark) mark(ctx, 2);
    const size_t lds = IsFp8<STORE>::value ? (size_t)4 * 64 * p.max_nzsteps : 0;
    const size_t glds = (size_t)2 * NT * MR<STORE>::BFRAG * 16 + (size_t)8 * p.max_nsteps + lds;
    if (p.max_nseg <= 64 && glds <= 65536)
        hipLaunchKernelGGL((k_umfma_group<STORE, NT>), dim3(p.num_tgroups), dim3(256), glds, st, p, k, alpha, beta, y,
                           ldy);
    else if (p.max_nseg <= 64)
        hipLaunchKernelGGL((k_umfma<STORE, NT, true>), dim3((p.num_tiles + 3) / 4), dim3(256), lds, st, p, k, alpha,
                           beta, y, ldy);
    else
        hipLaunchKernelGGL((k_umfma<STORE, NT, false>), dim3((p.num_tiles + 3) / 4), dim3(256), lds, st, p, k, alpha,
                           beta, y, ldy);
    if ((e = (int)hipGetLastError())) return e;
    if (mark) mark(ctx, 3);
    return 0;
}

template <int STORE>
int launch_mr_form(const DevPlanMR &p, int32_t k, float alpha, const float *x, int64_t ldx, float beta, float *y,
                   int64_t ldy, hipStream_t st, void (*mark)(void *, int), void *ctx) {
    switch ((k + 15) / 16) {
    case 1: return launch_mr_nt<STORE, 1>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 2: return launch_mr_nt<STORE, 2>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 3: return launch_mr_nt<STORE, 3>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 4: return launch_mr_nt<STORE, 4>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 5: return launch_mr_nt<STORE, 5>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 6: return launch_mr_nt<STORE, 6>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 7: return launch_mr_nt<STORE, 7>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    case 8: return launch_mr_nt<STORE, 8>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace

int launch_mr(const DevPlanMR &p, int32_t k, float alpha, const float *x, int64_t ldx, float beta, float *y,
              int64_t ldy, void *stream, void (*mark)(void *, int), void *ctx) {
    if (k < 1 || k > 128 || (k + 15) / 16 > p.ntmax) return (int)hipErrorInvalidValue;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        return launch_mr_form<HMAT_STORE_FP16_SCALED>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    if (p.storage == HMAT_STORE_FP8)
        return launch_mr_form<HMAT_STORE_FP8>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    if (p.storage == HMAT_STORE_FP8_F16D)
        return launch_mr_form<HMAT_STORE_FP8_F16D>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    if (p.storage == HMAT_STORE_BF16)
        return launch_mr_form<HMAT_STORE_BF16>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
    return launch_mr_form<HMAT_STORE_FP32>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
}

}  // namespace hmat
