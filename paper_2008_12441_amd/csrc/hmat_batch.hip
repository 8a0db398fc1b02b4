// Batched persistent launch (gfx950): many independent H-matrices applied by
// one kernel.
//
// The host lays every member's product out as a list of items (hmat_host.cpp)
// in stage bands: source side (V^T x, or X packing then V^T X), partial
// reduction, target side (U z + D x, writing y). Workgroups take items from
// one queue with an atomic ticket. An item that needs an earlier stage of its
// member waits on that member's stage counter; every item it can wait for was
// taken earlier by a running workgroup, so the queue always drains, however
// many workgroups are resident. The wait is bounded: past the poll limit it
// raises the error flag and goes on, so a fault in the dependency bookkeeping
// gives a reported error, never a hung GPU.
//
// Memory ordering: a producer item ends with every wave waiting for its own
// stores to complete, a workgroup barrier, then an agent-scope release
// increment of the stage counter by thread 0 (on gfx950 the release writes the
// L2 back, reaching across the XCDs, each of which has its own L2); a consumer's
// thread 0 polls the counter and takes an agent-scope acquire (L1/L2
// invalidate) before the workgroup barrier that releases the other waves.
//
// An item is a run of consecutive work indices of one stage of one member,
// grouped on the host up to a byte budget (the grain): waves take its indices
// in turn, whole-workgroup stages take them one after the other. The
// multi-RHS V products and target sides are whole-workgroup stages over unit
// groups and tile groups (four waves sharing one B sequence through LDS).
//
// The multi-RHS bodies read the n-tile scales that earlier items of the same
// launch wrote with vector loads into a register (one per lane) instead of
// through the scalar cache, whose contents are only valid for data constant
// during a launch.
#include "hmat_mr_device.h"
#include "hmat_sv_device.h"

namespace hmat {
namespace {

using namespace hmat::dev;

__global__ __launch_bounds__(256) void k_batch_clear(int32_t *ctl, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) ctl[i] = 0;
}

// Thread 0 of a workgroup: wait until ctl[idx] >= need, polling at most
// `limit` times; past that, raise the error flag and return.
__device__ inline void wait_counter(int32_t *ctl, int idx, int need, int limit) {
    int polls = 0;
    while (__hip_atomic_load(ctl + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++polls > limit) {
            __hip_atomic_fetch_or(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// A member's plan: the scalar fields in one read, each pointer on its own so
// that it is known to be global (see cptr).
#define HMAT_GLOBAL_FIELD(p, src, f) p.f = cptr(&src->f)

__device__ inline DevPlan load_plan(const DevPlan *m) {
    DevPlan p = cload(m);
    HMAT_GLOBAL_FIELD(p, m, V);
    HMAT_GLOBAL_FIELD(p, m, UD);
    HMAT_GLOBAL_FIELD(p, m, part);
    HMAT_GLOBAL_FIELD(p, m, slice);
    HMAT_GLOBAL_FIELD(p, m, zg);
    HMAT_GLOBAL_FIELD(p, m, chunks);
    HMAT_GLOBAL_FIELD(p, m, pbase);
    HMAT_GLOBAL_FIELD(p, m, zsegs);
    HMAT_GLOBAL_FIELD(p, m, dsegs);
    HMAT_GLOBAL_FIELD(p, m, dscale);
    HMAT_GLOBAL_FIELD(p, m, vtiles);
    HMAT_GLOBAL_FIELD(p, m, z1);
    HMAT_GLOBAL_FIELD(p, m, z2);
    return p;
}

__device__ inline DevPlanMR load_plan_mr(const DevPlanMR *m) {
    DevPlanMR p = cload(m);
    HMAT_GLOBAL_FIELD(p, m, V);
    HMAT_GLOBAL_FIELD(p, m, UD);
    HMAT_GLOBAL_FIELD(p, m, xpack);
    HMAT_GLOBAL_FIELD(p, m, zpack);
    HMAT_GLOBAL_FIELD(p, m, part);
    HMAT_GLOBAL_FIELD(p, m, sx);
    HMAT_GLOBAL_FIELD(p, m, sz);
    HMAT_GLOBAL_FIELD(p, m, dscale);
    HMAT_GLOBAL_FIELD(p, m, chunks);
    HMAT_GLOBAL_FIELD(p, m, vunits);
    HMAT_GLOBAL_FIELD(p, m, zitems);
    HMAT_GLOBAL_FIELD(p, m, zmembers);
    HMAT_GLOBAL_FIELD(p, m, segs);
    HMAT_GLOBAL_FIELD(p, m, tiles);
    HMAT_GLOBAL_FIELD(p, m, ustep);
    HMAT_GLOBAL_FIELD(p, m, scales);
    return p;
}

__device__ inline BArgs load_args(const BArgs *m) {
    BArgs a = cload(m);
    HMAT_GLOBAL_FIELD(a, m, x);
    HMAT_GLOBAL_FIELD(a, m, y);
    return a;
}

#undef HMAT_GLOBAL_FIELD

template <int STORE, bool HAS_S, bool HAS_M>
__global__ __launch_bounds__(256) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int s_ticket[2];  // double-buffered: written one iteration, read after its closing barrier
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave: work indices stay scalar
    if (tid == 0) s_ticket[0] = __hip_atomic_fetch_add(a.ctl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int t = __builtin_amdgcn_readfirstlane(s_ticket[0]);
    int par = 1;
    while (t < a.num_items) {
        // the next ticket is taken now; its value is needed only after this item
        int next = 0;
        if (tid == 0) next = __hip_atomic_fetch_add(a.ctl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const BItem it = cload(a.items, t);
        if (it.dep >= 0) {
            if (tid == 0) {
                wait_counter(a.ctl, it.dep, it.need, a.spin_limit);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
        }
        const BArgs ar = load_args(a.args + it.member);
        const int k = cload(a.members, it.member).k;
        if (HAS_S && it.kind <= BK_SU) {
            const DevPlan p = load_plan(&a.members[it.member].sp);
            if (it.kind == BK_SV) {
                for (int j = wave; j < it.count; j += 4) sv_vtile<STORE, float>(p, it.first + j, lane, ar.x);
            } else if (it.kind == BK_SZ1) {
                sv_z1_packed<float>(p, it.first, it.count, it.lanes, wave, lane);
            } else if (it.kind == BK_SZ2) {
                sv_z2_packed<float>(p, it.first, it.count, it.lanes, wave, lane);
            } else {
                for (int j = 0; j < it.count; ++j) {
                    if (j) __syncthreads();  // the previous chunk's operand is still being read from LDS
                    sv_chunk<STORE, float>(p, it.first + j, tid, reinterpret_cast<float *>(lds), ar.x, ar.y,
                                           ar.alpha, ar.beta);
                }
            }
        }
        if (HAS_M && it.kind >= BK_MX) {
            const DevPlanMR p = load_plan_mr(&a.members[it.member].mp);
            if (it.kind == BK_MX) {  // a wave per chunk; lane i loads the descriptor of the wave's i-th
                for (int j0 = 0; j0 < it.count; j0 += 256) {
                    const int jl = j0 + wave + 4 * lane;
                    MRChunk cl{};
                    if (jl < it.count) cl = p.chunks[it.first + jl];
                    for (int i = 0; j0 + wave + 4 * i < it.count && i < 64; ++i)
                        mr_xpack_wave<STORE>(p, it.first + j0 + wave + 4 * i, lane_bcast(cl, i), 0, ar.x, ar.ldx, k,
                                             lane);
                }
            } else if (it.kind == BK_MV) {  // unit groups, X fragments shared through the LDS ring
                for (int j = 0; j < it.count; ++j) mr_vunit_group<STORE, 1>(p, it.first + j, lds);
            } else if (it.kind == BK_MZ) {
                float(*zs)[16] = reinterpret_cast<float(*)[16]>(lds) + wave * a.zs_rank;
                for (int j0 = 0; j0 < it.count; j0 += 256) {  // lane i: the wave's i-th item and its first member
                    const int jl = j0 + wave + 4 * lane;
                    MRZItem zl{};
                    MRZMember ml{};
                    if (jl < it.count) {
                        zl = p.zitems[it.first + jl];
                        ml = p.zmembers[zl.m0];
                    }
                    for (int i = 0; j0 + wave + 4 * i < it.count && i < 64; ++i)
                        mr_zitem<STORE>(p, it.first + j0 + wave + 4 * i, lane_bcast(zl, i), lane_bcast(ml, i), 0, lane,
                                        zs);
                }
            } else {  // tile groups: the ring, then the chunk's step table
                int2 *stab = reinterpret_cast<int2 *>(lds + 2 * MR<STORE>::BFRAG * 16);
                for (int j = 0; j < it.count; ++j)
                    mr_tile_group<STORE, 1>(p, it.first + j, k, ar.alpha, ar.beta, ar.y, ar.ldy, lds, stab, nullptr);
            }
        }
        if (it.done >= 0) __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
        if (tid == 0) s_ticket[par] = next;
        __syncthreads();
        if (tid == 0 && it.done >= 0)
            __hip_atomic_fetch_add(a.ctl + it.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        t = __builtin_amdgcn_readfirstlane(s_ticket[par]);
        par ^= 1;
    }
}

template <int STORE, bool HAS_S, bool HAS_M>
int launch_form(const BatchArgs &a, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(256), 0, st, a.ctl, a.num_ctl);
    int e = (int)hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL((k_batch<STORE, HAS_S, HAS_M>), dim3(grid), dim3(256), lds, st, a);
    return (int)hipGetLastError();
}

template <int STORE>
int launch_mix(const BatchArgs &a, bool s, bool m, int grid, size_t lds, hipStream_t st) {
    if (s && m) return launch_form<STORE, true, true>(a, grid, lds, st);
    if (m) return launch_form<STORE, false, true>(a, grid, lds, st);
    return launch_form<STORE, true, false>(a, grid, lds, st);
}

template <int STORE, bool HAS_S, bool HAS_M>
int occupancy(size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<STORE, HAS_S, HAS_M>, 256, lds) != hipSuccess)
        return 0;
    return n;
}

template <int STORE>
int occupancy_mix(bool s, bool m, size_t lds) {
    if (s && m) return occupancy<STORE, true, true>(lds);
    if (m) return occupancy<STORE, false, true>(lds);
    return occupancy<STORE, true, false>(lds);
}

}  // namespace

int launch_batch(const BatchArgs &a, int32_t storage, bool has_single, bool has_multi, int grid, size_t lds,
                 void *stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (storage == HMAT_STORE_FP16_SCALED)
        return launch_mix<HMAT_STORE_FP16_SCALED>(a, has_single, has_multi, grid, lds, st);
    if (storage == HMAT_STORE_BF16) return launch_mix<HMAT_STORE_BF16>(a, has_single, has_multi, grid, lds, st);
    return launch_mix<HMAT_STORE_FP32>(a, has_single, has_multi, grid, lds, st);
}

int batch_max_wg_per_cu(int32_t storage, bool has_single, bool has_multi, size_t lds) {
    if (storage == HMAT_STORE_FP16_SCALED) return occupancy_mix<HMAT_STORE_FP16_SCALED>(has_single, has_multi, lds);
    if (storage == HMAT_STORE_BF16) return occupancy_mix<HMAT_STORE_BF16>(has_single, has_multi, lds);
    return occupancy_mix<HMAT_STORE_FP32>(has_single, has_multi, lds);
}

}  // namespace hmat
