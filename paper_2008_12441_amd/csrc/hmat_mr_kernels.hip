// HIP kernels (gfx950) of the multi-RHS H-matrix-vector product on MFMA.
//
// With k right-hand sides the local products of Sec. 4.1 become dense
// contractions: the source side Z = V^T X (Eq. (4.2) for k columns) and the
// target side Y += U Z and Y += D X (Eqs. (4.6)-(4.8)). Per group of at most
// 128 right-hand sides four launches run on the caller's stream:
//   k_xpack   X -> B fragments per chunk (FP16: hi + lo halves, one
//             power-of-two scale per chunk and column);
//   k_vmfma   per unit (level, source box, 64 V columns, up to 16 chunks):
//             partial sums of V^T X, accumulated across the unit's chunks;
//   k_zmfma   per low-rank block and n-tile: the fixed-order sum of its
//             partials (Steps 2-4 collapsed), times the block's scales, packed
//             as B fragments (FP16: with a power-of-two scale per column);
//   k_umfma   per row tile of one target leaf: Y over the z of every ancestor
//             block and over x of every source leaf, written once.
// Segment scales are powers of two, so moving the accumulators from one
// segment's scale to the next is exact.
#include <hip/hip_runtime.h>

#include "hmat.h"
#include "hmat_internal.h"

namespace hmat {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxRankMR = 128;

template <int STORE>
struct MR;

template <>
struct MR<HMAT_STORE_FP32> {
    static constexpr int KB = 16;     // inner indices per fragment
    static constexpr int VW = 4;      // per lane
    static constexpr int BFRAG = 64;  // 16-byte lane slots per B fragment
    static constexpr bool SCALED = false;
    using A = f32x4;
    struct B {
        f32x4 v;
    };
    __device__ static inline A loadA(const void *base, int64_t frag, int lane) {
        return __builtin_nontemporal_load(static_cast<const f32x4 *>(base) + frag * 64 + lane);
    }
    __device__ static inline B loadB(const void *base, int64_t frag, int lane) {
        B b;
        b.v = static_cast<const f32x4 *>(base)[frag * BFRAG + lane];
        return b;
    }
    __device__ static inline void storeB(void *base, int64_t frag, int lane, const float (&v)[VW]) {
        f32x4 t = {v[0], v[1], v[2], v[3]};
        static_cast<f32x4 *>(base)[frag * BFRAG + lane] = t;
    }
    __device__ static inline void mma(const A &a, const B &b, f32x4 &c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b.v[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b.v[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b.v[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b.v[3], c, 0, 0, 0);
    }
};

template <>
struct MR<HMAT_STORE_FP16_SCALED> {
    static constexpr int KB = 32;
    static constexpr int VW = 8;
    static constexpr int BFRAG = 128;  // hi (64 slots) then lo (64 slots)
    static constexpr bool SCALED = true;
    using A = f16x8;
    struct B {
        f16x8 hi, lo;
    };
    __device__ static inline A loadA(const void *base, int64_t frag, int lane) {
        return __builtin_nontemporal_load(static_cast<const f16x8 *>(base) + frag * 64 + lane);
    }
    __device__ static inline B loadB(const void *base, int64_t frag, int lane) {
        const f16x8 *p = static_cast<const f16x8 *>(base) + frag * BFRAG + lane;
        B b;
        b.hi = p[0];
        b.lo = p[64];
        return b;
    }
    // v is already divided by the column scale: split into two halves whose
    // sum carries about 22 significant bits
    __device__ static inline void storeB(void *base, int64_t frag, int lane, const float (&v)[VW]) {
        f16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            hi[e] = (_Float16)v[e];
            lo[e] = (_Float16)(v[e] - (float)hi[e]);
        }
        f16x8 *p = static_cast<f16x8 *>(base) + frag * BFRAG + lane;
        p[0] = hi;
        p[64] = lo;
    }
    __device__ static inline void mma(const A &a, const B &b, f32x4 &c) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b.lo, c, 0, 0, 0);
    }
};

// power of two with |v| / s <= 2^14 for |v| <= amax (1 for amax == 0)
__device__ inline float col_scale(float amax) {
    if (!(amax > 0.0f)) return 1.0f;
    int e = 0;
    const float m = frexpf(amax, &e);
    const int c = (m == 0.5f) ? e - 1 : e;
    return ldexpf(1.0f, c - 14);
}

__device__ inline float wave_max(float v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = fmaxf(v, __shfl_xor(v, s));
    return v;
}

__device__ inline int wave_id(int waves_per_block) {
    return __builtin_amdgcn_readfirstlane((int)blockIdx.x * waves_per_block + (int)(threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// X -> B fragments, one workgroup per chunk.
// ---------------------------------------------------------------------------
template <int STORE>
__global__ __launch_bounds__(256) void k_xpack(DevPlanMR p, const float *__restrict__ x, int64_t ldx, int k) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    __shared__ float sig[128];
    const int c = blockIdx.x;
    const MRChunk ch = p.chunks[c];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nt_used = (k + 15) / 16;
    const int ncol = p.ntmax * 16;
    if (F::SCALED) {
        for (int n = wave; n < nt_used * 16; n += 4) {
            float m = 0.0f;
            if (n < k)
                for (int i = lane; i < ch.rows; i += 64) m = fmaxf(m, fabsf(x[(int64_t)(ch.row_begin + i) + n * ldx]));
            m = wave_max(m);
            const float s = col_scale(m);
            if (lane == 0) {
                sig[n] = s;
                p.sx[(int64_t)c * ncol + n] = s;
            }
        }
        __syncthreads();
    }
    const int nfrag = ch.nkb * nt_used;
    for (int f = wave; f < nfrag; f += 4) {
        const int kb = f / nt_used, nt = f % nt_used;
        const int n = nt * 16 + (lane & 15);
        // the leaf holding this K-block (leaves start on K-block boundaries)
        int lf = 0;
        while (lf + 1 < ch.nleaf && p.leaves[ch.leaf_base + lf + 1].kb0 <= kb) ++lf;
        const MRLeaf L = p.leaves[ch.leaf_base + lf];
        const int off0 = (kb - L.kb0) * KB + VW * (lane >> 4);
        const float inv = F::SCALED ? 1.0f / sig[nt * 16 + (lane & 15)] : 1.0f;
        float v[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int o = off0 + e;
            v[e] = (n < k && o < L.rows) ? x[(int64_t)(L.row_begin + o) + n * ldx] * inv : 0.0f;
        }
        F::storeB(p.xpack, ch.xoff + (int64_t)kb * p.ntmax + nt, lane, v);
    }
}

// ---------------------------------------------------------------------------
// Source side: one wave per unit; acc[m-subtile][n-tile] are 16x16 tiles.
// ---------------------------------------------------------------------------
template <int STORE, int NT>
__global__ __launch_bounds__(256) void k_vmfma(DevPlanMR p) {
    using F = MR<STORE>;
    const int w = wave_id(4);
    if (w >= p.num_vunits) return;
    const int lane = threadIdx.x & 63;
    const MRVUnit u = p.vunits[w];
    const int nm = u.nm;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0, 0, 0, 0};
    float scur[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) scur[t] = 1.0f;
    const int ncol = p.ntmax * 16;
    int64_t af = u.aoff;
    for (int c = u.c0; c < u.c0 + u.nc; ++c) {
        const MRChunk ch = p.chunks[c];
        if (F::SCALED) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float s = p.sx[(int64_t)c * ncol + t * 16 + (lane & 15)];
                const float f = scur[t] / s;
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[m][t] *= f;
                scur[t] = s;
            }
        }
        for (int kb = 0; kb < ch.nkb; ++kb) {
            typename F::A a[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < nm) a[m] = F::loadA(p.V, af + (int64_t)kb * nm + m, lane);
            typename F::B b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = F::loadB(p.xpack, ch.xoff + (int64_t)kb * p.ntmax + t, lane);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < nm)
#pragma unroll
                    for (int t = 0; t < NT; ++t) F::mma(a[m], b[t], acc[m][t]);
        }
        af += (int64_t)ch.nkb * nm;
    }
    float *out = p.part + u.poff;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[(int64_t)(16 * m + 4 * (lane >> 4) + i) * ncol + t * 16 + (lane & 15)] = acc[m][t][i] * scur[t];
}

// ---------------------------------------------------------------------------
// Partial reduction and z packing: one wave per (low-rank block, n-tile).
// ---------------------------------------------------------------------------
template <int STORE>
__global__ __launch_bounds__(256) void k_zmfma(DevPlanMR p, int nt_used) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    __shared__ float zs[4][kMaxRankMR][16];
    const int w = wave_id(4);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (w >= p.num_zitems * nt_used) return;
    const int item = w / nt_used, nt = w % nt_used;
    const MRZItem z = p.zitems[item];
    const int ncol = p.ntmax * 16;
    const int nn = lane & 15, g = lane >> 4;
    const int n = nt * 16 + nn;
    const int64_t ustride = (int64_t)64 * ncol;
    float amax = 0.0f;
    for (int j = g; j < z.rank; j += 4) {
        const int col = z.vcol + j;
        const int64_t u0 = z.ubase + (int64_t)(col >> 6) * z.nu;
        const float *src = p.part + u0 * ustride + (int64_t)(col & 63) * ncol + n;
        float a0 = 0.0f, a1 = 0.0f;
        int i = 0;
        for (; i + 2 <= z.nu; i += 2) {
            a0 += src[(int64_t)i * ustride];
            a1 += src[(int64_t)(i + 1) * ustride];
        }
        if (i < z.nu) a0 += src[(int64_t)i * ustride];
        const float s = (a0 + a1) * z.scale;
        zs[wave][j][nn] = s;
        amax = fmaxf(amax, fabsf(s));
    }
    amax = fmaxf(amax, __shfl_xor(amax, 16));
    amax = fmaxf(amax, __shfl_xor(amax, 32));
    const float sig = F::SCALED ? col_scale(amax) : 1.0f;
    if (F::SCALED && g == 0) p.sz[(int64_t)item * ncol + n] = sig;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const float inv = 1.0f / sig;
    const int nkb = (z.rank + KB - 1) / KB;
    for (int kb = 0; kb < nkb; ++kb) {
        float v[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int j = kb * KB + VW * g + e;
            v[e] = j < z.rank ? zs[wave][j][nn] * inv : 0.0f;
        }
        F::storeB(p.zpack, z.zoff + (int64_t)kb * p.ntmax + nt, lane, v);
    }
}

// ---------------------------------------------------------------------------
// Target side: one wave per row tile (<= 64 rows of one target leaf).
// ---------------------------------------------------------------------------
template <int STORE, int NT>
__global__ __launch_bounds__(256) void k_umfma(DevPlanMR p, int k, float alpha, float beta, float *__restrict__ y,
                                               int64_t ldy) {
    using F = MR<STORE>;
    const int w = wave_id(4);
    if (w >= p.num_tiles) return;
    const int lane = threadIdx.x & 63;
    const MRTile tl = p.tiles[w];
    const MRChunk ch = p.chunks[tl.chunk];
    const int nm = tl.nm;
    const int ncol = p.ntmax * 16;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0, 0, 0, 0};
    float scur[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) scur[t] = 1.0f;
    int64_t af = tl.aoff;
    for (int si = ch.seg_base; si < ch.seg_base + ch.nseg; ++si) {
        const MRSeg sg = p.segs[si];
        if (F::SCALED) {
            const float ds = sg.kind ? p.dscale[ch.dscale_base + tl.tleaf * ch.nleaf + sg.leaf] : 1.0f;
            const float *srow = (sg.kind ? p.sx : p.sz) + (int64_t)sg.sidx * ncol;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float s = srow[t * 16 + (lane & 15)] * ds;
                const float f = scur[t] / s;
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[m][t] *= f;
                scur[t] = s;
            }
        }
        const void *bsrc = sg.kind ? p.xpack : p.zpack;
        for (int kb = 0; kb < sg.nkb; ++kb) {
            typename F::A a[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < nm) a[m] = F::loadA(p.UD, af + (int64_t)kb * nm + m, lane);
            typename F::B b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = F::loadB(bsrc, sg.src + (int64_t)kb * p.ntmax + t, lane);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < nm)
#pragma unroll
                    for (int t = 0; t < NT; ++t) F::mma(a[m], b[t], acc[m][t]);
        }
        af += (int64_t)sg.nkb * nm;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = t * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * m + 4 * (lane >> 4) + i;
                if (m < nm && row < tl.rows && n < k) {
                    float *yp = y + (int64_t)(tl.row0 + row) + (int64_t)n * ldy;
                    float v = alpha * (acc[m][t][i] * scur[t]);
                    if (beta != 0.0f) v = fmaf(beta, *yp, v);
                    *yp = v;
                }
            }
        }
}

template <int STORE, int NT>
int launch_mr_nt(const DevPlanMR &p, int32_t k, float alpha, const float *x, int64_t ldx, float beta, float *y,
                 int64_t ldy, hipStream_t st, void (*mark)(void *, int), void *ctx) {
    if (mark) mark(ctx, 0);
    hipLaunchKernelGGL(k_xpack<STORE>, dim3(p.num_chunks), dim3(256), 0, st, p, x, ldx, k);
    int e = (int)hipGetLastError();
    if (e) return e;
    if (p.num_vunits > 0) {
        hipLaunchKernelGGL((k_vmfma<STORE, NT>), dim3((p.num_vunits + 3) / 4), dim3(256), 0, st, p);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (mark) mark(ctx, 1);
    if (p.num_zitems > 0) {
        hipLaunchKernelGGL(k_zmfma<STORE>, dim3((p.num_zitems * NT + 3) / 4), dim3(256), 0, st, p, NT);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (mark) mark(ctx, 2);
    hipLaunchKernelGGL((k_umfma<STORE, NT>), dim3((p.num_tiles + 3) / 4), dim3(256), 0, st, p, k, alpha, beta, y,
                       ldy);
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
    return launch_mr_form<HMAT_STORE_FP32>(p, k, alpha, x, ldx, beta, y, ldy, st, mark, ctx);
}

}  // namespace hmat
