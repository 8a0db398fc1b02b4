// Device bodies of the single-vector product (one right-hand side), shared by
// the per-handle kernels and the batched persistent kernel.
//
//   sv_vtile   Step 1 on the source side (Eq. (4.2)): one wave, one vtile
//              (chunk, block of 64 V columns): partial sums of V^T x over the
//              chunk's rows, one column per lane;
//   sv_z1/z2   Steps 2-4 (tree-reduction, source-to-target transfer and
//              tree-broadcast) collapse to a fixed-order sum of those partials
//              over the chunks of each source box, written straight into the
//              target box's slot of z;
//   sv_chunk   Step 5 (Eqs. (4.6)-(4.8)): one workgroup, one chunk: every row
//              reads its U factors of all levels and its dense leaf row once,
//              against z and x staged in LDS, and writes y once.
//
// Every body is templated on its accumulator type: float for the product
// itself, double for the accuracy-check mode, where partial sums, z, the LDS
// operand and the row sums are all FP64 and y is rounded to FP32 at the store.
#pragma once

#include "hmat_device_common.h"

namespace hmat {
namespace dev {

template <int STORE>
struct Form;

template <>
struct Form<HMAT_STORE_FP32> {
    using Vec = f32x4;
    using Elem = float;
    static constexpr int VW = 4;
    __device__ static inline void load(const Vec *p, float (&v)[VW]) {
        const Vec t = __builtin_nontemporal_load(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
};

template <>
struct Form<HMAT_STORE_FP16_SCALED> {
    using Vec = f16x8;
    using Elem = _Float16;
    static constexpr int VW = 8;
    __device__ static inline void load(const Vec *p, float (&v)[VW]) {
        const Vec t = __builtin_nontemporal_load(p);
#pragma unroll
        for (int e = 0; e < VW; ++e) v[e] = (float)t[e];
    }
};

template <>
struct Form<HMAT_STORE_BF16> {
    using Vec = u32x4;
    using Elem = unsigned short;
    static constexpr int VW = 8;
    __device__ static inline void load(const Vec *p, float (&v)[VW]) {
        const Vec t = __builtin_nontemporal_load(p);
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // a BF16 code is the top half of an FP32 word
            v[2 * e] = __builtin_bit_cast(float, t[e] << 16);
            v[2 * e + 1] = __builtin_bit_cast(float, t[e] & 0xffff0000u);
        }
    }
};

#ifndef HMAT_VUNROLL
#define HMAT_VUNROLL 8
#endif
#ifndef HMAT_UUNROLL
#define HMAT_UUNROLL 8
#endif
constexpr int kVUnroll = HMAT_VUNROLL;  // 16-byte loads in flight per lane, V-phase
constexpr int kUUnroll = HMAT_UUNROLL;  // same for the U-phase

// ---------------------------------------------------------------------------
// V-phase: lane l owns column 64 cb + l of the chunk and accumulates
// sum_i V[i, col] x[i] over the chunk's rows. x is uniform across the wave,
// so its loads are scalar.
// ---------------------------------------------------------------------------
template <int STORE, class Acc>
__device__ inline void sv_vtile(const DevPlan &p, int w, int lane, const float *__restrict__ x) {
    using F = Form<STORE>;
    constexpr int VW = F::VW;
    const VTile vt = cload(p.vtiles, w);
    const int rows = cload(p.chunks, vt.chunk).rows;
    const float *__restrict__ xc = x + cload(p.chunks, vt.chunk).row_begin;
    const typename F::Vec *tile =
        reinterpret_cast<const typename F::Vec *>(static_cast<const typename F::Elem *>(p.V) + vt.off) + lane;
    Acc acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = 0;
    const int nfull = rows / VW;
    int q = 0;
    for (; q + kVUnroll <= nfull; q += kVUnroll) {
        float v[kVUnroll][VW];
#pragma unroll
        for (int u = 0; u < kVUnroll; ++u) F::load(tile + (int64_t)(q + u) * kWave, v[u]);
#pragma unroll
        for (int u = 0; u < kVUnroll; ++u)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = fma((Acc)v[u][e], (Acc)cload(xc, (q + u) * VW + e), acc[e]);
    }
    for (; q < nfull; ++q) {
        float v[VW];
        F::load(tile + (int64_t)q * kWave, v);
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = fma((Acc)v[e], (Acc)cload(xc, q * VW + e), acc[e]);
    }
    if (q * VW < rows) {  // ragged last vector: rows past the chunk hold zeros in V
        float v[VW];
        F::load(tile + (int64_t)q * kWave, v);
#pragma unroll
        for (int e = 0; e < VW; ++e)
            if (q * VW + e < rows) acc[e] = fma((Acc)v[e], (Acc)cload(xc, q * VW + e), acc[e]);
    }
    Acc s = 0;
#pragma unroll
    for (int e = 0; e < VW; ++e) s += acc[e];
    static_cast<Acc *>(p.part)[vt.pout + lane] = s;
}

// ---------------------------------------------------------------------------
// Partial reduction, stage 1: one wave per item; the item sums, in chunk
// order, the partials of one block over at most 32 consecutive chunks of its
// source box. Items of boxes that span more chunks write slices that stage 2
// adds up, also in order, so the result is deterministic.
// ---------------------------------------------------------------------------
template <class Acc>
__device__ inline void sv_z1(const DevPlan &p, int w, int lane) {
    const ZItem it = cload(p.z1, w);
    const int32_t *pb = p.pbase + it.chunk0;
    Acc *zg = static_cast<Acc *>(p.zg);
    for (int k = lane; k < it.rank; k += kWave) {
        // eight independent partial sums keep eight loads in flight; they are
        // combined in a fixed order, so the result stays deterministic
        Acc a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const Acc *src = static_cast<const Acc *>(p.part) + it.vcol + k;
        int c = 0;
        for (; c + 8 <= it.nchunks; c += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += src[cload(pb, c + u)];
        }
        for (; c < it.nchunks; ++c) a[0] += src[cload(pb, c)];
        const Acc s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        zg[it.dst + k] = s * (Acc)it.scale;
    }
}

template <class Acc>
__device__ inline void sv_z2(const DevPlan &p, int w, int lane) {
    const ZItem2 it = cload(p.z2, w);
    Acc *zg = static_cast<Acc *>(p.zg);
    for (int k = lane; k < it.rank; k += kWave) {
        Acc a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const Acc *src = zg + it.src + k;
        int c = 0;
        for (; c + 8 <= it.nslices; c += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += src[(c + u) * it.rank];
        }
        for (; c < it.nslices; ++c) a[0] += src[c * it.rank];
        const Acc s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        zg[it.dst + k] = s * (Acc)it.scale;
    }
}

// The two reduction stages over a run of items [first, first + count), for
// ranks well below 64: a wave takes 64 / R items at a time, lane l working
// on item l / R and rank index l % R (R a power of two; an item of larger
// rank loops). Each item's sums are the ones sv_z1 / sv_z2 form, in the same
// order, so the results are bitwise the same.
template <class Acc>
__device__ inline void sv_z1_packed(const DevPlan &p, int first, int count, int R, int wave, int lane) {
    const int per = 64 / R, sub = lane / R, kk = lane % R;
    Acc *zg = static_cast<Acc *>(p.zg);
    for (int j = wave * per + sub; j < count; j += 4 * per) {
        const ZItem it = p.z1[first + j];
        const int32_t *pb = p.pbase + it.chunk0;
        for (int k = kk; k < it.rank; k += R) {
            Acc a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const Acc *src = static_cast<const Acc *>(p.part) + it.vcol + k;
            int c = 0;
            for (; c + 8 <= it.nchunks; c += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += src[pb[c + u]];
            }
            for (; c < it.nchunks; ++c) a[0] += src[pb[c]];
            const Acc s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
            zg[it.dst + k] = s * (Acc)it.scale;
        }
    }
}

template <class Acc>
__device__ inline void sv_z2_packed(const DevPlan &p, int first, int count, int R, int wave, int lane) {
    const int per = 64 / R, sub = lane / R, kk = lane % R;
    Acc *zg = static_cast<Acc *>(p.zg);
    for (int j = wave * per + sub; j < count; j += 4 * per) {
        const ZItem2 it = p.z2[first + j];
        for (int k = kk; k < it.rank; k += R) {
            Acc a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const Acc *src = zg + it.src + k;
            int c = 0;
            for (; c + 8 <= it.nslices; c += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += src[(c + u) * it.rank];
            }
            for (; c < it.nslices; ++c) a[0] += src[c * it.rank];
            const Acc s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
            zg[it.dst + k] = s * (Acc)it.scale;
        }
    }
}

// ---------------------------------------------------------------------------
// U-phase + dense near field + output for one chunk, by a workgroup of 256
// threads. The chunk's vector operand (its ancestors' z segments, then x over
// each source leaf) is staged in LDS; each wave takes 64-row tiles, one row
// per lane, and reads VW columns per 16-byte load with the operand broadcast
// from LDS.
// ---------------------------------------------------------------------------
template <int STORE, class Acc>
__device__ inline Acc dot_range(const typename Form<STORE>::Vec *base, const Acc *vec, int q0, int q1) {
    using F = Form<STORE>;
    constexpr int VW = F::VW;
    Acc a[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) a[e] = 0;
    int q = q0;
    for (; q + kUUnroll <= q1; q += kUUnroll) {
        float v[kUUnroll][VW];
#pragma unroll
        for (int u = 0; u < kUUnroll; ++u) F::load(base + (int64_t)(q + u) * kWave, v[u]);
#pragma unroll
        for (int u = 0; u < kUUnroll; ++u)
#pragma unroll
            for (int e = 0; e < VW; ++e) a[e] = fma((Acc)v[u][e], vec[(q + u) * VW + e], a[e]);
    }
    for (; q < q1; ++q) {
        float v[VW];
        F::load(base + (int64_t)q * kWave, v);
#pragma unroll
        for (int e = 0; e < VW; ++e) a[e] = fma((Acc)v[e], vec[q * VW + e], a[e]);
    }
    Acc s = 0;
#pragma unroll
    for (int e = 0; e < VW; ++e) s += a[e];
    return s;
}

template <int STORE, class Acc>
__device__ inline void sv_chunk(const DevPlan &p, int c, int tid, Acc *vec, const float *__restrict__ x,
                                float *__restrict__ y, float alpha, float beta) {
    using F = Form<STORE>;
    constexpr int VW = F::VW;
    const Acc *zg = static_cast<const Acc *>(p.zg);
    const ChunkMeta m = cload(p.chunks, c);
    int pos = 0;
    for (int l = 0; l < p.num_levels; ++l) {
        const ZSeg zs = cload(p.zsegs, m.zseg_base + l);
        for (int j = tid; j < zs.len; j += 256) vec[pos + j] = zg[zs.off + j];
        pos += zs.len;
    }
    for (int j = pos + tid; j < m.nq_lr * VW; j += 256) vec[j] = 0;
    pos = m.nq_lr * VW;
    for (int s = 0; s < m.nleaf; ++s) {
        const DSeg ds = cload(p.dsegs, m.dseg_base + s);
        for (int j = tid; j < ds.nq * VW; j += 256) vec[pos + j] = j < ds.rows ? (Acc)x[ds.row_begin + j] : (Acc)0;
        pos += ds.nq * VW;
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int ntile = (m.rows + kWave - 1) / kWave;
    for (int tile = wave; tile < ntile; tile += 4) {
        const typename F::Vec *base =
            reinterpret_cast<const typename F::Vec *>(static_cast<const typename F::Elem *>(p.UD) + m.ud_off) +
            (int64_t)tile * m.nq * kWave + lane;
        const int row = tile * kWave + lane;
        Acc acc = dot_range<STORE, Acc>(base, vec, 0, m.nq_lr);
        int tleaf = 0;  // the row's target leaf: the target segments follow the source segments
        if (STORE == HMAT_STORE_FP16_SCALED)
            while (tleaf + 1 < m.ntleaf &&
                   m.row_begin + row >= cload(p.dsegs, m.dseg_base + m.nleaf + tleaf + 1).row_begin)
                ++tleaf;
        int q = m.nq_lr;
        for (int s = 0; s < m.nleaf; ++s) {
            const int nq = cload(p.dsegs, m.dseg_base + s).nq;
            const Acc part = dot_range<STORE, Acc>(base, vec, q, q + nq);
            if (STORE == HMAT_STORE_FP16_SCALED)
                acc = fma((Acc)cload(p.dscale, m.dscale_base + tleaf * m.nleaf + s), part, acc);
            else
                acc += part;
            q += nq;
        }
        if (row < m.rows) {
            float *yp = y + m.row_begin + row;
            Acc v = (Acc)alpha * acc;
            if (beta != 0.0f) v = fma((Acc)beta, (Acc)*yp, v);
            *yp = (float)v;  // the only rounding to FP32 of the output
        }
    }
}

}  // namespace dev
}  // namespace hmat
