// Device bodies of the multi-RHS product on MFMA, shared by the per-handle
// kernels and the batched persistent kernel.
//
// With k right-hand sides the local products of Sec. 4.1 become dense
// contractions: the source side Z = V^T X (Eq. (4.2) for k columns) and the
// target side Y += U Z and Y += D X (Eqs. (4.6)-(4.8)):
//   mr_xpack   X -> B fragments per chunk (FP16: hi + lo halves, one
//              power-of-two scale per chunk and n-tile of 16 columns);
//   mr_vunit_group  per group of up to four units (a unit: level, source
//              box, 64 V columns, up to 4 chunks): partial sums of V^T X,
//              accumulated across the unit's chunks;
//   mr_zitem   per z item (the low-rank blocks of one target box) and n-tile:
//              the fixed-order sum of each block's partials (Steps 2-4
//              collapsed), times the block's scales, stacked and packed as B
//              fragments (FP16: with a power-of-two scale per n-tile);
//   mr_tile_group, mr_tile  per group of up to four row tiles of one chunk,
//              or per row tile: Y over the z of every ancestor block and over
//              x of every source leaf, written once.
// Segment scales are powers of two, so moving the accumulators from one
// segment's scale to the next is exact.
#pragma once

#include "hmat_device_common.h"

#include <type_traits>

namespace hmat {
namespace dev {

constexpr int kMaxRankMR = 128;

// waves per SIMD the MFMA kernels are compiled for: two while the
// accumulators and the double-buffered fragments fit in 256 registers
template <int NT>
struct Occupancy {
    static constexpr int waves = NT <= 4 ? 2 : 1;
};

template <int STORE>
struct MR;

typedef __amdgpu_buffer_rsrc_t rsrc_t;

// A buffer resource starting at p (raw, byte offsets below 4 GiB).
__device__ inline rsrc_t make_rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, -1, 0x00020000);
}

constexpr int kNontemporal = 2;  // cache-policy bits of a streaming (read-once) load

// Uniform (wave-wide) values read through the scalar cache.
typedef __attribute__((address_space(4))) const float cfloat;
__device__ inline float sload(const float *p, int i) { return ((cfloat *)p)[i]; }

template <int AUX>
__device__ inline f32x4 buf16(rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}

template <>
struct MR<HMAT_STORE_FP32> {
    static constexpr int KB = 16;     // inner indices per fragment
    static constexpr int VW = 4;      // per lane
    static constexpr int BFRAG = 64;  // 16-byte lane slots per B fragment
    static constexpr bool SCALED = false;
    using A = f32x4;
    using Op = A;
    static constexpr bool FP8 = false;
    struct B {
        f32x4 v;
    };
    // A fragment at byte offset soff of r; lane l reads bytes [16 l, 16 l + 16)
    __device__ static inline A loadA(rsrc_t r, int soff, int lane) { return buf16<kNontemporal>(r, lane * 16, soff); }
    __device__ static inline B loadB(rsrc_t r, int soff, int lane) {
        B b;
        b.v = buf16<0>(r, lane * 16, soff);
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
    using Op = A;
    static constexpr bool FP8 = false;
    struct B {
        f16x8 hi, lo;
    };
    __device__ static inline A loadA(rsrc_t r, int soff, int lane) {
        return __builtin_bit_cast(f16x8, buf16<kNontemporal>(r, lane * 16, soff));
    }
    __device__ static inline B loadB(rsrc_t r, int soff, int lane) {
        B b;
        b.hi = __builtin_bit_cast(f16x8, buf16<0>(r, lane * 16, soff));
        b.lo = __builtin_bit_cast(f16x8, buf16<0>(r, lane * 16 + 1024, soff));
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

template <>
struct MR<HMAT_STORE_BF16> {
    static constexpr int KB = 32;
    static constexpr int VW = 8;
    static constexpr int BFRAG = 128;   // hi (64 slots) then lo (64 slots)
    static constexpr bool SCALED = false;  // BF16 keeps FP32's exponent range
    using A = bf16x8;
    using Op = A;
    static constexpr bool FP8 = false;
    struct B {
        bf16x8 hi, lo;
    };
    __device__ static inline A loadA(rsrc_t r, int soff, int lane) {
        return __builtin_bit_cast(bf16x8, buf16<kNontemporal>(r, lane * 16, soff));
    }
    __device__ static inline B loadB(rsrc_t r, int soff, int lane) {
        B b;
        b.hi = __builtin_bit_cast(bf16x8, buf16<0>(r, lane * 16, soff));
        b.lo = __builtin_bit_cast(bf16x8, buf16<0>(r, lane * 16 + 1024, soff));
        return b;
    }
    // two BF16 parts whose sum carries about 16 significant bits
    __device__ static inline void storeB(void *base, int64_t frag, int lane, const float (&v)[VW]) {
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            hi[e] = (__bf16)v[e];
            lo[e] = (__bf16)(v[e] - (float)hi[e]);
        }
        bf16x8 *p = static_cast<bf16x8 *>(base) + frag * BFRAG + lane;
        p[0] = hi;
        p[64] = lo;
    }
    __device__ static inline void mma(const A &a, const B &b, f32x4 &c) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.lo, c, 0, 0, 0);
    }
};

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// FP8 forms: U and V fragments hold per lane 8 E4M3 hi codes then 8 lo codes
// (OCP E4M3FN, converted exactly by the hardware), D fragments 8 BF16 codes
// (DBF16) or 8 FP16 codes; every A fragment reaches the MFMA as FP16, against
// FP16 hi + lo activations as in the FP16 form.
template <bool DBF16>
struct MRFp8 {
    static constexpr int KB = 32;
    static constexpr int VW = 8;
    static constexpr int BFRAG = 128;  // hi (64 slots) then lo (64 slots)
    static constexpr bool SCALED = true;
    static constexpr bool FP8 = true;
    using A = u32x4;                   // the lane's raw 16 bytes
    using Op = f16x8;
    struct B {
        f16x8 hi, lo;
    };
    __device__ static inline A loadA(rsrc_t r, int soff, int lane) {
        return __builtin_bit_cast(u32x4, buf16<kNontemporal>(r, lane * 16, soff));
    }
    __device__ static inline B loadB(rsrc_t r, int soff, int lane) {
        B b;
        b.hi = __builtin_bit_cast(f16x8, buf16<0>(r, lane * 16, soff));
        b.lo = __builtin_bit_cast(f16x8, buf16<0>(r, lane * 16 + 1024, soff));
        return b;
    }
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
    // RNE_f16(hi + s' lo) for the lane's 8 elements; s2[q] holds the lo
    // scales of elements 2q and 2q + 1. Both conversions are exact, so the
    // fused multiply-add rounds once.
    __device__ static inline Op hilo(const A &r, const h2 (&s2)[4]) {
        Op o;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const h2 h0 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(r[w], 1.0f, false);
            const h2 h1 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(r[w], 1.0f, true);
            const h2 l0 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(r[2 + w], 1.0f, false);
            const h2 l1 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(r[2 + w], 1.0f, true);
            const h2 v0 = __builtin_elementwise_fma(l0, s2[2 * w], h0);
            const h2 v1 = __builtin_elementwise_fma(l1, s2[2 * w + 1], h1);
            o[4 * w] = v0[0];
            o[4 * w + 1] = v0[1];
            o[4 * w + 2] = v1[0];
            o[4 * w + 3] = v1[1];
        }
        return o;
    }
    // D codes as FP16 (BF16 -> FP16 is exact for |value| >= 2^-14)
    __device__ static inline Op dense(const A &r) {
        if constexpr (DBF16) {
            Op o;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                o[2 * w] = (_Float16)__builtin_bit_cast(float, r[w] << 16);
                o[2 * w + 1] = (_Float16)__builtin_bit_cast(float, r[w] & 0xffff0000u);
            }
            return o;
        } else {
            return __builtin_bit_cast(Op, r);
        }
    }
    __device__ static inline void mma(const Op &a, const B &b, f32x4 &c) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b.lo, c, 0, 0, 0);
    }
};

template <>
struct MR<HMAT_STORE_FP8> : MRFp8<true> {};
template <>
struct MR<HMAT_STORE_FP8_F16D> : MRFp8<false> {};

// Forms whose fragments feed the MFMA as loaded.
template <int STORE>
struct IsFp8 {
    static constexpr bool value = STORE == HMAT_STORE_FP8 || STORE == HMAT_STORE_FP8_F16D;
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

// ---------------------------------------------------------------------------
// The K-block step loop shared by both contractions. Step s multiplies the A
// fragments af0 + s * nm + m (m < nm) with the B fragments that info(s)
// points at (n-tile t at + t * 16 * BFRAG bytes). In the scaled form the B
// values of step s carry the n-tile scales info(s).srow[t] * info(s).fac;
// whenever those change, the accumulators are moved to the new scales
// (powers of two, so the move is exact). info is called in increasing s.
//
// prep(a, m, info(s)) turns a loaded A fragment into the MFMA operand (the
// FP8 forms dequantise there; the other forms pass it through).
//
// Without LANE_SCALES the scales are read through the scalar cache from
// info(s).srow, which requires them to stay unchanged during the launch. With
// LANE_SCALES the caller has loaded the scales the wave needs into sv[t] (lane
// j: segment j's scale of n-tile t, with vector loads, so they may have been
// written earlier in the same launch), and step s takes lane info(s).sidx of
// them: no scalar memory access on the path of a step.
// ---------------------------------------------------------------------------
struct StepInfo {
    int64_t bofs;        // byte offset of the step's B fragments
    const float *srow;   // n-tile scales of the step's B (scaled form), read through the scalar cache
    float fac;           // extra power-of-two factor of those scales
    int32_t sidx;        // LANE_SCALES: lane of sv holding the step's scales (srow unused)
    int32_t dense;       // FP8 forms: the step multiplies D (else U or V)
    int32_t lofs;        // FP8 forms, U steps: offset of the step's 32 lo-scales in the wave's LDS table
};

// B fragment t of a scaled form times a power of two f <= 1: exact while the
// products stay normal FP16; below that, the rounding is at most 2^-24 of the
// common scale, far under FP32 resolution of the result.
template <class B>
__device__ inline void scale_b(B &b, float f) {
    const _Float16 h = (_Float16)f;
    b.hi *= h;
    b.lo *= h;
}

// The largest of the lanes' scales (lanes >= n hold none): the common scale of a tile.
__device__ inline float lanes_max(float v, int lane, int n) {
    float m = lane < n ? v : 0.0f;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
    return m > 0.0f ? m : 1.0f;
}

template <int STORE, int NT, bool LANE_SCALES, class Info, class Prep>
__device__ inline void mfma_steps(const void *A, const void *B, int64_t af0, int nm, int nsteps, int lane, Info info,
                                  Prep prep, f32x4 (&acc)[4][NT], float (&scur)[NT], const float (&sv)[NT],
                                  int nsv = 0) {
    using F = MR<STORE>;
    auto scale_of = [&](const StepInfo &i, int t) {
        return LANE_SCALES ? __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sv[t]), i.sidx))
                           : sload(i.srow, t);
    };
    if (nsteps <= 0) return;
    const rsrc_t ra = make_rsrc(static_cast<const char *>(A) + af0 * 1024);
    // Four register sets for A (loaded four steps ahead), two for B (one step
    // ahead). Every load is issued unconditionally, with indices clamped to
    // the last step and m-subtile (re-reading fragments already in cache):
    // loads under branches make the wait counters conservative and would
    // drain the prefetched fragments at every step.
    typename F::A a0[4], a1[4], a2[4], a3[4];
    typename F::B b0[NT], b1[NT];
    auto load_a = [&](typename F::A(&a)[4], int st) {
        const int sc = st < nsteps ? st : nsteps - 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) a[m] = F::loadA(ra, (sc * nm + (m < nm ? m : nm - 1)) * 1024, lane);
    };
    auto load_b = [&](typename F::B(&b)[NT], int64_t bofs) {
        const rsrc_t rb = make_rsrc(static_cast<const char *>(B) + bofs);
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = F::loadB(rb, t * 16 * F::BFRAG, lane);
    };
    // With lane scales (sv[t] holds nsv scales, the step's dense factor
    // already folded in) every n-tile keeps one common scale, the largest of
    // the tile's: each step's B is multiplied by its own scale over the common
    // one (a power of two <= 1), and the accumulators are never rescaled.
    // Without them, the accumulators move to each new scale as it comes.
    constexpr bool kCommon = LANE_SCALES && F::SCALED;
    if constexpr (kCommon) {
#pragma unroll
        for (int t = 0; t < NT; ++t) scur[t] = lanes_max(sv[t], lane, nsv);
    }
    // scales of the current step's B and whether they differ from the last
    // step's; the next step's are read one step ahead
    StepInfo ic = info(0), in_;
    float sc[NT], sn[NT];
    bool chg_c = true, chg_n = false;
    if (F::SCALED) {
#pragma unroll
        for (int t = 0; t < NT; ++t) sc[t] = scale_of(ic, t) * ic.fac;
    }
    auto step = [&](typename F::A(&a)[4], typename F::B(&b)[NT], typename F::B(&bn)[NT], int st) {
        in_ = info(st + 1 < nsteps ? st + 1 : nsteps - 1);
        load_b(bn, in_.bofs);
        if constexpr (kCommon) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                sn[t] = scale_of(in_, t) * in_.fac;
                const float f = sc[t] * __builtin_amdgcn_rcpf(scur[t]);  // powers of two: exact
                if (f != 1.0f) scale_b(b[t], f);
            }
        } else if (F::SCALED) {
            chg_n = in_.srow != ic.srow || in_.sidx != ic.sidx || in_.fac != ic.fac;
#pragma unroll
            for (int t = 0; t < NT; ++t) sn[t] = chg_n ? scale_of(in_, t) * in_.fac : sc[t];
            if (chg_c) {  // this step's B carries new n-tile scales: move the accumulators
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const float f = scur[t] * __builtin_amdgcn_rcpf(sc[t]);  // powers of two: exact
#pragma unroll
                    for (int m = 0; m < 4; ++m) acc[m][t] *= f;
                    scur[t] = sc[t];
                }
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (m < nm) {
                const typename F::Op op = prep(a[m], m, ic);  // the fragment as the MFMA takes it
#pragma unroll
                for (int t = 0; t < NT; ++t) F::mma(op, b[t], acc[m][t]);
            }
        load_a(a, st + 4);
        ic = in_;
        if (F::SCALED) {
            chg_c = chg_n;
#pragma unroll
            for (int t = 0; t < NT; ++t) sc[t] = sn[t];
        }
    };
    load_b(b0, ic.bofs);
    load_a(a0, 0);
    load_a(a1, 1);
    load_a(a2, 2);
    load_a(a3, 3);
    // whole groups of four steps without exits (the wait counts stay exact),
    // then the remaining ones
    int st = 0;
    for (; st + 4 <= nsteps; st += 4) {
        step(a0, b0, b1, st);
        step(a1, b1, b0, st + 1);
        step(a2, b0, b1, st + 2);
        step(a3, b1, b0, st + 3);
    }
    if (st < nsteps) step(a0, b0, b1, st);
    if (st + 1 < nsteps) step(a1, b1, b0, st + 1);
    if (st + 2 < nsteps) step(a2, b0, b1, st + 2);
}

// ---------------------------------------------------------------------------
// X -> B fragments for one (chunk, n-tile of 16 columns), by a workgroup of
// 256 threads; red (4 floats of LDS) takes the per-wave maxima. Lane l of
// wave w reads rows 8 (l / 16) .. of K-blocks w, w + 4, ... of column
// 16 nt + l % 16, which is where they sit in the fragment. The first four
// K-blocks of every wave stay in registers between the amax and the split, so
// a chunk of up to 16 K-blocks (512 rows in FP16) reads X once; the rest of a
// longer chunk is read a second time.
// ---------------------------------------------------------------------------
template <int STORE>
__device__ inline void mr_xpack(const DevPlanMR &p, int c, int nt, const float *__restrict__ x, int64_t ldx, int k,
                                float *red) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    constexpr int R = 4;  // K-blocks per wave held in registers
    const MRChunk ch = cload(p.chunks, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = nt * 16 + (lane & 15);
    const float *col = x + (int64_t)n * ldx + ch.row_begin;
    auto gather = [&](int kb, float (&v)[VW]) {  // zero past the chunk's rows and past column k
        const int off0 = kb * KB + VW * (lane >> 4);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int o = off0 + e;
            v[e] = (n < k && o < ch.rows) ? col[o] : 0.0f;
        }
    };
    auto store = [&](int kb, const float (&v)[VW], float inv) {
        float t[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) t[e] = v[e] * inv;
        F::storeB(p.xpack, ch.xoff + (int64_t)kb * p.ntmax + nt, lane, t);
    };
    float v[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (wave + 4 * r < ch.nkb) {
            gather(wave + 4 * r, v[r]);
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) v[r][e] = 0.0f;
        }
    }
    float inv = 1.0f;
    if (F::SCALED) {
        float m = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VW; ++e) m = fmaxf(m, fabsf(v[r][e]));
        for (int kb = wave + 4 * R; kb < ch.nkb; kb += 4) {
            float t[VW];
            gather(kb, t);
#pragma unroll
            for (int e = 0; e < VW; ++e) m = fmaxf(m, fabsf(t[e]));
        }
        m = wave_max(m);
        if (lane == 0) red[wave] = m;
        __syncthreads();
        const float s = col_scale(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
        if (tid == 0) p.sx[(int64_t)c * p.ntmax + nt] = s;
        inv = 1.0f / s;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (wave + 4 * r < ch.nkb) store(wave + 4 * r, v[r], inv);
    for (int kb = wave + 4 * R; kb < ch.nkb; kb += 4) {
        float t[VW];
        gather(kb, t);
        store(kb, t, inv);
    }
}

// Lane i's copy of a descriptor held one per lane (i uniform), word by word.
template <class T>
__device__ inline T lane_bcast(const T &v, int i) {
    static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
    struct W { int w[sizeof(T) / 4]; };
    W a = __builtin_bit_cast(W, v);
#pragma unroll
    for (int j = 0; j < (int)(sizeof(T) / 4); ++j) a.w[j] = __builtin_amdgcn_readlane(a.w[j], i);
    return __builtin_bit_cast(T, a);
}

// ---------------------------------------------------------------------------
// The same packing by one wave per (chunk, n-tile), for the batched kernel,
// whose chunks are mostly a few hundred rows or less: the four waves of a
// workgroup pack four chunks at once instead of one after the other. The
// first 128 rows stay in registers between the maximum and the split; the rest
// of a longer chunk is read a second time (from L2, as a rule). The fragments and the scale are the
// ones mr_xpack and mr_xpack_tile write. ch is chunk c's descriptor (row_begin, rows, nkb and xoff
// are read), which the caller loads ahead.
// ---------------------------------------------------------------------------
template <int STORE>
__device__ inline void mr_xpack_wave(const DevPlanMR &p, int c, const MRChunk &ch, int nt,
                                     const float *__restrict__ x, int64_t ldx, int k, int lane) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    constexpr int R = 128 / KB;  // K-blocks held in registers
    const int n = nt * 16 + (lane & 15);
    const float *col = x + (int64_t)n * ldx + ch.row_begin;
    auto gather = [&](int kb, float (&v)[VW]) {  // zero past the chunk's rows and past column k
        const int off0 = kb * KB + VW * (lane >> 4);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int o = off0 + e;
            v[e] = (n < k && o < ch.rows) ? col[o] : 0.0f;
        }
    };
    auto store = [&](int kb, const float (&v)[VW], float inv) {
        float t[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) t[e] = v[e] * inv;
        F::storeB(p.xpack, ch.xoff + (int64_t)kb * p.ntmax + nt, lane, t);
    };
    float v[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r < ch.nkb) {
            gather(r, v[r]);
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) v[r][e] = 0.0f;
        }
    }
    float inv = 1.0f;
    if (F::SCALED) {
        float m = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VW; ++e) m = fmaxf(m, fabsf(v[r][e]));
        for (int kb = R; kb < ch.nkb; ++kb) {
            float t[VW];
            gather(kb, t);
#pragma unroll
            for (int e = 0; e < VW; ++e) m = fmaxf(m, fabsf(t[e]));
        }
        const float s = col_scale(wave_max(m));
        if (lane == 0) p.sx[(int64_t)c * p.ntmax + nt] = s;
        inv = 1.0f / s;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < ch.nkb) store(r, v[r], inv);
    for (int kb = R; kb < ch.nkb; ++kb) {
        float t[VW];
        gather(kb, t);
        store(kb, t, inv);
    }
}

// ---------------------------------------------------------------------------
// The same packing for chunks of at most 512 rows, with X read coalesced: each
// wave reads four of the 16 columns, 64 consecutive rows per instruction, into
// an LDS tile (16 x (rows + 1) floats, the padding spreads the banks), and the
// fragments are then assembled from LDS. Same values as mr_xpack.
// ---------------------------------------------------------------------------
constexpr int kXpackMaxRows = 512;

template <int STORE>
__device__ inline void mr_xpack_tile(const DevPlanMR &p, int c, int nt, const float *__restrict__ x, int64_t ldx,
                                     int k, float *tile, float *red) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    const MRChunk ch = cload(p.chunks, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rs = ch.rows + 1;  // LDS row stride of a column
    float m = 0.0f;
    float v[4][kXpackMaxRows / 64];
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // all loads first: 32 in flight per thread
        const int n = nt * 16 + 4 * wave + j;
        const float *col = x + (int64_t)n * ldx + ch.row_begin;
#pragma unroll
        for (int i = 0; i < kXpackMaxRows / 64; ++i) {
            const int r = lane + 64 * i;
            v[j][i] = (n < k && r < ch.rows) ? col[r] : 0.0f;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < kXpackMaxRows / 64; ++i) {
            const int r = lane + 64 * i;
            if (r < ch.rows) tile[(4 * wave + j) * rs + r] = v[j][i];
            m = fmaxf(m, fabsf(v[j][i]));
        }
    float inv = 1.0f;
    if (F::SCALED) {
        m = wave_max(m);
        if (lane == 0) red[wave] = m;
    }
    __syncthreads();
    if (F::SCALED) {
        const float sc = col_scale(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
        if (tid == 0) p.sx[(int64_t)c * p.ntmax + nt] = sc;
        inv = 1.0f / sc;
    }
    const int j = lane & 15;
    const float *src = tile + j * rs;
    for (int kb = wave; kb < ch.nkb; kb += 4) {
        const int off0 = kb * KB + VW * (lane >> 4);
        float t[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) t[e] = off0 + e < ch.rows ? src[off0 + e] * inv : 0.0f;
        F::storeB(p.xpack, ch.xoff + (int64_t)kb * p.ntmax + nt, lane, t);
    }
}

// ---------------------------------------------------------------------------
// Partial reduction and z packing, one wave per (z item, n-tile): the z of the
// item's blocks stacked in their rows, then packed as B fragments with one
// power-of-two scale for the item and n-tile. zs is the wave's LDS scratch of
// kMaxRankMR x 16 floats; z is the item's descriptor and zm0 its first member's.
// ---------------------------------------------------------------------------
template <int STORE>
__device__ inline void mr_zitem(const DevPlanMR &p, int item, const MRZItem &z, const MRZMember &zm0, int nt,
                                int lane, float (*zs)[16]) {
    using F = MR<STORE>;
    constexpr int VW = F::VW;
    constexpr int KB = F::KB;
    const int ncol = p.ntmax * 16;
    const int nn = lane & 15, g = lane >> 4;
    const int n = nt * 16 + nn;
    const int64_t ustride = (int64_t)64 * ncol;
    float amax = 0.0f;
    // Columns j0 + step q (q < 8) of member zm, the loads of eight columns and
    // two units in flight (the addresses of columns past the rank are clamped,
    // their sums dropped); each sum runs over the units in order.
    auto columns = [&](const MRZMember &zm, int j0, int step) {
        const float *src[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + step * q < zm.rank ? j0 + step * q : zm.rank - 1;
            const int col = zm.vcol + j;
            src[q] = p.part + (zm.ubase + (int64_t)(col >> 6) * zm.nu) * ustride + (int64_t)(col & 63) * ncol + n;
        }
        float a[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        int i0 = 0;
        for (; i0 + 2 <= zm.nu; i0 += 2) {  // two units' loads, then their sums in order
            float t[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 8; ++q) t[u][q] = src[q][(int64_t)(i0 + u) * ustride];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 8; ++q) a[q] += t[u][q];
        }
        if (i0 < zm.nu)
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] += src[q][(int64_t)i0 * ustride];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + step * q;
            if (j < zm.rank) {
                float zsc = zm.scale;
                if constexpr (F::FP8) zsc = p.zcol[zm.col_off + j];  // s_j of U times s_j of V
                const float sj = a[q] * zsc;
                zs[zm.row + j][nn] = sj;
                amax = fmaxf(amax, fabsf(sj));
            }
        }
    };
    if (z.nmem == 1) {  // lane group g: columns g, g + 4, g + 8, ... of the block
        for (int j0 = g; j0 < zm0.rank; j0 += 32) columns(zm0, j0, 4);
    } else {  // lane group g: blocks g, g + 4, ... of the item, eight columns at a time
        for (int mi = z.m0 + g; mi < z.m0 + z.nmem; mi += 4) {
            const MRZMember zm = p.zmembers[mi];
            for (int j0 = 0; j0 < zm.rank; j0 += 8) columns(zm, j0, 1);
        }
    }
    amax = wave_max(amax);
    const float sig = F::SCALED ? col_scale(amax) : 1.0f;
    if (F::SCALED && lane == 0) p.sz[(int64_t)item * p.ntmax + nt] = sig;
    // the wave's LDS writes above precede its reads below: a wave's LDS operations run in order, so
    // only the compiler has to keep them so
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float inv = 1.0f / sig;
    const int nkb = (z.rows + KB - 1) / KB;
    for (int kb = 0; kb < nkb; ++kb) {
        float v[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int j = kb * KB + VW * g + e;
            v[e] = j < z.rows ? zs[j][nn] * inv : 0.0f;
        }
        F::storeB(p.zpack, z.zoff + (int64_t)kb * p.ntmax + nt, lane, v);
    }
}

// ---------------------------------------------------------------------------
// A chunk's step table held one entry per lane: lane l has the B offset (KiB)
// and the segment of step w0 + l; the following 64 steps are loaded when a
// window is entered and taken over when the next one is, so a step never
// waits on a load issued in it (a wait there would also drain the prefetched
// fragments). advance() is called with steps that grow by at most one.
struct StepWindow {
    int w0 = 0, bkib = 0, seg = 0, nb = 0, ns = 0;
    __device__ static inline int at(int st, int nsteps) { return st < nsteps ? st : nsteps - 1; }
    __device__ inline void init(const MRStep *steps, int nsteps, int lane) {
        const MRStep e = steps[at(lane, nsteps)];
        const MRStep f = steps[at(64 + lane, nsteps)];
        bkib = (int)(e.bofs >> 10);
        seg = e.lseg;
        nb = (int)(f.bofs >> 10);
        ns = f.lseg;
    }
    __device__ inline void advance(const MRStep *steps, int nsteps, int lane, int st) {
        if (st >= w0 + 64) {
            w0 += 64;
            bkib = nb;
            seg = ns;
            const MRStep f = steps[at(w0 + 64 + lane, nsteps)];
            nb = (int)(f.bofs >> 10);
            ns = f.lseg;
        }
    }
};

// ---------------------------------------------------------------------------
// Target side, one wave per row tile (<= 64 contiguous rows of a chunk): Y over
// the z of every ancestor block and over x of every source leaf, written once.
// ---------------------------------------------------------------------------
template <int STORE, int NT, bool LANE_SCALES>
__device__ inline void mr_tile(const DevPlanMR &p, int w, int lane, int k, float alpha, float beta,
                               float *__restrict__ y, int64_t ldy, uint32_t *lo_lds) {
    using F = MR<STORE>;
    const MRTile tl = cload(p.tiles, w);
    const MRChunk ch = cload(p.chunks, tl.chunk);
    const int nm = tl.nm;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0, 0, 0, 0};
    float scur[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) scur[t] = 1.0f;
    // A fragments are contiguous over the tile's steps; the chunk's step
    // table gives each step's B fragment (z of a block, or x of a source leaf).
    const MRStep *steps = p.ustep + ch.step_base;
    const float *drow = p.dscale + ch.dscale_base;  // the dense scale of each source leaf
    // LANE_SCALES (at most 64 segments): per lane j, segment j's n-tile scales,
    // its dense factor and kind; per lane l, step w0 + l of a window of 64
    // steps (its B offset in KiB and its segment). A step then reads them with
    // readlane: no scalar memory access on its path.
    float sv[NT];
    float fv = 1.0f;
    int vk = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) sv[t] = 1.0f;
    if (LANE_SCALES && lane < ch.nseg) {
        const MRSeg sg = p.segs[ch.seg_base + lane];  // per lane: vector loads
        const float *row = (sg.kind == 0 ? p.sz : p.sx) + (int64_t)sg.sidx * p.ntmax;
        vk = sg.kind;
        if (sg.kind == 1) fv = drow[sg.leaf];
        if (F::SCALED)  // the segment's scales with its dense factor folded in
#pragma unroll
            for (int t = 0; t < NT; ++t) sv[t] = row[t] * fv;
    }
    if constexpr (F::FP8) {  // the chunk's U lo-scales, 32 per z step, into this wave's LDS table
        const uint32_t *src = reinterpret_cast<const uint32_t *>(p.ulo + ch.ulo_base);
        for (int i = lane; i < ch.nzsteps * 16; i += 64) lo_lds[i] = src[i];
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
    // LANE_SCALES: the step table one entry per lane, 64 steps at a time, the
    // next 64 loaded a window ahead (so that using them waits for no recent load)
    StepWindow win;
    if constexpr (LANE_SCALES) win.init(steps, ch.nsteps, lane);
    auto info = [&](int st) {
        if constexpr (LANE_SCALES) {
            win.advance(steps, ch.nsteps, lane, st);
            const int seg = __builtin_amdgcn_readlane(win.seg, st - win.w0);
            return StepInfo{(int64_t)__builtin_amdgcn_readlane(win.bkib, st - win.w0) << 10, nullptr, 1.0f, seg,
                            __builtin_amdgcn_readlane(vk, seg), st * 32};
        } else {
            const MRStep e = cload(steps, st);
            return StepInfo{e.bofs, p.scales + (int64_t)e.srow * p.ntmax, e.sleaf >= 0 ? sload(drow, e.sleaf) : 1.0f,
                            0, e.sleaf >= 0 ? 1 : 0, st * 32};
        }
    };
    auto prep = [&](const typename F::A &a, int, const StepInfo &si) -> typename F::Op {
        if constexpr (F::FP8) {
            if (si.dense) return F::dense(a);
            // the 8 lo-scales of the lane's K indices of this step
            const h2 *q = reinterpret_cast<const h2 *>(lo_lds) + (si.lofs + 8 * (lane >> 4)) / 2;
            const h2 s2[4] = {q[0], q[1], q[2], q[3]};
            return F::hilo(a, s2);
        } else {
            return a;
        }
    };
    mfma_steps<STORE, NT, LANE_SCALES>(p.UD, p.zpack, tl.aoff, nm, ch.nsteps, lane, info, prep, acc, scur, sv,
                                       ch.nseg);
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

// ---------------------------------------------------------------------------
// The step loop of a workgroup of four waves that multiply one sequence of B
// fragments, each with its own A (row tiles of one chunk, or V units over the
// same chunks). B of every step is staged once in LDS for the workgroup
// instead of being read by every wave: two LDS slots (step s reads slot s & 1
// while B of step s + 1 is written to the other), one barrier per step, and B
// of step s + 3 loaded into registers (two staging sets) two steps before it
// is written. A wave without work (active false) takes part in the staging and
// the barriers, and loads some valid A it does not use: with every load
// unconditional and no exits inside a group of four steps, the wait counts
// stay exact and prefetched fragments are never drained.
// The scales are the common-scale scheme of mfma_steps: scur[t] is the n-tile's
// common scale, sv[t] (lane j) the scale of the j-th entry info(s).sidx points at.
// ring: 2 x NT x 16 x BFRAG bytes of LDS.
// ---------------------------------------------------------------------------
// Calls f(integral_constant<int, j>) for j = 0 .. N-1 (unrolled, j a constant).
template <int N, class Fn, int J = 0>
__device__ inline void static_for(Fn &&f) {
    if constexpr (J < N) {
        f(std::integral_constant<int, J>{});
        static_for<N, Fn, J + 1>(static_cast<Fn &&>(f));
    }
}

// Prefetch depths of the group step loop: KA steps of A fragments in
// registers, KS staging sets for B. The 16-bit forms from NT = 4 up use three
// and one, which keeps them within 256 registers at NT > 4 (two waves per
// SIMD) and within 168 at NT = 4 (three).
constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

template <int STORE, int NT>
struct GroupDepth {
    static constexpr bool lean = STORE != HMAT_STORE_FP32 && NT >= 4;
    static constexpr int KA = lean ? 3 : 4;
    static constexpr int KS = lean ? 1 : 2;
};

template <int STORE, int NT, class BOfs, class Info, class Prep>
__device__ inline void mfma_steps_group(const void *A, int64_t af0, int nm, const void *B, int nsteps, bool active,
                                        int tid, unsigned char *ring, BOfs bofs_of, Info info, Prep prep,
                                        f32x4 (&acc)[4][NT], const float (&scur)[NT], const float (&sv)[NT]) {
    using F = MR<STORE>;
    constexpr int KA = GroupDepth<STORE, NT>::KA, KS = GroupDepth<STORE, NT>::KS;
    constexpr int U = KA * KS / cgcd(KA, KS);  // lcm(KA, KS)
    constexpr int kUnits = NT * F::BFRAG;  // 16-byte pieces of one step's B
    constexpr int kSlot = kUnits * 16;
    constexpr int kPer = (kUnits + 255) / 256;
    const int lane = tid & 63;
    auto clamp = [&](int st) { return st < nsteps ? st : nsteps - 1; };
    auto scale_of = [&](const StepInfo &i, int t) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sv[t]), i.sidx));
    };
    const rsrc_t ra = make_rsrc(static_cast<const char *>(A) + af0 * 1024);
    typename F::A a[KA][4];
    u32x4 g[KS][kPer];
    auto load_a = [&](typename F::A(&as)[4], int st) {
        const int sc = clamp(st);
#pragma unroll
        for (int m = 0; m < 4; ++m) as[m] = F::loadA(ra, (sc * nm + (m < nm ? m : nm - 1)) * 1024, lane);
    };
    auto gload = [&](u32x4(&gs)[kPer], int st) {  // this thread's pieces of B(st), clamped to the last step
        const rsrc_t rb = make_rsrc(static_cast<const char *>(B) + bofs_of(clamp(st)));
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = tid + 256 * i;
            gs[i] = __builtin_bit_cast(
                u32x4, buf16<0>(rb, (kUnits % 256 == 0 ? u : (u < kUnits ? u : kUnits - 1)) * 16, 0));
        }
    };
    auto swrite = [&](const u32x4(&gs)[kPer], int slot) {
        u32x4 *dst = reinterpret_cast<u32x4 *>(ring + slot * kSlot);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = tid + 256 * i;
            if (kUnits % 256 == 0 || u < kUnits) dst[u] = gs[i];
        }
    };
    StepInfo ic = info(0), in_;
    // step st: A from set st % KA, B from slot st & 1; B(st + 1) goes from staging
    // set (st + 1) % KS into the other slot, and the set is refilled with B(st + 1 + KS)
    auto step = [&](auto JA, auto JG, int st) {
        constexpr int ja = decltype(JA)::value, jg = decltype(JG)::value;
        swrite(g[jg], (st + 1) & 1);
        gload(g[jg], st + 1 + KS);
        in_ = info(clamp(st + 1));
        if (active) {
            typename F::Op op[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) op[m] = prep(a[ja][m], m, ic);
            const unsigned char *slot = ring + (st & 1) * kSlot;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                typename F::B b;
                if constexpr (STORE == HMAT_STORE_FP32) {
                    b.v = *reinterpret_cast<const f32x4 *>(slot + t * 16 * F::BFRAG + lane * 16);
                } else {
                    b.hi = *reinterpret_cast<const decltype(b.hi) *>(slot + t * 16 * F::BFRAG + lane * 16);
                    b.lo = *reinterpret_cast<const decltype(b.lo) *>(slot + t * 16 * F::BFRAG + 1024 + lane * 16);
                }
                if constexpr (F::SCALED) {  // this step's scale over the common one: a power of two <= 1
                    const float f = scale_of(ic, t) * __builtin_amdgcn_rcpf(scur[t]);
                    if (f != 1.0f) scale_b(b, f);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    if (m < nm) F::mma(op[m], b, acc[m][t]);
            }
        }
        load_a(a[ja], st + KA);
        ic = in_;
        __syncthreads();  // slot st & 1 is free again; B(st + 1) is visible to every wave
    };
    gload(g[0], 0);
    swrite(g[0], 0);
    static_for<KS>([&](auto J) { gload(g[(decltype(J)::value + 1) % KS], decltype(J)::value + 1); });
    static_for<KA>([&](auto J) { load_a(a[decltype(J)::value], decltype(J)::value); });
    __syncthreads();
    int st = 0;  // whole groups of U steps without exits, then the remaining ones
    for (; st + U <= nsteps; st += U)
        static_for<U>([&](auto J) {
            constexpr int j = decltype(J)::value;
            step(std::integral_constant<int, j % KA>{}, std::integral_constant<int, (j + 1) % KS>{}, st + j);
        });
    static_for<U - 1>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if (st + j < nsteps)
            step(std::integral_constant<int, j % KA>{}, std::integral_constant<int, (j + 1) % KS>{}, st + j);
    });
}

// ---------------------------------------------------------------------------
// Target side, one workgroup of four waves per tile group (up to four row
// tiles of one chunk, which multiply the same B sequence): mfma_steps_group
// over the chunk's step table, copied into LDS once so that no step waits on
// a global load other than its fragments. The segment scales are held one per
// lane (at most 64 segments per chunk).
// stab: nsteps entries of LDS; lo_lds (FP8 forms): 16 x nzsteps words per wave.
// ---------------------------------------------------------------------------
template <int STORE, int NT>
__device__ inline void mr_tile_group(const DevPlanMR &p, int g, int k, float alpha, float beta,
                                     float *__restrict__ y, int64_t ldy, unsigned char *ring, int2 *stab,
                                     uint32_t *lo_lds) {
    using F = MR<STORE>;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const MRTileGroup tg = cload(p.tgroups, g);
    const bool active = wave < tg.ntiles;
    const MRTile tl = cload(p.tiles, tg.tile0 + (active ? wave : 0));
    const MRChunk ch = cload(p.chunks, tg.chunk);
    const int nm = tl.nm, nsteps = ch.nsteps;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0, 0, 0, 0};
    float scur[NT], sv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) scur[t] = sv[t] = 1.0f;
    const MRStep *steps = p.ustep + ch.step_base;
    const float *drow = p.dscale + ch.dscale_base;
    float fv = 1.0f;
    int vk = 0;
    if (lane < ch.nseg) {  // per lane j: segment j's n-tile scales (dense factor folded in) and kind
        const MRSeg sg = p.segs[ch.seg_base + lane];
        const float *row = (sg.kind == 0 ? p.sz : p.sx) + (int64_t)sg.sidx * p.ntmax;
        vk = sg.kind;
        if (sg.kind == 1) fv = drow[sg.leaf];
        if (F::SCALED)
#pragma unroll
            for (int t = 0; t < NT; ++t) sv[t] = row[t] * fv;
    }
    if (F::SCALED)
#pragma unroll
        for (int t = 0; t < NT; ++t)
            scur[t] = __builtin_bit_cast(
                float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, lanes_max(sv[t], lane, ch.nseg))));
    if constexpr (F::FP8) {  // the chunk's U lo-scales, into this wave's LDS table
        const uint32_t *src = reinterpret_cast<const uint32_t *>(p.ulo + ch.ulo_base);
        for (int i = lane; i < ch.nzsteps * 16; i += 64) lo_lds[i] = src[i];
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
    for (int i = tid; i < nsteps; i += 256) {  // step table: B offset in KiB, segment
        const MRStep e = steps[i];
        stab[i] = int2{(int)(e.bofs >> 10), e.lseg};
    }
    __syncthreads();
    auto bofs_of = [&](int st) -> int64_t { return (int64_t)__builtin_amdgcn_readfirstlane(stab[st].x) << 10; };
    auto info = [&](int st) {
        const int seg = __builtin_amdgcn_readfirstlane(stab[st].y);
        return StepInfo{0, nullptr, 1.0f, seg, __builtin_amdgcn_readlane(vk, seg), st * 32};
    };
    auto prep = [&](const typename F::A &a, int, const StepInfo &si) -> typename F::Op {
        if constexpr (F::FP8) {
            if (si.dense) return F::dense(a);
            const h2 *q = reinterpret_cast<const h2 *>(lo_lds) + (si.lofs + 8 * (lane >> 4)) / 2;
            const h2 s2[4] = {q[0], q[1], q[2], q[3]};
            return F::hilo(a, s2);
        } else {
            return a;
        }
    };
    mfma_steps_group<STORE, NT>(p.UD, tl.aoff, nm, p.zpack, nsteps, active, tid, ring, bofs_of, info, prep, acc,
                                scur, sv);
    if (!active) return;
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

// ---------------------------------------------------------------------------
// Source side, one workgroup of four waves per unit group (up to four V units
// over the same chunks, which multiply the same X fragments): mfma_steps_group
// with the X fragments of the chunks as B: each wave writes its unit's 64
// partial sums per right-hand side column.
// ---------------------------------------------------------------------------
template <int STORE, int NT>
__device__ inline void mr_vunit_group(const DevPlanMR &p, int g, unsigned char *ring) {
    using F = MR<STORE>;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const MRUnitGroup ug = cload(p.ugroups, g);
    const bool active = wave < ug.count;
    const MRVUnit u = cload(p.vunits, ug.u0 + (active ? wave : 0));
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0, 0, 0, 0};
    float scur[NT], sv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) scur[t] = sv[t] = 1.0f;
    int nsteps = 0;
    for (int c = u.c0; c < u.c0 + u.nc; ++c) nsteps += cload(p.chunks, c).nkb;
    int vn = 0;  // lane j: K-blocks of the unit's chunk j
    if (lane < u.nc) {
        vn = p.chunks[u.c0 + lane].nkb;
        if (F::SCALED)
#pragma unroll
            for (int t = 0; t < NT; ++t) sv[t] = p.sx[(int64_t)(u.c0 + lane) * p.ntmax + t];
    }
    if (F::SCALED)
#pragma unroll
        for (int t = 0; t < NT; ++t)
            scur[t] = __builtin_bit_cast(
                float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, lanes_max(sv[t], lane, u.nc))));
    h2 vl[4];  // FP8 forms: lo-scale of the lane's V column in each m-subtile, twice
    if constexpr (F::FP8) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const _Float16 sl = __builtin_bit_cast(_Float16, p.vlo[(int64_t)u.lo_off * 64 + 16 * m + (lane & 15)]);
            vl[m] = h2{sl, sl};
        }
    }
    auto prep = [&](const typename F::A &a, int m, const StepInfo &) -> typename F::Op {
        if constexpr (F::FP8) {
            const h2 s2[4] = {vl[m], vl[m], vl[m], vl[m]};
            return F::hilo(a, s2);
        } else {
            return a;
        }
    };
    const int64_t b0 = cload(p.chunks, u.c0).xoff, ntm = p.ntmax;
    constexpr int64_t bbytes = 16 * F::BFRAG;
    auto bofs_of = [&](int st) -> int64_t { return (b0 + (int64_t)st * ntm) * bbytes; };
    int c = 0, cend = 0;  // chunk (index in the unit) of the step asked for last, and the step where it ends
    cend = __builtin_amdgcn_readlane(vn, 0);
    auto info = [&](int st) {
        while (st >= cend) {
            ++c;
            cend += __builtin_amdgcn_readlane(vn, c);
        }
        return StepInfo{0, nullptr, 1.0f, c, 0, 0};
    };
    mfma_steps_group<STORE, NT>(p.V, u.aoff, u.nm, p.xpack, nsteps, active, tid, ring, bofs_of, info, prep, acc,
                                scur, sv);
    if (!active) return;
    const int ncol = p.ntmax * 16;
    float *out = p.part + u.poff;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[(int64_t)(16 * m + 4 * (lane >> 4) + i) * ncol + t * 16 + (lane & 15)] = acc[m][t][i] * scur[t];
}

}  // namespace dev
}  // namespace hmat
