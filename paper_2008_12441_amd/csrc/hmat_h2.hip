// HIP kernels (gfx950) of the H^2-matrix-vector product, one right-hand side.
//
// One product runs as up to 2 (L - 2) + 2 launches on the caller's stream:
//   k_h2_upward   one workgroup per chunk: x^ of each leaf (V_t^T x_t, lanes
//                 own rows, columns reduced across the wave), then the
//                 chunk's x^ = sum over its leaves of F_c^T x^_c;
//   k_h2_up       one wave per node, a level at a time upward from depth
//                 L - 2: x^_t = sum over its children of F_c^T x^_c;
//   k_h2_down     one wave per node, a level at a time downward from depth 1:
//                 y^_t = E_t y^_parent + sum over its couplings of S_ts x^_s;
//   k_h2_leaf     one workgroup per chunk: the chunk's y^ (as k_h2_down), each
//                 leaf's y^ = E_c y^_chunk, then every row y_i = U_t(i, :) y^_t
//                 + sum over its dense blocks of D_ts(i, :) x_s, written once.
// The leaf kernels stream the big arrays (leaf bases, dense blocks) from HBM
// with one contiguous 1 KiB per wave-load; the level kernels move the small
// transfer and coupling matrices and are bound by latency.
#include "hmat_sv_device.h"
#include "hmat_h2_internal.h"

namespace hmat {
namespace {

using namespace hmat::dev;

template <int STORE>
struct SmallOf {
    using T = float;
};
template <>
struct SmallOf<HMAT_STORE_FP16_SCALED> {
    using T = _Float16;
};

// One exchange of the butterfly below: the live columns are p[0..2H); lanes
// whose bit o is set keep the upper half and send the lower one, the others
// the reverse, and each adds what its partner (lane ^ o) sent. All indices
// are compile-time constants, so p stays in registers.
template <int K, int H>
__device__ inline void reduce_scatter_step(float (&p)[K], int lane) {
    if constexpr (H >= 1) {
        constexpr int o = 64 * H / K;
        const bool upper = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float keep = upper ? p[H + i] : p[i];
            const float send = upper ? p[i] : p[H + i];
            p[i] = keep + __shfl_xor(send, o, 64);
        }
        reduce_scatter_step<K, H / 2>(p, lane);
    }
}

// Sum over the 64 lanes of p[0..K) (K a power of two <= 64): a butterfly that
// halves the live columns at every exchange. On return lane l holds the sum
// of column l / (64 / K) over all lanes.
template <int K>
__device__ inline float lane_reduce_scatter(float (&p)[K], int lane) {
    reduce_scatter_step<K, K / 2>(p, lane);
    float s = p[0];
#pragma unroll
    for (int o = 32 / K; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// Entry j of a vector held one entry per lane (lane j), as a uniform value.
__device__ inline float lane_value(float v, int j) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}

template <class S>
struct SmallVec {
    using V = f32x4;
    static constexpr int W = 4;
};
template <>
struct SmallVec<_Float16> {
    using V = f16x8;
    static constexpr int W = 8;
};

// (M w)[lane] for a small matrix stored by rows: row `lane` of M at m + lane * ldm
// (16-byte aligned, zero past its cols <= 64 entries); lane j holds w[j]. Each
// lane reads its row in 16-byte loads, all in flight together.
template <class S>
__device__ inline float small_gemv(const S *__restrict__ m, int ldm, int cols, float w, int lane) {
    using SV = SmallVec<S>;
    constexpr int W = SV::W, NQ = 64 / W;
    const typename SV::V *row = reinterpret_cast<const typename SV::V *>(m + (int64_t)lane * ldm);
    typename SV::V v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q * W < cols) v[q] = row[q];
    float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q * W < cols) {
#pragma unroll
            for (int e = 0; e < W; e += 2) {
                a0 = fma((float)v[q][e], lane_value(w, q * W + e), a0);
                a1 = fma((float)v[q][e + 1], lane_value(w, q * W + e + 1), a1);
            }
        }
    return a0 + a1;
}

// One term of a node's x^ or y^: the vector w (cols entries of the workspace)
// read one entry per lane, then scale * (M w) for lane < rows (0 elsewhere).
template <class S>
__device__ inline float term_product(const DevPlanH2 &p, const H2Term &t, int rows, int lane) {
    const float *w = p.ws + t.src + (t.y_from ? p.ws_half : 0);
    const float wv = lane < t.cols ? w[lane] : 0.0f;
    float r = 0.0f;
    if (lane < rows) r = small_gemv(static_cast<const S *>(p.small) + t.m_off, t.ldm, t.cols, wv, lane) * t.scale;
    return r;
}

// sum_{q in [q0, q1)} <row's VW-vector q, vec[(q - q0) * VW ...]> for one lane's row.
template <int STORE>
__device__ inline float dot_span(const typename Form<STORE>::Vec *base, const float *vec, int q0, int q1) {
    using F = Form<STORE>;
    constexpr int VW = F::VW;
    float a[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) a[e] = 0.0f;
    int q = q0;
    for (; q + kUUnroll <= q1; q += kUUnroll) {
        float v[kUUnroll][VW];
#pragma unroll
        for (int u = 0; u < kUUnroll; ++u) F::load(base + (int64_t)(q + u) * kWave, v[u]);
#pragma unroll
        for (int u = 0; u < kUUnroll; ++u)
#pragma unroll
            for (int e = 0; e < VW; ++e) a[e] = fma(v[u][e], vec[(q + u - q0) * VW + e], a[e]);
    }
    for (; q < q1; ++q) {
        float v[VW];
        F::load(base + (int64_t)q * kWave, v);
#pragma unroll
        for (int e = 0; e < VW; ++e) a[e] = fma(v[e], vec[(q - q0) * VW + e], a[e]);
    }
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < VW; ++e) s += a[e];
    return s;
}

// ---------------------------------------------------------------------------
// Upward pass at the chunks: every leaf's x^ = V_t^T x_t (lane = row, the
// columns summed across the wave), times F_c^T into the chunk's x^ straight
// from the lanes that hold it. K: the leaf ranks rounded up to a power of
// two (>= VW). The chunks are at depth >= 1, so they have bases.
// ---------------------------------------------------------------------------
template <int STORE, int K>
__global__ __launch_bounds__(256) void k_h2_upward(DevPlanH2 p, const float *__restrict__ x) {
    using F = Form<STORE>;
    using S = typename SmallOf<STORE>::T;
    constexpr int VW = F::VW;
    static_assert(K >= VW && K <= 64 && (K & (K - 1)) == 0, "K: a power of two in [VW, 64]");
    __shared__ float red[256];  // per-wave partial sums of the chunk's x^
    const H2Chunk ch = cload(p.chunks, blockIdx.x);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    float part = 0.0f;
    for (int li = wave; li < ch.nleaf; li += 4) {
        const H2Leaf lf = cload(p.leaves, ch.leaf_base + li);
        float acc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = 0.0f;
        const int ntile = (lf.rows + kWave - 1) / kWave;
        for (int tile = 0; tile < ntile; ++tile) {
            const int row = tile * kWave + lane;
            const float xi = row < lf.rows ? x[lf.row_begin + row] : 0.0f;
            const typename F::Vec *base =
                reinterpret_cast<const typename F::Vec *>(static_cast<const typename F::Elem *>(p.V) + lf.v_off) +
                (int64_t)tile * lf.kq * kWave + lane;
#pragma unroll
            for (int q = 0; q < K / VW; ++q) {
                if (q < lf.kq) {
                    float v[VW];
                    F::load(base + (int64_t)q * kWave, v);
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[q * VW + e] = fma(v[e], xi, acc[q * VW + e]);
                }
            }
        }
        // column i of V^T x ends in lanes i * (64 / K) ...; the leaf's x^ is that times its V scale
        const float s = lane_reduce_scatter<K>(acc, lane);
        // lane j's row of F^T in 16-byte loads, all in flight at once
        using SV = SmallVec<S>;
        constexpr int W = SV::W;
        typename SV::V fv[K / W > 0 ? K / W : 1];
        const typename SV::V *ft =
            reinterpret_cast<const typename SV::V *>(static_cast<const S *>(p.small) + lf.ft_off + (int64_t)lane * lf.ft_ld);
#pragma unroll
        for (int q = 0; q * W < K; ++q)
            if (lane < ch.k && q * W < lf.k) fv[q] = ft[q];
            else fv[q] = typename SV::V{};
        float c0 = 0.0f, c1 = 0.0f;
#pragma unroll
        for (int i = 0; i < K; i += 2) {
            c0 = fma((float)fv[i / W][i % W], lane_value(s, i * (64 / K)), c0);
            c1 = fma((float)fv[(i + 1) / W][(i + 1) % W], lane_value(s, (i + 1) * (64 / K)), c1);
        }
        part = fma(c0 + c1, lf.sv * lf.sf, part);
    }
    red[tid] = part;
    __syncthreads();
    if (wave == 0 && lane < ch.k) p.ws[ch.xh + lane] = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
}

// Upward pass above the chunks, one level: one wave per node, lane = output
// index: x^_t = sum over its children of F_c^T x^_c.
template <int STORE>
__global__ __launch_bounds__(256) void k_h2_up(DevPlanH2 p, int first, int count) {
    using S = typename SmallOf<STORE>::T;
    const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= count) return;
    const int lane = threadIdx.x & 63;
    const H2Node nd = cload(p.nodes, first + w);
    float acc = 0.0f;
    for (int u = 0; u < nd.nup; ++u) acc += term_product<S>(p, cload(p.terms, nd.up_base + u), nd.k, lane);
    if (lane < nd.k) p.ws[nd.xh + lane] = acc;
}

// Downward pass, one level: one wave per node, lane = output index:
// y^_t = E_t y^_parent + sum over its couplings of S_ts x^_s.
template <int STORE>
__global__ __launch_bounds__(256) void k_h2_down(DevPlanH2 p, int first, int count) {
    using S = typename SmallOf<STORE>::T;
    const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= count) return;
    const int lane = threadIdx.x & 63;
    const H2Node nd = cload(p.nodes, first + w);
    float acc = 0.0f;
    for (int u = 0; u < nd.nterm; ++u) acc += term_product<S>(p, cload(p.terms, nd.term_base + u), nd.k, lane);
    if (lane < nd.k) p.ws[p.ws_half + nd.xh + lane] = acc;
}

// ---------------------------------------------------------------------------
// Leaf kernel: per chunk, its y^, its leaves' y^, then y for its rows.
// ---------------------------------------------------------------------------
template <int STORE>
__global__ __launch_bounds__(256) void k_h2_leaf(DevPlanH2 p, const float *__restrict__ x, float *__restrict__ y,
                                                 float alpha, float beta) {
    using F = Form<STORE>;
    using S = typename SmallOf<STORE>::T;
    constexpr int VW = F::VW;
    extern __shared__ __align__(16) float lds[];
    const H2Chunk ch = cload(p.chunks, blockIdx.x);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ku = ch.nq_u * VW;        // padded width of a leaf's y^
    float *red = lds;                   // [4][64]
    float *yc = lds + 256;              // [64]: the chunk's y^
    float *yl = lds + 320;              // [nleaf][ku]: each leaf's y^, times its U scale
    float *vec = yl + ch.nleaf * ku;    // x over the dense source leaves, each padded to VW
    if (ch.k > 0) {
        float part = 0.0f;
        for (int u = wave; u < ch.nterm; u += 4) part += term_product<S>(p, cload(p.terms, ch.term_base + u), ch.k, lane);
        red[tid] = part;
    }
    int pos = 0;
    for (int s = 0; s < ch.nsrc; ++s) {
        const DSeg ds = cload(p.dsegs, ch.dseg_base + s);
        for (int j = tid; j < ds.nq * VW; j += 256) vec[pos + j] = j < ds.rows ? x[ds.row_begin + j] : 0.0f;
        pos += ds.nq * VW;
    }
    __syncthreads();
    if (wave == 0) yc[lane] = ch.k > 0 && lane < ch.k ? (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])
                                                     : 0.0f;
    __syncthreads();
    const float ycv = yc[lane];
    for (int li = wave; li < ch.nleaf; li += 4) {
        const H2Leaf lf = cload(p.leaves, ch.leaf_base + li);
        float s = 0.0f;
        if (ch.k > 0 && lane < lf.k)
            s = small_gemv(static_cast<const S *>(p.small) + lf.e_off, lf.e_ld, ch.k, ycv, lane) * (lf.se * lf.su);
        if (lane < ku) yl[li * ku + lane] = s;
    }
    __syncthreads();
    const int ntile = (ch.rows + kWave - 1) / kWave;
    for (int tile = wave; tile < ntile; tile += 4) {
        const typename F::Vec *base =
            reinterpret_cast<const typename F::Vec *>(static_cast<const typename F::Elem *>(p.UD) + ch.ud_off) +
            (int64_t)tile * ch.nq * kWave + lane;
        const int row = tile * kWave + lane;
        int li = 0;  // the row's leaf
        while (li + 1 < ch.nleaf && ch.row_begin + row >= cload(p.leaves, ch.leaf_base + li + 1).row_begin) ++li;
        float acc = ch.nq_u > 0 ? dot_span<STORE>(base, yl + li * ku, 0, ch.nq_u) : 0.0f;
        int q = ch.nq_u, vq = 0;
        for (int s = 0; s < ch.nsrc; ++s) {
            const int nq = cload(p.dsegs, ch.dseg_base + s).nq;
            const float part = dot_span<STORE>(base, vec + vq * VW, q, q + nq);
            if (STORE == HMAT_STORE_FP16_SCALED)
                acc = fma(cload(p.dscale, ch.dscale_base + li * ch.nsrc + s), part, acc);
            else
                acc += part;
            q += nq;
            vq += nq;
        }
        if (row < ch.rows) {
            float *yp = y + ch.row_begin + row;
            float v = alpha * acc;
            if (beta != 0.0f) v = fma(beta, *yp, v);
            *yp = v;
        }
    }
}

template <int STORE>
void launch_upward_store(const DevPlanH2 &p, const float *x, hipStream_t st) {
    const dim3 g(p.num_chunks), b(256);
    int kp = Form<STORE>::VW;
    while (kp < p.kmax) kp *= 2;
    switch (kp) {
        case 4:
            if constexpr (Form<STORE>::VW <= 4) hipLaunchKernelGGL((k_h2_upward<STORE, 4>), g, b, 0, st, p, x);
            break;
        case 8: hipLaunchKernelGGL((k_h2_upward<STORE, 8>), g, b, 0, st, p, x); break;
        case 16: hipLaunchKernelGGL((k_h2_upward<STORE, 16>), g, b, 0, st, p, x); break;
        case 32: hipLaunchKernelGGL((k_h2_upward<STORE, 32>), g, b, 0, st, p, x); break;
        default: hipLaunchKernelGGL((k_h2_upward<STORE, 64>), g, b, 0, st, p, x); break;
    }
}

}  // namespace

int launch_h2_upward(const DevPlanH2 &p, const float *x, void *stream) {
    if (p.storage == HMAT_STORE_FP16_SCALED)
        launch_upward_store<HMAT_STORE_FP16_SCALED>(p, x, (hipStream_t)stream);
    else
        launch_upward_store<HMAT_STORE_FP32>(p, x, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_h2_up(const DevPlanH2 &p, int32_t first, int32_t count, void *stream) {
    const dim3 g((count + 3) / 4), b(256);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_h2_up<HMAT_STORE_FP16_SCALED>), g, b, 0, (hipStream_t)stream, p, first, count);
    else
        hipLaunchKernelGGL((k_h2_up<HMAT_STORE_FP32>), g, b, 0, (hipStream_t)stream, p, first, count);
    return (int)hipGetLastError();
}

int launch_h2_down(const DevPlanH2 &p, int32_t first, int32_t count, void *stream) {
    const dim3 g((count + 3) / 4), b(256);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_h2_down<HMAT_STORE_FP16_SCALED>), g, b, 0, (hipStream_t)stream, p, first, count);
    else
        hipLaunchKernelGGL((k_h2_down<HMAT_STORE_FP32>), g, b, 0, (hipStream_t)stream, p, first, count);
    return (int)hipGetLastError();
}

int launch_h2_leaf(const DevPlanH2 &p, const float *x, float *y, float alpha, float beta, void *stream) {
    const size_t lds = (size_t)p.lds_b_floats * sizeof(float);
    const dim3 g(p.num_chunks), b(256);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_h2_leaf<HMAT_STORE_FP16_SCALED>), g, b, lds, (hipStream_t)stream, p, x, y, alpha, beta);
    else
        hipLaunchKernelGGL((k_h2_leaf<HMAT_STORE_FP32>), g, b, lds, (hipStream_t)stream, p, x, y, alpha, beta);
    return (int)hipGetLastError();
}

}  // namespace hmat
