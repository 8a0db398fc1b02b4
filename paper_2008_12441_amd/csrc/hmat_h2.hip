// HIP kernels (gfx950) of the H^2-matrix-vector product, one right-hand side.
//
// One product runs as up to 2 (L - 2) + 2 launches on the caller's stream:
//   k_h2_upleaf   one workgroup per chunk: x^ of each leaf (V_t^T x_t, lanes
//                 own rows, columns reduced across the wave), then the
//                 chunk's x^ = sum over its leaves of F_c^T x^_c;
//   k_h2_up       one wave per node, a level at a time upward from depth
//                 L - 2: x^_t = sum over children of F_c^T x^_c;
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

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Sum over the 64 lanes of p[0..K) (K a power of two <= 64): a butterfly that
// halves the live columns at every exchange. On return lane l holds the sum
// of column l >> (6 - log2 K) over all lanes.
template <int K>
__device__ inline float lane_reduce_scatter(float (&p)[K], int lane) {
#pragma unroll
    for (int h = K / 2, o = 32; h >= 1; h >>= 1, o >>= 1) {
        const bool upper = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const float keep = upper ? p[h + i] : p[i];
            const float send = upper ? p[i] : p[h + i];
            p[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    float s = p[0];
#pragma unroll
    for (int o = 32 / K; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// s * (M w) for lane = row index of M (rows x cols, column-major, rows = ld),
// w read from `w` (uniform across the wave).
template <class S>
__device__ inline float small_gemv_row(const S *__restrict__ m, int rows, int cols, const float *w, int lane) {
    float s = 0.0f;
    for (int j = 0; j < cols; ++j) s = fma((float)m[lane + j * rows], w[j], s);
    return s;
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
// Upward pass at the leaves: per chunk, every leaf's x^ = V_t^T x_t, then the
// chunk's x^. K: the leaf ranks rounded up to a power of two (>= VW).
// ---------------------------------------------------------------------------
template <int STORE, int K>
__global__ __launch_bounds__(256) void k_h2_upleaf(DevPlanH2 p, const float *__restrict__ x) {
    using F = Form<STORE>;
    using S = typename SmallOf<STORE>::T;
    constexpr int VW = F::VW;
    static_assert(K >= VW && K <= 64 && (K & (K - 1)) == 0, "K: a power of two in [VW, 64]");
    extern __shared__ __align__(16) float lds[];
    const H2Chunk ch = cload(p.chunks, blockIdx.x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *xl = lds;                  // [nleaf][64]: x^ of each leaf
    float *red = lds + ch.nleaf * 64; // [4][64]: per-wave partial sums of the chunk's x^
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
        const float s = lane_reduce_scatter<K>(acc, lane);
        const int j = lane >> (6 - ilog2(K));
        if ((lane & (64 / K - 1)) == 0 && j < lf.k) xl[li * 64 + j] = s * lf.sv;
    }
    __syncthreads();
    if (ch.k == 0) return;
    float part = 0.0f;
    if (lane < ch.k)
        for (int li = wave; li < ch.nleaf; li += 4) {
            const H2Leaf lf = cload(p.leaves, ch.leaf_base + li);
            const float s = small_gemv_row(static_cast<const S *>(p.small) + lf.ft_off, ch.k, lf.k, xl + li * 64, lane);
            part = fma(s, lf.sf, part);
        }
    red[wave * 64 + lane] = part;
    __syncthreads();
    if (wave == 0 && lane < ch.k) p.ws[ch.xh + lane] = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
}

// One wave per node; lane = output index. up: x^_t from the children's x^;
// down: y^_t from y^_parent and the couplings' x^.
template <int STORE, bool UP>
__global__ __launch_bounds__(256) void k_h2_level(DevPlanH2 p, int first, int count) {
    using S = typename SmallOf<STORE>::T;
    const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= count) return;
    const int lane = threadIdx.x & 63;
    const H2Node nd = cload(p.nodes, first + w);
    if (lane >= nd.k) return;
    const int tb = UP ? nd.up_base : nd.term_base, nt = UP ? nd.nup : nd.nterm;
    float acc = 0.0f;
    for (int u = 0; u < nt; ++u) {
        const H2Term t = cload(p.terms, tb + u);
        const float *w = p.ws + t.src + (t.y_from ? p.ws_half : 0);
        acc = fma(small_gemv_row(static_cast<const S *>(p.small) + t.m_off, nd.k, t.cols, w, lane), t.scale, acc);
    }
    p.ws[nd.xh + (UP ? 0 : p.ws_half) + lane] = acc;
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
        if (lane < ch.k)
            for (int u = wave; u < ch.nterm; u += 4) {
                const H2Term t = cload(p.terms, ch.term_base + u);
                const float *w = p.ws + t.src + (t.y_from ? p.ws_half : 0);
                part = fma(small_gemv_row(static_cast<const S *>(p.small) + t.m_off, ch.k, t.cols, w, lane), t.scale,
                           part);
            }
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
    for (int li = wave; li < ch.nleaf; li += 4) {
        const H2Leaf lf = cload(p.leaves, ch.leaf_base + li);
        for (int i = lane; i < ku; i += kWave) {
            float s = 0.0f;
            if (ch.k > 0 && i < lf.k)
                s = small_gemv_row(static_cast<const S *>(p.small) + lf.e_off, lf.k, ch.k, yc, i) * (lf.se * lf.su);
            yl[li * ku + i] = s;
        }
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
void launch_upleaf_store(const DevPlanH2 &p, const float *x, hipStream_t st) {
    const size_t lds = (size_t)p.lds_a_floats * sizeof(float);
    const dim3 g(p.num_chunks), b(256);
    int kp = Form<STORE>::VW;
    while (kp < p.kmax) kp *= 2;
    switch (kp) {
        case 4:
            if constexpr (Form<STORE>::VW <= 4) hipLaunchKernelGGL((k_h2_upleaf<STORE, 4>), g, b, lds, st, p, x);
            break;
        case 8: hipLaunchKernelGGL((k_h2_upleaf<STORE, 8>), g, b, lds, st, p, x); break;
        case 16: hipLaunchKernelGGL((k_h2_upleaf<STORE, 16>), g, b, lds, st, p, x); break;
        case 32: hipLaunchKernelGGL((k_h2_upleaf<STORE, 32>), g, b, lds, st, p, x); break;
        default: hipLaunchKernelGGL((k_h2_upleaf<STORE, 64>), g, b, lds, st, p, x); break;
    }
}

}  // namespace

int launch_h2_upleaf(const DevPlanH2 &p, const float *x, void *stream) {
    if (p.storage == HMAT_STORE_FP16_SCALED)
        launch_upleaf_store<HMAT_STORE_FP16_SCALED>(p, x, (hipStream_t)stream);
    else
        launch_upleaf_store<HMAT_STORE_FP32>(p, x, (hipStream_t)stream);
    return (int)hipGetLastError();
}

int launch_h2_up(const DevPlanH2 &p, int32_t first, int32_t count, void *stream) {
    const dim3 g((count + 3) / 4), b(256);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_h2_level<HMAT_STORE_FP16_SCALED, true>), g, b, 0, (hipStream_t)stream, p, first, count);
    else
        hipLaunchKernelGGL((k_h2_level<HMAT_STORE_FP32, true>), g, b, 0, (hipStream_t)stream, p, first, count);
    return (int)hipGetLastError();
}

int launch_h2_down(const DevPlanH2 &p, int32_t first, int32_t count, void *stream) {
    const dim3 g((count + 3) / 4), b(256);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_h2_level<HMAT_STORE_FP16_SCALED, false>), g, b, 0, (hipStream_t)stream, p, first, count);
    else
        hipLaunchKernelGGL((k_h2_level<HMAT_STORE_FP32, false>), g, b, 0, (hipStream_t)stream, p, first, count);
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
