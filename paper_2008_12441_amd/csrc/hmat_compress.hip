// HIP kernels (gfx950) of the factor construction (hmat_compress).
//
// Dense blocks are the kernel entries themselves. A low-rank block is
// compressed by a randomized SVD whose kernel entries are generated on the fly
// from the points and never stored:
//   k_csample (mode 0)  Y = K_ts Omega on MFMA, the entries generated in the A
//                       fragments, the source points and their Rademacher rows
//                       staged through LDS;
//   k_cgram, k_ceig, k_capply (twice)  Q from Y: the FP64 Gram matrix Y^T Y,
//                       its Jacobi eigen-decomposition P D P^T, and
//                       Y <- Y P D^(-1/2) (directions with D below a relative
//                       floor dropped); the second pass makes the columns
//                       orthonormal to working precision (the SVQB scheme of
//                       Stathopoulos and Wu, SIAM J. Sci. Comput. 23, 2002);
//   k_csample (mode 1)  B^T = K_st Q on MFMA over the rows of s;
//   k_cgram, k_ceig     B B^T = (B^T)^T B^T = W L W^T; the leading r pairs give
//                       M_U = W_r L_r^(1/4) and M_V = W_r L_r^(-1/4);
//   k_capply            U = Q M_U, V = B^T M_V, so that U V^T = Q W_r W_r^T B,
//                       the rank-r truncation of Q B (Algorithm 5.1 of Halko,
//                       Martinsson and Tropp).
// Entries are FP32 and enter the sample products as exact three-part BF16
// splits with FP32 accumulation; Gram matrices, rotations and the eigenvalue
// arithmetic are FP64.
#include <hip/hip_runtime.h>

#include "hmat.h"
#include "hmat_compress.h"

namespace hmat {
namespace {

constexpr int kOther = 64;  // other-side points per LDS tile of the sample products

// Kernel function of Eq. (2.1) from the squared distance:
// -log(d) / (2 pi) = -log(d^2) / (4 pi), and 1 / (4 pi d) = rsqrt(d^2) / (4 pi).
__device__ inline float kernel_entry(int kind, float d2) {
    constexpr float kInv4Pi = 0.0795774715459476679f;
    return kind == HMAT_KERNEL_LOG ? -logf(d2) * kInv4Pi : rsqrtf(d2) * kInv4Pi;
}

// The same from the hardware's base-2 logarithm and reciprocal square root
// (v_log_f32, v_rsq_f32, about 1 ulp for the normal squared distances of
// distinct points): the sample products, where the low-rank truncation error
// dominates anyway.
template <int KIND>
__device__ inline float kernel_entry_hw(float d2) {
    constexpr float kLn2Inv4Pi = 0.05515890003816573f, kInv4Pi = 0.0795774715459476679f;
    if constexpr (KIND == HMAT_KERNEL_LOG) return -__builtin_amdgcn_logf(d2) * kLn2Inv4Pi;
    return __builtin_amdgcn_rsqf(d2) * kInv4Pi;
}

__device__ inline void point3(const CKernel &k, int64_t i, float (&p)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = a < k.dim ? k.pts[i * k.dim + a] : 0.0f;
}

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of the
// multiply-xor round on a four-word counter, the two-word key bumped by the
// Weyl constants between rounds.
__device__ inline void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
    constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kW0;
            k1 += kW1;
        }
        const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
        const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__global__ __launch_bounds__(256) void k_cdense(CKernel k, const CDense *__restrict__ blocks,
                                                const CTile *__restrict__ tiles, float *__restrict__ out) {
    const CTile tl = tiles[blockIdx.x];
    const CDense b = blocks[tl.block];
    const int64_t e = tl.first + threadIdx.x;
    if (e >= (int64_t)b.mt * b.ms) return;
    const int64_t gi = b.t0 + e % b.mt, gj = b.s0 + e / b.mt;
    float v = k.diag;
    if (gi != gj) {
        float p[3], q[3];
        point3(k, gi, p);
        point3(k, gj, q);
        float d2 = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float d = p[a] - q[a];
            d2 = fmaf(d, d, d2);
        }
        v = kernel_entry(k.kind, d2);
    }
    out[b.off + e] = v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// v = h + m + l exactly: each part carries 8 significant bits of the FP32 value
// (the remainders v - h and (v - h) - m are exact in FP32).
__device__ inline void split3(float v, __bf16 &h, __bf16 &m, __bf16 &l) {
    h = (__bf16)v;
    const float r = v - (float)h;
    m = (__bf16)r;
    l = (__bf16)(r - (float)m);
}

// Sample products on MFMA (16x16x32 BF16, FP32 accumulation): mode 0 rows of t
// against the source points weighted by Omega, mode 1 rows of s against the
// target points weighted by Q. A wave owns 64 rows (four 16-row tiles); a lane
// generates the entries of its A fragments itself: row 16 m + lane % 16 of the
// wave's rows against the 8 other points 8 (lane / 16) + e of a 32-point
// k-step. Each entry is split into three BF16 parts (exact); Omega's +-1 is
// exact in BF16 (three products per tile), Q is split the same way (the six
// products of parts whose orders add up to at most 2^-16). The weights are
// staged as B fragments in LDS, 64 other points per tile. Padding points and
// rows copy a valid point, so every entry stays finite against zero weights.
// The block's entries are symmetric in the two points (t and s are disjoint,
// so no diagonal entry occurs).
template <int NT, int MODE, int KIND>
__global__ __launch_bounds__(256) void k_csample(CKernel k, CWork w, const CTile *__restrict__ tiles) {
    constexpr int mode = MODE;
    __shared__ float4 opt[kOther];
    __shared__ bf16x8 wb[MODE == 0 ? 1 : 3][2][NT][64];  // [part][k-step][n-tile][lane]
    const CTile tl = tiles[blockIdx.x];
    const CLowRank b = w.blocks[tl.block];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = mode == 0 ? b.t0 : b.s0, oth0 = mode == 0 ? b.s0 : b.t0;
    const int nrows = mode == 0 ? b.mt : b.ms, noth = mode == 0 ? b.ms : b.mt;
    const int rbase = (int)tl.first + 64 * wave;
    float p[4][3];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int r = rbase + 16 * m + (lane & 15);
        point3(k, row0 + (r < nrows ? r : 0), p[m]);
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const float *q = w.fws + b.yoff;
    for (int o0 = 0; o0 < noth; o0 += kOther) {
        const int nv = min(kOther, noth - o0);
        __syncthreads();  // the previous tile has been read
        if (tid < kOther) {
            float o[3];
            point3(k, oth0 + o0 + (tid < nv ? tid : 0), o);
            opt[tid] = make_float4(o[0], o[1], o[2], 0.0f);
        }
        if constexpr (MODE == 0) {
            if (tid < kOther) {  // the Rademacher row of other point o0 + tid, into its B-fragment slots
                uint64_t c4[4] = {(uint64_t)(oth0 + o0 + tid), 0, 0, 0};
                philox4x64_10(c4, w.seed, 0);
                const int ks = tid >> 5, e = tid & 7, lhi = ((tid & 31) >> 3) * 16;
#pragma unroll
                for (int c = 0; c < NT * 16; ++c) {
                    const float v = (tid < nv && c < b.ell) ? (((c4[c >> 6] >> (c & 63)) & 1) ? -1.0f : 1.0f) : 0.0f;
                    reinterpret_cast<__bf16 *>(&wb[0][ks][c >> 4][lhi + (c & 15)])[e] = (__bf16)v;
                }
            }
        } else {
            for (int e2 = tid; e2 < kOther * NT * 16; e2 += 256) {
                const int j = e2 % kOther, c = e2 / kOther;
                const float v = (j < nv && c < b.ell) ? q[(int64_t)(o0 + j) + (int64_t)c * b.mt] : 0.0f;
                __bf16 h, mm, l;
                split3(v, h, mm, l);
                const int ks = j >> 5, e = j & 7, ln = ((j & 31) >> 3) * 16 + (c & 15);
                reinterpret_cast<__bf16 *>(&wb[0][ks][c >> 4][ln])[e] = h;
                reinterpret_cast<__bf16 *>(&wb[1][ks][c >> 4][ln])[e] = mm;
                reinterpret_cast<__bf16 *>(&wb[2][ks][c >> 4][ln])[e] = l;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            if (ks * 32 >= nv) break;
            float4 o[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) o[e] = opt[ks * 32 + 8 * (lane >> 4) + e];
            bf16x8 ah[4], am[4], al[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float dx = p[m][0] - o[e].x, dy = p[m][1] - o[e].y, dz = p[m][2] - o[e].z;
                    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    __bf16 h, mm, l;
                    split3(kernel_entry_hw<KIND>(d2), h, mm, l);
                    ah[m][e] = h;
                    am[m][e] = mm;
                    al[m][e] = l;
                }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16x8 bh = wb[0][ks][t][lane];
                if constexpr (MODE == 0) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bh, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], bh, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[m], bh, acc[m][t], 0, 0, 0);
                    }
                } else {
                    const bf16x8 bm = wb[1][ks][t][lane], bl = wb[2][ks][t][lane];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bh, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bm, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], bh, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bl, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], bm, acc[m][t], 0, 0, 0);
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[m], bh, acc[m][t], 0, 0, 0);
                    }
                }
            }
        }
    }
    float *out = w.fws + (mode == 0 ? b.yoff : b.boff);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rbase + 16 * m + 4 * (lane >> 4) + e;
                if (r < nrows && c < b.ell) out[r + (int64_t)c * nrows] = acc[m][t][e];
            }
        }
}

// Gram matrix A^T A in FP64 of a column-major FP32 block A (Y or B^T), one
// workgroup per block; each thread owns a fixed set of the ell (ell + 1) / 2
// entries on and above the diagonal.
template <int LC>
__global__ __launch_bounds__(256) void k_cgram(CWork w, int which) {
    constexpr int kPer = (LC * (LC + 1) / 2 + 255) / 256;
    __shared__ float tile[64][LC + 1];
    const CLowRank b = w.blocks[blockIdx.x];
    const int tid = threadIdx.x, ell = b.ell;
    const int nrows = which == 0 ? b.mt : b.ms;
    const float *a = w.fws + (which == 0 ? b.yoff : b.boff);
    const int npairs = ell * (ell + 1) / 2;
    int px[kPer], py[kPer];
    double acc[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int e = tid + 256 * i, x = 0;
        acc[i] = 0.0;
        if (e >= npairs) {
            px[i] = py[i] = 0;
            continue;
        }
        while (e >= ell - x) {
            e -= ell - x;
            ++x;
        }
        px[i] = x;
        py[i] = x + e;
    }
    for (int r0 = 0; r0 < nrows; r0 += 64) {
        const int nv = min(64, nrows - r0);
        __syncthreads();
        for (int e = tid; e < 64 * ell; e += 256) {
            const int ii = e % 64, c = e / 64;
            tile[ii][c] = ii < nv ? a[(int64_t)(r0 + ii) + (int64_t)c * nrows] : 0.0f;
        }
        __syncthreads();
        // pairs past npairs point at entry (0, 0) and are never written back
#pragma unroll 2
        for (int ii = 0; ii < 64; ++ii)
#pragma unroll
            for (int i = 0; i < kPer; ++i) acc[i] = fma((double)tile[ii][px[i]], (double)tile[ii][py[i]], acc[i]);
    }
    double *g = w.gram + b.goff;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        if (tid + 256 * i >= npairs) break;
        g[px[i] + (int64_t)py[i] * ell] = acc[i];
        g[py[i] + (int64_t)px[i] * ell] = acc[i];
    }
}

// Parallel cyclic Jacobi on the Gram matrix of one block (one workgroup per
// block, G and the accumulated rotations P in LDS, FP64). Each round applies
// n / 2 disjoint rotations (round-robin pairing of n = ell rounded up to even
// indices; a padding index is a zero row and column and never rotates): the
// rotation that zeroes G_pq (Golub and Van Loan, Matrix Computations,
// Algorithm 8.5.2), then G <- J^T G J and P <- P J. Sweeps repeat until one
// applies no rotation (every |G_pq| <= 1e-15 sqrt(|G_pp G_qq|)), at most 40.
// mode 0: T = P D^(-1/2) over the eigenvalues above 1e-13 of the largest
// (other columns zero), ell x ell at toff. mode 1: the leading `rank`
// eigenpairs by value, those above 1e-14 of the largest: M_U = w l^(1/4) at
// toff and M_V = w l^(-1/4) at toff + ell rank (ell x rank each; the rest zero).
__global__ __launch_bounds__(256) void k_ceig(CWork w, int mode) {
    extern __shared__ double sm[];
    __shared__ int s_changed;
    const CLowRank b = w.blocks[blockIdx.x];
    const int tid = threadIdx.x, ell = b.ell, n = ell + (ell & 1), half = n / 2;
    const int nmax = w.max_ell + (w.max_ell & 1);
    double *G = sm, *P = sm + nmax * nmax, *rc = P + nmax * nmax, *rs = rc + nmax / 2;
    int *rp = reinterpret_cast<int *>(rs + nmax / 2), *rq = rp + nmax / 2;
    const double *g0 = w.gram + b.goff;
    for (int e = tid; e < n * n; e += 256) {
        const int i = e % n, j = e / n;
        G[e] = (i < ell && j < ell) ? g0[i + (int64_t)j * ell] : 0.0;
        P[e] = i == j ? 1.0 : 0.0;
    }
    if (tid == 0) s_changed = 0;
    __syncthreads();
    for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
        for (int round = 0; round < n - 1; ++round) {
            if (tid < half) {
                int p, q;
                if (tid == 0) {
                    p = n - 1;
                    q = round;
                } else {
                    p = (round + tid) % (n - 1);
                    q = (round - tid + n - 1) % (n - 1);
                }
                const double gpp = G[p + p * n], gqq = G[q + q * n], gpq = G[p + q * n];
                double c = 1.0, s = 0.0;
                if (gpq != 0.0 && fabs(gpq) > 1e-15 * sqrt(fabs(gpp * gqq))) {
                    const double th = (gqq - gpp) / (2.0 * gpq);
                    const double t = fabs(th) > 1e150 ? 0.5 / th
                                                      : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    s_changed = 1;
                }
                rc[tid] = c;
                rs[tid] = s;
                rp[tid] = p;
                rq[tid] = q;
            }
            __syncthreads();
            for (int e = tid; e < half * n; e += 256) {  // rows p, q of G
                const int k = e % half, j = e / half;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double gp = G[p + j * n], gq = G[q + j * n];
                G[p + j * n] = c * gp - s * gq;
                G[q + j * n] = s * gp + c * gq;
            }
            __syncthreads();
            for (int e = tid; e < half * n; e += 256) {  // columns p, q of G and of P
                const int k = e % half, i = e / half;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double gp = G[i + p * n], gq = G[i + q * n];
                G[i + p * n] = c * gp - s * gq;
                G[i + q * n] = s * gp + c * gq;
                const double vp = P[i + p * n], vq = P[i + q * n];
                P[i + p * n] = c * vp - s * vq;
                P[i + q * n] = s * vp + c * vq;
            }
            __syncthreads();
        }
        const int changed = s_changed;
        __syncthreads();  // every thread has read the flag before it is cleared
        if (!changed) break;
        if (tid == 0) s_changed = 0;
        __syncthreads();
    }
    double lmax = 0.0;
    for (int i = 0; i < ell; ++i) lmax = fmax(lmax, G[i + i * n]);
    float *t = w.fws + b.toff;
    if (mode == 0) {
        for (int e = tid; e < ell * ell; e += 256) {
            const int k = e % ell, i = e / ell;
            const double l = G[i + i * n];
            const double f = (l > 1e-13 * lmax && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
            t[k + i * ell] = (float)(P[k + i * n] * f);
        }
        return;
    }
    const int rank = b.rank;
    for (int e = tid; e < 2 * ell * rank; e += 256) t[e] = 0.0f;
    __syncthreads();
    for (int e = tid; e < ell * ell; e += 256) {
        const int k = e % ell, i = e / ell;
        const double l = G[i + i * n];
        int pos = 0;  // place of eigenvalue i in descending order (ties by index)
        for (int j = 0; j < ell; ++j) {
            const double lj = G[j + j * n];
            pos += (lj > l || (lj == l && j < i)) ? 1 : 0;
        }
        if (pos >= rank || !(l > 1e-14 * lmax && l > 0.0)) continue;
        const double q4 = sqrt(sqrt(l));
        t[k + pos * ell] = (float)(P[k + i * n] * q4);
        t[ell * rank + k + pos * ell] = (float)(P[k + i * n] / q4);
    }
}

// out = A T row by row (one thread per row): what 0 Y <- Y T in place (T ell x
// ell), 1 U = Q M_U, 2 V = B^T M_V (ell x rank). T is staged transposed in
// LDS so that a thread reads one column of T as consecutive words.
template <int LC>
__global__ __launch_bounds__(256) void k_capply(CWork w, const CTile *__restrict__ tiles, int what) {
    __shared__ __align__(16) float tt[LC * LC];
    const CTile tl = tiles[blockIdx.x];
    const CLowRank b = w.blocks[tl.block];
    const int tid = threadIdx.x, ell = b.ell;
    const int nrows = what == 2 ? b.ms : b.mt;
    const int ncols = what == 0 ? ell : b.rank;
    const float *a = w.fws + (what == 2 ? b.boff : b.yoff);
    const float *t = w.fws + b.toff + (what == 2 ? (int64_t)ell * b.rank : 0);
    float *out = w.fws + (what == 0 ? b.yoff : what == 1 ? b.uoff : b.voff);
    for (int e = tid; e < LC * LC; e += 256) {
        const int c = e / LC, k = e % LC;
        tt[e] = (c < ncols && k < ell) ? t[k + c * ell] : 0.0f;
    }
    __syncthreads();
    const int r = (int)tl.first + tid;
    if (r >= nrows) return;
    float av[LC];
#pragma unroll
    for (int k = 0; k < LC; ++k) av[k] = k < ell ? a[r + (int64_t)k * nrows] : 0.0f;
    for (int c = 0; c < ncols; ++c) {
        const float *col = tt + c * LC;
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < LC; ++k) s = fmaf(av[k], col[k], s);
        out[r + (int64_t)c * nrows] = s;
    }
}

#define HMAT_LC_SWITCH(lc, CALL) \
    switch (lc) {                \
    case 16: CALL(16); break;    \
    case 32: CALL(32); break;    \
    case 48: CALL(48); break;    \
    case 64: CALL(64); break;    \
    case 80: CALL(80); break;    \
    case 96: CALL(96); break;    \
    default: return (int)hipErrorInvalidValue; \
    }

}  // namespace

int launch_compress_dense(const CKernel &k, const CDense *blocks, const CTile *tiles, int64_t ntiles, float *out,
                          void *stream) {
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL(k_cdense, dim3((unsigned)ntiles), dim3(256), 0, static_cast<hipStream_t>(stream), k, blocks,
                       tiles, out);
    return (int)hipGetLastError();
}

int launch_compress_sample(const CKernel &k, const CWork &w, const CTile *tiles, int64_t ntiles, int mode,
                           void *stream) {
    if (ntiles <= 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
#define HMAT_LAUNCH(L, M, K) \
    hipLaunchKernelGGL((k_csample<(L) / 16, M, K>), dim3((unsigned)ntiles), dim3(256), 0, st, k, w, tiles)
#define HMAT_CALL(L)                                                          \
    if (k.kind == HMAT_KERNEL_LOG) {                                           \
        if (mode == 0) HMAT_LAUNCH(L, 0, HMAT_KERNEL_LOG);                     \
        else HMAT_LAUNCH(L, 1, HMAT_KERNEL_LOG);                               \
    } else {                                                                   \
        if (mode == 0) HMAT_LAUNCH(L, 0, HMAT_KERNEL_INV);                     \
        else HMAT_LAUNCH(L, 1, HMAT_KERNEL_INV);                               \
    }
    HMAT_LC_SWITCH(w.lc, HMAT_CALL)
#undef HMAT_CALL
#undef HMAT_LAUNCH
    return (int)hipGetLastError();
}

int launch_compress_gram(const CWork &w, int64_t nblocks, int which, void *stream) {
    if (nblocks <= 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
#define HMAT_CALL(L) hipLaunchKernelGGL(k_cgram<L>, dim3((unsigned)nblocks), dim3(256), 0, st, w, which)
    HMAT_LC_SWITCH(w.lc, HMAT_CALL)
#undef HMAT_CALL
    return (int)hipGetLastError();
}

int launch_compress_eig(const CWork &w, int64_t nblocks, int mode, void *stream) {
    if (nblocks <= 0) return 0;
    const int n = w.max_ell + (w.max_ell & 1);
    const size_t lds = (size_t)2 * n * n * sizeof(double) + (size_t)(n / 2) * (2 * sizeof(double) + 2 * sizeof(int));
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_ceig),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(k_ceig, dim3((unsigned)nblocks), dim3(256), lds, static_cast<hipStream_t>(stream), w, mode);
    return (int)hipGetLastError();
}

int launch_compress_apply(const CWork &w, const CTile *tiles, int64_t ntiles, int what, void *stream) {
    if (ntiles <= 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
#define HMAT_CALL(L) hipLaunchKernelGGL(k_capply<L>, dim3((unsigned)ntiles), dim3(256), 0, st, w, tiles, what)
    HMAT_LC_SWITCH(w.lc, HMAT_CALL)
#undef HMAT_CALL
    return (int)hipGetLastError();
}

}  // namespace hmat
