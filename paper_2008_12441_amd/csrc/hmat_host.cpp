// Host side of libhmat: argument and structure validation, the level-ordered
// device layout, host-side quantisation, device memory, kernel launches and
// timing. The C ABI is declared in include/hmat.h.
#include "hmat.h"
#include "hmat_handle.h"
#include "hmat_compress.h"
#include "hmat_internal.h"
#include "hmat_structure.h"
#include "hmat_host_quant.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

using hmat::ChunkMeta;
using hmat::DevPlan;
using hmat::DSeg;
using hmat::VTile;
using hmat::ZItem;
using hmat::ZItem2;
using hmat::ZSeg;
using hmat::Tree;
using hmat::Structure;
using hmat::analyse_tree;
using hmat::parallel_for;
using hmat::validate_blocks;
using hmat::dense_group_amax;
using hmat::col_major_amax;
using hmat::f32_to_bf16_rne;
using hmat::f32_to_f16_rne;
using hmat::pow2_scale_f16;
using hmat::quant16;

namespace {

thread_local std::string t_err;
std::mutex g_mu;
std::unordered_set<const hmat_handle *> g_live;

hmat_status fail(hmat_status s, const std::string &msg) {
    t_err = msg;
    return s;
}

bool is_live(const hmat_handle *h) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_live.count(h) != 0;
}

}  // namespace

hmat_status hmat::set_error(hmat_status s, const std::string &msg) { return fail(s, msg); }

bool hmat::handle_live(const hmat_handle *h, int add_ref) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_live.count(h)) return false;
    const_cast<hmat_handle *>(h)->batch_refs += add_ref;
    return true;
}

namespace {

// FP8 E4M3 (OCP E4M3FN: bias 7, 3 mantissa bits, subnormals, largest finite
// 448, no infinities) code of x by round-to-nearest-even; |x| <= 448.
uint8_t e4m3_rne(double x) {
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    const double a = std::fabs(x);
    if (a == 0.0) return sign;
    int e = 0;
    std::frexp(a, &e);  // a = m 2^e, m in [0.5, 1): the leading bit has weight 2^(e-1)
    const int lead = std::max(e - 1, -6);                 // subnormals share the exponent of 2^-6
    const double q = std::nearbyint(std::ldexp(a, 3 - lead));  // significand in units of 2^(lead-3), RNE
    int32_t code;
    if (lead == -6 && q < 8.0)
        code = (int32_t)q;                                // subnormal (q = 8 is the smallest normal)
    else if (q >= 16.0)
        code = ((lead + 1 + 7) << 3);                     // rounded up to the next binade
    else
        code = ((lead + 7) << 3) | ((int32_t)q - 8);
    return (uint8_t)(sign | code);
}

double e4m3_value(uint8_t c) {
    const int ex = (c >> 3) & 0xF, m = c & 7;
    const double v = ex == 0 ? std::ldexp((double)m, -9) : std::ldexp(8.0 + m, ex - 10);
    return (c & 0x80) ? -v : v;
}

// Smallest power of two s with a / s <= 448 (1 for a == 0): the E4M3 column
// scale 2^ceil(log2(a / 448)), chosen without rounding error.
double pow2_scale_e4m3(double a) {
    if (!(a > 0.0)) return 1.0;
    int e = 0;
    std::frexp(a / 448.0, &e);
    int k = e;
    while (a > std::ldexp(448.0, k)) ++k;
    while (k > -1074 && a <= std::ldexp(448.0, k - 1)) --k;
    return std::ldexp(1.0, k);
}

// FP16 code of a power of two (0 below the FP16 range).
uint16_t f16_pow2_code(double s) {
    return f32_to_f16_rne((float)s);
}

// Column scales of an FP8 factor (rows x cols, column-major, ld): per column
// j, s[2 j] = s_j and s[2 j + 1] = s'_j.
void e4m3_column_scales(const float *a, int64_t rows, int64_t cols, int64_t ld, float *s) {
    for (int64_t j = 0; j < cols; ++j) {
        double am = 0.0;
        for (int64_t i = 0; i < rows; ++i) am = std::max(am, (double)std::fabs(a[i + j * ld]));
        const double sj = pow2_scale_e4m3(am);
        double ar = 0.0;
        for (int64_t i = 0; i < rows; ++i) {
            const double u = (double)a[i + j * ld] / sj;
            ar = std::max(ar, std::fabs(u - e4m3_value(e4m3_rne(u))));
        }
        s[2 * j] = (float)sj;
        s[2 * j + 1] = (float)pow2_scale_e4m3(ar);
    }
}

// hi and lo codes of v in a column with scales (sj, slj).
inline void e4m3_hilo(float v, float sj, float slj, uint8_t *hi, uint8_t *lo) {
    const double u = (double)v / sj;
    *hi = e4m3_rne(u);
    *lo = e4m3_rne((u - e4m3_value(*hi)) / slj);
}

// ---------------------------------------------------------------------------
// Level-ordered layout.
// ---------------------------------------------------------------------------
struct HostPlan {
    int32_t vw = 4;                 // elements per 16-byte vector
    bool bf16 = false;              // 16-bit codes are BF16 (else scaled FP16)
    int32_t chunk_depth = 0;
    std::vector<int32_t> chunk_node;
    std::vector<ChunkMeta> chunks;
    std::vector<ZSeg> zsegs;
    std::vector<DSeg> dsegs;
    std::vector<float> dscale;
    std::vector<VTile> vtiles;
    std::vector<ZItem> z1;
    std::vector<ZItem2> z2;
    std::vector<int32_t> anc;       // chunk x chunk_depth+1: ancestor at each depth
    std::vector<int32_t> vcol;      // per block
    std::vector<int32_t> zdst;      // per block
    std::vector<int32_t> zoff, zlen; // per node
    std::vector<float> sU, sV, sD;  // per block scales
    int64_t v_elems = 0, ud_elems = 0;
    int64_t part_floats = 0, slice_floats = 0, zg_floats = 0;
    int32_t lds_floats = 0, max_leaf_rows = 0;
};

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// The leaves below a chunk node: its children, or the node itself when the root is a leaf.
std::vector<int32_t> chunk_leaves(const Tree &t, int32_t node) {
    std::vector<int32_t> v;
    if (t.L == 0) v.push_back(node);
    else
        for (int32_t j = 0; j < t.nkids(node); ++j) v.push_back(t.kid(node, j));
    return v;
}

hmat_status build_plan(const Tree &t, const Structure &st, const hmat_block_desc *bl, int64_t nb,
                       int32_t storage, int32_t acc_bytes, HostPlan &hp) {
    hp.vw = storage == HMAT_STORE_FP32 ? 4 : 8;
    hp.bf16 = storage == HMAT_STORE_BF16;
    const int32_t vw = hp.vw;
    const int32_t L = t.L;
    const int32_t cd = std::max(L - 1, 0);
    hp.chunk_depth = cd;
    for (int32_t i = 0; i < t.num_nodes; ++i)
        if (t.depth[i] == cd) hp.chunk_node.push_back(i);
    std::sort(hp.chunk_node.begin(), hp.chunk_node.end(),
              [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
    const int32_t nc = (int32_t)hp.chunk_node.size();
    hp.anc.assign((size_t)nc * (cd + 1), 0);
    // chunk range of every node at depth <= cd
    std::vector<int32_t> cfirst(t.num_nodes, INT32_MAX), clast(t.num_nodes, -1);
    for (int32_t c = 0; c < nc; ++c) {
        int32_t a = hp.chunk_node[c];
        for (int32_t d = cd; d >= 0; --d) {
            hp.anc[(size_t)c * (cd + 1) + d] = a;
            cfirst[a] = std::min(cfirst[a], c);
            clast[a] = std::max(clast[a], c + 1);
            a = t.parent[a];
        }
    }
    auto rank_of = [&](int64_t b) { return bl[b].rank; };

    // per-block scales
    hp.sU.assign(nb, 1.0f);
    hp.sV.assign(nb, 1.0f);
    hp.sD.assign(nb, 1.0f);
    if (storage != HMAT_STORE_FP32) {
        const bool scaled = storage == HMAT_STORE_FP16_SCALED;
        std::atomic<bool> ok{true};
        std::vector<float> amax_d(nb, 0.0f);
        parallel_for(nb, [&](int64_t b) {
            bool fin = true;
            const hmat_block_desc &d = bl[b];
            const int64_t mt = t.size(d.target), ms = t.size(d.source);
            if (d.rank == 0) {
                amax_d[b] = col_major_amax(d.a, mt, ms, d.lda, &fin);
            } else {
                const float au = col_major_amax(d.a, mt, d.rank, d.lda, &fin);
                const float av = col_major_amax(d.b, ms, d.rank, d.ldb, &fin);
                if (scaled) {
                    hp.sU[b] = pow2_scale_f16(au);
                    hp.sV[b] = pow2_scale_f16(av);
                }
            }
            if (!fin) ok = false;
        });
        if (!ok) return fail(HMAT_ERR_INVALID_ARG, "factors contain non-finite values");
        if (scaled) {  // a dense block's scale covers its group (see dense_group_amax)
            dense_group_amax(t, bl, nb, amax_d);
            for (int64_t b = 0; b < nb; ++b)
                if (bl[b].rank == 0) hp.sD[b] = pow2_scale_f16(amax_d[b]);
        }
    }

    // z layout: per non-leaf node t at depth 1..L-1, the z vectors of its low-rank blocks (t, s)
    hp.zoff.assign(t.num_nodes, 0);
    hp.zlen.assign(t.num_nodes, 0);
    hp.zdst.assign(nb, -1);
    hp.vcol.assign(nb, -1);
    int64_t zcur = 0;
    for (int32_t a = 1; a < t.num_nodes && L >= 2; ++a) {
        if (t.depth[a] < 1 || t.depth[a] > L - 1) continue;
        hp.zoff[a] = (int32_t)zcur;
        int32_t off = 0;
        for (const int64_t b : st.by_target[a]) {
            hp.zdst[b] = (int32_t)(zcur + off);
            off += rank_of(b);
        }
        hp.zlen[a] = off;
        zcur += off;
    }
    hp.zg_floats = zcur;

    // chunks
    hp.chunks.resize(nc);
    int64_t ud_cur = 0, part_cur = 0;
    int32_t max_lds = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t node = hp.chunk_node[c];
        ChunkMeta &m = hp.chunks[c];
        std::memset(&m, 0, sizeof(m));
        m.row_begin = (int32_t)t.begin[node];
        m.rows = (int32_t)t.size(node);
        // V columns (source side) and their offsets
        int32_t wv = 0;
        for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
            const int32_t a = hp.anc[(size_t)c * (cd + 1) + lvl];
            for (const int64_t b : st.by_source[a]) {
                if (hp.vcol[b] < 0) hp.vcol[b] = wv;
                else if (hp.vcol[b] != wv)
                    return fail(HMAT_ERR_UNSUPPORTED, "inconsistent source column layout");
                wv += rank_of(b);
            }
        }
        const int32_t ncb = (wv + hmat::kWave - 1) / hmat::kWave;
        const int32_t nvec = (m.rows + vw - 1) / vw;
        m.part_base = (int32_t)part_cur;
        for (int32_t cb = 0; cb < ncb; ++cb) {
            VTile vt;
            vt.off = hp.v_elems;
            vt.chunk = c;
            vt.pout = (int32_t)(part_cur + (int64_t)cb * hmat::kWave);
            hp.vtiles.push_back(vt);
            hp.v_elems += (int64_t)nvec * hmat::kWave * vw;
        }
        part_cur += (int64_t)ncb * hmat::kWave;
        // U columns (target side): z segments of each ancestor level
        m.zseg_base = (int32_t)hp.zsegs.size();
        int32_t wlr = 0;
        for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
            const int32_t a = hp.anc[(size_t)c * (cd + 1) + lvl];
            hp.zsegs.push_back(ZSeg{hp.zoff[a], hp.zlen[a]});
            wlr += hp.zlen[a];
        }
        m.nq_lr = (wlr + vw - 1) / vw;
        // dense part: one segment per source leaf of the chunk's dense blocks, then
        // (for the row -> target leaf lookup) one per target leaf, the chunk's children
        m.dseg_base = (int32_t)hp.dsegs.size();
        const std::vector<int32_t> tleaves = chunk_leaves(t, node);
        const std::vector<int32_t> &sleaves = L == 0 ? tleaves : st.dense_src[node];
        m.nleaf = (int32_t)sleaves.size();
        m.ntleaf = (int32_t)tleaves.size();
        int32_t nq = m.nq_lr;
        for (int32_t pass = 0; pass < 2; ++pass)
            for (int32_t lf : pass == 0 ? sleaves : tleaves) {
                DSeg ds;
                ds.row_begin = (int32_t)t.begin[lf];
                ds.rows = (int32_t)t.size(lf);
                ds.nq = (ds.rows + vw - 1) / vw;
                ds.pad_ = 0;
                if (pass == 0) nq += ds.nq;
                hp.dsegs.push_back(ds);
                hp.max_leaf_rows = std::max(hp.max_leaf_rows, ds.rows);
            }
        m.nq = nq;
        m.dscale_base = (int32_t)hp.dscale.size();
        for (int32_t lt : tleaves)
            for (int32_t ls : sleaves) hp.dscale.push_back(hp.sD[L == 0 ? 0 : st.find(lt, ls)]);
        m.ud_off = ud_cur;
        const int32_t ntile = (m.rows + hmat::kWave - 1) / hmat::kWave;
        ud_cur += (int64_t)ntile * nq * hmat::kWave * vw;
        max_lds = std::max(max_lds, nq * vw);
    }
    hp.ud_elems = ud_cur;
    hp.part_floats = part_cur;
    hp.lds_floats = max_lds;
    if ((int64_t)max_lds * acc_bytes > hmat::kMaxLdsBytes)
        return fail(HMAT_ERR_UNSUPPORTED, "a chunk's vector operand (" + std::to_string(max_lds) +
                                              " values of " + std::to_string(acc_bytes) +
                                              " bytes) exceeds the U-phase LDS budget");
    if (hp.part_floats >= INT32_MAX || hp.zg_floats >= INT32_MAX)
        return fail(HMAT_ERR_UNSUPPORTED, "workspace too large");

    // partial reduction items: slices of at most 32 chunks; slice sums live in
    // the same buffer as z, after it
    const int32_t S = 32;
    int64_t slice_cur = hp.zg_floats;
    for (int64_t b = 0; b < nb && L >= 2; ++b) {
        if (bl[b].rank == 0) continue;
        const int32_t s = bl[b].source;
        const int32_t c0 = cfirst[s], c1 = clast[s];
        const int32_t r = bl[b].rank;
        const float scale = hp.sU[b] * hp.sV[b];
        if (c1 - c0 <= S) {
            hp.z1.push_back(ZItem{c0, c1 - c0, hp.vcol[b], r, hp.zdst[b], scale});
        } else {
            const int32_t nsl = (c1 - c0 + S - 1) / S;
            for (int32_t k = 0; k < nsl; ++k) {
                const int32_t a0 = c0 + k * S;
                hp.z1.push_back(ZItem{a0, std::min(S, c1 - a0), hp.vcol[b], r,
                                      (int32_t)(slice_cur + (int64_t)k * r), 1.0f});
            }
            hp.z2.push_back(ZItem2{(int32_t)slice_cur, nsl, r, hp.zdst[b], scale, 0});
            slice_cur += (int64_t)nsl * r;
        }
    }
    hp.slice_floats = slice_cur - hp.zg_floats;
    if (slice_cur >= INT32_MAX) return fail(HMAT_ERR_UNSUPPORTED, "workspace too large");
    return HMAT_OK;
}

// Fill the V panel (FP32 or FP16) for the chunks [c_lo, c_hi).
template <class T>
void fill_v(const Tree &t, const Structure &st, const hmat_block_desc *bl, const HostPlan &hp,
            T *out, int64_t base_elem) {
    const int32_t vw = hp.vw;
    const int32_t cd = hp.chunk_depth;
    const int32_t L = t.L;
    // first vtile of each chunk
    std::vector<int32_t> first(hp.chunks.size() + 1, (int32_t)hp.vtiles.size());
    for (int32_t i = (int32_t)hp.vtiles.size() - 1; i >= 0; --i) first[hp.vtiles[i].chunk] = i;
    for (int32_t c = (int32_t)hp.chunks.size() - 1; c >= 0; --c)
        first[c] = std::min(first[c], first[c + 1]);
    parallel_for((int64_t)hp.chunks.size(), [&](int64_t c) {
        const ChunkMeta &m = hp.chunks[c];
        if (first[c] >= (int32_t)hp.vtiles.size() || hp.vtiles[first[c]].chunk != c) return;
        const int32_t nvec = (m.rows + vw - 1) / vw;
        int32_t col = 0;
        for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
            const int32_t a = hp.anc[(size_t)c * (cd + 1) + lvl];
            const int64_t roff = m.row_begin - t.begin[a];
            for (const int64_t b : st.by_source[a]) {
                const hmat_block_desc &d = bl[b];
                const float inv = 1.0f / hp.sV[b];
                for (int32_t k = 0; k < d.rank; ++k, ++col) {
                    const VTile &vt = hp.vtiles[first[c] + col / hmat::kWave];
                    T *dst = out + (vt.off - base_elem);
                    const int32_t l = col % hmat::kWave;
                    const float *src = d.b + roff + (int64_t)k * d.ldb;
                    for (int32_t i = 0; i < nvec * vw; ++i) {
                        const float v = i < m.rows ? src[i] : 0.0f;
                        T q;
                        if constexpr (sizeof(T) == 4) q = v;
                        else q = quant16(v, inv, hp.bf16);
                        dst[((int64_t)(i / vw) * hmat::kWave + l) * vw + i % vw] = q;
                    }
                }
            }
        }
    });
}

template <class T>
void fill_ud(const Tree &t, const Structure &st, const hmat_block_desc *bl, const HostPlan &hp,
             T *out) {
    const int32_t vw = hp.vw;
    const int32_t cd = hp.chunk_depth;
    const int32_t L = t.L;
    parallel_for((int64_t)hp.chunks.size(), [&](int64_t c) {
        const ChunkMeta &m = hp.chunks[c];
        const int64_t tile_stride = (int64_t)m.nq * hmat::kWave * vw;
        auto put = [&](int32_t i, int32_t j, T q) {
            out[m.ud_off + (i / hmat::kWave) * tile_stride +
                ((int64_t)(j / vw) * hmat::kWave + i % hmat::kWave) * vw + j % vw] = q;
        };
        const int32_t ntile = (m.rows + hmat::kWave - 1) / hmat::kWave;
        const int32_t prow = ntile * hmat::kWave;
        int32_t col = 0;
        for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
            const int32_t a = hp.anc[(size_t)c * (cd + 1) + lvl];
            const int64_t roff = m.row_begin - t.begin[a];
            for (const int64_t b : st.by_target[a]) {
                const hmat_block_desc &d = bl[b];
                const float inv = 1.0f / hp.sU[b];
                for (int32_t k = 0; k < d.rank; ++k, ++col) {
                    const float *src = d.a + roff + (int64_t)k * d.lda;
                    for (int32_t i = 0; i < prow; ++i) {
                        const float v = i < m.rows ? src[i] : 0.0f;
                        if constexpr (sizeof(T) == 4) put(i, col, v);
                        else put(i, col, quant16(v, inv, hp.bf16));
                    }
                }
            }
        }
        for (; col < m.nq_lr * vw; ++col)
            for (int32_t i = 0; i < prow; ++i) put(i, col, T(0));
        // dense part, grouped by source leaf; the target leaf of a row selects the block
        const std::vector<int32_t> tleaves = chunk_leaves(t, hp.chunk_node[c]);
        const std::vector<int32_t> &sleaves = L == 0 ? tleaves : st.dense_src[hp.chunk_node[c]];
        const DSeg *tsegs = hp.dsegs.data() + m.dseg_base + m.nleaf;
        int32_t qcol = m.nq_lr * vw;
        for (int32_t is = 0; is < m.nleaf; ++is) {
            const DSeg &sseg = hp.dsegs[m.dseg_base + is];
            std::vector<int64_t> blk(m.ntleaf);
            for (int32_t it = 0; it < m.ntleaf; ++it) blk[it] = L == 0 ? 0 : st.find(tleaves[it], sleaves[is]);
            for (int32_t jj = 0; jj < sseg.nq * vw; ++jj, ++qcol) {
                for (int32_t it = 0, i = 0; i < prow; ++i) {
                    float v = 0.0f;
                    float inv = 1.0f;
                    if (i < m.rows && jj < sseg.rows) {
                        while (it + 1 < m.ntleaf && m.row_begin + i >= tsegs[it + 1].row_begin) ++it;
                        const DSeg &tseg = tsegs[it];
                        const int64_t b = blk[it];
                        const hmat_block_desc &d = bl[b];
                        v = d.a[(m.row_begin + i - tseg.row_begin) + (int64_t)jj * d.lda];
                        inv = 1.0f / hp.sD[b];
                    }
                    if constexpr (sizeof(T) == 4) put(i, qcol, v);
                    else put(i, qcol, quant16(v, inv, hp.bf16));
                }
            }
        }
    });
}


// ---------------------------------------------------------------------------
// Multi-RHS (MFMA) layout.
// ---------------------------------------------------------------------------
constexpr int32_t kUnitChunks = 4;    // chunks a V-phase unit accumulates over
constexpr int32_t kMaxRankMR = 128;

struct HostPlanMR {
    int32_t kb = 16, vw = 4, ntmax = 1;
    bool bf16 = false;
    bool fp8 = false;        // U, V as E4M3 hi + lo (HMAT_STORE_FP8, HMAT_STORE_FP8_F16D)
    bool dense_bf16 = false; // D as BF16 of v / s_D (HMAT_STORE_FP8)
    std::vector<std::vector<float>> colU, colV;  // FP8: per low-rank block, (s_j, s'_j) per column
    std::vector<uint16_t> vlo, ulo;              // FP8: FP16 lo-scale tables
    std::vector<float> zcol;                     // FP8: per z item and column, s_j(U) s_j(V)
    int32_t chunk_depth = 0;
    std::vector<int32_t> chunk_node;
    std::vector<int32_t> anc;                  // chunk x (chunk_depth + 1)
    std::vector<hmat::MRChunk> chunks;
    std::vector<hmat::MRLeaf> leaves;
    std::vector<int32_t> leaf_node;            // node id of each leaf entry
    std::vector<hmat::MRVUnit> vunits;
    std::vector<int32_t> unit_node, unit_group;
    std::vector<hmat::MRZItem> zitems;
    std::vector<hmat::MRZMember> zmembers;
    std::vector<int64_t> zmember_block;        // low-rank block of each z item member
    std::vector<std::vector<int32_t>> zrow_member;  // per z item: the member holding each row
    std::vector<hmat::MRSeg> segs;
    std::vector<int32_t> seg_chunk;            // source chunk of an x segment (-1 for z)
    std::vector<hmat::MRTile> tiles;
    std::vector<hmat::MRTileGroup> tgroups;
    std::vector<hmat::MRUnitGroup> ugroups;
    std::vector<hmat::MRStep> ustep;
    std::vector<float> dscale;
    std::vector<std::vector<std::pair<int64_t, int32_t>>> colmap;  // per node s: V column -> (block, j)
    std::vector<float> sU, sV, sD;
    int64_t v_frags = 0, ud_frags = 0, x_frags = 0, z_frags = 0, part_floats = 0;
};

hmat_status build_plan_mr(const Tree &t, const Structure &st, const hmat_block_desc *bl, int64_t nb,
                          int32_t storage, int32_t max_nrhs, HostPlanMR &hp) {
    hp.fp8 = storage == HMAT_STORE_FP8 || storage == HMAT_STORE_FP8_F16D;
    hp.dense_bf16 = storage == HMAT_STORE_FP8;
    const bool f16 = storage == HMAT_STORE_FP16_SCALED || hp.fp8;  // D (and U, V unless FP8) block-scaled
    const bool half = storage != HMAT_STORE_FP32;  // 16-bit lanes (FP16, BF16, or FP8 hi + lo pairs)
    hp.bf16 = storage == HMAT_STORE_BF16;
    hp.kb = half ? 32 : 16;
    hp.vw = half ? 8 : 4;
    hp.ntmax = (std::min(max_nrhs, 128) + 15) / 16;
    const int32_t KB = hp.kb, L = t.L, cd = std::max(L - 1, 0);
    hp.chunk_depth = cd;
    for (int64_t b = 0; b < nb; ++b)
        if (bl[b].rank > kMaxRankMR)
            return fail(HMAT_ERR_UNSUPPORTED, "multi-RHS handles support ranks up to 128");
    for (int32_t i = 0; i < t.num_nodes; ++i)
        if (t.depth[i] == cd) hp.chunk_node.push_back(i);
    std::sort(hp.chunk_node.begin(), hp.chunk_node.end(),
              [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
    const int32_t nc = (int32_t)hp.chunk_node.size();
    hp.anc.assign((size_t)nc * (cd + 1), 0);
    std::vector<int32_t> cfirst(t.num_nodes, INT32_MAX), clast(t.num_nodes, -1), chunk_of(t.num_nodes, -1);
    // the boxes at depth L - 1 whose leaves are the dense sources of a chunk's leaves (the
    // chunk itself when the root is a leaf), in row order
    auto dense_partners = [&](int32_t node) {
        std::vector<int32_t> out;
        if (L == 0) return std::vector<int32_t>{node};
        for (int32_t ls : st.dense_src[node])
            if (out.empty() || out.back() != t.parent[ls]) out.push_back(t.parent[ls]);
        return out;
    };
    for (int32_t c = 0; c < nc; ++c) {
        int32_t a = hp.chunk_node[c];
        chunk_of[a] = c;
        for (int32_t d = cd; d >= 0; --d) {
            hp.anc[(size_t)c * (cd + 1) + d] = a;
            cfirst[a] = std::min(cfirst[a], c);
            clast[a] = std::max(clast[a], c + 1);
            a = t.parent[a];
        }
    }
    hp.sU.assign(nb, 1.0f);
    hp.sV.assign(nb, 1.0f);
    hp.sD.assign(nb, 1.0f);
    if (half) {
        std::atomic<bool> ok{true};
        std::vector<float> amax_d(nb, 0.0f);
        parallel_for(nb, [&](int64_t b) {
            bool fin = true;
            const hmat_block_desc &d = bl[b];
            const int64_t mt = t.size(d.target), ms = t.size(d.source);
            if (d.rank == 0) {
                amax_d[b] = col_major_amax(d.a, mt, ms, d.lda, &fin);
            } else {
                const float au = col_major_amax(d.a, mt, d.rank, d.lda, &fin);
                const float av = col_major_amax(d.b, ms, d.rank, d.ldb, &fin);
                if (f16 && !hp.fp8) {
                    hp.sU[b] = pow2_scale_f16(au);
                    hp.sV[b] = pow2_scale_f16(av);
                }
            }
            if (!fin) ok = false;
        });
        if (!ok) return fail(HMAT_ERR_INVALID_ARG, "factors contain non-finite values");
        if (f16) {  // a dense block's scale covers its group (see dense_group_amax)
            dense_group_amax(t, bl, nb, amax_d);
            for (int64_t b = 0; b < nb; ++b)
                if (bl[b].rank == 0) hp.sD[b] = pow2_scale_f16(amax_d[b]);
        }
    }
    if (hp.fp8) {
        hp.colU.assign(nb, {});
        hp.colV.assign(nb, {});
        parallel_for(nb, [&](int64_t b) {
            const hmat_block_desc &d = bl[b];
            if (d.rank == 0) return;
            hp.colU[b].resize(2 * (size_t)d.rank);
            hp.colV[b].resize(2 * (size_t)d.rank);
            e4m3_column_scales(d.a, t.size(d.target), d.rank, d.lda, hp.colU[b].data());
            e4m3_column_scales(d.b, t.size(d.source), d.rank, d.ldb, hp.colV[b].data());
        });
    }
    // chunks: their rows are contiguous in the X fragments, padded once, at the chunk's end
    int64_t xf = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t node = hp.chunk_node[c];
        hmat::MRChunk m{};
        m.row_begin = (int32_t)t.begin[node];
        m.rows = (int32_t)t.size(node);
        m.nkb = (m.rows + KB - 1) / KB;
        m.leaf_base = (int32_t)hp.leaves.size();
        const std::vector<int32_t> lv = chunk_leaves(t, node);
        const std::vector<int32_t> pn = dense_partners(node);
        m.nleaf = (int32_t)lv.size();
        m.nsrc = (int32_t)pn.size();
        for (int32_t lf : lv) {
            hp.leaves.push_back(hmat::MRLeaf{(int32_t)t.begin[lf], (int32_t)t.size(lf)});
            hp.leaf_node.push_back(lf);
        }
        m.xoff = xf;
        xf += (int64_t)m.nkb * hp.ntmax;
        // one dense scale per partner box: the group of the dense blocks between the two (Def. 2.3
        // makes every pair of a leaf of the chunk and a leaf of a partner a dense block)
        m.dscale_base = (int32_t)hp.dscale.size();
        for (int32_t q : pn) hp.dscale.push_back(hp.sD[L == 0 ? 0 : st.find(lv[0], t.kid(q, 0))]);
        hp.chunks.push_back(m);
    }
    hp.x_frags = xf;
    // V units: per level-l source box s and 64-column group, at most kUnitChunks chunks each
    hp.colmap.assign(t.num_nodes, {});
    std::vector<int32_t> ubase(t.num_nodes, -1), nunit(t.num_nodes, 0), vcol(nb, -1);
    int64_t af = 0;
    for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
        std::vector<int32_t> boxes;
        for (int32_t i = 0; i < t.num_nodes; ++i)
            if (t.depth[i] == lvl) boxes.push_back(i);
        std::sort(boxes.begin(), boxes.end(), [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
        for (int32_t s : boxes) {
            auto &cm = hp.colmap[s];
            for (const int64_t b : st.by_source[s]) {
                vcol[b] = (int32_t)cm.size();
                for (int32_t k = 0; k < bl[b].rank; ++k) cm.emplace_back(b, k);
            }
            const int32_t W = (int32_t)cm.size();
            const int32_t ngroups = (W + 63) / 64;
            const int32_t c0 = cfirst[s], c1 = clast[s];
            const int32_t nu = (c1 - c0 + kUnitChunks - 1) / kUnitChunks;
            ubase[s] = (int32_t)hp.vunits.size();
            nunit[s] = nu;
            for (int32_t g = 0; g < ngroups; ++g) {
                const int32_t nm = std::min(4, (W - 64 * g + 15) / 16);
                const int32_t lo_off = (int32_t)(hp.vlo.size() / 64);
                if (hp.fp8)  // lo-scales of the group's 64 V columns (1 past the box's columns)
                    for (int32_t c = 0; c < 64; ++c) {
                        const int32_t col = 64 * g + c;
                        hp.vlo.push_back(col < W ? f16_pow2_code(hp.colV[cm[col].first][2 * cm[col].second + 1])
                                                 : f16_pow2_code(1.0));
                    }
                for (int32_t i = 0; i < nu; ++i) {
                    hmat::MRVUnit u{};
                    u.aoff = af;
                    u.lo_off = hp.fp8 ? lo_off : 0;
                    u.c0 = c0 + i * kUnitChunks;
                    u.nc = std::min(kUnitChunks, c1 - u.c0);
                    u.nm = nm;
                    u.poff = (int64_t)hp.vunits.size() * 64 * hp.ntmax * 16;
                    for (int32_t c = u.c0; c < u.c0 + u.nc; ++c) af += (int64_t)hp.chunks[c].nkb * nm;
                    hp.vunits.push_back(u);
                    hp.unit_node.push_back(s);
                    hp.unit_group.push_back(g);
                }
            }
        }
    }
    hp.v_frags = af;
    hp.part_floats = (int64_t)hp.vunits.size() * 64 * hp.ntmax * 16;
    // Launch order: the units of every level and column group that read the same
    // kUnitChunks chunks of X run next to each other (and, with the XCD-aware
    // numbering of the kernel, in one L2), so X is fetched from HBM about once
    // instead of once per level. A unit keeps its partial-sum slot (poff), which
    // the z items address by the unit's place in the level-ordered list.
    {
        std::vector<int32_t> perm(hp.vunits.size());
        for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int32_t)i;
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
            return hp.vunits[a].c0 / kUnitChunks < hp.vunits[b].c0 / kUnitChunks;
        });
        std::vector<hmat::MRVUnit> vu(perm.size());
        std::vector<int32_t> un(perm.size()), ug(perm.size());
        for (size_t i = 0; i < perm.size(); ++i) {
            vu[i] = hp.vunits[perm[i]];
            un[i] = hp.unit_node[perm[i]];
            ug[i] = hp.unit_group[perm[i]];
        }
        hp.vunits.swap(vu);
        hp.unit_node.swap(un);
        hp.unit_group.swap(ug);
    }
    // unit groups: up to four consecutive units over the same chunks (they share their X fragments)
    for (int32_t i = 0; i < (int32_t)hp.vunits.size();) {
        int32_t j = i + 1;
        while (j < (int32_t)hp.vunits.size() && j - i < 4 && hp.vunits[j].c0 == hp.vunits[i].c0 &&
               hp.vunits[j].nc == hp.vunits[i].nc)
            ++j;
        hp.ugroups.push_back(hmat::MRUnitGroup{i, j - i});
        i = j;
    }
    // z items: a block whose rank is a whole number of K-blocks is an item of its
    // own; the others of one target box, in its block order, are stacked into
    // shared K-blocks (a box whose stacked ranks add up to more than kMaxRankMR
    // continues in a further item)
    std::vector<int32_t> zfirst(t.num_nodes, 0), zcount(t.num_nodes, 0);
    int64_t zf = 0;
    for (int32_t a = 0; a < t.num_nodes && L >= 2; ++a) {
        if (st.by_target[a].empty()) continue;
        zfirst[a] = (int32_t)hp.zitems.size();
        hmat::MRZItem z{};
        auto finish = [&]() {
            z.zoff = zf;
            zf += (int64_t)((z.rows + KB - 1) / KB) * hp.ntmax;
            std::vector<int32_t> rm(z.rows);
            for (int32_t i = z.m0; i < z.m0 + z.nmem; ++i)
                for (int32_t j = 0; j < hp.zmembers[i].rank; ++j) rm[hp.zmembers[i].row + j] = i;
            hp.zrow_member.push_back(std::move(rm));
            hp.zitems.push_back(z);
        };
        z.m0 = (int32_t)hp.zmembers.size();
        std::vector<int64_t> order;  // the stacked blocks, then the whole-K-block ones
        for (const int64_t b : st.by_target[a])
            if (bl[b].rank % KB != 0) order.push_back(b);
        const size_t nstack = order.size();
        for (const int64_t b : st.by_target[a])
            if (bl[b].rank % KB == 0) order.push_back(b);
        for (size_t i = 0; i < order.size(); ++i) {
            const int64_t b = order[i];
            if (z.nmem > 0 && (i >= nstack || z.rows + bl[b].rank > kMaxRankMR)) {
                finish();
                z = hmat::MRZItem{};
                z.m0 = (int32_t)hp.zmembers.size();
            }
            const int32_t s = bl[b].source;
            hmat::MRZMember zm{};
            zm.ubase = ubase[s];
            zm.nu = nunit[s];
            zm.vcol = vcol[b];
            zm.rank = bl[b].rank;
            zm.scale = hp.sU[b] * hp.sV[b];
            zm.col_off = 0;
            zm.row = z.rows;
            if (hp.fp8) {
                zm.scale = 1.0f;
                zm.col_off = (int32_t)hp.zcol.size();
                for (int32_t j = 0; j < bl[b].rank; ++j) hp.zcol.push_back(hp.colU[b][2 * j] * hp.colV[b][2 * j]);
            }
            hp.zmembers.push_back(zm);
            hp.zmember_block.push_back(b);
            ++z.nmem;
            z.rows += bl[b].rank;
        }
        if (z.nmem > 0) finish();
        zcount[a] = (int32_t)hp.zitems.size() - zfirst[a];
    }
    hp.z_frags = zf;
    // U-phase segments per chunk, and row tiles per target leaf
    int64_t uf = 0;
    for (int32_t c = 0; c < nc; ++c) {
        hmat::MRChunk &m = hp.chunks[c];
        m.seg_base = (int32_t)hp.segs.size();
        int32_t seg_kb = 0;
        for (int32_t lvl = 1; lvl <= L - 1; ++lvl) {
            const int32_t a = hp.anc[(size_t)c * (cd + 1) + lvl];
            for (int32_t zi = zfirst[a]; zi < zfirst[a] + zcount[a]; ++zi) {
                const hmat::MRZItem &z = hp.zitems[zi];
                hmat::MRSeg sg{z.zoff, (z.rows + KB - 1) / KB, 0, zi, 0};
                seg_kb += sg.nkb;
                hp.segs.push_back(sg);
                hp.seg_chunk.push_back(-1);
            }
        }
        // x over the rows of each partner box (the sources of the dense blocks), contiguous, from
        // the X fragments of that chunk in contiguous row order
        const std::vector<int32_t> pn = dense_partners(hp.chunk_node[c]);
        for (int32_t ip = 0; ip < m.nsrc; ++ip) {
            const int32_t sc = L == 0 ? c : chunk_of[pn[ip]];
            const hmat::MRChunk &ms = hp.chunks[sc];
            hmat::MRSeg sg{ms.xoff, ms.nkb, 1, sc, ip};
            seg_kb += sg.nkb;
            hp.segs.push_back(sg);
            hp.seg_chunk.push_back(sc);
        }
        m.nseg = (int32_t)hp.segs.size() - m.seg_base;
        m.step_base = (int32_t)hp.ustep.size();
        m.nsteps = seg_kb;
        m.ulo_base = (int32_t)hp.ulo.size();
        m.nzsteps = 0;
        for (int32_t si = m.seg_base; si < m.seg_base + m.nseg; ++si) {
            const hmat::MRSeg &sg = hp.segs[si];
            if (sg.kind != 0) continue;
            m.nzsteps += sg.nkb;
            if (!hp.fp8) continue;
            const hmat::MRZItem &z = hp.zitems[sg.sidx];
            for (int32_t k = 0; k < sg.nkb * KB; ++k) {  // lo-scales of the item's U columns, K-block by K-block
                if (k >= z.rows) {
                    hp.ulo.push_back(f16_pow2_code(1.0));
                    continue;
                }
                const int32_t mi = hp.zrow_member[sg.sidx][k];
                hp.ulo.push_back(f16_pow2_code(hp.colU[hp.zmember_block[mi]][2 * (k - hp.zmembers[mi].row) + 1]));
            }
        }
        const int64_t bbytes = KB == 32 ? 2048 : 1024;
        for (int32_t si = m.seg_base; si < m.seg_base + m.nseg; ++si) {
            const hmat::MRSeg &sg = hp.segs[si];
            // B fragments: z fragments first, then X fragments, in one allocation;
            // scale rows likewise: one per z item, then one per chunk
            const int64_t base = sg.kind == 0 ? sg.src : hp.z_frags + sg.src;
            for (int32_t kb = 0; kb < sg.nkb; ++kb) {
                hmat::MRStep e;
                e.bofs = (base + (int64_t)kb * hp.ntmax) * bbytes;
                e.srow = sg.kind == 0 ? sg.sidx : (int32_t)hp.zitems.size() + sg.sidx;
                e.sleaf = sg.kind == 0 ? -1 : sg.leaf;
                e.lseg = si - m.seg_base;
                e.pad_ = 0;
                hp.ustep.push_back(e);
            }
        }
        // row tiles: the chunk's rows, contiguous, in four tiles per started 256
        // rows (so that a chunk of a few dozen rows still keeps the four waves of
        // a tile group busy), each a whole number of 16-row subtiles, at most 64;
        // a tile may hold rows of several target leaves
        const int32_t aim = 4 * ((m.rows + 255) / 256);  // tiles aimed at
        const int32_t th = std::min(64, ((m.rows + aim - 1) / aim + 15) / 16 * 16);
        for (int32_t r0 = 0; r0 < m.rows; r0 += th) {
            hmat::MRTile tl{};
            tl.aoff = uf;
            tl.chunk = c;
            tl.row0 = m.row_begin + r0;
            tl.rows = std::min(th, m.rows - r0);
            tl.nm = (tl.rows + 15) / 16;
            uf += (int64_t)seg_kb * tl.nm;
            hp.tiles.push_back(tl);
        }
    }
    hp.ud_frags = uf;
    // tile groups: up to four consecutive tiles of one chunk (they share the chunk's B sequence)
    for (int32_t i = 0; i < (int32_t)hp.tiles.size();) {
        int32_t j = i + 1;
        while (j < (int32_t)hp.tiles.size() && j - i < 4 && hp.tiles[j].chunk == hp.tiles[i].chunk) ++j;
        hp.tgroups.push_back(hmat::MRTileGroup{hp.tiles[i].chunk, i, j - i, 0});
        i = j;
    }
    return HMAT_OK;
}

template <class T>
inline T quant(float v, float scale, bool bf16) {
    if constexpr (sizeof(T) == 4) {
        (void)scale;
        (void)bf16;
        return v;
    } else {
        return quant16(v, 1.0f / scale, bf16);
    }
}

template <class T>
void fill_v_mr(const Tree &t, const hmat_block_desc *bl, const HostPlanMR &hp, T *out) {
    const int32_t vw = hp.vw, KB = hp.kb;
    parallel_for((int64_t)hp.vunits.size(), [&](int64_t ui) {
        const hmat::MRVUnit &u = hp.vunits[ui];
        const int32_t s = hp.unit_node[ui], g = hp.unit_group[ui];
        const auto &cm = hp.colmap[s];
        int64_t af = u.aoff;
        for (int32_t c = u.c0; c < u.c0 + u.nc; ++c) {
            const hmat::MRChunk &m = hp.chunks[c];
            for (int32_t kb = 0; kb < m.nkb; ++kb)
                for (int32_t ms = 0; ms < u.nm; ++ms) {
                    T *fr = out + (af + (int64_t)kb * u.nm + ms) * 64 * vw;
                    for (int32_t l = 0; l < 64; ++l) {
                        const int32_t col = 64 * g + 16 * ms + l % 16;
                        uint8_t hi[8] = {0, 0, 0, 0, 0, 0, 0, 0}, lo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                        for (int32_t e = 0; e < vw; ++e) {
                            const int32_t pr = kb * KB + vw * (l / 16) + e;  // the chunk's rows, contiguous
                            const int32_t gr = pr < m.rows ? m.row_begin + pr : -1;
                            float v = 0.0f, sc = 1.0f;
                            if (gr >= 0 && col < (int32_t)cm.size()) {
                                const int64_t b = cm[col].first;
                                const hmat_block_desc &d = bl[b];
                                v = d.b[(gr - t.begin[s]) + (int64_t)cm[col].second * d.ldb];
                                sc = hp.sV[b];
                                if (hp.fp8) {
                                    const float *cs = &hp.colV[b][2 * cm[col].second];
                                    e4m3_hilo(v, cs[0], cs[1], &hi[e], &lo[e]);
                                }
                            }
                            if (!hp.fp8) fr[l * vw + e] = quant<T>(v, sc, hp.bf16);
                        }
                        if (hp.fp8)  // 8 hi codes, then 8 lo codes
                            for (int32_t w = 0; w < 4; ++w) {
                                fr[l * vw + w] = (T)(hi[2 * w] | (hi[2 * w + 1] << 8));
                                fr[l * vw + 4 + w] = (T)(lo[2 * w] | (lo[2 * w + 1] << 8));
                            }
                    }
                }
            af += (int64_t)m.nkb * u.nm;
        }
    });
}

template <class T>
void fill_ud_mr(const Tree &t, const Structure &st, const hmat_block_desc *bl, const HostPlanMR &hp, T *out) {
    const int32_t vw = hp.vw, KB = hp.kb;
    parallel_for((int64_t)hp.tiles.size(), [&](int64_t ti) {
        const hmat::MRTile &tl = hp.tiles[ti];
        const hmat::MRChunk &m = hp.chunks[tl.chunk];
        // the target leaf of each of the tile's rows, as an index into the tile's target leaves
        std::vector<int32_t> tleaves, row_lt(tl.rows);
        for (int32_t r = 0, lf = -1; r < tl.rows; ++r) {
            while (lf + 1 < m.nleaf && tl.row0 + r >= hp.leaves[m.leaf_base + lf + 1].row_begin) ++lf;
            if (tleaves.empty() || tleaves.back() != hp.leaf_node[m.leaf_base + lf])
                tleaves.push_back(hp.leaf_node[m.leaf_base + lf]);
            row_lt[r] = (int32_t)tleaves.size() - 1;
        }
        int64_t af = tl.aoff;
        for (int32_t si = m.seg_base; si < m.seg_base + m.nseg; ++si) {
            const hmat::MRSeg &sg = hp.segs[si];
            const bool zseg = sg.kind == 0;
            // z segment: column kk is column kk - row of the member block holding
            // row kk of the z item; x segment: column kk is row kk of the source
            // chunk, a column of the dense block of the row's target leaf and the
            // source leaf holding it
            int32_t ncols = 0;
            std::vector<int32_t> col_ls, col_off;  // x: per column, the source leaf (index) and its column
            std::vector<int64_t> blk;               // x: per (target leaf, source leaf) of the tile, the block
            int32_t nls = 0;
            float dsc = 1.0f;
            if (zseg) {
                ncols = hp.zitems[sg.sidx].rows;
            } else {
                const hmat::MRChunk &ms = hp.chunks[hp.seg_chunk[si]];
                ncols = ms.rows;
                col_ls.resize(ncols);
                col_off.resize(ncols);
                for (int32_t k = 0, lf = 0; k < ncols; ++k) {
                    while (lf + 1 < ms.nleaf && ms.row_begin + k >= hp.leaves[ms.leaf_base + lf + 1].row_begin) ++lf;
                    col_ls[k] = lf;
                    col_off[k] = ms.row_begin + k - hp.leaves[ms.leaf_base + lf].row_begin;
                }
                nls = ms.nleaf;
                blk.resize((size_t)tleaves.size() * nls);
                for (size_t i = 0; i < tleaves.size(); ++i)
                    for (int32_t j = 0; j < nls; ++j)
                        blk[i * nls + j] = (t.L == 0) ? 0 : st.find(tleaves[i], hp.leaf_node[ms.leaf_base + j]);
                dsc = hp.sD[blk[0]];  // the same for every block of the pair of boxes
            }
            const bool hilo = hp.fp8 && zseg;
            for (int32_t kb = 0; kb < sg.nkb; ++kb)
                for (int32_t ms = 0; ms < tl.nm; ++ms) {
                    T *fr = out + (af + (int64_t)kb * tl.nm + ms) * 64 * vw;
                    for (int32_t l = 0; l < 64; ++l) {
                        const int32_t tr = 16 * ms + l % 16;
                        uint8_t hi[8] = {0, 0, 0, 0, 0, 0, 0, 0}, lo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                        for (int32_t e = 0; e < vw; ++e) {
                            const int32_t kk = kb * KB + vw * (l / 16) + e;
                            int64_t b = -1;
                            int32_t col = kk;
                            if (zseg && kk < ncols) {
                                const int32_t mi = hp.zrow_member[sg.sidx][kk];
                                b = hp.zmember_block[mi];
                                col = kk - hp.zmembers[mi].row;
                            }
                            const float sc = kk >= ncols ? 1.0f : zseg ? hp.sU[b] : dsc;
                            float v = 0.0f;
                            if (tr < tl.rows && kk < ncols) {
                                if (!zseg) {
                                    b = blk[(size_t)row_lt[tr] * nls + col_ls[kk]];
                                    col = col_off[kk];
                                }
                                const hmat_block_desc &d = bl[b];
                                v = d.a[(tl.row0 + tr - t.begin[d.target]) + (int64_t)col * d.lda];
                            }
                            if (hilo) {
                                if (kk < ncols) e4m3_hilo(v, hp.colU[b][2 * col], hp.colU[b][2 * col + 1], &hi[e], &lo[e]);
                            } else if (hp.dense_bf16 && !zseg) {
                                fr[l * vw + e] = (T)f32_to_bf16_rne(v * (1.0f / sc));  // BF16 of v / s_D
                            } else {
                                fr[l * vw + e] = quant<T>(v, sc, hp.bf16);
                            }
                        }
                        if (hilo)  // 8 hi codes, then 8 lo codes
                            for (int32_t w = 0; w < 4; ++w) {
                                fr[l * vw + w] = (T)(hi[2 * w] | (hi[2 * w + 1] << 8));
                                fr[l * vw + 4 + w] = (T)(lo[2 * w] | (lo[2 * w + 1] << 8));
                            }
                    }
                }
            af += (int64_t)sg.nkb * tl.nm;
        }
    });
}

void release(hmat_handle *h) {
    if (!h) return;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    for (void *p : h->dev_allocs) (void)hipFree(p);
    delete h;
}

bool fault_alloc_armed() {
    const char *e = std::getenv("HMAT_FAULT");
    return e && std::strcmp(e, "alloc") == 0;
}

hmat_status dev_alloc(hmat_handle *h, size_t bytes, void **p) {
    *p = nullptr;
    if (fault_alloc_armed()) return fail(HMAT_ERR_NOMEM, "injected device allocation failure (HMAT_FAULT=alloc)");
    if (h->dev_allocs.empty()) {
        const hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    const hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(HMAT_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes: out of memory");
    }
    if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    h->dev_allocs.push_back(*p);
    return HMAT_OK;
}

template <class V>
hmat_status upload(hmat_handle *h, const std::vector<V> &v, const V **dst) {
    void *p = nullptr;
    hmat_status s = dev_alloc(h, v.size() * sizeof(V), &p);
    if (s != HMAT_OK) return s;
    if (!v.empty()) {
        const hipError_t e = hipMemcpy(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *dst = static_cast<const V *>(p);
    return HMAT_OK;
}

template <class T>
hmat_status upload_panels(hmat_handle *h, const Tree &t, const Structure &st,
                          const hmat_block_desc *bl, const HostPlan &hp) {
    void *vdev = nullptr, *uddev = nullptr;
    hmat_status s = dev_alloc(h, hp.v_elems * sizeof(T), &vdev);
    if (s != HMAT_OK) return s;
    s = dev_alloc(h, hp.ud_elems * sizeof(T), &uddev);
    if (s != HMAT_OK) return s;
    try {
        if (hp.v_elems > 0) {
            std::vector<T> stage(hp.v_elems);
            fill_v<T>(t, st, bl, hp, stage.data(), 0);
            const hipError_t e = hipMemcpy(vdev, stage.data(), stage.size() * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        {
            std::vector<T> stage(hp.ud_elems);
            fill_ud<T>(t, st, bl, hp, stage.data());
            const hipError_t e = hipMemcpy(uddev, stage.data(), stage.size() * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
    } catch (const std::bad_alloc &) {
        return fail(HMAT_ERR_NOMEM, "host staging allocation failed");
    }
    h->plan.V = vdev;
    h->plan.UD = uddev;
    return HMAT_OK;
}


template <class T>
hmat_status upload_mr(hmat_handle *h, const Tree &t, const Structure &st, const hmat_block_desc *bl,
                      const HostPlanMR &hp) {
    hmat::DevPlanMR &p = h->mrp;
    const size_t frag = (size_t)64 * hp.vw * sizeof(T);  // A fragment bytes (1 KiB)
    const size_t bfrag = hp.kb == 32 ? 2048 : 1024;      // B fragment bytes
    void *q = nullptr;
    hmat_status s;
    if ((s = dev_alloc(h, (hp.z_frags + hp.x_frags) * bfrag, &q)) != HMAT_OK) return s;
    p.zpack = q;
    p.xpack = static_cast<char *>(q) + hp.z_frags * bfrag;
    if ((s = dev_alloc(h, hp.part_floats * 4, &q)) != HMAT_OK) return s;
    p.part = static_cast<float *>(q);
    if ((s = dev_alloc(h, (hp.zitems.size() + hp.chunks.size()) * hp.ntmax * 4, &q)) != HMAT_OK) return s;
    p.sz = static_cast<float *>(q);
    p.sx = p.sz + hp.zitems.size() * hp.ntmax;
    p.scales = p.sz;
    if ((s = upload(h, hp.dscale, &p.dscale)) != HMAT_OK) return s;
    if ((s = upload(h, hp.chunks, &p.chunks)) != HMAT_OK) return s;
    if ((s = upload(h, hp.vunits, &p.vunits)) != HMAT_OK) return s;
    if ((s = upload(h, hp.zitems, &p.zitems)) != HMAT_OK) return s;
    if ((s = upload(h, hp.zmembers, &p.zmembers)) != HMAT_OK) return s;
    if ((s = upload(h, hp.segs, &p.segs)) != HMAT_OK) return s;
    if ((s = upload(h, hp.tiles, &p.tiles)) != HMAT_OK) return s;
    if ((s = upload(h, hp.tgroups, &p.tgroups)) != HMAT_OK) return s;
    if ((s = upload(h, hp.ugroups, &p.ugroups)) != HMAT_OK) return s;
    if ((s = upload(h, hp.ustep, &p.ustep)) != HMAT_OK) return s;
    if (hp.fp8) {
        if ((s = upload(h, hp.vlo, &p.vlo)) != HMAT_OK) return s;
        if ((s = upload(h, hp.ulo, &p.ulo)) != HMAT_OK) return s;
        if ((s = upload(h, hp.zcol, &p.zcol)) != HMAT_OK) return s;
    }
    void *vdev = nullptr, *uddev = nullptr;
    if ((s = dev_alloc(h, hp.v_frags * frag, &vdev)) != HMAT_OK) return s;
    if ((s = dev_alloc(h, hp.ud_frags * frag, &uddev)) != HMAT_OK) return s;
    try {
        if (hp.v_frags > 0) {
            std::vector<T> stage((size_t)hp.v_frags * 64 * hp.vw);
            fill_v_mr<T>(t, bl, hp, stage.data());
            const hipError_t e = hipMemcpy(vdev, stage.data(), stage.size() * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        std::vector<T> stage((size_t)hp.ud_frags * 64 * hp.vw);
        fill_ud_mr<T>(t, st, bl, hp, stage.data());
        const hipError_t e = hipMemcpy(uddev, stage.data(), stage.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    } catch (const std::bad_alloc &) {
        return fail(HMAT_ERR_NOMEM, "host staging allocation failed");
    }
    p.V = vdev;
    p.UD = uddev;
    p.storage = h->storage;
    p.ntmax = hp.ntmax;
    p.num_chunks = (int32_t)hp.chunks.size();
    p.num_vunits = (int32_t)hp.vunits.size();
    p.num_zitems = (int32_t)hp.zitems.size();
    p.num_tiles = (int32_t)hp.tiles.size();
    p.num_tgroups = (int32_t)hp.tgroups.size();
    p.num_ugroups = (int32_t)hp.ugroups.size();
    p.max_nzsteps = 0;
    p.max_nseg = 0;
    p.max_nsteps = 0;
    p.max_chunk_rows = 0;
    for (const hmat::MRChunk &c : hp.chunks) {
        p.max_chunk_rows = std::max(p.max_chunk_rows, c.rows);
        p.max_nzsteps = std::max(p.max_nzsteps, c.nzsteps);
        p.max_nseg = std::max(p.max_nseg, c.nseg);
        p.max_nsteps = std::max(p.max_nsteps, c.nsteps);
    }
    if (hp.fp8 && (int64_t)p.max_nzsteps * 32 * 2 * 4 > 65536)
        return fail(HMAT_ERR_UNSUPPORTED, "FP8 form: a chunk's U lo-scale table exceeds the LDS budget");
    h->info.device_factor_bytes = (hp.v_frags + hp.ud_frags) * (int64_t)frag;
    h->info.workspace_bytes = (hp.x_frags + hp.z_frags) * (int64_t)bfrag + hp.part_floats * 4 +
                              (int64_t)(hp.chunks.size() + hp.zitems.size()) * hp.ntmax * 4;
    h->info.num_chunks = (int32_t)hp.chunks.size();
    return HMAT_OK;
}

// The blocks of K^T: (t, s) becomes (s, t); a low-rank block's U and V trade
// places; a dense block is copied transposed into `dense` (column-major, leading
// dimension |s|).
void transpose_blocks(const Tree &t, const hmat_block_desc *bl, int64_t nb, std::vector<hmat_block_desc> &out,
                      std::vector<float> &dense) {
    std::vector<int64_t> off(nb + 1, 0);
    for (int64_t b = 0; b < nb; ++b)
        off[b + 1] = off[b] + (bl[b].rank == 0 ? t.size(bl[b].target) * t.size(bl[b].source) : 0);
    dense.resize(off[nb]);
    out.resize(nb);
    parallel_for(nb, [&](int64_t b) {
        const hmat_block_desc &d = bl[b];
        hmat_block_desc &o = out[b];
        o = d;
        o.target = d.source;
        o.source = d.target;
        if (d.rank > 0) {
            o.a = d.b;
            o.lda = d.ldb;
            o.b = d.a;
            o.ldb = d.lda;
        } else {
            const int64_t m = t.size(d.target), n = t.size(d.source);
            float *dst = dense.data() + off[b];
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = 0; i < n; ++i) dst[i + j * n] = d.a[j + i * d.lda];
            o.a = dst;
            o.lda = n;
            o.b = nullptr;
            o.ldb = 0;
        }
    });
}

hmat_status create_impl(const hmat_tree_desc *tree, const hmat_block_desc *blocks, int64_t nb,
                        const hmat_options *opts, hmat_handle *h) {
    if (!opts) return fail(HMAT_ERR_INVALID_ARG, "options pointer is NULL");
    if (opts->storage < HMAT_STORE_FP32 || opts->storage > HMAT_STORE_FP8_F16D)
        return fail(HMAT_ERR_INVALID_ARG, "unknown storage form");
    if (opts->max_nrhs < 1) return fail(HMAT_ERR_INVALID_ARG, "max_nrhs must be >= 1");
    if (opts->device < 0) return fail(HMAT_ERR_INVALID_ARG, "device must be >= 0");
    if ((opts->flags & ~(HMAT_FLAG_FP64_ACCUM | HMAT_FLAG_TRANSPOSE)) != 0)
        return fail(HMAT_ERR_INVALID_ARG, "unknown option flags");
    const bool fp64 = (opts->flags & HMAT_FLAG_FP64_ACCUM) != 0;
    const int32_t acc_bytes = fp64 ? 8 : 4;
    Tree t;
    hmat_status s = analyse_tree(tree, t);
    if (s != HMAT_OK) return s;
    Structure st;
    s = validate_blocks(t, blocks, nb, st);
    if (s != HMAT_OK) return s;
    std::vector<hmat_block_desc> tblocks;  // K^T: the transposed blocks, and the transposed dense entries
    std::vector<float> tdense;
    if (opts->flags & HMAT_FLAG_TRANSPOSE) {
        transpose_blocks(t, blocks, nb, tblocks, tdense);
        blocks = tblocks.data();
        st = Structure();
        s = validate_blocks(t, blocks, nb, st);
        if (s != HMAT_OK) return s;
    }
    HostPlan hp;
    HostPlanMR hpm;
    const bool fp8 = opts->storage == HMAT_STORE_FP8 || opts->storage == HMAT_STORE_FP8_F16D;
    if (fp8 && (opts->max_nrhs < 2 || fp64))
        return fail(HMAT_ERR_UNSUPPORTED,
                    "the FP8 storage forms need a multi-RHS handle (max_nrhs > 1, no FP64 accumulation)");
    h->mr = opts->max_nrhs > 1 && !fp64;
    s = h->mr ? build_plan_mr(t, st, blocks, nb, opts->storage, opts->max_nrhs, hpm)
              : build_plan(t, st, blocks, nb, opts->storage, acc_bytes, hp);
    if (s != HMAT_OK) return s;

    h->device = opts->device;
    h->storage = opts->storage;
    h->max_nrhs = opts->max_nrhs;
    h->flags = opts->flags;
    for (int64_t b = 0; b < nb; ++b) h->max_rank = std::max(h->max_rank, blocks[b].rank);
    {
        // work estimates for the batched scheduler; kLatencyBytes prices one
        // round trip of a latency-bound reduction item in bytes of streaming
        constexpr float kLatencyBytes = 4096.0f;
        const float esz = opts->storage == HMAT_STORE_FP32 ? 4.0f : 2.0f;
        if (h->mr) {
            for (const hmat::MRZItem &z : hpm.zitems) h->max_zrows = std::max(h->max_zrows, z.rows);
            for (const hmat::MRChunk &c : hpm.chunks) {
                h->chunk_rows.push_back(c.rows);
                h->max_nseg = std::max(h->max_nseg, c.nseg);
            }
            // per unit group and tile group: the A fragments its waves stream (the B
            // sequence they share is read once), plus kGroupBytes for the latency of
            // its start (step table, first fragments) and end (y or partials)
            constexpr int64_t kGroupBytes = 32768;
            for (const hmat::MRUnitGroup &g : hpm.ugroups) {
                int64_t bytes = kGroupBytes;
                for (int32_t i = g.u0; i < g.u0 + g.count; ++i) {
                    const hmat::MRVUnit &u = hpm.vunits[i];
                    for (int32_t c = u.c0; c < u.c0 + u.nc; ++c) bytes += (int64_t)hpm.chunks[c].nkb * u.nm * 1024;
                }
                h->cost_src.push_back((float)bytes);
            }
            for (const hmat::MRTileGroup &g : hpm.tgroups) {
                int64_t bytes = kGroupBytes;
                for (int32_t i = g.tile0; i < g.tile0 + g.ntiles; ++i)
                    bytes += (int64_t)hpm.chunks[g.chunk].nsteps * hpm.tiles[i].nm * 1024;
                h->cost_tgt.push_back((float)bytes);
            }
            // partials read and B fragments written (one n-tile), plus a latency term: these small
            // items are bound by round trips, not bytes
            for (const hmat::MRZItem &z : hpm.zitems) {
                float c = (float)z.rows * 64 * 2 + kLatencyBytes;
                for (int32_t i = z.m0; i < z.m0 + z.nmem; ++i) c += (float)hpm.zmembers[i].nu * hpm.zmembers[i].rank * 64;
                h->cost_z1.push_back(c);
            }
        } else {
            for (const ChunkMeta &c : hp.chunks) {
                h->chunk_rows.push_back(c.rows);
                const int64_t ntile = (c.rows + hmat::kWave - 1) / hmat::kWave;
                h->cost_tgt.push_back((float)ntile * c.nq * hmat::kWave * hp.vw * esz);
            }
            for (const VTile &vt : hp.vtiles) {
                const int64_t nvec = (hp.chunks[vt.chunk].rows + hp.vw - 1) / hp.vw;
                h->cost_src.push_back((float)nvec * hmat::kWave * hp.vw * esz);
            }
            for (const ZItem &z : hp.z1) h->cost_z1.push_back((float)(z.nchunks + 1) * z.rank * 4 + kLatencyBytes);
            for (const ZItem2 &z : hp.z2) h->cost_z2.push_back((float)(z.nslices + 1) * z.rank * 4 + kLatencyBytes);
        }
    }
    hmat_info &in = h->info;
    in.n = t.n;
    in.leaf_depth = t.L;
    in.num_chunks = (int32_t)hp.chunks.size();
    int64_t elems = 0, nd = 0, nl = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t mt = t.size(blocks[b].target), ms = t.size(blocks[b].source);
        if (blocks[b].rank == 0) {
            elems += mt * ms;
            ++nd;
        } else {
            elems += (mt + ms) * blocks[b].rank;
            ++nl;
        }
    }
    in.num_dense_blocks = nd;
    in.num_lowrank_blocks = nl;
    in.stored_elements = elems;
    const int64_t esz = opts->storage == HMAT_STORE_FP32 ? 4 : 2;  // FP8 forms: a hi + lo byte pair
    int64_t scale_bytes = 0;
    if (opts->storage == HMAT_STORE_FP16_SCALED) scale_bytes = 4 * (nd + 2 * nl);
    if (fp8) {
        scale_bytes = 4 * nd;  // one per dense block, then s_j and s'_j per U and V column
        for (int64_t b = 0; b < nb; ++b) scale_bytes += 16 * (int64_t)blocks[b].rank;
    }
    in.factor_bytes = elems * esz + scale_bytes;
    in.device_factor_bytes = (hp.v_elems + hp.ud_elems) * esz;
    in.workspace_bytes = (hp.part_floats + hp.slice_floats + hp.zg_floats) * acc_bytes;
    in.storage = opts->storage;
    in.max_nrhs = opts->max_nrhs;
    in.flags = opts->flags;

    if (h->mr) {
        if (opts->storage != HMAT_STORE_FP32) return upload_mr<uint16_t>(h, t, st, blocks, hpm);
        return upload_mr<float>(h, t, st, blocks, hpm);
    }

    DevPlan &p = h->plan;
    p.storage = opts->storage;
    p.fp64 = fp64 ? 1 : 0;
    p.num_chunks = (int32_t)hp.chunks.size();
    p.num_vtiles = (int32_t)hp.vtiles.size();
    p.num_z1 = (int32_t)hp.z1.size();
    p.num_z2 = (int32_t)hp.z2.size();
    p.num_levels = std::max(t.L - 1, 0);
    p.lds_floats = hp.lds_floats;
    p.max_leaf_rows = hp.max_leaf_rows;

    h->ws_part_bytes = hp.part_floats * acc_bytes;
    h->ws_zg_bytes = hp.zg_floats * acc_bytes;
    h->ws_slice_bytes = hp.slice_floats * acc_bytes;
    void *ws = nullptr;
    if ((s = dev_alloc(h, hp.part_floats * acc_bytes, &ws)) != HMAT_OK) return s;
    p.part = ws;
    if ((s = dev_alloc(h, (hp.zg_floats + hp.slice_floats) * acc_bytes, &ws)) != HMAT_OK) return s;
    p.zg = ws;
    p.slice = static_cast<char *>(ws) + hp.zg_floats * acc_bytes;
    if ((s = upload(h, hp.chunks, &p.chunks)) != HMAT_OK) return s;
    {
        std::vector<int32_t> pb(hp.chunks.size());
        for (size_t c = 0; c < pb.size(); ++c) pb[c] = hp.chunks[c].part_base;
        if ((s = upload(h, pb, &p.pbase)) != HMAT_OK) return s;
    }
    if ((s = upload(h, hp.zsegs, &p.zsegs)) != HMAT_OK) return s;
    if ((s = upload(h, hp.dsegs, &p.dsegs)) != HMAT_OK) return s;
    if ((s = upload(h, hp.dscale, &p.dscale)) != HMAT_OK) return s;
    if ((s = upload(h, hp.vtiles, &p.vtiles)) != HMAT_OK) return s;
    if ((s = upload(h, hp.z1, &p.z1)) != HMAT_OK) return s;
    if ((s = upload(h, hp.z2, &p.z2)) != HMAT_OK) return s;
    if (opts->storage != HMAT_STORE_FP32)
        s = upload_panels<uint16_t>(h, t, st, blocks, hp);
    else
        s = upload_panels<float>(h, t, st, blocks, hp);
    return s;
}

// ---------------------------------------------------------------------------
// Construction of the block factors (hmat_compress): validation, block sets
// bounded by a workspace budget, the launches of hmat_compress.hip, and the
// copies into the caller's arrays.
// ---------------------------------------------------------------------------
struct DevMem {  // device allocations of one compress call, released on every exit
    std::vector<void *> ptrs;
    ~DevMem() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hmat_status alloc(size_t count, T **p) {
        *p = nullptr;
        if (fault_alloc_armed()) return fail(HMAT_ERR_NOMEM, "injected device allocation failure (HMAT_FAULT=alloc)");
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 256));
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            return fail(HMAT_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes: out of memory");
        }
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
        ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return HMAT_OK;
    }
    template <class T>
    hmat_status upload(const std::vector<T> &v, T **p) {
        hmat_status s = alloc(v.size(), p);
        if (s != HMAT_OK) return s;
        const hipError_t e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        return HMAT_OK;
    }
};

hmat_status hip_status(int e, const char *what) {
    if (e == 0) return HMAT_OK;
    return fail(HMAT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

constexpr int64_t kCompressSetFloats = int64_t(1) << 30;  // 4 GiB of float workspace per block set

int32_t sample_width(const Tree &t, const hmat_block_desc &d, int32_t oversample) {
    return (int32_t)std::min<int64_t>({(int64_t)d.rank + oversample, t.size(d.target), t.size(d.source)});
}

hmat_status compress_dense(const Tree &t, const hmat_block_desc *bl, const std::vector<int64_t> &ids,
                           const hmat::CKernel &ck, std::function<void()> &pending) {
    for (size_t i0 = 0; i0 < ids.size();) {
        DevMem mem;
        std::vector<hmat::CDense> db;
        std::vector<hmat::CTile> tiles;
        int64_t total = 0;
        size_t i1 = i0;
        for (; i1 < ids.size(); ++i1) {
            const hmat_block_desc &d = bl[ids[i1]];
            const int64_t ne = t.size(d.target) * t.size(d.source);
            if (i1 > i0 && total + ne > kCompressSetFloats) break;
            hmat::CDense c{t.begin[d.target], t.begin[d.source], (int32_t)t.size(d.target),
                           (int32_t)t.size(d.source), total};
            for (int64_t e = 0; e < ne; e += 256) tiles.push_back(hmat::CTile{(int32_t)db.size(), 0, e});
            db.push_back(c);
            total += ne;
        }
        hmat::CDense *ddb = nullptr;
        hmat::CTile *dtl = nullptr;
        float *out = nullptr;
        hmat_status s;
        if ((s = mem.upload(db, &ddb)) != HMAT_OK || (s = mem.upload(tiles, &dtl)) != HMAT_OK ||
            (s = mem.alloc((size_t)total, &out)) != HMAT_OK)
            return s;
        if ((s = hip_status(hmat::launch_compress_dense(ck, ddb, dtl, (int64_t)tiles.size(), out, nullptr),
                            "dense entries")) != HMAT_OK)
            return s;
        pending();
        auto host = std::make_shared<std::vector<float>>((size_t)total);
        if ((s = hip_status(hipMemcpy(host->data(), out, (size_t)total * 4, hipMemcpyDeviceToHost), "hipMemcpy")) !=
            HMAT_OK)
            return s;
        pending = [bl, &ids, db = std::move(db), host, i0, i1]() {
            for (size_t i = i0; i < i1; ++i) {
                const hmat_block_desc &d = bl[ids[i]];
                const hmat::CDense &c = db[i - i0];
                float *a = const_cast<float *>(d.a);
                for (int32_t j = 0; j < c.ms; ++j)
                    std::memcpy(a + (int64_t)j * d.lda, host->data() + c.off + (int64_t)j * c.mt, (size_t)c.mt * 4);
            }
        };
        i0 = i1;
    }
    return HMAT_OK;
}

// `pending` holds the copy of the last set's results into the caller's arrays:
// it runs once the next set's kernels are queued, so that the host copies
// overlap the GPU work; the caller runs what is left at the end.
hmat_status compress_lowrank(const Tree &t, const hmat_block_desc *bl, const std::vector<int64_t> &ids,
                             const hmat::CKernel &ck, int32_t oversample, uint64_t seed,
                             std::function<void()> &pending) {
    for (size_t i0 = 0; i0 < ids.size();) {
        DevMem mem;
        std::vector<hmat::CLowRank> lr;
        std::vector<hmat::CTile> ttiles, stiles;
        int64_t fl = 0, gl = 0;
        int32_t max_ell = 1;
        size_t i1 = i0;
        // Y and B^T, then the transforms, then U and V (contiguous, copied back in one piece)
        for (; i1 < ids.size(); ++i1) {
            const hmat_block_desc &d = bl[ids[i1]];
            const int64_t mt = t.size(d.target), ms = t.size(d.source);
            const int32_t ell = sample_width(t, d, oversample);
            const int64_t need = (mt + ms) * (ell + d.rank) + (int64_t)ell * std::max(ell, 2 * d.rank);
            if (i1 > i0 && fl + need > kCompressSetFloats) break;
            hmat::CLowRank c{};
            c.t0 = t.begin[d.target];
            c.s0 = t.begin[d.source];
            c.mt = (int32_t)mt;
            c.ms = (int32_t)ms;
            c.ell = ell;
            c.rank = d.rank;
            c.yoff = fl;
            c.boff = fl + mt * ell;
            c.toff = c.boff + ms * ell;
            fl = c.toff + (int64_t)ell * std::max(ell, 2 * d.rank);
            c.goff = gl;
            gl += (int64_t)ell * ell;
            for (int64_t r = 0; r < mt; r += 256) ttiles.push_back(hmat::CTile{(int32_t)lr.size(), 0, r});
            for (int64_t r = 0; r < ms; r += 256) stiles.push_back(hmat::CTile{(int32_t)lr.size(), 0, r});
            max_ell = std::max(max_ell, ell);
            lr.push_back(c);
        }
        const int64_t uv0 = fl;
        for (hmat::CLowRank &c : lr) {
            c.uoff = fl;
            c.voff = fl + (int64_t)c.mt * c.rank;
            fl = c.voff + (int64_t)c.ms * c.rank;
        }
        hmat::CLowRank *dlr = nullptr;
        hmat::CTile *dtt = nullptr, *dst = nullptr;
        float *fws = nullptr;
        double *gram = nullptr;
        hmat_status s;
        if ((s = mem.upload(lr, &dlr)) != HMAT_OK || (s = mem.upload(ttiles, &dtt)) != HMAT_OK ||
            (s = mem.upload(stiles, &dst)) != HMAT_OK || (s = mem.alloc((size_t)fl, &fws)) != HMAT_OK ||
            (s = mem.alloc((size_t)gl, &gram)) != HMAT_OK)
            return s;
        hmat::CWork w{dlr, fws, gram, seed, (max_ell + 15) / 16 * 16, max_ell};
        const int64_t nb = (int64_t)lr.size(), nt = (int64_t)ttiles.size(), ns = (int64_t)stiles.size();
        int e = hmat::launch_compress_sample(ck, w, dtt, nt, 0, nullptr);  // Y = K Omega
        for (int pass = 0; pass < 2 && !e; ++pass) {                       // Q: two SVQB passes over Y
            if (!(e = hmat::launch_compress_gram(w, nb, 0, nullptr)) && !(e = hmat::launch_compress_eig(w, nb, 0, nullptr)))
                e = hmat::launch_compress_apply(w, dtt, nt, 0, nullptr);
        }
        if (!e) e = hmat::launch_compress_sample(ck, w, dst, ns, 1, nullptr);  // B^T = K^T Q
        if (!e) e = hmat::launch_compress_gram(w, nb, 1, nullptr);             // B B^T
        if (!e) e = hmat::launch_compress_eig(w, nb, 1, nullptr);              // M_U, M_V
        if (!e) e = hmat::launch_compress_apply(w, dtt, nt, 1, nullptr);       // U = Q M_U
        if (!e) e = hmat::launch_compress_apply(w, dst, ns, 2, nullptr);       // V = B^T M_V
        if ((s = hip_status(e, "compress launch")) != HMAT_OK) return s;
        // the previous set's factors go to the caller's arrays while this set runs on the GPU
        pending();
        auto host = std::make_shared<std::vector<float>>((size_t)(fl - uv0));
        if ((s = hip_status(hipMemcpy(host->data(), fws + uv0, host->size() * 4, hipMemcpyDeviceToHost),
                            "hipMemcpy")) != HMAT_OK)
            return s;
        pending = [bl, &ids, lr = std::move(lr), host, i0, i1, uv0]() {
            for (size_t i = i0; i < i1; ++i) {
                const hmat_block_desc &d = bl[ids[i]];
                const hmat::CLowRank &c = lr[i - i0];
                float *a = const_cast<float *>(d.a), *b = const_cast<float *>(d.b);
                for (int32_t j = 0; j < c.rank; ++j) {
                    std::memcpy(a + (int64_t)j * d.lda, host->data() + (c.uoff - uv0) + (int64_t)j * c.mt,
                                (size_t)c.mt * 4);
                    std::memcpy(b + (int64_t)j * d.ldb, host->data() + (c.voff - uv0) + (int64_t)j * c.ms,
                                (size_t)c.ms * 4);
                }
            }
        };
        i0 = i1;
    }
    return HMAT_OK;
}

hmat_status compress_impl(const hmat_tree_desc *tree, const float *points, const hmat_block_desc *blocks,
                          int64_t nb, const hmat_compress_options *opts) {
    if (!opts) return fail(HMAT_ERR_INVALID_ARG, "options pointer is NULL");
    if (!points) return fail(HMAT_ERR_INVALID_ARG, "points pointer is NULL");
    if (opts->reserved != 0) return fail(HMAT_ERR_INVALID_ARG, "options reserved field must be 0");
    if (opts->kernel != HMAT_KERNEL_LOG && opts->kernel != HMAT_KERNEL_INV)
        return fail(HMAT_ERR_INVALID_ARG, "unknown kernel function");
    if (opts->dim < 1 || opts->dim > 3) return fail(HMAT_ERR_INVALID_ARG, "dim must be in [1, 3]");
    if (!std::isfinite(opts->diag)) return fail(HMAT_ERR_INVALID_ARG, "diag must be finite");
    if (opts->oversample < 0 || opts->oversample > hmat::kCompressMaxL)
        return fail(HMAT_ERR_INVALID_ARG, "oversample must be in [0, 96]");
    Tree t;
    hmat_status s = analyse_tree(tree, t);
    if (s != HMAT_OK) return s;
    Structure st;
    if ((s = validate_blocks(t, blocks, nb, st)) != HMAT_OK) return s;
    std::vector<int64_t> dense, lowrank;
    for (int64_t b = 0; b < nb; ++b) {
        if (blocks[b].rank == 0) {
            dense.push_back(b);
            continue;
        }
        if (sample_width(t, blocks[b], opts->oversample) > hmat::kCompressMaxL)
            return fail(HMAT_ERR_UNSUPPORTED, "block " + std::to_string(b) + ": min(rank + oversample, |t|, |s|) exceeds 96");
        lowrank.push_back(b);
    }
    for (int64_t i = 0; i < t.n * opts->dim; ++i)
        if (!std::isfinite(points[i])) return fail(HMAT_ERR_INVALID_ARG, "points must be finite");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opts->device < 0 || opts->device >= ndev)
        return fail(HMAT_ERR_INVALID_ARG, "device ordinal out of range");
    if ((s = hip_status(hipSetDevice(opts->device), "hipSetDevice")) != HMAT_OK) return s;
    DevMem mem;
    float *dpts = nullptr;
    if ((s = mem.upload(std::vector<float>(points, points + t.n * opts->dim), &dpts)) != HMAT_OK) return s;
    const hmat::CKernel ck{dpts, opts->dim, opts->kernel, opts->diag, 0};
    std::function<void()> pending = [] {};
    if ((s = compress_dense(t, blocks, dense, ck, pending)) != HMAT_OK) return s;
    if ((s = compress_lowrank(t, blocks, lowrank, ck, opts->oversample, opts->seed, pending)) != HMAT_OK) return s;
    pending();
    return HMAT_OK;
}

}  // namespace

extern "C" {

const char *hmat_status_string(hmat_status s) {
    switch (s) {
    case HMAT_OK: return "HMAT_OK";
    case HMAT_ERR_INVALID_ARG: return "HMAT_ERR_INVALID_ARG";
    case HMAT_ERR_BAD_TREE: return "HMAT_ERR_BAD_TREE";
    case HMAT_ERR_BAD_BLOCKS: return "HMAT_ERR_BAD_BLOCKS";
    case HMAT_ERR_UNSUPPORTED: return "HMAT_ERR_UNSUPPORTED";
    case HMAT_ERR_NOMEM: return "HMAT_ERR_NOMEM";
    case HMAT_ERR_DEVICE: return "HMAT_ERR_DEVICE";
    }
    return "HMAT_ERR_UNKNOWN";
}

const char *hmat_last_error(void) { return t_err.c_str(); }

hmat_status hmat_create(const hmat_tree_desc *tree, const hmat_block_desc *blocks, int64_t num_blocks,
                        const hmat_options *opts, hmat_t *out) {
    if (!out) return fail(HMAT_ERR_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    t_err.clear();
    hmat_handle *h = nullptr;
    try {
        h = new hmat_handle();
        const hmat_status s = create_impl(tree, blocks, num_blocks, opts, h);
        if (s != HMAT_OK) {
            release(h);
            return s;
        }
    } catch (const std::bad_alloc &) {
        release(h);
        return fail(HMAT_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        release(h);
        return fail(HMAT_ERR_INVALID_ARG, std::string("internal error: ") + e.what());
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(h);
    }
    *out = h;
    return HMAT_OK;
}

hmat_status hmat_compress(const hmat_tree_desc *tree, const float *points, const hmat_block_desc *blocks,
                          int64_t num_blocks, const hmat_compress_options *opts) {
    t_err.clear();
    try {
        return compress_impl(tree, points, blocks, num_blocks, opts);
    } catch (const std::bad_alloc &) {
        return fail(HMAT_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(HMAT_ERR_INVALID_ARG, std::string("internal error: ") + e.what());
    }
}

hmat_status hmat_destroy(hmat_t h) {
    if (!h) return HMAT_OK;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_live.count(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown or already destroyed handle");
        if (h->batch_refs > 0) return fail(HMAT_ERR_INVALID_ARG, "handle is still used by a batch");
        g_live.erase(h);
    }
    if (!h->dev_allocs.empty()) (void)hipSetDevice(h->device);
    release(h);
    return HMAT_OK;
}

hmat_status hmat_get_info(hmat_t h, hmat_info *info) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown handle");
    if (!info) return fail(HMAT_ERR_INVALID_ARG, "info pointer is NULL");
    *info = h->info;
    return HMAT_OK;
}

static hmat_status record_event(hmat_handle *h, hipStream_t stream) {
    if (h->events_used == h->events.size()) {
        hipEvent_t e;
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(err));
        h->events.push_back(e);
    }
    const hipError_t err = hipEventRecord(h->events[h->events_used++], stream);
    if (err != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(err));
    return HMAT_OK;
}

struct MarkCtx {
    hmat_handle *h;
    hipStream_t st;
    hmat_status err;
};

static void mark_phase(void *ctx, int) {
    MarkCtx *m = static_cast<MarkCtx *>(ctx);
    if (m->err == HMAT_OK) m->err = record_event(m->h, m->st);
}

// Argument checks shared by the product entry points; makes the handle's device current.
static hmat_status matvec_prologue(hmat_t h, int32_t nrhs, const float *x, int64_t ldx, const float *y,
                                   int64_t ldy) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown handle");
    const int64_t n = h->info.n;
    if (nrhs < 1 || nrhs > h->max_nrhs) return fail(HMAT_ERR_INVALID_ARG, "nrhs out of [1, max_nrhs]");
    if (!x || !y) return fail(HMAT_ERR_INVALID_ARG, "x and y must not be NULL");
    if (ldx < n || ldy < n) return fail(HMAT_ERR_INVALID_ARG, "leading dimension smaller than n");
    const uintptr_t xb = (uintptr_t)x, xe = (uintptr_t)(x + (nrhs - 1) * ldx + n);
    const uintptr_t yb = (uintptr_t)y, ye = (uintptr_t)(y + (nrhs - 1) * ldy + n);
    if (xb < ye && yb < xe) return fail(HMAT_ERR_INVALID_ARG, "x and y overlap");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
        const hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    return HMAT_OK;
}

hmat_status hmat_matvec(hmat_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx, float beta,
                        float *y, int64_t ldy, void *stream) {
    const hmat_status ps = matvec_prologue(h, nrhs, x, ldx, y, ldy);
    if (ps != HMAT_OK) return ps;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (h->mr) {
        for (int32_t c0 = 0; c0 < nrhs; c0 += 128) {
            const int32_t kk = std::min<int32_t>(128, nrhs - c0);
            MarkCtx mc{h, st, HMAT_OK};
            const int e = hmat::launch_mr(h->mrp, kk, alpha, x + c0 * ldx, ldx, beta, y + c0 * ldy, ldy, st,
                                          h->timing ? mark_phase : nullptr, &mc);
            if (mc.err != HMAT_OK) return mc.err;
            if (e != 0) return fail(HMAT_ERR_DEVICE, std::string("multi-RHS launch: ") + hipGetErrorString((hipError_t)e));
            if (h->timing) h->timed_calls++;
        }
        return HMAT_OK;
    }
    const DevPlan &p = h->plan;
    for (int32_t c = 0; c < nrhs; ++c) {
        const float *xc = x + c * ldx;
        float *yc = y + c * ldy;
        hmat_status s;
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        int e = 0;
        if (p.num_vtiles > 0 && (e = hmat::launch_vphase(p, xc, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("V-phase launch: ") + hipGetErrorString((hipError_t)e));
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if (p.num_z1 > 0 && (e = hmat::launch_zfinish(p, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("z-finish launch: ") + hipGetErrorString((hipError_t)e));
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if ((e = hmat::launch_uphase(p, xc, yc, alpha, beta, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("U-phase launch: ") + hipGetErrorString((hipError_t)e));
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if (h->timing) h->timed_calls++;
    }
    return HMAT_OK;
}

hmat_status hmat_matvec_noalloc(hmat_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx, float beta,
                                float *y, int64_t ldy, void *stream) {
    const hmat_status ps = matvec_prologue(h, nrhs, x, ldx, y, ldy);
    if (ps != HMAT_OK) return ps;
    if (h->mr)
        return fail(HMAT_ERR_UNSUPPORTED,
                    "hmat_matvec_noalloc: multi-RHS handles are not supported (create with max_nrhs = 1)");
    auto round256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t part_bytes = round256(h->ws_part_bytes);
    const int64_t need = part_bytes + round256(h->ws_zg_bytes + h->ws_slice_bytes);
    if (need > HMAT_NOALLOC_SCRATCH_BYTES)
        return fail(HMAT_ERR_UNSUPPORTED, "hmat_matvec_noalloc: the handle's workspace takes " + std::to_string(need) +
                                              " bytes, more than the " + std::to_string(HMAT_NOALLOC_SCRATCH_BYTES) +
                                              "-byte scratch");
    void *base = nullptr;
    int e = hmat::scratch_address(h->device, &base);
    if (e != 0)
        return fail(HMAT_ERR_DEVICE, std::string("scratch address (hipGetSymbolAddress): ") +
                                         hipGetErrorString((hipError_t)e));
    // the handle's plan with its workspace pointers moved into the scratch
    DevPlan p = h->plan;
    p.part = base;
    p.zg = static_cast<char *>(base) + part_bytes;
    p.slice = static_cast<char *>(p.zg) + h->ws_zg_bytes;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t c = 0; c < nrhs; ++c) {
        const float *xc = x + c * ldx;
        float *yc = y + c * ldy;
        if (p.num_vtiles > 0 && (e = hmat::launch_vphase(p, xc, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("V-phase launch: ") + hipGetErrorString((hipError_t)e));
        if (p.num_z1 > 0 && (e = hmat::launch_zfinish(p, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("z-finish launch: ") + hipGetErrorString((hipError_t)e));
        if ((e = hmat::launch_uphase(p, xc, yc, alpha, beta, st)) != 0)
            return fail(HMAT_ERR_DEVICE, std::string("U-phase launch: ") + hipGetErrorString((hipError_t)e));
    }
    return HMAT_OK;
}

hmat_status hmat_set_timing(hmat_t h, int32_t enable) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown handle");
    if (h->events_used > 0) {
        const hipError_t e = hipEventSynchronize(h->events[h->events_used - 1]);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    }
    h->timing = enable != 0;
    h->events_used = 0;
    h->timed_calls = 0;
    for (double &m : h->ms) m = 0.0;
    return HMAT_OK;
}

hmat_status hmat_get_timing(hmat_t h, double ms[HMAT_NUM_PHASES], int64_t *calls) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown handle");
    if (!ms || !calls) return fail(HMAT_ERR_INVALID_ARG, "output pointers must not be NULL");
    const size_t per = HMAT_NUM_PHASES + 1;
    const size_t sets = h->events_used / per;
    if (sets > 0) {
        const hipError_t e = hipEventSynchronize(h->events[sets * per - 1]);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    }
    for (size_t k = 0; k < sets; ++k)
        for (int ph = 0; ph < HMAT_NUM_PHASES; ++ph) {
            float t = 0.0f;
            const hipError_t e = hipEventElapsedTime(&t, h->events[k * per + ph], h->events[k * per + ph + 1]);
            if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
            h->ms[ph] += t;
        }
    h->events_used = 0;
    for (int ph = 0; ph < HMAT_NUM_PHASES; ++ph) ms[ph] = h->ms[ph];
    *calls = h->timed_calls;
    return HMAT_OK;
}

hmat_status hmat_probe_bandwidth(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream) {
    if (!src || !dst) return fail(HMAT_ERR_INVALID_ARG, "src and dst must not be NULL");
    if (bytes <= 0 || bytes % 16 != 0) return fail(HMAT_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
    if (mode != 0 && mode != 1) return fail(HMAT_ERR_INVALID_ARG, "mode must be 0 (read) or 1 (copy)");
    const int e = hmat::launch_probe(src, dst, bytes, mode, stream);
    if (e != 0) return fail(HMAT_ERR_DEVICE, std::string("probe launch: ") + hipGetErrorString((hipError_t)e));
    return HMAT_OK;
}

}  // extern "C"
