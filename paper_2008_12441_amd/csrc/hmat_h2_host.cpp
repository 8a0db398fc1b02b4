// Host side of the H^2-matrix-vector product: validation of the tree, the
// nested bases and the Def. 2.3 block set, the device layout (hmat_h2_internal.h),
// host-side quantisation, device memory, launches and timing. The C ABI is
// declared in include/hmat_h2.h.
#include "hmat_h2.h"
#include "hmat_h2_internal.h"
#include "hmat_handle.h"
#include "hmat_host_quant.h"
#include "hmat_structure.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

struct hmat_h2_handle {
    int32_t device = 0;
    int32_t storage = 0;
    hmat_h2_info info{};
    hmat::DevPlanH2 plan{};
    std::vector<int32_t> level_first, level_count;  // nodes above the chunks, per depth (index = depth)
    std::vector<void *> dev_allocs;
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    double ms[HMAT_NUM_PHASES] = {0, 0, 0};
    int64_t timed_calls = 0;
};

namespace {

using hmat::DSeg;
using hmat::H2Chunk;
using hmat::H2Leaf;
using hmat::H2Node;
using hmat::H2Term;
using hmat::Structure;
using hmat::Tree;

std::mutex g_mu;
std::unordered_set<const hmat_h2_handle *> g_live;

hmat_status fail(hmat_status s, const std::string &msg) { return hmat::set_error(s, msg); }

bool is_live(const hmat_h2_handle *h) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_live.count(h) != 0;
}

void release(hmat_h2_handle *h) {
    if (!h) return;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    for (void *p : h->dev_allocs) (void)hipFree(p);
    delete h;
}

hmat_status dev_alloc(hmat_h2_handle *h, size_t bytes, void **p) {
    *p = nullptr;
    const char *fe = std::getenv("HMAT_FAULT");
    if (fe && std::strcmp(fe, "alloc") == 0)
        return fail(HMAT_ERR_NOMEM, "injected device allocation failure (HMAT_FAULT=alloc)");
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
hmat_status upload(hmat_h2_handle *h, const V *data, size_t count, const V **dst) {
    void *p = nullptr;
    hmat_status s = dev_alloc(h, count * sizeof(V), &p);
    if (s != HMAT_OK) return s;
    if (count > 0) {
        const hipError_t e = hipMemcpy(p, data, count * sizeof(V), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *dst = static_cast<const V *>(p);
    return HMAT_OK;
}

template <class V>
hmat_status upload(hmat_h2_handle *h, const std::vector<V> &v, const V **dst) {
    return upload(h, v.data(), v.size(), dst);
}

constexpr int32_t kMaxLdsFloats = hmat::kMaxLdsBytes / 4;

// The leaves below a chunk node: its children, or the node itself when the root is a leaf.
std::vector<int32_t> chunk_leaves(const Tree &t, int32_t node) {
    std::vector<int32_t> v;
    if (t.L == 0) v.push_back(node);
    else
        for (int32_t j = 0; j < t.nkids(node); ++j) v.push_back(t.kid(node, j));
    return v;
}

// Per stored array: a power-of-two scale and its codes (FP16 form), or the values (FP32).
struct Quant {
    bool f16 = false;
    float scale(const float *a, int64_t rows, int64_t cols, int64_t ld, bool *finite) const {
        const float am = hmat::col_major_amax(a, rows, cols, ld, finite);
        return f16 ? hmat::pow2_scale_f16(am) : 1.0f;
    }
};

// Host-side layout before upload.
struct H2Host {
    int32_t vw = 4;
    std::vector<int32_t> chunk_node;
    std::vector<H2Chunk> chunks;
    std::vector<H2Leaf> leaves;
    std::vector<int32_t> leaf_node;      // node id of every leaf entry
    std::vector<DSeg> dsegs;
    std::vector<float> dscale;
    std::vector<H2Node> nodes;
    std::vector<H2Term> terms;
    std::vector<int32_t> xh;             // per node: workspace offset of x^ (-1 without a basis)
    int64_t ws_half = 0;
    // small matrices: (destination offset, source, rows, cols, ld, transpose, scale)
    struct SmallMat {          // stored by rows: row r at off + r * sld, entries [0, cols), zeros to sld
        int64_t off;
        const float *src;          // the given matrix (column-major, ld)
        int32_t rows, cols;        // of the stored matrix
        int32_t sld;
        int64_t ld;
        bool transpose;            // stored = given^T
        float scale;
    };
    std::vector<SmallMat> small;
    int64_t small_elems = 0;
    int64_t v_elems = 0, ud_elems = 0;
    int64_t stored = 0, leaf_kernel_elems = 0;
    int32_t lds_b = 0, kmax = 0;
};

hmat_status validate(const Tree &t, const hmat_h2_basis *bases, const hmat_h2_block *blocks, int64_t nb,
                     Structure &st) {
    if (!bases) return fail(HMAT_ERR_INVALID_ARG, "bases pointer is NULL");
    if (!blocks) return fail(HMAT_ERR_INVALID_ARG, "blocks pointer is NULL");
    if (nb < 1) return fail(HMAT_ERR_INVALID_ARG, "num_blocks must be >= 1");
    const bool has_bases = t.L >= 2;
    for (int32_t a = 0; a < t.num_nodes; ++a) {
        const hmat_h2_basis &b = bases[a];
        const std::string id = "basis of node " + std::to_string(a);
        if (b.reserved != 0) return fail(HMAT_ERR_INVALID_ARG, id + ": reserved field must be 0");
        const bool want = has_bases && a != 0;
        if (!want) {
            if (b.rank != 0)
                return fail(HMAT_ERR_INVALID_ARG, id + ": must have rank 0 (the root, or a tree without low-rank blocks)");
            continue;
        }
        if (b.rank < 1) return fail(HMAT_ERR_INVALID_ARG, id + ": every non-root node needs a basis (rank >= 1)");
        if (b.rank > HMAT_H2_MAX_RANK)
            return fail(HMAT_ERR_UNSUPPORTED, id + ": rank above HMAT_H2_MAX_RANK (" +
                                                  std::to_string(HMAT_H2_MAX_RANK) + ")");
        if (t.leaf(a)) {
            if (!b.u || !b.v) return fail(HMAT_ERR_INVALID_ARG, id + ": a leaf needs U and V");
            if (b.ldu < t.size(a) || b.ldv < t.size(a))
                return fail(HMAT_ERR_INVALID_ARG, id + ": ldu and ldv must be >= |t|");
        }
        if (t.parent[a] != 0) {   // the parent has a basis
            if (!b.e || !b.f) return fail(HMAT_ERR_INVALID_ARG, id + ": transfers E and F are NULL");
            if (b.lde < b.rank || b.ldf < b.rank) return fail(HMAT_ERR_INVALID_ARG, id + ": lde and ldf must be >= k_t");
        }
    }
    // the block set's shape, through the H-matrix validation (a coupling block
    // stands in as a rank-1 block with the sizes of (t, s))
    std::vector<hmat_block_desc> shadow(nb);
    for (int64_t b = 0; b < nb; ++b) {
        const hmat_h2_block &d = blocks[b];
        const std::string id = "block " + std::to_string(b);
        if (d.reserved != 0) return fail(HMAT_ERR_INVALID_ARG, id + ": reserved field must be 0");
        if (d.target < 0 || d.target >= t.num_nodes || d.source < 0 || d.source >= t.num_nodes)
            return fail(HMAT_ERR_INVALID_ARG, id + ": node id out of range");
        if (d.kind != 0 && d.kind != 1) return fail(HMAT_ERR_INVALID_ARG, id + ": kind must be 0 (dense) or 1 (coupling)");
        if (!d.a) return fail(HMAT_ERR_INVALID_ARG, id + ": matrix pointer is NULL");
        const int64_t mt = t.size(d.target), ms = t.size(d.source);
        if (d.kind == 0 && d.lda < mt) return fail(HMAT_ERR_INVALID_ARG, id + ": lda < |t|");
        if (d.kind == 1) {
            if (!has_bases) return fail(HMAT_ERR_BAD_BLOCKS, id + ": a tree with leaf depth < 2 has no low-rank blocks");
            if (d.lda < bases[d.target].rank) return fail(HMAT_ERR_INVALID_ARG, id + ": lda < k_t");
        }
        hmat_block_desc &s = shadow[b];
        s.target = d.target;
        s.source = d.source;
        s.rank = d.kind == 1 ? 1 : 0;
        s.reserved = 0;
        s.a = d.a;
        s.lda = mt;
        s.b = d.a;
        s.ldb = ms;
    }
    return hmat::validate_blocks(t, shadow.data(), nb, st);
}

hmat_status build(const Tree &t, const Structure &st, const hmat_h2_basis *bases, const hmat_h2_block *bl,
                  int64_t nb, int32_t storage, H2Host &hp) {
    const int32_t vw = storage == HMAT_STORE_FP32 ? 4 : 8;
    hp.vw = vw;
    const Quant qz{storage == HMAT_STORE_FP16_SCALED};
    const int32_t L = t.L;
    const int32_t cd = std::max(L - 1, 0);
    auto rank = [&](int32_t a) { return bases[a].rank; };
    bool finite = true;
    // workspace: x^ (and y^) of every node with a basis
    hp.xh.assign(t.num_nodes, -1);
    for (int32_t a = 0; a < t.num_nodes; ++a) {
        hp.kmax = std::max(hp.kmax, rank(a));
        if (rank(a) > 0 && !t.leaf(a)) {  // a leaf's x^ and y^ live in the leaf kernels' LDS only
            hp.xh[a] = (int32_t)hp.ws_half;
            hp.ws_half += rank(a);
        }
    }
    if (hp.ws_half >= INT32_MAX / 2) return fail(HMAT_ERR_UNSUPPORTED, "workspace too large");
    auto add_small = [&](const float *src, int32_t rows, int32_t cols, int64_t ld, bool transpose) {
        H2Host::SmallMat m;
        m.off = hp.small_elems;
        m.src = src;
        m.rows = transpose ? cols : rows;  // rows of the stored matrix
        m.cols = transpose ? rows : cols;
        m.sld = (m.cols + vw - 1) / vw * vw;
        m.ld = ld;
        m.transpose = transpose;
        m.scale = qz.scale(src, rows, cols, ld, &finite);
        hp.small.push_back(m);
        hp.small_elems += (int64_t)m.rows * m.sld;
        hp.stored += (int64_t)rows * cols;
        return hp.small.size() - 1;
    };
    // transfers of every node whose parent has a basis: E_t as given, F_t transposed
    std::vector<int64_t> e_idx(t.num_nodes, -1), ft_idx(t.num_nodes, -1);
    for (int32_t a = 1; a < t.num_nodes; ++a) {
        if (rank(a) == 0 || rank(t.parent[a]) == 0) continue;
        const hmat_h2_basis &b = bases[a];
        e_idx[a] = (int64_t)add_small(b.e, b.rank, rank(t.parent[a]), b.lde, false);
        ft_idx[a] = (int64_t)add_small(b.f, b.rank, rank(t.parent[a]), b.ldf, true);
    }
    // couplings
    std::vector<int64_t> s_idx(nb, -1);
    for (int64_t b = 0; b < nb; ++b)
        if (bl[b].kind == 1)
            s_idx[b] = (int64_t)add_small(bl[b].a, rank(bl[b].target), rank(bl[b].source), bl[b].lda, false);
    auto term_of_coupling = [&](int64_t b) {
        const H2Host::SmallMat &m = hp.small[s_idx[b]];
        return H2Term{(int32_t)m.off, hp.xh[bl[b].source], rank(bl[b].source), 0, m.scale, m.sld};
    };
    auto term_of_parent = [&](int32_t a) {
        const H2Host::SmallMat &m = hp.small[e_idx[a]];
        return H2Term{(int32_t)m.off, hp.xh[t.parent[a]], rank(t.parent[a]), 1, m.scale, m.sld};
    };
    // nodes above the chunks, by depth
    for (int32_t d = 1; d <= L - 2; ++d)
        for (int32_t a = 0; a < t.num_nodes; ++a) {
            if (t.depth[a] != d) continue;
            H2Node nd{};
            nd.k = rank(a);
            nd.xh = hp.xh[a];
            nd.up_base = (int32_t)hp.terms.size();
            for (int32_t j = 0; j < t.nkids(a); ++j) {
                const int32_t c = t.kid(a, j);
                const H2Host::SmallMat &m = hp.small[ft_idx[c]];
                hp.terms.push_back(H2Term{(int32_t)m.off, hp.xh[c], rank(c), 0, m.scale, m.sld});
            }
            nd.nup = (int32_t)hp.terms.size() - nd.up_base;
            nd.term_base = (int32_t)hp.terms.size();
            if (t.parent[a] > 0) hp.terms.push_back(term_of_parent(a));
            for (const int64_t b : st.by_target[a]) hp.terms.push_back(term_of_coupling(b));
            nd.nterm = (int32_t)hp.terms.size() - nd.term_base;
            hp.nodes.push_back(nd);
        }
    // chunks and their leaves
    for (int32_t a = 0; a < t.num_nodes; ++a)
        if (t.depth[a] == cd) hp.chunk_node.push_back(a);
    std::sort(hp.chunk_node.begin(), hp.chunk_node.end(), [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
    for (const int32_t node : hp.chunk_node) {
        H2Chunk m{};
        m.row_begin = (int32_t)t.begin[node];
        m.rows = (int32_t)t.size(node);
        m.k = rank(node);
        m.xh = hp.xh[node] < 0 ? 0 : hp.xh[node];
        m.term_base = (int32_t)hp.terms.size();
        if (m.k > 0) {
            if (t.parent[node] > 0) hp.terms.push_back(term_of_parent(node));
            for (const int64_t b : st.by_target[node]) hp.terms.push_back(term_of_coupling(b));
        }
        m.nterm = (int32_t)hp.terms.size() - m.term_base;
        const std::vector<int32_t> tleaves = chunk_leaves(t, node);
        m.leaf_base = (int32_t)hp.leaves.size();
        m.nleaf = (int32_t)tleaves.size();
        int32_t kq_max = 0;
        for (const int32_t lf : tleaves) {
            H2Leaf e{};
            e.row_begin = (int32_t)t.begin[lf];
            e.rows = (int32_t)t.size(lf);
            e.k = rank(lf);
            e.kq = (e.k + vw - 1) / vw;
            e.v_off = hp.v_elems;
            e.ft_off = ft_idx[lf] >= 0 ? (int32_t)hp.small[ft_idx[lf]].off : -1;
            e.e_off = e_idx[lf] >= 0 ? (int32_t)hp.small[e_idx[lf]].off : -1;
            e.ft_ld = ft_idx[lf] >= 0 ? hp.small[ft_idx[lf]].sld : 0;
            e.e_ld = e_idx[lf] >= 0 ? hp.small[e_idx[lf]].sld : 0;
            e.sf = ft_idx[lf] >= 0 ? hp.small[ft_idx[lf]].scale : 1.0f;
            e.se = e_idx[lf] >= 0 ? hp.small[e_idx[lf]].scale : 1.0f;
            e.sv = e.k > 0 ? qz.scale(bases[lf].v, e.rows, e.k, bases[lf].ldv, &finite) : 1.0f;
            e.su = e.k > 0 ? qz.scale(bases[lf].u, e.rows, e.k, bases[lf].ldu, &finite) : 1.0f;
            if (e.k > 0) {
                hp.v_elems += (int64_t)((e.rows + hmat::kWave - 1) / hmat::kWave) * e.kq * hmat::kWave * vw;
                hp.stored += 2 * (int64_t)e.rows * e.k;
                hp.leaf_kernel_elems += (int64_t)e.rows * e.k;       // U
                if (e.e_off >= 0) hp.leaf_kernel_elems += (int64_t)e.k * m.k;
            }
            kq_max = std::max(kq_max, e.kq);
            hp.leaves.push_back(e);
            hp.leaf_node.push_back(lf);
        }
        for (int32_t u = m.term_base; u < m.term_base + m.nterm; ++u)
            hp.leaf_kernel_elems += (int64_t)m.k * hp.terms[u].cols;
        m.nq_u = kq_max;
        const std::vector<int32_t> &sleaves = L == 0 ? tleaves : st.dense_src[node];
        m.dseg_base = (int32_t)hp.dsegs.size();
        m.nsrc = (int32_t)sleaves.size();
        int32_t nq = m.nq_u, vec = 0;
        for (const int32_t lf : sleaves) {
            DSeg ds;
            ds.row_begin = (int32_t)t.begin[lf];
            ds.rows = (int32_t)t.size(lf);
            ds.nq = (ds.rows + vw - 1) / vw;
            ds.pad_ = 0;
            nq += ds.nq;
            vec += ds.nq * vw;
            hp.dsegs.push_back(ds);
        }
        m.nq = nq;
        m.vec_floats = vec;
        m.dscale_base = (int32_t)hp.dscale.size();
        for (const int32_t lt : tleaves)
            for (const int32_t ls : sleaves) {
                const int64_t b = L == 0 ? 0 : st.find(lt, ls);
                const int64_t mt = t.size(lt), ms = t.size(ls);
                hp.dscale.push_back(qz.scale(bl[b].a, mt, ms, bl[b].lda, &finite));
                hp.stored += mt * ms;
                hp.leaf_kernel_elems += mt * ms;
            }
        m.ud_off = hp.ud_elems;
        hp.ud_elems += (int64_t)((m.rows + hmat::kWave - 1) / hmat::kWave) * nq * hmat::kWave * vw;
        hp.lds_b = std::max(hp.lds_b, 320 + m.nleaf * m.nq_u * vw + vec);
        hp.chunks.push_back(m);
    }
    if (!finite) return fail(HMAT_ERR_INVALID_ARG, "factors contain non-finite values");
    if (hp.lds_b > kMaxLdsFloats)
        return fail(HMAT_ERR_UNSUPPORTED, "a chunk's leaf-kernel operands (" + std::to_string(hp.lds_b) +
                                              " floats) exceed the LDS budget of " + std::to_string(kMaxLdsFloats));
    if (hp.small_elems >= INT32_MAX || hp.terms.size() >= (size_t)INT32_MAX)
        return fail(HMAT_ERR_UNSUPPORTED, "too many transfer and coupling entries");
    return HMAT_OK;
}

// The big panels and the small array, in the storage form (T = float or FP16 codes).
template <class T>
void fill(const Tree &t, const Structure &st, const hmat_h2_basis *bases, const hmat_h2_block *bl, const H2Host &hp,
          T *v, T *ud, T *small) {
    const int32_t vw = hp.vw;
    auto code = [](float x, float s) -> T {
        if constexpr (sizeof(T) == 4) return x;
        else return hmat::f32_to_f16_rne(x * (1.0f / s));
    };
    const int32_t L = t.L;
    // leaf V tiles
    hmat::parallel_for((int64_t)hp.leaves.size(), [&](int64_t i) {
        const H2Leaf &e = hp.leaves[i];
        if (e.k == 0) return;
        const hmat_h2_basis &b = bases[hp.leaf_node[i]];
        const int32_t ntile = (e.rows + hmat::kWave - 1) / hmat::kWave;
        for (int32_t tile = 0; tile < ntile; ++tile)
            for (int32_t j = 0; j < e.kq * vw; ++j)
                for (int32_t r = 0; r < hmat::kWave; ++r) {
                    const int32_t row = tile * hmat::kWave + r;
                    const float x = row < e.rows && j < e.k ? b.v[row + (int64_t)j * b.ldv] : 0.0f;
                    v[e.v_off + (int64_t)tile * e.kq * hmat::kWave * vw + ((int64_t)(j / vw) * hmat::kWave + r) * vw +
                      j % vw] = code(x, e.sv);
                }
    });
    // UD panels
    hmat::parallel_for((int64_t)hp.chunks.size(), [&](int64_t c) {
        const H2Chunk &m = hp.chunks[c];
        const int64_t tile_stride = (int64_t)m.nq * hmat::kWave * vw;
        auto put = [&](int32_t i, int32_t j, T q) {
            ud[m.ud_off + (i / hmat::kWave) * tile_stride + ((int64_t)(j / vw) * hmat::kWave + i % hmat::kWave) * vw +
               j % vw] = q;
        };
        const int32_t prow = ((m.rows + hmat::kWave - 1) / hmat::kWave) * hmat::kWave;
        const int32_t node = hp.chunk_node[c];
        const std::vector<int32_t> tleaves = chunk_leaves(t, node);
        const std::vector<int32_t> &sleaves = L == 0 ? tleaves : st.dense_src[node];
        int32_t it = 0;
        for (int32_t i = 0; i < prow; ++i) {
            if (i < m.rows)
                while (it + 1 < m.nleaf && m.row_begin + i >= hp.leaves[m.leaf_base + it + 1].row_begin) ++it;
            const H2Leaf &e = hp.leaves[m.leaf_base + it];
            const int32_t lr = m.row_begin + i - e.row_begin;  // row inside its leaf
            // U basis of the row's leaf
            for (int32_t j = 0; j < m.nq_u * vw; ++j) {
                float x = 0.0f;
                if (i < m.rows && j < e.k) x = bases[tleaves[it]].u[lr + (int64_t)j * bases[tleaves[it]].ldu];
                put(i, j, code(x, e.su));
            }
            // dense blocks, by source leaf
            int32_t col = m.nq_u * vw;
            for (int32_t is = 0; is < m.nsrc; ++is) {
                const DSeg &ds = hp.dsegs[m.dseg_base + is];
                const int64_t b = L == 0 ? 0 : st.find(tleaves[it], sleaves[is]);
                const float s = hp.dscale[m.dscale_base + it * m.nsrc + is];
                for (int32_t jj = 0; jj < ds.nq * vw; ++jj, ++col) {
                    float x = 0.0f;
                    if (i < m.rows && jj < ds.rows) x = bl[b].a[lr + (int64_t)jj * bl[b].lda];
                    put(i, col, code(x, s));
                }
            }
        }
    });
    // small matrices
    hmat::parallel_for((int64_t)hp.small.size(), [&](int64_t k) {
        const H2Host::SmallMat &m = hp.small[k];
        for (int32_t r = 0; r < m.rows; ++r)
            for (int32_t c = 0; c < m.sld; ++c) {
                float x = 0.0f;
                if (c < m.cols) x = m.transpose ? m.src[c + (int64_t)r * m.ld] : m.src[r + (int64_t)c * m.ld];
                small[m.off + (int64_t)r * m.sld + c] = code(x, m.scale);
            }
    });
}

template <class T>
hmat_status upload_all(hmat_h2_handle *h, const Tree &t, const Structure &st, const hmat_h2_basis *bases,
                       const hmat_h2_block *bl, const H2Host &hp) {
    hmat::DevPlanH2 &p = h->plan;
    try {
        std::vector<T> v(hp.v_elems), ud(hp.ud_elems), small(hp.small_elems);
        fill<T>(t, st, bases, bl, hp, v.data(), ud.data(), small.data());
        const T *dv = nullptr, *dud = nullptr, *dsmall = nullptr;
        hmat_status s;
        if ((s = upload(h, v, &dv)) != HMAT_OK) return s;
        if ((s = upload(h, ud, &dud)) != HMAT_OK) return s;
        if ((s = upload(h, small, &dsmall)) != HMAT_OK) return s;
        p.V = dv;
        p.UD = dud;
        p.small = dsmall;
    } catch (const std::bad_alloc &) {
        return fail(HMAT_ERR_NOMEM, "host staging allocation failed");
    }
    return HMAT_OK;
}

hmat_status create_impl(const hmat_tree_desc *tree, const hmat_h2_basis *bases, const hmat_h2_block *blocks,
                        int64_t nb, const hmat_h2_options *opts, hmat_h2_handle *h) {
    if (!opts) return fail(HMAT_ERR_INVALID_ARG, "options pointer is NULL");
    if (opts->storage != HMAT_STORE_FP32 && opts->storage != HMAT_STORE_FP16_SCALED)
        return fail(HMAT_ERR_INVALID_ARG, "the H^2 product takes HMAT_STORE_FP32 or HMAT_STORE_FP16_SCALED");
    if (opts->device < 0) return fail(HMAT_ERR_INVALID_ARG, "device must be >= 0");
    if (opts->flags != 0 || opts->reserved != 0) return fail(HMAT_ERR_INVALID_ARG, "flags and reserved must be 0");
    Tree t;
    hmat_status s = hmat::analyse_tree(tree, t);
    if (s != HMAT_OK) return s;
    Structure st;
    if ((s = validate(t, bases, blocks, nb, st)) != HMAT_OK) return s;
    H2Host hp;
    if ((s = build(t, st, bases, blocks, nb, opts->storage, hp)) != HMAT_OK) return s;
    h->device = opts->device;
    h->storage = opts->storage;
    hmat::DevPlanH2 &p = h->plan;
    p.storage = opts->storage;
    p.L = t.L;
    p.num_chunks = (int32_t)hp.chunks.size();
    p.kmax = hp.kmax;
    p.lds_b_floats = hp.lds_b;
    p.ws_half = (int32_t)hp.ws_half;
    // levels above the chunks: the node list holds depth 1, then depth 2, ... up to L-2
    h->level_first.assign(std::max(t.L, 1), 0);
    h->level_count.assign(std::max(t.L, 1), 0);
    {
        int32_t cur = 0;
        for (int32_t d = 1; d <= t.L - 2; ++d) {
            int32_t count = 0;
            for (int32_t a = 0; a < t.num_nodes; ++a) count += t.depth[a] == d;
            h->level_first[d] = cur;
            h->level_count[d] = count;
            cur += count;
        }
        if (cur != (int32_t)hp.nodes.size()) return fail(HMAT_ERR_INVALID_ARG, "internal error: level lists");
    }
    const int64_t esz = opts->storage == HMAT_STORE_FP32 ? 4 : 2;
    hmat_h2_info &in = h->info;
    in.n = t.n;
    in.leaf_depth = t.L;
    in.num_chunks = p.num_chunks;
    for (int64_t b = 0; b < nb; ++b) (blocks[b].kind == 0 ? in.num_dense_blocks : in.num_coupling_blocks)++;
    in.stored_elements = hp.stored;
    const int64_t nscales = opts->storage == HMAT_STORE_FP32 ? 0 : (int64_t)(hp.small.size() + hp.dscale.size()) +
                                                                      2 * (int64_t)hp.leaves.size();
    in.factor_bytes = hp.stored * esz + 4 * nscales;
    in.device_factor_bytes = (hp.v_elems + hp.ud_elems + hp.small_elems) * esz;
    in.workspace_bytes = 2 * hp.ws_half * 4;
    in.leaf_kernel_bytes = hp.leaf_kernel_elems * esz + 8 * t.n;
    in.storage = opts->storage;
    in.max_rank = hp.kmax;
    hmat_status u = opts->storage == HMAT_STORE_FP32 ? upload_all<float>(h, t, st, bases, blocks, hp)
                                                    : upload_all<uint16_t>(h, t, st, bases, blocks, hp);
    if (u != HMAT_OK) return u;
    void *ws = nullptr;
    if ((s = dev_alloc(h, 2 * hp.ws_half * 4, &ws)) != HMAT_OK) return s;
    p.ws = static_cast<float *>(ws);
    if ((s = upload(h, hp.chunks, &p.chunks)) != HMAT_OK) return s;
    if ((s = upload(h, hp.leaves, &p.leaves)) != HMAT_OK) return s;
    if ((s = upload(h, hp.dsegs, &p.dsegs)) != HMAT_OK) return s;
    if ((s = upload(h, hp.dscale, &p.dscale)) != HMAT_OK) return s;
    if ((s = upload(h, hp.nodes, &p.nodes)) != HMAT_OK) return s;
    if ((s = upload(h, hp.terms, &p.terms)) != HMAT_OK) return s;
    return HMAT_OK;
}

hmat_status record_event(hmat_h2_handle *h, hipStream_t stream) {
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

}  // namespace

extern "C" {

hmat_status hmat_h2_create(const hmat_tree_desc *tree, const hmat_h2_basis *bases, const hmat_h2_block *blocks,
                           int64_t num_blocks, const hmat_h2_options *opts, hmat_h2_t *out) {
    if (!out) return fail(HMAT_ERR_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    (void)hmat::set_error(HMAT_OK, "");
    hmat_h2_handle *h = nullptr;
    try {
        h = new hmat_h2_handle();
        const hmat_status s = create_impl(tree, bases, blocks, num_blocks, opts, h);
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

hmat_status hmat_h2_destroy(hmat_h2_t h) {
    if (!h) return HMAT_OK;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_live.count(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown or already destroyed H^2 handle");
        g_live.erase(h);
    }
    if (!h->dev_allocs.empty()) (void)hipSetDevice(h->device);
    release(h);
    return HMAT_OK;
}

hmat_status hmat_h2_get_info(hmat_h2_t h, hmat_h2_info *info) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown H^2 handle");
    if (!info) return fail(HMAT_ERR_INVALID_ARG, "info pointer is NULL");
    *info = h->info;
    return HMAT_OK;
}

hmat_status hmat_h2_matvec(hmat_h2_t h, int32_t nrhs, float alpha, const float *x, int64_t ldx, float beta,
                           float *y, int64_t ldy, void *stream) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown H^2 handle");
    const int64_t n = h->info.n;
    if (nrhs < 1) return fail(HMAT_ERR_INVALID_ARG, "nrhs must be >= 1");
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hmat::DevPlanH2 &p = h->plan;
    const int32_t L = p.L;
    auto dev_fail = [](const char *what, int e) {
        return fail(HMAT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
    };
    for (int32_t c = 0; c < nrhs; ++c) {
        const float *xc = x + c * ldx;
        float *yc = y + c * ldy;
        hmat_status s;
        int e = 0;
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if (L >= 2) {
            if ((e = hmat::launch_h2_upward(p, xc, st)) != 0) return dev_fail("upward launch", e);
            for (int32_t d = L - 2; d >= 1; --d)
                if ((e = hmat::launch_h2_up(p, h->level_first[d], h->level_count[d], st)) != 0)
                    return dev_fail("upward level launch", e);
        }
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        for (int32_t d = 1; d <= L - 2; ++d)
            if ((e = hmat::launch_h2_down(p, h->level_first[d], h->level_count[d], st)) != 0)
                return dev_fail("downward level launch", e);
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if ((e = hmat::launch_h2_leaf(p, xc, yc, alpha, beta, st)) != 0) return dev_fail("leaf launch", e);
        if (h->timing && (s = record_event(h, st)) != HMAT_OK) return s;
        if (h->timing) h->timed_calls++;
    }
    return HMAT_OK;
}

hmat_status hmat_h2_set_timing(hmat_h2_t h, int32_t enable) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown H^2 handle");
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

hmat_status hmat_h2_get_timing(hmat_h2_t h, double ms[HMAT_NUM_PHASES], int64_t *calls) {
    if (!h || !is_live(h)) return fail(HMAT_ERR_INVALID_ARG, "unknown H^2 handle");
    if (!ms || !calls) return fail(HMAT_ERR_INVALID_ARG, "output pointers must not be NULL");
    const size_t per = HMAT_NUM_PHASES + 1;
    const size_t sets = h->events_used / per;
    if (sets > 0) {
        const hipError_t e = hipEventSynchronize(h->events[sets * per - 1]);
        if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    }
    for (size_t k = 0; k < sets; ++k)
        for (int ph = 0; ph < HMAT_NUM_PHASES; ++ph) {
            float tms = 0.0f;
            const hipError_t e = hipEventElapsedTime(&tms, h->events[k * per + ph], h->events[k * per + ph + 1]);
            if (e != hipSuccess) return fail(HMAT_ERR_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
            h->ms[ph] += tms;
        }
    h->events_used = 0;
    for (int ph = 0; ph < HMAT_NUM_PHASES; ++ph) ms[ph] = h->ms[ph];
    *calls = h->timed_calls;
    return HMAT_OK;
}

}  // extern "C"
