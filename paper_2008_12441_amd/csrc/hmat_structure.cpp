// Domain tree analysis and validation of the Def. 2.3 block structure.
#include "hmat_structure.h"

#include "hmat_handle.h"

#include <string>

namespace hmat {
namespace {
hmat_status fail(hmat_status s, const std::string &msg) { return set_error(s, msg); }
}  // namespace

hmat_status analyse_tree(const hmat_tree_desc *td, Tree &t) {
    if (!td) return fail(HMAT_ERR_INVALID_ARG, "tree descriptor is NULL");
    if (td->n < 1 || td->n >= (int64_t(1) << 31))
        return fail(HMAT_ERR_INVALID_ARG, "tree n must be in [1, 2^31)");
    if (td->num_nodes < 1) return fail(HMAT_ERR_INVALID_ARG, "tree needs at least one node");
    if (td->reserved != 0) return fail(HMAT_ERR_INVALID_ARG, "tree reserved field must be 0");
    if (!td->parent || !td->begin || !td->end)
        return fail(HMAT_ERR_INVALID_ARG, "tree arrays must not be NULL");
    const int32_t nn = td->num_nodes;
    t.n = td->n;
    t.num_nodes = nn;
    t.parent.assign(td->parent, td->parent + nn);
    t.begin.assign(td->begin, td->begin + nn);
    t.end.assign(td->end, td->end + nn);
    if (t.parent[0] != -1) return fail(HMAT_ERR_BAD_TREE, "node 0 must be the root (parent -1)");
    if (t.begin[0] != 0 || t.end[0] != t.n)
        return fail(HMAT_ERR_BAD_TREE, "the root must own [0, n)");
    std::vector<int32_t> count(nn + 1, 0);
    for (int32_t i = 0; i < nn; ++i) {
        if (t.begin[i] < 0 || t.end[i] > t.n || t.begin[i] >= t.end[i])
            return fail(HMAT_ERR_BAD_TREE, "node " + std::to_string(i) + " has an empty or out-of-range index range");
        if (i > 0) {
            if (t.parent[i] < 0 || t.parent[i] >= i)
                return fail(HMAT_ERR_BAD_TREE, "node " + std::to_string(i) + " must have a parent with a smaller id");
            count[t.parent[i]]++;
        }
    }
    t.child_start.assign(nn + 1, 0);
    for (int32_t i = 0; i < nn; ++i) t.child_start[i + 1] = t.child_start[i] + count[i];
    t.child_list.assign(std::max(nn - 1, 0), 0);
    t.child_pos.assign(nn, 0);
    std::vector<int32_t> fill(nn, 0);
    for (int32_t i = 1; i < nn; ++i) {
        const int32_t p = t.parent[i];
        t.child_pos[i] = fill[p];
        t.child_list[t.child_start[p] + fill[p]++] = i;
    }
    t.depth.assign(nn, 0);
    for (int32_t i = 1; i < nn; ++i) t.depth[i] = t.depth[t.parent[i]] + 1;
    // children (in id order) tile the parent's range contiguously
    for (int32_t p = 0; p < nn; ++p) {
        const int32_t k = t.nkids(p);
        if (k == 0) continue;
        int64_t cur = t.begin[p];
        for (int32_t c = 0; c < k; ++c) {
            const int32_t ch = t.kid(p, c);
            if (t.begin[ch] != cur)
                return fail(HMAT_ERR_BAD_TREE, "children of node " + std::to_string(p) + " do not tile its range in id order");
            cur = t.end[ch];
        }
        if (cur != t.end[p])
            return fail(HMAT_ERR_BAD_TREE, "children of node " + std::to_string(p) + " do not cover its range");
    }
    int32_t L = -1;
    for (int32_t i = 0; i < nn; ++i) {
        if (!t.leaf(i)) continue;
        if (L < 0) L = t.depth[i];
        else if (t.depth[i] != L)
            return fail(HMAT_ERR_UNSUPPORTED, "leaves at different depths are not supported (the Def. 2.3 "
                                              "structure then has dense blocks between a leaf and a non-leaf)");
    }
    t.L = L;
    return HMAT_OK;
}

hmat_status validate_blocks(const Tree &t, const hmat_block_desc *bl, int64_t nb, Structure &st) {
    if (!bl) return fail(HMAT_ERR_INVALID_ARG, "blocks pointer is NULL");
    if (nb < 1) return fail(HMAT_ERR_INVALID_ARG, "num_blocks must be >= 1");
    const int32_t nn = t.num_nodes;
    for (int64_t b = 0; b < nb; ++b) {
        const hmat_block_desc &d = bl[b];
        const std::string id = "block " + std::to_string(b);
        if (d.reserved != 0) return fail(HMAT_ERR_INVALID_ARG, id + ": reserved field must be 0");
        if (d.target < 0 || d.target >= nn || d.source < 0 || d.source >= nn)
            return fail(HMAT_ERR_INVALID_ARG, id + ": node id out of range");
        if (d.rank < 0) return fail(HMAT_ERR_INVALID_ARG, id + ": negative rank");
        if (!d.a) return fail(HMAT_ERR_INVALID_ARG, id + ": factor pointer a is NULL");
        const int64_t mt = t.size(d.target), ms = t.size(d.source);
        if (d.lda < mt) return fail(HMAT_ERR_INVALID_ARG, id + ": lda < |t|");
        if (d.rank > 0) {
            if (!d.b) return fail(HMAT_ERR_INVALID_ARG, id + ": factor pointer b is NULL");
            if (d.ldb < ms) return fail(HMAT_ERR_INVALID_ARG, id + ": ldb < |s|");
            if (d.rank > std::min(mt, ms)) return fail(HMAT_ERR_INVALID_ARG, id + ": rank exceeds min(|t|, |s|)");
        }
    }
    if (t.L == 0) {
        if (nb != 1 || bl[0].target != 0 || bl[0].source != 0 || bl[0].rank != 0)
            return fail(HMAT_ERR_BAD_BLOCKS, "a tree whose root is a leaf takes exactly one dense block (0, 0)");
        return HMAT_OK;
    }
    auto name = [&](int64_t b) {
        return "block " + std::to_string(b) + " (" + std::to_string(bl[b].target) + ", " +
               std::to_string(bl[b].source) + ")";
    };
    st.index.reserve((size_t)nb * 2);
    for (int64_t b = 0; b < nb; ++b) {
        const hmat_block_desc &d = bl[b];
        if (d.target == 0 || d.source == 0)
            return fail(HMAT_ERR_BAD_BLOCKS, name(b) + ": the root pair is never a block of Def. 2.3");
        if (!st.index.emplace(Structure::key(d.target, d.source), b).second)
            return fail(HMAT_ERR_BAD_BLOCKS, name(b) + ": duplicate block");
    }
    // walk the recursion pairs level by level; every child pair must be a block or recurse
    std::vector<uint8_t> seen(nb, 0);
    std::vector<std::vector<int32_t>> partners(nn);
    std::vector<std::pair<int32_t, int32_t>> frontier{{0, 0}}, next;
    while (!frontier.empty()) {
        next.clear();
        for (const auto &pq : frontier) {
            const int32_t p = pq.first, q = pq.second;
            if (t.depth[p] == t.L - 1) partners[p].push_back(q);
            for (int32_t i = 0; i < t.nkids(p); ++i)
                for (int32_t j = 0; j < t.nkids(q); ++j) {
                    const int32_t ct = t.kid(p, i), cs = t.kid(q, j);
                    const int64_t b = st.find(ct, cs);
                    const bool leaves = t.leaf(ct);  // all leaves share one depth, and so do ct and cs
                    if (b < 0) {
                        if (leaves)
                            return fail(HMAT_ERR_BAD_BLOCKS, "missing block (" + std::to_string(ct) + ", " +
                                                                 std::to_string(cs) + ")");
                        next.emplace_back(ct, cs);
                        continue;
                    }
                    seen[b] = 1;
                    if (leaves) {
                        if (bl[b].rank != 0)
                            return fail(HMAT_ERR_UNSUPPORTED,
                                        name(b) + ": low-rank blocks between leaves are not supported (Def. 2.3 "
                                                  "makes them dense)");
                    } else {
                        if (ct == cs)
                            return fail(HMAT_ERR_BAD_BLOCKS,
                                        name(b) + ": (c, c) above the leaves is a recursion pair, not a block");
                        if (bl[b].rank == 0)
                            return fail(HMAT_ERR_UNSUPPORTED,
                                        name(b) + ": dense blocks between non-leaf boxes are not supported");
                    }
                }
        }
        frontier.swap(next);
    }
    for (int64_t b = 0; b < nb; ++b)
        if (!seen[b])
            return fail(HMAT_ERR_BAD_BLOCKS, name(b) + ": not a child pair of a recursion pair (it overlaps "
                                                       "another block or pairs boxes of different depths)");
    // low-rank blocks per node, and the dense sources of every depth-(L-1) node
    st.by_target.assign(nn, {});
    st.by_source.assign(nn, {});
    for (int64_t b = 0; b < nb; ++b)
        if (bl[b].rank > 0) {
            st.by_target[bl[b].target].push_back(b);
            st.by_source[bl[b].source].push_back(b);
        }
    for (int32_t a = 0; a < nn; ++a) {
        std::sort(st.by_target[a].begin(), st.by_target[a].end(),
                  [&](int64_t x, int64_t y) { return t.begin[bl[x].source] < t.begin[bl[y].source]; });
        std::sort(st.by_source[a].begin(), st.by_source[a].end(),
                  [&](int64_t x, int64_t y) { return t.begin[bl[x].target] < t.begin[bl[y].target]; });
    }
    st.dense_src.assign(nn, {});
    for (int32_t p = 0; p < nn; ++p) {
        auto &q = partners[p];
        std::sort(q.begin(), q.end(), [&](int32_t x, int32_t y) { return t.begin[x] < t.begin[y]; });
        for (int32_t r : q)
            for (int32_t j = 0; j < t.nkids(r); ++j) st.dense_src[p].push_back(t.kid(r, j));
    }
    return HMAT_OK;
}

void dense_group_amax(const Tree &t, const hmat_block_desc *bl, int64_t nb, std::vector<float> &amax) {
    std::unordered_map<uint64_t, float> group;  // (parent of the target, parent of the source) -> largest |entry|
    auto key = [&](int64_t b) { return Structure::key(t.parent[bl[b].target], t.parent[bl[b].source]); };
    for (int64_t b = 0; b < nb; ++b)
        if (bl[b].rank == 0) {
            float &g = group[key(b)];
            g = std::max(g, amax[b]);
        }
    for (int64_t b = 0; b < nb; ++b)
        if (bl[b].rank == 0) amax[b] = group[key(b)];
}

}  // namespace hmat
