// Domain tree and Def. 2.3 block structure: analysis and validation shared by
// the host sources (the H-matrix handles and the H^2 handles), plus the host
// thread pool they lay data out with.
#pragma once

#include "hmat.h"

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <thread>
#include <unordered_map>
#include <vector>

namespace hmat {

// Run f(0), ..., f(n - 1) on up to 16 host threads (any order).
template <class F>
void parallel_for(int64_t n, F f) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (n < 2 || nt == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    nt = (unsigned)std::min<int64_t>(nt, n);
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int64_t i = next.fetch_add(1);
            if (i >= n) break;
            f(i);
        }
    };
    std::vector<std::thread> th;
    for (unsigned k = 1; k < nt; ++k) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

// ---------------------------------------------------------------------------
// Tree analysis and structure validation.
// ---------------------------------------------------------------------------
struct Tree {
    int64_t n = 0;
    int32_t num_nodes = 0;
    std::vector<int32_t> parent, depth, child_start, child_list, child_pos;
    std::vector<int64_t> begin, end;
    int32_t L = 0;
    int32_t nkids(int32_t p) const { return child_start[p + 1] - child_start[p]; }
    int32_t kid(int32_t p, int32_t i) const { return child_list[child_start[p] + i]; }
    bool leaf(int32_t p) const { return nkids(p) == 0; }
    int64_t size(int32_t p) const { return end[p] - begin[p]; }
};

// Check a domain tree descriptor and derive children, depths and the common
// leaf depth L.
hmat_status analyse_tree(const hmat_tree_desc *td, Tree &t);

// The block structure of Def. 2.3: starting from the pair (root, root),
// every child pair of a recursion pair is a dense block (leaf pairs), a
// low-rank block (admissible pairs) or a recursion pair itself. The
// admissibility condition is the caller's: any block set of this shape is
// accepted, so weak admissibility (low-rank blocks between distinct siblings)
// and standard admissibility (low-rank blocks between boxes whose parents are
// neighbours, dense blocks between neighbouring parents' leaves) both are.
struct Structure {
    std::unordered_map<uint64_t, int64_t> index;             // (target, source) -> block
    std::vector<std::vector<int64_t>> by_target, by_source;  // low-rank blocks of a node, by the other node's first row
    std::vector<std::vector<int32_t>> dense_src;             // per node at depth L-1: the source leaves of its
                                                             // children's dense blocks, by first row
    static uint64_t key(int32_t a, int32_t b) { return (uint64_t)(uint32_t)a << 32 | (uint32_t)b; }
    int64_t find(int32_t a, int32_t b) const {
        const auto it = index.find(key(a, b));
        return it == index.end() ? -1 : it->second;
    }
};

// Check that the blocks have Def. 2.3's shape for the tree (see hmat_create)
// and index them.
hmat_status validate_blocks(const Tree &t, const hmat_block_desc *bl, int64_t nb, Structure &st);

// The scaled storage forms give the dense blocks one power-of-two scale per
// group: the dense blocks whose target leaves have one parent and whose source
// leaves have one parent (the near field between two boxes at depth L - 1).
// amax holds each dense block's largest |entry| (the entries of low-rank
// blocks are left alone); on return a dense block's entry holds the largest
// over its group.
void dense_group_amax(const Tree &t, const hmat_block_desc *bl, int64_t nb, std::vector<float> &amax);

}  // namespace hmat
