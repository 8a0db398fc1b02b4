// Sanitizer driver: runs the library's C ABI over one structure read from a
// file (written by tests/test_sanitize_cpu.py), with the HIP runtime replaced
// by the host stand-ins of sanitize_stubs.cpp. Every layout, plan, batch and
// validation path of the host code runs; malformed variants of the structure
// must be rejected with the documented status. Prints "OK" and exits 0 when
// every call returned what it should.
//
// File: int32 magic (1: H-matrix, 2: H^2), int64 n, int32 num_nodes, int32 nb,
// int32 d, int32 parent[num_nodes], int64 begin[num_nodes], int64 end[num_nodes],
// int32 target[nb], int32 source[nb], int32 rank_or_kind[nb], int64 off_a[nb],
// int64 off_b[nb], then for magic 2: int32 basis_rank[num_nodes], int64
// u_off, v_off, e_off, f_off [num_nodes]; then int64 pool_size, float
// pool[pool_size], float points[n * d].
#include "hmat.h"
#include "hmat_h2.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

int g_fail = 0, g_calls = 0;

void expect(hmat_status got, hmat_status want, const char *what) {
    ++g_calls;
    if (got != want) {
        std::printf("UNEXPECTED %s: status %d (%s), wanted %d: %s\n", what, (int)got, hmat_status_string(got),
                    (int)want, hmat_last_error());
        ++g_fail;
    }
}

template <class T>
void rd(FILE *f, T *p, size_t n) {
    if (n && std::fread(p, sizeof(T), n, f) != n) {
        std::printf("short read\n");
        std::exit(2);
    }
}

struct Input {
    int32_t magic = 0, nn = 0, nb = 0, d = 0;
    int64_t n = 0;
    std::vector<int32_t> parent, target, source, rk, brank;
    std::vector<int64_t> begin, end, off_a, off_b, u_off, v_off, e_off, f_off;
    std::vector<float> pool, points;
    int64_t size(int32_t a) const { return end[a] - begin[a]; }
};

Input load(const char *path) {
    Input in;
    FILE *f = std::fopen(path, "rb");
    if (!f) std::exit(2);
    rd(f, &in.magic, 1);
    rd(f, &in.n, 1);
    rd(f, &in.nn, 1);
    rd(f, &in.nb, 1);
    rd(f, &in.d, 1);
    in.parent.resize(in.nn);
    in.begin.resize(in.nn);
    in.end.resize(in.nn);
    rd(f, in.parent.data(), in.nn);
    rd(f, in.begin.data(), in.nn);
    rd(f, in.end.data(), in.nn);
    in.target.resize(in.nb);
    in.source.resize(in.nb);
    in.rk.resize(in.nb);
    in.off_a.resize(in.nb);
    in.off_b.resize(in.nb);
    rd(f, in.target.data(), in.nb);
    rd(f, in.source.data(), in.nb);
    rd(f, in.rk.data(), in.nb);
    rd(f, in.off_a.data(), in.nb);
    rd(f, in.off_b.data(), in.nb);
    if (in.magic == 2) {
        in.brank.resize(in.nn);
        rd(f, in.brank.data(), in.nn);
        for (auto *v : {&in.u_off, &in.v_off, &in.e_off, &in.f_off}) {
            v->resize(in.nn);
            rd(f, v->data(), in.nn);
        }
    }
    int64_t ps = 0;
    rd(f, &ps, 1);
    in.pool.resize(ps);
    rd(f, in.pool.data(), ps);
    in.points.resize(in.n * in.d);
    rd(f, in.points.data(), in.points.size());
    std::fclose(f);
    return in;
}

hmat_tree_desc tree_of(const Input &in) {
    return hmat_tree_desc{in.n, in.nn, 0, in.parent.data(), in.begin.data(), in.end.data()};
}

std::vector<hmat_block_desc> blocks_of(Input &in, float *pool) {
    std::vector<hmat_block_desc> b(in.nb);
    for (int32_t i = 0; i < in.nb; ++i) {
        b[i] = hmat_block_desc{in.target[i], in.source[i], in.rk[i], 0, pool + in.off_a[i], in.size(in.target[i]),
                               in.rk[i] > 0 ? pool + in.off_b[i] : nullptr, in.rk[i] > 0 ? in.size(in.source[i]) : 0};
    }
    return b;
}

void run_h(Input &in) {
    hmat_tree_desc t = tree_of(in);
    std::vector<hmat_block_desc> b = blocks_of(in, in.pool.data());
    const int64_t n = in.n;
    std::vector<float> x(n * 3, 1.0f), y(n * 3, 0.0f);
    struct Case {
        int32_t storage, max_nrhs, flags;
    };
    const Case cases[] = {{HMAT_STORE_FP32, 1, 0}, {HMAT_STORE_FP16_SCALED, 1, 0}, {HMAT_STORE_BF16, 1, 0},
                          {HMAT_STORE_FP32, 1, HMAT_FLAG_FP64_ACCUM}, {HMAT_STORE_FP32, 1, HMAT_FLAG_TRANSPOSE},
                          {HMAT_STORE_FP32, 16, 0}, {HMAT_STORE_FP16_SCALED, 16, 0}, {HMAT_STORE_BF16, 16, 0},
                          {HMAT_STORE_FP8, 16, 0}, {HMAT_STORE_FP8_F16D, 16, HMAT_FLAG_TRANSPOSE},
                          {HMAT_STORE_FP16_SCALED, 130, 0}};
    for (const Case &c : cases) {
        hmat_options o{c.storage, c.max_nrhs, 0, c.flags};
        hmat_t h = nullptr;
        const hmat_status s = hmat_create(&t, b.data(), in.nb, &o, &h);
        expect(s, HMAT_OK, "hmat_create");
        if (s != HMAT_OK) continue;
        hmat_info info;
        expect(hmat_get_info(h, &info), HMAT_OK, "hmat_get_info");
        expect(hmat_set_timing(h, 1), HMAT_OK, "hmat_set_timing");
        const int32_t k = c.max_nrhs < 3 ? c.max_nrhs : 3;
        expect(hmat_matvec(h, k, 1.0f, x.data(), n, 0.5f, y.data(), n, nullptr), HMAT_OK, "hmat_matvec");
        double ms[HMAT_NUM_PHASES];
        int64_t calls = 0;
        expect(hmat_get_timing(h, ms, &calls), HMAT_OK, "hmat_get_timing");
        expect(hmat_matvec_noalloc(h, 1, 1.0f, x.data(), n, 0.0f, y.data(), n, nullptr),
               c.max_nrhs == 1 || (c.flags & HMAT_FLAG_FP64_ACCUM) ? HMAT_OK : HMAT_ERR_UNSUPPORTED,
               "hmat_matvec_noalloc");
        expect(hmat_matvec(h, c.max_nrhs + 1, 1.0f, x.data(), n, 0.0f, y.data(), n, nullptr), HMAT_ERR_INVALID_ARG,
               "hmat_matvec nrhs > max");
        expect(hmat_destroy(h), HMAT_OK, "hmat_destroy");
    }
    {  // FP8 needs a multi-RHS handle
        hmat_options o{HMAT_STORE_FP8, 1, 0, 0};
        hmat_t h = nullptr;
        expect(hmat_create(&t, b.data(), in.nb, &o, &h), HMAT_ERR_UNSUPPORTED, "hmat_create fp8 single");
    }
    // a batch over a single-vector and a multi-RHS member, the autotuner with its cache
    {
        hmat_options o1{HMAT_STORE_FP16_SCALED, 1, 0, 0}, o2{HMAT_STORE_FP16_SCALED, 16, 0, 0};
        hmat_t h1 = nullptr, h2 = nullptr;
        expect(hmat_create(&t, b.data(), in.nb, &o1, &h1), HMAT_OK, "hmat_create member 1");
        expect(hmat_create(&t, b.data(), in.nb, &o2, &h2), HMAT_OK, "hmat_create member 2");
        if (h1 && h2) {
            hmat_t hs[2] = {h1, h2};
            int32_t k[2] = {1, 16};
            std::vector<float> x2(n * 16, 1.0f), y1(n, 0.0f), y2(n * 16, 0.0f);
            const float *xs[2] = {x.data(), x2.data()};
            float *ys[2] = {y1.data(), y2.data()};
            int64_t ld[2] = {n, n};
            hmat_batch_t bt = nullptr;
            expect(hmat_batch_create(hs, 2, k, nullptr, &bt), HMAT_OK, "hmat_batch_create");
            if (bt) {
                expect(hmat_batch_matvec(bt, 1.0f, xs, ld, 0.0f, ys, ld, nullptr), HMAT_OK, "hmat_batch_matvec");
                expect(hmat_batch_sync(bt, nullptr), HMAT_OK, "hmat_batch_sync");
                hmat_batch_options chosen;
                const std::string cache = std::string(std::getenv("HMAT_SANITIZE_TMP") ? std::getenv("HMAT_SANITIZE_TMP")
                                                                                        : "/tmp") +
                                          "/hmat_tune.json";
                expect(hmat_batch_autotune(bt, 1.0f, xs, ld, 0.0f, ys, ld, nullptr, cache.c_str(), 1, &chosen), HMAT_OK,
                       "hmat_batch_autotune");
                expect(hmat_batch_autotune(bt, 1.0f, xs, ld, 0.0f, ys, ld, nullptr, cache.c_str(), 1, &chosen), HMAT_OK,
                       "hmat_batch_autotune (cached)");
                hmat_batch_info bi;
                expect(hmat_batch_get_info(bt, &bi), HMAT_OK, "hmat_batch_get_info");
                expect(hmat_destroy(h1), HMAT_ERR_INVALID_ARG, "hmat_destroy of a batch member");
                expect(hmat_batch_destroy(bt), HMAT_OK, "hmat_batch_destroy");
            }
        }
        expect(hmat_destroy(h1), HMAT_OK, "hmat_destroy member 1");
        expect(hmat_destroy(h2), HMAT_OK, "hmat_destroy member 2");
    }
    // construction: dense entries and randomized SVDs written into a copy of the pool
    if (in.d >= 1 && in.d <= 3) {
        std::vector<float> pool2(in.pool.size(), 0.0f);
        std::vector<hmat_block_desc> b2 = blocks_of(in, pool2.data());
        hmat_compress_options co{HMAT_KERNEL_LOG, in.d, 1.0f, 10, 7, 0, 0};
        expect(hmat_compress(&t, in.points.data(), b2.data(), in.nb, &co), HMAT_OK, "hmat_compress");
    }
    // malformed variants, each rejected before any allocation
    hmat_options o{HMAT_STORE_FP32, 1, 0, 0};
    hmat_t h = nullptr;
    if (in.nb > 1) {
        expect(hmat_create(&t, b.data(), in.nb - 1, &o, &h), HMAT_ERR_BAD_BLOCKS, "missing block");
        std::vector<hmat_block_desc> dup(b);
        dup.push_back(b[0]);
        expect(hmat_create(&t, dup.data(), in.nb + 1, &o, &h), HMAT_ERR_BAD_BLOCKS, "duplicate block");
    }
    for (int32_t i = 0; i < in.nb; ++i)
        if (b[i].rank > 0) {
            std::vector<hmat_block_desc> bad(b);
            bad[i].rank = 0;
            expect(hmat_create(&t, bad.data(), in.nb, &o, &h), HMAT_ERR_UNSUPPORTED, "dense block above the leaves");
            bad = b;
            bad[i].rank = (int32_t)(in.size(b[i].target) + 1);
            expect(hmat_create(&t, bad.data(), in.nb, &o, &h), HMAT_ERR_INVALID_ARG, "rank too large");
            bad = b;
            bad[i].ldb = 1;
            expect(hmat_create(&t, bad.data(), in.nb, &o, &h), HMAT_ERR_INVALID_ARG, "ldb too small");
            break;
        }
    if (in.nn > 2) {
        std::vector<int64_t> e2(in.end);
        e2[1] -= 1;
        hmat_tree_desc t2{in.n, in.nn, 0, in.parent.data(), in.begin.data(), e2.data()};
        expect(hmat_create(&t2, b.data(), in.nb, &o, &h), HMAT_ERR_BAD_TREE, "children do not tile");
        std::vector<int32_t> p2(in.parent);
        p2[1] = in.nn - 1;
        hmat_tree_desc t3{in.n, in.nn, 0, p2.data(), in.begin.data(), in.end.data()};
        expect(hmat_create(&t3, b.data(), in.nb, &o, &h), HMAT_ERR_BAD_TREE, "parent after child");
    }
    expect(hmat_create(nullptr, b.data(), in.nb, &o, &h), HMAT_ERR_INVALID_ARG, "null tree");
}

void run_h2(Input &in) {
    hmat_tree_desc t = tree_of(in);
    float *P = in.pool.data();
    std::vector<hmat_h2_basis> bases(in.nn);
    for (int32_t a = 0; a < in.nn; ++a) {
        const int32_t k = in.brank[a];
        const int32_t kp = a > 0 ? in.brank[in.parent[a]] : 0;
        bases[a] = hmat_h2_basis{k, 0, in.u_off[a] >= 0 ? P + in.u_off[a] : nullptr, in.size(a),
                                 in.v_off[a] >= 0 ? P + in.v_off[a] : nullptr, in.size(a),
                                 in.e_off[a] >= 0 ? P + in.e_off[a] : nullptr, k,
                                 in.f_off[a] >= 0 ? P + in.f_off[a] : nullptr, k};
        (void)kp;
    }
    std::vector<hmat_h2_block> blocks(in.nb);
    for (int32_t i = 0; i < in.nb; ++i)
        blocks[i] = hmat_h2_block{in.target[i], in.source[i], in.rk[i], 0, P + in.off_a[i],
                                  in.rk[i] ? in.brank[in.target[i]] : in.size(in.target[i])};
    std::vector<float> x(in.n * 2, 1.0f), y(in.n * 2, 0.0f);
    for (int32_t st : {HMAT_STORE_FP32, HMAT_STORE_FP16_SCALED}) {
        hmat_h2_options o{st, 0, 0, 0};
        hmat_h2_t h = nullptr;
        const hmat_status s = hmat_h2_create(&t, bases.data(), blocks.data(), in.nb, &o, &h);
        expect(s, HMAT_OK, "hmat_h2_create");
        if (s != HMAT_OK) continue;
        hmat_h2_info info;
        expect(hmat_h2_get_info(h, &info), HMAT_OK, "hmat_h2_get_info");
        expect(hmat_h2_set_timing(h, 1), HMAT_OK, "hmat_h2_set_timing");
        expect(hmat_h2_matvec(h, 2, 1.0f, x.data(), in.n, 0.25f, y.data(), in.n, nullptr), HMAT_OK, "hmat_h2_matvec");
        double ms[HMAT_NUM_PHASES];
        int64_t calls = 0;
        expect(hmat_h2_get_timing(h, ms, &calls), HMAT_OK, "hmat_h2_get_timing");
        expect(hmat_h2_destroy(h), HMAT_OK, "hmat_h2_destroy");
    }
    hmat_h2_options o{HMAT_STORE_FP32, 0, 0, 0};
    hmat_h2_t h = nullptr;
    if (in.nb > 1)
        expect(hmat_h2_create(&t, bases.data(), blocks.data(), in.nb - 1, &o, &h), HMAT_ERR_BAD_BLOCKS,
               "h2 missing block");
    for (int32_t a = 1; a < in.nn; ++a)
        if (bases[a].rank > 0) {
            std::vector<hmat_h2_basis> bad(bases);
            bad[a].rank = HMAT_H2_MAX_RANK + 1;
            expect(hmat_h2_create(&t, bad.data(), blocks.data(), in.nb, &o, &h), HMAT_ERR_UNSUPPORTED, "h2 rank");
            break;
        }
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    Input in = load(argv[1]);
    if (in.magic == 1) run_h(in);
    else run_h2(in);
    std::printf("%s %d calls, %d unexpected\n", g_fail ? "FAILED" : "OK", g_calls, g_fail);
    return g_fail ? 1 : 0;
}
