// Host side of the batched persistent launch: the item queue (stage bands,
// dependency counters, cost order), the per-call operand table, the HIP graph
// of (counter clear, persistent kernel), and the autotuner with its JSON cache.
#include "hmat.h"
#include "hmat_handle.h"
#include "hmat_internal.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <unordered_set>
#include <vector>

using hmat::BArgs;
using hmat::BItem;
using hmat::BMember;

struct hmat_batch_handle {
    int32_t device = 0;
    int32_t storage = 0;
    bool has_s = false, has_m = false;
    std::vector<hmat_t> members;
    std::vector<int32_t> k;
    hmat_batch_options opts{};
    int32_t cus = 0;
    int32_t max_wg = 0;
    size_t lds = 0;
    int32_t zs_rank = 0;
    int64_t item_bytes = 0;
    // device
    BMember *d_members = nullptr;
    BArgs *d_args = nullptr;
    BItem *d_items = nullptr;
    int32_t *d_ctl = nullptr;
    int32_t num_items = 0, items_cap = 0, num_ctl = 0, grid = 0;
    BArgs *h_args = nullptr;        // pinned staging of the operand table
    std::vector<BArgs> cur_args;    // what d_args holds
    bool args_valid = false;
    hipEvent_t args_ev = nullptr;   // recorded after the last operand upload
    bool args_ev_pending = false;
    hipStream_t cap = nullptr;      // private stream the graph is captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

using hmat::set_error;

std::mutex g_bmu;
std::unordered_set<const hmat_batch_handle *> g_blive;

bool batch_live(const hmat_batch_handle *b) {
    std::lock_guard<std::mutex> lk(g_bmu);
    return g_blive.count(b) != 0;
}

hmat_status hip_fail(const char *what, hipError_t e) {
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return set_error(HMAT_ERR_NOMEM, std::string(what) + ": out of memory");
    }
    return set_error(HMAT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int32_t kDefaultSpin = 1 << 20;

// Stage band of each item kind: source side, then V products of the
// multi-RHS members (their X packing is in band 0), reduction, second
// reduction stage, target side.
int band_of(int32_t kind) {
    switch (kind) {
    case hmat::BK_SV:
    case hmat::BK_MX: return 0;
    case hmat::BK_MV: return 1;
    case hmat::BK_SZ1:
    case hmat::BK_MZ: return 2;
    case hmat::BK_SZ2: return 3;
    default: return 4;
    }
}

struct Costed {
    BItem it;
    float cost;
};

// Every member's items; counters 2 + 3 i + {0, 1, 2} belong to member i. An
// item is a run of consecutive work indices of one stage whose estimated
// traffic reaches the grain (or the end of the stage).
std::vector<Costed> member_items(const hmat_batch_handle *b, int32_t i, double grain) {
    std::vector<Costed> out;
    const hmat_handle *h = b->members[i];
    const int32_t c0 = 2 + 3 * i;
    // items of one stage over work indices [0, n) with costs cost[]; returns how many
    auto stage = [&](int32_t kind, int32_t n, const std::vector<float> &cost, int32_t dep, int32_t need,
                     int32_t done) {
        int32_t items = 0;
        for (int32_t f = 0; f < n;) {
            double c = 0.0;
            int32_t e = f;
            while (e < n && (e == f || c + cost[e] <= grain)) c += cost[e++];
            out.push_back(Costed{BItem{i, kind, f, e - f, dep, need, done, 0}, (float)c});
            ++items;
            f = e;
        }
        return items;
    };
    if (!h->mr) {
        const hmat::DevPlan &p = h->plan;
        const int32_t nsv = stage(hmat::BK_SV, p.num_vtiles, h->cost_src, -1, 0, c0);
        const size_t z0 = out.size();
        const int32_t nz1 = stage(hmat::BK_SZ1, p.num_z1, h->cost_z1, nsv ? c0 : -1, nsv, c0 + 1);
        const int32_t nz2 = stage(hmat::BK_SZ2, p.num_z2, h->cost_z2, c0 + 1, nz1, c0 + 2);
        // reduction items carry the lanes per unit: the member's largest rank rounded up to a power of
        // two (a wave then works on 64 / that many units at once)
        int32_t lanes = 1;
        while (lanes < std::min(h->max_rank, 64)) lanes *= 2;
        for (size_t i = z0; i < out.size(); ++i) out[i].it.lanes = lanes;
        int32_t dep = -1, need = 0;
        if (nz2) dep = c0 + 2, need = nz2;
        else if (nz1) dep = c0 + 1, need = nz1;
        else if (nsv) dep = c0, need = nsv;
        stage(hmat::BK_SU, p.num_chunks, h->cost_tgt, dep, need, -1);
    } else {
        const hmat::DevPlanMR &p = h->mrp;
        std::vector<float> xcost(p.num_chunks);
        // X read and fragments written, plus a round trip shared by the four chunks a workgroup packs at once
        for (int32_t c = 0; c < p.num_chunks; ++c) xcost[c] = (float)h->chunk_rows[c] * 16 * 4 * 2 + 4096.0f;
        const int32_t nmx = stage(hmat::BK_MX, p.num_chunks, xcost, -1, 0, c0);
        const int32_t nmv = stage(hmat::BK_MV, p.num_ugroups, h->cost_src, c0, nmx, c0 + 1);
        const int32_t nmz = stage(hmat::BK_MZ, p.num_zitems, h->cost_z1, nmv ? c0 + 1 : c0, nmv ? nmv : nmx, c0 + 2);
        stage(hmat::BK_MU, p.num_tgroups, h->cost_tgt, nmz ? c0 + 2 : c0, nmz ? nmz : nmx, -1);
    }
    return out;
}

// The queue: stage bands in order; inside a band, order 0 sorts items by cost
// (largest first), order 1 keeps members together, largest member first.
constexpr int32_t kDefaultGrainKb = 512;

std::vector<BItem> build_queue(const hmat_batch_handle *b, const hmat_batch_options &o, int64_t *bytes) {
    const int32_t order = o.order;
    const double grain = 1024.0 * (o.grain_kb > 0 ? o.grain_kb : kDefaultGrainKb);
    const int32_t n = (int32_t)b->members.size();
    std::vector<std::vector<Costed>> per(n);
    std::vector<double> total(n, 0.0);
    *bytes = 0;
    for (int32_t i = 0; i < n; ++i) {
        per[i] = member_items(b, i, grain);
        for (const Costed &c : per[i]) total[i] += c.cost;
        for (const Costed &c : per[i])
            if (c.it.kind != hmat::BK_SZ1 && c.it.kind != hmat::BK_SZ2 && c.it.kind != hmat::BK_MZ &&
                c.it.kind != hmat::BK_MX)
                *bytes += (int64_t)c.cost;
    }
    std::vector<int32_t> mo(n);
    std::iota(mo.begin(), mo.end(), 0);
    std::stable_sort(mo.begin(), mo.end(), [&](int32_t a, int32_t c) { return total[a] > total[c]; });
    std::vector<BItem> q;
    for (int band = 0; band <= 4; ++band) {
        std::vector<Costed> items;
        for (int32_t i : mo)
            for (const Costed &c : per[i])
                if (band_of(c.it.kind) == band) items.push_back(c);
        if (order == 0)
            std::stable_sort(items.begin(), items.end(), [](const Costed &a, const Costed &c) { return a.cost > c.cost; });
        for (const Costed &c : items) q.push_back(c.it);
    }
    return q;
}

hmat::BatchArgs kernel_args(const hmat_batch_handle *b) {
    hmat::BatchArgs a{};
    a.members = b->d_members;
    a.args = b->d_args;
    a.items = b->d_items;
    a.ctl = b->d_ctl;
    a.num_items = b->num_items;
    a.num_ctl = b->num_ctl;
    a.spin_limit = b->opts.spin_limit > 0 ? b->opts.spin_limit : kDefaultSpin;
    a.zs_rank = b->zs_rank;
    return a;
}

void drop_graph(hmat_batch_handle *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// (Re)build the queue and, with use_graph, the graph, for b->opts.
hmat_status configure(hmat_batch_handle *b) {
    drop_graph(b);
    int64_t bytes = 0;
    const std::vector<BItem> q = build_queue(b, b->opts, &bytes);
    b->item_bytes = bytes;
    hipError_t e;
    if ((int32_t)q.size() > b->items_cap) {  // the queue grows with a finer grain
        if (b->d_items) (void)hipFree(b->d_items);
        b->d_items = nullptr;
        b->items_cap = 0;
        if ((e = hipMalloc(&b->d_items, sizeof(BItem) * q.size())) != hipSuccess) return hip_fail("hipMalloc", e);
        b->items_cap = (int32_t)q.size();
    }
    b->num_items = (int32_t)q.size();
    e = hipMemcpy(b->d_items, q.data(), q.size() * sizeof(BItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail("hipMemcpy", e);
    const int32_t wg = b->opts.wg_per_cu > 0 ? std::min(b->opts.wg_per_cu, b->max_wg) : b->max_wg;
    b->grid = std::max(1, wg * b->cus);
    if (!b->opts.use_graph) return HMAT_OK;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail("hipStreamBeginCapture", e);
    const int le = hmat::launch_batch(kernel_args(b), b->storage, b->has_s, b->has_m, b->grid, b->lds, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (le != 0) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail("batched launch capture", (hipError_t)le);
    }
    if (e != hipSuccess) return hip_fail("hipStreamEndCapture", e);
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail("hipGraphInstantiate", e);
    }
    return HMAT_OK;
}

void release_batch(hmat_batch_handle *b) {
    if (!b) return;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->args_ev) (void)hipEventDestroy(b->args_ev);
    if (b->h_args) (void)hipHostFree(b->h_args);
    for (void *p : {(void *)b->d_members, (void *)b->d_args, (void *)b->d_items, (void *)b->d_ctl})
        if (p) (void)hipFree(p);
    for (hmat_t h : b->members) (void)hmat::handle_live(h, -1);
    delete b;
}

hmat_status check_options(const hmat_batch_options *o) {
    if (o->use_graph != 0 && o->use_graph != 1) return set_error(HMAT_ERR_INVALID_ARG, "use_graph must be 0 or 1");
    if (o->wg_per_cu < 0 || o->wg_per_cu > 64) return set_error(HMAT_ERR_INVALID_ARG, "wg_per_cu out of [0, 64]");
    if (o->order != 0 && o->order != 1) return set_error(HMAT_ERR_INVALID_ARG, "order must be 0 or 1");
    if (o->spin_limit < 0) return set_error(HMAT_ERR_INVALID_ARG, "spin_limit must be >= 0");
    if (o->grain_kb < 0 || o->grain_kb > (1 << 20)) return set_error(HMAT_ERR_INVALID_ARG, "grain_kb out of [0, 2^20]");
    return HMAT_OK;
}

hmat_status create_impl(const hmat_t *hs, int32_t count, const int32_t *nrhs, const hmat_batch_options *opts,
                        hmat_batch_handle *b) {
    if (!hs || !nrhs) return set_error(HMAT_ERR_INVALID_ARG, "members and nrhs must not be NULL");
    if (count < 1) return set_error(HMAT_ERR_INVALID_ARG, "count must be >= 1");
    if (count > (1 << 20)) return set_error(HMAT_ERR_INVALID_ARG, "too many members");
    b->opts = hmat_batch_options{1, 0, 0, 0, 0};
    if (opts) {
        hmat_status s = check_options(opts);
        if (s != HMAT_OK) return s;
        b->opts = *opts;
    }
    std::unordered_set<const hmat_handle *> seen;
    for (int32_t i = 0; i < count; ++i) {
        const hmat_handle *h = hs[i];
        if (!h || !hmat::handle_live(h)) return set_error(HMAT_ERR_INVALID_ARG, "member " + std::to_string(i) + " is not a live handle");
        if (!seen.insert(h).second) return set_error(HMAT_ERR_INVALID_ARG, "member " + std::to_string(i) + " appears twice");
        if (i == 0) {
            b->device = h->device;
            b->storage = h->storage;
        } else if (h->device != b->device || h->storage != b->storage) {
            return set_error(HMAT_ERR_INVALID_ARG, "members must share one device and one storage form");
        }
        if (h->flags & HMAT_FLAG_FP64_ACCUM)
            return set_error(HMAT_ERR_INVALID_ARG, "members must not use the FP64 accuracy-check mode");
        if (h->storage > HMAT_STORE_BF16)
            return set_error(HMAT_ERR_UNSUPPORTED, "batches take FP32, FP16 and BF16 members");
        if (!h->mr) {
            if (nrhs[i] != 1)
                return set_error(HMAT_ERR_INVALID_ARG, "member " + std::to_string(i) + ": single-vector handle takes nrhs 1");
            b->has_s = true;
            b->lds = std::max(b->lds, (size_t)h->plan.lds_floats * 4);
        } else {
            if (nrhs[i] < 1 || nrhs[i] > std::min(16, h->max_nrhs))
                return set_error(HMAT_ERR_INVALID_ARG, "member " + std::to_string(i) + ": nrhs out of [1, min(16, max_nrhs)]");
            if (h->max_nseg > 64)
                return set_error(HMAT_ERR_UNSUPPORTED, "member " + std::to_string(i) + ": more than 64 target-side segments per chunk");
            b->has_m = true;
            b->zs_rank = std::max(b->zs_rank, h->max_zrows);
            // group bodies: two B slots of one n-tile, then (target side) a chunk's step table
            const size_t ring = (size_t)2 * 16 * (h->storage == HMAT_STORE_FP32 ? 64 : 128);
            b->lds = std::max(b->lds, ring + (size_t)8 * h->mrp.max_nsteps);
        }
    }
    b->zs_rank = (b->zs_rank + 3) / 4 * 4;
    if (b->has_m)  // z packing: rank x 16 values per wave (X packing takes no LDS: a wave per chunk)
        b->lds = std::max(b->lds, (size_t)4 * b->zs_rank * 16 * 4);
    b->lds = std::max<size_t>((b->lds + 15) / 16 * 16, 16);
    // take the references now: release_batch drops one per member
    for (int32_t i = 0; i < count; ++i) {
        if (!hmat::handle_live(hs[i], 1)) {
            return set_error(HMAT_ERR_INVALID_ARG, "member destroyed during batch creation");
        }
        b->members.push_back(hs[i]);
        b->k.push_back(nrhs[i]);
    }

    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail("hipSetDevice", e);
    e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) return hip_fail("hipDeviceGetAttribute", e);
    b->max_wg = hmat::batch_max_wg_per_cu(b->storage, b->has_s, b->has_m, b->lds);
    if (b->max_wg < 1) return set_error(HMAT_ERR_UNSUPPORTED, "the batched kernel does not fit on a compute unit");

    std::vector<BMember> mem(count);
    for (int32_t i = 0; i < count; ++i) {
        std::memset(&mem[i], 0, sizeof(BMember));
        mem[i].sp = b->members[i]->plan;
        mem[i].mp = b->members[i]->mrp;
        mem[i].mr = b->members[i]->mr ? 1 : 0;
        mem[i].k = nrhs[i];
    }
    b->num_ctl = 2 + 3 * count;
    if ((e = hipMalloc(&b->d_members, sizeof(BMember) * count)) != hipSuccess) return hip_fail("hipMalloc", e);
    if ((e = hipMalloc(&b->d_args, sizeof(BArgs) * count)) != hipSuccess) return hip_fail("hipMalloc", e);
    if ((e = hipMalloc(&b->d_ctl, sizeof(int32_t) * b->num_ctl)) != hipSuccess) return hip_fail("hipMalloc", e);
    if ((e = hipHostMalloc((void **)&b->h_args, sizeof(BArgs) * count, hipHostMallocDefault)) != hipSuccess) {
        b->h_args = nullptr;
        return hip_fail("hipHostMalloc", e);
    }
    if ((e = hipMemcpy(b->d_members, mem.data(), sizeof(BMember) * count, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail("hipMemcpy", e);
    if ((e = hipMemset(b->d_ctl, 0, sizeof(int32_t) * b->num_ctl)) != hipSuccess) return hip_fail("hipMemset", e);
    if ((e = hipEventCreateWithFlags(&b->args_ev, hipEventDisableTiming)) != hipSuccess) {
        b->args_ev = nullptr;
        return hip_fail("hipEventCreate", e);
    }
    if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
        b->cap = nullptr;
        return hip_fail("hipStreamCreate", e);
    }
    return configure(b);
}

// Validate the per-call operands and bring the device table up to date.
hmat_status stage_args(hmat_batch_handle *b, float alpha, const float *const *x, const int64_t *ldx, float beta,
                       float *const *y, const int64_t *ldy, hipStream_t st) {
    if (!x || !ldx || !y || !ldy) return set_error(HMAT_ERR_INVALID_ARG, "operand arrays must not be NULL");
    const size_t n = b->members.size();
    std::vector<BArgs> a(n);
    for (size_t i = 0; i < n; ++i) {
        const int64_t rows = b->members[i]->info.n;
        if (!x[i] || !y[i]) return set_error(HMAT_ERR_INVALID_ARG, "x or y of member " + std::to_string(i) + " is NULL");
        if (ldx[i] < rows || ldy[i] < rows)
            return set_error(HMAT_ERR_INVALID_ARG, "leading dimension of member " + std::to_string(i) + " below n");
        const int64_t k = b->k[i];
        const uintptr_t xb = (uintptr_t)x[i], xe = (uintptr_t)(x[i] + (k - 1) * ldx[i] + rows);
        const uintptr_t yb = (uintptr_t)y[i], ye = (uintptr_t)(y[i] + (k - 1) * ldy[i] + rows);
        if (xb < ye && yb < xe) return set_error(HMAT_ERR_INVALID_ARG, "x and y of member " + std::to_string(i) + " overlap");
        a[i] = BArgs{x[i], y[i], ldx[i], ldy[i], alpha, beta};
    }
    if (b->args_valid && std::memcmp(a.data(), b->cur_args.data(), n * sizeof(BArgs)) == 0) return HMAT_OK;
    hipError_t e;
    if (b->args_ev_pending) {  // the staging buffer is reused: its previous copy must have run
        if ((e = hipEventSynchronize(b->args_ev)) != hipSuccess) return hip_fail("hipEventSynchronize", e);
    }
    std::memcpy(b->h_args, a.data(), n * sizeof(BArgs));
    if ((e = hipMemcpyAsync(b->d_args, b->h_args, n * sizeof(BArgs), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail("hipMemcpyAsync", e);
    if ((e = hipEventRecord(b->args_ev, st)) != hipSuccess) return hip_fail("hipEventRecord", e);
    b->args_ev_pending = true;
    b->cur_args = a;
    b->args_valid = true;
    return HMAT_OK;
}

hmat_status run(hmat_batch_handle *b, hipStream_t st) {
    if (b->opts.use_graph) {
        const hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
        return HMAT_OK;
    }
    const int e = hmat::launch_batch(kernel_args(b), b->storage, b->has_s, b->has_m, b->grid, b->lds, st);
    if (e != 0) return hip_fail("batched launch", (hipError_t)e);
    return HMAT_OK;
}

hmat_status ensure_device(const hmat_batch_handle *b) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != b->device) {
        const hipError_t e = hipSetDevice(b->device);
        if (e != hipSuccess) return hip_fail("hipSetDevice", e);
    }
    return HMAT_OK;
}

// ---- autotuner cache (JSON) ------------------------------------------------
uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

std::string batch_key(const hmat_batch_handle *b) {
    uint64_t h = 1469598103934665603ull;
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess)
        h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    h = fnv1a(h, &b->cus, sizeof(b->cus));
    h = fnv1a(h, &b->storage, sizeof(b->storage));
    for (size_t i = 0; i < b->members.size(); ++i) {
        const hmat_handle *m = b->members[i];
        const int64_t v[6] = {m->info.n, m->info.leaf_depth, m->info.stored_elements, m->mr ? 1 : 0, b->k[i],
                              (int64_t)m->cost_src.size() * 1000003 + (int64_t)m->cost_tgt.size()};
        h = fnv1a(h, v, sizeof(v));
    }
    char buf[17];
    std::snprintf(buf, sizeof(buf), "%016" PRIx64, h);
    return buf;
}

struct CacheEntry {
    std::string key;
    int wg = 0, order = 0, grain = 0;
    double ms = 0.0;
};

// Entries of a cache file written by save_cache (unknown text is skipped).
std::vector<CacheEntry> load_cache(const char *path) {
    std::vector<CacheEntry> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find("\"key\": \"", pos)) != std::string::npos) {
        pos += 8;
        const size_t end = s.find('"', pos);
        const size_t close = s.find('}', pos);
        if (end == std::string::npos || close == std::string::npos) break;
        CacheEntry c;
        c.key = s.substr(pos, end - pos);
        const std::string obj = s.substr(end, close - end);
        auto num = [&](const char *name, double *v) {
            const size_t q = obj.find(name);
            return q != std::string::npos && std::sscanf(obj.c_str() + q + std::strlen(name), " : %lf", v) == 1;
        };
        double wg = 0, order = 0, grain = 0, ms = 0;
        if (num("\"wg_per_cu\"", &wg) && num("\"order\"", &order) && num("\"grain_kb\"", &grain) &&
            num("\"ms\"", &ms)) {
            c.wg = (int)wg;
            c.order = (int)order;
            c.grain = (int)grain;
            c.ms = ms;
            out.push_back(c);
        }
        pos = close;
    }
    return out;
}

bool save_cache(const char *path, const std::vector<CacheEntry> &entries) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n  \"format\": \"hmat-batch-tuning-1\",\n  \"entries\": [";
        for (size_t i = 0; i < entries.size(); ++i) {
            char line[256];
            std::snprintf(line, sizeof(line),
                          "%s\n    {\"key\": \"%s\", \"wg_per_cu\": %d, \"order\": %d, \"grain_kb\": %d, \"ms\": %.6f}",
                          i ? "," : "", entries[i].key.c_str(), entries[i].wg, entries[i].order, entries[i].grain,
                          entries[i].ms);
            f << line;
        }
        f << "\n  ]\n}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

hmat_status hmat_batch_create(const hmat_t *members, int32_t count, const int32_t *nrhs,
                              const hmat_batch_options *opts, hmat_batch_t *out) {
    if (!out) return set_error(HMAT_ERR_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    set_error(HMAT_OK, "");
    hmat_batch_handle *b = nullptr;
    try {
        b = new hmat_batch_handle();
        const hmat_status s = create_impl(members, count, nrhs, opts, b);
        if (s != HMAT_OK) {
            release_batch(b);
            return s;
        }
    } catch (const std::bad_alloc &) {
        release_batch(b);
        return set_error(HMAT_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        release_batch(b);
        return set_error(HMAT_ERR_INVALID_ARG, std::string("internal error: ") + e.what());
    }
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        g_blive.insert(b);
    }
    *out = b;
    return HMAT_OK;
}

hmat_status hmat_batch_matvec(hmat_batch_t b, float alpha, const float *const *x, const int64_t *ldx, float beta,
                              float *const *y, const int64_t *ldy, void *stream) {
    if (!b || !batch_live(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown batch");
    hmat_status s = ensure_device(b);
    if (s != HMAT_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    try {
        if ((s = stage_args(b, alpha, x, ldx, beta, y, ldy, st)) != HMAT_OK) return s;
    } catch (const std::bad_alloc &) {
        return set_error(HMAT_ERR_NOMEM, "host allocation failed");
    }
    return run(b, st);
}

hmat_status hmat_batch_sync(hmat_batch_t b, void *stream) {
    if (!b || !batch_live(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown batch");
    hmat_status s = ensure_device(b);
    if (s != HMAT_OK) return s;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail("hipStreamSynchronize", e);
    int32_t flag = 0;
    if ((e = hipMemcpy(&flag, b->d_ctl + 1, sizeof(flag), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail("hipMemcpy", e);
    if (flag != 0)
        return set_error(HMAT_ERR_DEVICE, "a dependency wait of the batched kernel reached its poll limit");
    return HMAT_OK;
}

hmat_status hmat_batch_set_options(hmat_batch_t b, const hmat_batch_options *opts) {
    if (!b || !batch_live(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown batch");
    if (!opts) return set_error(HMAT_ERR_INVALID_ARG, "options pointer is NULL");
    hmat_status s = check_options(opts);
    if (s != HMAT_OK) return s;
    if ((s = ensure_device(b)) != HMAT_OK) return s;
    // the queue is rewritten in place: earlier calls on any stream must be done
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail("hipDeviceSynchronize", e);
    b->opts = *opts;
    try {
        return configure(b);
    } catch (const std::bad_alloc &) {
        return set_error(HMAT_ERR_NOMEM, "host allocation failed");
    }
}

hmat_status hmat_batch_get_info(hmat_batch_t b, hmat_batch_info *info) {
    if (!b || !batch_live(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown batch");
    if (!info) return set_error(HMAT_ERR_INVALID_ARG, "info pointer is NULL");
    hmat_batch_info r{};
    r.count = (int32_t)b->members.size();
    r.num_items = b->num_items;
    r.grid = b->grid;
    r.wg_per_cu = b->cus ? b->grid / b->cus : 0;
    r.max_wg_per_cu = b->max_wg;
    r.order = b->opts.order;
    r.use_graph = b->opts.use_graph;
    r.grain_kb = b->opts.grain_kb > 0 ? b->opts.grain_kb : kDefaultGrainKb;
    r.lds_bytes = (int64_t)b->lds;
    r.item_bytes = b->item_bytes;
    *info = r;
    return HMAT_OK;
}

hmat_status hmat_batch_autotune(hmat_batch_t b, float alpha, const float *const *x, const int64_t *ldx,
                                float beta, float *const *y, const int64_t *ldy, void *stream,
                                const char *cache_path, int32_t reps, hmat_batch_options *chosen) {
    if (!b || !batch_live(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown batch");
    if (reps < 1) return set_error(HMAT_ERR_INVALID_ARG, "reps must be >= 1");
    hmat_status s = ensure_device(b);
    if (s != HMAT_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    try {
        const std::string key = batch_key(b);
        std::vector<CacheEntry> cache;
        if (cache_path) cache = load_cache(cache_path);
        hmat_batch_options best = b->opts;
        bool hit = false;
        for (const CacheEntry &c : cache)
            if (c.key == key && c.wg >= 1 && c.wg <= b->max_wg && (c.order == 0 || c.order == 1) && c.grain >= 1 &&
                c.grain <= (1 << 20)) {
                best.wg_per_cu = c.wg;
                best.order = c.order;
                best.grain_kb = c.grain;
                hit = true;
            }
        double best_ms = 0.0;
        if (!hit) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            hipError_t e = hipEventCreate(&e0);
            if (e == hipSuccess) e = hipEventCreate(&e1);
            if (e != hipSuccess) {
                if (e0) (void)hipEventDestroy(e0);
                return hip_fail("hipEventCreate", e);
            }
            double best_t = 1e300;
            for (int wg : {1, 2, 4, 8}) {
                if (wg > b->max_wg) continue;
                for (int cand = 0; cand < 6; ++cand) {
                    hmat_batch_options o = b->opts;
                    o.wg_per_cu = wg;
                    o.order = cand & 1;
                    o.grain_kb = cand < 2 ? 128 : cand < 4 ? 512 : 2048;
                    if ((s = hmat_batch_set_options(b, &o)) != HMAT_OK) break;
                    for (int w = 0; w < 2 && s == HMAT_OK; ++w) s = hmat_batch_matvec(b, alpha, x, ldx, beta, y, ldy, st);
                    if (s == HMAT_OK && (e = hipEventRecord(e0, st)) != hipSuccess) s = hip_fail("hipEventRecord", e);
                    for (int r = 0; r < reps && s == HMAT_OK; ++r) s = hmat_batch_matvec(b, alpha, x, ldx, beta, y, ldy, st);
                    if (s == HMAT_OK && (e = hipEventRecord(e1, st)) != hipSuccess) s = hip_fail("hipEventRecord", e);
                    if (s == HMAT_OK) s = hmat_batch_sync(b, st);
                    float ms = 0.0f;
                    if (s == HMAT_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) s = hip_fail("hipEventElapsedTime", e);
                    if (s != HMAT_OK) break;
                    if (ms / reps < best_t) {
                        best_t = ms / reps;
                        best = o;
                    }
                }
                if (s != HMAT_OK) break;
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (s != HMAT_OK) return s;
            best_ms = best_t;
        }
        if ((s = hmat_batch_set_options(b, &best)) != HMAT_OK) return s;
        if (!hit && cache_path) {
            std::vector<CacheEntry> keep;
            for (const CacheEntry &c : cache)
                if (c.key != key) keep.push_back(c);
            keep.push_back(CacheEntry{key, best.wg_per_cu, best.order, best.grain_kb, best_ms});
            if (!save_cache(cache_path, keep))
                return set_error(HMAT_ERR_INVALID_ARG, std::string("cannot write the tuning cache ") + cache_path);
        }
        if (chosen) *chosen = best;
        return HMAT_OK;
    } catch (const std::bad_alloc &) {
        return set_error(HMAT_ERR_NOMEM, "host allocation failed");
    }
}

hmat_status hmat_batch_destroy(hmat_batch_t b) {
    if (!b) return HMAT_OK;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        if (!g_blive.erase(b)) return set_error(HMAT_ERR_INVALID_ARG, "unknown or already destroyed batch");
    }
    (void)hipSetDevice(b->device);
    release_batch(b);
    return HMAT_OK;
}

}  // extern "C"
