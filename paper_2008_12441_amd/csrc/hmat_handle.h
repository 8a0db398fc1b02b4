// Host-side state of a handle, shared by the sources of the host library
// (hmat_host.cpp: single handles; hmat_batch_host.cpp: batches).
#pragma once

#include "hmat.h"
#include "hmat_internal.h"

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

struct hmat_handle {
    int32_t device = 0;
    int32_t storage = 0;
    int32_t max_nrhs = 1;
    int32_t flags = 0;
    hmat_info info{};
    bool mr = false;               // multi-RHS (MFMA) layout
    hmat::DevPlan plan{};
    hmat::DevPlanMR mrp{};
    std::vector<void *> dev_allocs;
    // work estimates for schedulers: bytes streamed per source-side work index
    // (vtile, or V unit group) and per target-side work index (chunk, or row
    // tile group)
    std::vector<float> cost_src, cost_tgt;
    std::vector<float> cost_z1, cost_z2;  // per reduction item (multi-RHS: z items in cost_z1)
    std::vector<int32_t> chunk_rows;  // rows of each chunk
    int32_t max_nseg = 0;             // multi-RHS: most target-side segments of a chunk
    int32_t max_rank = 0;             // largest rank of a low-rank block
    int32_t max_zrows = 0;            // multi-RHS: most z rows of a z item (the blocks of one target box)
    // single-vector workspace sizes in bytes (partial sums; z vectors; stage-1 slices)
    int64_t ws_part_bytes = 0, ws_zg_bytes = 0, ws_slice_bytes = 0;
    int32_t batch_refs = 0;           // batches that reference this handle (guarded by the registry lock)
    // phase timing
    bool timing = false;
    std::vector<hipEvent_t> events;   // HMAT_NUM_PHASES + 1 per timed column
    size_t events_used = 0;
    double ms[HMAT_NUM_PHASES] = {0, 0, 0};
    int64_t timed_calls = 0;
};

namespace hmat {
// Record msg as the calling thread's last error and return s.
hmat_status set_error(hmat_status s, const std::string &msg);
// Whether h is a live handle; when add_ref is nonzero, also adjust its batch
// reference count by add_ref under the registry lock (only when live).
bool handle_live(const hmat_handle *h, int add_ref = 0);
}  // namespace hmat
