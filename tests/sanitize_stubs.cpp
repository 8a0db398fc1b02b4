// Host stand-ins for the HIP runtime and the library's kernel launchers, so that
// the library's host sources can be built for the CPU alone (with AddressSanitizer
// and UndefinedBehaviorSanitizer) and driven through the C ABI: "device" memory is
// host memory, copies are memcpy, launches do nothing, events and streams are
// empty objects. Used by tests/test_sanitize_cpu.py only.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>

#include "hmat.h"
#include "hmat_compress.h"
#include "hmat_h2_internal.h"
#include "hmat_internal.h"

namespace {
struct Dummy {
    int v = 0;
};
}  // namespace

extern "C" {
hipError_t hipMalloc(void **ptr, size_t size) {
    *ptr = std::calloc(1, size ? size : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *ptr) {
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int) { return hipMalloc(ptr, size); }
hipError_t hipHostFree(void *ptr) { return hipFree(ptr); }
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(dst, src, n, k);
}
hipError_t hipMemset(void *dst, int value, size_t n) {
    std::memset(dst, value, n);
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipGetDeviceCount(int *c) {
    *c = 1;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_t *prop, int) {
    std::memset(prop, 0, sizeof(*prop));
    std::strcpy(prop->gcnArchName, "gfx950");
    prop->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "stand-in"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = reinterpret_cast<hipEvent_t>(new Dummy);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<Dummy *>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    *s = reinterpret_cast<hipStream_t>(new Dummy);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<Dummy *>(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = reinterpret_cast<hipGraph_t>(new Dummy);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    *x = reinterpret_cast<hipGraphExec_t>(new Dummy);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<Dummy *>(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    delete reinterpret_cast<Dummy *>(x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
}

namespace hmat {
int launch_vphase(const DevPlan &, const float *, void *) { return 0; }
int launch_zfinish(const DevPlan &, void *) { return 0; }
int launch_uphase(const DevPlan &, const float *, float *, float, float, void *) { return 0; }
int launch_probe(const void *, void *, int64_t, int32_t, void *) { return 0; }
int launch_mr(const DevPlanMR &, int32_t, float, const float *, int64_t, float, float *, int64_t, void *,
              void (*mark)(void *, int), void *ctx) {
    if (mark)
        for (int ph = 0; ph < HMAT_NUM_PHASES + 1; ++ph) mark(ctx, ph);
    return 0;
}
int launch_batch(const BatchArgs &, int32_t, bool, bool, int, size_t, void *) { return 0; }
int batch_max_wg_per_cu(int32_t, bool, bool, size_t) { return 2; }
int scratch_address(int, void **ptr) {
    static void *p = std::calloc(1, (size_t)HMAT_NOALLOC_SCRATCH_BYTES);
    *ptr = p;
    return 0;
}
int launch_compress_dense(const CKernel &, const CDense *, const CTile *, int64_t, float *, void *) { return 0; }
int launch_compress_sample(const CKernel &, const CWork &, const CTile *, int64_t, int, void *) { return 0; }
int launch_compress_gram(const CWork &, int64_t, int, void *) { return 0; }
int launch_compress_eig(const CWork &, int64_t, int, void *) { return 0; }
int launch_compress_apply(const CWork &, const CTile *, int64_t, int, void *) { return 0; }
int launch_h2_upward(const DevPlanH2 &, const float *, void *) { return 0; }
int launch_h2_up(const DevPlanH2 &, int32_t, int32_t, void *) { return 0; }
int launch_h2_down(const DevPlanH2 &, int32_t, int32_t, void *) { return 0; }
int launch_h2_leaf(const DevPlanH2 &, const float *, float *, float, float, void *) { return 0; }
}  // namespace hmat
