// HIP kernels (gfx950) of the single-vector H-matrix-vector product.
//
// One product y = alpha K x + beta y runs as four launches on the caller's
// stream, the single-GPU form of the five steps of Sec. 4.1 (bodies in
// hmat_sv_device.h): k_vphase (one wave per vtile), k_zsum1/k_zsum2 (one wave
// per reduction item) and k_uphase (one workgroup per chunk). All streams are
// HBM-bound (two flops per stored element); the layouts make every wave-level
// load a contiguous 1 KiB.
#include "hmat_sv_device.h"

#include <mutex>

namespace hmat {
namespace {

using namespace hmat::dev;

__device__ inline int wave_id_in_grid(int waves_per_block) {
    return __builtin_amdgcn_readfirstlane((int)blockIdx.x * waves_per_block + (int)(threadIdx.x >> 6));
}

template <int STORE, class Acc>
__global__ __launch_bounds__(256) void k_vphase(DevPlan p, const float *__restrict__ x) {
    const int w = wave_id_in_grid(4);
    if (w >= p.num_vtiles) return;
    sv_vtile<STORE, Acc>(p, w, threadIdx.x & 63, x);
}

template <class Acc>
__global__ __launch_bounds__(256) void k_zsum1(DevPlan p) {
    const int w = wave_id_in_grid(4);
    if (w >= p.num_z1) return;
    sv_z1<Acc>(p, w, threadIdx.x & 63);
}

template <class Acc>
__global__ __launch_bounds__(256) void k_zsum2(DevPlan p) {
    const int w = wave_id_in_grid(4);
    if (w >= p.num_z2) return;
    sv_z2<Acc>(p, w, threadIdx.x & 63);
}

template <int STORE, class Acc>
__global__ __launch_bounds__(256) void k_uphase(DevPlan p, const float *__restrict__ x, float *__restrict__ y,
                                                float alpha, float beta) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    sv_chunk<STORE, Acc>(p, blockIdx.x, threadIdx.x, reinterpret_cast<Acc *>(lds_raw), x, y, alpha, beta);
}

// ---------------------------------------------------------------------------
// Bandwidth probe. Read: every wave streams one contiguous span of the buffer
// (the access pattern of the product kernels, whose waves each walk a panel),
// 16 nontemporal 16-byte loads per lane in flight, i.e. 16 KiB per wave; the
// grid is the number of workgroups that fit on the chip at once, so every
// wave stays resident for the whole read. The sum stays live. Copy: a
// grid-stride copy of 16-byte vectors.
// ---------------------------------------------------------------------------
constexpr int kProbeLoads = 16;

__global__ __launch_bounds__(256) void k_probe_read(const f32x4 *__restrict__ src, int64_t n4, int64_t span,
                                                    float *__restrict__ out) {
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t b0 = wave * span;
    const int64_t b1 = b0 + span < n4 ? b0 + span : n4;
    f32x4 acc = {0, 0, 0, 0};
    int64_t i = b0;
    for (; i + kProbeLoads * 64 <= b1; i += kProbeLoads * 64) {
        f32x4 v[kProbeLoads];
#pragma unroll
        for (int u = 0; u < kProbeLoads; ++u) v[u] = __builtin_nontemporal_load(src + i + u * 64 + lane);
#pragma unroll
        for (int u = 0; u < kProbeLoads; ++u) acc += v[u];
    }
    for (i += lane; i < b1; i += 64) acc += src[i];
    __shared__ float red[256];
    red[threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_probe_copy(const f32x4 *__restrict__ src, int64_t n4, f32x4 *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

template <class Acc>
static void launch_vphase_acc(const DevPlan &p, const float *x, hipStream_t st) {
    const int blocks = (p.num_vtiles + 3) / 4;
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_vphase<HMAT_STORE_FP16_SCALED, Acc>), dim3(blocks), dim3(256), 0, st, p, x);
    else if (p.storage == HMAT_STORE_BF16)
        hipLaunchKernelGGL((k_vphase<HMAT_STORE_BF16, Acc>), dim3(blocks), dim3(256), 0, st, p, x);
    else
        hipLaunchKernelGGL((k_vphase<HMAT_STORE_FP32, Acc>), dim3(blocks), dim3(256), 0, st, p, x);
}

int launch_vphase(const DevPlan &p, const float *x, void *stream) {
    if (p.fp64)
        launch_vphase_acc<double>(p, x, (hipStream_t)stream);
    else
        launch_vphase_acc<float>(p, x, (hipStream_t)stream);
    return (int)hipGetLastError();
}

template <class Acc>
static int launch_zfinish_acc(const DevPlan &p, hipStream_t st) {
    hipLaunchKernelGGL(k_zsum1<Acc>, dim3((p.num_z1 + 3) / 4), dim3(256), 0, st, p);
    int e = (int)hipGetLastError();
    if (e != 0 || p.num_z2 == 0) return e;
    hipLaunchKernelGGL(k_zsum2<Acc>, dim3((p.num_z2 + 3) / 4), dim3(256), 0, st, p);
    return (int)hipGetLastError();
}

int launch_zfinish(const DevPlan &p, void *stream) {
    return p.fp64 ? launch_zfinish_acc<double>(p, (hipStream_t)stream)
                  : launch_zfinish_acc<float>(p, (hipStream_t)stream);
}

template <class Acc>
static void launch_uphase_acc(const DevPlan &p, const float *x, float *y, float alpha, float beta,
                              hipStream_t st) {
    const size_t lds = (size_t)p.lds_floats * sizeof(Acc);
    if (p.storage == HMAT_STORE_FP16_SCALED)
        hipLaunchKernelGGL((k_uphase<HMAT_STORE_FP16_SCALED, Acc>), dim3(p.num_chunks), dim3(256), lds, st, p, x,
                           y, alpha, beta);
    else if (p.storage == HMAT_STORE_BF16)
        hipLaunchKernelGGL((k_uphase<HMAT_STORE_BF16, Acc>), dim3(p.num_chunks), dim3(256), lds, st, p, x, y,
                           alpha, beta);
    else
        hipLaunchKernelGGL((k_uphase<HMAT_STORE_FP32, Acc>), dim3(p.num_chunks), dim3(256), lds, st, p, x, y,
                           alpha, beta);
}

int launch_uphase(const DevPlan &p, const float *x, float *y, float alpha, float beta, void *stream) {
    if (p.fp64)
        launch_uphase_acc<double>(p, x, y, alpha, beta, (hipStream_t)stream);
    else
        launch_uphase_acc<float>(p, x, y, alpha, beta, (hipStream_t)stream);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Library-owned scratch of hmat_matvec_noalloc: the single-vector workspace
// of a product (partial sums of V^T x, stage-1 slice sums, z vectors) held in
// a static device array instead of the handle's own allocation. Every device
// the library runs on holds its own copy until the process ends. In host code
// the array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns on each device, fetched once per device below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HMAT_NOALLOC_SCRATCH_BYTES];

int scratch_address(int device, void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return 0;
}

int launch_probe(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream) {
    const int64_t n4 = bytes / 16;
    if (mode == 0) {
        // as many workgroups as are resident at once (at most 65536, the size of dst)
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_read, 256, 0);
        if (e != hipSuccess) return (int)e;
        int64_t blocks = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
        if (blocks > 65536) blocks = 65536;
        // each wave's span: whole 16 KiB steps, so only the last wave has a ragged end
        const int64_t waves = blocks * 4, step = kProbeLoads * 64;
        const int64_t span = ((n4 + waves - 1) / waves + step - 1) / step * step;
        hipLaunchKernelGGL(k_probe_read, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                           static_cast<const f32x4 *>(src), n4, span, static_cast<float *>(dst));
    } else {
        int64_t blocks = (n4 + 256 * 8 - 1) / (256 * 8);
        if (blocks > 4096) blocks = 4096;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                           static_cast<const f32x4 *>(src), n4, static_cast<f32x4 *>(dst));
    }
    return (int)hipGetLastError();
}

}  // namespace hmat
