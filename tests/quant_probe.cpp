// Test probe: exposes libhmat's host quantisers (compiled from the library
// source) on stdin/stdout. Input: float32 values; output per value: the FP16
// code of v * inv, the BF16 code of v, and the power-of-two FP16 scale of |v|.
#include "../paper_2008_12441_amd/csrc/hmat_host.cpp"

#include <cstdio>

// The probe never launches kernels; these stand in for the HIP launchers.
namespace hmat {
int launch_vphase(const DevPlan &, const float *, void *) { return 1; }
int launch_zfinish(const DevPlan &, void *) { return 1; }
int launch_uphase(const DevPlan &, const float *, float *, float, float, void *) { return 1; }
int launch_probe(const void *, void *, int64_t, int32_t, void *) { return 1; }
int launch_mr(const DevPlanMR &, int32_t, float, const float *, int64_t, float, float *, int64_t, void *,
              void (*)(void *, int), void *) {
    return 1;
}
}  // namespace hmat

int main(int argc, char **argv) {
    const float inv = argc > 1 ? std::strtof(argv[1], nullptr) : 1.0f;
    float v;
    while (std::fread(&v, 4, 1, stdin) == 1) {
        const uint16_t h = quant16(v, inv, false);
        const uint16_t b = quant16(v, inv, true);
        const float s = pow2_scale_f16(std::fabs(v));
        std::fwrite(&h, 2, 1, stdout);
        std::fwrite(&b, 2, 1, stdout);
        std::fwrite(&s, 4, 1, stdout);
    }
    return 0;
}
