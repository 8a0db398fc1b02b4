// Test probe: exposes libhmat's host quantisers (compiled from the library
// source) on stdin/stdout.
//   quant_probe INV        float32 values in; per value: the FP16 code of
//                          v * inv, the BF16 code of v, the FP16 scale of |v|
//   quant_probe e4m3       float32 values in; per value: the E4M3 code of v
//                          (|v| <= 448) and the E4M3 scale of |v| (double)
//   quant_probe fp8col     int32 rows, cols, then a column-major float32
//                          factor; out: per column s_j, s'_j (float32), then
//                          per element its hi and lo codes
//   quant_probe blk16      int32 mode, then one stored array (float32) as the
//                          library quantises a whole block array: mode 0 the
//                          FP16 form (per-array scale s, FP16 codes of v / s),
//                          mode 1 the FP8 forms' dense rule (BF16 codes of
//                          v / s with the same s); out: s (float32), then one
//                          16-bit code per value
#include "../paper_2008_12441_amd/csrc/hmat_host.cpp"
#include "../paper_2008_12441_amd/csrc/hmat_structure.cpp"

#include <cstdio>

// The probe never launches kernels; these stand in for the HIP launchers.
namespace hmat {
int launch_vphase(const DevPlan &, const float *, void *) { return 1; }
int launch_zfinish(const DevPlan &, void *) { return 1; }
int launch_uphase(const DevPlan &, const float *, float *, float, float, void *) { return 1; }
int launch_probe(const void *, void *, int64_t, int32_t, void *) { return 1; }
int scratch_address(int, void **) { return 1; }
int launch_mr(const DevPlanMR &, int32_t, float, const float *, int64_t, float, float *, int64_t, void *,
              void (*)(void *, int), void *) {
    return 1;
}
int launch_compress_dense(const CKernel &, const CDense *, const CTile *, int64_t, float *, void *) { return 1; }
int launch_compress_sample(const CKernel &, const CWork &, const CTile *, int64_t, int, void *) { return 1; }
int launch_compress_gram(const CWork &, int64_t, int, void *) { return 1; }
int launch_compress_eig(const CWork &, int64_t, int, void *) { return 1; }
int launch_compress_apply(const CWork &, const CTile *, int64_t, int, void *) { return 1; }
}  // namespace hmat

int main(int argc, char **argv) {
    if (argc > 1 && std::strcmp(argv[1], "e4m3") == 0) {
        float v;
        while (std::fread(&v, 4, 1, stdin) == 1) {
            const uint8_t c = std::fabs(v) <= 448.0f ? e4m3_rne(v) : 0;
            const double s = pow2_scale_e4m3(std::fabs((double)v));
            std::fwrite(&c, 1, 1, stdout);
            std::fwrite(&s, 8, 1, stdout);
        }
        return 0;
    }
    if (argc > 1 && std::strcmp(argv[1], "fp8col") == 0) {
        int32_t dims[2];
        if (std::fread(dims, 4, 2, stdin) != 2) return 1;
        std::vector<float> a((size_t)dims[0] * dims[1]);
        if (std::fread(a.data(), 4, a.size(), stdin) != a.size()) return 1;
        std::vector<float> sc(2 * (size_t)dims[1]);
        e4m3_column_scales(a.data(), dims[0], dims[1], dims[0], sc.data());
        std::fwrite(sc.data(), 4, sc.size(), stdout);
        for (int32_t j = 0; j < dims[1]; ++j)
            for (int32_t i = 0; i < dims[0]; ++i) {
                uint8_t hl[2];
                e4m3_hilo(a[i + (size_t)j * dims[0]], sc[2 * j], sc[2 * j + 1], &hl[0], &hl[1]);
                std::fwrite(hl, 1, 2, stdout);
            }
        return 0;
    }
    if (argc > 1 && std::strcmp(argv[1], "blk16") == 0) {
        int32_t mode = 0;
        if (std::fread(&mode, 4, 1, stdin) != 1) return 1;
        std::vector<float> a;
        float v;
        while (std::fread(&v, 4, 1, stdin) == 1) a.push_back(v);
        bool finite = true;
        const float amax = col_major_amax(a.data(), (int64_t)a.size(), 1, (int64_t)a.size(), &finite);
        const float sc = pow2_scale_f16(amax);
        std::fwrite(&sc, 4, 1, stdout);
        for (float e : a) {
            const uint16_t c = mode == 0 ? quant16(e, 1.0f / sc, false) : f32_to_bf16_rne(e * (1.0f / sc));
            std::fwrite(&c, 2, 1, stdout);
        }
        return 0;
    }
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
