// Issue rates of the transcendental 2^x (v_exp_f32), the fused multiply-add
// (v_fma_f32) and the gap-junction pair term's instruction mix on this GPU:
// a stand-alone measurement program, not part of the library. The ALU
// rooflines count work in FMA issue slots; this program measures what an
// exponential costs in them, and whether it overlaps with the FMA-class
// operations around it (the pair term: a subtraction, a multiply, the
// exponential and a fused multiply-add).
//
// Each thread runs eight independent chains in registers (no memory access
// until one store of the result per thread): x <- 2^(-x), which stays in
// [0.5, 1]; x <- x * a + b with |a| < 1, which stays bounded; and
// v = x - 1/2, x <- 2^(-v*v) * 1/2 + 1/4, which stays in (0.25, 0.75]. The
// grid holds eight 256-thread workgroups per compute unit.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o probe_exp_rate probe_exp_rate.hip && ./probe_exp_rate
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

constexpr int kChains = 8;
constexpr int kIters = 8192;

__global__ __launch_bounds__(256) void k_exp_chain(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fma_chain(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
    const float a = 0.999f, b = 1e-3f;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_pair_chain(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * c + 1e-6f * threadIdx.x;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const float v = x[c] - 0.5f;
            x[c] = __builtin_fmaf(__builtin_amdgcn_exp2f(-(v * v)), 0.5f, 0.25f);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename K>
double rate(K kernel, int blocks, float* d_out) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, 0, d_out, 0.5f);   // warm-up
    CHECK(hipGetLastError());
    float best = 1e30f;
    for (int r = 0; r < 5; ++r) {
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, 0, d_out, 0.5f);
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        best = ms < best ? ms : best;
    }
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return (double)blocks * 256 * kIters * kChains / (best * 1e-3);
}

int main() {
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = 8 * cus;
    float* d_out = nullptr;
    CHECK(hipMalloc(&d_out, sizeof(float) * blocks * 256));
    const double ex = rate(k_exp_chain, blocks, d_out);
    const double fm = rate(k_fma_chain, blocks, d_out);
    const double pr = rate(k_pair_chain, blocks, d_out);
    std::printf("{\"compute_units\": %d, \"exp_per_s\": %.4g, \"fma_per_s\": %.4g, \"fma_slots_per_exp\": %.3f, "
                "\"pair_mix_per_s\": %.4g, \"fma_slots_per_pair_mix\": %.3f}\n",
                cus, ex, fm, fm / ex, pr, fm / pr);
    CHECK(hipFree(d_out));
    return 0;
}
