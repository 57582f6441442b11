// issue_probe.hip -- vector issue rate of the instruction classes the step
// kernel is made of, measured on the device it runs on.
//
// The step kernel's roofline prices every operation at the FP64 vector rate
// (64 lanes x 2 flops per FMA per CU and clock).  That is the rate of FP32
// arithmetic too only while FP32 is issued unpacked, which is how this
// library is compiled.  This program checks it: each kernel runs eight
// independent dependency chains of one instruction per thread (enough
// independent work to hide the pipeline latency), on 32 wavefronts of
// 256 threads per CU, and prints the measured lane-instructions per second
// and the implied clocks per wave64 instruction per SIMD (at 2.4 GHz, 256
// CUs x 4 SIMDs).
//
//   fp32 fma      v_fma_f32 (packed FP32 disabled at compile time)
//   fp64 fma      v_fma_f64
//   mad_u64_u32   the 32x32->64 product-add of the Philox rounds
//   bitop3        the three-input XOR of the Philox rounds
//   log/sqrt/sin/rcp_f32, rcp/rsq_f64   the hardware transcendental and
//                 reciprocal instructions of the FP32 form's elementary
//                 functions and the FP64 form's quotients and square roots
//
// Build: hipcc --offload-arch=gfx950 -O3 (with packed FP32 disabled, as for
// the library); run: ./issue_probe.  Exit status 0 on success.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kChains = 8, kUnroll = 8;

__global__ __launch_bounds__(256) void k_fp32(float *out, int iters, float a, float b) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-7f + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = fmaf(x[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fp64(double *out, int iters, double a, double b) {
    double x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-7 + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = fma(x[k], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mad_u64(uint64_t *out, int iters, uint32_t m) {
    uint64_t x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 7u + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = (uint64_t)(uint32_t)x[k] * m + x[k];
    }
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s ^= x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_bitop3(uint32_t *out, int iters, uint32_t c) {
    uint32_t x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 7u + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_bitop3_b32(x[k], x[(k + 1) % kChains], c, 0x96);
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s ^= x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// transcendental and reciprocal classes: one hardware instruction per step
// (|x| is a free source modifier; the values may reach infinities or NaN,
// which does not change the issue rate)
template <int kOp>
__global__ __launch_bounds__(256) void k_trans32(float *out, int iters) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-7f + k + 0.5f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (kOp == 0) x[k] = __builtin_amdgcn_logf(fabsf(x[k]));
                if constexpr (kOp == 1) x[k] = __builtin_amdgcn_sqrtf(fabsf(x[k]));
                if constexpr (kOp == 2) x[k] = __builtin_amdgcn_sinf(x[k]);
                if constexpr (kOp == 3) x[k] = __builtin_amdgcn_rcpf(x[k]);
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int kOp>
__global__ __launch_bounds__(256) void k_trans64(double *out, int iters) {
    double x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-7 + k + 0.5;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (kOp == 0) x[k] = __builtin_amdgcn_rcp(x[k]);
                if constexpr (kOp == 1) x[k] = __builtin_amdgcn_rsq(fabs(x[k]));
            }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

bool ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    std::fprintf(stderr, "issue_probe: %s: %s\n", what, hipGetErrorString(e));
    return false;
}

}  // namespace

int main() {
    const int blocks = 256 * 32, threads = 256, iters = 4096;
    const size_t n = (size_t)blocks * threads;
    void *buf = nullptr;
    if (!ok(hipMalloc(&buf, n * sizeof(uint64_t)), "hipMalloc")) return 1;
    hipEvent_t e0, e1;
    if (!ok(hipEventCreate(&e0), "hipEventCreate") || !ok(hipEventCreate(&e1), "hipEventCreate")) return 1;
    const double lane_instr = (double)n * iters * kUnroll * kChains;
    const char *names[10] = {"fp32 fma", "fp64 fma", "mad_u64_u32", "bitop3", "log_f32", "sqrt_f32",
                             "sin_f32", "rcp_f32", "rcp_f64", "rsq_f64"};
    std::printf("%-12s %10s %22s %30s\n", "class", "ms", "lane-instr/s (1e12)", "clocks per wave64 instr/SIMD");
    for (int rep = 0; rep < 2; ++rep) {
        for (int w = 0; w < 10; ++w) {
            if (!ok(hipEventRecord(e0, 0), "hipEventRecord")) return 1;
            if (w == 0) hipLaunchKernelGGL(k_fp32, dim3(blocks), dim3(threads), 0, 0, (float *)buf, iters, 0.999f, 1e-3f);
            if (w == 1) hipLaunchKernelGGL(k_fp64, dim3(blocks), dim3(threads), 0, 0, (double *)buf, iters, 0.999, 1e-3);
            if (w == 2) hipLaunchKernelGGL(k_mad_u64, dim3(blocks), dim3(threads), 0, 0, (uint64_t *)buf, iters, 0xD2511F53u);
            if (w == 3) hipLaunchKernelGGL(k_bitop3, dim3(blocks), dim3(threads), 0, 0, (uint32_t *)buf, iters, 0x9E3779B9u);
            if (w == 4) hipLaunchKernelGGL(k_trans32<0>, dim3(blocks), dim3(threads), 0, 0, (float *)buf, iters);
            if (w == 5) hipLaunchKernelGGL(k_trans32<1>, dim3(blocks), dim3(threads), 0, 0, (float *)buf, iters);
            if (w == 6) hipLaunchKernelGGL(k_trans32<2>, dim3(blocks), dim3(threads), 0, 0, (float *)buf, iters);
            if (w == 7) hipLaunchKernelGGL(k_trans32<3>, dim3(blocks), dim3(threads), 0, 0, (float *)buf, iters);
            if (w == 8) hipLaunchKernelGGL(k_trans64<0>, dim3(blocks), dim3(threads), 0, 0, (double *)buf, iters);
            if (w == 9) hipLaunchKernelGGL(k_trans64<1>, dim3(blocks), dim3(threads), 0, 0, (double *)buf, iters);
            if (!ok(hipGetLastError(), "launch") || !ok(hipEventRecord(e1, 0), "hipEventRecord") ||
                !ok(hipEventSynchronize(e1), "kernel"))
                return 1;
            float ms = 0.0f;
            if (!ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) return 1;
            const double rate = lane_instr / (ms * 1e-3);
            const double clocks = 256.0 * 4 * 2.4e9 / (rate / 64.0);
            if (rep == 1) std::printf("%-12s %10.3f %22.2f %30.2f\n", names[w], ms, rate / 1e12, clocks);
        }
    }
    ok(hipFree(buf), "hipFree");
    return 0;
}
