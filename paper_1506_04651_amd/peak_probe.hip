/*
 * peak_probe.hip -- measured vector FMA throughput of the device, the
 * denominators of the roofline fractions: eight independent FMA chains per
 * lane, FP64 and FP32 (built without packed-FP32 instruction selection, as
 * the library is), best of five launches.  Prints one line per case.
 */
#include <hip/hip_runtime.h>

#include <cstdio>

__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__global__ void __launch_bounds__(256) k_fma(T* out, int iters, T b, T c) {
    T a0 = threadIdx.x * T(1e-3), a1 = a0 + T(1), a2 = a0 + T(2), a3 = a0 + T(3);
    T a4 = a0 + T(4), a5 = a0 + T(5), a6 = a0 + T(6), a7 = a0 + T(7);
    for (int i = 0; i < iters; ++i) {
        a0 = fma_t(a0, b, c); a1 = fma_t(a1, b, c); a2 = fma_t(a2, b, c); a3 = fma_t(a3, b, c);
        a4 = fma_t(a4, b, c); a5 = fma_t(a5, b, c); a6 = fma_t(a6, b, c); a7 = fma_t(a7, b, c);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            return -1.0;                                                           \
        }                                                                          \
    } while (0)

template <typename T>
static double tflops(int blocks, int iters) {
    T* d = nullptr;
    CHECK(hipMalloc((void**)&d, sizeof(T) * (size_t)blocks * 256));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    float best = 1e30f;
    for (int r = 0; r < 6; ++r) {
        CHECK(hipEventRecord(e0, nullptr));
        hipLaunchKernelGGL(k_fma<T>, dim3(blocks), dim3(256), 0, nullptr, d, iters, T(0.999999),
                           T(1e-7));
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, nullptr));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0 && ms < best) best = ms;
    }
    CHECK(hipFree(d));
    return 2.0 * 8.0 * iters * (double)blocks * 256 / (best * 1e-3) / 1e12;
}

int main() {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 2;
    printf("{\"cus\": %d, \"clock_khz\": %d", p.multiProcessorCount, p.clockRate);
    for (int blocks : {4096, 16384, 65536}) {
        printf(", \"fp64_fma_tflops_%d\": %.2f", blocks, tflops<double>(blocks, 4096));
        printf(", \"fp32_fma_tflops_%d\": %.2f", blocks, tflops<float>(blocks, 4096));
    }
    printf("}\n");
    return 0;
}
