// Microbenchmarks for the roofline denominators on this GPU: FP64 MFMA
// (16x16x4 and 4x4x4), INT8 MFMA (16x16x64), FP64 VALU FMA, and a
// device-to-device streaming copy.
// Every kernel keeps its results live and writes one value per thread.
#include <hip/hip_runtime.h>
#include <stdio.h>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

// Two workgroups per CU requested, so that the accumulators stay in VGPRs:
// with one, the compiler keeps them in VGPRs across the loop and copies them
// to and from AGPRs around every iteration's MFMAs, which halves the rate.
__global__ __launch_bounds__(256, 2) void mfma16_kernel(double *out, int iters, double a0)
{
    d4 acc[16];
    for (int i = 0; i < 16; ++i)
        acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const double a = a0 + threadIdx.x * 1e-3, b = a0 - threadIdx.x * 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
    for (int i = 0; i < 16; ++i)
        s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256, 2) void mfma4_kernel(double *out, int iters, double a0)
{
    double acc[16];
    for (int i = 0; i < 16; ++i)
        acc[i] = 0.0;
    const double a = a0 + threadIdx.x * 1e-3, b = a0 - threadIdx.x * 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
    for (int i = 0; i < 16; ++i)
        s += acc[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256, 2) void mfma_i8_kernel(int *out, int iters, int a0)
{
    v4i acc[16];
    for (int i = 0; i < 16; ++i)
        acc[i] = v4i{0, 0, 0, 0};
    const v4i a = v4i{a0 + (int)threadIdx.x, a0, a0 ^ 0x01010101, a0}, b = v4i{a0, a0 - (int)threadIdx.x, a0, a0 + 3};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[i], 0, 0, 0);
    }
    int s = 0;
    for (int i = 0; i < 16; ++i)
        s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void fma_kernel(double *out, int iters, double a0)
{
    double x[32];
    for (int i = 0; i < 32; ++i)
        x[i] = a0 + i;
    const double m = 1.0000001, c = 1e-9;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 32; ++i)
            x[i] = fma(x[i], m, c);
    }
    double s = 0.0;
    for (int i = 0; i < 32; ++i)
        s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        dst[i] = src[i];
}

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));        \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    double *out;
    CHECK(hipMalloc(&out, sizeof(double) * 256 * (size_t)cus * 8));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    float ms = 0.0f;
    printf("device: %s, %d CUs\n", prop.name, cus);
    for (int wps = 1; wps <= 2; ++wps) {
        const int blocks = cus * wps, iters = 2000;
        hipLaunchKernelGGL(mfma16_kernel, dim3(blocks), dim3(256), 0, 0, out, 10, 1.0);
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(mfma16_kernel, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        printf("v_mfma_f64_16x16x4_f64, %d wave(s)/SIMD: %.1f TFLOP/s\n", wps,
               (double)blocks * 4 * iters * 16 * 2048.0 / ms / 1e9);
        hipLaunchKernelGGL(mfma4_kernel, dim3(blocks), dim3(256), 0, 0, out, 10, 1.0);
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(mfma4_kernel, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        // four 4x4x4 products per instruction: 512 flops
        printf("v_mfma_f64_4x4x4_4b_f64, %d wave(s)/SIMD: %.1f TFLOP/s\n", wps,
               (double)blocks * 4 * iters * 16 * 512.0 / ms / 1e9);
    }
    for (int wps = 1; wps <= 2; ++wps) {
        const int blocks = cus * wps, iters = 2000;
        hipLaunchKernelGGL(mfma_i8_kernel, dim3(blocks), dim3(256), 0, 0, (int *)out, 10, 0x01020304);
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(mfma_i8_kernel, dim3(blocks), dim3(256), 0, 0, (int *)out, iters, 0x01020304);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        // 16 x 16 x 64 multiply-adds per instruction: 32768 operations
        printf("v_mfma_i32_16x16x64_i8, %d wave(s)/SIMD: %.1f TOP/s\n", wps,
               (double)blocks * 4 * iters * 16 * 32768.0 / ms / 1e9);
    }
    for (int wps = 1; wps <= 8; wps *= 2) {
        const int blocks = cus * wps, iters = 10000;
        hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(256), 0, 0, out, 10, 1.0);
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        printf("v_fma_f64 (VALU), %d wave(s)/SIMD: %.1f TFLOP/s\n", wps,
               (double)blocks * 256 * iters * 32 * 2.0 / ms / 1e9);
    }
    const size_t bytes = (size_t)4 << 30;  // 4 GiB each way
    double2 *src, *dst;
    CHECK(hipMalloc(&src, bytes));
    CHECK(hipMalloc(&dst, bytes));
    CHECK(hipMemset(src, 0, bytes));
    const size_t n = bytes / sizeof(double2);
    hipLaunchKernelGGL(copy_kernel, dim3(cus * 16), dim3(256), 0, 0, src, dst, n);
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r)
        hipLaunchKernelGGL(copy_kernel, dim3(cus * 16), dim3(256), 0, 0, src, dst, n);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    printf("streaming copy 4 GiB: %.2f TB/s (read + write)\n", 5.0 * 2.0 * bytes / (ms / 1e3) / 1e12);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));
    CHECK(hipFree(out));
    return 0;
}
