// Back-substitution R c = (Q^T b)[0:M] (Sec. Theory: c = R^-1 Q^T b, solved as
// a series of back substitutions) and small vector utilities.
#include "kernels.h"

namespace gap {

constexpr int TB = 64;

// Solve the bw x bw diagonal block at (b0, b0) with one wave; rhs is updated
// in place, c[b0 .. b0+bw) written.
__global__ __launch_bounds__(64) void trsv_diag_kernel(const double *R, int64_t ld, int64_t b0, int bw,
                                                       double *rhs, double *c)
{
    __shared__ double S[TB][TB + 1];
    __shared__ double x[TB];
    const int l = threadIdx.x;
    for (int cc = 0; cc < bw; ++cc)
        if (l < bw)
            S[l][cc] = R[(b0 + cc) * ld + b0 + l];
    double r = (l < bw) ? rhs[b0 + l] : 0.0;
    __syncthreads();
    for (int i = bw - 1; i >= 0; --i) {
        if (l == i)
            x[i] = r / S[i][i];
        __syncthreads();
        if (l < i)
            r -= S[l][i] * x[i];
    }
    if (l < bw)
        c[b0 + l] = x[l];
}

// rhs[r] -= sum_i R[r][b0+i] c[b0+i] for r < b0.
__global__ __launch_bounds__(256) void trsv_gemv_kernel(const double *R, int64_t ld, int64_t b0, int bw,
                                                        double *rhs, const double *c)
{
    __shared__ double x[TB];
    if (threadIdx.x < bw)
        x[threadIdx.x] = c[b0 + threadIdx.x];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= b0)
        return;
    double s = 0.0;
    for (int i = 0; i < bw; ++i)
        s += R[(b0 + i) * ld + r] * x[i];
    rhs[r] -= s;
}

hipError_t launch_trsv_upper(const double *R, int64_t ld, int64_t n, double *rhs, double *c,
                             int32_t *status, hipStream_t s)
{
    const int64_t nb = (n + TB - 1) / TB;
    for (int64_t b = nb - 1; b >= 0; --b) {
        const int64_t b0 = b * TB;
        const int bw = (int)((n - b0) < TB ? (n - b0) : TB);
        hipLaunchKernelGGL(trsv_diag_kernel, dim3(1), dim3(64), 0, s, R, ld, b0, bw, rhs, c);
        if (b0 > 0)
            hipLaunchKernelGGL(trsv_gemv_kernel, dim3((unsigned)((b0 + 255) / 256)), dim3(256), 0, s, R,
                               ld, b0, bw, rhs, (const double *)c);
    }
    return launch_check_finite(c, n, status, s);
}

__global__ __launch_bounds__(256) void sumsq_kernel(const double *x, int64_t n, double *out, double *part,
                                                    unsigned *counter)
{
    __shared__ double red[4];
    __shared__ int flag;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v += x[i] * x[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    release_writes();
    if (!arrive_last(counter, gridDim.x, &flag))
        return;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b)
            s += part[b];
        *out = s;
    }
}

hipError_t launch_sumsq(const double *x, int64_t n, double *out, double *part, unsigned *counter,
                        hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 256)
        g = 256;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)g), dim3(256), 0, s, x, n, out, part, counter);
    return hipGetLastError();
}

__global__ void assemble_b_kernel(const double *y, const double *sigma, int64_t N, double *bcol,
                                  int64_t lda)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < N)
        bcol[r] = y[r] / sigma[r];
    else if (r < lda)
        bcol[r] = 0.0;
}

hipError_t launch_assemble_b(const double *y, const double *sigma, int64_t N, double *bcol,
                             int64_t lda, hipStream_t s)
{
    hipLaunchKernelGGL(assemble_b_kernel, dim3((unsigned)((lda + 255) / 256)), dim3(256), 0, s, y, sigma,
                       N, bcol, lda);
    return hipGetLastError();
}

__global__ void fill_kernel(double *p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void zero_block_kernel(double *A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int64_t c1)
{
    const int64_t rows = r1 - r0;
    const int64_t total = rows * (c1 - c0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t c = c0 + i / rows, r = r0 + i % rows;
        A[c * lda + r] = 0.0;
    }
}

hipError_t launch_zero_block(double *A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                             hipStream_t s)
{
    if (r1 <= r0 || c1 <= c0)
        return hipSuccess;
    int64_t g = ((r1 - r0) * (c1 - c0) + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(zero_block_kernel, dim3((unsigned)g), dim3(256), 0, s, A, lda, r0, r1, c0, c1);
    return hipGetLastError();
}

__global__ void check_finite_kernel(const double *x, int64_t n, int32_t *status)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        if (!isfinite(x[i])) {
            set_status(status, DST_ENONFINITE);
            return;
        }
}

hipError_t launch_check_finite(const double *x, int64_t n, int32_t *status, hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 1024)
        g = 1024;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)g), dim3(256), 0, s, x, n, status);
    return hipGetLastError();
}

}  // namespace gap
