// Back-substitution R c = (Q^T b)[0:M] (Sec. Theory: c = R^-1 Q^T b, solved as
// a series of back substitutions) and small vector utilities.
#include "kernels.h"

namespace gap {

constexpr int TB = 64;

// Back-substitution R x = rhs for the n x n upper triangle of R (column-major,
// ld), blocks of 64 from the bottom: one wave solves a diagonal block, then a
// GEMV removes the block's contribution from the rows above.  rhs is used as
// work.  R may be stored in FP32 (TR = float); the arithmetic is FP64.  When
// skip is non-null and *skip != 0 the kernels return at once.

// Solve the bw x bw diagonal block at (b0, b0) with one wave.
template <class TR>
__global__ __launch_bounds__(64) void trsv_diag_kernel(const TR *R, int64_t ld, int64_t b0, int bw, double *rhs,
                                                       double *x, const int32_t *skip)
{
    __shared__ double S[TB][TB + 1];
    __shared__ double xs[TB];
    if (skip && *skip)
        return;
    const int l = threadIdx.x;
    for (int cc = 0; cc < bw; ++cc)
        if (l < bw)
            S[l][cc] = (double)R[(b0 + cc) * ld + b0 + l];
    double r = (l < bw) ? rhs[b0 + l] : 0.0;
    __syncthreads();
    for (int i = bw - 1; i >= 0; --i) {
        if (l == i)
            xs[i] = r / S[i][i];
        __syncthreads();
        if (l < i)
            r -= S[l][i] * xs[i];
    }
    if (l < bw)
        x[b0 + l] = xs[l];
}

// rhs[r] -= sum_i R[r][b0+i] x[b0+i] for r < b0.
template <class TR>
__global__ __launch_bounds__(256) void trsv_gemv_kernel(const TR *R, int64_t ld, int64_t b0, int bw, double *rhs,
                                                        const double *x, const int32_t *skip)
{
    __shared__ double xs[TB];
    if (skip && *skip)
        return;
    if (threadIdx.x < bw)
        xs[threadIdx.x] = x[b0 + threadIdx.x];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= b0)
        return;
    double s = 0.0;
    for (int i = 0; i < bw; ++i)
        s += (double)R[(b0 + i) * ld + r] * xs[i];
    rhs[r] -= s;
}

// Forward substitution R^T x = rhs (R upper, so R^T is lower), blocks from the
// top: one wave per diagonal block, then rhs[i] -= sum_j R[j][i] x[j] for the
// rows below (column i of R holds the R[j][i], contiguous in j).
template <class TR>
__global__ __launch_bounds__(64) void trsv_t_diag_kernel(const TR *R, int64_t ld, int64_t b0, int bw, double *rhs,
                                                         double *x, const int32_t *skip)
{
    __shared__ double S[TB][TB + 1];
    __shared__ double xs[TB];
    if (skip && *skip)
        return;
    const int l = threadIdx.x;
    for (int cc = 0; cc < bw; ++cc)
        if (l < bw)
            S[l][cc] = (double)R[(b0 + cc) * ld + b0 + l];  // S[j][i] = R[b0+j][b0+i]
    double r = (l < bw) ? rhs[b0 + l] : 0.0;
    __syncthreads();
    for (int i = 0; i < bw; ++i) {
        if (l == i)
            xs[i] = r / S[i][i];
        __syncthreads();
        if (l > i && l < bw)
            r -= S[i][l] * xs[i];
    }
    if (l < bw)
        x[b0 + l] = xs[l];
}

template <class TR>
__global__ __launch_bounds__(256) void trsv_t_gemv_kernel(const TR *R, int64_t ld, int64_t n, int64_t b0, int bw,
                                                          double *rhs, const double *x, const int32_t *skip)
{
    __shared__ double xs[TB];
    if (skip && *skip)
        return;
    if (threadIdx.x < bw)
        xs[threadIdx.x] = x[b0 + threadIdx.x];
    __syncthreads();
    const int64_t i = b0 + bw + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const TR *col = R + i * ld + b0;
    double s = 0.0;
    for (int j = 0; j < bw; ++j)
        s += (double)col[j] * xs[j];
    rhs[i] -= s;
}

template <class TR>
static hipError_t trsv_upper(const TR *R, int64_t ld, int64_t n, double *rhs, double *x, const int32_t *skip,
                             hipStream_t s)
{
    const int64_t nb = (n + TB - 1) / TB;
    for (int64_t b = nb - 1; b >= 0; --b) {
        const int64_t b0 = b * TB;
        const int bw = (int)((n - b0) < TB ? (n - b0) : TB);
        hipLaunchKernelGGL(trsv_diag_kernel<TR>, dim3(1), dim3(64), 0, s, R, ld, b0, bw, rhs, x, skip);
        if (b0 > 0)
            hipLaunchKernelGGL(trsv_gemv_kernel<TR>, dim3((unsigned)((b0 + 255) / 256)), dim3(256), 0, s, R, ld,
                               b0, bw, rhs, (const double *)x, skip);
    }
    return hipGetLastError();
}

template <class TR>
static hipError_t trsv_upper_t(const TR *R, int64_t ld, int64_t n, double *rhs, double *x, const int32_t *skip,
                               hipStream_t s)
{
    const int64_t nb = (n + TB - 1) / TB;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t b0 = b * TB;
        const int bw = (int)((n - b0) < TB ? (n - b0) : TB);
        hipLaunchKernelGGL(trsv_t_diag_kernel<TR>, dim3(1), dim3(64), 0, s, R, ld, b0, bw, rhs, x, skip);
        const int64_t rest = n - b0 - bw;
        if (rest > 0)
            hipLaunchKernelGGL(trsv_t_gemv_kernel<TR>, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, R, ld,
                               n, b0, bw, rhs, (const double *)x, skip);
    }
    return hipGetLastError();
}

hipError_t launch_trsv_upper(const double *R, int64_t ld, int64_t n, double *rhs, double *c, int32_t *status,
                             hipStream_t s)
{
    hipError_t e = trsv_upper<double>(R, ld, n, rhs, c, nullptr, s);
    if (e != hipSuccess)
        return e;
    return launch_check_finite(c, n, status, s);
}

hipError_t launch_trsv_upper_f32(const float *R, int64_t ld, int64_t n, double *rhs, double *x, const int32_t *skip,
                                 hipStream_t s)
{
    return trsv_upper<float>(R, ld, n, rhs, x, skip, s);
}

hipError_t launch_trsv_upper_t_f32(const float *R, int64_t ld, int64_t n, double *rhs, double *x,
                                   const int32_t *skip, hipStream_t s)
{
    return trsv_upper_t<float>(R, ld, n, rhs, x, skip, s);
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

__global__ void copy_f32_f64_kernel(const float *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        dst[i] = (double)src[i];
}

hipError_t launch_copy_f32_f64(const float *src, double *dst, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(copy_f32_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
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
