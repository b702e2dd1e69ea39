// Mixed precision: iterative refinement of the least-squares solution in FP64
// against the FP64 stacked matrix, using the FP32 Householder factor R as the
// preconditioner (corrected semi-normal equations, Bjorck 1987):
//   r = b - A c,  s = A^T r,  solve R^T R dc = s,  c += dc.
// A and b are the FP64 [A | b] kept from the build; R is the upper triangle of
// the FP32 factorisation.  Iterations stop on the device once
// ||dc|| <= tol ||c|| (or once ||dc|| stops halving at a level <= 1e-9 ||c||,
// the FP64 rounding floor of the residual): later iterations' kernels see the
// flag and return at once, so the loop needs no host synchronisation.
#include "kernels.h"

namespace gap {

constexpr int RB = 256;   // rows per workgroup in the residual
constexpr int RCH = 8;    // column chunks of the residual product
constexpr double STALL_OK = 1e-9;  // a stalled correction this small counts as converged

__global__ void convert_f64_f32_kernel(const double *__restrict__ a, float *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        b[i] = (float)a[i];
}

hipError_t launch_convert_f64_f32(const double *a, float *b, int64_t n, hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(convert_f64_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

// Column-chunk partials of A c for rows [blockIdx.x*256, +256).
__global__ __launch_bounds__(256) void resid_part_kernel(RefineWork w)
{
    if (*w.done)
        return;
    const int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x;
    const int64_t ch = blockIdx.y;
    const int64_t per = (w.n + RCH - 1) / RCH;
    const int64_t j0 = ch * per;
    const int64_t j1 = (j0 + per) < w.n ? (j0 + per) : w.n;
    double acc0 = 0.0, acc1 = 0.0;
    if (r < w.m) {
        int64_t j = j0;
        for (; j + 1 < j1; j += 2) {
            acc0 += w.A[j * w.lda + r] * w.c[j];
            acc1 += w.A[(j + 1) * w.lda + r] * w.c[j + 1];
        }
        if (j < j1)
            acc0 += w.A[j * w.lda + r] * w.c[j];
        w.part[ch * w.m + r] = acc0 + acc1;
    }
}

// r = b - sum of the partials (chunks in order); partial ||r||^2 per workgroup.
__global__ __launch_bounds__(256) void resid_sum_kernel(RefineWork w)
{
    __shared__ double red[4];
    if (*w.done)
        return;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (r < w.m) {
        double ac = 0.0;
        for (int ch = 0; ch < RCH; ++ch)
            ac += w.part[ch * w.m + r];
        v = w.A[w.n * w.lda + r] - ac;  // b is column n of [A | b]
        w.r[r] = v;
    }
    double sq = wave_sum(v * v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0)
        w.rnorm_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// s_j = sum_i A[i][j] r[i], one column per workgroup (fixed-order reduction).
__global__ __launch_bounds__(256) void atr_kernel(RefineWork w)
{
    __shared__ double red[4];
    if (*w.done)
        return;
    const int64_t j = blockIdx.x;
    const double *col = w.A + j * w.lda;
    double a0 = 0.0, a1 = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 256 < w.m; i += 512) {
        a0 += col[i] * w.r[i];
        a1 += col[i + 256] * w.r[i + 256];
    }
    if (i < w.m)
        a0 += col[i] * w.r[i];
    const double v = wave_sum(a0 + a1);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        w.s[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// c += dc; convergence test on ||dc|| / ||c|| (one workgroup).
__global__ __launch_bounds__(256) void refine_update_kernel(RefineWork w, int64_t nparts)
{
    __shared__ double red[2][4];
    if (*w.done)
        return;
    double dd = 0.0, cc = 0.0;
    for (int64_t j = threadIdx.x; j < w.n; j += 256) {
        const double d = w.dc[j];
        const double c = w.c[j] + d;
        w.c[j] = c;
        dd += d * d;
        cc += c * c;
    }
    dd = wave_sum(dd);
    cc = wave_sum(cc);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = dd;
        red[1][threadIdx.x >> 6] = cc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double d2 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double c2 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        double rn = 0.0;
        for (int64_t b = 0; b < nparts; ++b)
            rn += w.rnorm_part[b];
        const double ratio = (c2 > 0.0) ? sqrt(d2 / c2) : 0.0;
        const double prev = w.stats[1];
        w.stats[0] = rn;                       // ||r||^2 before this correction
        w.stats[1] = ratio;
        w.iters[0] += 1;
        // converged: the correction is below tol; or it has reached the FP64
        // rounding floor (stopped halving) at a level already below STALL_OK
        const bool small = d2 <= w.tol * w.tol * c2;
        const bool stalled = w.iters[0] > 1 && ratio > 0.5 * prev && ratio <= STALL_OK;
        if (small || stalled)
            *w.done = 1;
    }
}

// ||r||^2 at the final c (after the loop): sum of the residual kernel's partials.
__global__ void refine_final_kernel(RefineWork w, int64_t nparts)
{
    if (threadIdx.x != 0)
        return;
    double rn = 0.0;
    for (int64_t b = 0; b < nparts; ++b)
        rn += w.rnorm_part[b];
    w.stats[0] = rn;
}

// After the loop: remember whether it converged (status ENOCONV otherwise) and
// re-arm the residual kernels for the final residual.
__global__ void refine_reset_done_kernel(RefineWork w)
{
    if (threadIdx.x == 0) {
        if (!*w.done)
            set_status(w.status, DST_ENOCONV);
        *w.done = 0;
    }
}

__global__ void refine_reset_kernel(RefineWork w)
{
    if (threadIdx.x == 0) {
        *w.done = 0;
        w.iters[0] = 0;
        w.stats[0] = 0.0;
        w.stats[1] = 0.0;
    }
}

static void residual(const RefineWork &w, hipStream_t s)
{
    const unsigned gr = (unsigned)((w.m + RB - 1) / RB);
    hipLaunchKernelGGL(resid_part_kernel, dim3(gr, RCH), dim3(256), 0, s, w);
    hipLaunchKernelGGL(resid_sum_kernel, dim3((unsigned)((w.m + 255) / 256)), dim3(256), 0, s, w);
}

hipError_t launch_refine(const RefineWork &w, int max_iters, hipStream_t s)
{
    hipLaunchKernelGGL(refine_reset_kernel, dim3(1), dim3(64), 0, s, w);
    const int64_t nparts = (w.m + 255) / 256;
    for (int it = 0; it < max_iters; ++it) {
        residual(w, s);
        hipLaunchKernelGGL(atr_kernel, dim3((unsigned)w.n), dim3(256), 0, s, w);
        // dc = R^-1 R^-T s (R from the FP32 factorisation, FP64 arithmetic)
        hipError_t e = launch_trsv_upper_t_f32(w.R32, w.lda, w.n, w.s, w.z, w.sync, w.done, s);
        if (e != hipSuccess)
            return e;
        e = launch_trsv_upper_f32(w.R32, w.lda, w.n, w.z, w.dc, w.sync, w.done, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(refine_update_kernel, dim3(1), dim3(256), 0, s, w, nparts);
    }
    // final residual at the returned c
    hipLaunchKernelGGL(refine_reset_done_kernel, dim3(1), dim3(64), 0, s, w);
    residual(w, s);
    hipLaunchKernelGGL(refine_final_kernel, dim3(1), dim3(64), 0, s, w, nparts);
    return hipGetLastError();
}

}  // namespace gap
