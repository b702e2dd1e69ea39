// Mixed precision: iterative refinement of the least-squares solution in FP64
// against the FP64 stacked matrix [A | b] kept from the build, preconditioned
// by R, the upper triangle of the FP32 Householder factorisation (triangular
// solves with R take FP64 arithmetic).
//
// Stage 1, corrected semi-normal equations (Bjorck 1987):
//   r = b - A c,  s = A^T r,  solve R^T R dc = s,  c += dc.
// Each step scales the error by roughly u_32 kappa(A), which nears or passes 1
// once kappa(A) nears 1/u_32.  When a correction, from the second on, fails to
// halve and is not yet small, the loop keeps c (without that correction when it
// grew) and moves to stage 2.
//
// Stage 2, CGLS on the right-preconditioned problem min ||A R^-1 v - b||,
// c = R^-1 v, carried out in c's coordinates (preconditioned CGLS, Bjorck,
// Numerical Methods for Least Squares Problems, 1996):
//   start  r = b - A c,  z = R^-T A^T r,  p = R^-1 z,  gamma = ||z||^2
//   step   q = A p,  alpha = gamma / ||q||^2,  c += alpha p,  r -= alpha q,
//          z = R^-T A^T r,  gamma' = ||z||^2,  p = R^-1 z + (gamma' / gamma) p.
// Its rate is set by the spread of the singular values of A R^-1, so it needs
// no bound on u_32 kappa(A).
//
// Both stages run the same kernel sequence per iteration, steered by a mode
// word on the device.  Iterations stop on the device once the step is
// <= tol ||c|| (or once it stops halving at a level <= 1e-9 ||c||, the FP64
// rounding floor): later iterations' kernels see the flag and return at once,
// so the loop needs no host synchronisation.
#include "kernels.h"

namespace gap {

constexpr int RB = 256;   // rows per workgroup in the residual
constexpr int RCH = 8;    // column chunks of the residual product
constexpr double STALL_OK = 1e-9;  // a stalled correction this small counts as converged
constexpr int MODE_CSNE = 0, MODE_CG_START = 1, MODE_CG = 2;

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

// b[r, c] = a[r, c] for rows [r0, r1) of columns [c0, c1) (column-major, ld).
__global__ void convert_block_f64_f32_kernel(const double *__restrict__ a, float *__restrict__ b, int64_t ld,
                                             int64_t r0, int64_t r1, int64_t c0, int64_t c1)
{
    const int64_t nr = r1 - r0, total = nr * (c1 - c0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t c = c0 + i / nr, r = r0 + i % nr;
        b[c * ld + r] = (float)a[c * ld + r];
    }
}

hipError_t launch_convert_block_f64_f32(const double *a, float *b, int64_t ld, int64_t r0, int64_t r1, int64_t c0,
                                        int64_t c1, hipStream_t s)
{
    const int64_t total = (r1 - r0) * (c1 - c0);
    if (total <= 0)
        return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(convert_block_f64_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, a, b, ld, r0, r1, c0, c1);
    return hipGetLastError();
}

// Fixed-order sum of a 256-thread workgroup (identical in every workgroup for
// identical inputs).
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Column-chunk partials of A v for rows [blockIdx.x*256, +256); v is c, or p
// in the CGLS steps.
__global__ __launch_bounds__(256) void resid_part_kernel(RefineWork w)
{
    if (*w.done)
        return;
    const double *v = (*w.mode == MODE_CG) ? w.p : w.c;
    const int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x;
    const int64_t ch = blockIdx.y;
    const int64_t per = (w.n + RCH - 1) / RCH;
    const int64_t j0 = ch * per;
    const int64_t j1 = (j0 + per) < w.n ? (j0 + per) : w.n;
    double acc0 = 0.0, acc1 = 0.0;
    if (r < w.m) {
        int64_t j = j0;
        for (; j + 1 < j1; j += 2) {
            acc0 += w.A[j * w.lda + r] * v[j];
            acc1 += w.A[(j + 1) * w.lda + r] * v[j + 1];
        }
        if (j < j1)
            acc0 += w.A[j * w.lda + r] * v[j];
        w.part[ch * w.m + r] = acc0 + acc1;
    }
}

// Sum of the partials (chunks in order): r = b - A c, or q = A p in the CGLS
// steps; partial ||r||^2 (||q||^2) per workgroup.
__global__ __launch_bounds__(256) void resid_sum_kernel(RefineWork w)
{
    __shared__ double red[4];
    if (*w.done)
        return;
    const bool cg = *w.mode == MODE_CG;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (r < w.m) {
        double ac = 0.0;
        for (int ch = 0; ch < RCH; ++ch)
            ac += w.part[ch * w.m + r];
        if (cg) {
            v = ac;
            w.q[r] = v;
        } else {
            v = w.A[w.n * w.lda + r] - ac;  // b is column n of [A | b]
            w.r[r] = v;
        }
    }
    const double sq = block_sum(v * v, red);
    if (threadIdx.x == 0)
        w.rnorm_part[blockIdx.x] = sq;
}

// CGLS step, rows: alpha = gamma / ||q||^2 (every workgroup sums the same
// partials in the same order), r -= alpha q.
__global__ __launch_bounds__(256) void cg_step_kernel(RefineWork w, int64_t nparts)
{
    __shared__ double red[4];
    if (*w.done || *w.mode != MODE_CG)
        return;
    double a = 0.0;
    for (int64_t b = threadIdx.x; b < nparts; b += 256)
        a += w.rnorm_part[b];
    const double qq = block_sum(a, red);
    const double alpha = qq > 0.0 ? w.stats[3] / qq : 0.0;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < w.m)
        w.r[r] -= alpha * w.q[r];
    if (blockIdx.x == 0 && threadIdx.x == 0)
        w.stats[2] = alpha;
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
    const double v = block_sum(a0 + a1, red);
    if (threadIdx.x == 0)
        w.s[j] = v;
}

// End of an iteration (one workgroup).  After the triangular solves z holds
// R^-T A^T r and dc holds R^-1 z.
//   CSNE:       c += dc unless the switch to CGLS drops a grown correction;
//               convergence test on ||dc|| / ||c + dc||.
//   CGLS start: p = dc, gamma = ||z||^2.
//   CGLS step:  c += alpha p (alpha from cg_step_kernel), convergence test on
//               ||alpha p|| / ||c||, then p = dc + (||z||^2 / gamma) p.
__global__ __launch_bounds__(256) void refine_update_kernel(RefineWork w, int64_t nparts)
{
    __shared__ double red[3][4];
    __shared__ int act;
    __shared__ double beta;
    if (*w.done)
        return;
    const int mode = *w.mode;
    const double alpha = w.stats[2];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t j = threadIdx.x; j < w.n; j += 256) {
        if (mode == MODE_CSNE) {
            const double d = w.dc[j];
            const double c = w.c[j] + d;
            a0 += d * d;
            a1 += c * c;
        } else if (mode == MODE_CG_START) {
            const double z = w.z[j];
            a2 += z * z;
        } else {
            const double st = alpha * w.p[j];
            const double c = w.c[j] + st;
            w.c[j] = c;
            a0 += st * st;
            a1 += c * c;
            const double z = w.z[j];
            a2 += z * z;
        }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a0;
        red[1][threadIdx.x >> 6] = a1;
        red[2][threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double d2 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double c2 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const double g2 = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
        const double ratio = (c2 > 0.0) ? sqrt(d2 / c2) : 0.0;
        const double prev = w.stats[1];
        const bool small = d2 <= w.tol * w.tol * c2;
        w.iters[0] += 1;
        int a = 0;  // 0: nothing, 1: c += dc, 2: p = dc, 3: p = dc + beta p
        if (mode == MODE_CSNE) {
            double rn = 0.0;
            for (int64_t b = 0; b < nparts; ++b)
                rn += w.rnorm_part[b];
            w.stats[0] = rn;  // ||r||^2 before this correction
            const bool halving = ratio <= 0.5 * prev;
            // converged: the correction is below tol; or it has reached the FP64
            // rounding floor (stopped halving) at a level already below STALL_OK
            const bool stalled = w.iters[0] > 1 && !halving && ratio <= STALL_OK;
            const bool slow = w.iters[0] > 1 && !halving && !small && !stalled;
            a = (!slow || ratio < prev) ? 1 : 0;
            if (slow)
                *w.mode = MODE_CG_START;
            if (small || stalled)
                *w.done = 1;
            w.stats[1] = ratio;
        } else if (mode == MODE_CG_START) {
            w.stats[3] = g2;
            *w.mode = MODE_CG;
            a = 2;
        } else {
            w.iters[1] += 1;
            const bool stalled = w.iters[1] > 1 && !(ratio <= 0.5 * prev) && ratio <= STALL_OK;
            if (small || stalled)
                *w.done = 1;
            const double g = w.stats[3];
            beta = g > 0.0 ? g2 / g : 0.0;
            w.stats[3] = g2;
            w.stats[1] = ratio;
            a = 3;
        }
        act = a;
    }
    __syncthreads();
    const int a = act;
    if (a == 1) {
        for (int64_t j = threadIdx.x; j < w.n; j += 256)
            w.c[j] += w.dc[j];
    } else if (a == 2) {
        for (int64_t j = threadIdx.x; j < w.n; j += 256)
            w.p[j] = w.dc[j];
    } else if (a == 3) {
        const double b = beta;
        for (int64_t j = threadIdx.x; j < w.n; j += 256)
            w.p[j] = w.dc[j] + b * w.p[j];
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
// re-arm the residual kernels for the final residual r = b - A c.
__global__ void refine_reset_done_kernel(RefineWork w)
{
    if (threadIdx.x == 0) {
        if (!*w.done)
            set_status(w.status, DST_ENOCONV);
        *w.done = 0;
        *w.mode = MODE_CSNE;
    }
}

__global__ void refine_reset_kernel(RefineWork w)
{
    if (threadIdx.x == 0) {
        *w.done = 0;
        *w.mode = MODE_CSNE;
        w.iters[0] = 0;
        w.iters[1] = 0;
        for (int k = 0; k < 4; ++k)
            w.stats[k] = 0.0;
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
        hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)nparts), dim3(256), 0, s, w, nparts);
        hipLaunchKernelGGL(atr_kernel, dim3((unsigned)w.n), dim3(256), 0, s, w);
        // z = R^-T s, dc = R^-1 z (R from the FP32 factorisation, FP64 arithmetic)
        hipError_t e = launch_trsv_upper_t_f32(w.R32, w.lda, w.n, w.s, w.z, w.sync, w.done, s);
        if (e != hipSuccess)
            return e;
        e = launch_trsv_upper_f32(w.R32, w.lda, w.n, w.z, w.dc, w.sync, w.done, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(refine_update_kernel, dim3(1), dim3(256), 0, s, w, nparts);
    }
    // final residual r = b - A c at the returned c, ||r||^2, and s = A^T r
    hipLaunchKernelGGL(refine_reset_done_kernel, dim3(1), dim3(64), 0, s, w);
    residual(w, s);
    hipLaunchKernelGGL(refine_final_kernel, dim3(1), dim3(64), 0, s, w, nparts);
    hipLaunchKernelGGL(atr_kernel, dim3((unsigned)w.n), dim3(256), 0, s, w);
    return hipGetLastError();
}

}  // namespace gap
