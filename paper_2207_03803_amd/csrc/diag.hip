// Diagnostics of a solved fit: the normal-equation residual of the returned
// weights and, on request, an estimate of their relative error from the
// condition number of the stacked matrix (kappa_2(A) = kappa_2(R)).
//
//   eta = ||A^T (b - A c)|| / (||A||_F (||A||_F ||c|| + ||b||))
//
// is the zero gradient of the loss (Sec. Theory, Eq. GP_sparse: A^T A c = A^T b)
// measured relative to the sizes involved.  Mixed precision forms A^T r with
// the FP64 A kept for the refinement.  FP64 factors A in place, so it forms
// A^T r in the factored basis, A^T r = R^T ((Q^T b)[0:M] - R c), which
// measures the back-substitution (the Householder QR's own backward error,
// about u, is not part of it).  ||A||_F = ||R||_F in both cases (Q has
// orthonormal columns; in mixed precision R is the FP32 factor's).
//
// The error estimate is u (kappa + kappa^2 ||r|| / (||A||_2 ||c||)), the
// first-order sensitivity of a least-squares solution to perturbations of
// relative size u in A and b, with sigma_max(R) from power iteration on
// R^T R and sigma_min(R) from inverse iteration (a fixed number of steps of
// each; both converge from inside, so kappa is an underestimate until they
// have converged).
#include "kernels.h"

namespace gap {

constexpr int DCH = 8;  // column chunks of the R c product

DEV double dblock_sum(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// part[j] = sum_{i <= j} R(i, j)^2, one workgroup per column.
template <class TR>
__global__ __launch_bounds__(256) void sumsq_upper_kernel(const TR *__restrict__ R, int64_t ld, int64_t n,
                                                          double *part)
{
    __shared__ double red[4];
    const int64_t j = blockIdx.x;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i <= j; i += 256) {
        const double v = (double)R[j * ld + i];
        a += v * v;
    }
    const double s = dblock_sum(a, red);
    if (threadIdx.x == 0)
        part[j] = s;
}

// Column-chunk partials of R x for the upper triangle: part[ch * n + i] =
// sum_{j in chunk ch, j >= i} R(i, j) x(j).
template <class TR>
__global__ __launch_bounds__(256) void rx_part_kernel(const TR *__restrict__ R, int64_t ld, int64_t n,
                                                      const double *__restrict__ x, double *part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ch = blockIdx.y;
    const int64_t per = (n + DCH - 1) / DCH;
    int64_t j0 = ch * per;
    const int64_t j1 = (j0 + per) < n ? (j0 + per) : n;
    if (i >= n)
        return;
    if (j0 < i)
        j0 = i;
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j)
        acc += (double)R[j * ld + i] * x[j];
    part[ch * n + i] = acc;
}

// out(i) = base(i) - sum_ch part (base null: 0 - ...; negate = false gives +sum).
__global__ __launch_bounds__(256) void rx_sum_kernel(const double *part, int64_t n, const double *base, bool sub,
                                                     double *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double s = 0.0;
    for (int ch = 0; ch < DCH; ++ch)
        s += part[ch * n + i];
    out[i] = sub ? base[i] - s : s;
}

// out(j) = sum_{i <= j} R(i, j) t(i), one workgroup per column.
template <class TR>
__global__ __launch_bounds__(256) void rtx_kernel(const TR *__restrict__ R, int64_t ld, int64_t n,
                                                  const double *__restrict__ t, double *out)
{
    __shared__ double red[4];
    const int64_t j = blockIdx.x;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i <= j; i += 256)
        a += (double)R[j * ld + i] * t[i];
    const double s = dblock_sum(a, red);
    if (threadIdx.x == 0)
        out[j] = s;
}

// One workgroup: x = z / ||z||, q[slot] = ||y||^2 (the Rayleigh quotient of the
// previous unit x).  First call (init): x = 1 / sqrt(n).
__global__ __launch_bounds__(256) void power_normalise_kernel(const double *y, const double *z, double *x,
                                                              int64_t n, double *q, int init)
{
    __shared__ double red[4];
    if (init) {
        for (int64_t i = threadIdx.x; i < n; i += 256)
            x[i] = 1.0 / sqrt((double)n);
        return;
    }
    double ay = 0.0, az = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        ay += y[i] * y[i];
        az += z[i] * z[i];
    }
    const double sy = dblock_sum(ay, red);
    const double sz = dblock_sum(az, red);
    const double inv = sz > 0.0 ? 1.0 / sqrt(sz) : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256)
        x[i] = z[i] * inv;
    if (threadIdx.x == 0)
        *q = sy;
}

// One workgroup: eta and the error estimate from the pieces.
//   s [n] A^T r;  c [n];  partR [n] column sums of R^2;  sc[0] ||b||^2 (plus
//   *tail2 when non-null), sc[1] ||r||^2, sc[2] sigma_max^2 and sc[3]
//   1 / sigma_min^2 (0: no estimate).  out[0] eta, out[1] the error estimate
//   (-1 without one), out[2] kappa.
__global__ __launch_bounds__(256) void diag_final_kernel(const double *s, const double *c, const double *partR,
                                                         int64_t n, const double *sc, const double *tail2,
                                                         double *out)
{
    __shared__ double red[4];
    double as = 0.0, ac = 0.0, ar = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        as += s[i] * s[i];
        ac += c[i] * c[i];
        ar += partR[i];
    }
    const double s2 = dblock_sum(as, red);
    const double c2 = dblock_sum(ac, red);
    const double r2 = dblock_sum(ar, red);
    if (threadIdx.x != 0)
        return;
    const double b2 = sc[0] + (tail2 ? *tail2 : 0.0);
    const double nA = sqrt(r2), nc = sqrt(c2), nb = sqrt(b2);
    const double den = nA * (nA * nc + nb);
    out[0] = den > 0.0 ? sqrt(s2) / den : 0.0;
    out[1] = -1.0;
    if (sc[2] > 0.0 && sc[3] > 0.0 && nc > 0.0) {
        const double smax = sqrt(sc[2]), smin = 1.0 / sqrt(sc[3]);
        const double kappa = smax / smin;
        const double u = 1.1102230246251565e-16;  // 2^-53
        const double rn = sqrt(sc[1] > 0.0 ? sc[1] : 0.0);
        out[1] = u * (kappa + kappa * kappa * rn / (smax * nc));
        out[2] = kappa;
    }
}

__global__ void diag_scalars_kernel(double *sc, const double *r2)
{
    if (threadIdx.x == 0) {
        sc[0] = 0.0;
        sc[1] = r2 ? *r2 : 0.0;
        sc[2] = 0.0;
        sc[3] = 0.0;
    }
}

template <class TR>
static void rx(const TR *R, int64_t ld, int64_t n, const double *x, const double *base, bool sub, double *part,
               double *out, hipStream_t s)
{
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((rx_part_kernel<TR>), dim3(g, DCH), dim3(256), 0, s, R, ld, n, x, part);
    hipLaunchKernelGGL(rx_sum_kernel, dim3(g), dim3(256), 0, s, part, n, base, sub, out);
}

// sc[2] = sigma_max(R)^2 (power iteration), sc[3] = 1 / sigma_min(R)^2 (inverse iteration).
template <class TR>
static hipError_t estimate(const DiagWork &d, const TR *R, hipStream_t s)
{
    const int64_t n = d.n;
    double *x = d.x, *y = d.y, *z = d.z;
    hipLaunchKernelGGL(power_normalise_kernel, dim3(1), dim3(256), 0, s, y, z, x, n, d.sc + 2, 1);
    for (int it = 0; it < d.iters; ++it) {
        rx<TR>(R, d.ld, n, x, nullptr, false, d.part, y, s);
        hipLaunchKernelGGL((rtx_kernel<TR>), dim3((unsigned)n), dim3(256), 0, s, R, d.ld, n, y, z);
        hipLaunchKernelGGL(power_normalise_kernel, dim3(1), dim3(256), 0, s, y, z, x, n, d.sc + 2, 0);
    }
    hipLaunchKernelGGL(power_normalise_kernel, dim3(1), dim3(256), 0, s, y, z, x, n, d.sc + 3, 1);
    for (int it = 0; it < d.iters; ++it) {
        hipError_t e;
        if constexpr (sizeof(TR) == 8) {
            e = launch_trsv_upper_t(reinterpret_cast<const double *>(R), d.ld, n, x, y, d.sync, s);
            if (e == hipSuccess)
                e = launch_trsv_upper_nc(reinterpret_cast<const double *>(R), d.ld, n, y, z, d.sync, s);
        } else {
            e = launch_trsv_upper_t_f32(reinterpret_cast<const float *>(R), d.ld, n, x, y, d.sync, nullptr, s);
            if (e == hipSuccess)
                e = launch_trsv_upper_f32(reinterpret_cast<const float *>(R), d.ld, n, y, z, d.sync, nullptr, s);
        }
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(power_normalise_kernel, dim3(1), dim3(256), 0, s, y, z, x, n, d.sc + 3, 0);
    }
    return hipGetLastError();
}

hipError_t launch_diag_fp64(const DiagWork &d, const double *R, const double *qtb, const double *c, double *out,
                            hipStream_t s)
{
    const int64_t n = d.n;
    // ||r||^2 of the QR solution is the minimum loss ||(Q^T b)[n:]||^2 (*d.tail2)
    hipLaunchKernelGGL(diag_scalars_kernel, dim3(1), dim3(64), 0, s, d.sc, d.tail2);
    hipLaunchKernelGGL((sumsq_upper_kernel<double>), dim3((unsigned)n), dim3(256), 0, s, R, d.ld, n, d.partR);
    // t = (Q^T b)[0:n] - R c, then A^T r = R^T t
    rx<double>(R, d.ld, n, c, qtb, true, d.part, d.t, s);
    hipLaunchKernelGGL((rtx_kernel<double>), dim3((unsigned)n), dim3(256), 0, s, R, d.ld, n, d.t, d.g);
    // ||b||^2 = ||(Q^T b)[0:n]||^2 + ||(Q^T b)[n:]||^2
    hipError_t e = launch_sumsq(qtb, n, d.sc, d.sum_part, d.counter, s);
    if (e == hipSuccess && d.iters > 0)
        e = estimate<double>(d, R, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, d.g, c, d.partR, n, d.sc, d.tail2, out);
    return hipGetLastError();
}

hipError_t launch_diag_mixed(const DiagWork &d, const float *R32, const double *bcol, int64_t m, const double *r2,
                             const double *c, double *out, hipStream_t s)
{
    const int64_t n = d.n;
    // d.g holds A^T r at the returned c (the refinement's last pass); ||r||^2 = *r2
    hipLaunchKernelGGL(diag_scalars_kernel, dim3(1), dim3(64), 0, s, d.sc, r2);
    hipLaunchKernelGGL((sumsq_upper_kernel<float>), dim3((unsigned)n), dim3(256), 0, s, R32, d.ld, n, d.partR);
    hipError_t e = launch_sumsq(bcol, m, d.sc, d.sum_part, d.counter, s);
    if (e == hipSuccess && d.iters > 0)
        e = estimate<float>(d, R32, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, d.g, c, d.partR, n, d.sc, nullptr, out);
    return hipGetLastError();
}

}  // namespace gap
