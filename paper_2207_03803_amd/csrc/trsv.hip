// Back-substitution R c = (Q^T b)[0:M] (Sec. Theory: c = R^-1 Q^T b, solved as
// a series of back substitutions) and small vector utilities.
#include "kernels.h"

namespace gap {

constexpr int TB = 64;          // rows per block row
constexpr int TS_GRID = 256;    // workgroups of one solve (all co-resident)
// A workgroup waiting for a block row gives up after this many 100 MHz ticks
// (10 s) and reports DST_EDEVICE, so that every wave always exits.
constexpr uint64_t TS_WAIT_TICKS = 1000000000ull;

// Triangular solves with the n x n upper triangle of R (column-major, ld):
// R x = rhs (back substitution, Sec. Theory: c = R^-1 Q^T b) and R^T x = rhs
// (forward substitution, used by the refinement).  R may be stored in FP32
// (TR = float); the arithmetic is FP64.
//
// One launch solves the whole system.  The block rows (64 rows each) are
// numbered in dependency order q = 0 .. nb-1 (the last block row first for
// R x = rhs, the first one first for R^T x = rhs).  A workgroup takes its next
// item from an atomic ticket when it starts it, so items are handed out in
// order to workgroups that are already running: every item a workgroup waits
// on (a smaller q) belongs to a running workgroup, whatever the dispatch order
// of the launch or the other work on the GPU, and the lowest unfinished q can
// always proceed.  A block row first accumulates the products with the blocks
// of every earlier block row, in order, waiting for each one's ready flag (its
// R values are loaded before the wait), then one wave solves the diagonal
// block and publishes x with a release and the flag.  The last workgroup to
// finish clears the flags and the ticket for the next solve (they must be zero
// before the first one).  When skip is non-null and *skip != 0 the kernel
// returns at once.

struct TrsvArgs {
    int64_t ld, n, nb;
    const double *rhs;
    double *x;
    int32_t *flags;     // [nb + 2]: ready flag per block row; [nb] = abort; [nb + 1] = ticket
    unsigned *counter;  // arrival counter (zero between solves)
    const int32_t *skip;
    int32_t *status;
};

DEV double load_x(const double *p)
{
    // bypass the non-coherent caches: x is written by other workgroups in this launch
    unsigned long long v =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}

// Make the dependency items [from, q) usable: thread 0 waits until item `from`
// is published, extends over every later item already published, and takes
// one agent-scope acquire for all of them.  Returns the new end of the ready
// range (uniform), or -1 when the wait was abandoned.
template <bool TRANS>
DEV int64_t acquire_ready(const TrsvArgs &a, int64_t from, int64_t q, int64_t *lds)
{
    if (threadIdx.x == 0) {
        auto row = [&](int64_t qq) { return TRANS ? qq : a.nb - 1 - qq; };
        int64_t upto = from;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(&a.flags[row(from)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (__hip_atomic_load(&a.flags[a.nb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                upto = -1;
                break;
            }
            if (__builtin_amdgcn_s_memrealtime() - t0 > TS_WAIT_TICKS) {
                set_status(a.status, DST_EDEVICE);
                __hip_atomic_store(&a.flags[a.nb], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                upto = -1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (upto >= 0) {
            upto = from + 1;
            while (upto < q && __hip_atomic_load(&a.flags[row(upto)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                ++upto;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        *lds = upto;
    }
    __syncthreads();
    return *lds;
}

template <class TR, bool TRANS>
__global__ __launch_bounds__(256) void trsv_fused_kernel(const TR *__restrict__ R, TrsvArgs a)
{
    __shared__ double D[TB][TB + 1];  // diagonal block: D[c][l] = R[b0+l][b0+c]
    __shared__ double red[4][TB];
    __shared__ double xs[TB];
    __shared__ int64_t ready_lds;
    __shared__ int last_lds;
    __shared__ int32_t ticket_lds;
    if (a.skip && *a.skip)
        return;
    const int t = threadIdx.x, lane = t & 63, grp = t >> 6;
    const int64_t ld = a.ld, n = a.n, nb = a.nb;
    bool alive = true;
    auto take = [&]() -> int64_t {
        __syncthreads();  // every thread is done with the previous item's shared state
        if (t == 0)
            ticket_lds = __hip_atomic_fetch_add(&a.flags[nb + 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        return ticket_lds;
    };
    for (int64_t q = take(); q < nb && alive; q = take()) {
        const int64_t i = TRANS ? q : nb - 1 - q;
        const int64_t b0 = i * TB;
        const int bw = (int)((n - b0) < TB ? (n - b0) : TB);
        // stage the diagonal block (independent of x): D[c][l] = R[b0+l][b0+c]
        {
            double dv[TB / 4];
#pragma unroll
            for (int e = 0; e < TB / 4; ++e) {
                const int c = grp + 4 * e;
                dv[e] = (c < bw && lane < bw) ? (double)R[(b0 + c) * ld + b0 + lane] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < TB / 4; ++e)
                D[grp + 4 * e][lane] = dv[e];
        }
        // products with the blocks of every earlier block row
        double acc[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            acc[e] = 0.0;
        int64_t ready = 0;  // dependency items [0, ready) are published and acquired
        for (int64_t qq = 0; qq < q && alive; ++qq) {
            const int64_t j = TRANS ? qq : nb - 1 - qq;
            const int64_t j0 = j * TB;
            const int jw = (int)((n - j0) < TB ? (n - j0) : TB);
            double rv[16];
            if (!TRANS) {
                // thread (row lane, columns grp + 4e): R[b0+lane][j0+c], coalesced over lanes
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int c = grp + 4 * e;
                    rv[e] = (c < jw && lane < bw) ? (double)R[(j0 + c) * ld + b0 + lane] : 0.0;
                }
            } else {
                // thread (x index lane, rows grp + 4e of the block row): R[j0+lane][b0+k]
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int k = grp + 4 * e;
                    rv[e] = (k < bw && lane < jw) ? (double)R[(b0 + k) * ld + j0 + lane] : 0.0;
                }
            }
            if (qq >= ready) {
                ready = acquire_ready<TRANS>(a, qq, q, &ready_lds);
                if (ready < 0) {
                    alive = false;
                    break;
                }
            }
            if (t < TB)
                xs[t] = (t < jw) ? load_x(a.x + j0 + t) : 0.0;
            __syncthreads();
            if (!TRANS) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    acc[0] += rv[e] * xs[grp + 4 * e];
            } else {
                const double xv = xs[lane];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    acc[e] += rv[e] * xv;
            }
            __syncthreads();
        }
        if (!alive)
            break;
        // r = rhs - (sum of the products), fixed reduction order
        if (!TRANS) {
            red[grp][lane] = acc[0];
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const double v = wave_sum(acc[e]);
                if (lane == 0)
                    red[0][grp + 4 * e] = v;
            }
        }
        __syncthreads();
        if (t < TB) {
            double r = 0.0, inv = 0.0;
            if (lane < bw) {
                const double sub = TRANS ? red[0][lane] : (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
                r = a.rhs[b0 + lane] - sub;
                inv = 1.0 / D[lane][lane];
            }
            double xl = 0.0;
            if (!TRANS) {
                for (int c = bw - 1; c >= 0; --c) {
                    const double xc = __shfl(r, c, 64) * __shfl(inv, c, 64);
                    if (lane == c)
                        xl = xc;
                    else if (lane < c)
                        r -= D[c][lane] * xc;
                }
            } else {
                for (int c = 0; c < bw; ++c) {
                    const double xc = __shfl(r, c, 64) * __shfl(inv, c, 64);
                    if (lane == c)
                        xl = xc;
                    else if (lane > c)
                        r -= D[lane][c] * xc;
                }
            }
            if (lane < bw)
                a.x[b0 + lane] = xl;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(&a.flags[i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
    // the last workgroup to finish clears the flags for the next solve
    if (!arrive_last(a.counter, gridDim.x, &last_lds))
        return;
    for (int64_t k = t; k <= nb + 1; k += 256)
        a.flags[k] = 0;
}

template <class TR, bool TRANS>
static hipError_t trsv_fused(const TR *R, int64_t ld, int64_t n, const double *rhs, double *x, const TrsvSync &sync,
                             const int32_t *skip, hipStream_t s)
{
    TrsvArgs a{};
    a.ld = ld;
    a.n = n;
    a.nb = (n + TB - 1) / TB;
    a.rhs = rhs;
    a.x = x;
    a.flags = sync.flags;
    a.counter = sync.counter;
    a.skip = skip;
    a.status = sync.status;
    const unsigned g = (unsigned)(a.nb < TS_GRID ? a.nb : TS_GRID);
    hipLaunchKernelGGL((trsv_fused_kernel<TR, TRANS>), dim3(g), dim3(256), 0, s, R, a);
    return hipGetLastError();
}

int64_t trsv_sync_ints(int64_t n) { return (n + TB - 1) / TB + 1 + 64; }

hipError_t launch_trsv_upper(const double *R, int64_t ld, int64_t n, const double *rhs, double *c,
                             const TrsvSync &sync, hipStream_t s)
{
    hipError_t e = trsv_fused<double, false>(R, ld, n, rhs, c, sync, nullptr, s);
    if (e != hipSuccess)
        return e;
    return launch_check_finite(c, n, sync.status, s);
}

hipError_t launch_trsv_upper_nc(const double *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                const TrsvSync &sync, hipStream_t s)
{
    return trsv_fused<double, false>(R, ld, n, rhs, x, sync, nullptr, s);
}

hipError_t launch_trsv_upper_t(const double *R, int64_t ld, int64_t n, const double *rhs, double *x,
                               const TrsvSync &sync, hipStream_t s)
{
    return trsv_fused<double, true>(R, ld, n, rhs, x, sync, nullptr, s);
}

hipError_t launch_trsv_upper_f32(const float *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                 const TrsvSync &sync, const int32_t *skip, hipStream_t s)
{
    return trsv_fused<float, false>(R, ld, n, rhs, x, sync, skip, s);
}

hipError_t launch_trsv_upper_t_f32(const float *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                   const TrsvSync &sync, const int32_t *skip, hipStream_t s)
{
    return trsv_fused<float, true>(R, ld, n, rhs, x, sync, skip, s);
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
