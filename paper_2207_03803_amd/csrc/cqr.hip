// Panel factorisation of the blocked Householder QR by shifted CholeskyQR3
// (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020), followed by the
// same Householder reconstruction as the TSQR panel (Ballard et al. 2015):
//
//   P = Q1 R1   from the Gram matrix P^T P + s I (shift s = 11 (mk pw + pw (pw+1)) u ||P||_F^2)
//   Q1 = Q2 R2, Q2 = Q R3  (two unshifted Cholesky QR passes)
//   R = S R3 R2 R1 with S and the unit lower Y1 from the LU of Q[0:pw] - S
//   Y (rows below the top block) = Q2 (U R3)^-1,  T = -U S Y1^-T,  tau = diag(T)
//
// so the panel leaves the LAPACK-form representation H = I - Y T Y^T, R above
// the diagonal, exactly as the TSQR panel does.  Every pass streams the panel
// (Gram products on FP64 MFMA, row-parallel triangular solves), so the panel
// costs a few reads of mk x 64 values instead of 64 dependent column steps.
// The intermediate Q's are kept in an FP64 scratch panel; the factored matrix
// may be stored in FP32 (arithmetic stays FP64).
#include "kernels.h"

namespace gap {

constexpr int CB = QR_NB;        // panel width bound (64)
constexpr int CQ_ROWS = 256;     // rows per workgroup of the row passes
using GS = TileShape<64, 64, 16, 2, 2>;

template <int N>
DEV void load_run_cvt(const double *__restrict__ p, double (&v)[N])
{
    load_run(p, v);
}

template <int N>
DEV void load_run_cvt(const float *__restrict__ p, double (&v)[N])
{
    static_assert(N % 4 == 0, "runs of a multiple of 4 floats");
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int e = 0; e < N / 4; ++e) {
        const float4 f = q[e];
        v[4 * e] = f.x;
        v[4 * e + 1] = f.y;
        v[4 * e + 2] = f.z;
        v[4 * e + 3] = f.w;
    }
}

// Partial Gram matrices: part[ch] = sum over rows [ch*chunk, +chunk) of
// P[r][:]^T P[r][:] for the pw columns of P (column-major, ld; 64 x 64 with
// zeros outside pw).
template <class T>
__global__ __launch_bounds__(256, 2) void cqr_gram_kernel(const T *__restrict__ P, int64_t ld, int64_t rows, int pw,
                                                          int64_t chunk, double *__restrict__ part)
{
    __shared__ double lds[2 * GS::STAGE];
    const int64_t ch = blockIdx.x;
    const int64_t lo = ch * chunk;
    const int64_t hi = (lo + chunk) < rows ? (lo + chunk) : rows;
    d4 acc[GS::FM][GS::FN];
    zero_acc<GS>(acc);
    constexpr int V = GS::BM * GS::BK / GS::NT;
    auto f = [&](int p, int64_t k, double (&v)[V]) {
        const int64_t r = lo + k;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                v[e] = 0.0;
        } else if (r + V <= hi) {
            load_run_cvt(P + p * ld + r, v);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e)
                v[e] = (r + e < hi) ? (double)P[p * ld + r + e] : 0.0;
        }
    };
    if (lo < hi)
        gemm_tile_runs<GS, true, true>(acc, lds, hi - lo, f, f);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / GS::WN, wn = wave % GS::WN;
    double *out = part + ch * (CB * CB);
#pragma unroll
    for (int i = 0; i < GS::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < GS::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                out[acc_row<GS>(wm, i, lane, e) * CB + acc_col<GS>(wn, jj, lane, e)] = acc[i][jj][e];
}

// Four partial sums of the chunk partials: G4[q][e] = sum over chunks
// c = q, q + 4, ... in order (grid 16 x 4; entries e of block x).
__global__ __launch_bounds__(256) void cqr_gsum_kernel(const double *__restrict__ part, int64_t nch,
                                                       double *__restrict__ G4)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    double s0 = 0.0, s1 = 0.0;
    int64_t c = q;
    for (; c + 4 < nch; c += 8) {
        s0 += part[c * (CB * CB) + e];
        s1 += part[(c + 4) * (CB * CB) + e];
    }
    if (c < nch)
        s0 += part[c * (CB * CB) + e];
    G4[q * (CB * CB) + e] = s0 + s1;
}

// Value of v in lane `lane` (uniform) of the wave.
DEV double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Order the wave's LDS accesses (the steps below run on one wave).
DEV void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Gram matrix into S by a 256-thread workgroup (all loads in flight at
// once): the sum of the four partial sums, identity beyond pw, and
// shift_coef * trace added to the diagonal.  Ends with a barrier.
DEV void gram_lds(const double *__restrict__ G4, int pw, double shift_coef, double (&S)[CB][CB + 1])
{
    const int t = threadIdx.x;
    double g[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u;
        g[u] = (G4[e] + G4[CB * CB + e]) + (G4[2 * CB * CB + e] + G4[3 * CB * CB + e]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u, i = e / CB, l = e % CB;
        S[i][l] = (i < pw && l < pw) ? g[u] : (i == l ? 1.0 : 0.0);
    }
    __syncthreads();
    if (t < 64) {
        const double d = (t < pw) ? S[t][t] : 0.0;
        const double tr = wave_sum(d);
        if (t < pw)
            S[t][t] = d + shift_coef * tr;
    }
    __syncthreads();
}

// Cholesky S = R^T R in place (one wave; lane l owns column l, S[i][l] for
// i <= l, in registers; row k of each step is shared through LDS): on exit S
// holds R (zeros below the diagonal).  A pivot that is not positive is
// replaced by 1 and reported through the return value.
DEV bool chol_lds(double (&S)[CB][CB + 1], double *rrow)
{
    const int l = threadIdx.x & 63;
    double x[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i)
        x[i] = S[i][l];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        if (l == k)
            rrow[k] = x[k];
        wave_sync();
        const double dkk = rrow[k];
        double rkk = sqrt(dkk);
        if (!(dkk > 0.0) || !(rkk < INFINITY)) {
            ok = false;
            rkk = 1.0;
        }
        const double rkj = (l > k) ? x[k] / rkk : (l == k ? rkk : 0.0);
        wave_sync();
        rrow[l] = rkj;
        wave_sync();
        x[k] = rkj;
        if (l > k) {
#pragma unroll
            for (int i = k + 1; i < CB; ++i)
                x[i] -= rrow[i] * rkj;  // rows past l are below the diagonal: zeroed below
        }
        wave_sync();
    }
#pragma unroll
    for (int i = 0; i < CB; ++i)
        S[i][l] = (i <= l) ? x[i] : 0.0;
    wave_sync();
    return ok;
}

// R_out = chol(G + shift I) (row-major 64 x 64, identity beyond pw); when
// Rprev is given, also Rprod = R_out Rprev (both upper triangular).  The
// factorisation runs on the first wave; loads and products on all four.
__global__ __launch_bounds__(256) void cqr_chol_kernel(const double *__restrict__ G4, int pw, double shift_coef,
                                                       double *__restrict__ Rout, const double *__restrict__ Rprev,
                                                       double *__restrict__ Rprod, int32_t *status)
{
    __shared__ double S[CB][CB + 1];
    __shared__ double Pv[CB][CB + 1];
    __shared__ double rrow[CB];
    const int t = threadIdx.x;
    double pv[16];
    if (Rprev) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            pv[u] = Rprev[t + 256 * u];
    }
    gram_lds(G4, pw, shift_coef, S);
    if (t < 64 && !chol_lds(S, rrow) && t == 0)
        set_status(status, DST_ERANK);
    if (Rprev) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            Pv[(t + 256 * u) / CB][(t + 256 * u) % CB] = pv[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u, i = e / CB, l = e % CB;
        Rout[e] = S[i][l];
        if (Rprev) {
            // entry (i, l) of R Rprev: sum over p in [i, l] of R[i][p] Rprev[p][l]
            double v = 0.0;
#pragma unroll 8
            for (int p = i; p <= l; ++p)
                v += S[i][p] * Pv[p][l];
            Rprod[e] = v;
        }
    }
}

// Row pass: dst[r][:] = src[r][:] R^-1 (R upper 64 x 64 row-major) for rows
// r0 .. rows-1, pw columns; one row per thread.
template <class TS, class TD>
__global__ __launch_bounds__(256) void cqr_pass_kernel(const TS *__restrict__ src, int64_t lds_, TD *__restrict__ dst,
                                                       int64_t ldd, int64_t r0, int64_t rows, int pw,
                                                       const double *__restrict__ R)
{
    __shared__ double Rs[CB][CB + 1];
    __shared__ double rinv[CB];
    {
        double rv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            rv[u] = R[threadIdx.x + 256 * u];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            Rs[(threadIdx.x + 256 * u) / CB][(threadIdx.x + 256 * u) % CB] = rv[u];
    }
    __syncthreads();
    if (threadIdx.x < CB)
        rinv[threadIdx.x] = 1.0 / Rs[threadIdx.x][threadIdx.x];
    __syncthreads();
    const int64_t r = r0 + (int64_t)blockIdx.x * CQ_ROWS + threadIdx.x;
    if (r >= rows)
        return;
    double y[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
        y[c] = (c < pw) ? (double)src[c * lds_ + r] : 0.0;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        if (c < pw) {
            double v = y[c];
#pragma unroll
            for (int i = 0; i < c; ++i)
                v -= y[i] * Rs[i][c];
            y[c] = v * rinv[c];
        }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (c < pw)
            dst[c * ldd + r] = (TD)y[c];
}

// The last Cholesky pass and the reconstruction of the top block (one
// workgroup): R3 = chol(G), Q_top = Q2[0:pw] R3^-1, LU of Q_top - S, the
// compact-WY T, R = S R3 R2 R1 and Y1 into the panel's top block, tau, and
// U R3 for the row pass that forms Y below the top block.  The sequential
// 64-step parts (Cholesky, triangular solve, LU) run on one wave; the
// products on all four.
template <class T>
__global__ __launch_bounds__(256) void cqr_top_kernel(QrWork w, int64_t j0, int pw, double *__restrict__ Tout)
{
    __shared__ double R3[CB][CB + 1];  // R3[i][l], upper
    __shared__ double B[CB][CB + 1];   // Q_top, then its LU (U on and above, multipliers below)
    __shared__ double X[CB][CB + 1];   // R2 R1, then Y1^-1
    __shared__ double sg[CB];
    __shared__ double tmp[CB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    {
        double xv[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u, r = e / CB, c = e % CB;
            xv[u] = w.cq_R[2 * CB * CB + e];  // R2 R1
            bv[u] = (r < pw && c < pw) ? w.cq_S[c * w.cq_ld + r] : 0.0;
        }
        gram_lds(w.cq_G, pw, 0.0, R3);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            X[e / CB][e % CB] = xv[u];
            B[e / CB][e % CB] = bv[u];
        }
    }
    if (wave == 0 && !chol_lds(R3, tmp) && lane == 0)
        set_status(w.status, DST_ERANK);
    __syncthreads();
    if (wave == 0) {
        // lane = row of Q_top, held in registers (columns past pw are zero)
        double q[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c)
            q[c] = B[lane][c];
        // Q_top = Q2_top R3^-1
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            if (c < pw) {
                double v = q[c];
#pragma unroll
                for (int i = 0; i < c; ++i)
                    v -= q[i] * R3[i][c];
                q[c] = v / R3[c][c];
            }
        }
        // LU of Q_top - S (s_k = -sign(pivot), sign(0) = +1); row k read from lane k
#pragma unroll
        for (int k = 0; k < CB; ++k) {
            if (k < pw) {
                const double d = readlane_d(q[k], k);
                const double sk = (d >= 0.0) ? -1.0 : 1.0;
                const double piv = d - sk;
                const bool below = lane > k && lane < pw;
                const double li = below ? q[k] / piv : 0.0;
#pragma unroll
                for (int c = k + 1; c < CB; ++c) {
                    const double u = readlane_d(q[c], k);
                    if (below)
                        q[c] -= li * u;
                }
                if (below)
                    q[k] = li;
                if (lane == k) {
                    q[k] = piv;
                    sg[k] = sk;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c)
            B[lane][c] = q[c];
    }
    __syncthreads();
    // Rc = R3 (R2 R1), upper, into registers (X is reused below)
    double rv[16];
    for (int idx = t, cnt = 0; idx < CB * CB; idx += 256, ++cnt) {
        const int r = idx / CB, c = idx % CB;
        double v = 0.0;
#pragma unroll 8
        for (int p = r; p <= c; ++p)
            v += R3[r][p] * X[p][c];
        rv[cnt] = v;
    }
    __syncthreads();
    // X := Y1^-1 (unit lower), lane = row, 16 columns per wave at once
    {
        double x[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            x[jj] = (lane == wave + 4 * jj) ? 1.0 : 0.0;
        for (int k = 0; k < pw; ++k) {
            const double yk = (lane > k && lane < pw) ? B[lane][k] : 0.0;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                x[jj] -= yk * readlane_d(x[jj], k);
            }
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int c = wave + 4 * jj;
            X[lane][c] = (lane < pw && c < pw) ? x[jj] : 0.0;
        }
    }
    __syncthreads();
    T *Ap = (sizeof(T) == 8) ? reinterpret_cast<T *>(w.A) : reinterpret_cast<T *>(w.A32);
    for (int idx = t, cnt = 0; idx < CB * CB; idx += 256, ++cnt) {
        const int r = idx / CB, c = idx % CB;
        // T = -U S Y1^-T:  T[r][c] = -sum_{p=r..c} U[r][p] s_p (Y1^-1)[c][p]
        double tv = 0.0;
        if (r < pw && c < pw && r <= c) {
#pragma unroll 8
            for (int p = r; p <= c; ++p)
                tv -= B[r][p] * sg[p] * X[c][p];
        }
        Tout[idx] = tv;
        if (r < pw && c < pw) {
            const double out = (r <= c) ? sg[r] * rv[cnt] : B[r][c];
            Ap[(j0 + c) * w.lda + j0 + r] = (T)out;
        }
        if (r == c && r < pw)
            w.tau[j0 + r] = tv;
        // U R3 (upper) for the row pass below the top block; identity beyond pw
        double ur = 0.0;
        if (r < pw && c < pw) {
            if (r <= c) {
#pragma unroll 8
                for (int p = r; p <= c; ++p)
                    ur += B[r][p] * R3[p][c];
            }
        } else if (r == c) {
            ur = 1.0;
        }
        w.cq_R[3 * CB * CB + idx] = ur;
    }
}

template <class T>
static void cqr_panel(const QrWork &w, int64_t j0, int pw, double *Tout, hipStream_t s)
{
    T *base = ((sizeof(T) == 8) ? reinterpret_cast<T *>(w.A) : reinterpret_cast<T *>(w.A32)) + j0 * w.lda + j0;
    const int64_t mk = w.m - j0;
    int64_t chunk = (mk + CQ_MAX_CHUNKS - 1) / CQ_MAX_CHUNKS;
    chunk = (chunk + CQ_ROWS - 1) / CQ_ROWS * CQ_ROWS;
    if (chunk < CQ_ROWS)
        chunk = CQ_ROWS;
    const unsigned nch = (unsigned)((mk + chunk - 1) / chunk);
    const unsigned nrow = (unsigned)((mk + CQ_ROWS - 1) / CQ_ROWS);
    const double u = 0x1p-53;
    const double shift = 11.0 * ((double)mk * pw + (double)pw * (pw + 1)) * u;
    double *R1 = w.cq_R, *R2 = w.cq_R + CB * CB, *R21 = w.cq_R + 2 * CB * CB, *UR3 = w.cq_R + 3 * CB * CB;
    const dim3 gsum_grid(CB * CB / 256, 4);
    // pass 1 (shifted): Gram of P, R1, Q1 = P R1^-1 into the scratch
    hipLaunchKernelGGL(cqr_gram_kernel<T>, dim3(nch), dim3(256), 0, s, (const T *)base, w.lda, mk, pw, chunk,
                       w.cq_part);
    hipLaunchKernelGGL(cqr_gsum_kernel, gsum_grid, dim3(256), 0, s, (const double *)w.cq_part, (int64_t)nch, w.cq_G);
    hipLaunchKernelGGL(cqr_chol_kernel, dim3(1), dim3(256), 0, s, (const double *)w.cq_G, pw, shift, R1,
                       (const double *)nullptr, (double *)nullptr, w.status);
    hipLaunchKernelGGL((cqr_pass_kernel<T, double>), dim3(nrow), dim3(256), 0, s, (const T *)base, w.lda, w.cq_S,
                       w.cq_ld, (int64_t)0, mk, pw, (const double *)R1);
    // pass 2: Q2 = Q1 R2^-1 in place
    hipLaunchKernelGGL(cqr_gram_kernel<double>, dim3(nch), dim3(256), 0, s, (const double *)w.cq_S, w.cq_ld, mk, pw,
                       chunk, w.cq_part);
    hipLaunchKernelGGL(cqr_gsum_kernel, gsum_grid, dim3(256), 0, s, (const double *)w.cq_part, (int64_t)nch, w.cq_G);
    hipLaunchKernelGGL(cqr_chol_kernel, dim3(1), dim3(256), 0, s, (const double *)w.cq_G, pw, 0.0, R2,
                       (const double *)R1, R21, w.status);
    hipLaunchKernelGGL((cqr_pass_kernel<double, double>), dim3(nrow), dim3(256), 0, s, (const double *)w.cq_S,
                       w.cq_ld, w.cq_S, w.cq_ld, (int64_t)0, mk, pw, (const double *)R2);
    // pass 3: R3 from the Gram of Q2, the top block's reconstruction, then Y below it
    hipLaunchKernelGGL(cqr_gram_kernel<double>, dim3(nch), dim3(256), 0, s, (const double *)w.cq_S, w.cq_ld, mk, pw,
                       chunk, w.cq_part);
    hipLaunchKernelGGL(cqr_gsum_kernel, gsum_grid, dim3(256), 0, s, (const double *)w.cq_part, (int64_t)nch, w.cq_G);
    hipLaunchKernelGGL(cqr_top_kernel<T>, dim3(1), dim3(256), 0, s, w, j0, pw, Tout);
    if (mk > pw) {
        const unsigned nb = (unsigned)((mk - pw + CQ_ROWS - 1) / CQ_ROWS);
        hipLaunchKernelGGL((cqr_pass_kernel<double, T>), dim3(nb), dim3(256), 0, s, (const double *)w.cq_S, w.cq_ld,
                           base, w.lda, (int64_t)pw, mk, pw, (const double *)UR3);
    }
}

void cqr_panel_f64(const QrWork &w, int64_t j0, int pw, double *Tout, hipStream_t s)
{
    cqr_panel<double>(w, j0, pw, Tout, s);
}

void cqr_panel_f32(const QrWork &w, int64_t j0, int pw, double *Tout, hipStream_t s)
{
    cqr_panel<float>(w, j0, pw, Tout, s);
}

}  // namespace gap
