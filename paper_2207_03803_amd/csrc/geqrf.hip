// Blocked Householder QR of the augmented stacked matrix [A | b] in FP64
// (Sec. Implementation: the factorisation leaves R in the upper triangle and
// the reflectors below it with their weights tau; Q^T b is obtained by
// carrying b along as an extra column, which is what applying the stored
// reflectors to b computes).
//
// Per panel of QR_NB columns:
//   1. column steps: each reflector from the column's norm (two-pass, FP64),
//      applied to the rest of the panel (three small kernels per column,
//      partial sums finished by the last workgroup to arrive);
//   2. split-K MFMA product P = V^T [V | C] over row chunks;
//   3. T of the compact WY form from V^T V and tau (one workgroup);
//   4. W = T^T V^T C (chunk partials summed in a fixed order);
//   5. C -= V W on MFMA.
// Reflector convention: H = I - tau v v^T, v(0) = 1, beta = -sign(alpha)
// ||(alpha, x)||, tau = (beta - alpha) / beta, v(1:) = x / (alpha - beta);
// tau = 0 when x is exactly zero.
#include "kernels.h"

namespace gap {

constexpr int NB = QR_NB;
constexpr int CR = QR_ROWS_PER_WG;  // rows per workgroup in the column steps (1 per thread)
constexpr int64_t MAX_CHUNKS = 64;

int64_t qr_max_chunks() { return MAX_CHUNKS; }
int64_t qr_max_col_wgs(int64_t m) { return (m + CR - 1) / CR; }

// Deterministic block sum of one value per thread (256 threads).
DEV double block_sum256(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

// Sum of n partials (stride `stride`) in a fixed order by a 256-thread block.
DEV double block_sum_partials(const double *p, int64_t n, int64_t stride, double *red)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256)
        s += p[i * stride];
    return block_sum256(s, red);
}

// Finish reflector j from alpha = A[j][j] and ||A[j+1:m, j]||^2 (thread 0).
DEV void finalize_reflector(double *A, int64_t lda, int64_t j, double xnorm2, double *tau,
                            double *refl)
{
    double *ajj = A + j * lda + j;
    const double alpha = *ajj;
    if (xnorm2 == 0.0) {
        tau[j] = 0.0;
        refl[0] = 0.0;
        return;
    }
    const double norm = sqrt(alpha * alpha + xnorm2);
    const double beta = (alpha >= 0.0) ? -norm : norm;
    tau[j] = (beta - alpha) / beta;
    refl[0] = 1.0 / (alpha - beta);
    *ajj = beta;
}

// Norm of column j below the diagonal; the last workgroup finalises reflector j.
__global__ __launch_bounds__(256) void qr_norm_kernel(QrWork w, int64_t j)
{
    __shared__ double red[4];
    __shared__ int flag;
    const int64_t r = j + (int64_t)blockIdx.x * CR + threadIdx.x;
    double x = 0.0;
    if (r > j && r < w.m) {
        x = w.A[j * w.lda + r];
        x *= x;
    }
    const double s = block_sum256(x, red);
    if (threadIdx.x == 0)
        w.colpart[blockIdx.x] = s;
    release_writes();
    if (!arrive_last(w.counters, gridDim.x, &flag))
        return;
    const double tot = block_sum_partials(w.colpart, gridDim.x, 1, red);
    if (threadIdx.x == 0)
        finalize_reflector(w.A, w.lda, j, tot, w.tau, w.refl);
}

// Scale column j into v and form partial dots v^T A[:, p] for panel columns
// j < p < je; the last workgroup stores w_p = tau_j * (v^T A[:, p]).
__global__ __launch_bounds__(256) void qr_dots_kernel(QrWork w, int64_t j, int64_t je)
{
    __shared__ double red[4][NB];
    __shared__ double red4[4];
    __shared__ int flag;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = j + (int64_t)blockIdx.x * CR + threadIdx.x;
    const double scale = w.refl[0];
    const bool zero_tau = (w.tau[j] == 0.0);
    double v = 0.0;
    if (r == j) {
        v = 1.0;
    } else if (r > j && r < w.m) {
        double *p = w.A + j * w.lda + r;
        v = zero_tau ? *p : *p * scale;
        if (!zero_tau)
            *p = v;
    }
    const int npc = (int)(je - j - 1);
    if (zero_tau || npc <= 0)
        return;  // nothing to apply (grid-uniform condition)
    for (int q = 0; q < npc; ++q) {
        double x = 0.0;
        if (r >= j && r < w.m)
            x = v * w.A[(j + 1 + q) * w.lda + r];
        x = wave_sum(x);
        if (lane == 0)
            red[wave][q] = x;
    }
    __syncthreads();
    double *part = w.colpart + (int64_t)blockIdx.x * (NB + 1);
    for (int q = threadIdx.x; q < npc; q += 256)
        part[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    release_writes();
    if (!arrive_last(w.counters + 1, gridDim.x, &flag))
        return;
    const double t = w.tau[j];
    for (int q = threadIdx.x; q < npc; q += 256) {
        double s = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b)
            s += w.colpart[(int64_t)b * (NB + 1) + q];
        w.refl[1 + q] = t * s;
    }
    (void)red4;
}

// A[:, p] -= w_p v for panel columns j < p < je, then the norm of column j+1
// below its diagonal (the last workgroup finalises reflector j+1).
__global__ __launch_bounds__(256) void qr_upd_kernel(QrWork w, int64_t j, int64_t je)
{
    __shared__ double red[4];
    __shared__ double wv[NB];
    __shared__ int flag;
    const int64_t r = j + (int64_t)blockIdx.x * CR + threadIdx.x;
    const int npc = (int)(je - j - 1);
    const bool zero_tau = (w.tau[j] == 0.0);
    for (int q = threadIdx.x; q < npc; q += 256)
        wv[q] = zero_tau ? 0.0 : w.refl[1 + q];
    __syncthreads();
    double nx = 0.0;
    if (r >= j && r < w.m) {
        const double v = (r == j) ? 1.0 : w.A[j * w.lda + r];
        if (!zero_tau) {
            for (int q = 0; q < npc; ++q) {
                double *p = w.A + (j + 1 + q) * w.lda + r;
                *p -= wv[q] * v;
            }
        }
        if (r > j + 1) {
            const double x = w.A[(j + 1) * w.lda + r];
            nx = x * x;
        }
    }
    const double s = block_sum256(nx, red);
    if (threadIdx.x == 0)
        w.colpart[blockIdx.x] = s;
    release_writes();
    if (!arrive_last(w.counters + 2, gridDim.x, &flag))
        return;
    const double tot = block_sum_partials(w.colpart, gridDim.x, 1, red);
    if (threadIdx.x == 0)
        finalize_reflector(w.A, w.lda, j + 1, tot, w.tau, w.refl);
}

// Reflector matrix V of the panel at (j0, j0): unit lower trapezoidal.
DEV double vpanel(const double *A, int64_t lda, int64_t m, int64_t j0, int pw, int64_t r, int p)
{
    if (p >= pw || r >= m)
        return 0.0;
    const int64_t d = r - (j0 + p);
    if (d < 0)
        return 0.0;
    if (d == 0)
        return 1.0;
    return A[(j0 + p) * lda + r];
}

using WS = TileShape<NB, 128, 16, 1, 4>;   // split-K V^T [V | C]
using US = TileShape<128, 128, 16, 2, 2>;  // C -= V W

// P[ch] = V^T X over the rows of chunk ch, X = [V | C] (columns j0 ...).
__global__ __launch_bounds__(256) void qr_wpart_kernel(QrWork w, int64_t j0, int pw, int64_t chunk,
                                                       int64_t width)
{
    __shared__ double lds[2 * WS::STAGE];
    const int64_t ch = blockIdx.y;
    const int64_t q0 = (int64_t)blockIdx.x * WS::BN;
    const int64_t rlo = j0 + ch * chunk;
    int64_t rhi = rlo + chunk;
    if (rhi > w.m)
        rhi = w.m;
    if (rlo >= rhi)
        return;
    d4 acc[WS::FM][WS::FN];
    zero_acc<WS>(acc);
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m;
    auto fa = [&](int p, int64_t k) -> double {
        const int64_t r = rlo + k;
        return (r < rhi) ? vpanel(A, lda, m, j0, pw, r, p) : 0.0;
    };
    auto fb = [&](int q, int64_t k) -> double {
        const int64_t r = rlo + k;
        const int64_t qq = q0 + q;
        if (r >= rhi || qq >= width)
            return 0.0;
        if (qq < pw)
            return vpanel(A, lda, m, j0, pw, r, (int)qq);
        return A[(j0 + qq) * lda + r];
    };
    gemm_tile<WS, true, true>(acc, lds, rhi - rlo, fa, fb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WS::WN, wn = wave % WS::WN;
    const int64_t ldw = NB + w.ncols;
    double *P = w.wpart + ch * NB * ldw;
#pragma unroll
    for (int i = 0; i < WS::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < WS::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = acc_row<WS>(wm, i, lane, e);
                const int64_t q = q0 + acc_col<WS>(wn, jj, lane);
                if (q < width)
                    P[p * ldw + q] = acc[i][jj][e];
            }
}

// T (upper triangular, compact WY) from G = V^T V and tau; one workgroup.
__global__ __launch_bounds__(256) void qr_tbuild_kernel(QrWork w, int64_t j0, int pw, int64_t nch)
{
    __shared__ double G[NB][NB + 1];
    __shared__ double T[NB][NB + 1];
    const int64_t ldw = NB + w.ncols;
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
        const int p = idx / NB, q = idx % NB;
        double s = 0.0;
        if (p < pw && q < pw)
            for (int64_t ch = 0; ch < nch; ++ch)
                s += w.wpart[ch * NB * ldw + p * ldw + q];
        G[p][q] = s;
        T[p][q] = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < pw; ++i) {
        const double ti = w.tau[j0 + i];
        const int r = threadIdx.x;
        double val = 0.0;
        if (r < i) {
            for (int s = r; s < i; ++s)
                val += T[r][s] * G[s][i];
            val = -ti * val;
        }
        __syncthreads();
        if (r < i)
            T[r][i] = val;
        if (r == i)
            T[i][i] = ti;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256)
        w.T[idx] = T[idx / NB][idx % NB];
}

// W[p][q] = sum_{s<=p} T[s][p] (V^T C)[s][q], the chunk partials summed in order.
__global__ __launch_bounds__(256) void qr_wred_kernel(QrWork w, int pw, int64_t nch, int64_t nt)
{
    __shared__ double T[NB][NB + 1];
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256)
        T[idx / NB][idx % NB] = w.T[idx];
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nt)
        return;
    const int64_t ldw = NB + w.ncols;
    double v[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        double s = 0.0;
        if (p < pw)
            for (int64_t ch = 0; ch < nch; ++ch)
                s += w.wpart[ch * NB * ldw + p * ldw + pw + q];
        v[p] = s;
    }
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r <= p; ++r)
            s += T[r][p] * v[r];
        w.W[p * w.ncols + q] = (p < pw) ? s : 0.0;
    }
}

// C[r][q] -= sum_p V[r][p] W[p][q] for rows j0.. and columns j0+pw..
__global__ __launch_bounds__(256) void qr_update_kernel(QrWork w, int64_t j0, int pw, int64_t nt)
{
    __shared__ double lds[2 * US::STAGE];
    const int64_t r0 = j0 + (int64_t)blockIdx.x * US::BM;
    const int64_t q0 = (int64_t)blockIdx.y * US::BN;
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m, ldW = w.ncols;
    const double *W = w.W;
    d4 acc[US::FM][US::FN];
    zero_acc<US>(acc);
    auto fa = [&](int mi, int64_t p) -> double { return vpanel(A, lda, m, j0, pw, r0 + mi, (int)p); };
    auto fb = [&](int ni, int64_t p) -> double {
        const int64_t q = q0 + ni;
        return (q < nt && p < pw) ? W[p * ldW + q] : 0.0;
    };
    gemm_tile<US, false, false>(acc, lds, pw, fa, fb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / US::WN, wn = wave % US::WN;
    double *C = w.A + (j0 + pw) * lda;
#pragma unroll
    for (int i = 0; i < US::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = r0 + acc_row<US>(wm, i, lane, e);
                const int64_t q = q0 + acc_col<US>(wn, jj, lane);
                if (r < m && q < nt)
                    C[q * lda + r] -= acc[i][jj][e];
            }
}

hipError_t launch_geqrf(const QrWork &w, hipStream_t s)
{
    for (int64_t j0 = 0; j0 < w.n; j0 += NB) {
        const int pw = (int)((w.n - j0) < NB ? (w.n - j0) : NB);
        const int64_t je = j0 + pw;
        const int64_t rows = w.m - j0;
        const unsigned gcol = (unsigned)((rows + CR - 1) / CR);
        // reflector for the panel's first column
        hipLaunchKernelGGL(qr_norm_kernel, dim3(gcol), dim3(256), 0, s, w, j0);
        for (int64_t j = j0; j < je; ++j) {
            const unsigned g = (unsigned)((w.m - j + CR - 1) / CR);
            hipLaunchKernelGGL(qr_dots_kernel, dim3(g), dim3(256), 0, s, w, j, je);
            if (j + 1 < je)
                hipLaunchKernelGGL(qr_upd_kernel, dim3(g), dim3(256), 0, s, w, j, je);
        }
        const int64_t nt = w.ncols - je;  // trailing columns incl. b and padding
        if (nt <= 0)
            continue;
        const int64_t width = pw + nt;
        const int64_t ncb = (width + WS::BN - 1) / WS::BN;
        int64_t nch = (2048 + ncb - 1) / ncb;
        if (nch > MAX_CHUNKS)
            nch = MAX_CHUNKS;
        int64_t chunk = (rows + nch - 1) / nch;
        chunk = (chunk + 15) & ~int64_t(15);
        if (chunk < 256)
            chunk = 256;
        nch = (rows + chunk - 1) / chunk;
        hipLaunchKernelGGL(qr_wpart_kernel, dim3((unsigned)ncb, (unsigned)nch), dim3(256), 0, s, w, j0,
                           pw, chunk, width);
        hipLaunchKernelGGL(qr_tbuild_kernel, dim3(1), dim3(256), 0, s, w, j0, pw, nch);
        hipLaunchKernelGGL(qr_wred_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, w, pw,
                           nch, nt);
        hipLaunchKernelGGL(qr_update_kernel, dim3((unsigned)((rows + US::BM - 1) / US::BM),
                                                  (unsigned)((nt + US::BN - 1) / US::BN)),
                           dim3(256), 0, s, w, j0, pw, nt);
    }
    return hipGetLastError();
}

}  // namespace gap
