// Blocked right-looking Cholesky factorisation K = U^T U (U = L^T, upper
// triangular), in place, FP64 (Sec. Theory: the lower block of A is L_MM^T).
// Per 64-column step: factor the diagonal block in LDS, solve the block row
// U_kk^T X = A_kj by forward substitution, then update the trailing upper
// triangle with an FP64 MFMA product A_ij -= U_ki^T U_kj.
#include "kernels.h"

namespace gap {

constexpr int CNB = CHOL_NB;
constexpr int CLD = CNB + 1;

// Factor the kb x kb diagonal block starting at (k0, k0).
__global__ __launch_bounds__(256) void chol_diag_kernel(double *U, int64_t ld, int64_t k0, int kb,
                                                        int32_t *status)
{
    __shared__ double S[CNB * CLD];
    __shared__ int failed;
    const int t = threadIdx.x;
    for (int idx = t; idx < kb * kb; idx += 256) {
        const int r = idx % kb, c = idx / kb;
        S[r * CLD + c] = (r <= c) ? U[(k0 + c) * ld + k0 + r] : 0.0;
    }
    if (t == 0)
        failed = 0;
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        if (t == 0) {
            double piv = S[j * CLD + j];
            if (!(piv > 0.0) || !isfinite(piv)) {
                if (!failed)
                    set_status(status, DST_ENOTPD);
                failed = 1;
                piv = 1.0;  // keep the (discarded) rest finite
            }
            S[j * CLD + j] = sqrt(piv);
        }
        __syncthreads();
        const double dj = S[j * CLD + j];
        for (int c = j + 1 + t; c < kb; c += 256)
            S[j * CLD + c] /= dj;
        __syncthreads();
        // trailing: S[r][c] -= U[j][r] U[j][c] for j < r <= c
        const int w = kb - j - 1;
        for (int idx = t; idx < w * w; idx += 256) {
            const int r = j + 1 + idx % w, c = j + 1 + idx / w;
            if (r <= c)
                S[r * CLD + c] -= S[j * CLD + r] * S[j * CLD + c];
        }
        __syncthreads();
    }
    for (int idx = t; idx < kb * kb; idx += 256) {
        const int r = idx % kb, c = idx / kb;
        U[(k0 + c) * ld + k0 + r] = (r <= c) ? S[r * CLD + c] : 0.0;
    }
}

// Block row: X = U_kk^-T B for the 64-column block `blockIdx.x` right of the
// diagonal block (forward substitution, right-looking, in LDS).
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *U, int64_t ld, int64_t k0, int kb,
                                                        int64_t n)
{
    __shared__ double Ukk[CNB * CLD];
    __shared__ double B[CNB * CLD];
    const int t = threadIdx.x;
    const int64_t c0 = k0 + kb + (int64_t)blockIdx.x * CNB;
    const int cw = (int)((n - c0) < CNB ? (n - c0) : CNB);
    for (int idx = t; idx < kb * kb; idx += 256) {
        const int r = idx % kb, c = idx / kb;
        Ukk[r * CLD + c] = U[(k0 + c) * ld + k0 + r];
    }
    for (int idx = t; idx < kb * cw; idx += 256) {
        const int r = idx % kb, c = idx / kb;
        B[r * CLD + c] = U[(c0 + c) * ld + k0 + r];
    }
    __syncthreads();
    for (int i = 0; i < kb; ++i) {
        const double di = Ukk[i * CLD + i];
        for (int c = t; c < cw; c += 256)
            B[i * CLD + c] /= di;
        __syncthreads();
        const int rows = kb - i - 1;
        for (int idx = t; idx < rows * cw; idx += 256) {
            const int r = i + 1 + idx % rows, c = idx / rows;
            B[r * CLD + c] -= Ukk[i * CLD + r] * B[i * CLD + c];
        }
        __syncthreads();
    }
    for (int idx = t; idx < kb * cw; idx += 256) {
        const int r = idx % kb, c = idx / kb;
        U[(c0 + c) * ld + k0 + r] = B[r * CLD + c];
    }
}

using SS = TileShape<128, 128, 16, 2, 2>;

// Trailing update of the upper triangle: A[r][c] -= sum_p U[k0+p][r] U[k0+p][c]
// for k1 <= r <= c < n, one 128 x 128 tile per workgroup (upper tiles only).
__global__ __launch_bounds__(256) void chol_syrk_kernel(double *U, int64_t ld, int64_t k0, int kb,
                                                        int64_t n)
{
    __shared__ double lds[2 * SS::STAGE];
    const int64_t k1 = k0 + kb;
    // linear id -> (ti, tj), ti <= tj, enumerated column by column
    const int64_t L = blockIdx.x;
    int64_t tj = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
    while ((tj + 1) * (tj + 2) / 2 <= L)
        ++tj;
    while (tj * (tj + 1) / 2 > L)
        --tj;
    const int64_t ti = L - tj * (tj + 1) / 2;
    const int64_t r0 = k1 + ti * SS::BM, c0 = k1 + tj * SS::BN;

    // The tile is computed transposed, acc(c, r), so that consecutive lanes
    // update consecutive rows of the column-major matrix.
    d4 acc[SS::FM][SS::FN];
    zero_acc<SS>(acc);
    const double *P = U + k0;  // element (row x, p) = U[k0 + p][x] at x * ld + p
    auto fa = [&](int mi, int64_t p) -> double {
        const int64_t x = c0 + mi;
        return (x < n && p < kb) ? P[x * ld + p] : 0.0;
    };
    auto fb = [&](int ni, int64_t p) -> double {
        const int64_t x = r0 + ni;
        return (x < n && p < kb) ? P[x * ld + p] : 0.0;
    };
    gemm_tile<SS, true, true>(acc, lds, kb, fa, fb);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / SS::WN, wn = wave % SS::WN;
#pragma unroll
    for (int i = 0; i < SS::FM; ++i)
#pragma unroll
        for (int j = 0; j < SS::FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + acc_row<SS>(wm, i, lane, e);
                const int64_t r = r0 + acc_col<SS>(wn, j, lane, e);
                if (r <= c && c < n)
                    U[c * ld + r] -= acc[i][j][e];
            }
}

hipError_t launch_potrf_upper(double *U, int64_t ld, int64_t n, int32_t *status, hipStream_t s)
{
    for (int64_t k0 = 0; k0 < n; k0 += CNB) {
        const int kb = (int)((n - k0) < CNB ? (n - k0) : CNB);
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, U, ld, k0, kb, status);
        const int64_t rest = n - k0 - kb;
        if (rest <= 0)
            break;
        const int64_t nbr = (rest + CNB - 1) / CNB;
        hipLaunchKernelGGL(chol_trsm_kernel, dim3((unsigned)nbr), dim3(256), 0, s, U, ld, k0, kb, n);
        const int64_t nt = (rest + SS::BM - 1) / SS::BM;
        const int64_t pairs = nt * (nt + 1) / 2;
        hipLaunchKernelGGL(chol_syrk_kernel, dim3((unsigned)pairs), dim3(256), 0, s, U, ld, k0, kb, n);
    }
    return hipGetLastError();
}

}  // namespace gap
