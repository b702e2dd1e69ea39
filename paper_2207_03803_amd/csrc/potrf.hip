// Blocked right-looking Cholesky factorisation K = U^T U (U = L^T, upper
// triangular), in place, FP64 (Sec. Theory: the lower block of A is L_MM^T).
// Per 64-column step: factor the diagonal block in LDS, solve the block row
// U_kk^T X = A_kj by forward substitution, then update the trailing upper
// triangle with an FP64 MFMA product A_ij -= U_ki^T U_kj.
#include "kernels.h"

namespace gap {

constexpr int CNB = CHOL_NB;
constexpr int CLD = CNB + 1;

// Order the LDS accesses of one wave's lanes (no workgroup barrier: one wave).
DEV void lane_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Factor the kb x kb diagonal block starting at (k0, k0) on one wave: lane c
// holds column c of the block in registers (rows and columns past kb padded
// with the identity), and row j of each step is shared through LDS.  Each
// element sees the right-looking order: U[j][j] = sqrt(pivot), U[j][c] /=
// U[j][j], then U[r][c] -= U[j][r] U[j][c].
__global__ __launch_bounds__(64) void chol_diag_kernel(double *U, int64_t ld, int64_t k0, int kb, int32_t *status)
{
    __shared__ double row[CNB];
    const int c = threadIdx.x;
    double x[CNB];
    const double *col = U + (k0 + c) * ld + k0;
#pragma unroll
    for (int r = 0; r < CNB; ++r)
        x[r] = (c < kb) ? ((r <= c) ? col[r] : 0.0) : (r == c ? 1.0 : 0.0);
#pragma unroll
    for (int j = 0; j < CNB; ++j) {
        if (c == j) {
            double piv = x[j];
            if (!(piv > 0.0) || !isfinite(piv)) {
                set_status(status, DST_ENOTPD);  // the first failure is kept
                piv = 1.0;                       // keep the (discarded) rest finite
            }
            x[j] = sqrt(piv);
            row[j] = x[j];
        }
        lane_sync();
        const double dj = row[j];
        if (c > j) {
            x[j] = x[j] / dj;
            row[c] = x[j];
        }
        lane_sync();
        if (c > j) {
            const double xj = x[j];
#pragma unroll
            for (int r = j + 1; r < CNB; ++r)
                x[r] -= row[r] * xj;  // rows past c are below the diagonal: never stored
        }
        lane_sync();
    }
    if (c < kb) {
        double *out = U + (k0 + c) * ld + k0;
#pragma unroll
        for (int r = 0; r < CNB; ++r)
            if (r < kb)
                out[r] = (r <= c) ? x[r] : 0.0;
    }
}

// Block row: X = U_kk^-T B for the 64-column block `blockIdx.x` right of the
// diagonal block, one wave per block and one column per lane (each column's
// forward substitution is independent: no barriers), U_kk staged in LDS.
__global__ __launch_bounds__(64) void chol_trsm_kernel(double *U, int64_t ld, int64_t k0, int kb, int64_t n)
{
    __shared__ double Ukk[CNB * CLD];
    const int c = threadIdx.x;
    const int64_t c0 = k0 + kb + (int64_t)blockIdx.x * CNB;
    const int cw = (int)((n - c0) < CNB ? (n - c0) : CNB);
    {
        const double *col = U + (k0 + c) * ld + k0;
#pragma unroll
        for (int r = 0; r < CNB; ++r)
            Ukk[r * CLD + c] = (c < kb && r <= c) ? col[r] : 0.0;
    }
    lane_sync();
    if (c >= cw)
        return;
    double x[CNB];
    double *bc = U + (c0 + c) * ld + k0;
#pragma unroll
    for (int r = 0; r < CNB; ++r)
        x[r] = (r < kb) ? bc[r] : 0.0;
#pragma unroll
    for (int i = 0; i < CNB; ++i) {
        if (i < kb) {
            x[i] = x[i] / Ukk[i * CLD + i];
#pragma unroll
            for (int r = i + 1; r < CNB; ++r)
                x[r] -= Ukk[i * CLD + r] * x[i];  // U_kk rows past kb are zero
        }
    }
#pragma unroll
    for (int r = 0; r < CNB; ++r)
        if (r < kb)
            bc[r] = x[r];
}
using SS = TileShape<128, 128, 16, 2, 2>;

// Trailing update of the upper triangle: A[r][c] -= sum_{p < kb} U[k0+p][r] U[k0+p][c]
// for k1 <= r <= c < n and r < rlim, one 128 x 128 tile per workgroup.  With
// rlim = n the tiles are the upper ones of the trailing triangle (enumerated
// column by column); with rlim < n (a strip of at most 128 rows) they are one
// row of tiles across the columns.
__global__ __launch_bounds__(256) void chol_syrk_kernel(double *U, int64_t ld, int64_t k0, int kb, int64_t k1,
                                                        int64_t rlim, int64_t n)
{
    __shared__ double lds[2 * SS::STAGE];
    const int64_t L = blockIdx.x;
    int64_t ti = 0, tj = L;
    if (rlim >= n) {  // linear id -> (ti, tj), ti <= tj
        tj = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
        while ((tj + 1) * (tj + 2) / 2 <= L)
            ++tj;
        while (tj * (tj + 1) / 2 > L)
            --tj;
        ti = L - tj * (tj + 1) / 2;
    }
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
                if (r <= c && c < n && r < rlim)
                    U[c * ld + r] -= acc[i][j][e];
            }
}

static void syrk(double *U, int64_t ld, int64_t k0, int kb, int64_t k1, int64_t rlim, int64_t n, hipStream_t s)
{
    const int64_t nc = (n - k1 + SS::BN - 1) / SS::BN;
    const int64_t tiles = (rlim >= n) ? nc * (nc + 1) / 2 : nc;
    hipLaunchKernelGGL(chol_syrk_kernel, dim3((unsigned)tiles), dim3(256), 0, s, U, ld, k0, kb, k1, rlim, n);
}

// Steps are taken in pairs: block k's rows update only block k + 1's rows
// (a thin strip), block k + 1 is factored, then one trailing update of depth
// 128 applies both blocks to everything below (half the trailing passes, each
// twice as deep).
hipError_t launch_potrf_upper(double *U, int64_t ld, int64_t n, int32_t *status, hipStream_t s)
{
    auto factor_row = [&](int64_t k0, int kb) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(64), 0, s, U, ld, k0, kb, status);
        const int64_t rest = n - k0 - kb;
        if (rest > 0)
            hipLaunchKernelGGL(chol_trsm_kernel, dim3((unsigned)((rest + CNB - 1) / CNB)), dim3(64), 0, s, U, ld, k0,
                               kb, n);
        return rest;
    };
    int64_t k0 = 0;
    while (k0 < n) {
        const int kb = (int)((n - k0) < CNB ? (n - k0) : CNB);
        const int64_t rest = factor_row(k0, kb);
        if (rest <= 0)
            break;
        const int64_t k1 = k0 + kb;
        if (rest <= CNB) {  // one block left
            syrk(U, ld, k0, kb, k1, n, n, s);
            k0 = k1;
            continue;
        }
        syrk(U, ld, k0, kb, k1, k1 + CNB, n, s);  // block k's rows into block k + 1's rows
        factor_row(k1, CNB);
        syrk(U, ld, k0, kb + CNB, k1 + CNB, n, n, s);  // both blocks into the rest
        k0 = k1 + CNB;
    }
    return hipGetLastError();
}

}  // namespace gap
