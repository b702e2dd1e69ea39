// K_NM / K_MM builder: descriptor GEMM on FP64 MFMA with the dot-product
// covariance, the per-configuration segment-sum and the Sigma^-1/2 row scale
// fused into the epilogue (Sec. Theory: definition of K_MN; the upper block of
// A; Eqs. 1-2).  The n_atoms x M matrix of atom-level covariances is never
// written to HBM.
#include "kernels.h"

namespace gap {

// ---------------------------------------------------------------------------
// Tile plan: pack whole configurations, in order, into tiles of at most
// KNM_CAP atoms and KNM_MAX_SEG configurations (greedy).  A configuration with
// more than KNM_CAP atoms gets a tile of its own, processed in several atom
// chunks.  Also validates the offsets.  The plan is a sequential scan of the
// n_configs + 1 offsets by one thread; the workgroup stages them through LDS.
// ---------------------------------------------------------------------------
constexpr int PLAN_SEG = 4096;  // offsets staged in LDS per step of the scan

__global__ __launch_bounds__(256) void plan_tiles_kernel(const int64_t *__restrict__ offsets, int64_t N,
                                                         int64_t n_atoms, int32_t *__restrict__ tile_cfg,
                                                         int32_t *__restrict__ n_tiles, int64_t max_tiles,
                                                         int32_t *status)
{
    __shared__ int64_t seg[PLAN_SEG + 1];
    __shared__ int bad_s;
    // scan state, owned by thread 0
    int64_t t = 0, tile_atoms = 0, tile_n = 0, prev = 0;
    bool bad = false;
    if (threadIdx.x == 0) {
        bad_s = 0;
        tile_cfg[0] = 0;
    }
    for (int64_t base = 0; base < N; base += PLAN_SEG) {
        const int64_t cnt = (N - base) < PLAN_SEG ? (N - base) : PLAN_SEG;
        __syncthreads();
        for (int64_t i = threadIdx.x; i <= cnt; i += 256)
            seg[i] = offsets[base + i];
        __syncthreads();
        if (threadIdx.x == 0 && !bad) {
            if (base == 0) {
                prev = seg[0];
                bad = (prev != 0);
            }
            for (int64_t i = 0; i < cnt && !bad; ++i) {
                const int64_t nx = seg[i + 1];
                const int64_t na = nx - prev;
                if (na < 0) {
                    bad = true;
                    break;
                }
                if (tile_n > 0 && (tile_atoms + na > KNM_CAP || tile_n == KNM_MAX_SEG)) {
                    if (++t >= max_tiles) {
                        bad = true;
                        break;
                    }
                    tile_cfg[t] = (int32_t)(base + i);
                    tile_atoms = 0;
                    tile_n = 0;
                }
                tile_atoms += na;
                ++tile_n;
                prev = nx;
            }
            bad_s = bad ? 1 : 0;
        }
        __syncthreads();
        if (bad_s)
            break;
    }
    if (threadIdx.x != 0)
        return;
    if (prev != n_atoms)
        bad = true;
    if (bad) {
        *n_tiles = 0;
        set_status(status, DST_EINVAL);
        return;
    }
    tile_cfg[t + 1] = (int32_t)N;
    *n_tiles = (int32_t)(t + 1);
}

int64_t knm_max_tiles(int64_t N, int64_t n_atoms)
{
    // Two consecutive tiles hold more than KNM_CAP atoms between them unless the
    // first was closed by the configuration cap.
    int64_t bound = 2 * ((n_atoms + KNM_CAP - 1) / KNM_CAP) + (N + KNM_MAX_SEG - 1) / KNM_MAX_SEG + 1;
    return bound < N ? bound : N;
}

// 256 threads, 4 waves of 64 x 64, BK = 8: about 45 KB of LDS, so two or three
// workgroups share a CU and cover each other's barriers.
using KS = TileShape<KNM_BM, KNM_BN, 8, 4, 1>;
static_assert(KS::NT == 256, "K_NM kernel assumes 256 threads");
static_assert(KNM_BM == 256 && KNM_BN == 64, "loader mapping assumes a 256 x 64 tile");

constexpr int EPC = 16;           // epilogue columns per pass (one 16-column block)
constexpr int EPLD = EPC + 1;     // padded LDS row of the epilogue buffer

// Load one BK-slice (8 descriptor components) of the atom tile (256 rows) and
// the sparse tile (64 rows) into registers.  Rows past the valid range and k
// past d read as zero.
struct KnmLoads {
    double a[8];
    double b[2];
};

DEV void knm_load(KnmLoads &r, const double *__restrict__ X, int64_t row0, int64_t row_end,
                  const double *__restrict__ XM, int64_t col0, int64_t M, int d, int k0)
{
    const int tid = threadIdx.x;
    {
        const int64_t row = row0 + tid;
        const int kb = k0;
        const bool rv = row < row_end;
        const double *p = X + row * (int64_t)d + kb;
        if (rv && kb + 8 <= d) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                r.a[e] = p[e];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                r.a[e] = (rv && kb + e < d) ? p[e] : 0.0;
        }
    }
    {
        const int64_t row = col0 + (tid >> 2);
        const int kb = k0 + (tid & 3) * 2;
        const bool rv = row < M;
        const double *p = XM + row * (int64_t)d + kb;
        if (rv && kb + 2 <= d) {
            r.b[0] = p[0];
            r.b[1] = p[1];
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                r.b[e] = (rv && kb + e < d) ? p[e] : 0.0;
        }
    }
}

DEV void knm_store(const KnmLoads &r, double *As, double *Bs)
{
    const int tid = threadIdx.x;
    {
        const int row = tid;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            As[e * KS::LDA + row] = r.a[e];
    }
    {
        const int row = tid >> 2, kb = (tid & 3) * 2;
#pragma unroll
        for (int e = 0; e < 2; ++e)
            Bs[(kb + e) * KS::LDB + row] = r.b[e];
    }
}

// G = X[row0 : row0+256) . XM[col0 : col0+64)^T, accumulated in registers.
DEV void knm_gemm(d4 (&acc)[KS::FM][KS::FN], double *lds, const double *__restrict__ X, int64_t row0,
                  int64_t row_end, const double *__restrict__ XM, int64_t col0, int64_t M, int d)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / KS::WN, wn = wave % KS::WN;
    zero_acc<KS>(acc);
    const int nk = (d + KS::BK - 1) / KS::BK;
    KnmLoads r;
    knm_load(r, X, row0, row_end, XM, col0, M, d, 0);
    knm_store(r, lds, lds + KS::A_ELEMS);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        double *cur = lds + (kt & 1) * KS::STAGE;
        double *nxt = lds + ((kt + 1) & 1) * KS::STAGE;
        const bool more = kt + 1 < nk;
        if (more)
            knm_load(r, X, row0, row_end, XM, col0, M, d, (kt + 1) * KS::BK);
        mma_stage<KS>(cur, cur + KS::A_ELEMS, acc, wm, wn, lane);
        if (more)
            knm_store(r, nxt, nxt + KS::A_ELEMS);
        __syncthreads();
    }
}

constexpr int KNM_LDS_DOUBLES =
    (2 * KS::STAGE > KNM_BM * EPLD) ? 2 * KS::STAGE : KNM_BM * EPLD;

__global__ __launch_bounds__(256, 2) void knm_kernel(KnmArgs a)
{
    __shared__ double lds[KNM_LDS_DOUBLES];
    __shared__ int32_t sstart[KNM_MAX_SEG + 1];
    __shared__ double carry[KNM_BN];

    // The grid is sized for the largest possible tile count; the remap uses
    // the actual count so that all eight XCDs get an equal share of the tiles.
    const bool unit = (a.offsets == nullptr);
    const int64_t n_tiles = unit ? (a.n_rows_unit + KNM_BM - 1) / KNM_BM : (int64_t)*a.n_tiles_dev;
    const int64_t total = n_tiles * a.n_ct;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if ((int64_t)blockIdx.x >= total_pad)
        return;
    const int64_t lw = xcd_remap(blockIdx.x, total_pad);
    if (lw >= total)
        return;
    const int64_t t = lw / a.n_ct, ct = lw % a.n_ct;

    int64_t seg_lo, seg_hi, atom_lo, atom_hi;
    if (unit) {
        seg_lo = t * KNM_BM;
        seg_hi = seg_lo + KNM_BM < a.n_rows_unit ? seg_lo + KNM_BM : a.n_rows_unit;
        atom_lo = seg_lo;
        atom_hi = seg_hi;
    } else {
        seg_lo = a.tile_cfg[t];
        seg_hi = a.tile_cfg[t + 1];
        atom_lo = a.offsets[seg_lo];
        atom_hi = a.offsets[seg_hi];
    }
    const int n_seg = (int)(seg_hi - seg_lo);
    const int64_t col0 = ct * KNM_BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / KS::WN, wn = wave % KS::WN;

    // Segment boundaries relative to the tile's first atom.
    for (int s = tid; s <= n_seg; s += KS::NT)
        sstart[s] = unit ? s : (int32_t)(a.offsets[seg_lo + s] - atom_lo);

    auto emit = [&](int s, int64_t colg, double sum) {
        const int64_t seg = seg_lo + s;
        double v = sum;
        if (unit) {
            if (seg == colg)
                v += a.jitter;
            if (a.upper_only && seg > colg)
                v = 0.0;
        }
        if (a.sigma)
            v = v / a.sigma[seg];
        a.out[colg * a.ldo + a.row_off + seg] = v;
    };

    if (atom_hi == atom_lo) {  // only empty configurations: their sums are zero
        for (int item = tid; item < n_seg * KNM_BN; item += KS::NT) {
            const int s = item % n_seg, c = item / n_seg;
            const int64_t colg = col0 + c;
            if (colg < a.M)
                emit(s, colg, 0.0);
        }
        return;
    }

    const bool multi = (atom_hi - atom_lo) > KNM_BM;  // then n_seg == 1
    d4 acc[KS::FM][KS::FN];
    for (int64_t cs = atom_lo; cs < atom_hi; cs += KNM_BM) {
        const bool first = (cs == atom_lo), last = (cs + KNM_BM >= atom_hi);
        __syncthreads();
        knm_gemm(acc, lds, a.X, cs, atom_hi, a.XM, col0, a.M, a.d);

        // k = sigma_w^2 g^zeta, in registers.
#pragma unroll
        for (int i = 0; i < KS::FM; ++i)
#pragma unroll
            for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[i][j][e] = a.sw2 * ipow(acc[i][j][e], a.zeta);

        double *E = lds;  // [256][EPLD], reused after the GEMM
        for (int p = 0; p < KNM_BN / EPC; ++p) {
            // waves owning columns [p*16, p*16+16) park their values in LDS
            if (wn == (p * EPC) / KS::TN) {
#pragma unroll
                for (int i = 0; i < KS::FM; ++i)
#pragma unroll
                    for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int cl = acc_col<KS>(wn, j, lane, e) - p * EPC;
                            if (cl >= 0 && cl < EPC)
                                E[acc_row<KS>(wm, i, lane, e) * EPLD + cl] = acc[i][j][e];
                        }
            }
            __syncthreads();
            if (!multi) {
                for (int item = tid; item < n_seg * EPC; item += KS::NT) {
                    const int s = item % n_seg, c = item / n_seg;
                    const int64_t colg = col0 + p * EPC + c;
                    if (colg >= a.M)
                        continue;
                    double sum = 0.0;
                    for (int r = sstart[s]; r < sstart[s + 1]; ++r)
                        sum += E[r * EPLD + c];
                    emit(s, colg, sum);
                }
            } else if (tid < EPC) {
                const int c = tid;
                const int64_t colg = col0 + p * EPC + c;
                const int nr = (int)((atom_hi - cs) < KNM_BM ? (atom_hi - cs) : KNM_BM);
                double sum = 0.0;
                for (int r = 0; r < nr; ++r)
                    sum += E[r * EPLD + c];
                const double tot = first ? sum : carry[p * EPC + c] + sum;
                carry[p * EPC + c] = tot;
                if (last && colg < a.M)
                    emit(0, colg, tot);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Prediction (Eqs. 1-2): y_A = sum_{i in A} sum_j c_j sigma_w^2 (x_i . x_j)^zeta.
// Workgroup w owns configurations [w*C, (w+1)*C); it walks their atoms in
// chunks of 256, accumulates each atom's energy over all sparse tiles in LDS
// (the atom-by-sparse covariances stay in registers), then one thread per
// configuration adds its atoms' energies in atom order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void predict_kernel(const double *__restrict__ X, const int64_t *offsets,
                                                      int64_t N, const double *__restrict__ XM, int64_t M,
                                                      int d, int zeta, double sw2,
                                                      const double *__restrict__ c, double *y, int64_t C)
{
    __shared__ double lds[2 * KS::STAGE];
    __shared__ double eps[KNM_BM];
    __shared__ double part[KS::WN][KNM_BM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / KS::WN, wn = wave % KS::WN;
    const int64_t cfg_lo = (int64_t)blockIdx.x * C;
    int64_t cfg_hi = cfg_lo + C;
    if (cfg_hi > N)
        cfg_hi = N;
    if (cfg_lo >= cfg_hi)
        return;
    const int64_t atom_lo = offsets[cfg_lo], atom_hi = offsets[cfg_hi];
    const int ncfg = (int)(cfg_hi - cfg_lo);
    int64_t my_lo = 0, my_hi = 0;
    if (tid < ncfg) {
        my_lo = offsets[cfg_lo + tid];
        my_hi = offsets[cfg_lo + tid + 1];
    }
    double ysum = 0.0;
    const int64_t n_ct = (M + KNM_BN - 1) / KNM_BN;
    d4 acc[KS::FM][KS::FN];
    for (int64_t cs = atom_lo; cs < atom_hi; cs += KNM_BM) {
        __syncthreads();  // the previous chunk's sums have read eps
        if (tid < KNM_BM)
            eps[tid] = 0.0;
        for (int64_t ct = 0; ct < n_ct; ++ct) {
            const int64_t col0 = ct * KNM_BN;
            __syncthreads();
            knm_gemm(acc, lds, X, cs, atom_hi, XM, col0, M, d);
            double cw[KS::FN][4];
#pragma unroll
            for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t col = col0 + acc_col<KS>(wn, j, lane, e);
                    cw[j][e] = (col < M) ? c[col] : 0.0;
                }
#pragma unroll
            for (int i = 0; i < KS::FM; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        s += cw[j][e] * (sw2 * ipow(acc[i][j][e], zeta));
                // the 4 lanes that differ in l % 4 share this row
                s += __shfl_xor(s, 1, 64);
                s += __shfl_xor(s, 2, 64);
                if ((lane & 3) == 0)
                    part[wn][acc_row<KS>(wm, i, lane, 0)] = s;
            }
            __syncthreads();
            if (tid < KNM_BM) {
                double add = 0.0;
#pragma unroll
                for (int q = 0; q < KS::WN; ++q)
                    add += part[q][tid];
                eps[tid] += add;
            }
        }
        __syncthreads();
        if (tid < ncfg) {
            const int64_t lo = my_lo > cs ? my_lo : cs;
            const int64_t hi = my_hi < cs + KNM_BM ? my_hi : cs + KNM_BM;
            for (int64_t a = lo; a < hi; ++a)
                ysum += eps[a - cs];
        }
    }
    if (tid < ncfg)
        y[cfg_lo + tid] = ysum;
}

hipError_t launch_predict(const double *X, int64_t n_atoms, const int64_t *offsets, int64_t N,
                          const double *XM, int64_t M, int d, int zeta, double sw2, const double *c,
                          double *y, hipStream_t s)
{
    if (N <= 0)
        return hipSuccess;
    int64_t C = n_atoms > 0 ? (224 * N) / n_atoms : N;
    if (C < 1)
        C = 1;
    if (C > 256)
        C = 256;
    const int64_t grid = (N + C - 1) / C;
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)grid), dim3(KS::NT), 0, s, X, offsets, N, XM, M, d,
                       zeta, sw2, c, y, C);
    return hipGetLastError();
}

hipError_t launch_plan_tiles(const int64_t *offsets, int64_t N, int64_t n_atoms, int32_t *tile_cfg,
                             int32_t *n_tiles, int64_t max_tiles, int32_t *status, hipStream_t s)
{
    hipLaunchKernelGGL(plan_tiles_kernel, dim3(1), dim3(256), 0, s, offsets, N, n_atoms, tile_cfg,
                       n_tiles, max_tiles, status);
    return hipGetLastError();
}

hipError_t launch_knm(KnmArgs a, int64_t max_tiles, hipStream_t s)
{
    a.n_ct = (a.M + KNM_BN - 1) / KNM_BN;
    const int64_t total = max_tiles * a.n_ct;
    a.total_pad = (total + 7) & ~int64_t(7);
    if (a.total_pad == 0)
        return hipSuccess;
    hipLaunchKernelGGL(knm_kernel, dim3((unsigned)a.total_pad), dim3(KS::NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace gap
