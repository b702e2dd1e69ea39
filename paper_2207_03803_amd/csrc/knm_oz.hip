// FP64-accurate K_NM on INT8 MFMA (Ozaki scheme).  The descriptor dot
// products of the K_MN definition (Sec. Theory) are formed exactly in integer
// arithmetic from 8-bit slices of the FP64 values, then the power, the
// per-configuration segment sum and the Sigma^-1/2 row scale run in FP64 as in
// the FP64 build.
//
// Slicing (Ozaki, Ogita, Oishi & Rump 2012, with integer slice products as in
// Ootomo, Ozaki & Yokota 2024).  Row r of a descriptor array gets an exponent
// e_r with max_k |x_rk| < 2^e_r, and every entry becomes the integer
// N = rint(x 2^(54 - e_r)), |N| < 2^54, so x = N 2^(e_r - 54) up to half a unit
// of 2^(e_r - 54).  N is written in OZ_S = 7 balanced base-256 digits,
// N = sum_t D_t 256^(6 - t) with D_t in [-128, 127] (t = 0 the most significant,
// |D_0| <= 64).  Then
//   x_i . x_j = 2^(e_i + e_j - 12) sum_delta 2^(-8 delta) S_delta,
//   S_delta = sum_{t + u = delta} D_t(x_i) . D_u(x_j),
// with every S_delta exact in INT32 (at most 7 products of dp <= 4096 terms of
// at most 2^14 each).  Diagonals delta <= 6 are kept (28 slice products): the
// first dropped one is below 2^-56 of the leading term, so the dot product
// carries the error of the rounding to 54 bits, about FP64's own.
#include "knm.h"

namespace gap {

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int OZ_S = 7;                          // slices
constexpr int OZ_PAIRS = OZ_S * (OZ_S + 1) / 2;  // slice products kept
constexpr int OZ_BITS = 54;                      // |N| < 2^54

// (t, u) of the slice products, by diagonal delta = t + u from the smallest
// terms (delta = 6) to the largest, t ascending within a diagonal.
__constant__ int8_t oz_pt[OZ_PAIRS] = {0, 1, 2, 3, 4, 5, 6, 0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 0, 1, 2, 3, 0, 1, 2, 0, 1, 0};
__constant__ int8_t oz_pu[OZ_PAIRS] = {6, 5, 4, 3, 2, 1, 0, 5, 4, 3, 2, 1, 0, 4, 3, 2, 1, 0, 3, 2, 1, 0, 2, 1, 0, 1, 0, 0};

int knm_oz_dpad(int d) { return (d + 63) / 64 * 64; }
int knm_oz_slices() { return OZ_S; }

// One wave per row: the row's exponent, then its digits, four entries (one
// 32-bit word per slice) per lane and step.  Slice t of row r starts at
// out + t * rows * dp + r * dp; entries k >= d are zero.
__global__ __launch_bounds__(256) void oz_split_kernel(const double *__restrict__ x, int64_t rows, int d, int dp,
                                                       int8_t *__restrict__ out, int32_t *__restrict__ ex)
{
    const int lane = threadIdx.x & 63;
    const int64_t slice = rows * (int64_t)dp;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; r < rows; r += waves) {
        const double *src = x + r * (int64_t)d;
        double m = 0.0;
        for (int k = lane; k < d; k += 64)
            m = fmax(m, fabs(src[k]));
        for (int o = 32; o > 0; o >>= 1)
            m = fmax(m, __shfl_xor(m, o));
        int e = 0;
        if (m > 0.0)
            (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1): every |x| < 2^e
        if (lane == 0)
            ex[r] = e;
        for (int w = lane; w < dp / 4; w += 64) {
            uint32_t word[OZ_S];
#pragma unroll
            for (int t = 0; t < OZ_S; ++t)
                word[t] = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * w + q;
                int64_t n = k < d ? (int64_t)rint(ldexp(src[k], OZ_BITS - e)) : 0;
#pragma unroll
                for (int t = OZ_S - 1; t > 0; --t) {
                    const int8_t dg = (int8_t)(uint8_t)(n & 0xff);  // n - dg is a multiple of 256
                    word[t] |= (uint32_t)(uint8_t)dg << (8 * q);
                    n = (n - dg) >> 8;
                }
                word[0] |= (uint32_t)(uint8_t)(int8_t)n << (8 * q);
            }
#pragma unroll
            for (int t = 0; t < OZ_S; ++t)
                reinterpret_cast<uint32_t *>(out + t * slice + r * (int64_t)dp)[w] = word[t];
        }
    }
}

// ---------------------------------------------------------------------------
// Tile: the plan's tile of up to 256 atoms (whole configurations) x 128 sparse
// points, 512 threads = 8 waves of 64 x 64 (4 along the atoms, 2 along the
// sparse points), each a 4 x 4 grid of 16 x 16 INT32 accumulator blocks and the
// matching FP64 sums.  A workgroup takes OCT consecutive column tiles of one
// atom tile.  The k loop runs over the 28 slice products, each in steps of 64
// bytes (one MFMA), staged in LDS as [row][k] with rows padded to 80 bytes; the
// next step's global loads are in flight during the MFMAs.  After the last
// product of a diagonal, its INT32 sums are scaled by 2^(-8 delta) into the FP64
// sums (exact).
//
// Operand layout of v_mfma_i32_16x16x64_i8: lane l supplies row (A) or column
// (B) l % 16 and the sixteen k of group l / 16; A and B use the same k
// assignment.  Accumulator element e of lane l is C(4 (l / 16) + e, l % 16).
// ---------------------------------------------------------------------------
constexpr int OBM = KNM_BM;   // atoms per tile (the plan's tiles)
constexpr int OBN = 128;      // sparse points per tile
constexpr int OBK = 64;       // k (bytes) per step
constexpr int OLDK = OBK + 16;
constexpr int ONT = 512;
constexpr int OCT = 8;        // column tiles per workgroup
constexpr int OEPC = 32;      // epilogue columns per pass
constexpr int OEPLD = OEPC + 1;
constexpr int OA_BYTES = OBM * OLDK, OB_BYTES = OBN * OLDK, OSTAGE = OA_BYTES + OB_BYTES;
constexpr int O_LDS_GEMM = 2 * OSTAGE;
constexpr int O_LDS_EPI = OBM * OEPLD * 8;
constexpr int O_LDS = O_LDS_GEMM > O_LDS_EPI ? O_LDS_GEMM : O_LDS_EPI;
static_assert(OBM == 256 && ONT == 512, "loader mapping assumes 256 atoms and 512 threads");

struct KnmOzArgs {
    const int8_t *X, *XM;     // slices: X + t * x_slice + atom * dp, XM + t * xm_slice + col * dp
    int64_t x_slice, xm_slice;
    const int32_t *xe, *xme;  // row exponents
    int dp;
    const int64_t *offsets;
    const int32_t *tile_start, *cfg_list, *n_tiles_dev;
    int64_t M;
    int zeta;
    double sw2;
    const double *sigma;
    double *out;              // column-major: out[col * ldo + configuration]
    int64_t ldo;
    int64_t n_ct, n_cg;
};

DEV double ipow_oz(double g, int zeta)
{
    double p = g;
    for (int z = 1; z < zeta; ++z)
        p *= g;
    return p;
}

__global__ __launch_bounds__(ONT) __attribute__((amdgpu_waves_per_eu(2, 2))) void knm_oz_kernel(KnmOzArgs a)
{
    __shared__ __align__(16) unsigned char lds[O_LDS];
    __shared__ int32_t sstart[KNM_MAX_SEG + 1];
    __shared__ int64_t sbase[KNM_MAX_SEG];
    __shared__ int32_t srow[KNM_MAX_SEG];
    __shared__ double carry[OBN];
    __shared__ int32_t scan[KNM_MAX_SEG];
    __shared__ int32_t sexp[OBM];
    __shared__ int32_t cexp[OBN];

    const int64_t n_tiles = (int64_t)*a.n_tiles_dev;
    const int64_t total = n_tiles * a.n_cg;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if ((int64_t)blockIdx.x >= total_pad)
        return;
    const int64_t lw = xcd_remap(blockIdx.x, total_pad);
    if (lw >= total)
        return;
    const int64_t t_id = lw / a.n_cg, cg = lw % a.n_cg;
    const int64_t ct_lo = cg * OCT, ct_hi = (ct_lo + OCT) < a.n_ct ? (ct_lo + OCT) : a.n_ct;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // segments (configurations) of the tile and their atom offsets within it
    const int64_t p0 = a.tile_start[t_id];
    const int n_seg = (int)(a.tile_start[t_id + 1] - p0);
    if (tid < KNM_MAX_SEG) {
        int64_t sz = 0;
        if (tid < n_seg) {
            const int32_t cfg = a.cfg_list[p0 + tid];
            const int64_t lo = a.offsets[cfg];
            sz = a.offsets[cfg + 1] - lo;
            sbase[tid] = lo;
            srow[tid] = cfg;
        }
        scan[tid] = (int32_t)sz;
    }
    __syncthreads();
    for (int off = 1; off < KNM_MAX_SEG; off <<= 1) {
        int32_t v = 0;
        if (tid < KNM_MAX_SEG && tid >= off)
            v = scan[tid - off];
        __syncthreads();
        if (tid < KNM_MAX_SEG)
            scan[tid] += v;
        __syncthreads();
    }
    if (tid < KNM_MAX_SEG)
        sstart[tid + 1] = scan[tid];
    if (tid == 0)
        sstart[0] = 0;
    __syncthreads();
    const int64_t n_at = sstart[n_seg];

    auto emit = [&](int s, int64_t colg, double sum) {
        const int64_t row = srow[s];
        a.out[colg * a.ldo + row] = sum / a.sigma[row];
    };
    if (n_at == 0) {  // only empty configurations: their sums are zero
        const int ncol = (int)((ct_hi - ct_lo) * OBN);
        for (int item = tid; item < n_seg * ncol; item += ONT) {
            const int s = item % n_seg, c = item / n_seg;
            const int64_t colg = ct_lo * OBN + c;
            if (colg < a.M)
                emit(s, colg, 0.0);
        }
        return;
    }
    const bool multi = n_at > OBM;  // then n_seg == 1: one configuration in several atom chunks

    auto atom_of = [&](int r) -> int64_t {
        int lo = 0, hi = n_seg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sstart[mid] <= r)
                lo = mid;
            else
                hi = mid - 1;
        }
        return sbase[lo] + (r - sstart[lo]);
    };
    // this thread's two A chunks (rows ra0, ra0 + 128; 16-byte part pa) and one B chunk (row rb, part pb)
    const int ra0 = tid >> 2, pa = tid & 3;
    const int rb = tid >> 2, pb = tid & 3;
    const int nk = a.dp / OBK;
    const int n_steps = OZ_PAIRS * nk;

    i32x4 acc[4][4];
    double sum[4][4][4];
    for (int64_t ct = ct_lo; ct < ct_hi; ++ct) {
        const int64_t col0 = ct * OBN;
        const int64_t colb = col0 + rb;
        const int8_t *bsrc = (colb < a.M) ? a.XM + colb * (int64_t)a.dp + pb * 16 : nullptr;
        for (int64_t cs = 0; cs < n_at; cs += OBM) {
            const bool first = (cs == 0), last = (cs + OBM >= n_at);
            const int8_t *asrc[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = ra0 + 128 * h;
                asrc[h] = nullptr;
                if (multi) {
                    if (cs + r < n_at)
                        asrc[h] = a.X + (sbase[0] + cs + r) * (int64_t)a.dp + pa * 16;
                } else if (r < n_at) {
                    asrc[h] = a.X + atom_of(r) * (int64_t)a.dp + pa * 16;
                }
            }
            __syncthreads();  // the previous pass's epilogue is done with the LDS and the exponents
            for (int r = tid; r < OBM; r += ONT) {
                int64_t at = -1;
                if (multi) {
                    if (cs + r < n_at)
                        at = sbase[0] + cs + r;
                } else if (r < n_at) {
                    at = atom_of(r);
                }
                sexp[r] = at >= 0 ? a.xe[at] : 0;
            }
            if (tid < OBN)
                cexp[tid] = (col0 + tid < a.M) ? a.xme[col0 + tid] : 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] = i32x4{0, 0, 0, 0};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        sum[i][j][e] = 0.0;
                }

            i32x4 ra[2], rbv;
            const i32x4 zero4 = {0, 0, 0, 0};
            auto load = [&](int st) {
                const int p = st / nk, kc = st - p * nk;
                const int64_t ka = (int64_t)oz_pt[p] * a.x_slice + kc * OBK;
                const int64_t kb = (int64_t)oz_pu[p] * a.xm_slice + kc * OBK;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    ra[h] = asrc[h] ? *reinterpret_cast<const i32x4 *>(asrc[h] + ka) : zero4;
                rbv = bsrc ? *reinterpret_cast<const i32x4 *>(bsrc + kb) : zero4;
            };
            auto store = [&](unsigned char *As, unsigned char *Bs) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    *reinterpret_cast<i32x4 *>(As + (ra0 + 128 * h) * OLDK + pa * 16) = ra[h];
                *reinterpret_cast<i32x4 *>(Bs + rb * OLDK + pb * 16) = rbv;
            };
            load(0);
            store(lds, lds + OA_BYTES);
            __syncthreads();
            int p = 0, kc = 0;  // the current step's slice product and k step
            for (int st = 0; st < n_steps; ++st) {
                unsigned char *cur = lds + (st & 1) * OSTAGE;
                unsigned char *nxt = lds + ((st + 1) & 1) * OSTAGE;
                const bool more = st + 1 < n_steps;
                if (more)
                    load(st + 1);
                const unsigned char *As = cur, *Bs = cur + OA_BYTES;
                i32x4 af[4], bfr[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    af[i] = *reinterpret_cast<const i32x4 *>(As + (wm * 64 + i * 16 + (lane & 15)) * OLDK +
                                                             (lane >> 4) * 16);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bfr[j] = *reinterpret_cast<const i32x4 *>(Bs + (wn * 64 + j * 16 + (lane & 15)) * OLDK +
                                                              (lane >> 4) * 16);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bfr[j], acc[i][j], 0, 0, 0);
                if (kc == nk - 1 && oz_pu[p] == 0) {
                    // the diagonal delta = t ends with u = 0: fold it into the FP64 sums
                    const double sc = ldexp(1.0, -8 * (int)oz_pt[p]);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                sum[i][j][e] = fma((double)acc[i][j][e], sc, sum[i][j][e]);
                            acc[i][j] = i32x4{0, 0, 0, 0};
                        }
                }
                if (++kc == nk) {
                    kc = 0;
                    ++p;
                }
                if (more)
                    store(nxt, nxt + OA_BYTES);
                __syncthreads();
            }

            // g = 2^(e_i + e_j - 12) sum, k = sigma_w^2 g^zeta, in registers
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = wm * 64 + i * 16 + 4 * (lane >> 4) + e;
                        const int c = wn * 64 + j * 16 + (lane & 15);
                        const double g = ldexp(sum[i][j][e], sexp[r] + cexp[c] - 12);
                        sum[i][j][e] = a.sw2 * ipow_oz(g, a.zeta);
                    }

            double *E = reinterpret_cast<double *>(lds);  // [256][OEPLD], reused after the GEMM
            for (int q = 0; q < OBN / OEPC; ++q) {
                // columns [32 q, 32 q + 32) are blocks j = 2 (q & 1), 2 (q & 1) + 1 of waves wn = q / 2
                if (wn == (q >> 1)) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jj = 0; jj < 2; ++jj) {
                            const int j = 2 * (q & 1) + jj;
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                E[(wm * 64 + i * 16 + 4 * (lane >> 4) + e) * OEPLD + jj * 16 + (lane & 15)] =
                                    sum[i][j][e];
                        }
                }
                __syncthreads();
                if (!multi) {
                    for (int item = tid; item < n_seg * OEPC; item += ONT) {
                        const int s = item % n_seg, c = item / n_seg;
                        const int64_t colg = col0 + q * OEPC + c;
                        if (colg >= a.M)
                            continue;
                        const int a1 = sstart[s + 1];
                        double acc_s = 0.0;
                        for (int r = sstart[s]; r < a1; ++r)  // atom order
                            acc_s += E[r * OEPLD + c];
                        emit(s, colg, acc_s);
                    }
                } else if (tid < OEPC) {
                    const int c = tid;
                    const int64_t colg = col0 + q * OEPC + c;
                    const int nr = (int)((n_at - cs) < OBM ? (n_at - cs) : OBM);
                    double acc_s = 0.0;
                    for (int r = 0; r < nr; ++r)
                        acc_s += E[r * OEPLD + c];
                    const double tot = first ? acc_s : carry[q * OEPC + c] + acc_s;
                    carry[q * OEPC + c] = tot;
                    if (last && colg < a.M)
                        emit(0, colg, tot);
                }
                __syncthreads();
            }
        }
    }  // column tiles of the group
}

hipError_t launch_oz_split(const double *x, int64_t rows, int d, int8_t *out, int32_t *ex, hipStream_t s)
{
    if (rows <= 0)
        return hipSuccess;
    int64_t g = (rows + 3) / 4;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(oz_split_kernel, dim3((unsigned)g), dim3(256), 0, s, x, rows, d, knm_oz_dpad(d), out, ex);
    return hipGetLastError();
}

hipError_t launch_knm_oz(const KnmOzLaunch &l, hipStream_t s)
{
    KnmOzArgs a{};
    a.dp = knm_oz_dpad(l.d);
    a.X = l.X;
    a.XM = l.XM;
    a.x_slice = l.n_atoms * (int64_t)a.dp;
    a.xm_slice = l.M * (int64_t)a.dp;
    a.xe = l.xe;
    a.xme = l.xme;
    a.offsets = l.offsets;
    a.tile_start = l.tile_start;
    a.cfg_list = l.cfg_list;
    a.n_tiles_dev = l.n_tiles_dev;
    a.M = l.M;
    a.zeta = l.zeta;
    a.sw2 = l.sw2;
    a.sigma = l.sigma;
    a.out = l.out;
    a.ldo = l.ldo;
    a.n_ct = (l.M + OBN - 1) / OBN;
    a.n_cg = (a.n_ct + OCT - 1) / OCT;
    const int64_t total = l.max_tiles * a.n_cg;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if (total_pad == 0)
        return hipSuccess;
    hipLaunchKernelGGL(knm_oz_kernel, dim3((unsigned)total_pad), dim3(ONT), 0, s, a);
    return hipGetLastError();
}

}  // namespace gap
