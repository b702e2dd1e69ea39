// Low-precision K_NM for the mixed-precision form: the descriptor dot products
// run on BF16 or FP16 MFMA (v_mfma_f32_16x16x32_bf16 / _f16) with FP32
// accumulation; the power, the per-configuration segment sum (Sec. Theory:
// definition of K_MN) and the Sigma^-1/2 row scale run in FP32 in the epilogue,
// and the rows land in the FP32 copy of the stacked matrix that the FP32
// Householder QR factors.  The FP64 K_NM is still built: the refinement's
// residuals need the FP64 problem's A.
#include "knm.h"

namespace gap {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// FP64 -> FP32 rounded to odd: of the two floats around x, the one whose last
// significand bit is 1 (x itself when it is a float).  Rounding that float to a
// format with at least two fewer significand bits (BF16: 8, FP16: 11) gives
// the correctly rounded result, with no double-rounding error.
DEV float f64_to_f32_odd(double x)
{
    const float f = (float)x;
    const double fd = (double)f;
    if (fd == x)
        return f;
    uint32_t u = __float_as_uint(f);
    if (f == 0.0f)
        return __uint_as_float(x > 0.0 ? 1u : 0x80000001u);
    if ((u & 1u) == 0u) {
        const bool up = x > fd;                 // x lies above f
        u = ((f > 0.0f) == up) ? u + 1u : u - 1u;  // the neighbour on x's side
    }
    return __uint_as_float(u);
}

// Bits of x rounded to nearest (ties to even) in BF16 or FP16.
template <bool BF>
DEV uint16_t to_lp_bits(double x)
{
    const float f = f64_to_f32_odd(x);
    if constexpr (BF) {
        uint32_t u = __float_as_uint(f);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    } else {
        const _Float16 h = (_Float16)f;
        return __builtin_bit_cast(uint16_t, h);
    }
}

// out[r * dp + k] = x[r * d + k] rounded (k < d), 0 for d <= k < dp; eight
// elements (16 bytes) per thread.
template <bool BF>
__global__ __launch_bounds__(256) void convert_lp_kernel(const double *__restrict__ x, int64_t rows, int d,
                                                         uint16_t *__restrict__ out, int dp)
{
    const int64_t per_row = dp / 8;
    const int64_t total = rows * per_row;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / per_row;
        const int k0 = (int)(i % per_row) * 8;
        const double *src = x + r * (int64_t)d;
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            v[e] = (k0 + e < d) ? to_lp_bits<BF>(src[k0 + e]) : (uint16_t)0;
        u32x4 w;
        w[0] = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        w[1] = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
        w[2] = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
        w[3] = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<u32x4 *>(out + r * (int64_t)dp + k0) = w;
    }
}

// ---------------------------------------------------------------------------
// Tile: the plan's tile of up to 256 atoms (whole configurations) x 128 sparse
// points, 512 threads = 8 waves of 64 x 64 (4 along the atoms, 2 along the
// sparse points), each a 4 x 4 grid of 16 x 16 accumulator blocks.  A
// workgroup takes LCT consecutive column tiles of one atom tile, so the tile's
// set-up (segment table, atom rows) is shared and the atom rows stay in L2.  K runs in
// slices of 32 (one MFMA), staged in LDS as [row][k] with the row padded to 40
// elements; the next slice's global loads are in flight during the MFMAs.
//
// Operand layout of v_mfma_f32_16x16x32_{bf16,f16}: lane l supplies row (A) or
// column (B) l % 16 and the eight k of group l / 16; A and B use the same k
// assignment, so any order of k within the 32 gives the same dot products.
// Accumulator element e of lane l is C(4 (l / 16) + e, l % 16).
// ---------------------------------------------------------------------------
constexpr int LBM = KNM_BM;   // atoms per tile (the plan's tiles)
constexpr int LBN = 128;      // sparse points per tile
constexpr int LBK = 32;       // k per slice
constexpr int LDSK = LBK + 8; // padded LDS row (elements)
constexpr int LNT = 512;
constexpr int LCT = 8;        // column tiles per workgroup (the tile's setup is shared)
constexpr int LEPC = 64;      // epilogue columns per pass (the columns of one wn)
constexpr int LEPLD = LEPC + 1;
constexpr int LA_ELEMS = LBM * LDSK, LB_ELEMS = LBN * LDSK, LSTAGE = LA_ELEMS + LB_ELEMS;
constexpr int LDS_BYTES_GEMM = 2 * LSTAGE * 2;
constexpr int LDS_BYTES_EPI = LBM * LEPLD * 4;
constexpr int LDS_BYTES = LDS_BYTES_GEMM > LDS_BYTES_EPI ? LDS_BYTES_GEMM : LDS_BYTES_EPI;
static_assert(LBM == 256 && LNT == 512, "loader mapping assumes 256 atoms and 512 threads");

struct KnmLpArgs {
    const uint16_t *X;          // [n_atoms x dp] rounded descriptors
    const uint16_t *XM;         // [M x dp] rounded sparse points
    int dp;                     // padded descriptor length (multiple of 32)
    const int64_t *offsets;
    const int32_t *tile_start, *cfg_list, *n_tiles_dev;
    int64_t M;
    int zeta;
    float sw2;
    const double *sigma;
    float *out;                 // column-major: out[col * ldo + configuration]
    int64_t ldo;
    int64_t n_ct, n_cg, total_pad;  // column tiles, groups of LCT of them
};

template <bool BF>
DEV f4 mfma_lp(const u32x4 &a, const u32x4 &b, const f4 &c)
{
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
}

DEV float ipowf(float g, int zeta)
{
    float p = g;
    for (int z = 1; z < zeta; ++z)
        p *= g;
    return p;
}

template <bool BF>
__global__ __launch_bounds__(LNT) __attribute__((amdgpu_waves_per_eu(4, 4))) void knm_lp_kernel(KnmLpArgs a)
{
    __shared__ __align__(16) unsigned char lds_raw[LDS_BYTES];
    __shared__ int32_t sstart[KNM_MAX_SEG + 1];
    __shared__ int64_t sbase[KNM_MAX_SEG];
    __shared__ int32_t srow[KNM_MAX_SEG];
    __shared__ float carry[LBN];
    __shared__ int32_t scan[KNM_MAX_SEG];
    uint16_t *lds = reinterpret_cast<uint16_t *>(lds_raw);

    const int64_t n_tiles = (int64_t)*a.n_tiles_dev;
    const int64_t total = n_tiles * a.n_cg;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if ((int64_t)blockIdx.x >= total_pad)
        return;
    const int64_t lw = xcd_remap(blockIdx.x, total_pad);
    if (lw >= total)
        return;
    const int64_t t = lw / a.n_cg, cg = lw % a.n_cg;
    const int64_t ct_lo = cg * LCT, ct_hi = (ct_lo + LCT) < a.n_ct ? (ct_lo + LCT) : a.n_ct;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // segments (configurations) of the tile and their atom offsets within it
    const int64_t p0 = a.tile_start[t];
    const int n_seg = (int)(a.tile_start[t + 1] - p0);
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
        int32_t x = 0;
        if (tid < KNM_MAX_SEG && tid >= off)
            x = scan[tid - off];
        __syncthreads();
        if (tid < KNM_MAX_SEG)
            scan[tid] += x;
        __syncthreads();
    }
    if (tid < KNM_MAX_SEG)
        sstart[tid + 1] = scan[tid];
    if (tid == 0)
        sstart[0] = 0;
    __syncthreads();
    const int64_t n_at = sstart[n_seg];

    auto emit = [&](int s, int64_t colg, float sum) {
        const int64_t row = srow[s];
        a.out[colg * a.ldo + row] = (float)((double)sum / a.sigma[row]);
    };
    if (n_at == 0) {  // only empty configurations: their sums are zero
        const int ncol = (int)((ct_hi - ct_lo) * LBN);
        for (int item = tid; item < n_seg * ncol; item += LNT) {
            const int s = item % n_seg, c = item / n_seg;
            const int64_t colg = ct_lo * LBN + c;
            if (colg < a.M)
                emit(s, colg, 0.0f);
        }
        return;
    }
    const bool multi = n_at > LBM;  // then n_seg == 1: one configuration in several atom chunks

    // atom row of tile row r (packed tiles): segment by binary search
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
    // this thread's two A chunks (rows ra0, ra0 + 128; part pa) and one B chunk (row rb, part pb)
    const int ra0 = tid >> 2, pa = tid & 3;
    const int rb = tid >> 2, pb = tid & 3;
    const int nk = a.dp / LBK;

    f4 acc[4][4];
    for (int64_t ct = ct_lo; ct < ct_hi; ++ct) {
    const int64_t col0 = ct * LBN;
    const int64_t colb = col0 + rb;
    const uint16_t *bsrc = (colb < a.M) ? a.XM + colb * (int64_t)a.dp + pb * 8 : nullptr;
    for (int64_t cs = 0; cs < n_at; cs += LBM) {
        const bool first = (cs == 0), last = (cs + LBM >= n_at);
        const uint16_t *asrc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = ra0 + 128 * h;
            asrc[h] = nullptr;
            if (multi) {
                if (cs + r < n_at)
                    asrc[h] = a.X + (sbase[0] + cs + r) * (int64_t)a.dp + pa * 8;
            } else if (r < n_at) {
                asrc[h] = a.X + atom_of(r) * (int64_t)a.dp + pa * 8;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

        u32x4 ra[2], rbv;
        const u32x4 zero4 = {0u, 0u, 0u, 0u};
        auto load = [&](int kt) {
            const int k0 = kt * LBK;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                ra[h] = asrc[h] ? *reinterpret_cast<const u32x4 *>(asrc[h] + k0) : zero4;
            rbv = bsrc ? *reinterpret_cast<const u32x4 *>(bsrc + k0) : zero4;
        };
        auto store = [&](uint16_t *As, uint16_t *Bs) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                *reinterpret_cast<u32x4 *>(As + (ra0 + 128 * h) * LDSK + pa * 8) = ra[h];
            *reinterpret_cast<u32x4 *>(Bs + rb * LDSK + pb * 8) = rbv;
        };
        __syncthreads();  // the previous chunk's epilogue is done with the LDS
        load(0);
        store(lds, lds + LA_ELEMS);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            uint16_t *cur = lds + (kt & 1) * LSTAGE;
            uint16_t *nxt = lds + ((kt + 1) & 1) * LSTAGE;
            const bool more = kt + 1 < nk;
            if (more)
                load(kt + 1);
            const uint16_t *As = cur, *Bs = cur + LA_ELEMS;
            u32x4 af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const u32x4 *>(As + (wm * 64 + i * 16 + (lane & 15)) * LDSK + (lane >> 4) * 8);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bfr[j] = *reinterpret_cast<const u32x4 *>(Bs + (wn * 64 + j * 16 + (lane & 15)) * LDSK + (lane >> 4) * 8);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = mfma_lp<BF>(af[i], bfr[j], acc[i][j]);
            if (more)
                store(nxt, nxt + LA_ELEMS);
            __syncthreads();
        }

        // k = sigma_w^2 g^zeta in FP32, in registers
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[i][j][e] = a.sw2 * ipowf(acc[i][j][e], a.zeta);

        float *E = reinterpret_cast<float *>(lds_raw);  // [256][LEPLD], reused after the GEMM
        for (int p = 0; p < LBN / LEPC; ++p) {
            // columns [64 p, 64 p + 64) are the blocks of the waves wn = p
            if (wn == p) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            E[(wm * 64 + i * 16 + 4 * (lane >> 4) + e) * LEPLD + j * 16 + (lane & 15)] = acc[i][j][e];
            }
            __syncthreads();
            if (!multi) {
                for (int item = tid; item < n_seg * LEPC; item += LNT) {
                    const int s = item % n_seg, c = item / n_seg;
                    const int64_t colg = col0 + p * LEPC + c;
                    if (colg >= a.M)
                        continue;
                    const int a1 = sstart[s + 1];
                    float sum = 0.0f;
                    int r = sstart[s];
                    for (; r + 8 <= a1; r += 8) {  // atom order; the loads of 8 rows issued together
                        float v[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            v[k] = E[(r + k) * LEPLD + c];
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            sum += v[k];
                    }
                    for (; r < a1; ++r)
                        sum += E[r * LEPLD + c];
                    emit(s, colg, sum);
                }
            } else if (tid < LEPC) {
                const int c = tid;
                const int64_t colg = col0 + p * LEPC + c;
                const int nr = (int)((n_at - cs) < LBM ? (n_at - cs) : LBM);
                float sum = 0.0f;
                for (int r = 0; r < nr; ++r)
                    sum += E[r * LEPLD + c];
                const float tot = first ? sum : carry[p * LEPC + c] + sum;
                carry[p * LEPC + c] = tot;
                if (last && colg < a.M)
                    emit(0, colg, tot);
            }
            __syncthreads();
        }
    }
    }  // column tiles of the group
}

int knm_lp_dpad(int d) { return (d + LBK - 1) / LBK * LBK; }

hipError_t launch_convert_lp(const double *x, int64_t rows, int d, uint16_t *out, bool bf16, hipStream_t s)
{
    const int dp = knm_lp_dpad(d);
    int64_t g = (rows * (dp / 8) + 255) / 256;
    if (g > 65536)
        g = 65536;
    if (g < 1)
        return hipSuccess;
    if (bf16)
        hipLaunchKernelGGL(convert_lp_kernel<true>, dim3((unsigned)g), dim3(256), 0, s, x, rows, d, out, dp);
    else
        hipLaunchKernelGGL(convert_lp_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, x, rows, d, out, dp);
    return hipGetLastError();
}

hipError_t launch_knm_lp(const KnmLpLaunch &l, hipStream_t s)
{
    KnmLpArgs a{};
    a.X = l.X;
    a.XM = l.XM;
    a.dp = knm_lp_dpad(l.d);
    a.offsets = l.offsets;
    a.tile_start = l.tile_start;
    a.cfg_list = l.cfg_list;
    a.n_tiles_dev = l.n_tiles_dev;
    a.M = l.M;
    a.zeta = l.zeta;
    a.sw2 = (float)l.sw2;
    a.sigma = l.sigma;
    a.out = l.out;
    a.ldo = l.ldo;
    a.n_ct = (l.M + LBN - 1) / LBN;
    a.n_cg = (a.n_ct + LCT - 1) / LCT;
    const int64_t total = l.max_tiles * a.n_cg;
    a.total_pad = (total + 7) & ~int64_t(7);
    if (a.total_pad == 0)
        return hipSuccess;
    if (l.bf16)
        hipLaunchKernelGGL(knm_lp_kernel<true>, dim3((unsigned)a.total_pad), dim3(LNT), 0, s, a);
    else
        hipLaunchKernelGGL(knm_lp_kernel<false>, dim3((unsigned)a.total_pad), dim3(LNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace gap
