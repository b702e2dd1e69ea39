// K_NM / K_MM and predict kernel interfaces of the GAP fit library.  Every
// launcher enqueues on the given stream and returns the launch error
// (hipSuccess when none).
#pragma once

#include "common.h"

namespace gap {

// ----------------------------------------------------------------- K_NM / K_MM
constexpr int KNM_BM = 256;       // atoms per chunk (GEMM rows)
constexpr int KNM_BN = 64;        // sparse points per tile (GEMM columns)
constexpr int KNM_CAP = KNM_BM;   // atom capacity of a packed tile
constexpr int KNM_MAX_SEG = 256;  // configurations per tile

struct KnmArgs {
    const double *X;           // [rows x d] row-major descriptors
    const int64_t *offsets;    // [N+1] CSR offsets; nullptr = unit segments (row r is segment r)
    const int32_t *tile_start; // [n_tiles+1] first position of each tile in cfg_list (from the plan)
    const int32_t *cfg_list;   // [N] configurations, tile by tile
    const int32_t *n_tiles_dev;
    int64_t n_rows_unit;       // unit segments: number of rows
    const double *XM;          // [M x d] sparse points
    int64_t M;
    int d, zeta;
    double sw2;                // sigma_w^2
    const double *sigma;       // [N] or nullptr: the segment sum is divided by sigma
    double *out;               // column-major: out[col * ldo + row_off + segment]
    int64_t ldo, row_off;
    double jitter;             // unit segments: added where segment == column
    int upper_only;            // unit segments: write 0 where segment > column
    int64_t n_ct, total_pad;   // filled by launch_knm
    int32_t *status;
    int bn;                    // column tile: 64 sparse points (0 or 64) or 32
    // derivative observation rows (launch_kdm only): the segments are observations over
    // positions p (offsets is their CSR); row p reads X[pos_grad[p]], X = the descriptor
    // gradients, and its products are scaled by zeta sw2 pos_weight[p] D(grad_atom[g], j)
    const int64_t *pos_grad;   // [n_pos]
    const double *pos_weight;  // [n_pos]
    const int64_t *grad_atom;  // [n_grad]
    const double *D;           // row-major, D[i * ldd + j] = (x_i . x_j)^(zeta - 1); null: 1 (zeta = 1)
    int64_t ldd;
    int64_t n_grad, n_src;     // bounds of pos_grad and grad_atom values (out of range: zero row, DST_EINVAL)
};

int64_t knm_max_tiles(int64_t N, int64_t n_atoms);
int64_t knm_plan_chunks(int64_t N);
// Plan arrays (device): tile_start [max_tiles + 1], n_tiles [1], cfg_list [N],
// lstart [n_chunks * 2049], lcount [n_chunks] (n_chunks = knm_plan_chunks(N)).
struct KnmPlan {
    int32_t *tile_start, *n_tiles, *cfg_list, *lstart, *lcount;
};
hipError_t launch_plan_tiles(const int64_t *offsets, int64_t N, int64_t n_atoms, const KnmPlan &p, int64_t max_tiles,
                             int32_t *status, hipStream_t s);
hipError_t launch_knm(KnmArgs a, int64_t max_tiles, hipStream_t s);
// Derivative observation rows (forces, virials): with the tile plan built over the
// observations' positions, row o of out is sum_p w_p zeta sw2 D(i(p), j) (x'_{g(p)} . x_j),
// divided by sigma[o].  a.X holds the gradients, a.zeta the kernel exponent.
hipError_t launch_kdm(KnmArgs a, int64_t max_tiles, hipStream_t s);
// The K_NM of n fits as grouped launches (up to KNM_GROUP fits per launch, the
// table passed as the kernel argument); each fit's tiles compute exactly what
// launch_knm computes for it.
constexpr int KNM_GROUP = 16;
struct KnmGroup {
    int n;
    int64_t base[KNM_GROUP + 1];  // first workgroup of each fit (multiples of 8)
    KnmArgs f[KNM_GROUP];
};
hipError_t launch_knm_group(const KnmArgs *fits, const int64_t *max_tiles, int n, hipStream_t s);

// ------------------------------------------------- low-precision K_NM (mixed form)
// Descriptors rounded to BF16 or FP16 (round to nearest, ties to even) into
// rows of knm_lp_dpad(d) elements, zero-padded.
int knm_lp_dpad(int d);
hipError_t launch_convert_lp(const double *x, int64_t rows, int d, uint16_t *out, bool bf16, hipStream_t s);
struct KnmLpLaunch {
    const uint16_t *X, *XM;     // rounded descriptors [n_atoms x dpad], sparse points [M x dpad]
    int d;
    const int64_t *offsets;     // CSR offsets and the tile plan of the FP64 build
    const int32_t *tile_start, *cfg_list, *n_tiles_dev;
    int64_t max_tiles;
    int64_t M;
    int zeta;
    double sw2;
    const double *sigma;        // [N]: rows divided by sigma
    float *out;                 // FP32 column-major: out[col * ldo + configuration]
    int64_t ldo;
    bool bf16;                  // BF16 (true) or FP16 MFMA
};
hipError_t launch_knm_lp(const KnmLpLaunch &l, hipStream_t s);

// ------------------------------------------ FP64-accurate K_NM on INT8 MFMA
// Descriptor rows split into knm_oz_slices() signed 8-bit slices of
// knm_oz_dpad(d) bytes per row (slice-major: slice t of row r at
// out + (t * rows + r) * dpad) and one exponent per row.
int knm_oz_dpad(int d);
int knm_oz_slices();
hipError_t launch_oz_split(const double *x, int64_t rows, int d, int8_t *out, int32_t *ex, hipStream_t s);
struct KnmOzLaunch {
    const int8_t *X, *XM;       // slices of the descriptors [n_atoms rows] and sparse points [M rows]
    const int32_t *xe, *xme;    // their row exponents
    int64_t n_atoms;
    int d;
    const int64_t *offsets;     // CSR offsets and the tile plan of the FP64 build
    const int32_t *tile_start, *cfg_list, *n_tiles_dev;
    int64_t max_tiles;
    int64_t M;
    int zeta;
    double sw2;
    const double *sigma;        // [N]: rows divided by sigma
    double *out;                // FP64 column-major: out[col * ldo + configuration]
    int64_t ldo;
};
hipError_t launch_knm_oz(const KnmOzLaunch &l, hipStream_t s);
// --------------------------------------------------------------------- predict
// Configurations whose offsets are not a range inside [0, n_atoms) (or offsets[0] != 0,
// offsets[N] != n_atoms) get NaN energies and DST_EINVAL in *status (when non-null);
// no descriptor outside [0, n_atoms) is read.
hipError_t launch_predict(const double *X, int64_t n_atoms, const int64_t *offsets, int64_t N,
                          const double *XM, int64_t M, int d, int zeta, double sw2, const double *c,
                          double *y, int32_t *status, hipStream_t s);

}  // namespace gap
