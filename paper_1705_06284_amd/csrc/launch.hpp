// launch.hpp -- host launchers of the estimator kernels (internal to libbispec).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace bispec {

hipError_t launch_mean(const float *x, int n, int batch, double *partial, int nparts, double *mean, hipStream_t st);

// Forward 3D DFT of batch maps (mean subtracted on load, then multiplied by
// scale, a power of two) into the half spectra.
hipError_t launch_forward(const float *delta, const double *mean, int n, int batch, const float2 *tw,
                          float2 *spec, hipStream_t st, double scale);

// Pruned inverse transform (see k_inv_z_prune): passes Z and Y of every pair
// in pd, one launch each, block tables (pair, first column) in ztab / ytab;
// the compact rows land in bc at each pair's boff.  Pass X (launch_inverse_x)
// reads one pair's compact rows (row stride Wp) and writes F_b1 to f1 and
// F_b2 to f2 (f2 may be null).
// Complex entries of one map's half spectrum [N][N][spec_ld<N>()].
int64_t spec_elems(int n);
hipError_t launch_inverse_zy(const float2 *spec, int64_t spec_stride, int n, int batch, const float2 *tw,
                             const PairDev *pd, const int2 *ztab, int nz_blk, const int2 *ytab, int ny_blk,
                             const int *cols, float2 *abox, float2 *bc, hipStream_t st);
hipError_t launch_inverse_x(const float2 *bc, int64_t bc_stride, int n, int batch, const float2 *tw,
                            const PairGeom &g, float *f1, float *f2, int64_t field_stride, hipStream_t st);
// Pass X of every pair in one launch: pair q (reading its compact rows at
// pd[q].boff + map pd[q].bstride) writes F_2q and F_2q+1 (if 2q+1 < nb) of
// fields [batch][nb][N^3].  npairs = ceil(nb / 2).
hipError_t launch_inverse_x_pairs(const float2 *bc, int n, int batch, const float2 *tw, const PairDev *pd, int npairs,
                                  int nb, float *fields, hipStream_t st);
// Unit-amplitude (count) fields I_b of one pair in FP64 (one map).
hipError_t launch_inverse_unit_f64(int n, const double2 *tw, const PairDev *pd, const PairGeom &g,
                                   const int2 *ztab, int nz_blk, const int2 *ytab, int ny_blk, const int *cols,
                                   double2 *abox, double2 *bc, double *f1, double *f2, hipStream_t st);
// Pencils per block of the FFT kernels (the column-chunk size of the tables).
int fft_pencils_per_block(int n, bool fp64);

hipError_t launch_contract_terms_f32(const float *fields, int64_t npix, int nb, int64_t map_stride, int batch,
                                     const uchar4 *terms, int nterm, int nblk, double *partial, hipStream_t st);
// Ill-conditioned triplets on the vector ALUs (k_refine_terms): FP64 sums
// over FP32 fields [batch][*][fl] (fl a multiple of 4), the products in FP64
// (f64_products) or FP32.
// One launch contracts the slots [slot0, slot0 + refine_slots_per_launch)
// of the slot table (uchar4 (x, y, z, f): staged rows x, y, z; f = 0x80 an
// empty slot, which reads rows 0 and is not written),
// staging the nbs fields bins[0..nbs) (nbs <= refine_rows_bucket(nbs_plan));
// nbs_plan, the most rows any launch of the plan stages, fixes the slots per
// wave.  partial: [batch][nblk][nslot_total] FP64, this launch's slots
// written.
int refine_rows_bucket(int nbs);
int refine_slots_per_wave(int nbs_plan);
int refine_slots_per_launch(int nbs_plan);
hipError_t launch_refine_terms(const float *fields, int64_t fl, int64_t map_stride, int batch, const int *bins,
                               int nbs, int nbs_plan, const uchar4 *slots, int slot0, int nslot_total, int nblk,
                               double *partial, hipStream_t st, bool f64_products);
// out[map][list[i]] = scale[i] src[map][i], i < n, list[i] >= 0 (src [batch][n], out [batch][nout]).
hipError_t launch_scatter_list(const double *src, int n, const int *list, const double *scale, int batch,
                               double *out, int nout, hipStream_t st);
hipError_t launch_contract_terms_f64(const double *fields, int64_t npix, int nb, const uchar4 *terms, int nterm,
                                     int nblk, double *partial, hipStream_t st);

hipError_t launch_finalize(const double *partial, int nblk, int nterm, int batch, const double *scale, double *o0,
                           int n0, double *o1, int n1, double *o2, int n2, hipStream_t st);

// Product-Gram contraction on MFMA (mfma.hip).  pairs: [n_mtile*32] row
// factors (field row indices; 32 = zeros, 33 = ones); column nb < 32 is a
// field of ones.  partial: [batch][nblk][n_mtile + want_t][32][32] FP64.
constexpr int PG_MODE_F32 = 0;
constexpr int PG_MODE_SPLIT = 1;
constexpr int PG_ROW_ZERO = 32;
constexpr int PG_ROW_ONE = 33;
// The fused tail's work is counted in units of 512 grid points
// (tail_units(n) = N^3 / 512 per map); one block contracts at most
// PG_CHUNK_TILES units.
constexpr int PG_CHUNK_TILES = 64;
int64_t tail_units(int n);
size_t pgram_partial_doubles(int n_mtile, bool want_t);
// Fused pass X + product-Gram over the compact rows of all shell pairs.
struct TailPairs {
    int R[16];
    int W[16];              // row stride (Wp) of pair q's compact rows
    long long off[16];      // float2 offset of pair q's compact rows of map 0
    int npairs;
};
// Block shapes of launch_tail (mfma.hip): wide (16 waves, one output tile
// each), deep (8 waves, up to three), twin (8 waves, one tile, 256-point
// tiles, two blocks per CU; N <= 256).  A shape that does not fit the tile
// count falls back to wide, else deep (tail_shape).  nblk blocks per map,
// at least ceil(tail_units(n) / PG_CHUNK_TILES) (else hipErrorInvalidValue).
constexpr int PG_SHAPE_DEEP = 0, PG_SHAPE_WIDE = 1, PG_SHAPE_TWIN = 2;
hipError_t launch_tail(int mode, bool want_t, const float2 *bc, const TailPairs &tp, int n, int nb, int batch,
                       const uchar2 *pairs, int n_mtile, const float2 *tw, int nblk, double *partial,
                       hipStream_t st, int shape);
bool tail_shape_fits(int n, int n_mtile, bool want_t, int shape);
int tail_shape(int n, int n_mtile, bool want_t, int shape);
// K parts per pair tile of the launched shape (summed inside the block:
// each block writes one partial set of n_mtile + want_t tiles).
int tail_ksplit(int n, int n_mtile, bool want_t, int shape);
// Product-Gram over bin fields in HBM (33..128 bins, split-BF16; mfma.hip),
// one group of 64 columns per launch: fields [batch][nb][npix] FP32 (npix:
// the field stride, a multiple of 128; entries beyond the grid are zero);
// columns c < 64 are the fields col0 + c (zero at or beyond nb; col0 a
// multiple of 64 below nb); pairs [n_mtile*32] row factors of the group (field
// rows 0..nb-1, pgf_row_zero(nb) = zeros); partial
// [batch][nblk][tiles_total][32][64] FP64, the launch writing tiles tile0 ..
// tile0 + n_mtile - 1 of every block's set.  nblk blocks per map, each
// contracting pgram_fields_chunk(n, nblk) <= PGF_MAX_CHUNK points (else
// hipErrorInvalidValue).  squares: the product-Gram of the squares (rows
// (a,a), a < nb, n_mtile = pgf_sq_tiles(nb), pairs unused; columns F_b^2 of
// the group and ones at column nb - col0 when that is below 64), with
// pgram_fields_kparts K parts per block, each its own partial set: partial
// [batch][nblk * kparts][tiles_total][32][64].
constexpr int PGF_ROW_ZERO = 64;        // zero row of plans of up to 64 bins
constexpr int PGF_ROW_ZERO_XL = 128;    // and of 65..128 bins
constexpr int PGF_MAX_BINS = 128;
inline int pgf_row_zero(int nb) { return nb <= PGF_ROW_ZERO ? PGF_ROW_ZERO : PGF_ROW_ZERO_XL; }
// Points one block contracts in FP32 accumulation: 512 split-mode MFMA
// steps.  The matrix cores' FP32 accumulation drifts with the length of the
// sum (on one-k_f shells at 256^3, spans of 2048 steps left errors of 5e-5 of
// the noise level on equilateral triplets, 512 steps 2e-5).
constexpr int64_t PGF_MAX_CHUNK = 8192;
int64_t pgram_fields_chunk(int64_t npix, int nblk);
int pgram_fields_kparts(int n_mtile, bool squares);
int pgf_sq_tiles(int nb);               // 1, 2 or 4 row tiles of (a,a)
hipError_t launch_pgram_fields(const float *fields, int64_t npix, int nb, int batch, const uchar2 *pairs, int n_mtile,
                               int col0, int tile0, int tiles_total, int nblk, double *partial, hipStream_t st,
                               bool squares);
// dense[map][e] = sum over the nblk partial sets; tmp holds
// PG_REDUCE_SEGS * n_dense * batch doubles of segment sums (or null: one pass).
constexpr int PG_REDUCE_SEGS = 32;
hipError_t launch_reduce_dense(const double *partial, int nblk, int64_t n_dense, int batch, double *dense,
                               double *tmp, hipStream_t st);
// Terms whose idx carries PG_IDX_ALT read alt (block stride alt_stride) at
// idx & ~PG_IDX_ALT instead of partial: the refinement pass's dense tiles.
constexpr int PG_IDX_ALT = 1 << 30;
hipError_t launch_finalize_gather(const double *partial, int nblk, int64_t blk_stride, const double *alt,
                                  int64_t alt_stride, const int *idx, int nterm, int batch, const double *scale,
                                  double *o0, int n0, double *o1, int n1, double *o2, int n2, hipStream_t st);
// out[map][list[i]] = scale[t] * alt[map][idx[t] & ~PG_IDX_ALT], t = list[i]
// (the refined triplets of the vector-ALU route, written over its values).
hipError_t launch_scatter_alt(const double *alt, int64_t alt_stride, const int *idx, const double *scale,
                              const int *list, int nlist, int batch, double *out, int nout, hipStream_t st);
// FP64 product-Gram over bin fields in HBM (the refinement rows of
// ill-conditioned triplets, any plan of up to 128 bins): same tables, column
// groups and partial layout as launch_pgram_fields, one pair tile per wave,
// nblk blocks of pgram_fields_chunk(n, nblk) points.
hipError_t launch_pgram_fields_f64(const float *fields, int64_t npix, int nb, int batch, const uchar2 *pairs,
                                   int n_mtile, int col0, int tile0, int tiles_total, int nblk, double *partial,
                                   hipStream_t st);

// out[map][g] = sum_{group[t] = g} count[t] B[map][t] / sum count[t] (NaN if empty).
hipError_t launch_rebin(const double *B, int n_tri, const double *count, const int *group, int n_group, int batch,
                        double *out, hipStream_t st);

hipError_t launch_shell_hist(int n, int nb, const int *lo2, const int *hi2, unsigned long long *counts,
                             hipStream_t st);

}  // namespace bispec
