// general.hpp -- host launchers of the transforms on grids that are not cubic
// powers of two (internal to libbispec; general.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bispec {

// Largest prime factor outside 2, 3, 5 an axis may have (one per axis; its
// pass is a direct DFT of that length).
constexpr int GEN_MAX_PRIME = 127;
constexpr int GEN_MAX_RADICES = 16;

// One axis: length n = product of radix[0 .. nrad), twiddles W_n^j (j < n) at
// tw_off of the twiddle table.
struct GenAxis {
    int n, nrad, tw_off, pad;
    int radix[GEN_MAX_RADICES];
};

// Grid N_z x N_y x N_x (axes ax[0] = z, ax[1] = y, ax[2] = x), q scales
// s_i = P / N_i, and npix = N_z N_y N_x.
struct GenGrid {
    GenAxis ax[3];
    int nz, ny, nx, pad;
    long long sz, sy, sx;
    long long npix;
};

// Membership thresholds of a shell pair: mode m is in bin b1 iff
// lo1 <= q < hi1 (lo2 = hi2 = 0 for a lone bin).
struct GenPair {
    long long lo1, hi1, lo2, hi2;
};

// Radices of an axis of length n (8, 4, 2, 3, 5 first, then at most one
// prime <= GEN_MAX_PRIME); false if n has another factor.
bool gen_factor(int n, GenAxis &ax);
// Pencils per block of the axis kernels.
int gen_pencils(int n, size_t elem_bytes);

hipError_t gen_mean(const float *x, const GenGrid &g, int batch, double *part, int nparts, double *mean,
                    hipStream_t st);
// Forward transform of batch maps [batch][npix] (mean subtracted, then
// multiplied by scale, a power of two) into the full complex spectra
// [batch][npix]; tw: the three axis tables.
hipError_t gen_forward(const float *delta, const double *mean, const GenGrid &g, int batch, const float2 *tw,
                       float2 *spec, hipStream_t st, double scale);
// The same in FP64 for one real map x [npix] (no mean, no scale).
hipError_t gen_forward_f64(const double *x, const GenGrid &g, const double2 *tw, double2 *spec, hipStream_t st);
// Inverse transform of one shell pair: work [batch][npix] complex scratch;
// fields F_b1 to f1 and F_b2 to f2 (may be null), map m at m * map_stride.
hipError_t gen_inverse_pair(const float2 *spec, float2 *work, const GenGrid &g, const GenPair &pr, int batch,
                            const float2 *tw, float *f1, float *f2, int64_t map_stride, hipStream_t st);
// Unit-amplitude (count) fields of one pair in FP64 (one map).
hipError_t gen_inverse_unit_f64(double2 *work, const GenGrid &g, const GenPair &pr, const double2 *tw, double *f1,
                                double *f2, hipStream_t st);
hipError_t gen_zero_pads_f32(float *fields, int64_t npix, int64_t stride, int nfields, hipStream_t st);
hipError_t gen_zero_pads_f64(double *fields, int64_t npix, int64_t stride, int nfields, hipStream_t st);
hipError_t gen_shell_hist(const GenGrid &g, int nb, const long long *qlo, const long long *qhi,
                          unsigned long long *counts, hipStream_t st);

}  // namespace bispec
