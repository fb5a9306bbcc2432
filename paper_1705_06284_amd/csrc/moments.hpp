// moments.hpp -- host launchers of the per-shell spectral moments and the
// connected collapsed trispectrum (internal to libbispec; kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bispec {

// X_b = sum |Delta|^2 and Y_b = sum |Delta|^4 over shell b of each map's half
// spectrum spec [batch][spec_stride] (rows padded as spec_elems lays them
// out); thr [2 nb] holds the integer thresholds lo2 then hi2 (a mode is in
// shell b iff lo2 <= |m|^2 < hi2, m != 0).  Writes block partials
// partial [batch][nblk][nb][2] for launch_reduce_dense (n_dense = 2 nb).
hipError_t launch_shell_moments(const float2 *spec, int64_t spec_stride, int n, int nb, int batch, const int *thr,
                                int nblk, double *partial, hipStream_t st);

// Tc [batch][nq] = T - scale N_pix S_D per collapsed quad (quads: the plan's
// [nq] quad terms, any order of (a,a,b,b)); mom [batch][nb][2] = (X, Y).
hipError_t launch_trispec_connected(const double *T, const double *mom, const uchar4 *quads, const double *scale,
                                    double npix, int nq, int nb, int batch, double *Tc, hipStream_t st);

}  // namespace bispec
