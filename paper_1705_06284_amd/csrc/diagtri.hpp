// diagtri.hpp -- launchers of the diagonal-binned trispectrum's elementwise
// steps and shell sums (internal to libbispec; diagtri.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "general.hpp"

namespace bispec {

// One shell sum: the modes idx[off .. off + len) (linear indices of the full
// grid), operands xa and xb (array indices: base + xa * stride), and for the
// |D|^4 sums the diagonal thresholds elo <= q < ehi.
struct DtTask {
    int off, len, xa, xb;
    long long elo, ehi;
};

hipError_t dt_mul_f32(const float *a, const float *b, float *out, int64_t n, hipStream_t st);
hipError_t dt_mul_f64(const double *a, const double *b, double *out, int64_t n, hipStream_t st);
// out = |spec|^2 (imaginary parts zero)
hipError_t dt_power(const float2 *spec, float2 *out, int64_t n, hipStream_t st);
// cnt = rint(Re spec / npix); *bad |= 1 if a residual exceeds 0.01
hipError_t dt_round_counts(const double2 *spec, double *cnt, int64_t n, double npix, unsigned int *bad,
                           hipStream_t st);
// out[t] for t < ntask, fixed-order FP64 sums over nblk blocks per task:
// mode 0 Re(x conj y) of FP32 complex arrays, 1 x y of FP64 arrays, 2 Re x;
// partial holds ntask * nblk doubles.
hipError_t dt_shell_sums(int mode, const void *base, int64_t stride, const int *idx, const DtTask *tasks, int ntask,
                         int nblk, double *partial, double *out, hipStream_t st);
// out[t] = sum_{k in task t's shell, 2k in [elo, ehi)} |spec(k)|^4
hipError_t dt_pow4_sums(const float2 *spec, const GenGrid &g, const int *idx, const DtTask *tasks, int ntask,
                        int nblk, double *partial, double *out, hipStream_t st);
// Td = coef[t] sums[t]; Tdc = coef[t] (sums[t] - npix coef[n+t] sums[n+t]
// + npix^2 coef[2n+t] sums[2n+t]) when Tdc is not null.
hipError_t dt_finalize(const double *sums, const double *coef, int n, double npix, double *Td, double *Tdc,
                       hipStream_t st);

}  // namespace bispec
