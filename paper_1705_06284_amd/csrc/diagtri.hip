// diagtri.hip -- the diagonal-binned trispectrum (gfx950).
//
// Four shells leave the quadrilateral k1 + k2 + k3 + k4 = 0 free to fold
// along the diagonal q = k1 + k2 = -(k3 + k4); binning |q| as well fixes its
// shape (Section 2, Eq. Jeong_gen with p = 4).  With the pair-product field
// Pi_ab(x) = F_a(x) F_b(x) and its DFT Pi_ab^(q) = N_pix sum_{k1 + k2 = q}
// D(k1) D(k2) (k1 in S_a, k2 in S_b), the sum over closed quadruples whose
// diagonal lies in shell e is
//
//     S(a,b,c,d; e) = N_pix^-2 sum_{q in S_e} Pi_ab^(q) conj(Pi_cd^(q)),
//
// a dot product over the modes of one shell (the fields are real, so
// Pi_cd^(-q) = conj Pi_cd^(q)).  The counts use the unit fields I_b in FP64,
// whose pair products transform to integer pair counts C_ab(q) N_pix.
// The Gaussian pairings of Wick's theorem that survive a diagonal q != 0 are
// k3 = -k1, k4 = -k2 (shells a = c, b = d) and k4 = -k1, k3 = -k2 (a = d,
// b = c), both over pairs (k1, k2) with k1 + k2 in S_e, each
//     S2(a,b; e) = N_pix^-1 sum_{q in S_e} U_ab^(q),
// U_ab = U_a U_b with U_b the inverse transform of |D|^2 on S_b; they share
// the quadruples (k, k, -k, -k), S4(a; e) = sum_{k in S_a, 2k in S_e} |D(k)|^4.
// The kernels here are the elementwise steps and the shell sums; the
// transforms are those of the mixed-radix path (general.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "diagtri.hpp"

namespace bispec {

namespace {

constexpr int DT_NT = 256;

__device__ __forceinline__ double dt_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order block sum of one value per thread (DT_NT threads).
__device__ __forceinline__ double dt_block_sum(double v) {
    __shared__ double red[DT_NT / 64];
    v = dt_wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < DT_NT / 64; ++w) s += red[w];
    return s;
}

template <typename T>
__global__ __launch_bounds__(DT_NT) void k_dt_mul(const T *__restrict__ a, const T *__restrict__ b,
                                                  T *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * DT_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT_NT)
        out[i] = a[i] * b[i];
}

__global__ __launch_bounds__(DT_NT) void k_dt_power(const float2 *__restrict__ spec, float2 *__restrict__ out,
                                                    int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * DT_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT_NT) {
        const float2 v = spec[i];
        out[i] = float2{v.x * v.x + v.y * v.y, 0.0f};
    }
}

// cnt = rint(Re s / N_pix); flags a residual above 0.01 in the real or
// imaginary part (the FP64 transform no longer resolves single counts).
__global__ __launch_bounds__(DT_NT) void k_dt_round(const double2 *__restrict__ spec, double *__restrict__ cnt,
                                                    int64_t n, double inv, unsigned int *__restrict__ bad) {
    bool off = false;
    for (int64_t i = (int64_t)blockIdx.x * DT_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT_NT) {
        const double c = spec[i].x * inv, r = rint(c);
        cnt[i] = r;
        off = off || fabs(c - r) > 0.01 || fabs(spec[i].y * inv) > 0.01;
    }
    if (__any(off) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// partial[t][blk] = sum over the modes idx[off_t .. off_t + len_t) of
// MODE 0: Re(x conj y) (FP32 complex spectra), 1: x y (FP64 counts),
// 2: Re x (FP32 complex), with x = base + xa_t stride, y = base + xb_t stride.
template <int MODE>
__global__ __launch_bounds__(DT_NT) void k_dt_shell_sum(const void *__restrict__ base, int64_t stride,
                                                        const int *__restrict__ idx, const DtTask *__restrict__ tasks,
                                                        double *__restrict__ partial) {
    const DtTask tk = tasks[blockIdx.y];
    double v = 0.0;
    for (int i = blockIdx.x * DT_NT + threadIdx.x; i < tk.len; i += gridDim.x * DT_NT) {
        const int64_t m = idx[tk.off + i];
        if constexpr (MODE == 1) {
            const double *p = reinterpret_cast<const double *>(base);
            v += p[tk.xa * stride + m] * p[tk.xb * stride + m];
        } else {
            const float2 *p = reinterpret_cast<const float2 *>(base);
            const float2 x = p[tk.xa * stride + m];
            if constexpr (MODE == 0) {
                const float2 y = p[tk.xb * stride + m];
                v += (double)x.x * y.x + (double)x.y * y.y;
            } else {
                v += (double)x.x;
            }
        }
    }
    const double s = dt_block_sum(v);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// partial[t][blk] = sum over the modes k of shell a (idx segment of task t)
// with 2k, reduced modulo the grid, in [elo, ehi): |D(k)|^4.
__global__ __launch_bounds__(DT_NT) void k_dt_pow4(const float2 *__restrict__ spec, GenGrid g,
                                                   const int *__restrict__ idx, const DtTask *__restrict__ tasks,
                                                   double *__restrict__ partial) {
    const DtTask tk = tasks[blockIdx.y];
    double v = 0.0;
    auto fq = [](int i, int n) { return i < n - n / 2 ? i : i - n; };
    auto red = [](long long c, int n) {            // c mod n into the signed frequency range
        long long r = ((c % n) + n) % n;
        return r < n - n / 2 ? r : r - n;
    };
    for (int i = blockIdx.x * DT_NT + threadIdx.x; i < tk.len; i += gridDim.x * DT_NT) {
        const int64_t m = idx[tk.off + i];
        const int x = (int)(m % g.nx), y = (int)((m / g.nx) % g.ny), z = (int)(m / ((int64_t)g.nx * g.ny));
        const long long qz = g.sz * red(2LL * fq(z, g.nz), g.nz), qy = g.sy * red(2LL * fq(y, g.ny), g.ny),
                        qx = g.sx * red(2LL * fq(x, g.nx), g.nx);
        const long long q = qz * qz + qy * qy + qx * qx;
        if (q > 0 && q >= tk.elo && q < tk.ehi) {
            const float2 d = spec[m];
            const double a = (double)d.x * d.x + (double)d.y * d.y;
            v += a * a;
        }
    }
    const double s = dt_block_sum(v);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// out[t] = sum_blk partial[t][blk] in block order (one block per task).
__global__ __launch_bounds__(DT_NT) void k_dt_reduce(const double *__restrict__ partial, int nblk,
                                                     double *__restrict__ out) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += DT_NT) v += partial[(int64_t)blockIdx.x * nblk + i];
    const double s = dt_block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Td[t] = scale_t P_t; Tdc[t] = scale_t (P_t - N_pix c2_t U_t + N_pix^2 c4_t Q_t)
// (sums[0..n) P, [n..2n) U, [2n..3n) Q; U and Q read only when Tdc is set).
__global__ __launch_bounds__(DT_NT) void k_dt_finalize(const double *__restrict__ sums,
                                                       const double *__restrict__ coef, int n, double npix,
                                                       double *__restrict__ Td, double *__restrict__ Tdc) {
    const int t = blockIdx.x * DT_NT + threadIdx.x;
    if (t >= n) return;
    const double scale = coef[t], c2 = coef[n + t], c4 = coef[2 * n + t];
    const double p = sums[t];
    Td[t] = scale * p;
    if (Tdc) {
        double g = 0.0;
        if (c2 != 0.0) g += npix * c2 * sums[n + t];
        if (c4 != 0.0) g -= npix * npix * c4 * sums[2 * n + t];
        Tdc[t] = scale * (p - g);
    }
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + DT_NT - 1) / DT_NT;
    return (unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

hipError_t dt_mul_f32(const float *a, const float *b, float *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_dt_mul<float>, dim3(grid_for(n)), dim3(DT_NT), 0, st, a, b, out, n);
    return hipGetLastError();
}

hipError_t dt_mul_f64(const double *a, const double *b, double *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_dt_mul<double>, dim3(grid_for(n)), dim3(DT_NT), 0, st, a, b, out, n);
    return hipGetLastError();
}

hipError_t dt_power(const float2 *spec, float2 *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_dt_power, dim3(grid_for(n)), dim3(DT_NT), 0, st, spec, out, n);
    return hipGetLastError();
}

hipError_t dt_round_counts(const double2 *spec, double *cnt, int64_t n, double npix, unsigned int *bad,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_dt_round, dim3(grid_for(n)), dim3(DT_NT), 0, st, spec, cnt, n, 1.0 / npix, bad);
    return hipGetLastError();
}

hipError_t dt_shell_sums(int mode, const void *base, int64_t stride, const int *idx, const DtTask *tasks, int ntask,
                         int nblk, double *partial, double *out, hipStream_t st) {
    if (ntask < 1) return hipSuccess;
    if (nblk < 1 || mode < 0 || mode > 2) return hipErrorInvalidValue;
    const dim3 grid(nblk, ntask);
    if (mode == 0)
        hipLaunchKernelGGL(k_dt_shell_sum<0>, grid, dim3(DT_NT), 0, st, base, stride, idx, tasks, partial);
    else if (mode == 1)
        hipLaunchKernelGGL(k_dt_shell_sum<1>, grid, dim3(DT_NT), 0, st, base, stride, idx, tasks, partial);
    else
        hipLaunchKernelGGL(k_dt_shell_sum<2>, grid, dim3(DT_NT), 0, st, base, stride, idx, tasks, partial);
    hipLaunchKernelGGL(k_dt_reduce, dim3(ntask), dim3(DT_NT), 0, st, partial, nblk, out);
    return hipGetLastError();
}

hipError_t dt_pow4_sums(const float2 *spec, const GenGrid &g, const int *idx, const DtTask *tasks, int ntask,
                        int nblk, double *partial, double *out, hipStream_t st) {
    if (ntask < 1) return hipSuccess;
    hipLaunchKernelGGL(k_dt_pow4, dim3(nblk, ntask), dim3(DT_NT), 0, st, spec, g, idx, tasks, partial);
    hipLaunchKernelGGL(k_dt_reduce, dim3(ntask), dim3(DT_NT), 0, st, partial, nblk, out);
    return hipGetLastError();
}

hipError_t dt_finalize(const double *sums, const double *coef, int n, double npix, double *Td, double *Tdc,
                       hipStream_t st) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_dt_finalize, dim3((n + DT_NT - 1) / DT_NT), dim3(DT_NT), 0, st, sums, coef, n, npix, Td,
                       Tdc);
    return hipGetLastError();
}

}  // namespace bispec
