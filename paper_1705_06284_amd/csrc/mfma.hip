// mfma.hip -- all-triplet contraction as an MFMA product-Gram (gfx950).
//
// The bispectrum numerators of Eq. (Jeong_BI), sum_n F_i F_j F_k for every
// i <= j <= k, are the entries of the product-Gram matrix
//
//     G[(i,j), k] = sum_n (F_i F_j)(n) F_k(n),
//
// a GEMM whose reduction dimension is the grid.  Rows are the pair products
// (i,j), i <= j < nb, followed by rows (b, ONE) whose product is F_b itself,
// so that G[(b, ONE), b] = sum_n F_b^2 gives the power-spectrum numerator of
// Eq. (Jeong_PS).  Columns are the bin fields F_k, k < 32.  An optional extra
// tile holds the collapsed p = 4 numerators sum_n F_a^2 F_b^2 (rows F_a^2,
// columns F_b^2).
//
// MODE_SPLIT: each FP32 operand x is split into x_hi = bf16_rne(x) and
// x_lo = bf16_rne(x - x_hi) (the difference is exact in FP32); the product
// is A_hi B_hi + A_hi B_lo + A_lo B_hi on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation.  MODE_F32: the same GEMM on v_mfma_f32_32x32x2f32.
// In both modes the FP32 accumulators are flushed into FP64 registers every
// 4096 grid points, and every block writes its FP64 tile partials; a
// fixed-order FP64 reduction over blocks follows (k_finalize_gather).
//
// Lane layouts (checked on the device): for the 32x32x16 bf16 operation lane
// l holds A[l%32][8(l/32)+j] and B[8(l/32)+j][l%32], j < 8; for 32x32x2 f32
// lane l holds A[l%32][l/32] and B[l/32][l%32]; both write
// C[8(r/4)+4(l/32)+r%4][l%32] to accumulator register r.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace bispec {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int PG_TK = 256;                // grid points per LDS tile
constexpr int PG_THREADS = 512;           // 8 waves
constexpr int PG_WAVES = PG_THREADS / 64;
constexpr int PG_MAXT = 3;                // output tiles per wave
constexpr int PG_FLUSH = 16;              // LDS tiles between FP64 flushes (4096 points)
constexpr int PG_FS = PG_TK + 4;          // LDS row stride of a field, floats
constexpr int PG_BS = PG_TK + 8;          // LDS row stride of a bf16 operand row
constexpr int PG_ZERO = PG_ROW_ZERO;      // field row of zeros (padding rows)
constexpr int PG_ONE = PG_ROW_ONE;        // field row of ones (F_b * 1 rows)
constexpr int PG_FROWS = 34;

__device__ __forceinline__ void split2(float x0, float x1, bf16x2 &h, bf16x2 &l) {
    const f32x2 v = {x0, x1};
    h = __builtin_convertvector(v, bf16x2);
    const f32x2 hf = __builtin_convertvector(h, f32x2);
    l = __builtin_convertvector(v - hf, bf16x2);
}

__device__ __forceinline__ void split8(const float *x, bf16x8 &h, bf16x8 &l) {
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        bf16x2 hh, ll;
        split2(x[j], x[j + 1], hh, ll);
        h[j] = hh[0];
        h[j + 1] = hh[1];
        l[j] = ll[0];
        l[j + 1] = ll[1];
    }
}

template <int MODE, bool WANT_T>
__global__ __launch_bounds__(PG_THREADS) void k_pgram(const float *__restrict__ fields, int64_t npix, int nb,
                                                      int64_t map_stride, const uchar2 *__restrict__ pairs,
                                                      int n_mtile, int64_t chunk, double *__restrict__ partial) {
    __shared__ float Ft[PG_FROWS * PG_FS];
    constexpr int BSZ = MODE == PG_MODE_SPLIT ? 32 * PG_BS : 1;
    constexpr int QSZ = (MODE == PG_MODE_SPLIT && WANT_T) ? 32 * PG_BS : 1;
    __shared__ __bf16 Bh[BSZ], Bl[BSZ], Qh[QSZ], Ql[QSZ];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 31, half = lane >> 5;
    const int map = blockIdx.y;
    const float *f = fields + map * map_stride;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = p_begin + chunk < npix ? p_begin + chunk : npix;
    const int n_out = n_mtile + (WANT_T ? 1 : 0);

    int tile_of[PG_MAXT];
    uchar2 rp[PG_MAXT];
#pragma unroll
    for (int t = 0; t < PG_MAXT; ++t) {
        const int tile = wave + t * PG_WAVES;
        tile_of[t] = tile < n_out ? tile : -1;
        if (tile < n_mtile) rp[t] = pairs[tile * 32 + col];
        else rp[t] = uchar2{(unsigned char)(col < nb ? col : PG_ZERO), (unsigned char)(col < nb ? col : PG_ZERO)};
    }
    f32x16 acc[PG_MAXT];
    double dacc[PG_MAXT][16];
#pragma unroll
    for (int t = 0; t < PG_MAXT; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc[t][r] = 0.0f;
            dacc[t][r] = 0.0;
        }
    }
    // rows nb..31 and the zero row stay 0, the ONE row stays 1
    for (int e = tid; e < (PG_FROWS - nb) * PG_FS; e += PG_THREADS) {
        const int row = nb + e / PG_FS;
        Ft[row * PG_FS + e % PG_FS] = row == PG_ONE ? 1.0f : 0.0f;
    }

    int since_flush = 0;
    for (int64_t p = p_begin; p < p_end; p += PG_TK) {
        __syncthreads();
        for (int e = tid; e < nb * (PG_TK / 4); e += PG_THREADS) {
            const int b = e / (PG_TK / 4), q = e % (PG_TK / 4);
            const float4 v = *reinterpret_cast<const float4 *>(f + (int64_t)b * npix + p + 4 * q);
            *reinterpret_cast<float4 *>(&Ft[b * PG_FS + 4 * q]) = v;
        }
        __syncthreads();
        if constexpr (MODE == PG_MODE_SPLIT) {
            for (int e = tid; e < 32 * (PG_TK / 2); e += PG_THREADS) {
                const int c = e / (PG_TK / 2), q = 2 * (e % (PG_TK / 2));
                const float x0 = Ft[c * PG_FS + q], x1 = Ft[c * PG_FS + q + 1];
                bf16x2 h, l;
                split2(x0, x1, h, l);
                *reinterpret_cast<bf16x2 *>(&Bh[c * PG_BS + q]) = h;
                *reinterpret_cast<bf16x2 *>(&Bl[c * PG_BS + q]) = l;
                if constexpr (WANT_T) {
                    split2(x0 * x0, x1 * x1, h, l);
                    *reinterpret_cast<bf16x2 *>(&Qh[c * PG_BS + q]) = h;
                    *reinterpret_cast<bf16x2 *>(&Ql[c * PG_BS + q]) = l;
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int s = 0; s < PG_TK / 16; ++s) {
                const int kp = s * 16 + half * 8;
                const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&Bh[col * PG_BS + kp]);
                const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&Bl[col * PG_BS + kp]);
#pragma unroll
                for (int t = 0; t < PG_MAXT; ++t) {
                    if (tile_of[t] < 0) continue;
                    const bool tq = WANT_T && tile_of[t] == n_mtile;
                    const float4 i0 = *reinterpret_cast<const float4 *>(&Ft[rp[t].x * PG_FS + kp]);
                    const float4 i1 = *reinterpret_cast<const float4 *>(&Ft[rp[t].x * PG_FS + kp + 4]);
                    const float4 j0 = *reinterpret_cast<const float4 *>(&Ft[rp[t].y * PG_FS + kp]);
                    const float4 j1 = *reinterpret_cast<const float4 *>(&Ft[rp[t].y * PG_FS + kp + 4]);
                    float a[8] = {i0.x * j0.x, i0.y * j0.y, i0.z * j0.z, i0.w * j0.w,
                                  i1.x * j1.x, i1.y * j1.y, i1.z * j1.z, i1.w * j1.w};
                    bf16x8 ah, al;
                    split8(a, ah, al);
                    bf16x8 uh = bh, ul = bl;
                    if (tq) {
                        uh = *reinterpret_cast<const bf16x8 *>(&Qh[col * PG_BS + kp]);
                        ul = *reinterpret_cast<const bf16x8 *>(&Ql[col * PG_BS + kp]);
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, uh, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, ul, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, uh, acc[t], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 1
            for (int s = 0; s < PG_TK / 2; ++s) {
                const int k = 2 * s + half;
                const float bk = Ft[(col < nb ? col : PG_ZERO) * PG_FS + k];
#pragma unroll
                for (int t = 0; t < PG_MAXT; ++t) {
                    if (tile_of[t] < 0) continue;
                    const bool tq = WANT_T && tile_of[t] == n_mtile;
                    const float a = Ft[rp[t].x * PG_FS + k] * Ft[rp[t].y * PG_FS + k];
                    const float b = tq ? bk * bk : bk;
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        if (++since_flush == PG_FLUSH) {
            since_flush = 0;
#pragma unroll
            for (int t = 0; t < PG_MAXT; ++t) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    dacc[t][r] += (double)acc[t][r];
                    acc[t][r] = 0.0f;
                }
            }
        }
    }
    const int64_t blk = (int64_t)map * gridDim.x + blockIdx.x;
#pragma unroll
    for (int t = 0; t < PG_MAXT; ++t) {
        if (tile_of[t] < 0) continue;
        double *out = partial + (blk * n_out + tile_of[t]) * 1024;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * half + (r & 3);
            out[row * 32 + col] = dacc[t][r] + (double)acc[t][r];
        }
    }
}

// Fixed-order FP64 sum over blocks of the dense tile partials, gathered at
// idx[t] and scaled: segment layout as in k_finalize.
__global__ __launch_bounds__(256) void k_finalize_gather(const double *__restrict__ partial, int nblk,
                                                         int64_t blk_stride, const int *__restrict__ idx, int nterm,
                                                         const double *__restrict__ scale, double *o0, int n0,
                                                         double *o1, int n1, double *o2, int n2) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int map = blockIdx.y;
    if (t >= nterm) return;
    const double *p = partial + (int64_t)map * nblk * blk_stride + idx[t];
    double acc = 0.0, comp = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double x = p[(int64_t)b * blk_stride];
        const double s = acc + x;
        comp += fabs(acc) >= fabs(x) ? (acc - s) + x : (x - s) + acc;
        acc = s;
    }
    const double v = (acc + comp) * scale[t];
    if (t < n0) {
        if (o0) o0[(int64_t)map * n0 + t] = v;
    } else if (t < n0 + n1) {
        if (o1) o1[(int64_t)map * n1 + (t - n0)] = v;
    } else if (t < n0 + n1 + n2) {
        if (o2) o2[(int64_t)map * n2 + (t - n0 - n1)] = v;
    }
}

size_t pgram_partial_doubles(int n_mtile, bool want_t) { return (size_t)(n_mtile + (want_t ? 1 : 0)) * 1024; }

hipError_t launch_pgram(int mode, bool want_t, const float *fields, int64_t npix, int nb, int64_t map_stride,
                        int batch, const uchar2 *pairs, int n_mtile, int nblk, double *partial, hipStream_t st) {
    if (nb > 32 || n_mtile + (want_t ? 1 : 0) > PG_MAXT * PG_WAVES) return hipErrorInvalidValue;
    const int64_t chunk = ((npix + nblk - 1) / nblk + PG_TK - 1) / PG_TK * PG_TK;
    const dim3 grid(nblk, batch), block(PG_THREADS);
    if (mode == PG_MODE_SPLIT) {
        if (want_t)
            hipLaunchKernelGGL((k_pgram<PG_MODE_SPLIT, true>), grid, block, 0, st, fields, npix, nb, map_stride, pairs,
                               n_mtile, chunk, partial);
        else
            hipLaunchKernelGGL((k_pgram<PG_MODE_SPLIT, false>), grid, block, 0, st, fields, npix, nb, map_stride,
                               pairs, n_mtile, chunk, partial);
    } else {
        if (want_t)
            hipLaunchKernelGGL((k_pgram<PG_MODE_F32, true>), grid, block, 0, st, fields, npix, nb, map_stride, pairs,
                               n_mtile, chunk, partial);
        else
            hipLaunchKernelGGL((k_pgram<PG_MODE_F32, false>), grid, block, 0, st, fields, npix, nb, map_stride, pairs,
                               n_mtile, chunk, partial);
    }
    return hipGetLastError();
}

hipError_t launch_finalize_gather(const double *partial, int nblk, int64_t blk_stride, const int *idx, int nterm,
                                  int batch, const double *scale, double *o0, int n0, double *o1, int n1, double *o2,
                                  int n2, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_gather, dim3((nterm + 255) / 256, batch), dim3(256), 0, st, partial, nblk,
                       blk_stride, idx, nterm, scale, o0, n0, o1, n1, o2, n2);
    return hipGetLastError();
}

}  // namespace bispec
