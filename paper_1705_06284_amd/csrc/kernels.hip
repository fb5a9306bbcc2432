// kernels.hip -- HIP kernels of the FFT polyspectrum estimator (gfx950).
//
// Pipeline for one map (Watkinson et al. 2017, Section 2):
//   k_sum_f64 / k_mean_final   FP64 mean of the FP32 input
//   k_fwd_x, k_fft_strided     forward 3D DFT, Eq. (DeltaFFTtoDelta), FP32,
//                              to the half spectrum m_x >= 0
//   k_inv_z_prune              shell masks of two bins fused into the first
//                              inverse pass (Eq. delta_nr): the two real bin
//                              fields come out as the real and imaginary
//                              parts of one complex inverse transform
//   k_inv_y_prune, k_inv_x_pairs, k_inv_x_compact  remaining inverse passes
//                              (up to 32 bins the x pass is fused into the
//                              contraction on the estimate path, mfma.hip;
//                              k_inv_x_pairs writes every bin field to HBM
//                              in one launch, k_inv_x_compact the FP64
//                              count fields of one pair)
//   k_contract_terms           sum_n of products of 2, 3 or 4 bin fields
//                              (numerators and denominators of Eqs. Jeong_PS,
//                              Jeong_BI, Jeong_gen), per-block FP64 partials
//   k_finalize                 fixed-order FP64 cross-block sum and the
//                              normalisation H^p / V over the FFT count
//   k_rebin                    count-weighted averages of B over groups of
//                              triplets (configuration binning)
//   k_shell_hist               modes per shell (wave ballot + popcount)
//   k_shell_moments, k_trispec_connected  per-shell sums of |Delta|^2 and
//                              |Delta|^4, and the collapsed T with its
//                              Gaussian pairings removed
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fft_core.hpp"
#include "launch.hpp"
#include "moments.hpp"

namespace bispec {

// ---------------------------------------------------------------------------
// FP64 mean (block partials, then one block sums them in fixed order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_sum_f64(const float *__restrict__ x, int64_t n,
                                                 int64_t map_stride, double *__restrict__ partial) {
    const float *xm = x + (int64_t)blockIdx.y * map_stride;
    double acc = 0.0, acc2 = 0.0;
    // n = N^3 is a multiple of 512: 16-byte loads, two independent sums
    const float4 *x4 = reinterpret_cast<const float4 *>(xm);
    const int64_t n4 = n / 4;
#pragma unroll 4
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
        const float4 v = x4[i];
        acc += (double)v.x + (double)v.y;
        acc2 += (double)v.z + (double)v.w;
    }
    acc += acc2;
    acc = wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_mean_final(const double *__restrict__ partial, int nparts,
                                                   double inv_n, double *__restrict__ mean) {
    const double *p = partial + (int64_t)blockIdx.x * nparts;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 64) acc += p[i];
    acc = wave_sum(acc);
    if (threadIdx.x == 0) mean[blockIdx.x] = acc * inv_n;
}

// ---------------------------------------------------------------------------
// FFT kernels.  Volumes are [z][y][x] with N^3 entries.
// ---------------------------------------------------------------------------
template <typename C, int N>
__device__ __forceinline__ void load_twiddles(C *tw_s, const C *tw) {
    for (int i = threadIdx.x; i < N; i += 256) tw_s[i] = tw[i];
}

// Forward pass along x: real input minus the FP64 mean, half-spectrum output
// [z][y][m_x = 0..N/2] with row length spec_ld<N>() (pad entries zero).  Two
// real rows a, b share one complex transform Z of a + i b; then
// A(k) = (Z(k) + conj Z(N-k)) / 2 and B(k) = (Z(k) - conj Z(N-k)) / (2i).
template <int N>
__global__ __launch_bounds__(256) void k_fwd_x(const float *__restrict__ delta, const double *__restrict__ mean,
                                               const float2 *__restrict__ tw, float2 *__restrict__ spec,
                                               double scale) {
    constexpr int G0 = pencils_per_block<float, N>();
    constexpr int G = G0 < N * N / 2 ? G0 : N * N / 2;      // complex pencils = 2G real rows
    constexpr int HP = spec_ld<N>();
    constexpr int LD = pencil_ld<N>();
    constexpr int PER = 2 * G * N / 256;
    static_assert((2 * G * N) % 256 == 0, "row pairs must divide the block");
    __shared__ float2 s[G * LD];
    __shared__ float2 tws[N];
    load_twiddles<float2, N>(tws, tw);
    const int64_t vol = (int64_t)N * N * N;
    const int map = blockIdx.y;
    const float *src = delta + map * vol;
    float2 *dst = spec + map * (int64_t)N * N * HP;
    const double mu = mean[map];
    const int64_t row0 = (int64_t)blockIdx.x * 2 * G;
    float x[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) x[k] = src[row0 * N + threadIdx.x + k * 256];   // all loads in flight
    float *sf = reinterpret_cast<float *>(s);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        const int r = e / N, i = e % N;          // real row r of the block: pencil r / 2, part r % 2
        sf[2 * ((r >> 1) * LD + pad_idx(i)) + (r & 1)] = (float)(((double)x[k] - mu) * scale);
    }
    __syncthreads();
    fft_pencils<float2, N, LD, G, -1>(s, tws);
    for (int e = threadIdx.x; e < G * HP; e += 256) {
        const int p = e / HP, k = e % HP;
        float2 a = float2{0.0f, 0.0f}, b = float2{0.0f, 0.0f};
        if (k <= N / 2) {
            const float2 z = s[p * LD + pad_idx(k)];
            const float2 zm = s[p * LD + pad_idx((N - k) & (N - 1))];
            a = float2{0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y)};
            b = float2{0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x)};
        }
        dst[(row0 + 2 * p) * HP + k] = a;
        dst[(row0 + 2 * p + 1) * HP + k] = b;
    }
}

// In-place transform along y (AXIS = 1) or z (AXIS = 2) of a complex volume
// whose rows hold W entries ([z][y][W]; W = spec_ld<N>() for the half
// spectrum).  A block takes G pencils that are adjacent in the row, so every
// load and store instruction touches contiguous runs.
template <typename R, int N, int DIR, int AXIS, int W>
__global__ __launch_bounds__(256) void k_fft_strided(cplx<R> *__restrict__ vol_base, const cplx<R> *__restrict__ tw,
                                                     int64_t map_stride) {
    using C = cplx<R>;
    constexpr int G = pencils_per_block<R, N>();
    static_assert((N * W) % G == 0, "pencil groups must tile the volume");
    __shared__ C s[G * pencil_ld<N>()];
    __shared__ C tws[N];
    load_twiddles<C, N>(tws, tw);
    C *v = vol_base + (int64_t)blockIdx.y * map_stride;
    const int64_t p0 = (int64_t)blockIdx.x * G;   // first pencil (c * W + x)
    const int64_t stride = AXIS == 1 ? W : (int64_t)N * W;
    auto addr = [&](int p, int i) {
        const int64_t pl = p0 + p;
        return AXIS == 1 ? (pl / W) * N * W + i * stride + pl % W : (int64_t)i * stride + pl;
    };
    if constexpr (N >= 16) {
        // loads feed the first radix-8 pass in registers, the last pass stores
        // to memory; tasks run pencil-fastest
        constexpr int NB1 = N / 8, PER1 = G * NB1 / 256;
        static_assert((G * NB1) % 256 == 0, "first-pass tasks must fill the block");
        C x[PER1][8];
#pragma unroll
        for (int k = 0; k < PER1; ++k) {
            const int task = threadIdx.x + k * 256;
#pragma unroll
            for (int t = 0; t < 8; ++t) x[k][t] = v[addr(task % G, task / G + t * NB1)];
        }
#pragma unroll
        for (int k = 0; k < PER1; ++k) {
            const int task = threadIdx.x + k * 256;
            first_pass_butterfly<C, N, pencil_ld<N>(), DIR>(s, task % G, task / G, x[k]);
        }
        __syncthreads();
        fft_pencils_to<C, N, pencil_ld<N>(), G, DIR, 256, true, true>(s, tws, G,
                                                                      [&](int p, int i, C val) { v[addr(p, i)] = val; });
    } else {
        constexpr int PER = G * N / 256;
        C x[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + k * 256;
            x[k] = v[addr(e % G, e / G)];
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + k * 256;
            s[(e % G) * pencil_ld<N>() + pad_idx(e / G)] = x[k];
        }
        __syncthreads();
        fft_pencils<C, N, pencil_ld<N>(), G, DIR>(s, tws);
        for (int e = threadIdx.x; e < G * N; e += 256) v[addr(e % G, e / G)] = s[(e % G) * pencil_ld<N>() + pad_idx(e / G)];
    }
}

// ---------------------------------------------------------------------------
// Pruned inverse transform of a shell pair (b1, b2), Eq. (delta_nr).
//
// Pass Z: only the columns (m_y, m_x) with m_y^2 + m_x^2 < hmax can hold a
// shell mode.  Each such column gathers [m in S_b1] Delta(m) +
// i [m in S_b2] Delta(m) along m_z (the shell masks fused into the load),
// transforms along z and writes the box A[n_z][m_y + R][m_x + R] (W x W per
// z-plane; entries outside the disk are never written nor read).  Since both
// masked spectra are Hermitian the 3D transform is F_b1 + i F_b2.
// UNIT = true sets Delta = 1 (the count fields I_b).
//
// Pass Y: each column (n_z, m_x), |m_x| <= R, gathers A along m_y (zero
// outside the disk), transforms along y and writes the compact rows
// Bc[n_z][n_y][m_x + R].
//
// Pass X (k_inv_x_compact, or fused into the contraction kernel): each row
// (n_z, n_y) places Bc at m_x mod N, transforms along x, and the real and
// imaginary parts are F_b1 and F_b2.
// ---------------------------------------------------------------------------
// One launch covers every pair: block b reads (pair q, first column c0) from
// the block table, so small and large pairs share the machine.
template <typename R, int N, bool UNIT>
__global__ __launch_bounds__(256) void k_inv_z_prune(const cplx<R> *__restrict__ spec, int64_t spec_stride,
                                                     cplx<R> *__restrict__ abox, const PairDev *__restrict__ pd,
                                                     const int2 *__restrict__ ztab, const int *__restrict__ cols,
                                                     const cplx<R> *__restrict__ tw) {
    using C = cplx<R>;
    constexpr int G = pencils_per_block<R, N>();
    __shared__ C s[G * pencil_ld<N>()];
    __shared__ C tws[N];
    load_twiddles<C, N>(tws, tw);
    const int map = blockIdx.y;
    const int2 ent = ztab[blockIdx.x];
    const PairDev P = pd[ent.x];
    const int c0 = ent.y;
    const C *sp = UNIT ? nullptr : spec + map * spec_stride;
    C *o = abox + P.aoff + map * P.astride;
    const int Wp = P.g.Wp, Rr = P.g.R;
    const int *cl = cols + P.col_off;
    constexpr int PER = G * N / 256;
    // this thread's column is fixed (p = tid % G since 256 is a multiple of G)
    const int p = threadIdx.x % G;
    const bool live = c0 + p < P.ncols;
    const int box = live ? cl[c0 + p] : 0;           // (m_y + R) * Wp + (m_x + R)
    const int my = box / Wp - Rr, mx = box % Wp - Rr;
    // half spectrum: m_x < 0 is read as conj Delta(-m)
    constexpr int HP = spec_ld<N>();
    const bool neg = mx < 0;
    const int64_t col_addr = neg ? (int64_t)((-my) & (N - 1)) * HP - mx : (int64_t)(my & (N - 1)) * HP + mx;
    const int64_t plane = (int64_t)P.g.W * Wp;
    // the shell masks of the two bins fused into the load: b1 real, b2 imaginary
    auto masked = [&](int i) {
        const int mz = signed_freq(i, N);
        const int r2 = mz * mz + my * my + mx * mx;
        const bool in1 = live && r2 >= P.g.lo1 && r2 < P.g.hi1;
        const bool in2 = live && r2 >= P.g.lo2 && r2 < P.g.hi2;
        C d = C{R(0), R(0)};
        if (in1 || in2) {
            if constexpr (UNIT) {
                d = C{R(1), R(0)};
            } else {
                const int iz = neg ? (N - i) & (N - 1) : i;
                const C v = sp[(int64_t)iz * N * HP + col_addr];
                d = neg ? C{v.x, -v.y} : v;
            }
        }
        const R a1 = in1 ? R(1) : R(0), a2 = in2 ? R(1) : R(0);
        return C{d.x * a1 - d.y * a2, d.y * a1 + d.x * a2};
    };
    if constexpr (N >= 16) {
        // The loads feed the first radix-8 pass in registers and the last pass
        // stores to memory; tasks run pencil-fastest (every task of this
        // thread is on its column p).
        constexpr int NB1 = N / 8, PER1 = G * NB1 / 256;
        static_assert((G * NB1) % 256 == 0, "first-pass tasks must fill the block");
        C v[PER1][8];
#pragma unroll
        for (int k = 0; k < PER1; ++k) {             // all loads in flight first
            const int jj = (threadIdx.x + k * 256) / G;
#pragma unroll
            for (int t = 0; t < 8; ++t) v[k][t] = masked(jj + t * NB1);
        }
#pragma unroll
        for (int k = 0; k < PER1; ++k)
            first_pass_butterfly<C, N, pencil_ld<N>(), +1>(s, p, (threadIdx.x + k * 256) / G, v[k]);
        __syncthreads();
        fft_pencils_to<C, N, pencil_ld<N>(), G, +1, 256, true, true>(s, tws, G, [&](int q, int i, C val) {
            if (c0 + q < P.ncols) o[(int64_t)i * plane + cl[c0 + q]] = val;
        });
    } else {
        C d[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) d[k] = masked((threadIdx.x + k * 256) / G);
#pragma unroll
        for (int k = 0; k < PER; ++k) s[p * pencil_ld<N>() + pad_idx((threadIdx.x + k * 256) / G)] = d[k];
        __syncthreads();
        fft_pencils<C, N, pencil_ld<N>(), G, +1>(s, tws);
        for (int e = threadIdx.x; e < G * N; e += 256) {
            const int q = e % G, i = e / G;
            if (c0 + q < P.ncols) o[(int64_t)i * plane + cl[c0 + q]] = s[q * pencil_ld<N>() + pad_idx(i)];
        }
    }
}

// Columns (n_z, xi) of a pair are numbered c = n_z * Wp + xi; those with
// xi >= W are row padding and are skipped.
template <typename R, int N>
__global__ __launch_bounds__(256) void k_inv_y_prune(const cplx<R> *__restrict__ abox, cplx<R> *__restrict__ bc,
                                                     const PairDev *__restrict__ pd, const int2 *__restrict__ ytab,
                                                     const cplx<R> *__restrict__ tw) {
    using C = cplx<R>;
    constexpr int G = pencils_per_block<R, N>();
    __shared__ C s[G * pencil_ld<N>()];
    __shared__ C tws[N];
    load_twiddles<C, N>(tws, tw);
    const int map = blockIdx.y;
    const int2 ent = ytab[blockIdx.x];
    const PairDev P = pd[ent.x];
    const int c0 = ent.y;
    const C *a = abox + P.aoff + map * P.astride;
    C *o = bc + P.boff + map * P.bstride;
    const int W = P.g.W, Wp = P.g.Wp, Rr = P.g.R;
    const int ncols = N * Wp;
    const int64_t plane = (int64_t)W * Wp;
    if constexpr (N >= 16) {
        // The loads feed the first radix-8 pass in registers and the last pass
        // stores to memory; tasks run pencil-fastest, so consecutive threads
        // touch consecutive columns xi.
        constexpr int NB1 = N / 8, PER1 = G * NB1 / 256;
        static_assert((G * NB1) % 256 == 0, "first-pass tasks must fill the block");
        // this thread's column p = tid % G is the same for all its tasks
        const int p = threadIdx.x % G;
        const int c = c0 + p;
        const int nz = c / Wp, xi = c % Wp;
        const bool live = c < ncols && xi < W;
        const int mx = xi - Rr;
        const C *col = a + (int64_t)nz * plane + xi;
        C v[PER1][8];
#pragma unroll
        for (int k = 0; k < PER1; ++k) {             // all loads in flight first
            const int jj = (threadIdx.x + k * 256) / G;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int my = signed_freq(jj + t * NB1, N);
                v[k][t] = C{R(0), R(0)};
                if (live && my >= -Rr && my <= Rr && my * my + mx * mx < P.g.hmax) v[k][t] = col[(int64_t)(my + Rr) * Wp];
            }
        }
#pragma unroll
        for (int k = 0; k < PER1; ++k)
            first_pass_butterfly<C, N, pencil_ld<N>(), +1>(s, p, (threadIdx.x + k * 256) / G, v[k]);
        __syncthreads();
        // the row padding xi >= W is written too (zeros: no input there), so
        // that every store fills whole 128-byte lines
        fft_pencils_to<C, N, pencil_ld<N>(), G, +1, 256, true, true>(s, tws, G, [&](int p, int i, C val) {
            const int c = c0 + p;
            const int nz = c / Wp, xi = c % Wp;
            if (c < ncols) o[((int64_t)nz * N + i) * Wp + xi] = val;
        });
    } else {
        constexpr int PER = G * N / 256;
        {
            const int p = threadIdx.x % G;               // fixed column of this thread
            const int c = c0 + p;
            const int nz = c / Wp, xi = c % Wp;
            const bool live = c < ncols && xi < W;
            const int mx = xi - Rr;
            const C *col = a + (int64_t)nz * plane + xi;
            C v[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int my = signed_freq((threadIdx.x + k * 256) / G, N);
                v[k] = C{R(0), R(0)};
                if (live && my >= -Rr && my <= Rr && my * my + mx * mx < P.g.hmax) v[k] = col[(int64_t)(my + Rr) * Wp];
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) s[p * pencil_ld<N>() + pad_idx((threadIdx.x + k * 256) / G)] = v[k];
        }
        __syncthreads();
        fft_pencils<C, N, pencil_ld<N>(), G, +1>(s, tws);
        for (int e = threadIdx.x; e < G * N; e += 256) {
            const int p = e % G, i = e / G;
            const int c = c0 + p;
            const int nz = c / Wp, xi = c % Wp;
            if (c < ncols && xi < W) o[((int64_t)nz * N + i) * Wp + xi] = s[p * pencil_ld<N>() + pad_idx(i)];
        }
    }
}

// Pass X over the G rows from row0 of one pair's compact rows src (row
// stride Wp, radius Rr): the real parts go to d1, the imaginary parts to d2
// (or nowhere).
template <typename R, int N>
__device__ __forceinline__ void inv_x_rows(const cplx<R> *__restrict__ src, int Wp, int Rr, int64_t row0,
                                           cplx<R> *s, const cplx<R> *tws, R *__restrict__ d1,
                                           R *__restrict__ d2) {
    using C = cplx<R>;
    constexpr int G = pencils_per_block<R, N>();
    constexpr int PER = G * N / 256;
    C v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        const int p = e / N, mx = signed_freq(e % N, N);
        v[k] = (mx >= -Rr && mx <= Rr) ? src[(row0 + p) * Wp + mx + Rr] : C{R(0), R(0)};
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        s[(e / N) * pencil_ld<N>() + pad_idx(e % N)] = v[k];
    }
    __syncthreads();
    fft_pencils<C, N, pencil_ld<N>(), G, +1>(s, tws);
    for (int e = threadIdx.x; e < G * N; e += 256) d1[row0 * N + e] = s[(e / N) * pencil_ld<N>() + pad_idx(e % N)].x;
    if (d2)
        for (int e = threadIdx.x; e < G * N; e += 256)
            d2[row0 * N + e] = s[(e / N) * pencil_ld<N>() + pad_idx(e % N)].y;
}

// Pass X writing the two bin fields of one pair (the FP64 count fields).
template <typename R, int N>
__global__ __launch_bounds__(256) void k_inv_x_compact(const cplx<R> *__restrict__ bc, int64_t bc_stride,
                                                       PairGeom g, const cplx<R> *__restrict__ tw,
                                                       R *__restrict__ f1, R *__restrict__ f2, int64_t field_stride) {
    using C = cplx<R>;
    constexpr int G = pencils_per_block<R, N>();
    __shared__ C s[G * pencil_ld<N>()];
    __shared__ C tws[N];
    load_twiddles<C, N>(tws, tw);
    const int map = blockIdx.y;
    inv_x_rows<R, N>(bc + map * bc_stride, g.Wp, g.R, (int64_t)blockIdx.x * G, s, tws, f1 + map * field_stride,
                     f2 ? f2 + map * field_stride : nullptr);
}

// Pass X of every pair in one launch (bin_fields, the vector-ALU terms and
// the fields product-Gram): block (x, map, q) transforms rows x G .. x G + G - 1
// of pair q into F_2q and F_2q+1 of fields [batch][nb][N^3].
template <int N>
__global__ __launch_bounds__(256) void k_inv_x_pairs(const float2 *__restrict__ bc, const PairDev *__restrict__ pd,
                                                     const float2 *__restrict__ tw, int nb,
                                                     float *__restrict__ fields) {
    constexpr int G = pencils_per_block<float, N>();
    constexpr int64_t VOL = (int64_t)N * N * N;
    __shared__ float2 s[G * pencil_ld<N>()];
    __shared__ float2 tws[N];
    load_twiddles<float2, N>(tws, tw);
    const int map = blockIdx.y, q = blockIdx.z;
    const PairDev P = pd[q];
    float *f1 = fields + ((int64_t)map * nb + 2 * q) * VOL;
    inv_x_rows<float, N>(bc + P.boff + map * P.bstride, P.g.Wp, P.g.R, (int64_t)blockIdx.x * G, s, tws, f1,
                         2 * q + 1 < nb ? f1 + VOL : nullptr);
}


// ---------------------------------------------------------------------------
// Product sums over the grid: term t multiplies the fields named by the four
// bytes of terms[t] (0xFF = absent).  Block b sums the points
// [b*chunk, (b+1)*chunk) and writes one FP64 partial per term.
// FP32 inputs: products and per-tile (64 point) sums in FP32, then FP64.
// ---------------------------------------------------------------------------
constexpr int CT_TILE = 64;
constexpr int CT_MAXT = 16;   // terms per thread per launch

// Neumaier compensated addition: (s, c) += x.
__device__ __forceinline__ void comp_add(double &s, double &c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// FP32 fields: products and per-tile (64 point) sums in FP32, then FP64.
// FP64 fields (the count fields of the plan): every product is added with
// compensated FP64 summation, so sums of integer-valued count products stay
// exact well beyond 2^53 / N_pix.
template <typename R>
__global__ __launch_bounds__(256) void k_contract_terms(const R *__restrict__ fields, int64_t npix, int nb,
                                                        int64_t map_stride, const uchar4 *__restrict__ terms,
                                                        int t0, int nterm_launch, int nterm_total,
                                                        int64_t chunk, double *__restrict__ partial) {
    constexpr bool F64 = sizeof(R) == 8;
    using P = R;                                   // product and tile-sum type
    extern __shared__ unsigned char smem_raw[];
    R *tile = reinterpret_cast<R *>(smem_raw);   // [CT_TILE][nb]
    const int map = blockIdx.y;
    const R *f = fields + map * map_stride;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = p_begin + chunk < npix ? p_begin + chunk : npix;
    uchar4 my_terms[CT_MAXT];
    double acc[CT_MAXT], comp[CT_MAXT];
    int nmine = 0;
#pragma unroll
    for (int q = 0; q < CT_MAXT; ++q) {
        const int t = threadIdx.x + q * 256;
        acc[q] = 0.0;
        comp[q] = 0.0;
        if (t < nterm_launch) {
            my_terms[q] = terms[t0 + t];
            nmine = q + 1;
        } else {
            my_terms[q] = uchar4{0xFF, 0xFF, 0xFF, 0xFF};
        }
    }
    for (int64_t p = p_begin; p < p_end; p += CT_TILE) {
        const int cnt = (int)((p_end - p) < CT_TILE ? (p_end - p) : CT_TILE);
        __syncthreads();
        for (int e = threadIdx.x; e < CT_TILE * nb; e += 256) {
            const int b = e / CT_TILE, pt = e % CT_TILE;
            tile[pt * nb + b] = pt < cnt ? f[(int64_t)b * npix + p + pt] : R(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CT_MAXT; ++q) {
            if (q >= nmine) break;
            const uchar4 tm = my_terms[q];
            P s = P(0);
            for (int pt = 0; pt < CT_TILE; ++pt) {
                const R *row = tile + pt * nb;
                P v = (P)row[tm.x] * (P)row[tm.y];
                if (tm.z != 0xFF) v *= (P)row[tm.z];
                if (tm.w != 0xFF) v *= (P)row[tm.w];
                if constexpr (F64) comp_add(acc[q], comp[q], v);
                else s += v;
            }
            if constexpr (!F64) acc[q] += (double)s;
            (void)s;
        }
    }
    double *out = partial + ((int64_t)map * gridDim.x + blockIdx.x) * nterm_total + t0;
#pragma unroll
    for (int q = 0; q < CT_MAXT; ++q) {
        const int t = threadIdx.x + q * 256;
        if (t < nterm_launch) out[t] = acc[q] + comp[q];
    }
}

// ---------------------------------------------------------------------------
// Ill-conditioned triplets on the vector ALUs (narrow shells near the
// triangle edge): sum_n F_x F_y F_z with FP64 sums.  F64P: the products are
// formed in FP64 (the pair product of two FP32 values is exact), for plans in
// FP32 mode, whose bar is tighter; otherwise in FP32 with a 4-point FP32 sum
// per lane before the FP64 one: a relative rounding of a few 2^-24 per
// product, far below the 2^-9..2^-17 of the split-BF16 operands the
// refinement replaces, at half the vector-ALU work.
//
// A block of RF_WAVES waves takes a span of grid points in tiles of RF_TP
// points.  The fields the launch reads (bins[r], r < nbs) are staged per
// tile into LDS as rows of RF_TP floats; lane l reads points 4l..4l+3 of a
// row with one 16-byte load, so a wave's reads cover a row without bank
// conflicts.  Wave w owns the slots [w*S, (w+1)*S) of the launch's slot
// table (S = SLOTS), one per lane of a register, read out with v_readlane:
// slot x | y << 8 | z << 16 | f << 24 adds F_x F_y F_z (staged rows) to its
// sum; f = 0x80 marks an empty slot (rows 0, not written).  The slots carry
// no branches, so the loads of later slots overlap the products of earlier
// ones.  Each lane keeps one FP64 running sum per slot over all its points;
// at the end the lanes' sums are added in a fixed order and the block
// writes one FP64 partial per slot, partial[map][block][slot0 + slot].  The
// next tile's global loads are issued into registers before the current
// tile's products.
// ---------------------------------------------------------------------------
constexpr int RF_WAVES = 16;
constexpr int RF_TP = 256;

template <int NBS, int SLOTS, bool F64P>
__global__ __launch_bounds__(RF_WAVES * 64) void k_refine_terms(const float *__restrict__ fields, int64_t fl,
                                                                int64_t map_stride, const int *__restrict__ bins,
                                                                int nbs, const uchar4 *__restrict__ slots, int slot0,
                                                                int nslot_total, int64_t chunk,
                                                                double *__restrict__ partial) {
    constexpr int PF = NBS / RF_WAVES;             // staged rows per wave
    static_assert(SLOTS <= 64, "one slot per lane");
    __shared__ __attribute__((aligned(16))) float tile[NBS * RF_TP];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float *f = fields + (int64_t)blockIdx.y * map_stride;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = p_begin + chunk < fl ? p_begin + chunk : fl;
    const unsigned *tab = reinterpret_cast<const unsigned *>(slots + slot0) + w * SLOTS;
    const unsigned desc = lane < SLOTS ? tab[lane] : 0u;
    float4 pf[PF];
    auto load = [&](int64_t p) {
        const int64_t pt = p + 4 * lane;
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int r = w + RF_WAVES * j;
            if (r < nbs)
                pf[j] = pt < p_end ? *reinterpret_cast<const float4 *>(f + (int64_t)bins[r] * fl + pt)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto row = [&](unsigned r) { return *reinterpret_cast<const float4 *>(&tile[r * RF_TP + 4 * lane]); };
    double acc[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) acc[q] = 0.0;
    if (p_begin < p_end) load(p_begin);
    for (int64_t p = p_begin; p < p_end; p += RF_TP) {
        __syncthreads();                           // the previous tile is read
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int r = w + RF_WAVES * j;
            if (r < nbs) *reinterpret_cast<float4 *>(&tile[r * RF_TP + 4 * lane]) = pf[j];
        }
        __syncthreads();
        if (p + RF_TP < p_end) load(p + RF_TP);
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const unsigned d = __builtin_amdgcn_readlane(desc, q);
            const float4 a = row(d & 0xFF), b = row((d >> 8) & 0xFF), c = row((d >> 16) & 0xFF);
            if constexpr (F64P) {
                acc[q] = fma((double)a.x * (double)b.x, (double)c.x, acc[q]);
                acc[q] = fma((double)a.y * (double)b.y, (double)c.y, acc[q]);
                acc[q] = fma((double)a.z * (double)b.z, (double)c.z, acc[q]);
                acc[q] = fma((double)a.w * (double)b.w, (double)c.w, acc[q]);
            } else {
                float t = (a.x * b.x) * c.x;
                t = fmaf(a.y * b.y, c.y, t);
                t = fmaf(a.z * b.z, c.z, t);
                t = fmaf(a.w * b.w, c.w, t);
                acc[q] += (double)t;
            }
        }
    }
    double *out = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nslot_total + slot0 + w * SLOTS;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0 && !(__builtin_amdgcn_readlane(desc, q) >> 31)) out[q] = v;
    }
}

int refine_rows_bucket(int nbs) { return nbs <= 32 ? 32 : nbs <= 64 ? 64 : 128; }
int refine_slots_per_wave(int nbs) { return refine_rows_bucket(nbs) <= 64 ? 32 : 24; }
int refine_slots_per_launch(int nbs) { return RF_WAVES * refine_slots_per_wave(nbs); }
int64_t refine_chunk(int64_t fl, int nblk) { return ((fl + nblk - 1) / nblk + RF_TP - 1) / RF_TP * RF_TP; }

hipError_t launch_refine_terms(const float *fields, int64_t fl, int64_t map_stride, int batch, const int *bins,
                               int nbs, int nbs_plan, const uchar4 *slots, int slot0, int nslot_total, int nblk,
                               double *partial, hipStream_t st, bool f64_products) {
    const int bucket = refine_rows_bucket(nbs_plan);
    if (fl % 4 || nblk < 1 || nbs < 1 || nbs > bucket || nbs_plan > 128) return hipErrorInvalidValue;
    const int64_t chunk = refine_chunk(fl, nblk);
    const dim3 grid(nblk, batch), block(RF_WAVES * 64);
    auto go = [&](auto f64c) {
        constexpr bool F = decltype(f64c)::value;
        if (bucket == 32)
            hipLaunchKernelGGL((k_refine_terms<32, 32, F>), grid, block, 0, st, fields, fl, map_stride, bins, nbs,
                               slots, slot0, nslot_total, chunk, partial);
        else if (bucket == 64)
            hipLaunchKernelGGL((k_refine_terms<64, 32, F>), grid, block, 0, st, fields, fl, map_stride, bins, nbs,
                               slots, slot0, nslot_total, chunk, partial);
        else
            hipLaunchKernelGGL((k_refine_terms<128, 24, F>), grid, block, 0, st, fields, fl, map_stride, bins, nbs,
                               slots, slot0, nslot_total, chunk, partial);
    };
    if (f64_products) go(std::true_type{});
    else go(std::false_type{});
    return hipGetLastError();
}

// Fixed-order compensated FP64 sum over blocks, then scale: out = scale[t] * sum.
// Terms [0, n0) go to o0, [n0, n0+n1) to o1, [n0+n1, n0+n1+n2) to o2.
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partial, int nblk, int nterm,
                                                  const double *__restrict__ scale, double *o0, int n0,
                                                  double *o1, int n1, double *o2, int n2) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int map = blockIdx.y;
    if (t >= nterm) return;
    const double *p = partial + (int64_t)map * nblk * nterm + t;
    double acc = 0.0, comp = 0.0;
    for (int b = 0; b < nblk; ++b) comp_add(acc, comp, p[(int64_t)b * nterm]);
    const double v = (acc + comp) * scale[t];
    if (t < n0) {
        if (o0) o0[(int64_t)map * n0 + t] = v;
    } else if (t < n0 + n1) {
        if (o1) o1[(int64_t)map * n1 + (t - n0)] = v;
    } else if (t < n0 + n1 + n2) {
        if (o2) o2[(int64_t)map * n2 + (t - n0 - n1)] = v;
    }
}

// Further binning of B over groups of triplets (Section 3: measure in narrow
// shells, then bin the configurations): block (g, map) forms
// sum_{t: group[t] = g} N_t B[map][t] / sum N_t, the estimator of the union of
// the group's closed triangles.  Each thread sums a fixed strided subset, the
// wave and block sums run in a fixed order, so the result is deterministic.
// Triplets with N_t = 0 (B = NaN) contribute nothing; an empty group is NaN.
constexpr int RB_NT = 1024;

__global__ __launch_bounds__(RB_NT) void k_rebin(const double *__restrict__ B, int n_tri,
                                                 const double *__restrict__ count, const int *__restrict__ group,
                                                 int n_group, double *__restrict__ out) {
    const int g = blockIdx.x, map = blockIdx.y;
    const double *b = B + (int64_t)map * n_tri;
    double num = 0.0, den = 0.0;
#pragma unroll 4
    for (int t = threadIdx.x; t < n_tri; t += RB_NT) {
        if (group[t] == g) {
            const double w = count[t];
            if (w > 0.0) {
                num += w * b[t];
                den += w;
            }
        }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    __shared__ double red[2][RB_NT / 64];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = num;
        red[1][threadIdx.x >> 6] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sn = 0.0, sd = 0.0;
        for (int w = 0; w < RB_NT / 64; ++w) {
            sn += red[0][w];
            sd += red[1][w];
        }
        out[(int64_t)map * n_group + g] = sd > 0.0 ? sn / sd : __builtin_nan("");
    }
}

// Per-shell moments of the half spectrum: X_b = sum_{m in S_b} |D(m)|^2 and
// Y_b = sum_{m in S_b} |D(m)|^4 over the full spectrum (an entry with
// m_x > 0 stands for m and -m, which have the same modulus; the m_x = 0
// plane holds both of each pair).  Each step covers 256 entries: the block
// finds their |m|^2 range, and for every shell that meets it sums the
// members' values with wave shuffles and a fixed-order combination of the
// four wave sums into an LDS accumulator of the shell.  Block partials
// partial[map][block][b][2] are summed in a fixed order afterwards.
constexpr int SM_MAXB = 128;

__global__ __launch_bounds__(256) void k_shell_moments(const float2 *__restrict__ spec, int64_t spec_stride, int n,
                                                       int hp, int nb, const int *__restrict__ thr,
                                                       double *__restrict__ partial) {
    __shared__ int lo2s[SM_MAXB], hi2s[SM_MAXB];
    __shared__ double acc[2][SM_MAXB];
    __shared__ double red[2][4];
    __shared__ int rng[2][4];
    const int map = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int xw = n / 2 + 1;
    const int64_t total = (int64_t)n * n * xw;
    const float2 *sp = spec + (int64_t)map * spec_stride;
    if (tid < nb) {
        lo2s[tid] = thr[tid];
        hi2s[tid] = thr[nb + tid];
        acc[0][tid] = 0.0;
        acc[1][tid] = 0.0;
    }
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * 256; base < total; base += (int64_t)gridDim.x * 256) {
        const int64_t e = base + tid;
        int r2 = -1;
        double v2 = 0.0, v4 = 0.0;
        if (e < total) {
            const int x = (int)(e % xw);
            const int64_t row = e / xw;
            const int y = (int)(row % n), z = (int)(row / n);
            const int mz = signed_freq(z, n), my = signed_freq(y, n);
            r2 = mz * mz + my * my + x * x;
            const float2 v = sp[row * hp + x];
            const double a = (double)v.x * v.x + (double)v.y * v.y;
            const double w = x == 0 ? 1.0 : 2.0;
            v2 = w * a;
            v4 = w * a * a;
        }
        // |m|^2 range of the step's entries (the mean mode and padding excluded)
        int rmin = r2 > 0 ? r2 : INT32_MAX, rmax = r2 > 0 ? r2 : -1;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            rmin = min(rmin, __shfl_xor(rmin, o, 64));
            rmax = max(rmax, __shfl_xor(rmax, o, 64));
        }
        if (lane == 0) {
            rng[0][wave] = rmin;
            rng[1][wave] = rmax;
        }
        __syncthreads();
        rmin = min(min(rng[0][0], rng[0][1]), min(rng[0][2], rng[0][3]));
        rmax = max(max(rng[1][0], rng[1][1]), max(rng[1][2], rng[1][3]));
        for (int b = 0; b < nb; ++b) {
            const int lo = lo2s[b], hi = hi2s[b];
            if (hi <= rmin || lo > rmax) continue;          // block-uniform
            const bool in = r2 > 0 && r2 >= lo && r2 < hi;
            double x2 = wave_sum(in ? v2 : 0.0), x4 = wave_sum(in ? v4 : 0.0);
            if (lane == 0) {
                red[0][wave] = x2;
                red[1][wave] = x4;
            }
            __syncthreads();
            if (tid == 0) {
                acc[0][b] += (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
                acc[1][b] += (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
            }
            __syncthreads();
        }
        __syncthreads();   // rng is rewritten by the next step
    }
    if (tid < nb) {
        double *o = partial + (((int64_t)map * gridDim.x + blockIdx.x) * nb + tid) * 2;
        o[0] = acc[0][tid];
        o[1] = acc[1][tid];
    }
}

// Connected T: Tc = T - scale N_pix S_D; S_D = 0 unless the quad is (a,a,b,b),
// S_D = X_a X_b, plus 2 X_a^2 - 3 Y_a when a = b (the three Gaussian
// pairings of k1..k4, inclusion-exclusion over their common quadruples
// (k,-k,-k,k) and the like; for disjoint shells a != b only k2 = -k1,
// k4 = -k3 pairs).  mom [map][nb][2] = (X, Y); scale is the raw T's
// normalisation per quad, V^3 / N_pix^4 / (N_pix N_q).
__global__ __launch_bounds__(256) void k_trispec_connected(const double *__restrict__ T,
                                                           const double *__restrict__ mom,
                                                           const uchar4 *__restrict__ quads,
                                                           const double *__restrict__ scale, double npix, int nq,
                                                           int nb, double *__restrict__ Tc) {
    const int q = blockIdx.x * 256 + threadIdx.x, map = blockIdx.y;
    if (q >= nq) return;
    const uchar4 t = quads[q];
    int s[4] = {t.x, t.y, t.z, t.w};
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && s[j] < s[j - 1]; --j) {
            const int u = s[j];
            s[j] = s[j - 1];
            s[j - 1] = u;
        }
    const int a = s[0], b = s[2];
    const double *m = mom + (int64_t)map * nb * 2;
    const double xa = m[2 * a], xb = m[2 * b], ya = m[2 * a + 1];
    // with identical or disjoint shells only (a, a, b, b) has pairings
    const bool coll = s[0] == s[1] && s[2] == s[3];
    const double sd = coll ? xa * xb + (a == b ? 2.0 * xa * xa - 3.0 * ya : 0.0) : 0.0;
    Tc[(int64_t)map * nq + q] = T[(int64_t)map * nq + q] - scale[q] * npix * sd;
}

// ---------------------------------------------------------------------------
// Modes per shell: each thread classifies one grid mode; a wave ballot and a
// popcount give the wave's count per bin, one integer atomic per wave.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shell_hist(int n, int nb, const int *__restrict__ lo2,
                                                    const int *__restrict__ hi2,
                                                    unsigned long long *__restrict__ counts) {
    const int64_t vol = (int64_t)n * n * n;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int r2 = -1;
    if (g < vol) {
        const int x = (int)(g % n), y = (int)((g / n) % n), z = (int)(g / ((int64_t)n * n));
        const int mz = signed_freq(z, n), my = signed_freq(y, n), mx = signed_freq(x, n);
        r2 = mz * mz + my * my + mx * mx;
    }
    for (int b = 0; b < nb; ++b) {
        const bool in = r2 > 0 && r2 >= lo2[b] && r2 < hi2[b];
        const unsigned long long m = __ballot(in);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(&counts[b], (unsigned long long)__popcll(m));
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

// Runs f(std::integral_constant<int, N>) for the supported grid sides.
template <class F> hipError_t dispatch_n(int n, F &&f) {
    switch (n) {
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 16: f(std::integral_constant<int, 16>{}); break;
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        case 128: f(std::integral_constant<int, 128>{}); break;
        case 256: f(std::integral_constant<int, 256>{}); break;
        case 512: f(std::integral_constant<int, 512>{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mean(const float *x, int n, int batch, double *partial, int nparts, double *mean,
                       hipStream_t st) {
    const int64_t vol = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_sum_f64, dim3(nparts, batch), dim3(256), 0, st, x, vol, vol, partial);
    hipLaunchKernelGGL(k_mean_final, dim3(batch), dim3(64), 0, st, partial, nparts, 1.0 / (double)vol, mean);
    return hipGetLastError();
}

hipError_t launch_forward(const float *delta, const double *mean, int n, int batch, const float2 *tw,
                          float2 *spec, hipStream_t st, double scale) {
    return dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        constexpr int G = pencils_per_block<float, NN>();
        constexpr int GX = G < NN * NN / 2 ? G : NN * NN / 2;
        constexpr int HP = spec_ld<NN>();
        const int64_t hvol = (int64_t)NN * NN * HP;
        hipLaunchKernelGGL((k_fwd_x<NN>), dim3(NN * NN / (2 * GX), batch), dim3(256), 0, st, delta, mean, tw, spec,
                           scale);
        hipLaunchKernelGGL((k_fft_strided<float, NN, -1, 1, HP>), dim3(NN * HP / G, batch), dim3(256), 0, st, spec,
                           tw, hvol);
        hipLaunchKernelGGL((k_fft_strided<float, NN, -1, 2, HP>), dim3(NN * HP / G, batch), dim3(256), 0, st, spec,
                           tw, hvol);
    });
}

template <typename R>
hipError_t launch_inverse_zy_t(const cplx<R> *spec, int64_t spec_stride, int n, int batch, const cplx<R> *tw,
                               const PairDev *pd, const int2 *ztab, int nz_blk, const int2 *ytab, int ny_blk,
                               const int *cols, cplx<R> *abox, cplx<R> *bc, hipStream_t st) {
    return dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        if (nz_blk > 0) {
            if (spec)
                hipLaunchKernelGGL((k_inv_z_prune<R, NN, false>), dim3(nz_blk, batch), dim3(256), 0, st, spec,
                                   spec_stride, abox, pd, ztab, cols, tw);
            else
                hipLaunchKernelGGL((k_inv_z_prune<R, NN, true>), dim3(nz_blk, batch), dim3(256), 0, st, spec,
                                   spec_stride, abox, pd, ztab, cols, tw);
        }
        if (ny_blk > 0)
            hipLaunchKernelGGL((k_inv_y_prune<R, NN>), dim3(ny_blk, batch), dim3(256), 0, st, abox, bc, pd, ytab,
                               tw);
    });
}

template <typename R>
hipError_t launch_inverse_x_t(const cplx<R> *bc, int64_t bc_stride, int n, int batch, const cplx<R> *tw,
                              const PairGeom &g, R *f1, R *f2, int64_t field_stride, hipStream_t st) {
    return dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        constexpr int G = pencils_per_block<R, NN>();
        hipLaunchKernelGGL((k_inv_x_compact<R, NN>), dim3(NN * NN / G, batch), dim3(256), 0, st, bc, bc_stride, g,
                           tw, f1, f2, field_stride);
    });
}

hipError_t launch_inverse_zy(const float2 *spec, int64_t spec_stride, int n, int batch, const float2 *tw,
                             const PairDev *pd, const int2 *ztab, int nz_blk, const int2 *ytab, int ny_blk,
                             const int *cols, float2 *abox, float2 *bc, hipStream_t st) {
    return launch_inverse_zy_t<float>(spec, spec_stride, n, batch, tw, pd, ztab, nz_blk, ytab, ny_blk, cols, abox,
                                      bc, st);
}

hipError_t launch_inverse_x(const float2 *bc, int64_t bc_stride, int n, int batch, const float2 *tw,
                            const PairGeom &g, float *f1, float *f2, int64_t field_stride, hipStream_t st) {
    return launch_inverse_x_t<float>(bc, bc_stride, n, batch, tw, g, f1, f2, field_stride, st);
}

hipError_t launch_inverse_x_pairs(const float2 *bc, int n, int batch, const float2 *tw, const PairDev *pd, int npairs,
                                  int nb, float *fields, hipStream_t st) {
    if (npairs < 1 || 2 * npairs < nb || 2 * (npairs - 1) >= nb) return hipErrorInvalidValue;
    return dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        constexpr int G = pencils_per_block<float, NN>();
        hipLaunchKernelGGL((k_inv_x_pairs<NN>), dim3(NN * NN / G, batch, npairs), dim3(256), 0, st, bc, pd, tw, nb,
                           fields);
    });
}

hipError_t launch_inverse_unit_f64(int n, const double2 *tw, const PairDev *pd, const PairGeom &g,
                                   const int2 *ztab, int nz_blk, const int2 *ytab, int ny_blk, const int *cols,
                                   double2 *abox, double2 *bc, double *f1, double *f2, hipStream_t st) {
    const int64_t vol = (int64_t)n * n * n;
    hipError_t e = launch_inverse_zy_t<double>(nullptr, 0, n, 1, tw, pd, ztab, nz_blk, ytab, ny_blk, cols, abox, bc,
                                               st);
    if (e != hipSuccess) return e;
    return launch_inverse_x_t<double>(bc, 0, n, 1, tw, g, f1, f2, vol, st);
}

int64_t spec_elems(int n) {
    int64_t e = 0;
    dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        e = (int64_t)NN * NN * spec_ld<NN>();
    });
    return e;
}

int fft_pencils_per_block(int n, bool fp64) {
    int g = 0;
    dispatch_n(n, [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        g = fp64 ? pencils_per_block<double, NN>() : pencils_per_block<float, NN>();
    });
    return g;
}

template <typename R>
hipError_t launch_contract_terms_t(const R *fields, int64_t npix, int nb, int64_t map_stride, int batch,
                                   const uchar4 *terms, int nterm, int nblk, double *partial, hipStream_t st) {
    const int64_t chunk = ((npix + nblk - 1) / nblk + CT_TILE - 1) / CT_TILE * CT_TILE;
    const size_t smem = (size_t)CT_TILE * nb * sizeof(R);
    for (int t0 = 0; t0 < nterm; t0 += 256 * CT_MAXT) {
        const int nt = nterm - t0 < 256 * CT_MAXT ? nterm - t0 : 256 * CT_MAXT;
        hipLaunchKernelGGL((k_contract_terms<R>), dim3(nblk, batch), dim3(256), smem, st, fields, npix, nb,
                           map_stride, terms, t0, nt, nterm, chunk, partial);
    }
    return hipGetLastError();
}

hipError_t launch_contract_terms_f32(const float *fields, int64_t npix, int nb, int64_t map_stride, int batch,
                                     const uchar4 *terms, int nterm, int nblk, double *partial, hipStream_t st) {
    return launch_contract_terms_t<float>(fields, npix, nb, map_stride, batch, terms, nterm, nblk, partial, st);
}


// out[map][list[i]] = scale[i] src[map][i]
__global__ __launch_bounds__(256) void k_scatter_list(const double *__restrict__ src, int n,
                                                      const int *__restrict__ list, const double *__restrict__ scale,
                                                      double *__restrict__ out, int nout) {
    const int i = blockIdx.x * 256 + threadIdx.x, map = blockIdx.y;
    if (i < n && list[i] >= 0) out[(int64_t)map * nout + list[i]] = scale[i] * src[(int64_t)map * n + i];
}

hipError_t launch_scatter_list(const double *src, int n, const int *list, const double *scale, int batch,
                               double *out, int nout, hipStream_t st) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_list, dim3((n + 255) / 256, batch), dim3(256), 0, st, src, n, list, scale, out,
                       nout);
    return hipGetLastError();
}

hipError_t launch_contract_terms_f64(const double *fields, int64_t npix, int nb, const uchar4 *terms, int nterm,
                                     int nblk, double *partial, hipStream_t st) {
    return launch_contract_terms_t<double>(fields, npix, nb, npix * nb, 1, terms, nterm, nblk, partial, st);
}

hipError_t launch_finalize(const double *partial, int nblk, int nterm, int batch, const double *scale, double *o0,
                           int n0, double *o1, int n1, double *o2, int n2, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3((nterm + 255) / 256, batch), dim3(256), 0, st, partial, nblk, nterm, scale,
                       o0, n0, o1, n1, o2, n2);
    return hipGetLastError();
}

hipError_t launch_rebin(const double *B, int n_tri, const double *count, const int *group, int n_group, int batch,
                        double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rebin, dim3(n_group, batch), dim3(RB_NT), 0, st, B, n_tri, count, group, n_group, out);
    return hipGetLastError();
}

hipError_t launch_shell_moments(const float2 *spec, int64_t spec_stride, int n, int nb, int batch, const int *thr,
                                int nblk, double *partial, hipStream_t st) {
    if (nb < 1 || nb > SM_MAXB || nblk < 1) return hipErrorInvalidValue;
    const int hp = (int)(spec_elems(n) / ((int64_t)n * n));
    hipLaunchKernelGGL(k_shell_moments, dim3(nblk, batch), dim3(256), 0, st, spec, spec_stride, n, hp, nb, thr,
                       partial);
    return hipGetLastError();
}

hipError_t launch_trispec_connected(const double *T, const double *mom, const uchar4 *quads, const double *scale,
                                    double npix, int nq, int nb, int batch, double *Tc, hipStream_t st) {
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_trispec_connected, dim3((nq + 255) / 256, batch), dim3(256), 0, st, T, mom, quads, scale,
                       npix, nq, nb, Tc);
    return hipGetLastError();
}

hipError_t launch_shell_hist(int n, int nb, const int *lo2, const int *hi2, unsigned long long *counts,
                             hipStream_t st) {
    const int64_t vol = (int64_t)n * n * n;
    const int nblk = (int)((vol + 255) / 256);
    hipLaunchKernelGGL(k_shell_hist, dim3(nblk), dim3(256), 0, st, n, nb, lo2, hi2, counts);
    return hipGetLastError();
}

}  // namespace bispec
