// general.hip -- transforms of the polyspectrum estimator on grids that are
// not cubic powers of two (gfx950).
//
// A grid N_z x N_y x N_x of cubic cells (the non-cubic footnote of Section 2:
// one fundamental per axis) whose sides are products of 2, 3, 4, 5, 8 and at
// most one other prime up to GEN_MAX_PRIME (the paper's 600^3 toy boxes of
// Section 3.3, its 536^3 = 8 x 67 N-body grid of Section 3.2).  Every axis is
// a Stockham autosort FFT with radices chosen on the host; a block holds a
// group of G pencils in LDS, twice (the passes alternate between the two
// copies), and runs the passes of its axis in order.  In a pass of radix R
// over sub-transforms of span Ns, butterfly jj of a pencil reads the R inputs
// a[jj + t n/R], multiplies input t by w^(t k), k = jj mod Ns,
// w = exp(dir 2 pi i / (Ns R)), takes the R-point DFT and writes output u to
// (jj / Ns) Ns R + k + u Ns.  Every twiddle is an integer power of
// W_n = exp(-2 pi i / n) read from a table built on the host in FP64 from the
// exactly reduced argument (the inverse direction conjugates it).
//
// The forward transform keeps the full complex spectrum [m_z][m_y][m_x]
// (Eq. DeltaFFTtoDelta).  Each shell pair (b1, b2) is transformed back in the
// full work volume: pass Z gathers [m in S_b1] Delta + i [m in S_b2] Delta
// (both masked spectra are Hermitian, so the inverse is F_b1 + i F_b2,
// Eq. delta_nr), passes Y and X follow, and the last pass writes the real and
// imaginary parts as the two bin fields.  Membership is the integer test
// qlo <= q < qhi on q = (s_z m_z)^2 + (s_y m_y)^2 + (s_x m_x)^2, s_i = P / N_i
// with P the lcm of the sides.
// The passes are pruned to the pair's reach, qmax = max(hi1, hi2): pass Z
// runs on the columns of the disk (s_y m_y)^2 + (s_x m_x)^2 < qmax only (a
// column outside it holds no shell mode) and writes nothing elsewhere; pass
// Y runs on the columns (n_z, x) with (s_x m_x)^2 < qmax and reads the
// entries outside the disk as zeros; pass X reads only those x, the rest of
// each row as zeros.  Blocks whose pencils all fall outside return at once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"
#include "general.hpp"

namespace bispec {

namespace {

constexpr int GEN_NT = 256;

// Signed frequency of index i on an axis of n points: 0..n - n/2 - 1, then
// -(n/2)..-1.
__device__ __forceinline__ int gen_freq(int i, int n) { return i < n - n / 2 ? i : i - n; }

// q contributions of the y and x frequencies, and the pair's reach.
__device__ __forceinline__ int64_t gen_qy(const GenGrid &g, int y) {
    const int64_t m = g.sy * gen_freq(y, g.ny);
    return m * m;
}
__device__ __forceinline__ int64_t gen_qx(const GenGrid &g, int x) {
    const int64_t m = g.sx * gen_freq(x, g.nx);
    return m * m;
}
__device__ __forceinline__ int64_t gen_reach(const GenPair &pr) { return pr.hi1 > pr.hi2 ? pr.hi1 : pr.hi2; }

template <int DIR, typename C> __device__ __forceinline__ C gen_tw(const C *tw, int j) {
    C w = tw[j];
    if constexpr (DIR > 0) w = cconj(w);
    return w;
}

// 3- and 5-point DFTs with w = exp(DIR 2 pi i / R) (cosines and sines of
// 2 pi / 3, 2 pi / 5, 4 pi / 5).
template <int DIR, typename C> __device__ __forceinline__ void dft3(C *v) {
    using R = decltype(v[0].x);
    const R c = R(-0.5), s = R(0.86602540378443864676372317075294);
    const C a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    const C m = C{v[0].x + c * a.x, v[0].y + c * a.y};
    const C ib = mul_di<DIR>(C{s * b.x, s * b.y});          // i DIR s (x1 - x2)
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, ib);
    v[2] = csub(m, ib);
}

template <int DIR, typename C> __device__ __forceinline__ void dft5(C *v) {
    using R = decltype(v[0].x);
    const R c1 = R(0.30901699437494742410229341718282), c2 = R(-0.80901699437494742410229341718282);
    const R s1 = R(0.95105651629515357211643933337938), s2 = R(0.58778525229247312916870595463907);
    const C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const C m1 = C{v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const C m2 = C{v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const C j1 = mul_di<DIR>(C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    const C j2 = mul_di<DIR>(C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, j1);
    v[4] = csub(m1, j1);
    v[2] = cadd(m2, j2);
    v[3] = csub(m2, j2);
}

template <int R, int DIR, typename C> __device__ __forceinline__ void gen_dft(C *v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 3) dft3<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 5) dft5<DIR>(v);
    else if constexpr (R == 8) dft8<DIR>(v);
}

// q = a / b and r = a % b for 0 <= a < 2^24 and b >= 1, given rcp = 1 / b in
// FP32: the FP32 quotient is off by at most one and is corrected once (the
// divisors vary per pass, so the integer division would not be strength-
// reduced by the compiler).
__device__ __forceinline__ int gen_divmod(int a, int b, float rcp, int &r) {
    int q = (int)((float)a * rcp);
    r = a - q * b;
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    return q;
}

// One pass of radix R (2, 3, 4, 5 or 8) from src to dst over G pencils of n
// points (pencil stride n).  The twiddle exponent t k n / (ns R) stays
// below n (t < R, k < ns), so it needs no reduction.
template <int R, int DIR, typename C>
__device__ void gen_pass(const C *src, C *dst, const C *tw, int n, int ns, int G) {
    const int nb = n / R, tstep = n / (ns * R);
    const float rnb = 1.0f / (float)nb, rns = 1.0f / (float)ns;
    for (int task = threadIdx.x; task < G * nb; task += GEN_NT) {
        int jj, k;
        const int p = gen_divmod(task, nb, rnb, jj);
        const int blk = gen_divmod(jj, ns, rns, k);
        const C *s = src + p * n;
        C v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            v[t] = s[jj + t * nb];
            if (t > 0 && ns > 1) v[t] = cmul(v[t], gen_tw<DIR>(tw, t * k * tstep));
        }
        gen_dft<R, DIR>(v);
        C *d = dst + p * n + blk * ns * R + k;
#pragma unroll
        for (int u = 0; u < R; ++u) d[u * ns] = v[u];
    }
}

// A pass of a prime radix R > 5: one output per task, y_u = sum_t x_t' w_R^(t u)
// with x_t' the twiddled inputs (w_R^m = W_n^(m n / R) from the table).
template <int DIR, typename C>
__device__ void gen_pass_prime(const C *src, C *dst, const C *tw, int n, int ns, int R, int G) {
    const int nb = n / R, tstep = n / (ns * R), step_r = n / R;
    const float rn = 1.0f / (float)n, rr = 1.0f / (float)R, rns = 1.0f / (float)ns;
    for (int task = threadIdx.x; task < G * n; task += GEN_NT) {
        int rem, u, k;
        const int p = gen_divmod(task, n, rn, rem);
        const int jj = gen_divmod(rem, R, rr, u);
        const int blk = gen_divmod(jj, ns, rns, k);
        const C *s = src + p * n;
        C acc = C{0, 0};
        int tu = 0;                                  // t u mod R
        for (int t = 0; t < R; ++t) {
            C x = s[jj + t * nb];
            if (t > 0 && ns > 1) x = cmul(x, gen_tw<DIR>(tw, t * k * tstep));
            acc = cadd(acc, cmul(x, gen_tw<DIR>(tw, tu * step_r)));
            tu += u;
            if (tu >= R) tu -= R;
        }
        dst[p * n + blk * ns * R + k + u * ns] = acc;
    }
}

// All passes of one axis on the G pencils in a (copy b is the other buffer);
// returns the buffer that holds the result.  Expects a filled and a barrier.
template <int DIR, typename C>
__device__ C *gen_fft(C *a, C *b, const C *tw, const GenAxis &ax, int G) {
    int ns = 1;
    for (int i = 0; i < ax.nrad; ++i) {
        const int R = ax.radix[i];
        switch (R) {
            case 2: gen_pass<2, DIR>(a, b, tw, ax.n, ns, G); break;
            case 3: gen_pass<3, DIR>(a, b, tw, ax.n, ns, G); break;
            case 4: gen_pass<4, DIR>(a, b, tw, ax.n, ns, G); break;
            case 5: gen_pass<5, DIR>(a, b, tw, ax.n, ns, G); break;
            case 8: gen_pass<8, DIR>(a, b, tw, ax.n, ns, G); break;
            default: gen_pass_prime<DIR>(a, b, tw, ax.n, ns, R, G); break;
        }
        __syncthreads();
        C *t = a;
        a = b;
        b = t;
        ns *= R;
    }
    return a;
}

// Forward pass along x: real rows (minus the FP64 mean, if any, times
// scale) to complex rows of the full spectrum; block (x, map) holds rows
// x G .. x G + G - 1.
template <typename C, typename Rr>
__global__ __launch_bounds__(GEN_NT) void k_gen_fwd_x(const Rr *__restrict__ delta,
                                                      const double *__restrict__ mean, C *__restrict__ spec,
                                                      const C *__restrict__ tw, GenGrid g, int G, double scale) {
    using R = decltype(C{}.x);
    extern __shared__ __attribute__((aligned(16))) unsigned char gsm_raw[];
    C *gsm = reinterpret_cast<C *>(gsm_raw);
    const GenAxis &ax = g.ax[2];
    const int n = ax.n;
    C *a = gsm, *b = gsm + G * n;
    const int map = blockIdx.y;
    const int64_t rows = (int64_t)g.nz * g.ny;
    const int64_t r0 = (int64_t)blockIdx.x * G;
    const Rr *src = delta + (int64_t)map * g.npix;
    const double mu = mean ? mean[map] : 0.0;
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e / n, i = e % n;
        a[e] = r0 + p < rows ? C{(R)(((double)src[(r0 + p) * n + i] - mu) * scale), R(0)} : C{R(0), R(0)};
    }
    __syncthreads();
    const C *res = gen_fft<-1>(a, b, tw + ax.tw_off, ax, G);
    C *dst = spec + (int64_t)map * g.npix;
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e / n, i = e % n;
        if (r0 + p < rows) dst[(r0 + p) * n + i] = res[e];
    }
}

// In-place transform along y (AXIS 1) or z (AXIS 2) of a complex volume
// [z][y][x].  A block takes G pencils adjacent in x (AXIS 1: (z, x0 + p);
// AXIS 2: columns c0 + p of the y-x plane), so loads and stores run along x.
template <typename C, int DIR, int AXIS>
__global__ __launch_bounds__(GEN_NT) void k_gen_axis(C *__restrict__ vol, const C *__restrict__ tw, GenGrid g,
                                                     int G) {
    extern __shared__ __attribute__((aligned(16))) unsigned char gsm_raw[];
    C *a = reinterpret_cast<C *>(gsm_raw);
    const GenAxis &ax = g.ax[AXIS == 1 ? 1 : 0];
    const int n = ax.n;
    C *b = a + G * n;
    C *v = vol + (int64_t)blockIdx.y * g.npix;
    const int gx = (g.nx + G - 1) / G;               // groups per x row (AXIS 1)
    const int64_t ncol = (int64_t)g.ny * g.nx;       // columns of the y-x plane (AXIS 2)
    auto addr = [&](int p, int i, bool &ok) -> int64_t {
        if constexpr (AXIS == 1) {
            const int z = blockIdx.x / gx, x = (blockIdx.x % gx) * G + p;
            ok = x < g.nx;
            return ((int64_t)z * g.ny + i) * g.nx + x;
        } else {
            const int64_t c = (int64_t)blockIdx.x * G + p;
            ok = c < ncol;
            return (int64_t)i * ncol + c;
        }
    };
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G;
        bool ok;
        const int64_t at = addr(p, i, ok);
        a[p * n + i] = ok ? v[at] : C{0, 0};
    }
    __syncthreads();
    const C *res = gen_fft<DIR>(a, b, tw + ax.tw_off, ax, G);
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G;
        bool ok;
        const int64_t at = addr(p, i, ok);
        if (ok) v[at] = res[p * n + i];
    }
}

// Pass Z of the inverse transform of one shell pair: column c = y N_x + x of
// the y-x plane gathers along m_z the masked spectrum
// [q in S_b1] Delta + i [q in S_b2] Delta (UNIT: Delta = 1) and transforms it.
template <typename C, bool UNIT>
__global__ __launch_bounds__(GEN_NT) void k_gen_inv_z(const C *__restrict__ spec, C *__restrict__ work,
                                                      const C *__restrict__ tw, GenGrid g, GenPair pr, int G) {
    extern __shared__ __attribute__((aligned(16))) unsigned char gsm_raw[];
    C *a = reinterpret_cast<C *>(gsm_raw);
    const GenAxis &ax = g.ax[0];
    const int n = ax.n;
    C *b = a + G * n;
    const int map = blockIdx.y;
    const int64_t ncol = (int64_t)g.ny * g.nx;
    const C *sp = UNIT ? nullptr : spec + (int64_t)map * g.npix;
    C *w = work + (int64_t)map * g.npix;
    using Rr = decltype(C{}.x);
    const int64_t reach = gen_reach(pr);
    auto in_disk = [&](int64_t c) {
        return c < ncol && gen_qy(g, (int)(c / g.nx)) + gen_qx(g, (int)(c % g.nx)) < reach;
    };
    // the block's columns all outside the disk: nothing to do (block-uniform)
    const int64_t cfirst = (int64_t)blockIdx.x * G;
    if (!__syncthreads_or(threadIdx.x < G && in_disk(cfirst + threadIdx.x))) return;
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G;
        const int64_t c = (int64_t)blockIdx.x * G + p;
        C val = C{0, 0};
        if (c < ncol) {
            const int y = (int)(c / g.nx), x = (int)(c % g.nx);
            const int64_t mz = gen_freq(i, g.nz), my = gen_freq(y, g.ny), mx = gen_freq(x, g.nx);
            const int64_t q = (g.sz * mz) * (g.sz * mz) + (g.sy * my) * (g.sy * my) + (g.sx * mx) * (g.sx * mx);
            const bool in1 = q > 0 && q >= pr.lo1 && q < pr.hi1;
            const bool in2 = q > 0 && q >= pr.lo2 && q < pr.hi2;
            if (in1 || in2) {
                C d = C{Rr(1), Rr(0)};
                if constexpr (!UNIT) d = sp[(int64_t)i * ncol + c];
                const Rr a1 = in1 ? Rr(1) : Rr(0), a2 = in2 ? Rr(1) : Rr(0);
                val = C{d.x * a1 - d.y * a2, d.y * a1 + d.x * a2};
            }
        }
        a[p * n + i] = val;
    }
    __syncthreads();
    const C *res = gen_fft<+1>(a, b, tw + ax.tw_off, ax, G);
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G;
        const int64_t c = (int64_t)blockIdx.x * G + p;
        if (in_disk(c)) w[(int64_t)i * ncol + c] = res[p * n + i];
    }
}

// Pass Y of the inverse transform of one shell pair, in place on the work
// volume: block (z, x group) transforms the columns (z, x) with
// (s_x m_x)^2 < reach along y, reading the entries outside the disk as zeros
// (pass Z left them unwritten).
template <typename C>
__global__ __launch_bounds__(GEN_NT) void k_gen_inv_y(C *__restrict__ work, const C *__restrict__ tw, GenGrid g,
                                                      GenPair pr, int G) {
    extern __shared__ __attribute__((aligned(16))) unsigned char gsm_raw[];
    C *a = reinterpret_cast<C *>(gsm_raw);
    const GenAxis &ax = g.ax[1];
    const int n = ax.n;
    C *b = a + G * n;
    C *v = work + (int64_t)blockIdx.y * g.npix;
    const int gx = (g.nx + G - 1) / G;
    const int z = blockIdx.x / gx, x0 = (blockIdx.x % gx) * G;
    const int64_t reach = gen_reach(pr);
    auto live = [&](int x) { return x < g.nx && gen_qx(g, x) < reach; };
    if (!__syncthreads_or(threadIdx.x < G && live(x0 + threadIdx.x))) return;
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G, x = x0 + p;
        const bool ok = live(x) && gen_qy(g, i) + gen_qx(g, x) < reach;
        a[p * n + i] = ok ? v[((int64_t)z * g.ny + i) * g.nx + x] : C{0, 0};
    }
    __syncthreads();
    const C *res = gen_fft<+1>(a, b, tw + ax.tw_off, ax, G);
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e % G, i = e / G, x = x0 + p;
        if (live(x)) v[((int64_t)z * g.ny + i) * g.nx + x] = res[p * n + i];
    }
}

// Pass X of the inverse transform: rows of the work volume transformed along
// x; the real parts are F_b1, the imaginary parts F_b2 (f2 may be null).
// Fields of map m start at m * map_stride.
template <typename C, typename Rr>
__global__ __launch_bounds__(GEN_NT) void k_gen_inv_x(const C *__restrict__ work, Rr *__restrict__ f1,
                                                      Rr *__restrict__ f2, int64_t map_stride,
                                                      const C *__restrict__ tw, GenGrid g, GenPair pr, int G) {
    extern __shared__ __attribute__((aligned(16))) unsigned char gsm_raw[];
    C *a = reinterpret_cast<C *>(gsm_raw);
    const GenAxis &ax = g.ax[2];
    const int n = ax.n;
    C *b = a + G * n;
    const int map = blockIdx.y;
    const int64_t rows = (int64_t)g.nz * g.ny;
    const int64_t r0 = (int64_t)blockIdx.x * G;
    const C *src = work + (int64_t)map * g.npix;
    const int64_t reach = gen_reach(pr);
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e / n, i = e % n;
        a[e] = r0 + p < rows && gen_qx(g, i) < reach ? src[(r0 + p) * n + i] : C{0, 0};
    }
    __syncthreads();
    const C *res = gen_fft<+1>(a, b, tw + ax.tw_off, ax, G);
    Rr *d1 = f1 + (int64_t)map * map_stride;
    Rr *d2 = f2 ? f2 + (int64_t)map * map_stride : nullptr;
    for (int e = threadIdx.x; e < G * n; e += GEN_NT) {
        const int p = e / n, i = e % n;
        if (r0 + p < rows) {
            d1[(r0 + p) * n + i] = res[e].x;
            if (d2) d2[(r0 + p) * n + i] = res[e].y;
        }
    }
}

// Zeros in the padding [npix, stride) of every field (so that sums over the
// padded length equal sums over the grid).
template <typename Rr>
__global__ void k_gen_zero_pads(Rr *__restrict__ fields, int64_t npix, int64_t stride, int nfields) {
    const int64_t pad = stride - npix;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pad * nfields) return;
    fields[(e / pad) * stride + npix + e % pad] = Rr(0);
}

// FP64 mean of each map: block partials with scalar loads (any grid size).
__global__ __launch_bounds__(256) void k_gen_sum(const float *__restrict__ x, int64_t n, double *__restrict__ part) {
    const float *xm = x + (int64_t)blockIdx.y * n;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += xm[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_gen_mean(const double *__restrict__ part, int nparts, double inv_n,
                                                 double *__restrict__ mean) {
    const double *p = part + (int64_t)blockIdx.x * nparts;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 64) acc += p[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (threadIdx.x == 0) mean[blockIdx.x] = acc * inv_n;
}

// Modes per shell: one grid mode per thread, wave ballot + popcount per bin.
__global__ __launch_bounds__(256) void k_gen_shell_hist(GenGrid g, int nb, const long long *__restrict__ qlo,
                                                        const long long *__restrict__ qhi,
                                                        unsigned long long *__restrict__ counts) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t q = -1;
    if (e < g.npix) {
        const int x = (int)(e % g.nx), y = (int)((e / g.nx) % g.ny), z = (int)(e / ((int64_t)g.nx * g.ny));
        const int64_t mz = gen_freq(z, g.nz), my = gen_freq(y, g.ny), mx = gen_freq(x, g.nx);
        q = (g.sz * mz) * (g.sz * mz) + (g.sy * my) * (g.sy * my) + (g.sx * mx) * (g.sx * mx);
    }
    for (int b = 0; b < nb; ++b) {
        const bool in = q > 0 && q >= qlo[b] && q < qhi[b];
        const unsigned long long m = __ballot(in);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(&counts[b], (unsigned long long)__popcll(m));
    }
}

}  // namespace

int gen_pencils(int n, size_t elem_bytes) {
    // two copies of G pencils within 64 KiB of LDS, G a power of two <= 64
    int g = 1;
    while (2 * g <= 64 && (size_t)2 * (2 * g) * n * elem_bytes <= 65536) g *= 2;
    return g;
}

bool gen_factor(int n, GenAxis &ax) {
    ax = GenAxis{};
    ax.n = n;
    if (n < 2) return false;
    int r = n, k = 0;
    for (int f : {8, 4, 2, 3, 5})
        while (r % f == 0) {
            if (k >= GEN_MAX_RADICES) return false;
            ax.radix[k++] = f;
            r /= f;
        }
    if (r > 1) {
        if (r > GEN_MAX_PRIME || k >= GEN_MAX_RADICES) return false;
        for (int d = 2; d * d <= r; ++d)
            if (r % d == 0) return false;       // a composite rest (e.g. 7 x 7) is not handled
        ax.radix[k++] = r;
    }
    ax.nrad = k;
    return true;
}

namespace {
template <typename C> size_t gen_smem(int n, int G) { return (size_t)2 * G * n * sizeof(C); }
}  // namespace

hipError_t gen_mean(const float *x, const GenGrid &g, int batch, double *part, int nparts, double *mean,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_gen_sum, dim3(nparts, batch), dim3(256), 0, st, x, (int64_t)g.npix, part);
    hipLaunchKernelGGL(k_gen_mean, dim3(batch), dim3(64), 0, st, part, nparts, 1.0 / (double)g.npix, mean);
    return hipGetLastError();
}

template <typename C, typename Rr>
static hipError_t gen_forward_t(const Rr *delta, const double *mean, const GenGrid &g, int batch, const C *tw,
                                C *spec, hipStream_t st, double scale) {
    // rows are contiguous: half the rows per block, for occupancy (as in pass X
    // of the inverse)
    const int gpx = gen_pencils(g.nx, sizeof(C)), Gx = gpx >= 4 ? gpx / 2 : gpx;
    const int64_t rows = (int64_t)g.nz * g.ny;
    hipLaunchKernelGGL((k_gen_fwd_x<C, Rr>), dim3((unsigned)((rows + Gx - 1) / Gx), batch), dim3(GEN_NT),
                       gen_smem<C>(g.nx, Gx), st, delta, mean, spec, tw, g, Gx, scale);
    const int Gy = gen_pencils(g.ny, sizeof(C));
    hipLaunchKernelGGL((k_gen_axis<C, -1, 1>), dim3((unsigned)(g.nz * ((g.nx + Gy - 1) / Gy)), batch),
                       dim3(GEN_NT), gen_smem<C>(g.ny, Gy), st, spec, tw, g, Gy);
    const int Gz = gen_pencils(g.nz, sizeof(C));
    const int64_t ncol = (int64_t)g.ny * g.nx;
    hipLaunchKernelGGL((k_gen_axis<C, -1, 2>), dim3((unsigned)((ncol + Gz - 1) / Gz), batch), dim3(GEN_NT),
                       gen_smem<C>(g.nz, Gz), st, spec, tw, g, Gz);
    return hipGetLastError();
}

hipError_t gen_forward(const float *delta, const double *mean, const GenGrid &g, int batch, const float2 *tw,
                       float2 *spec, hipStream_t st, double scale) {
    return gen_forward_t<float2, float>(delta, mean, g, batch, tw, spec, st, scale);
}

hipError_t gen_forward_f64(const double *x, const GenGrid &g, const double2 *tw, double2 *spec, hipStream_t st) {
    return gen_forward_t<double2, double>(x, nullptr, g, 1, tw, spec, st, 1.0);
}

template <typename C, typename Rr, bool UNIT>
static hipError_t gen_inverse_t(const C *spec, C *work, const GenGrid &g, const GenPair &pr, int batch,
                                const C *tw, Rr *f1, Rr *f2, int64_t map_stride, hipStream_t st) {
    const int64_t ncol = (int64_t)g.ny * g.nx, rows = (int64_t)g.nz * g.ny;
    const int Gz = gen_pencils(g.nz, sizeof(C));
    hipLaunchKernelGGL((k_gen_inv_z<C, UNIT>), dim3((unsigned)((ncol + Gz - 1) / Gz), batch), dim3(GEN_NT),
                       gen_smem<C>(g.nz, Gz), st, spec, work, tw, g, pr, Gz);
    const int Gy = gen_pencils(g.ny, sizeof(C));
    hipLaunchKernelGGL((k_gen_inv_y<C>), dim3((unsigned)(g.nz * ((g.nx + Gy - 1) / Gy)), batch), dim3(GEN_NT),
                       gen_smem<C>(g.ny, Gy), st, work, tw, g, pr, Gy);
    // pass X: rows are contiguous, so fewer rows per block cost no coalescing
    // and buy occupancy (at 600 points, 2 rows in 19 KiB: eight blocks per CU)
    const int gpx = gen_pencils(g.nx, sizeof(C)), Gx = gpx >= 4 ? gpx / 2 : gpx;
    hipLaunchKernelGGL((k_gen_inv_x<C, Rr>), dim3((unsigned)((rows + Gx - 1) / Gx), batch), dim3(GEN_NT),
                       gen_smem<C>(g.nx, Gx), st, work, f1, f2, map_stride, tw, g, pr, Gx);
    return hipGetLastError();
}

hipError_t gen_inverse_pair(const float2 *spec, float2 *work, const GenGrid &g, const GenPair &pr, int batch,
                            const float2 *tw, float *f1, float *f2, int64_t map_stride, hipStream_t st) {
    return gen_inverse_t<float2, float, false>(spec, work, g, pr, batch, tw, f1, f2, map_stride, st);
}

hipError_t gen_inverse_unit_f64(double2 *work, const GenGrid &g, const GenPair &pr, const double2 *tw, double *f1,
                                double *f2, hipStream_t st) {
    return gen_inverse_t<double2, double, true>(nullptr, work, g, pr, 1, tw, f1, f2, 0, st);
}

hipError_t gen_zero_pads_f32(float *fields, int64_t npix, int64_t stride, int nfields, hipStream_t st) {
    const int64_t tot = (stride - npix) * nfields;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_zero_pads<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, fields, npix,
                       stride, nfields);
    return hipGetLastError();
}

hipError_t gen_zero_pads_f64(double *fields, int64_t npix, int64_t stride, int nfields, hipStream_t st) {
    const int64_t tot = (stride - npix) * nfields;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_zero_pads<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, fields, npix,
                       stride, nfields);
    return hipGetLastError();
}

hipError_t gen_shell_hist(const GenGrid &g, int nb, const long long *qlo, const long long *qhi,
                          unsigned long long *counts, hipStream_t st) {
    hipLaunchKernelGGL(k_gen_shell_hist, dim3((unsigned)((g.npix + 255) / 256)), dim3(256), 0, st, g, nb, qlo, qhi,
                       counts);
    return hipGetLastError();
}

}  // namespace bispec
