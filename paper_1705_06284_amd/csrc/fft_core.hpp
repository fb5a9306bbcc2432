// fft_core.hpp -- LDS-resident Stockham FFT of a group of pencils (gfx950).
//
// A block of NT threads (256 unless stated) holds G pencils of length N in
// LDS ([G][N] complex).
// The transform is a Stockham autosort sequence of radix-8 passes followed by
// at most one radix-2 or radix-4 pass, so N = 8^p * {1, 2, 4}.  In a pass of
// radix R over sub-transforms of span Ns, butterfly jj of a pencil reads the R
// inputs a[jj + t N/R], multiplies input t by w^(t k) with k = jj mod Ns and
// w = exp(dir 2 pi i / (Ns R)), takes an R-point DFT and writes output u to
// ((jj / Ns) Ns R + k + u Ns).  Every twiddle is an integer power of
// W_N = exp(-2 pi i / N) read from a table built on the host in FP64 from the
// exactly reduced argument; the inverse direction uses the conjugate.
//
// Direction: DIR = -1 is the forward transform of Eq. (DeltaFFTtoDelta),
// DIR = +1 the unnormalised inverse of Eq. (delta_nr).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bispec {

__device__ __forceinline__ int signed_freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Geometry of one shell pair (b1, b2) of the pruned inverse transform: mode m
// is in bin b1 iff lo1 <= |m|^2 < hi1 (likewise b2; lo2 = hi2 = 0 for a lone
// bin); every mode of either shell has components in [-R, R] and
// |m|^2 < hmax, and the compact intermediates span W = 2R + 1 values stored
// with row stride Wp (W rounded up to 16 complex = 128 bytes).
struct PairGeom {
    int lo1, hi1, lo2, hi2;
    int hmax, R, W, Wp;
};

// Where one pair's intermediates live (complex elements).  z-pass box of map
// m: aoff + m * astride, planes of W x Wp; compact rows of map m:
// boff + m * bstride, [N][N] rows of stride Wp.  The z-pass columns are
// cols[col_off .. col_off + ncols), each (m_y + R) * Wp + (m_x + R).
struct PairDev {
    PairGeom g;
    long long aoff, astride, boff, bstride;
    int col_off, ncols, pad0, pad1;
};

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename R> using cplx = typename cplx_of<R>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
// a * (DIR i)
template <int DIR, typename C> __device__ __forceinline__ C mul_di(C a) {
    return DIR > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <int DIR, typename C> __device__ __forceinline__ void dft2(C *v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C *v) {
    C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    C a2 = cadd(v[1], v[3]), a3 = mul_di<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
}

// y_u = sum_t x_t w8^(t u), w8 = exp(DIR 2 pi i / 8): split into even/odd
// outputs, each a 4-point DFT of (x_t +- x_{t+4}) (odd ones twiddled by w8^t).
template <int DIR, typename C> __device__ __forceinline__ void dft8(C *v) {
    using R = decltype(v[0].x);
    const R h = R(0.70710678118654752440084436210484904);
    C a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        a[t] = cadd(v[t], v[t + 4]);
        b[t] = csub(v[t], v[t + 4]);
    }
    // b_t * w8^t : w8 = h (1 + DIR i), w8^2 = DIR i, w8^3 = h (-1 + DIR i)
    {
        C x = b[1];
        C dx = mul_di<DIR>(x);
        b[1] = C{h * (x.x + dx.x), h * (x.y + dx.y)};
        b[2] = mul_di<DIR>(b[2]);
        C y = b[3];
        C dy = mul_di<DIR>(y);
        b[3] = C{h * (dy.x - y.x), h * (dy.y - y.y)};
    }
    dft4<DIR>(a);
    dft4<DIR>(b);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        v[2 * u] = a[u];
        v[2 * u + 1] = b[u];
    }
}

template <int RADIX, int DIR, typename C> __device__ __forceinline__ void dft_r(C *v) {
    if constexpr (RADIX == 8) dft8<DIR>(v);
    else if constexpr (RADIX == 4) dft4<DIR>(v);
    else if constexpr (RADIX == 2) dft2<DIR>(v);
}

// LDS layout of a pencil group: element i of pencil p sits at
// p * pencil_ld<N>() + pad_idx(i).  One padding slot per 8 elements breaks
// the power-of-two strides of the Stockham exchange (stride-8 writes of the
// first pass hit 16 distinct bank pairs), and the odd pencil stride staggers
// pencils that are read at the same position.
template <int N> constexpr int pencil_ld() { return N + N / 8 + 1; }
__device__ __forceinline__ int pad_idx(int i) { return i + (i >> 3); }

// Row length of the half spectrum m_x = 0..N/2 (the other half follows from
// Hermitian symmetry), rounded up to 16 entries so that rows stay 128-byte
// aligned and every pencil group of the strided passes stays whole.
template <int N> constexpr int spec_ld() { return (N / 2 + 1 + 15) / 16 * 16; }

constexpr int ilog8_floor(int n) { return n >= 8 ? 1 + ilog8_floor(n / 8) : 0; }
constexpr int ipow8(int p) { return p == 0 ? 1 : 8 * ipow8(p - 1); }

// One Stockham pass over the first g_act of the G pencils of the block (NT
// threads); the others are left untouched.  Output u of a butterfly goes to
// store(pencil, position, value) once every thread has read its inputs.
// Task t is butterfly t mod NB of pencil t / NB, or with PFAST butterfly
// t / G of pencil t mod G (consecutive threads on consecutive pencils, for
// stores that go straight to memory where pencils are adjacent).
template <typename C, int N, int LD, int G, int DIR, int RADIX, int NS, int NT, bool PFAST = false,
          typename Store>
__device__ __forceinline__ void stockham_pass_to(C *s, const C *tw, int g_act, Store store) {
    constexpr int NB = N / RADIX;          // butterflies per pencil
    constexpr int TASKS = G * NB;
    static_assert(TASKS % NT == 0 || TASKS < NT, "pencil group must fill the block or fit in it");
    constexpr int PER = TASKS < NT ? 1 : TASKS / NT;
    constexpr bool PARTIAL = TASKS < NT;   // some threads idle (tiny grids)
    constexpr int TSTEP = N / (NS * RADIX);
    const int tid = threadIdx.x;
    const int act_tasks = g_act * NB;
    C v[PER][RADIX];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int task = tid + q * NT;
        if ((!PFAST && task >= act_tasks) || (PARTIAL && tid >= TASKS)) break;
        const int p = PFAST ? task % G : task / NB, jj = PFAST ? task / G : task % NB;
        if (PFAST && p >= g_act) continue;
        const int k = jj % NS;
#pragma unroll
        for (int t = 0; t < RADIX; ++t) v[q][t] = s[p * LD + pad_idx(jj + t * NB)];
        if constexpr (NS > 1) {
#pragma unroll
            for (int t = 1; t < RADIX; ++t) {
                C w = tw[(t * k * TSTEP) & (N - 1)];
                if constexpr (DIR > 0) w = cconj(w);
                v[q][t] = cmul(v[q][t], w);
            }
        }
        dft_r<RADIX, DIR>(v[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int task = tid + q * NT;
        if ((!PFAST && task >= act_tasks) || (PARTIAL && tid >= TASKS)) break;
        const int p = PFAST ? task % G : task / NB, jj = PFAST ? task / G : task % NB;
        if (PFAST && p >= g_act) continue;
        const int k = jj % NS;
        const int base = (jj / NS) * NS * RADIX + k;
#pragma unroll
        for (int u = 0; u < RADIX; ++u) store(p, base + u * NS, v[q][u]);
    }
    __syncthreads();
}

template <typename C, int N, int LD, int G, int DIR, int RADIX, int NS, int NT, bool PFAST = false>
__device__ __forceinline__ void stockham_pass(C *s, const C *tw, int g_act) {
    stockham_pass_to<C, N, LD, G, DIR, RADIX, NS, NT, PFAST>(
        s, tw, g_act, [s](int p, int pos, C v) { s[p * LD + pad_idx(pos)] = v; });
}

// Full length-N transform of the first g_act (default all G) pencils held in
// s (pencil stride LD, positions mapped by pad_idx).
// Expects s filled and a __syncthreads() issued by the caller; leaves the
// result in s (natural order) followed by a barrier.
template <typename C, int N, int LD, int G, int DIR, int NT = 256>
__device__ __forceinline__ void fft_pencils(C *s, const C *tw, int g_act = G) {
    constexpr int P8 = ilog8_floor(N);
    constexpr int RL = N / ipow8(P8);
    if constexpr (P8 >= 1) stockham_pass<C, N, LD, G, DIR, 8, 1, NT>(s, tw, g_act);
    if constexpr (P8 >= 2) stockham_pass<C, N, LD, G, DIR, 8, 8, NT>(s, tw, g_act);
    if constexpr (P8 >= 3) stockham_pass<C, N, LD, G, DIR, 8, 64, NT>(s, tw, g_act);
    if constexpr (P8 >= 4) stockham_pass<C, N, LD, G, DIR, 8, 512, NT>(s, tw, g_act);
    if constexpr (RL > 1) stockham_pass<C, N, LD, G, DIR, RL, ipow8(P8), NT>(s, tw, g_act);
}

// As fft_pencils, but the last pass hands its outputs (pencil, position in
// natural order, value) to store instead of writing them back to s; s may be
// overwritten by store, since every read of the pass precedes it.
// SKIP_FIRST: the caller has already done the first radix-8 pass
// (first_pass_butterfly); needs N >= 16, so that it is not also the last.
template <typename C, int N, int LD, int G, int DIR, int NT, bool SKIP_FIRST = false, bool PFAST = false,
          typename Store>
__device__ __forceinline__ void fft_pencils_to(C *s, const C *tw, int g_act, Store store) {
    constexpr int P8 = ilog8_floor(N);
    constexpr int RL = N / ipow8(P8);
    constexpr int LAST8 = RL > 1 ? P8 : P8 - 1;     // radix-8 passes written back to s
    static_assert(!SKIP_FIRST || N >= 16, "the first pass is the last one");
    if constexpr (LAST8 >= 1 && !SKIP_FIRST) stockham_pass<C, N, LD, G, DIR, 8, 1, NT, PFAST>(s, tw, g_act);
    if constexpr (LAST8 >= 2) stockham_pass<C, N, LD, G, DIR, 8, 8, NT, PFAST>(s, tw, g_act);
    if constexpr (LAST8 >= 3) stockham_pass<C, N, LD, G, DIR, 8, 64, NT, PFAST>(s, tw, g_act);
    if constexpr (LAST8 >= 4) stockham_pass<C, N, LD, G, DIR, 8, 512, NT, PFAST>(s, tw, g_act);
    if constexpr (RL > 1)
        stockham_pass_to<C, N, LD, G, DIR, RL, ipow8(P8), NT, PFAST>(s, tw, g_act, store);
    else
        stockham_pass_to<C, N, LD, G, DIR, 8, ipow8(P8 - 1), NT, PFAST>(s, tw, g_act, store);
}

// First radix-8 Stockham pass of one butterfly whose 8 inputs x[jj + t N/8]
// (t < 8) the caller holds in v: no twiddles (span 1); output u goes to
// position 8 jj + u of pencil p.  Followed by a barrier and
// fft_pencils_to<..., SKIP_FIRST = true>.
template <typename C, int N, int LD, int DIR>
__device__ __forceinline__ void first_pass_butterfly(C *s, int p, int jj, C *v) {
    dft8<DIR>(v);
#pragma unroll
    for (int u = 0; u < 8; ++u) s[p * LD + pad_idx(8 * jj + u)] = v[u];
}

// Pencils per block: at least one butterfly task per thread, at most 80 KiB
// of LDS for the pencil tile (16 FP32 pencils of 512: the pencil-fastest
// stores of the strided passes then fill whole 128-byte lines), and no more
// than the N^2 pencils of one axis.
template <typename R, int N> constexpr int pencils_per_block() {
    constexpr int bytes = (int)sizeof(R) * 2;
    constexpr int by_lds = 81920 / (pencil_ld<N>() * bytes);
    constexpr int by_tasks = (2048 + N - 1) / N;
    constexpr int want = by_tasks > 16 ? by_tasks : 16;
    constexpr int gl = want < by_lds ? want : by_lds;
    constexpr int g = 1 << (31 - __builtin_clz(gl));          // power of two
    return g < N * N ? g : N * N;
}

}  // namespace bispec
