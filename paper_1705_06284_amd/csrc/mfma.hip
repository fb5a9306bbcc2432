// mfma.hip -- all-triplet contraction as an MFMA product-Gram (gfx950).
//
// The bispectrum numerators of Eq. (Jeong_BI), sum_n F_i F_j F_k for every
// i <= j <= k, are the entries of the product-Gram matrix
//
//     G[(i,j), k] = sum_n (F_i F_j)(n) F_k(n),
//
// a GEMM whose reduction dimension is the grid.  Rows are pair products
// (x,y): the (b,b) pairs first (pair tile 0 holds row (r,r) in lane r), then a
// cover of the requested triplets chosen on the host (each triplet is read
// from one of its three pairs), then rows (b, ONE) only when nb = 32.
// Columns are the bin fields F_k, k < 32; column nb < 32 is a field of ones,
// so G[(b,b), nb] = sum_n F_b^2 is the power-spectrum numerator of
// Eq. (Jeong_PS).  An optional extra tile holds the collapsed p = 4
// numerators sum_n F_a^2 F_b^2 (rows F_a^2, columns F_b^2), issued from the A
// operand of pair tile 0.
//
// MODE_SPLIT: each FP32 operand x is split into x_hi = bf16_rne(x) and
// x_lo = bf16_rne(x - x_hi) (the difference is exact in FP32); the product
// is A_hi B_hi + A_hi B_lo + A_lo B_hi on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation.  MODE_F32: the same GEMM on v_mfma_f32_32x32x2f32.
// Every block contracts one chunk of at most PG_CHUNK_TILES tiles and writes
// its FP64 tile partials; a fixed-order FP64 reduction over chunks follows
// (k_reduce_dense).  A chunk is at most 2048 split-mode MFMA steps, so the
// FP32 accumulators of split mode are converted only at the end of a chunk;
// FP32 mode (two points per step) adds its accumulators into FP64 registers
// every 32 MFMAs.  Triplets whose sums cancel strongly (ill-conditioned ones)
// are not read from these tiles but from an FP64 product-Gram over the bin
// fields (k_pgram_fields_f64).
//
// Lane layouts (checked on the device): for the 32x32x16 bf16 operation lane
// l holds A[l%32][8(l/32)+j] and B[8(l/32)+j][l%32], j < 8; for 32x32x2 f32
// lane l holds A[l%32][l/32] and B[l/32][l%32]; both write
// C[8(r/4)+4(l/32)+r%4][l%32] to accumulator register r.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fft_core.hpp"
#include "launch.hpp"

namespace bispec {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int PG_TK_TAIL = 512;           // grid points per LDS tile of the fused tail
// Block shapes of the fused tail (threads, output tiles per wave, points per
// LDS tile; tiles are at least one x-row of N points):
//   wide: 1024 threads, one tile per wave, 512 points (up to 16 pair
//         tiles, 4 waves per SIMD);
//   deep: 512 threads, up to three tiles per wave, 512 points (no prefetch:
//         its registers spilled, and without them the shape is 15 % faster);
//   twin: 512 threads, one tile per wave, 256 points (N <= 256, up to 8
//         pair tiles): half the LDS of the others, so two blocks share a CU
//         and one block's transforms overlap the other's contraction.
constexpr int PG_NT_WIDE = 1024, PG_MAXT_WIDE = 1;
constexpr int PG_NT_DEEP = 512, PG_MAXT_DEEP = 3;
constexpr int PG_NT_TWIN = 512, PG_MAXT_TWIN = 1, PG_TK_TWIN = 256;
constexpr bool PG_TWIN_PREFETCH = false;   // the co-resident block hides the loads
constexpr bool PG_WIDE_PREFETCH = false;   // the prefetch registers cost more (spills) than they hide
constexpr int PG_FLUSH_POINTS = 4096;     // FP32 mode: flush at least this often (whole tiles)
constexpr int PG_F32_FLUSH_STEPS = 32;    // FP32 mode: MFMAs (of 2 points) per FP32 accumulation span
constexpr int PG_ZERO = PG_ROW_ZERO;      // field row of zeros (padding rows)
constexpr int PG_ONE = PG_ROW_ONE;        // field row of ones (F_b * 1 rows)
constexpr int PG_FROWS = 34;

// x = hi + lo with hi = bf16_rne(x) and lo = bf16_rne(x - hi); x - hi is
// exact in FP32.
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

// Per-wave state of the product-Gram.  The work items are (pair tile, K
// part) pairs: with ksplit K parts, tile u / ksplit takes the 16-point steps
// s = kpart (mod ksplit) of every LDS tile, kpart = u mod ksplit.  Wave w owns
// items w + t WAVES (t < MAXT); with several items per wave, WAVES is a
// multiple of ksplit, so all items of a wave share one K part.
// The p = 4 tile (WANT_T; rows F_a^2, columns F_b^2) rides on pair tile 0,
// whose lane r < nb holds row (r, r): its A operand at lane r is F_r^2 at the
// lane's points, which is also what lane r must supply as the B operand of
// the p = 4 tile.  So the items of tile 0 add three more MFMAs with their own
// A halves as both operands (entries of rows or columns >= nb are unused).
template <int MODE, bool WANT_T, int NT, int MAXT>
struct PgState {
    static constexpr int WAVES = NT / 64;
    static constexpr int DT = MODE == PG_MODE_F32 ? MAXT + 1 : 1;    // FP64 flush registers (FP32 mode)
    int tile_of[MAXT];
    int kpart, ksplit;
    bool t_here;                          // WANT_T and one of this wave's items is tile 0
    uchar2 rp[MAXT];
    f32x16 acc[MAXT];
    f32x16 acct;                          // the p = 4 tile (when t_here)
    double dacc[DT][16];

    __device__ __forceinline__ void init(const uchar2 *__restrict__ pairs, int n_mtile, int nb, int wave, int col,
                                         int ks) {
        ksplit = ks;
        kpart = wave % ks;
        t_here = false;
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int u = wave + t * WAVES;
            const int tile = u / ks;
            tile_of[t] = tile < n_mtile ? tile : -1;
            t_here = t_here || (WANT_T && tile == 0);
            rp[t] = tile < n_mtile ? pairs[tile * 32 + col] : uchar2{PG_ZERO, PG_ZERO};
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) acct[r] = 0.0f;
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) dacc[t][r] = 0.0;
    }

    // Split-mode steps of this wave's K part.  HAS_T: t_here.
    template <int TK, int FS, bool HAS_T>
    __device__ __forceinline__ void contract_split(const float *Ft, const __bf16 *bh_row, const __bf16 *bl_row,
                                                   int half) {
#pragma unroll 1
        for (int s = kpart; s < TK / 16; s += ksplit) {
            const int kp = s * 16 + half * 8;
            const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&bh_row[kp]);
            const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&bl_row[kp]);
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                if (tile_of[t] < 0) continue;
                const float4 i0 = *reinterpret_cast<const float4 *>(&Ft[rp[t].x * FS + kp]);
                const float4 i1 = *reinterpret_cast<const float4 *>(&Ft[rp[t].x * FS + kp + 4]);
                const float4 j0 = *reinterpret_cast<const float4 *>(&Ft[rp[t].y * FS + kp]);
                const float4 j1 = *reinterpret_cast<const float4 *>(&Ft[rp[t].y * FS + kp + 4]);
                float a[8] = {i0.x * j0.x, i0.y * j0.y, i0.z * j0.z, i0.w * j0.w,
                              i1.x * j1.x, i1.y * j1.y, i1.z * j1.z, i1.w * j1.w};
                bf16x8 ah, al;
                split8(a, ah, al);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[t], 0, 0, 0);
                if (HAS_T && tile_of[t] == 0) {
                    acct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, ah, acct, 0, 0, 0);
                    acct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, al, acct, 0, 0, 0);
                    acct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, ah, acct, 0, 0, 0);
                }
            }
        }
    }

    // Contract TK points of the LDS field tile Ft (row stride FS); in split
    // mode bh_row/bl_row are this lane's column F_col in bf16 halves.
    template <int TK, int FS>
    __device__ __forceinline__ void contract(const float *Ft, const __bf16 *bh_row, const __bf16 *bl_row, int col,
                                             int half) {
        if constexpr (MODE == PG_MODE_SPLIT) {
            if (t_here)
                contract_split<TK, FS, WANT_T>(Ft, bh_row, bl_row, half);
            else
                contract_split<TK, FS, false>(Ft, bh_row, bl_row, half);
        } else {
            // every PG_F32_FLUSH_STEPS MFMAs (2 points each) the FP32
            // accumulators move into the FP64 ones, so each FP32 sum spans at
            // most 64 points of its K part
            int steps = 0;
#pragma unroll 1
            for (int s = kpart; s < TK / 2; s += ksplit) {
                const int k = 2 * s + half;
                const float bk = Ft[col * FS + k];
#pragma unroll
                for (int t = 0; t < MAXT; ++t) {
                    if (tile_of[t] < 0) continue;
                    const float a = Ft[rp[t].x * FS + k] * Ft[rp[t].y * FS + k];
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bk, acc[t], 0, 0, 0);
                    if (WANT_T && tile_of[t] == 0) acct = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, acct, 0, 0, 0);
                }
                if (++steps == PG_F32_FLUSH_STEPS) {
                    steps = 0;
                    flush();
                }
            }
        }
    }

    __device__ __forceinline__ void flush() {
        if constexpr (MODE == PG_MODE_F32) {
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    dacc[t][r] += (double)acc[t][r];
                    acc[t][r] = 0.0f;
                }
            }
            if (WANT_T) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    dacc[DT - 1][r] += (double)acct[r];
                    acct[r] = 0.0f;
                }
            }
        }
    }

    // The K parts of a tile are summed inside the block: parts 1..ksplit-1
    // leave their sums in scr ([ksplit-1][n_mtile + WANT_T][32][32] FP32,
    // over the LDS buffers once every tile is done), then part 0 adds them in
    // order and writes the block's FP64 partials [n_mtile + WANT_T][32][32]
    // (the p = 4 tile is tile n_mtile).  Called by every thread.
    __device__ __forceinline__ void write(double *__restrict__ partial, int64_t blk, int n_mtile, int col, int half,
                                          float *scr) {
        const int n_out = n_mtile + (WANT_T ? 1 : 0);
        auto own = [&](int t, int r) -> double {
            return (MODE == PG_MODE_F32 ? dacc[t < DT ? t : 0][r] : 0.0) + (double)acc[t][r];
        };
        auto own_t = [&](int r) -> double { return (MODE == PG_MODE_F32 ? dacc[DT - 1][r] : 0.0) + (double)acct[r]; };
        __syncthreads();
        if (kpart > 0) {
            float *o = scr + (int64_t)(kpart - 1) * n_out * 1024;
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                if (tile_of[t] < 0) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    o[tile_of[t] * 1024 + (8 * (r >> 2) + 4 * half + (r & 3)) * 32 + col] = (float)own(t, r);
            }
            if (WANT_T && t_here) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    o[n_mtile * 1024 + (8 * (r >> 2) + 4 * half + (r & 3)) * 32 + col] = (float)own_t(r);
            }
        }
        __syncthreads();
        if (kpart == 0) {
            double *base = partial + blk * n_out * 1024;
            auto put = [&](int tile, int r, double v) {
                const int e = tile * 1024 + (8 * (r >> 2) + 4 * half + (r & 3)) * 32 + col;
                for (int k = 1; k < ksplit; ++k) v += (double)scr[(int64_t)(k - 1) * n_out * 1024 + e];
                base[e] = v;
            };
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                if (tile_of[t] < 0) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) put(tile_of[t], r, own(t, r));
            }
            if (WANT_T && t_here) {
#pragma unroll
                for (int r = 0; r < 16; ++r) put(n_mtile, r, own_t(r));
            }
        }
    }
};

// Field rows nb..31 and the ZERO row hold 0, the ONE row holds 1; when
// nb < 32, row nb (a column of the product-Gram) holds 1 as well, so that
// G[(b,b), nb] = sum_n F_b^2.
template <int FS, int NT>
__device__ __forceinline__ void init_field_tile(float *Ft, int nb) {
    for (int e = threadIdx.x; e < (PG_FROWS - nb) * FS; e += NT) {
        const int row = nb + e / FS;
        Ft[row * FS + e % FS] = (row == PG_ONE || row == nb) ? 1.0f : 0.0f;
    }
}

// Fused last inverse pass + product-Gram.  A tile is TK = max(N, TKP) grid
// points: RT = TK/N consecutive x-rows (n_z, n_y).  For every row and shell
// pair the compact rows Bc[n_z][n_y][m_x + R] are placed at m_x mod N and
// transformed along x in LDS; the real and imaginary parts are the bin
// fields F_2q and F_2q+1 at the tile's points, contracted at once.
template <int MODE, bool WANT_T, int N, int NT, int MAXT, int TKP, int MINW, bool PREFETCH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW))) void k_tail(const float2 *__restrict__ bc, TailPairs tp, int nb,
                                             const uchar2 *__restrict__ pairs, int n_mtile,
                                             const float2 *__restrict__ tw, int tiles_per_blk, int ksplit,
                                             double *__restrict__ partial) {
    constexpr int TK = N >= TKP ? N : TKP;
    constexpr int RT = TK / N;
    constexpr int G = 16 * RT;                 // pencil slots: 16 pairs x RT rows
    constexpr int FS = TK + 4, BS = TK + 8;
    constexpr int LDP = pencil_ld<N>();
    constexpr int FFT_BYTES = G * LDP * 8;
    constexpr int SPLIT_BYTES = MODE == PG_MODE_SPLIT ? 2 * 32 * BS * 2 : 0;
    constexpr int UBYTES = FFT_BYTES > SPLIT_BYTES ? FFT_BYTES : SPLIT_BYTES;
    constexpr int PF = G * N / NT;             // loaded elements per thread and tile
    static_assert((G * N) % NT == 0, "tile loads must divide the block");
    constexpr int CBS = MODE == PG_MODE_SPLIT ? 2 * BS : 8;
    __shared__ float Ft[PG_FROWS * FS];
    __shared__ __attribute__((aligned(16))) unsigned char ubuf[UBYTES];
    __shared__ float2 tws[N];
    __shared__ __attribute__((aligned(16))) __bf16 Bconst[CBS];   // bf16 rows of ones and of zeros
    float2 *fb = reinterpret_cast<float2 *>(ubuf);
    __bf16 *Bh = reinterpret_cast<__bf16 *>(ubuf);       // over the FFT buffer once it is read
    __bf16 *Bl = Bh + 32 * BS;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, kept in SGPRs
    const int col = lane & 31, half = lane >> 5;
    const int map = blockIdx.y;
    const int64_t nrow = (int64_t)N * N;
    const int64_t total = (int64_t)N * N * N / TK;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_blk;
    const int64_t t_end = t_begin + tiles_per_blk < total ? t_begin + tiles_per_blk : total;
    for (int i = tid; i < N; i += NT) tws[i] = tw[i];
    for (int i = tid; i < CBS; i += NT) Bconst[i] = (__bf16)(i < CBS / 2 ? 1.0f : 0.0f);
    PgState<MODE, WANT_T, NT, MAXT> st;
    st.init(pairs, n_mtile, nb, wave, col, ksplit);
    init_field_tile<FS, NT>(Ft, nb);
    // This lane's column operand F_col in bf16 halves: the tile's split field,
    // or for col >= nb the constant column (ones at col = nb, else zeros).
    const __bf16 *bh_row = col < nb ? Bh + col * BS : (col == nb ? Bconst : Bconst + CBS / 2);
    const __bf16 *bl_row = col < nb ? Bl + col * BS : Bconst + CBS / 2;

    // Slot sl = q RT + r holds pair q of tile row r; only the first
    // npairs RT slots are loaded, transformed and read.
    static_assert(NT % N == 0, "block size must be a multiple of the row length");
    const int gact = tp.npairs * RT;
    // The last pass writes the fields straight into the tile: F_2q and
    // F_2q+1 in FP32 and, in split mode, their bf16 halves (which overwrite
    // the FFT buffer after the pass has read it).
    auto store = [&](int sl, int n, float2 f) {
        const int q = sl / RT, r = sl % RT;
        const int i = r * N + n;
        const bool odd = 2 * q + 1 < nb;
        Ft[(2 * q) * FS + i] = f.x;
        if (odd) Ft[(2 * q + 1) * FS + i] = f.y;
        if constexpr (MODE == PG_MODE_SPLIT) {
            bf16x2 h, l;
            split2(f.x, f.y, h, l);
            Bh[(2 * q) * BS + i] = h[0];
            Bl[(2 * q) * BS + i] = l[0];
            if (odd) {
                Bh[(2 * q + 1) * BS + i] = h[1];
                Bl[(2 * q + 1) * BS + i] = l[1];
            }
        }
    };
    int since_flush = 0;
    if constexpr (N >= 16) {
        // The loads feed the first radix-8 pass directly: task (slot p,
        // butterfly jj) loads x[jj + t N/8], t < 8, from the compact row
        // (zero where |m_x| > R), so the first pass reads no LDS.  A task's
        // row base, stride and radius are fixed over the tiles.
        constexpr int NB1 = N / 8;
        constexpr int T1 = G * NB1;
        constexpr int PER1 = T1 < NT ? 1 : T1 / NT;
        static_assert(T1 % NT == 0 || T1 < NT, "first-pass tasks must fill the block or fit in it");
        int64_t fbase[PER1];
        int fw[PER1], fr[PER1];
        bool fact[PER1];
#pragma unroll
        for (int k = 0; k < PER1; ++k) {
            const int task = tid + k * NT;
            const int p = task / NB1;
            const int q = p / RT, r = p % RT;
            fact[k] = (T1 >= NT || tid < T1) && p < gact;
            fw[k] = fact[k] ? tp.W[q] : 0;
            fr[k] = fact[k] ? tp.R[q] : -1;
            fbase[k] = fact[k] ? tp.off[q] + (map * nrow + r) * fw[k] + fr[k] : 0;
        }
        auto fetch = [&](int64_t tile, float2 (*v)[8]) {
#pragma unroll
            for (int k = 0; k < PER1; ++k) {
                const int jj = (tid + k * NT) % NB1;
                const int64_t row = fbase[k] + tile * RT * fw[k];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int mx = signed_freq(jj + t * NB1, N);
                    v[k][t] = float2{0.0f, 0.0f};
                    if (mx >= -fr[k] && mx <= fr[k]) v[k][t] = bc[row + mx];
                }
            }
        };
        // PREFETCH: the loads of tile t + 1 are issued right after tile t's
        // first pass and stay in flight through its transform and
        // contraction (else a co-resident block hides their latency).
        float2 v[PER1][8];
        if (PREFETCH && t_begin < t_end) fetch(t_begin, v);
        for (int64_t tile = t_begin; tile < t_end; ++tile) {
            if (!PREFETCH) fetch(tile, v);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PER1; ++k) {
                const int task = tid + k * NT;
                if (fact[k]) first_pass_butterfly<float2, N, LDP, +1>(fb, task / NB1, task % NB1, v[k]);
            }
            if (PREFETCH && tile + 1 < t_end) fetch(tile + 1, v);
            __syncthreads();
            fft_pencils_to<float2, N, LDP, G, +1, NT, true>(fb, tws, gact, store);
            st.template contract<TK, FS>(Ft, bh_row, bl_row, col, half);
            since_flush += TK;
            if (since_flush >= PG_FLUSH_POINTS) {
                since_flush = 0;
                st.flush();
            }
        }
    } else {
        // N = 8: the one radix-8 pass is also the last.  Element k of this
        // thread's share of a tile is e = tid + k NT: slot e / N at
        // position tid % N; a wave covers 64/N consecutive rows of one pair.
        const int mx = signed_freq(tid % N, N);
        auto fetch = [&](int64_t tile, float2 *v) {
            const int64_t row0 = tile * RT;
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int sl = tid / N + k * (NT / N);
                const int q = __builtin_amdgcn_readfirstlane(sl / RT);
                const int r = sl % RT;
                v[k] = float2{0.0f, 0.0f};
                if (q < tp.npairs) {
                    const int R = tp.R[q];
                    if (mx >= -R && mx <= R) v[k] = bc[tp.off[q] + (map * nrow + row0 + r) * tp.W[q] + mx + R];
                }
            }
        };
        float2 v[PF];
        for (int64_t tile = t_begin; tile < t_end; ++tile) {
            fetch(tile, v);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int e = tid + k * NT;
                if (e / N < gact) fb[(e / N) * LDP + pad_idx(e % N)] = v[k];
            }
            __syncthreads();
            fft_pencils_to<float2, N, LDP, G, +1, NT>(fb, tws, gact, store);
            st.template contract<TK, FS>(Ft, bh_row, bl_row, col, half);
            since_flush += TK;
            if (since_flush >= PG_FLUSH_POINTS) {
                since_flush = 0;
                st.flush();
            }
        }
    }
    st.write(partial, (int64_t)map * gridDim.x + blockIdx.x, n_mtile, col, half, reinterpret_cast<float *>(ubuf));
}

// Product-Gram over bin fields resident in HBM, for plans of 33..128 bins
// (narrow shells): G[(x,y), z] = sum_n (F_x F_y)(n) F_z(n) in split-BF16.
// One launch covers one group of 64 columns, fields col0 .. col0 + 63 (two
// 32-column MFMA tiles; columns at or beyond nb are zero), and the pair rows
// chosen for that group.  Block (c, map, g) contracts the points
// [c chunk, (c+1) chunk) for the pair tiles g T .. (g+1) T - 1
// of the group (T = PGF_TILES = 32); each of the 16 waves owns the tiles
// g T + w + r WAVES, r < 2.  With ZR = 128 a step stages pgf_tk(ZR, SQ) = 64
// points (the stage of 128 fields at 128 points would leave the registers
// for one accumulator pair only).
// Every step stages pgf_tk points of each field in LDS, all nb in FP32 for
// the row products and the group's columns as bf16 halves, so one split of a
// row product feeds both column tiles; the next step's loads are in flight
// during a step's contraction.  A chunk is at most PGF_MAX_CHUNK points, the
// split-mode span of FP32 accumulation; the block writes its FP64 tile
// partials into tiles tile0 .. tile0 + n_mtile - 1 of its set of
// tiles_total tiles (its own tiles only).  ZR: the zero row of the FP32
// stage (64 for plans of up to 64 bins, else 128).
// SQ: the product-Gram of the squares instead, rows (a,a) for a < nb (tile t
// row r is a = 32 t + r) against the columns F_b^2 of the group, and a column
// of ones at b = nb when nb - col0 < 64: G[(a,a), b] = sum_n F_a^2 F_b^2 (the
// collapsed p = 4 numerators) and G[(a,a), nb] = sum_n F_a^2 (the P
// numerators).  Its few row tiles would leave most waves idle, so the waves
// split the K steps instead: wave w takes tile w % n_mtile and the steps
// s = w / n_mtile (mod KS), KS = WAVES / n_mtile, and each K part writes its
// own partial set (partial [batch][nblk][KS][tiles_total][32][64]); the
// fixed-order reduction over nblk KS sets adds them.
constexpr int PGF_NT = 1024, PGF_TK = 128, PGF_TILES = 32;
__host__ __device__ constexpr int pgf_maxr(int zr, bool sq) { return sq && zr == PGF_ROW_ZERO_XL ? 1 : 2; }
__host__ __device__ constexpr int pgf_tk(int zr, bool sq) { return zr == PGF_ROW_ZERO_XL && !sq ? 64 : PGF_TK; }
static_assert(PGF_NT / 64 * pgf_maxr(PGF_ROW_ZERO, false) == PGF_TILES &&
                  PGF_NT / 64 * pgf_maxr(PGF_ROW_ZERO_XL, false) == PGF_TILES,
              "every triplet-pass block holds PGF_TILES pair tiles");

template <bool SQ, int ZR>
__global__ __launch_bounds__(PGF_NT) void k_pgram_fields(const float *__restrict__ fields, int64_t npix, int nb,
                                                         int64_t map_stride, const uchar2 *__restrict__ pairs,
                                                         int n_mtile, int col0, int tile0, int tiles_total,
                                                         int64_t chunk, double *__restrict__ partial) {
    constexpr int NT = PGF_NT;
    constexpr int TK = pgf_tk(ZR, SQ), FS = TK + 4, BS = TK + 8, WAVES = NT / 64, MAXR = pgf_maxr(ZR, SQ);
    static_assert(PGF_TK % TK == 0, "a chunk holds whole steps");
    __shared__ __attribute__((aligned(16))) float Ft[(ZR + 1) * FS];   // field rows, then a row of zeros
    __shared__ __attribute__((aligned(16))) __bf16 Bh[64 * BS];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[64 * BS];
    static_assert((BS * 2) % 16 == 0, "bf16 rows must keep 16-byte alignment");
    const int tid = threadIdx.x, lane = tid & 63, col = lane & 31, half = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int map = blockIdx.y;
    // rows nb..ZR-1 and the zero row are never loaded: zero them once
    for (int i = tid; i < (ZR + 1 - nb) * FS; i += NT) Ft[nb * FS + i] = 0.0f;
    // the group's column fields col0 .. col0 + ncf - 1; SQ: column nb - col0
    // is the ones column when it falls in the group
    const int ncf = nb - col0 < 64 ? nb - col0 : 64;
    const int one_col = SQ && nb - col0 < 64 ? nb - col0 : -1;
    const int zr = one_col >= 0 ? ncf + 1 : ncf;
    for (int i = tid; i < (64 - zr) * BS; i += NT) {
        Bh[zr * BS + i] = (__bf16)0.0f;
        Bl[zr * BS + i] = (__bf16)0.0f;
    }
    if (one_col >= 0)
        for (int i = tid; i < BS; i += NT) {
            Bh[one_col * BS + i] = (__bf16)1.0f;
            Bl[one_col * BS + i] = (__bf16)0.0f;
        }
    int tile_of[MAXR];
    uchar2 rp[MAXR];
    f32x16 acc[MAXR][2];
    const int ks = SQ ? WAVES / n_mtile : 1;           // K parts (SQ: n_mtile divides WAVES)
    const int kpart = SQ ? wave / n_mtile : 0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if constexpr (SQ) {
            const int t = wave % n_mtile, a = t * 32 + col;
            tile_of[r] = r == 0 ? t : -1;
            rp[r] = a < nb ? uchar2{(unsigned char)a, (unsigned char)a} : uchar2{ZR, ZR};
        } else {
            const int t = blockIdx.z * PGF_TILES + wave + r * WAVES;
            tile_of[r] = t < n_mtile ? t : -1;
            rp[r] = t < n_mtile ? pairs[t * 32 + col] : uchar2{ZR, ZR};
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            acc[r][0][i] = 0.0f;
            acc[r][1][i] = 0.0f;
        }
    }
    const float *f = fields + (int64_t)map * map_stride;
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = p0 + chunk < npix ? p0 + chunk : npix;
    // the loads of step p + TK are issued before step p's contraction and
    // land in registers; after the step they go to LDS
    constexpr int LPT = ZR * (TK / 4) / NT;   // float4 per thread at ZR bins
    static_assert(ZR * (TK / 4) % NT == 0, "field loads must divide the block");
    float4 pre[LPT];
    auto fetch = [&](int64_t p) {
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = tid + j * NT;
            if (e < nb * (TK / 4)) {
                const int b = e / (TK / 4), k = (e % (TK / 4)) * 4;
                pre[j] = *reinterpret_cast<const float4 *>(f + (int64_t)b * npix + p + k);
            }
        }
    };
    if (p0 < p1) fetch(p0);
    for (int64_t p = p0; p < p1; p += TK) {
        __syncthreads();   // the previous step's reads are done
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = tid + j * NT;
            if (e >= nb * (TK / 4)) continue;
            const int b = e / (TK / 4), k = (e % (TK / 4)) * 4;
            const float4 v = pre[j];
            *reinterpret_cast<float4 *>(&Ft[b * FS + k]) = v;
            const int c = b - col0;
            if (c < 0 || c >= 64) continue;
            const float4 w = SQ ? float4{v.x * v.x, v.y * v.y, v.z * v.z, v.w * v.w} : v;
            bf16x2 h0, l0, h1, l1;
            split2(w.x, w.y, h0, l0);
            split2(w.z, w.w, h1, l1);
            // 8-byte stores: (c BS + k) 2 bytes is a multiple of 8 (BS = TK + 8, k = 0 mod 4)
            *reinterpret_cast<bf16x4 *>(&Bh[c * BS + k]) = bf16x4{h0[0], h0[1], h1[0], h1[1]};
            *reinterpret_cast<bf16x4 *>(&Bl[c * BS + k]) = bf16x4{l0[0], l0[1], l1[0], l1[1]};
        }
        __syncthreads();
        if (p + TK < p1) fetch(p + TK);
#pragma unroll 1
        for (int s = kpart; s < TK / 16; s += ks) {
            const int kp = s * 16 + half * 8;
            const bf16x8 bh0 = *reinterpret_cast<const bf16x8 *>(&Bh[col * BS + kp]);
            const bf16x8 bl0 = *reinterpret_cast<const bf16x8 *>(&Bl[col * BS + kp]);
            const bf16x8 bh1 = *reinterpret_cast<const bf16x8 *>(&Bh[(32 + col) * BS + kp]);
            const bf16x8 bl1 = *reinterpret_cast<const bf16x8 *>(&Bl[(32 + col) * BS + kp]);
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                if (tile_of[r] < 0) continue;
                const float4 i0 = *reinterpret_cast<const float4 *>(&Ft[rp[r].x * FS + kp]);
                const float4 i1 = *reinterpret_cast<const float4 *>(&Ft[rp[r].x * FS + kp + 4]);
                const float4 j0 = *reinterpret_cast<const float4 *>(&Ft[rp[r].y * FS + kp]);
                const float4 j1 = *reinterpret_cast<const float4 *>(&Ft[rp[r].y * FS + kp + 4]);
                float a[8] = {i0.x * j0.x, i0.y * j0.y, i0.z * j0.z, i0.w * j0.w,
                              i1.x * j1.x, i1.y * j1.y, i1.z * j1.z, i1.w * j1.w};
                bf16x8 ah, al;
                split8(a, ah, al);
                acc[r][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh0, acc[r][0], 0, 0, 0);
                acc[r][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh1, acc[r][1], 0, 0, 0);
                acc[r][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl0, acc[r][0], 0, 0, 0);
                acc[r][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl1, acc[r][1], 0, 0, 0);
                acc[r][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh0, acc[r][0], 0, 0, 0);
                acc[r][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh1, acc[r][1], 0, 0, 0);
            }
        }
    }
    double *base = partial + (((int64_t)map * gridDim.x + blockIdx.x) * ks + kpart) * ((int64_t)tiles_total * 2048) +
                   (int64_t)tile0 * 2048;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (tile_of[r] < 0) continue;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = 8 * (i >> 2) + 4 * half + (i & 3);
            base[tile_of[r] * 2048 + row * 64 + col] = (double)acc[r][0][i];
            base[tile_of[r] * 2048 + row * 64 + 32 + col] = (double)acc[r][1][i];
        }
    }
}

// The same product-Gram on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
// for the rows of ill-conditioned triplets, whose sums cancel so strongly
// that FP32 (or split-BF16) rounding of the products and their accumulation
// would show: the pair product of two FP32 fields is exact in FP64, and so
// are the products with the column fields up to FP64 rounding.  64 columns
// (fields col0 .. col0 + 63 of one column group; columns at or beyond nb are
// zero).  Block (c, map, g) contracts the points [c chunk, (c+1) chunk) for
// the 32-row pair tile g WAVES + w of wave w.
// Each step stages PGF64_TK points of every field in LDS; one K step (4
// points) is 8 MFMAs 16x16x4: row halves (lanes l % 16 and 16 + l % 16) times
// the four 16-column quarters.  Lane layout (checked on the device): lane l
// feeds A[l % 16][l / 16] and B[l / 16][l % 16], and holds
// C[4 r + l / 16][l % 16] in accumulator register r.  Partials
// [batch][nblk][tiles_total][32][64] FP64 (this launch: tiles tile0 ..
// tile0 + n_mtile - 1), as the split kernel writes them.
constexpr int PGF64_NT = 256, PGF64_TK = 128;
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int ZR>
__global__ __launch_bounds__(PGF64_NT) void k_pgram_fields_f64(const float *__restrict__ fields, int64_t npix,
                                                               int nb, int64_t map_stride,
                                                               const uchar2 *__restrict__ pairs, int n_mtile,
                                                               int col0, int tile0, int tiles_total, int64_t chunk,
                                                               double *__restrict__ partial) {
    constexpr int TK = PGF64_TK, FS = TK + 4, WAVES = PGF64_NT / 64;
    __shared__ __attribute__((aligned(16))) float Ft[(ZR + 1) * FS];
    const int tid = threadIdx.x, lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int map = blockIdx.y;
    for (int i = tid; i < (ZR + 1 - nb) * FS; i += PGF64_NT) Ft[nb * FS + i] = 0.0f;
    const int tile = blockIdx.z * WAVES + wave;
    const bool live = tile < n_mtile;
    const uchar2 zero = uchar2{ZR, ZR};
    // column c of quarter q reads field row col0 + 16 q + c (the zero row past nb)
    int brow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) brow[q] = col0 + 16 * q + r16 < nb ? col0 + 16 * q + r16 : ZR;
    const uchar2 rp0 = live ? pairs[tile * 32 + r16] : zero;
    const uchar2 rp1 = live ? pairs[tile * 32 + 16 + r16] : zero;
    f64x4 c[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[h][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    const float *f = fields + (int64_t)map * map_stride;
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = p0 + chunk < npix ? p0 + chunk : npix;
    constexpr int LPT = ZR * (TK / 4) / PGF64_NT;   // float4 per thread at ZR bins
    static_assert(ZR * (TK / 4) % PGF64_NT == 0, "field loads must divide the block");
    for (int64_t p = p0; p < p1; p += TK) {
        float4 v[LPT];
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = tid + j * PGF64_NT;
            if (e < nb * (TK / 4)) {
                const int b = e / (TK / 4), k = (e % (TK / 4)) * 4;
                v[j] = *reinterpret_cast<const float4 *>(f + (int64_t)b * npix + p + k);
            }
        }
        __syncthreads();   // the previous step's reads are done
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = tid + j * PGF64_NT;
            if (e < nb * (TK / 4)) {
                const int b = e / (TK / 4), k = (e % (TK / 4)) * 4;
                *reinterpret_cast<float4 *>(&Ft[b * FS + k]) = v[j];
            }
        }
        __syncthreads();
        if (!live) continue;
#pragma unroll 2
        for (int s = 0; s < TK / 4; ++s) {
            const int k = 4 * s + kq;
            const double a0 = (double)Ft[rp0.x * FS + k] * (double)Ft[rp0.y * FS + k];
            const double a1 = (double)Ft[rp1.x * FS + k] * (double)Ft[rp1.y * FS + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double b = (double)Ft[brow[q] * FS + k];
                c[0][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, c[0][q], 0, 0, 0);
                c[1][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, c[1][q], 0, 0, 0);
            }
        }
    }
    if (!live) return;
    double *base = partial + ((int64_t)map * gridDim.x + blockIdx.x) * ((int64_t)tiles_total * 2048) +
                   (int64_t)(tile0 + tile) * 2048;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) base[(16 * h + 4 * r + kq) * 64 + 16 * q + r16] = c[h][q][r];
}

// Fixed-order compensated FP64 sum over blocks of every dense tile entry,
// in segments: out[map][z][e] = sum_{b in segment z} partial[map][b][e],
// segment z = [z seg, min((z+1) seg, nblk)) for z = blockIdx.z.  Consecutive
// threads read consecutive entries, so every partial is read once, coalesced.
__global__ __launch_bounds__(256) void k_reduce_dense(const double *__restrict__ partial, int nblk, int seg,
                                                      int64_t n_dense, double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int map = blockIdx.y, z = blockIdx.z;
    if (e >= n_dense) return;
    const double *p = partial + (int64_t)map * nblk * n_dense + e;
    const int b0 = z * seg, b1 = b0 + seg < nblk ? b0 + seg : nblk;
    double acc = 0.0, comp = 0.0;
#pragma unroll 8
    for (int b = b0; b < b1; ++b) {
        const double x = p[(int64_t)b * n_dense];
        const double s = acc + x;
        comp += fabs(acc) >= fabs(x) ? (acc - s) + x : (x - s) + acc;
        acc = s;
    }
    out[((int64_t)map * gridDim.z + z) * n_dense + e] = acc + comp;
}

// Fixed-order FP64 sum over blocks of the dense tile partials, gathered at
// idx[t] and scaled: segment layout as in k_finalize.
__global__ __launch_bounds__(256) void k_finalize_gather(const double *__restrict__ partial, int nblk,
                                                         int64_t blk_stride, const double *__restrict__ alt,
                                                         int64_t alt_stride, const int *__restrict__ idx, int nterm,
                                                         const double *__restrict__ scale, double *o0, int n0,
                                                         double *o1, int n1, double *o2, int n2) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int map = blockIdx.y;
    if (t >= nterm) return;
    // entries flagged PG_IDX_ALT live in the refinement pass's dense tiles
    const int it = idx[t];
    const bool in_alt = (it & PG_IDX_ALT) != 0;
    if (in_alt) blk_stride = alt_stride;
    const double *p = in_alt ? alt + (int64_t)map * nblk * alt_stride + (it & ~PG_IDX_ALT)
                             : partial + (int64_t)map * nblk * blk_stride + it;
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

int64_t tail_units(int n) { return (int64_t)n * n * n / PG_TK_TAIL; }

bool tail_shape_fits(int n, int n_mtile, bool want_t, int shape) {
    (void)want_t;                      // the p = 4 tile rides on pair tile 0
    const int n_out = n_mtile;
    switch (shape) {
        case PG_SHAPE_WIDE: return n_out <= PG_MAXT_WIDE * (PG_NT_WIDE / 64);
        case PG_SHAPE_DEEP: return n_out <= PG_MAXT_DEEP * (PG_NT_DEEP / 64);
        case PG_SHAPE_TWIN: return n <= PG_TK_TWIN && n_out <= PG_MAXT_TWIN * (PG_NT_TWIN / 64);
        default: return false;
    }
}

int tail_shape(int n, int n_mtile, bool want_t, int shape) {
    if (tail_shape_fits(n, n_mtile, want_t, shape)) return shape;
    return tail_shape_fits(n, n_mtile, want_t, PG_SHAPE_WIDE) ? PG_SHAPE_WIDE : PG_SHAPE_DEEP;
}

// Bytes of the FFT buffer of a shape (the LDS the K-part sums may reuse).
int tail_fft_bytes(int n, int shape) {
    const int tkp = shape == PG_SHAPE_TWIN ? PG_TK_TWIN : PG_TK_TAIL;
    const int tk = n >= tkp ? n : tkp;
    return 16 * (tk / n) * (n + n / 8 + 1) * 8;
}

int tail_ksplit(int n, int n_mtile, bool want_t, int shape) {
    const int n_out = n_mtile;
    const int sh = tail_shape(n, n_mtile, want_t, shape);
    const int nt = sh == PG_SHAPE_WIDE ? PG_NT_WIDE : sh == PG_SHAPE_DEEP ? PG_NT_DEEP : PG_NT_TWIN;
    const int maxt = sh == PG_SHAPE_WIDE ? PG_MAXT_WIDE : sh == PG_SHAPE_DEEP ? PG_MAXT_DEEP : PG_MAXT_TWIN;
    const int waves = nt / 64, cap = maxt * waves;
    // the sums of K parts 1.. must fit the FFT buffer
    const int scr_tiles = tail_fft_bytes(n, sh) / 4096;
    const int parts = n_mtile + (want_t ? 1 : 0);
    auto fits = [&](int k) { return (k - 1) * parts <= scr_tiles; };
    // one item per wave: any count of K parts; several: a power of two that
    // divides the wave count (all items of a wave then share one K part)
    if (maxt == 1) {
        int k = std::max(1, std::min(waves / n_out, PG_TK_TAIL / 32));
        while (k > 1 && !fits(k)) --k;
        return k;
    }
    int k = 1;
    while (2 * k <= waves && n_out * 2 * k <= cap && fits(2 * k)) k *= 2;
    return k;
}

template <int MODE, bool WANT_T>
hipError_t launch_tail_m(const float2 *bc, const TailPairs &tp, int n, int nb, int batch, const uchar2 *pairs,
                         int n_mtile, const float2 *tw, int nblk, double *partial, hipStream_t st, int shape) {
    const int sh = tail_shape(n, n_mtile, WANT_T, shape);
    const int ks = tail_ksplit(n, n_mtile, WANT_T, shape);
    const int64_t units = tail_units(n);
    const int per = (int)((units + nblk - 1) / nblk);       // 512-point units per block
    if (nblk < 1 || per > PG_CHUNK_TILES) return hipErrorInvalidValue;
    auto go = [&](auto nc) -> hipError_t {
        constexpr int NN = decltype(nc)::value;
        constexpr int TKW = NN >= PG_TK_TAIL ? NN : PG_TK_TAIL;
        const int per_w = (int)((int64_t)per * PG_TK_TAIL / TKW);
        if (sh == PG_SHAPE_WIDE)
            hipLaunchKernelGGL((k_tail<MODE, WANT_T, NN, PG_NT_WIDE, PG_MAXT_WIDE, PG_TK_TAIL, 4, PG_WIDE_PREFETCH>), dim3(nblk, batch),
                               dim3(PG_NT_WIDE), 0, st, bc, tp, nb, pairs, n_mtile, tw, per_w, ks, partial);
        else if (sh == PG_SHAPE_DEEP)
            hipLaunchKernelGGL((k_tail<MODE, WANT_T, NN, PG_NT_DEEP, PG_MAXT_DEEP, PG_TK_TAIL, 2, false>), dim3(nblk, batch),
                               dim3(PG_NT_DEEP), 0, st, bc, tp, nb, pairs, n_mtile, tw, per_w, ks, partial);
        else if constexpr (NN <= PG_TK_TWIN) {
            constexpr int TKT = NN >= PG_TK_TWIN ? NN : PG_TK_TWIN;
            const int per_t = (int)((int64_t)per * PG_TK_TAIL / TKT);
            hipLaunchKernelGGL((k_tail<MODE, WANT_T, NN, PG_NT_TWIN, PG_MAXT_TWIN, PG_TK_TWIN, 4, PG_TWIN_PREFETCH>), dim3(nblk, batch),
                               dim3(PG_NT_TWIN), 0, st, bc, tp, nb, pairs, n_mtile, tw, per_t, ks, partial);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    };
    switch (n) {
        case 8: return go(std::integral_constant<int, 8>{});
        case 16: return go(std::integral_constant<int, 16>{});
        case 32: return go(std::integral_constant<int, 32>{});
        case 64: return go(std::integral_constant<int, 64>{});
        case 128: return go(std::integral_constant<int, 128>{});
        case 256: return go(std::integral_constant<int, 256>{});
        case 512: return go(std::integral_constant<int, 512>{});
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tail(int mode, bool want_t, const float2 *bc, const TailPairs &tp, int n, int nb, int batch,
                       const uchar2 *pairs, int n_mtile, const float2 *tw, int nblk, double *partial,
                       hipStream_t st, int shape) {
    if (nb > 32 || tp.npairs > 16 || !tail_shape_fits(n, n_mtile, want_t, PG_SHAPE_DEEP)) return hipErrorInvalidValue;
    if (mode == PG_MODE_SPLIT)
        return want_t ? launch_tail_m<PG_MODE_SPLIT, true>(bc, tp, n, nb, batch, pairs, n_mtile, tw, nblk, partial, st,
                                                           shape)
                      : launch_tail_m<PG_MODE_SPLIT, false>(bc, tp, n, nb, batch, pairs, n_mtile, tw, nblk, partial,
                                                            st, shape);
    return want_t ? launch_tail_m<PG_MODE_F32, true>(bc, tp, n, nb, batch, pairs, n_mtile, tw, nblk, partial, st,
                                                     shape)
                  : launch_tail_m<PG_MODE_F32, false>(bc, tp, n, nb, batch, pairs, n_mtile, tw, nblk, partial, st,
                                                      shape);
}

int pgram_fields_kparts(int n_mtile, bool squares) { return squares ? PGF_NT / 64 / n_mtile : 1; }

int pgf_sq_tiles(int nb) {
    const int t = (nb + 31) / 32;
    return t <= 2 ? t : 4;
}

int64_t pgram_fields_chunk(int64_t npix, int nblk) {
    const int64_t c = (npix + nblk - 1) / nblk;
    return (c + PGF_TK - 1) / PGF_TK * PGF_TK;
}

hipError_t launch_pgram_fields(const float *fields, int64_t npix, int nb, int batch, const uchar2 *pairs, int n_mtile,
                               int col0, int tile0, int tiles_total, int nblk, double *partial, hipStream_t st,
                               bool squares) {
    if (nb < 1 || nb > PGF_MAX_BINS || n_mtile < 1 || nblk < 1 || batch < 1) return hipErrorInvalidValue;
    if (col0 < 0 || col0 % 64 != 0 || col0 >= nb || tile0 < 0 || tile0 + n_mtile > tiles_total)
        return hipErrorInvalidValue;
    if (squares ? (n_mtile != pgf_sq_tiles(nb) || (PGF_NT / 64) % n_mtile != 0) : !pairs) return hipErrorInvalidValue;
    const int64_t chunk = pgram_fields_chunk(npix, nblk);
    if (npix % PGF_TK != 0 || chunk > PGF_MAX_CHUNK) return hipErrorInvalidValue;
    const unsigned groups = squares ? 1u : (unsigned)((n_mtile + PGF_TILES - 1) / PGF_TILES);
    const int64_t ms = (int64_t)nb * npix;
    if (nb <= PGF_ROW_ZERO) {
        if (squares)
            hipLaunchKernelGGL((k_pgram_fields<true, PGF_ROW_ZERO>), dim3(nblk, batch, groups), dim3(PGF_NT), 0, st,
                               fields, npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
        else
            hipLaunchKernelGGL((k_pgram_fields<false, PGF_ROW_ZERO>), dim3(nblk, batch, groups), dim3(PGF_NT), 0, st,
                               fields, npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
    } else {
        if (squares)
            hipLaunchKernelGGL((k_pgram_fields<true, PGF_ROW_ZERO_XL>), dim3(nblk, batch, groups), dim3(PGF_NT), 0,
                               st, fields, npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
        else
            hipLaunchKernelGGL((k_pgram_fields<false, PGF_ROW_ZERO_XL>), dim3(nblk, batch, groups), dim3(PGF_NT), 0,
                               st, fields, npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_dense(const double *partial, int nblk, int64_t n_dense, int batch, double *dense,
                               double *tmp, hipStream_t st) {
    const unsigned gx = (unsigned)((n_dense + 255) / 256);
    if (nblk <= 2 * PG_REDUCE_SEGS || !tmp) {
        hipLaunchKernelGGL(k_reduce_dense, dim3(gx, batch, 1), dim3(256), 0, st, partial, nblk, nblk, n_dense, dense);
        return hipGetLastError();
    }
    // PG_REDUCE_SEGS segment sums, then their sum (both in a fixed order)
    const int seg = (nblk + PG_REDUCE_SEGS - 1) / PG_REDUCE_SEGS;
    const int nseg = (nblk + seg - 1) / seg;
    hipLaunchKernelGGL(k_reduce_dense, dim3(gx, batch, nseg), dim3(256), 0, st, partial, nblk, seg, n_dense, tmp);
    hipLaunchKernelGGL(k_reduce_dense, dim3(gx, batch, 1), dim3(256), 0, st, (const double *)tmp, nseg, nseg, n_dense,
                       dense);
    return hipGetLastError();
}

hipError_t launch_finalize_gather(const double *partial, int nblk, int64_t blk_stride, const double *alt,
                                  int64_t alt_stride, const int *idx, int nterm, int batch, const double *scale,
                                  double *o0, int n0, double *o1, int n1, double *o2, int n2, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_gather, dim3((nterm + 255) / 256, batch), dim3(256), 0, st, partial, nblk,
                       blk_stride, alt, alt_stride, idx, nterm, scale, o0, n0, o1, n1, o2, n2);
    return hipGetLastError();
}

// out[map][t] = scale[t] * alt[map][idx[t] & ~PG_IDX_ALT] for the listed t.
__global__ __launch_bounds__(256) void k_scatter_alt(const double *__restrict__ alt, int64_t alt_stride,
                                                     const int *__restrict__ idx, const double *__restrict__ scale,
                                                     const int *__restrict__ list, int nlist,
                                                     double *__restrict__ out, int nout) {
    const int i = blockIdx.x * 256 + threadIdx.x, map = blockIdx.y;
    if (i >= nlist) return;
    const int t = list[i];
    out[(int64_t)map * nout + t] = scale[t] * alt[(int64_t)map * alt_stride + (idx[t] & ~PG_IDX_ALT)];
}

hipError_t launch_scatter_alt(const double *alt, int64_t alt_stride, const int *idx, const double *scale,
                              const int *list, int nlist, int batch, double *out, int nout, hipStream_t st) {
    if (nlist < 1) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_alt, dim3((nlist + 255) / 256, batch), dim3(256), 0, st, alt, alt_stride, idx, scale,
                       list, nlist, out, nout);
    return hipGetLastError();
}

hipError_t launch_pgram_fields_f64(const float *fields, int64_t npix, int nb, int batch, const uchar2 *pairs,
                                   int n_mtile, int col0, int tile0, int tiles_total, int nblk, double *partial,
                                   hipStream_t st) {
    if (nb < 1 || nb > PGF_MAX_BINS || n_mtile < 1 || nblk < 1 || batch < 1 || !pairs) return hipErrorInvalidValue;
    if (col0 < 0 || col0 % 64 != 0 || col0 >= nb || tile0 < 0 || tile0 + n_mtile > tiles_total)
        return hipErrorInvalidValue;
    const int64_t chunk = pgram_fields_chunk(npix, nblk);
    if (npix % PGF64_TK != 0 || chunk % PGF64_TK != 0) return hipErrorInvalidValue;
    const unsigned groups = (unsigned)((n_mtile + PGF64_NT / 64 - 1) / (PGF64_NT / 64));
    const int64_t ms = (int64_t)nb * npix;
    if (nb <= PGF_ROW_ZERO)
        hipLaunchKernelGGL(k_pgram_fields_f64<PGF_ROW_ZERO>, dim3(nblk, batch, groups), dim3(PGF64_NT), 0, st, fields,
                           npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
    else
        hipLaunchKernelGGL(k_pgram_fields_f64<PGF_ROW_ZERO_XL>, dim3(nblk, batch, groups), dim3(PGF64_NT), 0, st,
                           fields, npix, nb, ms, pairs, n_mtile, col0, tile0, tiles_total, chunk, partial);
    return hipGetLastError();
}

}  // namespace bispec
