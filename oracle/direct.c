/*
 * oracle/direct.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 direct k-space sums that define what the FFT polyspectrum
 * estimator computes (Watkinson et al. 2017, arXiv:1705.06284).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library; the product path never does.
 *
 * The estimator of Eq. (Jeong_gen) equals, exactly up to rounding, a direct
 * sum over ordered tuples of shell modes whose vector sum vanishes modulo the
 * grid size N (the Kronecker delta written as a sum of phases over the grid,
 * Section 2, the identity just before Eq. gen_Nspec4).  These routines walk
 * those tuples literally:
 *
 *   pair loop  : m1 in shell A, m2 in shell B, m3 = -(m1+m2) reduced mod N;
 *                the product Delta(m1) Delta(m2) Delta(m3) is added to every
 *                requested bin that contains m3               (p = 3, Eq. gen_Nspec3)
 *   triple loop: m1, m2, m3 in shells A, B, C, m4 = -(m1+m2+m3) mod N  (p = 4)
 *
 * A tuple is "strict" when the unreduced closing vector already lies inside
 * the grid's fundamental cell, i.e. k1+k2+k3 = 0 holds in Z^3 and not only
 * modulo N (the aliasing discussion of Section 3, Eq. delta_sefusatti).
 *
 * Delta is the full complex DFT on the nz x ny x nx grid, layout [z][y][x],
 * entry (m mod N) per axis.  Passing re == NULL makes every amplitude 1, which
 * turns the sums into the polygon counts of the denominator of Eq. gen_Nspec3.
 *
 * Bin membership comes from a bit mask indexed by the integer
 * q = (sz mz)^2 + (sy my)^2 + (sx mx)^2 built by the caller (sz, sy, sx = 1
 * on a cubic grid, where q = |m|^2; on a grid of cubic cells q is |k|^2 in
 * units of 2 pi / (lcm of the sides) cells): bit b of mask[q] is set when mode
 * vectors of that q belong to bin b.
 *
 * Output layout per bin b (ORC_NACC doubles):
 *   [0] Re S   [1] Im S   [2] count   [3] Re S_strict   [4] Im S_strict
 *   [5] strict count      [6] sum |product|^2
 * Per-thread partials are merged in thread order, so a fixed thread count
 * gives a fixed result.  Small loops run on fewer threads (one per 2^18
 * tuples), which keeps the many short calls of narrow-shell plans cheap.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_NACC 7

/* Reduce c modulo n into [-n/2, n/2) (odd n: [-(n-1)/2, (n-1)/2]). */
static inline int wrap_c(int c, int n) {
    int r = ((c % n) + n) % n;
    return r >= n - n / 2 ? r - n : r;
}

typedef struct { int nz, ny, nx, sz, sy, sx; } grid_t;

static inline int64_t grid_index(int mz, int my, int mx, const grid_t *g) {
    int z = mz < 0 ? mz + g->nz : mz;
    int y = my < 0 ? my + g->ny : my;
    int x = mx < 0 ? mx + g->nx : mx;
    return ((int64_t)z * g->ny + y) * g->nx + x;
}

static inline int64_t grid_q(int mz, int my, int mx, const grid_t *g) {
    int64_t a = (int64_t)g->sz * mz, b = (int64_t)g->sy * my, c = (int64_t)g->sx * mx;
    return a * a + b * b + c * c;
}

static inline void amp(const double *re, const double *im, int64_t g,
                       double *ar, double *ai) {
    if (re) { *ar = re[g]; *ai = im[g]; }
    else    { *ar = 1.0;   *ai = 0.0;   }
}

static int threads_for(double work) {
    int nt = omp_get_max_threads();
    const double want = 1.0 + work / 262144.0;
    return want < (double)nt ? (int)want : nt;
}

static void merge(double *out, double *part, int nthreads, int nb) {
    memset(out, 0, sizeof(double) * (size_t)nb * ORC_NACC);
    for (int t = 0; t < nthreads; ++t)
        for (int i = 0; i < nb * ORC_NACC; ++i)
            out[i] += part[(size_t)t * nb * ORC_NACC + i];
}

static inline void accumulate(double *acc, uint64_t bits, double pr, double pi,
                              int strict) {
    while (bits) {
        int b = __builtin_ctzll(bits);
        bits &= bits - 1;
        double *a = acc + (size_t)b * ORC_NACC;
        a[0] += pr;
        a[1] += pi;
        a[2] += 1.0;
        if (strict) { a[3] += pr; a[4] += pi; a[5] += 1.0; }
        a[6] += pr * pr + pi * pi;
    }
}

/* p = 3: ordered pairs (m1 in A, m2 in B) closed by m3 = -(m1+m2) mod N. */
int orc_pair_sums(int nz, int ny, int nx, int sz, int sy, int sx, const double *re, const double *im,
                  int na, const int32_t *ma, int nb_modes, const int32_t *mb,
                  const uint64_t *mask, int64_t mask_len, uint64_t want,
                  int n_bins, double *out) {
    if (nz <= 0 || ny <= 0 || nx <= 0 || n_bins <= 0 || n_bins > 64) return -1;
    const grid_t G = {nz, ny, nx, sz, sy, sx};
    const grid_t *g = &G;
    int nt = threads_for((double)na * nb_modes);
    double *part = (double *)calloc((size_t)nt * n_bins * ORC_NACC, sizeof(double));
    if (!part) return -2;
#pragma omp parallel num_threads(nt)
    {
        double *acc = part + (size_t)omp_get_thread_num() * n_bins * ORC_NACC;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            int z1 = ma[3 * a], y1 = ma[3 * a + 1], x1 = ma[3 * a + 2];
            double r1, i1;
            amp(re, im, grid_index(z1, y1, x1, g), &r1, &i1);
            for (int b = 0; b < nb_modes; ++b) {
                int z2 = mb[3 * b], y2 = mb[3 * b + 1], x2 = mb[3 * b + 2];
                int uz = -(z1 + z2), uy = -(y1 + y2), ux = -(x1 + x2);
                int z3 = wrap_c(uz, nz), y3 = wrap_c(uy, ny), x3 = wrap_c(ux, nx);
                int64_t q = grid_q(z3, y3, x3, g);
                if (q >= mask_len) continue;
                uint64_t bits = mask[q] & want;
                if (!bits) continue;
                int strict = (z3 == uz) && (y3 == uy) && (x3 == ux);
                double r2a, i2a, r3a, i3a;
                amp(re, im, grid_index(z2, y2, x2, g), &r2a, &i2a);
                amp(re, im, grid_index(z3, y3, x3, g), &r3a, &i3a);
                double pr = r1 * r2a - i1 * i2a;
                double pi = r1 * i2a + i1 * r2a;
                double qr = pr * r3a - pi * i3a;
                double qi = pr * i3a + pi * r3a;
                accumulate(acc, bits, qr, qi, strict);
            }
        }
    }
    merge(out, part, nt, n_bins);
    free(part);
    return 0;
}

/* p = 4 with the diagonal fixed: ordered triples (m1 in A, m2 in B, m3 in C)
 * closed by m4 = -(m1+m2+m3) mod N whose diagonal q = m1 + m2, reduced
 * mod N, has (sz qz)^2 + (sy qy)^2 + (sx qx)^2 in [dlo2, dhi2) and is not 0
 * (the diagonal-binned trispectrum; Section 2, Eq. Jeong_gen with p = 4 and
 * the two-vector diagonal that four shells leave free). */
int orc_triple_sums_diag(int nz, int ny, int nx, int sz, int sy, int sx, const double *re, const double *im,
                         int na, const int32_t *ma, int nb_modes, const int32_t *mb,
                         int nc, const int32_t *mc,
                         const uint64_t *mask, int64_t mask_len, uint64_t want,
                         double dlo2, double dhi2, int n_bins, double *out) {
    if (nz <= 0 || ny <= 0 || nx <= 0 || n_bins <= 0 || n_bins > 64) return -1;
    const grid_t G = {nz, ny, nx, sz, sy, sx};
    const grid_t *g = &G;
    int nt = threads_for((double)na * nb_modes * nc);
    double *part = (double *)calloc((size_t)nt * n_bins * ORC_NACC, sizeof(double));
    if (!part) return -2;
#pragma omp parallel num_threads(nt)
    {
        double *acc = part + (size_t)omp_get_thread_num() * n_bins * ORC_NACC;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            int z1 = ma[3 * a], y1 = ma[3 * a + 1], x1 = ma[3 * a + 2];
            double r1, i1;
            amp(re, im, grid_index(z1, y1, x1, g), &r1, &i1);
            for (int b = 0; b < nb_modes; ++b) {
                int z2 = mb[3 * b], y2 = mb[3 * b + 1], x2 = mb[3 * b + 2];
                const double dq = (double)grid_q(wrap_c(z1 + z2, nz), wrap_c(y1 + y2, ny), wrap_c(x1 + x2, nx), g);
                if (dq <= 0.0 || dq < dlo2 || dq >= dhi2) continue;
                double r2a, i2a;
                amp(re, im, grid_index(z2, y2, x2, g), &r2a, &i2a);
                double pr = r1 * r2a - i1 * i2a;
                double pi = r1 * i2a + i1 * r2a;
                for (int c = 0; c < nc; ++c) {
                    int z3 = mc[3 * c], y3 = mc[3 * c + 1], x3 = mc[3 * c + 2];
                    int uz = -(z1 + z2 + z3), uy = -(y1 + y2 + y3), ux = -(x1 + x2 + x3);
                    int z4 = wrap_c(uz, nz), y4 = wrap_c(uy, ny), x4 = wrap_c(ux, nx);
                    int64_t q = grid_q(z4, y4, x4, g);
                    if (q >= mask_len) continue;
                    uint64_t bits = mask[q] & want;
                    if (!bits) continue;
                    int strict = (z4 == uz) && (y4 == uy) && (x4 == ux);
                    double r3a, i3a, r4a, i4a;
                    amp(re, im, grid_index(z3, y3, x3, g), &r3a, &i3a);
                    amp(re, im, grid_index(z4, y4, x4, g), &r4a, &i4a);
                    double qr = pr * r3a - pi * i3a;
                    double qi = pr * i3a + pi * r3a;
                    double sr = qr * r4a - qi * i4a;
                    double si = qr * i4a + qi * r4a;
                    accumulate(acc, bits, sr, si, strict);
                }
            }
        }
    }
    merge(out, part, nt, n_bins);
    free(part);
    return 0;
}

/* p = 4: ordered triples (m1 in A, m2 in B, m3 in C) closed by
 * m4 = -(m1+m2+m3) mod N. */
int orc_triple_sums(int nz, int ny, int nx, int sz, int sy, int sx, const double *re, const double *im,
                    int na, const int32_t *ma, int nb_modes, const int32_t *mb,
                    int nc, const int32_t *mc,
                    const uint64_t *mask, int64_t mask_len, uint64_t want,
                    int n_bins, double *out) {
    if (nz <= 0 || ny <= 0 || nx <= 0 || n_bins <= 0 || n_bins > 64) return -1;
    const grid_t G = {nz, ny, nx, sz, sy, sx};
    const grid_t *g = &G;
    int nt = threads_for((double)na * nb_modes * nc);
    double *part = (double *)calloc((size_t)nt * n_bins * ORC_NACC, sizeof(double));
    if (!part) return -2;
#pragma omp parallel num_threads(nt)
    {
        double *acc = part + (size_t)omp_get_thread_num() * n_bins * ORC_NACC;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            int z1 = ma[3 * a], y1 = ma[3 * a + 1], x1 = ma[3 * a + 2];
            double r1, i1;
            amp(re, im, grid_index(z1, y1, x1, g), &r1, &i1);
            for (int b = 0; b < nb_modes; ++b) {
                int z2 = mb[3 * b], y2 = mb[3 * b + 1], x2 = mb[3 * b + 2];
                double r2a, i2a;
                amp(re, im, grid_index(z2, y2, x2, g), &r2a, &i2a);
                double pr = r1 * r2a - i1 * i2a;
                double pi = r1 * i2a + i1 * r2a;
                for (int c = 0; c < nc; ++c) {
                    int z3 = mc[3 * c], y3 = mc[3 * c + 1], x3 = mc[3 * c + 2];
                    int uz = -(z1 + z2 + z3), uy = -(y1 + y2 + y3), ux = -(x1 + x2 + x3);
                    int z4 = wrap_c(uz, nz), y4 = wrap_c(uy, ny), x4 = wrap_c(ux, nx);
                    int64_t q = grid_q(z4, y4, x4, g);
                    if (q >= mask_len) continue;
                    uint64_t bits = mask[q] & want;
                    if (!bits) continue;
                    int strict = (z4 == uz) && (y4 == uy) && (x4 == ux);
                    double r3a, i3a, r4a, i4a;
                    amp(re, im, grid_index(z3, y3, x3, g), &r3a, &i3a);
                    amp(re, im, grid_index(z4, y4, x4, g), &r4a, &i4a);
                    double qr = pr * r3a - pi * i3a;
                    double qi = pr * i3a + pi * r3a;
                    double sr = qr * r4a - qi * i4a;
                    double si = qr * i4a + qi * r4a;
                    accumulate(acc, bits, sr, si, strict);
                }
            }
        }
    }
    merge(out, part, nt, n_bins);
    free(part);
    return 0;
}
