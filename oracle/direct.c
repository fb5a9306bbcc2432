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
 * Delta is the full complex DFT on the N^3 grid, layout [z][y][x], entry
 * (m mod N).  Passing re == NULL makes every amplitude 1, which turns the
 * sums into the polygon counts of the denominator of Eq. gen_Nspec3.
 *
 * Bin membership comes from a per-|m|^2 bit mask built by the caller:
 * bit b of mask[r2] is set when mode vectors with |m|^2 = r2 belong to bin b.
 *
 * Output layout per bin b (ORC_NACC doubles):
 *   [0] Re S   [1] Im S   [2] count   [3] Re S_strict   [4] Im S_strict
 *   [5] strict count      [6] sum |product|^2
 * Per-thread partials are merged in thread order, so a fixed thread count
 * gives a fixed result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_NACC 7

static inline int wrap_c(int c, int n) {
    int h = n / 2;
    if (c >= h) return c - n;
    if (c < -h) return c + n;
    return c;
}

static inline int64_t grid_index(int mz, int my, int mx, int n) {
    int z = mz < 0 ? mz + n : mz;
    int y = my < 0 ? my + n : my;
    int x = mx < 0 ? mx + n : mx;
    return ((int64_t)z * n + y) * n + x;
}

static inline void amp(const double *re, const double *im, int64_t g,
                       double *ar, double *ai) {
    if (re) { *ar = re[g]; *ai = im[g]; }
    else    { *ar = 1.0;   *ai = 0.0;   }
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
int orc_pair_sums(int n, const double *re, const double *im,
                  int na, const int32_t *ma, int nb_modes, const int32_t *mb,
                  const uint64_t *mask, int64_t mask_len, uint64_t want,
                  int n_bins, double *out) {
    if (n <= 0 || n_bins <= 0 || n_bins > 64) return -1;
    int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt * n_bins * ORC_NACC, sizeof(double));
    if (!part) return -2;
#pragma omp parallel num_threads(nt)
    {
        double *acc = part + (size_t)omp_get_thread_num() * n_bins * ORC_NACC;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            int z1 = ma[3 * a], y1 = ma[3 * a + 1], x1 = ma[3 * a + 2];
            double r1, i1;
            amp(re, im, grid_index(z1, y1, x1, n), &r1, &i1);
            for (int b = 0; b < nb_modes; ++b) {
                int z2 = mb[3 * b], y2 = mb[3 * b + 1], x2 = mb[3 * b + 2];
                int uz = -(z1 + z2), uy = -(y1 + y2), ux = -(x1 + x2);
                int z3 = wrap_c(uz, n), y3 = wrap_c(uy, n), x3 = wrap_c(ux, n);
                int64_t r2 = (int64_t)z3 * z3 + (int64_t)y3 * y3 + (int64_t)x3 * x3;
                if (r2 >= mask_len) continue;
                uint64_t bits = mask[r2] & want;
                if (!bits) continue;
                int strict = (z3 == uz) && (y3 == uy) && (x3 == ux);
                double r2a, i2a, r3a, i3a;
                amp(re, im, grid_index(z2, y2, x2, n), &r2a, &i2a);
                amp(re, im, grid_index(z3, y3, x3, n), &r3a, &i3a);
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

/* p = 4: ordered triples (m1 in A, m2 in B, m3 in C) closed by
 * m4 = -(m1+m2+m3) mod N. */
int orc_triple_sums(int n, const double *re, const double *im,
                    int na, const int32_t *ma, int nb_modes, const int32_t *mb,
                    int nc, const int32_t *mc,
                    const uint64_t *mask, int64_t mask_len, uint64_t want,
                    int n_bins, double *out) {
    if (n <= 0 || n_bins <= 0 || n_bins > 64) return -1;
    int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt * n_bins * ORC_NACC, sizeof(double));
    if (!part) return -2;
#pragma omp parallel num_threads(nt)
    {
        double *acc = part + (size_t)omp_get_thread_num() * n_bins * ORC_NACC;
#pragma omp for schedule(static)
        for (int a = 0; a < na; ++a) {
            int z1 = ma[3 * a], y1 = ma[3 * a + 1], x1 = ma[3 * a + 2];
            double r1, i1;
            amp(re, im, grid_index(z1, y1, x1, n), &r1, &i1);
            for (int b = 0; b < nb_modes; ++b) {
                int z2 = mb[3 * b], y2 = mb[3 * b + 1], x2 = mb[3 * b + 2];
                double r2a, i2a;
                amp(re, im, grid_index(z2, y2, x2, n), &r2a, &i2a);
                double pr = r1 * r2a - i1 * i2a;
                double pi = r1 * i2a + i1 * r2a;
                for (int c = 0; c < nc; ++c) {
                    int z3 = mc[3 * c], y3 = mc[3 * c + 1], x3 = mc[3 * c + 2];
                    int uz = -(z1 + z2 + z3), uy = -(y1 + y2 + y3), ux = -(x1 + x2 + x3);
                    /* three shell components each lie in (-N/2, N/2), so one
                     * reduction step may not suffice: reduce fully. */
                    int z4 = ((uz % n) + n) % n, y4 = ((uy % n) + n) % n, x4 = ((ux % n) + n) % n;
                    z4 = wrap_c(z4, n); y4 = wrap_c(y4, n); x4 = wrap_c(x4, n);
                    int64_t r2 = (int64_t)z4 * z4 + (int64_t)y4 * y4 + (int64_t)x4 * x4;
                    if (r2 >= mask_len) continue;
                    uint64_t bits = mask[r2] & want;
                    if (!bits) continue;
                    int strict = (z4 == uz) && (y4 == uy) && (x4 == ux);
                    double r3a, i3a, r4a, i4a;
                    amp(re, im, grid_index(z3, y3, x3, n), &r3a, &i3a);
                    amp(re, im, grid_index(z4, y4, x4, n), &r4a, &i4a);
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
