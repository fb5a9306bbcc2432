/*
 * bispec.h -- C ABI of the MI355X FFT polyspectrum estimator.
 *
 * Implements the estimator of Watkinson, Majumdar, Pritchard & Mondal (2017),
 * "A fast estimator for the bispectrum and beyond", arXiv:1705.06284,
 * Section 2:
 *
 *   Delta_fft(m) = sum_n delta(n) exp(-2 pi i m.n/N)          Eq. (DeltaFFTtoDelta)
 *   F_b(n)       = sum_{m in S_b} Delta_fft(m) exp(+2 pi i m.n/N)   Eq. (delta_nr), first line
 *   I_b(n)       = sum_{m in S_b} exp(+2 pi i m.n/N)                Eq. (delta_nr), second line
 *   P_b          = V/N_pix^2   sum_n F_b^2       / sum_n I_b^2      Eq. (Jeong_PS)
 *   B_ijk        = V^2/N_pix^3 sum_n F_i F_j F_k / sum_n I_i I_j I_k  Eq. (Jeong_BI)
 *   T_abcd       = V^3/N_pix^4 sum_n F_a F_b F_c F_d / sum_n I_a I_b I_c I_d
 *                                                               Eq. (Jeong_gen), p = 4
 *
 * with V = L^3 the box volume, N_pix = N^3, and S_b the spherical shell of
 * bin b: the integer mode vectors m (components in [-N/2, N/2)) with
 * k_lo[b]^2 <= |m|^2 < k_hi[b]^2, m != 0, edges in units of k_f = 2 pi / L
 * (the bin rule of Eq. gen_Nspec3 read as a spherical shell; the mean mode is
 * never in a shell, and k_hi <= N/2 keeps every Nyquist mode out, Eq. nyqvist).
 *
 * The denominators sum_n I...I equal N_pix times the number of ordered closed
 * tuples (closure modulo N, the phase-sum identity before Eq. gen_Nspec4).
 * The plan evaluates them once, in FP64 with the same FFT pipeline, and
 * stores the exact integer tuple counts.
 *
 * Conventions for every call:
 *  - Real fields are row-major [z][y][x] FP32 arrays of N^3 values on the
 *    device.  Batched arguments are [batch][...] with maps back to back.
 *  - All work is enqueued on the plan's stream and is asynchronous; outputs
 *    are valid once that stream has been synchronised.  bispec_plan itself
 *    synchronises the stream before it returns.
 *  - The caller owns every input, output and workspace buffer.  A plan owns
 *    only host metadata (bins, configuration lists, counts).  bispec_plan
 *    allocates temporary device memory for the count fields and frees it
 *    before returning.
 *  - No exception crosses the ABI.  Errors are negative status codes; on an
 *    error the outputs are undefined and the plan stays usable.
 *  - A plan is not thread safe: one plan per stream.  Plans may share a device.
 */
#ifndef BISPEC_H
#define BISPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bispec_plan_s *bispec_plan_t;   /* opaque, owned by the library */

typedef enum {
    BISPEC_OK = 0,
    BISPEC_E_INVALID = -1,        /* null pointer, bad index, batch out of range  */
    BISPEC_E_UNSUPPORTED_N = -2,  /* a side outside [2, 1024], or a prime factor
                                     other than 2, 3, 5 and one prime <= 127     */
    BISPEC_E_BIN_RANGE = -3,      /* need 0 <= k_lo < k_hi <= N/2, finite         */
    BISPEC_E_EMPTY_BIN = -4,      /* a shell holds no mode                        */
    BISPEC_E_NO_WORKSPACE = -5,   /* workspace missing or smaller than footprint  */
    BISPEC_E_OOM = -6,            /* temporary device allocation failed           */
    BISPEC_E_HIP = -7,            /* a HIP runtime call or kernel launch failed   */
    BISPEC_E_NUMERIC = -8         /* an FFT count was not within 0.01 of an integer */
} bispec_status;

/* Arithmetic of the contraction sum_n F_i F_j F_k (and of the P and T sums).
 * The FFTs are FP32 in every mode; cross-block sums and the normalisation are
 * FP64 in every mode.  Modes 0 and 1 evaluate the product-Gram
 * G[(x,y),k] = sum_n (F_x F_y) F_k on the matrix cores, for every column k
 * and for pair rows (x,y) that cover the requested triplets (each triplet is
 * read from one of its three pairs).  With n_bins <= 32 the product-Gram is
 * fused with the last inverse pass and also yields P and the collapsed T.
 * With 33..128 bins (narrow shells; Section 3.2 and the Conclusion advise
 * shells one k_f wide, e.g. 127 one-pixel shells at 256^3) mode 1 keeps the
 * bin fields in HBM and runs the triplets on a product-Gram over them, one
 * pass per group of 64 columns with pair rows chosen per group, and P and the
 * collapsed quads on a pass over the squared fields (rows F_a^2, columns
 * F_b^2 and ones); general quads, and P and T when n_bins is 64 or 128, run
 * on the vector ALUs.  Mode 0 runs as mode 2 there.
 * In modes 0 and 1, triplets whose condition number
 * kappa_t = sqrt(M_i M_j M_k / (N_pix N_t)) exceeds 2.5 (shells narrower than
 * k_f near the edge of the triangle inequality; bispec_plan_condition) are
 * computed again over the bin fields in HBM with FP64 sums: on product-Gram
 * rows of their own on the FP64 matrix cores, or, when those rows would be
 * sparse (about one such triplet per pair, as with one-pixel shells), as
 * terms on the vector ALUs with FP64 products in mode 0 and FP32 products in
 * mode 1.  Their error stays near that of the FP32 FFTs (about 2.5e-7 kappa
 * relative to the noise level of B).  Such plans keep the bin fields in the
 * workspace (bispec_plan_footprint). */
enum {
    BISPEC_FP32 = 0,        /* product-Gram, FP32 MFMA, FP32 accumulation            */
    BISPEC_SPLIT_BF16 = 1,  /* product-Gram, BF16 MFMA on hi/lo splits (3 products),
                               FP32 accumulation                                      */
    BISPEC_FP32_VALU = 2    /* only the requested sums, FP32 vector ALU               */
};

/* Grids.  A cubic grid of side N = 2^k, 8 <= N <= 512 (the paper advises 2^n
 * grids, Section 2) runs the pruned transforms fused with the contraction.
 * Any other grid N_z x N_y x N_x (n_side, n_y, n_x), each side in [2, 1024]
 * and a product of 2, 3, 5 and at most one other prime <= 127 (the paper's
 * 600^3 toy boxes, Section 3.3; its 536^3 = 8 x 67 N-body grid, Section 3.2),
 * runs mixed-radix Stockham transforms, keeps the bin fields in HBM and
 * contracts them on the fields product-Gram.  Non-cubic grids
 * have cubic cells (the footnote on pixel coordinates, Section 2: one
 * fundamental 2 pi / L_i per axis): box_len is L_x, L_i = L_x N_i / N_x,
 * V = L_x L_y L_z, and shell edges are in units of the x-axis fundamental
 * 2 pi / L_x, |k| / k_f = sqrt(sum_i (m_i N_x / N_i)^2).  Membership is exact:
 * with P the lcm of the sides and s_i = P / N_i, q = sum_i (s_i m_i)^2 is
 * compared with (lo s_x)^2 and (hi s_x)^2 formed in FP64 as (lo lo)(s_x s_x). */
typedef struct {
    int32_t n_side;        /* N (cubic) or N_z                                        */
    double box_len;        /* L (L_x); <= 0 means L_x = N_x (grid units, H = 1)       */
    int32_t n_bins;        /* 1..128                                                  */
    const double *k_lo;    /* [n_bins] lower shell edges in k_f units (inclusive)     */
    const double *k_hi;    /* [n_bins] upper shell edges in k_f units (exclusive)     */
    int32_t n_tri;         /* number of triplets; 0 = every closed triplet i<=j<=k    */
    const int32_t *tri;    /* [n_tri][3] bin indices, any order; NULL when n_tri = 0  */
    int32_t n_quad;        /* number of p = 4 configurations; 0 = all (a,a,b,b), a<=b */
    const int32_t *quad;   /* [n_quad][4] bin indices; NULL when n_quad = 0           */
    int32_t precision;     /* BISPEC_FP32, BISPEC_SPLIT_BF16 or BISPEC_FP32_VALU      */
    int32_t max_batch;     /* largest batch any later call will pass, >= 1            */
    void *stream;          /* hipStream_t for all work of this plan (NULL = default) */
    int32_t n_y;           /* N_y; 0 = n_side                                         */
    int32_t n_x;           /* N_x; 0 = n_side (edges: 0 <= k_lo < k_hi <= N_x / 2)    */
    int32_t n_dquad;       /* diagonal-binned p = 4 configurations (0: none)          */
    const int32_t *dquad;  /* [n_dquad][5] bin indices a, b, c, d, e (e: the shell of
                              the diagonal k1 + k2); NULL when n_dquad = 0           */
} bispec_plan_desc;

/* Process-wide limit on the device memory a plan's count pass may hold in
 * FP64 unit fields (8 N_pix bytes per bin); 0 (the default) means half the
 * free device memory at plan time.  Beyond the limit the bins are taken in
 * groups and the fields of every set of groups that some term touches are
 * made in turn (more transforms, the same integer counts).  Affects plans
 * built after the call. */
bispec_status bispec_set_count_memory(size_t bytes);

/* Build a plan: validate the descriptor, tabulate the shells, evaluate the
 * FFT counts (Eq. Jeong_BI denominator, Section 3: FFT-counted triangles) in
 * FP64 and, when n_tri = 0, keep every i<=j<=k whose shells admit a triangle
 * (each lower edge below the sum of the other two upper edges) and whose
 * count is non-zero.  *out is set only on BISPEC_OK. */
bispec_status bispec_plan(const bispec_plan_desc *desc, bispec_plan_t *out);

/* Device workspace bytes a call with this batch needs.  The footprint
 * depends on the precision mode: BISPEC_FP32_VALU, more than 32 bins or
 * non-collapsed quads keep all bin fields in HBM (n_bins * N^3 * 4 bytes per
 * map).  After bispec_set_precision to a mode that needs them, attach a
 * workspace of the new footprint, or calls return BISPEC_E_NO_WORKSPACE. */
bispec_status bispec_plan_footprint(bispec_plan_t plan, int32_t batch, size_t *bytes);

/* Attach caller-owned device memory (at least the footprint of max_batch,
 * 256-byte aligned).  Uploads the plan's small tables into it. */
bispec_status bispec_set_workspace(bispec_plan_t plan, void *dev_ptr, size_t bytes);

/* Switch the contraction arithmetic of an existing plan; counts and tables
 * are unchanged. */
bispec_status bispec_set_precision(bispec_plan_t plan, int32_t precision);

/* Change the stream later calls enqueue on. */
bispec_status bispec_set_stream(bispec_plan_t plan, void *stream);

/* Triplet list and FFT counts.  Each output pointer may be NULL.
 * tri_out: [n_tri][3] as stored (canonical i<=j<=k for automatic lists);
 * counts_out: [n_tri] ordered closed triples N_t (exact integers as double);
 * quad_counts_out: [n_quad] ordered closed quadruples N_q, rounded to the
 * nearest integer (exact while the FP64 sum resolves single units; beyond
 * that accurate to a relative 1e-9). */
bispec_status bispec_plan_query(bispec_plan_t plan, int32_t *n_tri, int32_t *tri_out,
                                double *counts_out, double *quad_counts_out);

/* p = 4 configuration list ([n_quad][4]) and the mode count M_b of each shell. */
bispec_status bispec_plan_query_quads(bispec_plan_t plan, int32_t *n_quad, int32_t *quad_out);
bispec_status bispec_plan_mode_counts(bispec_plan_t plan, int64_t *modes_out /*[n_bins]*/);

/* The bin fields F_b(n) of Eq. (delta_nr): fields is a device buffer
 * [batch][n_bins][N^3] FP32 (unnormalised inverse transform, so
 * sum_n F_b(n)^2 = N_pix sum_{m in S_b} |Delta_fft(m)|^2).
 * fields = NULL keeps them resident instead, in the plan's workspace (plans
 * whose workspace holds the field region: more than 32 bins, general grids,
 * general quads, ill-conditioned triplets or BISPEC_FP32_VALU; else
 * BISPEC_E_NO_WORKSPACE), for polyspec_estimate with delta = NULL.  Any
 * polyspec_estimate with a map on such a plan also leaves that map's fields
 * resident. */
bispec_status bispec_bin_fields(bispec_plan_t plan, const float *delta, int32_t batch,
                                float *fields);

/* Bispectrum of every planned triplet (Eq. Jeong_BI) and, if P != NULL, the
 * power spectrum of every bin (Eq. Jeong_PS).  delta: device [batch][N^3];
 * B: device [batch][n_tri] FP64; P: device [batch][n_bins] FP64.
 * A triplet whose count is zero (explicit lists only) yields NaN. */
bispec_status bispec_estimate(bispec_plan_t plan, const float *delta, int32_t batch,
                              double *B, double *P);

/* p = 4 polyspectrum of every planned quad (Eq. Jeong_gen with four fields).
 * T: device [batch][n_quad] FP64.  T is the raw four-point mean, including
 * its disconnected part. */
bispec_status trispec_estimate(bispec_plan_t plan, const float *delta, int32_t batch,
                               double *T);

/* Connected trispectrum (cubic power-of-two grids; BISPEC_E_UNSUPPORTED_N
 * on other grids): the raw T of Eq. Jeong_gen (p = 4) for every planned quad,
 * and Tc, the same estimate with the quadruples that split into two pairs
 * k_i = -k_j removed -- the Gaussian (disconnected) pairings of Wick's
 * theorem, measured on the map itself.  With the shells of each quad
 * identical or disjoint only a collapsed quad (a,a,b,b) has such quadruples,
 * so for any other quad Tc = T; for (a,a,b,b)
 *     Tc = T - V^3 / N_pix^4 * S_D / N_q,
 *     S_D = X_a X_b              (a != b, disjoint shells)
 *     S_D = 3 X_a^2 - 3 Y_a      (a = b; inclusion-exclusion over the three
 *                                 pairings, which share the quadruples
 *                                 (k,-k,-k,k), (k,-k,k,-k), (k,k,-k,-k))
 * with X_b = sum_{m in S_b} |Delta(m)|^2 and Y_b = sum |Delta(m)|^4 in FP64
 * over the FP32 spectrum.  For a Gaussian field Tc has zero mean.  The paper
 * names the trispectrum but evaluates none (Section 2); this removal of the
 * disconnected part is a reading of "connected".
 * T, Tc: device [batch][n_quad] FP64.  BISPEC_E_INVALID if two different
 * shells of a quad overlap, or for NULL pointers. */
bispec_status trispec_connected_estimate(bispec_plan_t plan, const float *delta, int32_t batch,
                                         double *T, double *Tc);

/* Diagonal-binned trispectrum (Section 2, Eq. Jeong_gen with p = 4: four
 * shells leave the quadrilateral k1 + k2 + k3 + k4 = 0 free to fold along its
 * diagonal q = k1 + k2; binning |q| fixes it).  For each planned
 * configuration (a, b, c, d, e) (bispec_plan_desc.dquad):
 *     Td = V^3 / N_pix^4 * S / N_q(e),
 *     S  = sum over closed quadruples (mod N) with k1..k4 in S_a..S_d and
 *          k1 + k2, reduced mod N, in S_e of Delta(k1) Delta(k2) Delta(k3) Delta(k4),
 * evaluated as N_pix^-2 sum_{q in S_e} Pi_ab(q) conj(Pi_cd(q)), Pi_ab the
 * FP32 DFT of the pair-product field F_a F_b (mixed-radix transforms on any
 * grid); N_q(e) from the FP64 unit fields at plan time (exact integers,
 * bispec_plan_query_dquads).  Tdc (may be NULL): Td with the Gaussian
 * pairings removed -- k3 = -k1, k4 = -k2 (a = c, b = d) and k4 = -k1,
 * k3 = -k2 (a = d, b = c), sharing (k, k, -k, -k) when all four shells are
 * one (k2 = -k1 has q = 0, in no shell):
 *     Tdc = Td - V^3 / N_pix^4 * (c2 S2(a,b;e) - c4 S4(a;e)) / N_q(e),
 *     S2 = sum_{k1 in S_a, k2 in S_b, k1 + k2 in S_e} |D(k1)|^2 |D(k2)|^2,
 *     S4 = sum_{k in S_a, 2k in S_e} |D(k)|^4,
 * c2 the number of the two pairings that apply, c4 = 1 if a = b = c = d.
 * The paper defines no diagonal binning; this is a reading of its "and
 * beyond" for p = 4.  Maps run one at a time.  Td, Tdc: device
 * [batch][n_dquad] FP64.  BISPEC_E_INVALID if the plan has no dquads, if Tdc
 * is requested and two different shells of a configuration overlap, or for
 * NULL pointers. */
bispec_status trispec_diag_estimate(bispec_plan_t plan, const float *delta, int32_t batch,
                                    double *Td, double *Tdc);
/* n_dquad and the counts N_q(e) (exact integers as double; either may be NULL). */
bispec_status bispec_plan_query_dquads(bispec_plan_t plan, int32_t *n_dquad, double *counts_out);

/* P, B and T from one set of bin fields (lower orders at no extra FFT cost,
 * Section 2 after Eq. Jeong_BI).  Any of P, B, T may be NULL.  delta = NULL
 * contracts the fields resident in the workspace (the last
 * bispec_bin_fields(fields = NULL) or estimate on a field-region plan, of
 * the same batch; BISPEC_E_INVALID otherwise, and on plans whose contraction
 * is fused with the last transform). */
bispec_status polyspec_estimate(bispec_plan_t plan, const float *delta, int32_t batch,
                                double *P, double *B, double *T);

/* polyspec_estimate without any device allocation and without the plan's
 * workspace, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as polyspec_estimate.  The kernels run
 * on a static scratch that the library keeps on every device it runs on
 * (64 MiB each, held until the process ends); the call needs the device that
 * is current at the call to be the plan's device.  BISPEC_E_NO_WORKSPACE
 * when the plan's workspace at its max_batch (bispec_plan_footprint) is
 * larger than the scratch (a 64^3 plan of a few bins fits; 128^3 does not).
 * The first call of a plan after another plan used the scratch copies the
 * plan's small tables into it and synchronises the plan's stream.  Every call
 * on one device shares that device's scratch, which keeps the last call's
 * contents: calls that overlap on one device race and give undefined
 * results.  No graph capture or replay happens in this call. */
bispec_status polyspec_estimate_noalloc(bispec_plan_t plan, const float *delta, int32_t batch,
                                        double *P, double *B, double *T);

/* Stage timing (diagnostics).  While enabled, every estimate or bin-field
 * call records HIP events on the plan's stream at its stage boundaries:
 * [0] FP64 mean + forward FFT, [1] shell-masked inverse FFTs (all bins),
 * [2] contraction kernel(s), [3] FP64 cross-block reduction.
 * bispec_timing_read waits for the recorded events, returns the summed
 * milliseconds per stage and the number of calls, and clears the record. */
enum { BISPEC_N_STAGES = 4 };
bispec_status bispec_timing_enable(bispec_plan_t plan, int32_t on);
bispec_status bispec_timing_read(bispec_plan_t plan, double *stage_ms /*[BISPEC_N_STAGES]*/,
                                 int32_t *calls);

/* Block shapes of the fused last-pass + contraction kernel. */
enum {
    BISPEC_TAIL_DEEP = 0, /* 512 threads, up to three output tiles per wave */
    BISPEC_TAIL_WIDE = 1, /* 1024 threads, one output tile per wave (<= 16 tiles) */
    BISPEC_TAIL_TWIN = 2  /* 512 threads, one tile per wave, half the LDS: two
                             blocks per CU (N <= 256, <= 8 tiles) */
};

/* Autotuner: times the fused last-pass + contraction kernel on the attached
 * workspace, on the compact rows of the map delta (device [N^3] FP32, or
 * NULL: zero rows; the kernel's speed can depend on the data), for every shape that fits the plan's
 * output tiles and for the default block count per map (one per CU, and
 * enough that no block contracts more than 64 units of 512 points) and two
 * and four times it, within the partial buffer the footprint reserves, each
 * timed as the median of five launches after a warm-up; keeps the fastest (a
 * candidate after the first must win by 3 %: wide, twin, deep, fewer blocks
 * first) and reports it.  Synchronises the stream.
 * bispec_set_tuning restores a stored choice; BISPEC_E_INVALID if nblk is
 * below the 64-unit limit or above the buffer, or the shape is unknown.  A
 * shape that does not fit the tiles of a call runs as wide, else deep. */
bispec_status bispec_autotune(bispec_plan_t plan, const float *delta, int32_t *nblk_out, int32_t *shape_out);
bispec_status bispec_set_tuning(bispec_plan_t plan, int32_t nblk, int32_t shape);

/* Condition number of each planned triplet's real-space sum,
 * kappa_t = sqrt(M_i M_j M_k / (N_pix N_t)) (infinity when N_t = 0): the
 * factor by which rounding in the FFTs and the contraction is amplified
 * relative to the random-phase noise level of B_t.  Triplets near the edge
 * of the triangle inequality with few closed triples have large kappa. */
bispec_status bispec_plan_condition(bispec_plan_t plan, double *kappa_out /*[n_tri]*/);

/* Configuration binning of narrow-shell measurements (Section 3.2 and the
 * Conclusion: measure B with shells one k_f wide, then bin further).
 *
 * bispec_theta_groups assigns the plan's triplets to bins of the angle theta
 * between the sides k1 and k2 of the triangle, at fixed k1 in bin b1 and k2
 * in bin b2 (Section 3, Fig. theta_illus: k3 = -k1 - k2 closes the triangle;
 * Eqs. ratio and alpha fix k2/k1 and the angle).  Triplet t belongs when its
 * three bins are b1, b2 and one more bin b3 (as a multiset); then, with bin
 * centres c = (lo + hi) / 2,
 *     cos theta_t = (c1^2 + c2^2 - c3^2) / (2 c1 c2)      (law of cosines)
 * and group_out[t] = floor((cos theta_t + 1) n_cos / 2), clamped to n_cos - 1:
 * n_cos equal bins of cos theta over [-1, 1] (n_cos = 20 gives the paper's
 * +-0.05).  group_out[t] = -1 when t does not hold b1 and b2, or when the
 * centres form no triangle (|cos theta| > 1).  cos_out (or NULL) receives
 * cos theta_t, NaN where t does not hold b1 and b2.  Host only: group_out
 * and cos_out are host [n_tri] arrays; no workspace is needed.
 * BISPEC_E_BIN_RANGE for a bin index outside the plan, BISPEC_E_INVALID for
 * n_cos < 1 or a NULL group_out.
 *
 * bispec_rebin averages B over groups of triplets, weighted by the FFT
 * triangle counts N_t of the plan:
 *     out[map][g] = sum_{t: group[t] = g} N_t B[map][t] / sum_{t: group[t] = g} N_t
 * which is the estimator of Eq. Jeong_BI over the union of the groups'
 * closed triangles (the sums S_t of disjoint triangle sets add).  B: device
 * [batch][n_tri] FP64 as written by bispec_estimate; group: device [n_tri]
 * int32 (values outside [0, n_group) join no group); out: device
 * [batch][n_group] FP64, NaN for a group without a triplet of non-zero
 * count.  Stream-ordered on the plan's stream; the counts live in the
 * workspace, so it needs one attached (BISPEC_E_NO_WORKSPACE).  The sums run
 * in a fixed order (bitwise reproducible).  BISPEC_E_INVALID for NULL
 * pointers, n_group < 1, or batch outside [1, max_batch]. */
bispec_status bispec_theta_groups(bispec_plan_t plan, int32_t b1, int32_t b2, int32_t n_cos,
                                  int32_t *group_out /*[n_tri]*/, double *cos_out /*[n_tri] or NULL*/);
bispec_status bispec_rebin(bispec_plan_t plan, const double *B, int32_t batch, const int32_t *group,
                           int32_t n_group, double *out);

/* Graph replay.  While enabled, polyspec_estimate (and bispec_estimate,
 * trispec_estimate) captures its launch sequence on the plan's stream into a
 * HIP graph the first time it sees a (delta, P, B, T, batch, precision)
 * combination and replays that graph on later calls with the same
 * arguments (up to 8 cached; the contents behind the pointers may change
 * freely).  Calls fall back to direct launches on the legacy NULL stream or
 * while stage timing is on.  Changing the workspace, precision or stream
 * discards the captured graphs. */
bispec_status bispec_graph_enable(bispec_plan_t plan, int32_t on);

bispec_status bispec_destroy(bispec_plan_t plan);
const char *bispec_status_string(bispec_status status);

/* Text of the last failure seen by the calling thread (the HIP call or
 * allocation and its runtime message); empty if none. */
const char *bispec_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BISPEC_H */
