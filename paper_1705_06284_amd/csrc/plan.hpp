// plan.hpp -- host-side plan state of libbispec (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "fft_core.hpp"
#include "general.hpp"

struct bispec_plan_s {
    unsigned long long uid = 0;  // unique per plan in the process (never reused)
    int n = 0;                 // grid side N (cubic grids; N_z otherwise)
    double box_len = 0;        // L (V = L^3); L_x on a non-cubic grid
    // grids that are not cubic powers of two: sides N_z x N_y x N_x of cubic
    // cells, mixed-radix transforms (general.hip), bin fields in HBM
    bool general = false;
    bispec::GenGrid gg{};
    std::vector<long long> qlo, qhi;     // member iff qlo <= q < qhi (general grids)
    int64_t npix = 0;                    // N_z N_y N_x
    int64_t fstride = 0;                 // stride of one bin field in HBM (padded to 128)
    int nb = 0;                // bins
    std::vector<double> lo, hi;          // edges in k_f units
    std::vector<int> ilo2, ihi2;         // member iff ilo2 <= |m|^2 < ihi2 (integers)
    std::vector<int64_t> modes;          // M_b
    std::vector<int> tri;                // [n_tri][3]
    std::vector<double> tri_count;       // N_t (exact integers)
    std::vector<int> quad;               // [n_quad][4]
    std::vector<double> quad_count;      // N_q
    // diagonal-binned p = 4 configurations (a, b, c, d, e): shells of k1..k4
    // and of the diagonal k1 + k2 (diagtri.hip), on the mixed-radix transforms
    std::vector<int> dquad;              // [n_dquad][5]
    std::vector<double> dq_count;        // N_q(e), exact integers
    std::vector<double> dq_coef;         // [3][n_dquad]: normalisation, pairing coefficients c2, c4
    std::vector<int> dbins;              // shells whose fields the pass builds; slot = position
    std::vector<int2> dpairs;            // slot pairs (x <= y) of the pair products
    std::vector<int> dq_pp;              // [n_dquad][2]: pair of (a,b), of (c,d)
    std::vector<int2> dupairs;           // slot pairs of the |D|^2 products (connected part)
    std::vector<int> dq_up;              // per dquad: index into dupairs, or -1
    std::vector<int> didx;               // linear mode indices of the listed shells
    std::vector<int2> dseg;              // per bin: (offset, length) in didx; length 0 if unlisted
    bool dconn_ok = false;               // every dquad's shells are identical or disjoint
    bispec::GenGrid gd{};                // the grid as the mixed-radix transforms see it
    int precision = 0;
    int max_batch = 1;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_fields = false;              // workspace holds the bin-field region
    int resident = 0;                    // maps whose bin fields the region holds (0: none)
    // pruned inverse transform: bins paired (2q, 2q+1)
    std::vector<bispec::PairGeom> pairs;
    std::vector<int> cols;               // active z-pass columns of all pairs
    std::vector<int> col_off, col_n;     // per pair: offset into cols, count
    std::vector<int64_t> bc_off;         // per pair: sum of Wp of earlier pairs
    std::vector<int64_t> ab_off;         // per pair: sum of W*Wp of earlier pairs
    int wmax = 1, wpmax = 16;            // largest W and Wp
    int64_t wsum = 0;                    // sum of Wp over pairs
    int64_t absum = 0;                   // sum of W*Wp over pairs
    std::vector<int2> ztab, ytab;        // FP32 pass block tables (pair, first column)
    int nblk = 1;                        // blocks of the term contraction
    std::vector<uchar4> terms;           // [triplets | (b,b) | quads]
    std::vector<double> scale;           // normalisation over the FFT count, per term
    // The spectrum is computed from (delta - mean) 2^-spec_shift, with
    // spec_shift = floor(log2 N_pix), so that bin fields are of the order of
    // the map's r.m.s. and products of four of them stay inside the FP32
    // range at any grid size (at 512^3, F^4 of a high shell reaches 1e39
    // unscaled).  A power of two scales exactly; the per-term normalisation
    // carries 2^(p spec_shift) back in FP64.
    int spec_shift = 0;
    // product-Gram (MFMA) contraction
    bool mfma_ok = false;                // n_bins <= 32
    bool quads_collapsed = false;        // every quad is (a,a,b,b) up to order
    bool pg_wide = false;                // 33..128 bins, general grids: product-Gram over the fields in HBM
    int nblk_wide = 1;                   // blocks per map of that product-Gram
    int n_cgroup = 1;                    // its groups of 64 columns
    std::vector<int> pg_gtile;           // first row tile of each column group, and the total
    int pg_sq_tiles = 0;                 // row tiles per group of its squares pass (P, collapsed T)
    bool pg_sq_ok = false;               // the squares pass has a ones column (nb not a multiple of 64)
    int n_mtile = 0;                     // 32-row tiles of pair rows
    int nblk_pg = 1;                     // blocks of the product-Gram kernel (tuned)
    int nblk_pg_min = 1;                 // fewest blocks (chunk span limit)
    int nblk_pg_max = 1;                 // partial buffer capacity in blocks
    int tail_shape = 1;                  // tail block shape, PG_SHAPE_* (tuned; 1 = wide)
    std::vector<uchar2> pg_pairs;        // [n_mtile*32] row factors
    std::vector<int> pg_idx;             // per term: index into a block's dense tiles
                                         // (| PG_IDX_ALT: into the refinement tiles)
    // refinement rows: triplets whose condition number exceeds kRefineKappa
    // run on FP32-mode product-Gram rows of their own in every precision
    std::vector<unsigned char> refine;   // per triplet: 1 = read from the refinement tiles
    std::vector<int> refine_t;           // the indices of those triplets
    std::vector<uchar2> pg_pairs_r;      // [n_mtile_r*32] row factors of those rows
    std::vector<int> pg_gtile_r;         // first refinement tile of each column group, and the total
    int n_mtile_r = 0;                   // 32-row tiles of refinement rows (0: none)
    // when those rows would use few of their 2048 entries per tile, the
    // triplets run instead as FP64-product terms on the vector ALUs
    // (k_refine_terms): a slot table of launches of
    // refine_slots_per_launch(refine_nbs) slots each
    bool refine_valu = false;
    std::vector<uchar4> refine_terms;    // per slot: staged rows x, y, z and 0x80 if empty
    std::vector<double> refine_scale;    // per slot: the triplet's normalisation (0: empty)
    std::vector<int> refine_list;        // per slot: the triplet (-1: empty)
    std::vector<int> refine_bins;        // each launch's staged bins, concatenated
    std::vector<int> refine_bins_off;    // launch l stages refine_bins[off[l] .. off[l+1])
    int refine_nbs = 0;                  // most bins a launch stages
    int refine_nblk = 1;                 // blocks per map of each launch
    int nblk_r = 1;                      // blocks per map of the refinement pass
    // stage timing: one event per stage boundary per call
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;     // free events
    std::vector<hipEvent_t> ev_rec;      // 5 per recorded call
    hipEvent_t ev_cur[5] = {};
    // captured launch sequences of polyspec_estimate, keyed by the call's
    // pointers, batch and precision (replayed with hipGraphLaunch)
    struct GraphEntry {
        const void *delta;
        const void *P, *B, *T;
        int batch, precision;
        hipGraphExec_t exec;
    };
    bool use_graph = false;
    std::vector<GraphEntry> graphs;
    void drop_graphs();
    ~bispec_plan_s();
};

namespace bispec {

// Blocks of the per-shell spectral moments (connected trispectrum).
constexpr int kMomBlocks = 2048;

// Byte offsets of the workspace regions (256-byte aligned).
struct Layout {
    size_t tw, terms, scale, tcount, thr, mom_partial, mom_tmp, mom, pg_pairs, pg_idx, pg_pairs_r, cols, pd, ztab,
        ytab, mean_partial, mean, spec, abox, bc, fields, partial, pg_partial, pg_dense, pg_tmp, pg_partial_r,
        pg_dense_r, pg_tmp_r, refine_t, ref_terms, ref_scale, ref_list, ref_bins, ref_partial, ref_out, ref_tmp,
        // diagonal-binned trispectrum pass (one map at a time)
        dtw, dspec, dwork, dfields, dtmp, dpspec, didx, dtask, dpart, dsums, dcoef, total;
};

// Triplets with a condition number sqrt(M_i M_j M_k / (N_pix N_t)) above
// this run on the FP64 refinement rows: split-BF16 rounding measures up to
// about 3e-5 kappa relative to the noise level on narrow shells (plus a
// kappa-independent part from the FP32 accumulation), so the bar of 1e-4
// keeps a margin of about 1.3 at kappa = 2.5.  Linear bins of a few k_f
// stay below it (max 2.03 at 256^3 with 24 bins, 2.07 at 512^3 with 32).
constexpr double kRefineKappa = 2.5;

// Doubles of the refinement pass's dense tiles per map.
size_t refine_dense_doubles(const bispec_plan_s &p);

Layout make_layout(const bispec_plan_s &p, int batch);
bool needs_fields(const bispec_plan_s &p);

}  // namespace bispec
