// api.cpp -- plan construction and the C ABI of libbispec (see include/bispec.h).
//
// A plan holds the shells of the bins as integer |m|^2 thresholds, the
// configuration lists (triplets for Eq. Jeong_BI, bins for Eq. Jeong_PS,
// quads for Eq. Jeong_gen with p = 4), and their exact FFT counts.  The counts
// are the denominators of those equations, sum_n I_i I_j ..., evaluated once
// in FP64 with the same FFT pipeline and divided by N_pix, which makes them
// integers (the number of ordered closed tuples, closure modulo N).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <numeric>
#include <tuple>
#include <vector>

#include "../../include/bispec.h"
#include "diagtri.hpp"
#include "general.hpp"
#include "launch.hpp"
#include "moments.hpp"
#include "noalloc.hpp"
#include "plan.hpp"

using namespace bispec;

namespace {

constexpr int kMeanParts = 1024;
constexpr int kDtBlocks = 64;            // blocks per shell sum of the diagonal-binned pass
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2_in_range(int n) { return n >= 8 && n <= 512 && (n & (n - 1)) == 0; }

// Text of the last failure on this thread (bispec_last_error).
thread_local char g_last_error[512] = "";

bispec_status record(bispec_status s, const char *what, hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return s;
}

#define CK(call)                                                        \
    do {                                                                \
        const hipError_t ck_e_ = (call);                                \
        if (ck_e_ != hipSuccess) return record(BISPEC_E_HIP, #call, ck_e_); \
    } while (0)

int contract_blocks(int64_t npix) {
    // about 4096 points per block, at most 2048 blocks, at least 1
    int64_t b = (npix + 4095) / 4096;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

// ceil(x) for the FP64 squared edges: integer r2 >= lo^2 <=> r2 >= ceil(lo^2)
// and r2 < hi^2 <=> r2 < ceil(hi^2).
int ceil_int(double x) { return (int)std::ceil(x); }

}  // namespace

namespace bispec {

int64_t field_len(const bispec_plan_s &p) { return p.general ? p.fstride : (int64_t)p.n * p.n * p.n; }

double spec_scale(const bispec_plan_s &p) { return std::ldexp(1.0, -p.spec_shift); }

bool needs_fields(const bispec_plan_s &p) {
    return p.general || !p.mfma_ok || !p.quads_collapsed || p.precision == BISPEC_FP32_VALU || p.n_mtile_r > 0;
}

size_t refine_dense_doubles(const bispec_plan_s &p) { return p.refine_valu ? 0 : (size_t)p.n_mtile_r * 2048; }

// Dense tile entries of the fields product-Gram (33..128 bins, general
// grids): [n_mtile][32][64], or the squares pass's [n_cgroup*sq_tiles][32][64].
size_t wide_dense_doubles(const bispec_plan_s &p) {
    return (size_t)std::max(p.n_mtile, p.n_cgroup * p.pg_sq_tiles) * 2048;
}

Layout make_layout(const bispec_plan_s &p, int batch) {
    Layout L{};
    const int64_t vol = field_len(p);
    size_t off = 0;
    const int ntw = p.general ? p.gg.nz + p.gg.ny + p.gg.nx : p.n;
    L.tw = off;           off = align_up(off + sizeof(float2) * ntw);
    L.terms = off;        off = align_up(off + sizeof(uchar4) * p.terms.size());
    L.scale = off;        off = align_up(off + sizeof(double) * p.scale.size());
    L.tcount = off;       off = align_up(off + sizeof(double) * p.tri_count.size());
    L.thr = off;          off = align_up(off + sizeof(int) * 2 * p.nb);
    L.mom_partial = off;  off = align_up(off + sizeof(double) * kMomBlocks * 2 * p.nb * batch);
    L.mom_tmp = off;      off = align_up(off + sizeof(double) * PG_REDUCE_SEGS * 2 * p.nb * batch);
    L.mom = off;          off = align_up(off + sizeof(double) * 2 * p.nb * batch);
    L.pg_pairs = off;     off = align_up(off + sizeof(uchar2) * p.pg_pairs.size());
    L.pg_idx = off;       off = align_up(off + sizeof(int) * p.pg_idx.size());
    L.pg_pairs_r = off;   off = align_up(off + sizeof(uchar2) * p.pg_pairs_r.size());
    L.cols = off;         off = align_up(off + sizeof(int) * p.cols.size());
    L.pd = off;           off = align_up(off + sizeof(PairDev) * p.pairs.size());
    L.ztab = off;         off = align_up(off + sizeof(int2) * p.ztab.size());
    L.ytab = off;         off = align_up(off + sizeof(int2) * p.ytab.size());
    L.mean_partial = off; off = align_up(off + sizeof(double) * kMeanParts * batch);
    L.mean = off;         off = align_up(off + sizeof(double) * batch);
    if (p.general) {
        // full complex spectrum, and one pair's inverse transform at a time
        L.spec = off;     off = align_up(off + sizeof(float2) * (size_t)p.npix * batch);
        L.abox = off;     off = align_up(off + sizeof(float2) * (size_t)p.npix * batch);
        L.bc = off;
    } else {
        L.spec = off;     off = align_up(off + sizeof(float2) * spec_elems(p.n) * batch);
        L.abox = off;     off = align_up(off + sizeof(float2) * (size_t)p.n * p.absum * batch);
        L.bc = off;       off = align_up(off + sizeof(float2) * (size_t)p.n * p.n * p.wsum * batch);
    }
    L.partial = off;      off = align_up(off + sizeof(double) * (size_t)p.nblk * p.terms.size() * batch);
    L.pg_partial = off;
    if (p.mfma_ok) {
        off = align_up(off + sizeof(double) * pgram_partial_doubles(p.n_mtile, true) * p.nblk_pg_max * batch);
    } else if (p.pg_wide) {
        // per block: the triplet pass's tiles, or the K-part sets of the squares pass
        const size_t sets = std::max((size_t)p.n_mtile, (size_t)p.n_cgroup * p.pg_sq_tiles *
                                                            pgram_fields_kparts(p.pg_sq_tiles, true));
        off = align_up(off + sizeof(double) * 2048 * sets * p.nblk_wide * batch);
    }
    L.pg_dense = off;
    if (p.mfma_ok) off = align_up(off + sizeof(double) * pgram_partial_doubles(p.n_mtile, true) * batch);
    else if (p.pg_wide) off = align_up(off + sizeof(double) * wide_dense_doubles(p) * batch);
    L.pg_tmp = off;
    if (p.mfma_ok)
        off = align_up(off + sizeof(double) * pgram_partial_doubles(p.n_mtile, true) * PG_REDUCE_SEGS * batch);
    else if (p.pg_wide)
        off = align_up(off + sizeof(double) * wide_dense_doubles(p) * PG_REDUCE_SEGS * batch);
    // refinement pass: FP64 partials of its blocks, their reduction
    const size_t rd = refine_dense_doubles(p);
    const size_t rblk = (size_t)p.nblk_r;
    L.pg_partial_r = off; off = align_up(off + sizeof(double) * rd * rblk * batch);
    L.pg_dense_r = off;   off = align_up(off + sizeof(double) * rd * batch);
    L.pg_tmp_r = off;     off = align_up(off + sizeof(double) * rd * PG_REDUCE_SEGS * batch);
    L.refine_t = off;     off = align_up(off + sizeof(int) * p.refine_t.size());
    L.ref_terms = off;    off = align_up(off + sizeof(uchar4) * p.refine_terms.size());
    L.ref_scale = off;    off = align_up(off + sizeof(double) * p.refine_scale.size());
    L.ref_list = off;     off = align_up(off + sizeof(int) * p.refine_list.size());
    L.ref_bins = off;     off = align_up(off + sizeof(int) * p.refine_bins.size());
    L.ref_partial = off;
    off = align_up(off + sizeof(double) * p.refine_terms.size() * (p.refine_valu ? p.refine_nblk : 0) * batch);
    L.ref_out = off;      off = align_up(off + sizeof(double) * p.refine_terms.size() * batch);
    L.ref_tmp = off;      off = align_up(off + sizeof(double) * p.refine_terms.size() * PG_REDUCE_SEGS * batch);
    // bin fields in HBM: only the vector-ALU contraction and general quads read them
    L.fields = off;
    if (needs_fields(p)) off = align_up(off + sizeof(float) * vol * p.nb * batch);
    // the diagonal-binned trispectrum pass, one map at a time: the full
    // spectrum, a transform scratch, the fields of its shells, a product
    // field and the spectra of the pair products
    const size_t ndq = p.dquad.size() / 5;
    const size_t np = ndq ? (size_t)p.npix : 0;
    const size_t ndtw = ndq && !p.general ? (size_t)(p.gd.nz + p.gd.ny + p.gd.nx) : 0;
    L.dtw = off;          off = align_up(off + sizeof(float2) * ndtw);
    L.dspec = off;        off = align_up(off + sizeof(float2) * np);
    L.dwork = off;        off = align_up(off + sizeof(float2) * np);
    L.dfields = off;      off = align_up(off + sizeof(float) * np * p.dbins.size());
    L.dtmp = off;         off = align_up(off + sizeof(float) * np);
    L.dpspec = off;       off = align_up(off + sizeof(float2) * np * std::max(p.dpairs.size(), p.dupairs.size()));
    L.didx = off;         off = align_up(off + sizeof(int) * p.didx.size());
    L.dtask = off;        off = align_up(off + sizeof(DtTask) * 3 * ndq);
    L.dpart = off;        off = align_up(off + sizeof(double) * 3 * ndq * kDtBlocks);
    L.dsums = off;        off = align_up(off + sizeof(double) * 3 * ndq);
    L.dcoef = off;        off = align_up(off + sizeof(double) * 3 * ndq);
    L.total = off;
    return L;
}

}  // namespace bispec

void bispec_plan_s::drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

bispec_plan_s::~bispec_plan_s() {
    drop_graphs();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_rec) (void)hipEventDestroy(e);
}

namespace {

// Stage stamps: stamp(p, 0) opens a record, stamp(p, 1..4) close stages.
hipEvent_t take_event(bispec_plan_s &p) {
    if (!p.ev_pool.empty()) {
        hipEvent_t e = p.ev_pool.back();
        p.ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void stamp(bispec_plan_s &p, int k) {
    if (!p.timing) return;
    if (k == 0)
        for (int i = 0; i < 5; ++i) p.ev_cur[i] = nullptr;
    hipEvent_t e = take_event(p);
    if (!e) return;
    (void)hipEventRecord(e, p.stream);
    p.ev_cur[k] = e;
    if (k == 4) {
        bool whole = true;
        for (int i = 0; i < 5; ++i) whole = whole && p.ev_cur[i];
        if (whole)
            for (int i = 0; i < 5; ++i) p.ev_rec.push_back(p.ev_cur[i]);
    }
}

// Close the stages not yet closed in this call at the current point.
void stamp_rest(bispec_plan_s &p, int from) {
    if (!p.timing) return;
    for (int k = from; k <= 4; ++k)
        if (!p.ev_cur[k]) stamp(p, k);
}

// Shell pairs (2q, 2q+1) of the pruned inverse transform and the list of
// z-pass columns (m_y, m_x) with m_y^2 + m_x^2 < hmax of each pair.
void build_pairs(bispec_plan_s &p) {
    p.pairs.clear();
    p.cols.clear();
    p.col_off.clear();
    p.col_n.clear();
    p.bc_off.clear();
    p.ab_off.clear();
    p.ztab.clear();
    p.ytab.clear();
    p.wmax = 1;
    p.wpmax = 16;
    p.wsum = 0;
    p.absum = 0;
    const int G = fft_pencils_per_block(p.n, false);
    for (int b = 0; b < p.nb; b += 2) {
        PairGeom g{};
        g.lo1 = p.ilo2[b];
        g.hi1 = p.ihi2[b];
        const bool two = b + 1 < p.nb;
        g.lo2 = two ? p.ilo2[b + 1] : 0;
        g.hi2 = two ? p.ihi2[b + 1] : 0;
        g.hmax = std::max(g.hi1, g.hi2);
        int r = 0;
        while ((int64_t)(r + 1) * (r + 1) < g.hmax) ++r;   // largest r with r^2 < hmax
        g.R = r;
        g.W = 2 * r + 1;
        g.Wp = (g.W + 15) / 16 * 16;
        const int q = (int)p.pairs.size();
        p.col_off.push_back((int)p.cols.size());
        // Pass Z columns: the disk m_y^2 + m_x^2 < hmax, each m_y row widened
        // to whole 16-column groups (128-byte aligned runs of the z-box
        // rows, so its stores fill whole lines); the extra columns hold no
        // shell mode and transform to zeros that pass Y never reads.
        for (int my = -r; my <= r; ++my) {
            int xa = r + 1, xb = -r - 1;
            for (int mx = -r; mx <= r; ++mx)
                if (my * my + mx * mx < g.hmax) {
                    xa = std::min(xa, mx);
                    xb = std::max(xb, mx);
                }
            if (xa > xb) continue;
            const int c0 = (xa + r) / 16 * 16, c1 = (xb + r + 1 + 15) / 16 * 16;
            for (int xi = c0; xi < c1; ++xi) p.cols.push_back((my + r) * g.Wp + xi);
        }
        p.col_n.push_back((int)p.cols.size() - p.col_off.back());
        for (int c0 = 0; c0 < p.col_n.back(); c0 += G) p.ztab.push_back(int2{q, c0});
        for (int c0 = 0; c0 < p.n * g.Wp; c0 += G) p.ytab.push_back(int2{q, c0});
        p.bc_off.push_back(p.wsum);
        p.wsum += g.Wp;
        p.ab_off.push_back(p.absum);
        p.absum += (int64_t)g.W * g.Wp;
        p.wmax = std::max(p.wmax, g.W);
        p.wpmax = std::max(p.wpmax, g.Wp);
        p.pairs.push_back(g);
    }
}

// Device descriptors of the pairs for the estimate path (all pairs resident).
std::vector<PairDev> pair_devs(const bispec_plan_s &p) {
    std::vector<PairDev> v;
    const long long n = p.n, mb = p.max_batch;
    for (size_t q = 0; q < p.pairs.size(); ++q) {
        PairDev d{};
        d.g = p.pairs[q];
        d.astride = n * d.g.W * d.g.Wp;
        d.aoff = p.ab_off[q] * n * mb;
        d.bstride = n * n * d.g.Wp;
        d.boff = p.bc_off[q] * n * n * mb;
        d.col_off = p.col_off[q];
        d.ncols = p.col_n[q];
        v.push_back(d);
    }
    return v;
}

// Greedy set cover of triplets by pair rows: repeatedly the pair (x <= y,
// index x*nb + y) that reads the most not-yet-covered triplets (lowest pair
// index on ties).  row_of holds the rows already present (-1: none) and is
// extended; add(x, y) appends a row.  A triplet a <= b <= c can be read from
// G[(x,y), z] for any of its three pairs, a repeated bin from its (b,b) row,
// and among three distinct bins two share a parity, so the equal-parity pairs
// (about nb^2/4) always suffice; the greedy cover is smaller.
template <class Add>
void greedy_cover(int nitem, const std::vector<int> &tp, const std::vector<int> &tris, std::vector<int> &row_of,
                  Add add) {
    auto covered = [&](int t) {
        return row_of[tp[3 * t]] >= 0 || row_of[tp[3 * t + 1]] >= 0 || row_of[tp[3 * t + 2]] >= 0;
    };
    std::vector<int> open;
    for (int t : tris)
        if (!covered(t)) open.push_back(t);
    std::vector<int> cnt(nitem);
    while (!open.empty()) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int t : open)
            for (int k = 0; k < 3; ++k) ++cnt[tp[3 * t + k]];
        const int best = (int)(std::max_element(cnt.begin(), cnt.end()) - cnt.begin());
        add(best);
        std::vector<int> left;
        for (int t : open)
            if (!covered(t)) left.push_back(t);
        open.swap(left);
    }
}

// Slot table of the vector-ALU refinement (k_refine_terms): the refined
// triplets in bin order, in launches of refine_slots_per_launch slots split
// evenly over the waves, each launch staging the bins its slots read.
void build_refine_slots(bispec_plan_s &p, const std::vector<int> &ref_t) {
    p.refine_terms.clear();
    p.refine_scale.clear();
    p.refine_list.clear();
    p.refine_bins.clear();
    p.refine_bins_off.assign(1, 0);
    p.refine_nbs = 0;
    if (!p.refine_valu) return;
    const int nb = p.nb;
    struct Entry { int x, y, z, t; };
    std::vector<Entry> es;
    for (int t : ref_t) {
        int a[3] = {p.tri[3 * t], p.tri[3 * t + 1], p.tri[3 * t + 2]};
        std::sort(a, a + 3);
        es.push_back(Entry{a[0], a[1], a[2], t});
    }
    std::sort(es.begin(), es.end(), [](const Entry &a, const Entry &b) {
        return std::make_tuple(a.x, a.y, a.z, a.t) < std::make_tuple(b.x, b.y, b.z, b.t);
    });
    // the most bins any launch stages fixes the slots per wave; a launch of
    // the larger size can only stage more, so settle it from the top
    int nbs_plan = 128;
    for (int pass = 0; pass < 2; ++pass) {
        const int spl = refine_slots_per_launch(nbs_plan);
        int most = 0;
        for (size_t l0 = 0; l0 < es.size(); l0 += spl) {
            std::vector<char> used(nb, 0);
            for (size_t i = l0; i < std::min(es.size(), l0 + spl); ++i) used[es[i].x] = used[es[i].y] = used[es[i].z] = 1;
            most = std::max(most, (int)std::count(used.begin(), used.end(), 1));
        }
        if (refine_rows_bucket(most) == refine_rows_bucket(nbs_plan)) break;
        nbs_plan = most;
    }
    // (every launch of spl slots stages at most refine_rows_bucket(nbs_plan)
    // bins: either the last pass confirmed it, or that bucket is 128 >= nb)
    p.refine_nbs = nbs_plan;
    const int spw = refine_slots_per_wave(nbs_plan), spl = refine_slots_per_launch(nbs_plan);
    const int waves = spl / spw;
    for (size_t l0 = 0; l0 < es.size(); l0 += spl) {
        const int m = (int)std::min<size_t>(spl, es.size() - l0);
        std::vector<int> row(nb, -1);
        for (int i = 0; i < m; ++i)
            for (int b : {es[l0 + i].x, es[l0 + i].y, es[l0 + i].z}) row[b] = 0;
        const int off = (int)p.refine_bins.size();
        for (int b = 0; b < nb; ++b)
            if (row[b] == 0) {
                row[b] = (int)p.refine_bins.size() - off;
                p.refine_bins.push_back(b);
            }
        p.refine_bins_off.push_back((int)p.refine_bins.size());
        for (int w = 0; w < waves; ++w) {
            const int i0 = (int)((int64_t)m * w / waves), i1 = (int)((int64_t)m * (w + 1) / waves);
            for (int q = 0; q < spw; ++q) {
                if (i0 + q < i1) {
                    const Entry &e = es[l0 + i0 + q];
                    p.refine_terms.push_back(uchar4{(unsigned char)row[e.x], (unsigned char)row[e.y],
                                                    (unsigned char)row[e.z], 0});
                    p.refine_scale.push_back(p.scale.empty() ? 0.0 : p.scale[e.t]);
                    p.refine_list.push_back(e.t);
                } else {
                    p.refine_terms.push_back(uchar4{0, 0, 0, 0x80});   // empty: reads row 0, not written
                    p.refine_scale.push_back(0.0);
                    p.refine_list.push_back(-1);
                }
            }
        }
    }
    // about 32 tiles of 256 points per block, at most 1024 blocks per map
    const int64_t fl = field_len(p);
    p.refine_nblk = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (fl + 8191) / 8192));
}

// Rows of the product-Gram.  Fused tail (up to 32 bins): every (b,b) row is
// kept (rows 0..nb-1, so pair tile 0 holds row (r,r) in lane r, which the
// p = 4 tile relies on); when nb < 32 column nb is a field of ones, so
// G[(b,b), nb] is the power-spectrum numerator, else rows (b, ONE) are added
// for it.  The other rows are a greedy cover of the well-conditioned
// triplets; the ill-conditioned ones (kappa above kRefineKappa) get a cover of
// their own, the refinement rows, which run on the FP64 product-Gram over the
// bin fields.  Over fields in HBM (33..128 bins, or any general grid) the
// columns come in groups of 64 and a cover item is a pair read against one
// group; each group's rows fill whole tiles of their own (ZERO padding).  A
// term's dense index in a block's tiles is tile*32*ncol + row_in_tile*ncol +
// column within the group (ncol = 32 for the tail, else 64), with PG_IDX_ALT
// set for the refinement tiles.
void build_pgram_tables(bispec_plan_s &p) {
    const int nb = p.nb;
    p.mfma_ok = !p.general && nb <= 32;
    p.pg_wide = p.general ? nb <= PGF_MAX_BINS : (nb > 32 && nb <= PGF_MAX_BINS);
    p.pg_pairs.clear();
    p.pg_idx.clear();
    p.pg_pairs_r.clear();
    p.pg_gtile.assign(1, 0);
    p.pg_gtile_r.assign(1, 0);
    p.n_mtile_r = 0;
    if (!p.mfma_ok && !p.pg_wide) return;
    // over fields in HBM the rows are the cover of the triplets alone (P and
    // collapsed quads come from the squares pass)
    const bool wide = p.pg_wide;
    const int G = wide ? (nb + 63) / 64 : 1;                // column groups of the main rows
    const int Gr = (nb + 63) / 64;                          // and of the refinement rows
    p.n_cgroup = G;
    const int row_zero = wide ? pgf_row_zero(nb) : PG_ROW_ZERO;
    const uchar2 zero2{(unsigned char)row_zero, (unsigned char)row_zero};
    const uchar2 zero2r{(unsigned char)pgf_row_zero(nb), (unsigned char)pgf_row_zero(nb)};
    // cover item of pair x*nb + y (x <= y) against column group g: (x*nb + y)*G + g
    std::vector<int> row_of(nb * nb * G, -1), row_one(nb, -1), row_of_r(nb * nb * Gr, -1);
    std::vector<std::vector<int>> grp(G), grp_r(Gr);       // items per group, in the order chosen
    auto add = [&](int item) {
        if (row_of[item] >= 0) return;
        if (wide) {
            row_of[item] = 0;                               // row numbers follow the group layout
            grp[item % G].push_back(item);
        } else {
            row_of[item] = (int)p.pg_pairs.size();
            p.pg_pairs.push_back(uchar2{(unsigned char)(item / nb), (unsigned char)(item % nb)});
        }
    };
    auto add_r = [&](int item) {
        if (row_of_r[item] >= 0) return;
        row_of_r[item] = 0;
        grp_r[item % Gr].push_back(item);
    };
    if (!wide)
        for (int b = 0; b < nb; ++b) add(b * nb + b);
    const bool one_col = nb < 32;
    if (!one_col && !wide)
        for (int b = 0; b < nb; ++b) {
            row_one[b] = (int)p.pg_pairs.size();
            p.pg_pairs.push_back(uchar2{(unsigned char)b, (unsigned char)PG_ROW_ONE});
        }
    const int ntri = (int)p.tri.size() / 3;
    // the three (pair, column) readings of each sorted triplet
    std::vector<int> tpair(3 * ntri), rest(3 * ntri), tp(3 * ntri), tp_r(3 * ntri);
    for (int t = 0; t < ntri; ++t) {
        int a[3] = {p.tri[3 * t], p.tri[3 * t + 1], p.tri[3 * t + 2]};
        std::sort(a, a + 3);
        const int c[3][3] = {{a[0], a[1], a[2]}, {a[0], a[2], a[1]}, {a[1], a[2], a[0]}};
        for (int k = 0; k < 3; ++k) {
            tpair[3 * t + k] = c[k][0] * nb + c[k][1];
            rest[3 * t + k] = c[k][2];
            tp[3 * t + k] = tpair[3 * t + k] * G + (G > 1 ? c[k][2] / 64 : 0);
            tp_r[3 * t + k] = tpair[3 * t + k] * Gr + (Gr > 1 ? c[k][2] / 64 : 0);
        }
    }
    // condition numbers decide which cover reads a triplet
    const double npix = (double)p.npix;
    p.refine.assign(ntri, 0);
    p.refine_t.clear();
    std::vector<int> main_t, ref_t;
    for (int t = 0; t < ntri; ++t) {
        const double m = (double)p.modes[p.tri[3 * t]] * (double)p.modes[p.tri[3 * t + 1]] *
                         (double)p.modes[p.tri[3 * t + 2]];
        const double c = p.tri_count.empty() ? 0.0 : p.tri_count[t];
        if (c > 0 && std::sqrt(m / (npix * c)) > kRefineKappa) {
            p.refine[t] = 1;
            ref_t.push_back(t);
            p.refine_t.push_back(t);
        } else {
            main_t.push_back(t);
        }
    }
    greedy_cover(nb * nb * G, tp, main_t, row_of, add);
    greedy_cover(nb * nb * Gr, tp_r, ref_t, row_of_r, add_r);
    // group layouts: each group's rows in whole tiles, tiles in group order
    auto lay_out = [&](std::vector<std::vector<int>> &gr, int ng, std::vector<int> &rof, std::vector<uchar2> &rows,
                       std::vector<int> &gtile, const uchar2 &z) {
        gtile.assign(1, 0);
        for (int g = 0; g < ng; ++g) {
            for (int item : gr[g]) {
                rof[item] = (int)rows.size();
                const int pr = item / ng;
                rows.push_back(uchar2{(unsigned char)(pr / nb), (unsigned char)(pr % nb)});
            }
            while (rows.size() % 32) rows.push_back(z);
            gtile.push_back((int)rows.size() / 32);
        }
    };
    if (wide) {
        lay_out(grp, G, row_of, p.pg_pairs, p.pg_gtile, zero2);
        if (p.pg_pairs.empty()) {
            // no triplet rows: one tile of zeros in group 0
            p.pg_pairs.assign(32, zero2);
            for (int g = 1; g <= G; ++g) p.pg_gtile[g] = 1;
        }
    } else {
        if (p.pg_pairs.empty()) p.pg_pairs.push_back(zero2);
        while (p.pg_pairs.size() % 32) p.pg_pairs.push_back(zero2);
        p.pg_gtile = {0, (int)p.pg_pairs.size() / 32};
    }
    p.n_mtile = (int)p.pg_pairs.size() / 32;
    lay_out(grp_r, Gr, row_of_r, p.pg_pairs_r, p.pg_gtile_r, zero2r);
    p.n_mtile_r = (int)p.pg_pairs_r.size() / 32;
    // an FP64 tile computes 32 x 64 sums per point at a third of the vector
    // ALUs' cost per sum; with fewer than a third of them wanted (one-k_f
    // shells: about one flattened triplet per row) the vector ALUs are cheaper
    p.refine_valu = !ref_t.empty() && (double)ref_t.size() < (2048.0 / 3.0) * p.n_mtile_r;
    build_refine_slots(p, ref_t);
    const int ncol = wide ? 64 : 32;
    auto dense = [ncol](int row, int c) { return (row / 32) * 32 * ncol + (row % 32) * ncol + c; };
    for (int t = 0; t < ntri; ++t) {
        const bool r = p.refine[t];
        const std::vector<int> &ro = r ? row_of_r : row_of;
        const std::vector<int> &it = r ? tp_r : tp;
        int idx = -1;
        if (r && p.refine_valu) idx = 0;   // written over afterwards (the vector-ALU terms)
        for (int k = 0; k < 3 && idx < 0; ++k)
            if (ro[it[3 * t + k]] >= 0) {
                const int row = ro[it[3 * t + k]], c = rest[3 * t + k];
                // refinement rows: 64-column tiles over the fields
                idx = r ? ((row / 32) * 2048 + (row % 32) * 64 + c % 64) | PG_IDX_ALT
                        : (wide ? dense(row, c % 64) : dense(row, c));
            }
        p.pg_idx.push_back(idx);
    }
    // blocks of the product-Gram kernels over fields in HBM: about 16384
    // points each (at least 256 blocks, at least one 128-point step per block)
    const int64_t npix_i = field_len(p);
    p.nblk_r = (int)std::min<int64_t>(std::max<int64_t>(256, npix_i / 16384), npix_i / 128);
    if (wide) {
        // blocks of at most PGF_MAX_CHUNK points, the FP32 accumulation span
        const int64_t need = (npix_i + PGF_MAX_CHUNK - 1) / PGF_MAX_CHUNK;
        p.nblk_wide = (int)std::max<int64_t>(need, std::min<int64_t>(p.nblk_r, 256));
        // P and collapsed quads from the product-Gram of the squares (rows
        // (a,a), columns F_b^2 of each group, ones at column nb): -1 leaves a
        // term to the vector ALUs (when nb is a multiple of 64, or general quads)
        p.pg_sq_tiles = pgf_sq_tiles(nb);
        p.pg_sq_ok = nb % 64 != 0;
        const int S = p.pg_sq_tiles;
        auto dsq = [S](int a, int c) { return ((c / 64) * S + a / 32) * 2048 + (a % 32) * 64 + c % 64; };
        for (int b = 0; b < nb; ++b) p.pg_idx.push_back(p.pg_sq_ok ? dsq(b, nb) : -1);
        const int nq = (int)p.quad.size() / 4;
        p.quads_collapsed = true;
        for (int q = 0; q < nq; ++q) {
            int a[4] = {p.quad[4 * q], p.quad[4 * q + 1], p.quad[4 * q + 2], p.quad[4 * q + 3]};
            std::sort(a, a + 4);
            const bool coll = a[0] == a[1] && a[2] == a[3];
            p.quads_collapsed = p.quads_collapsed && coll;
            p.pg_idx.push_back(coll && p.pg_sq_ok ? dsq(a[0], a[2]) : -1);
        }
        return;
    }
    for (int b = 0; b < nb; ++b)
        p.pg_idx.push_back(one_col ? dense(row_of[b * nb + b], nb) : dense(row_one[b], b));
    const int nq = (int)p.quad.size() / 4;
    p.quads_collapsed = true;
    for (int q = 0; q < nq; ++q) {
        int a[4] = {p.quad[4 * q], p.quad[4 * q + 1], p.quad[4 * q + 2], p.quad[4 * q + 3]};
        std::sort(a, a + 4);
        if (a[0] != a[1] || a[2] != a[3]) {
            p.quads_collapsed = false;
            p.pg_idx.push_back(-1);
        } else {
            p.pg_idx.push_back(p.n_mtile * 1024 + a[0] * 32 + a[2]);
        }
    }
}

void build_terms(bispec_plan_s &p) {
    p.terms.clear();
    p.scale.clear();
    const double npix = (double)p.npix;
    // cubic cells: L_i = L_x N_i / N_x on a non-cubic grid
    const double V = p.box_len * p.box_len * p.box_len *
                     (p.general ? ((double)p.gg.nz / p.gg.nx) * ((double)p.gg.ny / p.gg.nx) : 1.0);
    const double nan = std::numeric_limits<double>::quiet_NaN();
    // the bin fields carry 2^-spec_shift: a product of p of them 2^(-p spec_shift)
    const double u2 = std::ldexp(1.0, 2 * p.spec_shift), u3 = std::ldexp(1.0, 3 * p.spec_shift),
                 u4 = std::ldexp(1.0, 4 * p.spec_shift);
    const int ntri = (int)p.tri.size() / 3;
    for (int t = 0; t < ntri; ++t) {
        p.terms.push_back(uchar4{(unsigned char)p.tri[3 * t], (unsigned char)p.tri[3 * t + 1],
                                 (unsigned char)p.tri[3 * t + 2], 0xFF});
        const double c = p.tri_count.empty() ? 0.0 : p.tri_count[t];
        p.scale.push_back(c > 0 ? V * V / (npix * npix * npix) / (npix * c) * u3 : nan);
    }
    for (int b = 0; b < p.nb; ++b) {
        p.terms.push_back(uchar4{(unsigned char)b, (unsigned char)b, 0xFF, 0xFF});
        p.scale.push_back(V / (npix * npix) / (npix * (double)p.modes[b]) * u2);
    }
    const int nq = (int)p.quad.size() / 4;
    for (int q = 0; q < nq; ++q) {
        p.terms.push_back(uchar4{(unsigned char)p.quad[4 * q], (unsigned char)p.quad[4 * q + 1],
                                 (unsigned char)p.quad[4 * q + 2], (unsigned char)p.quad[4 * q + 3]});
        const double c = p.quad_count.empty() ? 0.0 : p.quad_count[q];
        p.scale.push_back(c > 0 ? V * V * V / (npix * npix * npix * npix) / (npix * c) * u4 : nan);
    }
    build_pgram_tables(p);
}

// Triangle inequality on the shells: each lower edge below the sum of the
// other two upper edges (necessary for a triangle closed in Z^3).
bool admits_triangle(const bispec_plan_s &p, int i, int j, int k) {
    return p.lo[k] < p.hi[i] + p.hi[j] && p.lo[j] < p.hi[i] + p.hi[k] && p.lo[i] < p.hi[j] + p.hi[k];
}

// Integer tuple counts from the FP64 grid sums sum_n I...I of the count
// fields (terms: triplets, then (b,b) per bin, then quads), divided by N_pix.
bispec_status counts_from_sums(const bispec_plan_s &p, const std::vector<double> &sums, int ntri, double npix,
                               std::vector<double> &tri_cnt, std::vector<double> &quad_cnt) {
    const int nb = p.nb, nq = (int)p.quad.size() / 4;
    auto to_count = [&](double s, double *out) -> bool {
        const double c = s / npix;
        const double r = std::nearbyint(c);
        *out = r;
        return std::fabs(c - r) <= 0.01;
    };
    tri_cnt.assign(ntri, 0.0);
    for (int t = 0; t < ntri; ++t)
        if (!to_count(sums[t], &tri_cnt[t])) return BISPEC_E_NUMERIC;
    for (int b = 0; b < nb; ++b) {
        double m;
        if (!to_count(sums[ntri + b], &m) || m != (double)p.modes[b]) return BISPEC_E_NUMERIC;
    }
    // p = 4 counts grow like M^3 and outrun what an FP64 sum resolves to one
    // unit once N_pix N_q passes ~2^53 ulp-scale: they are rounded to the
    // nearest integer and checked to a relative 1e-9.
    quad_cnt.assign(nq, 0.0);
    for (int q = 0; q < nq; ++q) {
        const double c = sums[ntri + nb + q] / npix;
        quad_cnt[q] = std::nearbyint(c);
        if (std::fabs(c - quad_cnt[q]) > std::max(0.01, 1e-9 * std::fabs(c))) return BISPEC_E_NUMERIC;
    }
    return BISPEC_OK;
}

// Count terms: candidate triplets, (b,b) per bin (the mode-count check), quads.
std::vector<uchar4> count_terms(const bispec_plan_s &p, const std::vector<int> &cand_tri) {
    std::vector<uchar4> terms;
    const int ntri = (int)cand_tri.size() / 3;
    for (int t = 0; t < ntri; ++t)
        terms.push_back(uchar4{(unsigned char)cand_tri[3 * t], (unsigned char)cand_tri[3 * t + 1],
                               (unsigned char)cand_tri[3 * t + 2], 0xFF});
    for (int b = 0; b < p.nb; ++b) terms.push_back(uchar4{(unsigned char)b, (unsigned char)b, 0xFF, 0xFF});
    const int nq = (int)p.quad.size() / 4;
    for (int q = 0; q < nq; ++q)
        terms.push_back(uchar4{(unsigned char)p.quad[4 * q], (unsigned char)p.quad[4 * q + 1],
                               (unsigned char)p.quad[4 * q + 2], (unsigned char)p.quad[4 * q + 3]});
    return terms;
}

// Twiddle tables W_n^j = exp(-2 pi i j / n), j < n, of the axes z, y, x of a
// general grid (at each axis's tw_off), from the exactly reduced argument.
template <typename C, typename R> std::vector<C> gen_twiddles(const GenGrid &g) {
    std::vector<C> tw;
    for (int a = 0; a < 3; ++a) {
        const int n = g.ax[a].n;
        for (int j = 0; j < n; ++j) {
            const double ang = 2.0 * M_PI * (double)j / (double)n;
            tw.push_back(C{(R)std::cos(ang), (R)-std::sin(ang)});
        }
    }
    return tw;
}

// Pair (b, b + 1) of a general grid's shells.
GenPair gen_pair(const bispec_plan_s &p, int b) {
    const bool two = b + 1 < p.nb;
    return GenPair{p.qlo[b], p.qhi[b], two ? p.qlo[b + 1] : 0, two ? p.qhi[b + 1] : 0};
}

// Diagonal-binned p = 4 configurations: the grid as the mixed-radix passes
// see it, the shells whose fields the pass builds (slots), the pair products,
// the pairing coefficients of the connected part and the mode lists of the
// diagonal shells (and of the shells whose |D|^4 sum the connected part
// needs).
bispec_status build_dquads(bispec_plan_s &p, const bispec_plan_desc *d) {
    p.dquad.clear();
    p.dbins.clear();
    p.dpairs.clear();
    p.dq_pp.clear();
    p.dupairs.clear();
    p.dq_up.clear();
    p.didx.clear();
    p.dseg.assign(p.nb, int2{0, 0});
    p.dq_coef.clear();
    const int ndq = d->n_dquad;
    if (ndq == 0) return BISPEC_OK;
    p.dquad.assign(d->dquad, d->dquad + 5 * ndq);
    if (p.general) {
        p.gd = p.gg;
    } else {
        GenGrid g{};
        int off = 0;
        for (int a = 0; a < 3; ++a) {
            if (!gen_factor(p.n, g.ax[a])) return BISPEC_E_UNSUPPORTED_N;
            g.ax[a].tw_off = off;
            off += p.n;
        }
        g.nz = g.ny = g.nx = p.n;
        g.sz = g.sy = g.sx = 1;
        g.npix = p.npix;
        p.gd = g;
    }
    const int nb = p.nb;
    std::vector<int> slot(nb, -1);
    auto use = [&](int b) {
        if (slot[b] < 0) {
            slot[b] = (int)p.dbins.size();
            p.dbins.push_back(b);
        }
        return slot[b];
    };
    auto pair_of = [&](std::vector<int2> &v, int x, int y) {
        int sx = use(x), sy = use(y);
        if (sx > sy) std::swap(sx, sy);
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].x == sx && v[i].y == sy) return (int)i;
        v.push_back(int2{sx, sy});
        return (int)v.size() - 1;
    };
    auto overlap = [&](int x, int y) { return x != y && p.qlo[x] < p.qhi[y] && p.qlo[y] < p.qhi[x]; };
    p.dconn_ok = true;
    std::vector<double> c2(ndq), c4(ndq);
    std::vector<char> listed(nb, 0);
    for (int t = 0; t < ndq; ++t) {
        const int *q = &p.dquad[5 * t];
        const int a = q[0], b = q[1], c = q[2], dd = q[3], e = q[4];
        p.dq_pp.push_back(pair_of(p.dpairs, a, b));
        p.dq_pp.push_back(pair_of(p.dpairs, c, dd));
        const int sh[4] = {a, b, c, dd};
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) p.dconn_ok = p.dconn_ok && !overlap(sh[i], sh[j]);
        c2[t] = (a == c && b == dd ? 1.0 : 0.0) + (a == dd && b == c ? 1.0 : 0.0);
        c4[t] = a == b && b == c && c == dd ? 1.0 : 0.0;
        p.dq_up.push_back(c2[t] > 0 ? pair_of(p.dupairs, a, b) : -1);
        listed[e] = 1;
        if (c4[t] > 0) listed[a] = 1;
    }
    // mode lists of the listed shells, in grid order
    std::vector<int> lb;
    for (int b = 0; b < nb; ++b)
        if (listed[b]) lb.push_back(b);
    std::vector<std::vector<int>> lists(lb.size());
    const GenGrid &g = p.gd;
    auto fq = [](int i, int n) { return (long long)(i < n - n / 2 ? i : i - n); };
    for (int z = 0; z < g.nz; ++z) {
        const long long qz = g.sz * fq(z, g.nz);
        for (int y = 0; y < g.ny; ++y) {
            const long long qy = g.sy * fq(y, g.ny);
            for (int x = 0; x < g.nx; ++x) {
                const long long qx = g.sx * fq(x, g.nx);
                const long long qq = qz * qz + qy * qy + qx * qx;
                if (qq == 0) continue;
                for (size_t i = 0; i < lb.size(); ++i)
                    if (qq >= p.qlo[lb[i]] && qq < p.qhi[lb[i]])
                        lists[i].push_back((int)(((int64_t)z * g.ny + y) * g.nx + x));
            }
        }
    }
    for (size_t i = 0; i < lb.size(); ++i) {
        p.dseg[lb[i]] = int2{(int)p.didx.size(), (int)lists[i].size()};
        p.didx.insert(p.didx.end(), lists[i].begin(), lists[i].end());
    }
    p.dq_coef.assign(3 * ndq, 0.0);
    for (int t = 0; t < ndq; ++t) {
        p.dq_coef[ndq + t] = c2[t];
        p.dq_coef[2 * ndq + t] = c4[t];
    }
    return BISPEC_OK;
}

// Shell-sum tasks of the diagonal pass: [0, n) the pair-product dot products
// over the diagonal shell, [n, 2n) the |D|^2 product sums, [2n, 3n) the |D|^4
// sums over shell a with 2k in the diagonal shell.
std::vector<DtTask> dquad_tasks(const bispec_plan_s &p) {
    const int ndq = (int)p.dquad.size() / 5;
    std::vector<DtTask> tk(3 * ndq);
    for (int t = 0; t < ndq; ++t) {
        const int a = p.dquad[5 * t], e = p.dquad[5 * t + 4];
        const int2 se = p.dseg[e];
        tk[t] = DtTask{se.x, se.y, p.dq_pp[2 * t], p.dq_pp[2 * t + 1], 0, 0};
        tk[ndq + t] = p.dq_up[t] >= 0 ? DtTask{se.x, se.y, p.dq_up[t], 0, 0, 0} : DtTask{0, 0, 0, 0, 0, 0};
        tk[2 * ndq + t] = p.dq_coef[2 * ndq + t] > 0
                              ? DtTask{p.dseg[a].x, p.dseg[a].y, 0, 0, p.qlo[e], p.qhi[e]}
                              : DtTask{0, 0, 0, 0, 0, 0};
    }
    return tk;
}

GenPair dquad_genpair(const bispec_plan_s &p, int i) {
    const int b1 = p.dbins[i];
    const bool two = i + 1 < (int)p.dbins.size();
    const int b2 = two ? p.dbins[i + 1] : 0;
    return GenPair{p.qlo[b1], p.qhi[b1], two ? p.qlo[b2] : 0, two ? p.qhi[b2] : 0};
}

// N_q(e) of every diagonal quad in FP64: the unit fields of the slots, their
// pair products transformed to N_pix C_xy(q) and rounded to the integer pair
// counts C_xy(q), then sum_{q in S_e} C_ab(q) C_cd(q).  Also the
// normalisation V^3 / N_pix^4 / N_q, over N_pix^2 for the dot products and
// times 2^(4 spec_shift) for the scaled fields.
bispec_status compute_dquad_counts(bispec_plan_s &p) {
    const int ndq = (int)p.dquad.size() / 5;
    if (ndq == 0) return BISPEC_OK;
    hipStream_t st = p.stream;
    const int64_t np = p.npix;
    const int nbd = (int)p.dbins.size(), npr = (int)p.dpairs.size();
    const std::vector<double2> tw = gen_twiddles<double2, double>(p.gd);
    const std::vector<DtTask> tk = dquad_tasks(p);
    size_t off = 0;
    const size_t o_tw = off;     off = align_up(off + sizeof(double2) * tw.size());
    const size_t o_f = off;      off = align_up(off + sizeof(double) * (size_t)np * nbd);
    const size_t o_tmp = off;    off = align_up(off + sizeof(double) * (size_t)np);
    const size_t o_spec = off;   off = align_up(off + sizeof(double2) * (size_t)np);
    const size_t o_work = off;   off = align_up(off + sizeof(double2) * (size_t)np);
    const size_t o_cnt = off;    off = align_up(off + sizeof(double) * (size_t)np * npr);
    const size_t o_idx = off;    off = align_up(off + sizeof(int) * p.didx.size());
    const size_t o_task = off;   off = align_up(off + sizeof(DtTask) * ndq);
    const size_t o_part = off;   off = align_up(off + sizeof(double) * (size_t)ndq * kDtBlocks);
    const size_t o_sums = off;   off = align_up(off + sizeof(double) * ndq);
    const size_t o_bad = off;    off = align_up(off + sizeof(unsigned int));
    char *mem = nullptr;
    {
        const hipError_t e = hipMalloc((void **)&mem, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            char what[128];
            std::snprintf(what, sizeof(what), "hipMalloc of %zu bytes for the diagonal count fields", off);
            return record(BISPEC_E_OOM, what, e);
        }
    }
    struct Free {
        char *m;
        ~Free() { (void)hipFree(m); }
    } guard{mem};
    const double2 *dtw = (const double2 *)(mem + o_tw);
    double *f = (double *)(mem + o_f);
    CK(hipMemcpyAsync(mem + o_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice, st));
    if (!p.didx.empty())
        CK(hipMemcpyAsync(mem + o_idx, p.didx.data(), sizeof(int) * p.didx.size(), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(mem + o_task, tk.data(), sizeof(DtTask) * ndq, hipMemcpyHostToDevice, st));
    CK(hipMemsetAsync(mem + o_bad, 0, sizeof(unsigned int), st));
    for (int i = 0; i < nbd; i += 2)
        CK(gen_inverse_unit_f64((double2 *)(mem + o_work), p.gd, dquad_genpair(p, i), dtw, f + (int64_t)i * np,
                                i + 1 < nbd ? f + (int64_t)(i + 1) * np : nullptr, st));
    for (int i = 0; i < npr; ++i) {
        CK(dt_mul_f64(f + (int64_t)p.dpairs[i].x * np, f + (int64_t)p.dpairs[i].y * np, (double *)(mem + o_tmp), np,
                      st));
        CK(gen_forward_f64((const double *)(mem + o_tmp), p.gd, dtw, (double2 *)(mem + o_spec), st));
        CK(dt_round_counts((const double2 *)(mem + o_spec), (double *)(mem + o_cnt) + (int64_t)i * np, np,
                           (double)np, (unsigned int *)(mem + o_bad), st));
    }
    CK(dt_shell_sums(1, mem + o_cnt, np, (const int *)(mem + o_idx), (const DtTask *)(mem + o_task), ndq, kDtBlocks,
                     (double *)(mem + o_part), (double *)(mem + o_sums), st));
    std::vector<double> sums(ndq);
    unsigned int bad = 0;
    CK(hipMemcpyAsync(sums.data(), mem + o_sums, sizeof(double) * ndq, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&bad, mem + o_bad, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (bad) return record(BISPEC_E_NUMERIC, "a diagonal pair count was not within 0.01 of an integer", hipSuccess);
    const double npix = (double)np;
    const double V = p.box_len * p.box_len * p.box_len *
                     (p.general ? ((double)p.gg.nz / p.gg.nx) * ((double)p.gg.ny / p.gg.nx) : 1.0);
    const double u4 = std::ldexp(1.0, 4 * p.spec_shift);
    p.dq_count = sums;
    for (int t = 0; t < ndq; ++t)
        p.dq_coef[t] = sums[t] > 0 ? V * V * V / (npix * npix * npix * npix) / sums[t] / (npix * npix) * u4
                                   : std::numeric_limits<double>::quiet_NaN();
    return BISPEC_OK;
}

// Temporary memory the count passes may hold in unit fields (0: half the
// free device memory at plan time); bispec_set_count_memory.
std::atomic<size_t> g_count_memory{0};

// Grid sums sum_n prod I_b(n) of every term over the FP64 unit fields (field
// length flen), the bins made in pairs (2q, 2q+1) by make_pair(q, f1, f2).
// When the fields of all pairs fit the count memory they are made once and
// every term is contracted over them.  Else the pairs go in groups of
// g = (pairs that fit) / 4; for each set of at most four groups that some
// term touches, in turn, the fields of its pairs are made and its terms
// contracted -- the fields are made again for every set, the memory stays
// within the limit.
template <class MakePair>
bispec_status count_term_sums(bispec_plan_s &p, const std::vector<uchar4> &terms, int64_t flen, MakePair make_pair,
                              std::vector<double> &sums) {
    hipStream_t st = p.stream;
    const int nb = p.nb, npairs = (nb + 1) / 2, nterm = (int)terms.size();
    const size_t pair_bytes = 2 * sizeof(double) * (size_t)flen;
    size_t limit = g_count_memory.load();
    if (limit == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = 0;
        }
        limit = fr / 2;
    }
    const int cap = (int)std::min<size_t>((size_t)npairs, std::max<size_t>(1, limit / pair_bytes));
    const int g = cap >= npairs ? npairs : std::max(1, cap / 4);
    // terms by the set of pair groups they touch
    std::vector<std::pair<std::vector<int>, std::vector<int>>> buckets;
    {
        std::vector<std::vector<int>> keys(nterm);
        for (int t = 0; t < nterm; ++t) {
            const unsigned char b[4] = {terms[t].x, terms[t].y, terms[t].z, terms[t].w};
            for (int i = 0; i < 4; ++i)
                if (b[i] != 0xFF) keys[t].push_back((b[i] / 2) / g);
            std::sort(keys[t].begin(), keys[t].end());
            keys[t].erase(std::unique(keys[t].begin(), keys[t].end()), keys[t].end());
        }
        std::vector<int> order(nterm);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return keys[a] < keys[b]; });
        for (int t : order) {
            if (buckets.empty() || buckets.back().first != keys[t]) buckets.push_back({keys[t], {}});
            buckets.back().second.push_back(t);
        }
    }
    size_t max_terms = 0, max_pairs = 0;
    for (const auto &bk : buckets) {
        max_terms = std::max(max_terms, bk.second.size());
        size_t np = 0;
        for (int grp : bk.first) np += (size_t)std::min(g, npairs - grp * g);
        max_pairs = std::max(max_pairs, np);
    }
    const int nblk = contract_blocks(flen);
    size_t off = 0;
    const size_t o_fields = off;  off = align_up(off + pair_bytes * max_pairs);
    const size_t o_terms = off;   off = align_up(off + sizeof(uchar4) * max_terms);
    const size_t o_ones = off;    off = align_up(off + sizeof(double) * max_terms);
    const size_t o_out = off;     off = align_up(off + sizeof(double) * max_terms);
    const size_t o_partial = off; off = align_up(off + sizeof(double) * (size_t)nblk * max_terms);
    char *mem = nullptr;
    {
        const hipError_t e = hipMalloc((void **)&mem, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            char what[128];
            std::snprintf(what, sizeof(what), "hipMalloc of %zu bytes for the count fields", off);
            return record(BISPEC_E_OOM, what, e);
        }
    }
    struct Free {
        char *m;
        ~Free() { (void)hipFree(m); }
    } guard{mem};
    double *fields = (double *)(mem + o_fields);
    const std::vector<double> ones(max_terms, 1.0);
    CK(hipMemcpyAsync(mem + o_ones, ones.data(), sizeof(double) * max_terms, hipMemcpyHostToDevice, st));
    sums.assign(nterm, 0.0);
    std::vector<int> slot(npairs, -1);
    std::vector<uchar4> mapped;
    std::vector<double> out;
    for (const auto &bk : buckets) {
        std::fill(slot.begin(), slot.end(), -1);
        int ns = 0;
        for (int grp : bk.first)
            for (int q = grp * g; q < std::min(npairs, (grp + 1) * g); ++q) {
                slot[q] = ns;
                CK(make_pair(q, fields + (int64_t)(2 * ns) * flen,
                             2 * q + 1 < nb ? fields + (int64_t)(2 * ns + 1) * flen : nullptr));
                ++ns;
            }
        const int n = (int)bk.second.size();
        mapped.resize(n);
        auto remap = [&](unsigned char b) {
            return b == 0xFF ? b : (unsigned char)(2 * slot[b / 2] + (b % 2));
        };
        for (int i = 0; i < n; ++i) {
            const uchar4 u = terms[bk.second[i]];
            mapped[i] = uchar4{remap(u.x), remap(u.y), remap(u.z), remap(u.w)};
        }
        CK(hipMemcpyAsync(mem + o_terms, mapped.data(), sizeof(uchar4) * n, hipMemcpyHostToDevice, st));
        CK(launch_contract_terms_f64(fields, flen, 2 * ns, (const uchar4 *)(mem + o_terms), n, nblk,
                                     (double *)(mem + o_partial), st));
        CK(launch_finalize((const double *)(mem + o_partial), nblk, n, 1, (const double *)(mem + o_ones),
                           (double *)(mem + o_out), n, nullptr, 0, nullptr, 0, st));
        out.resize(n);
        CK(hipMemcpyAsync(out.data(), mem + o_out, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) sums[bk.second[i]] = out[i];
    }
    return BISPEC_OK;
}

// Count fields and sums of a general grid: unit-amplitude fields of every
// bin in FP64 by the mixed-radix transforms, then the compensated FP64 term sums.
bispec_status compute_counts_general(bispec_plan_s &p, std::vector<int> &cand_tri, std::vector<double> &tri_cnt,
                                     std::vector<double> &quad_cnt) {
    hipStream_t st = p.stream;
    const std::vector<uchar4> terms = count_terms(p, cand_tri);
    const int ntri = (int)cand_tri.size() / 3;
    const int64_t fs = p.fstride;
    const std::vector<double2> tw = gen_twiddles<double2, double>(p.gg);
    size_t off = 0;
    const size_t o_tw = off;      off = align_up(off + sizeof(double2) * tw.size());
    const size_t o_work = off;    off = align_up(off + sizeof(double2) * (size_t)p.npix);
    char *mem = nullptr;
    {
        const hipError_t e = hipMalloc((void **)&mem, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return record(BISPEC_E_OOM, "hipMalloc for the count transforms", e);
        }
    }
    struct Free {
        char *m;
        ~Free() { (void)hipFree(m); }
    } guard{mem};
    CK(hipMemcpyAsync(mem + o_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice, st));
    auto make_pair = [&](int q, double *f1, double *f2) -> hipError_t {
        hipError_t e = gen_inverse_unit_f64((double2 *)(mem + o_work), p.gg, gen_pair(p, 2 * q),
                                            (const double2 *)(mem + o_tw), f1, f2, st);
        if (e == hipSuccess) e = gen_zero_pads_f64(f1, p.npix, fs, 1, st);
        if (e == hipSuccess && f2) e = gen_zero_pads_f64(f2, p.npix, fs, 1, st);
        return e;
    };
    std::vector<double> sums;
    bispec_status s = count_term_sums(p, terms, fs, make_pair, sums);
    if (s != BISPEC_OK) return s;
    return counts_from_sums(p, sums, ntri, (double)p.npix, tri_cnt, quad_cnt);
}

// FP64 count fields I_b and their product sums, evaluated on the device.
bispec_status compute_counts(bispec_plan_s &p, std::vector<int> &cand_tri, std::vector<double> &tri_cnt,
                             std::vector<double> &quad_cnt) {
    const int n = p.n;
    const int64_t vol = (int64_t)n * n * n;
    hipStream_t st = p.stream;
    // term list: candidate triplets, (b,b) for the mode-count check, quads
    const std::vector<uchar4> terms = count_terms(p, cand_tri);
    const int ntri = (int)cand_tri.size() / 3;

    std::vector<double2> tw(n);
    for (int i = 0; i < n; ++i) {
        const double a = 2.0 * M_PI * (double)i / (double)n;
        tw[i] = double2{std::cos(a), -std::sin(a)};
    }
    size_t off = 0;
    const size_t o_tw = off;      off = align_up(off + sizeof(double2) * n);
    const size_t o_cols = off;    off = align_up(off + sizeof(int) * p.cols.size());
    const size_t o_abox = off;    off = align_up(off + sizeof(double2) * (size_t)n * p.wmax * p.wpmax);
    const size_t o_bc = off;      off = align_up(off + sizeof(double2) * (size_t)n * n * p.wpmax);
    // one pair at a time: a one-entry pair table and its block tables
    const int G64 = fft_pencils_per_block(n, true);
    size_t max_tab = 0;
    for (size_t q = 0; q < p.pairs.size(); ++q)
        max_tab = std::max(max_tab, (size_t)(p.col_n[q] + G64 - 1) / G64 + (size_t)(n * p.pairs[q].Wp + G64 - 1) / G64);
    const size_t o_pd = off;      off = align_up(off + sizeof(PairDev) * p.pairs.size());
    const size_t o_tab = off;     off = align_up(off + sizeof(int2) * max_tab * p.pairs.size());
    char *mem = nullptr;
    {
        const hipError_t e = hipMalloc((void **)&mem, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return record(BISPEC_E_OOM, "hipMalloc for the count transforms", e);
        }
    }
    struct Free {
        char *m;
        ~Free() { (void)hipFree(m); }
    } guard{mem};
    CK(hipMemcpyAsync(mem + o_tw, tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(mem + o_cols, p.cols.data(), sizeof(int) * p.cols.size(), hipMemcpyHostToDevice, st));
    std::vector<PairDev> pd;
    std::vector<int2> tabs;
    std::vector<size_t> ztab_at, ytab_at;
    std::vector<int> nz, ny;
    for (size_t q = 0; q < p.pairs.size(); ++q) {
        PairDev d{};
        d.g = p.pairs[q];
        d.col_off = p.col_off[q];
        d.ncols = p.col_n[q];
        pd.push_back(d);                    // boxes shared by all pairs: offsets 0
        ztab_at.push_back(tabs.size());
        for (int c0 = 0; c0 < d.ncols; c0 += G64) tabs.push_back(int2{(int)q, c0});
        nz.push_back((int)(tabs.size() - ztab_at.back()));
        ytab_at.push_back(tabs.size());
        for (int c0 = 0; c0 < n * d.g.Wp; c0 += G64) tabs.push_back(int2{(int)q, c0});
        ny.push_back((int)(tabs.size() - ytab_at.back()));
    }
    CK(hipMemcpyAsync(mem + o_pd, pd.data(), sizeof(PairDev) * pd.size(), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(mem + o_tab, tabs.data(), sizeof(int2) * tabs.size(), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));   // host vectors above must outlive the copies
    const int2 *tab = (const int2 *)(mem + o_tab);
    auto make_pair = [&](int q, double *f1, double *f2) -> hipError_t {
        return launch_inverse_unit_f64(n, (const double2 *)(mem + o_tw), (const PairDev *)(mem + o_pd), p.pairs[q],
                                       tab + ztab_at[q], nz[q], tab + ytab_at[q], ny[q], (const int *)(mem + o_cols),
                                       (double2 *)(mem + o_abox), (double2 *)(mem + o_bc), f1, f2, st);
    };
    std::vector<double> sums;
    bispec_status s = count_term_sums(p, terms, vol, make_pair, sums);
    if (s != BISPEC_OK) return s;
    return counts_from_sums(p, sums, ntri, (double)vol, tri_cnt, quad_cnt);
}

bispec_status plan_impl(const bispec_plan_desc *d, bispec_plan_t *out) {
    if (!d || !out) return BISPEC_E_INVALID;
    // grid: N_z = n_side, N_y and N_x default to it; a cubic power of two in
    // [8, 512] takes the pruned path, any other grid the mixed-radix one
    const int nz = d->n_side, ny = d->n_y > 0 ? d->n_y : d->n_side, nx = d->n_x > 0 ? d->n_x : d->n_side;
    if (d->n_y < 0 || d->n_x < 0) return BISPEC_E_INVALID;
    const bool general = !(nz == ny && ny == nx && is_pow2_in_range(nz));
    GenGrid gg{};
    if (general) {
        const int sides[3] = {nz, ny, nx};
        int off = 0;
        for (int a = 0; a < 3; ++a) {
            if (sides[a] < 2 || sides[a] > 1024 || !gen_factor(sides[a], gg.ax[a])) return BISPEC_E_UNSUPPORTED_N;
            gg.ax[a].tw_off = off;
            off += sides[a];
        }
        const long long P = std::lcm(std::lcm((long long)nz, (long long)ny), (long long)nx);
        gg.nz = nz;
        gg.ny = ny;
        gg.nx = nx;
        gg.sz = P / nz;
        gg.sy = P / ny;
        gg.sx = P / nx;
        gg.npix = (long long)nz * ny * nx;
    }
    if (d->n_bins < 1 || d->n_bins > PGF_MAX_BINS || !d->k_lo || !d->k_hi) return BISPEC_E_INVALID;
    if (d->precision < BISPEC_FP32 || d->precision > BISPEC_FP32_VALU) return BISPEC_E_INVALID;
    if (d->max_batch < 1) return BISPEC_E_INVALID;
    if (d->n_tri < 0 || (d->n_tri > 0 && !d->tri)) return BISPEC_E_INVALID;
    if (d->n_quad < 0 || (d->n_quad > 0 && !d->quad)) return BISPEC_E_INVALID;
    const int n = d->n_side, nb = d->n_bins;
    // edges in units of the x-axis fundamental; k below the Nyquist wave
    // number pi / cell keeps every component below N_i / 2
    for (int b = 0; b < nb; ++b) {
        const double lo = d->k_lo[b], hi = d->k_hi[b];
        if (!std::isfinite(lo) || !std::isfinite(hi) || lo < 0.0 || lo >= hi || hi > 0.5 * nx)
            return BISPEC_E_BIN_RANGE;
    }
    for (int t = 0; t < 3 * d->n_tri; ++t)
        if (d->tri[t] < 0 || d->tri[t] >= nb) return BISPEC_E_INVALID;
    for (int t = 0; t < 4 * d->n_quad; ++t)
        if (d->quad[t] < 0 || d->quad[t] >= nb) return BISPEC_E_INVALID;
    if (d->n_dquad < 0 || (d->n_dquad > 0 && !d->dquad)) return BISPEC_E_INVALID;
    for (int t = 0; t < 5 * d->n_dquad; ++t)
        if (d->dquad[t] < 0 || d->dquad[t] >= nb) return BISPEC_E_INVALID;

    static std::atomic<unsigned long long> next_uid{1};
    bispec_plan_s *p = new bispec_plan_s();
    p->uid = next_uid++;
    p->n = n;
    p->general = general;
    p->gg = gg;
    p->npix = (int64_t)nz * ny * nx;
    p->fstride = (p->npix + 127) / 128 * 128;
    p->spec_shift = std::ilogb((double)p->npix);
    p->box_len = d->box_len > 0 ? d->box_len : (double)nx;
    p->nb = nb;
    p->lo.assign(d->k_lo, d->k_lo + nb);
    p->hi.assign(d->k_hi, d->k_hi + nb);
    p->precision = d->precision;
    p->max_batch = d->max_batch;
    p->stream = (hipStream_t)d->stream;
    for (int b = 0; b < nb; ++b) {
        if (general) {
            // q = sum (s_i m_i)^2 against (lo s_x)^2 and (hi s_x)^2, formed as (lo lo)(s_x s_x)
            const double sx2 = (double)(gg.sx * gg.sx);
            p->qlo.push_back(std::max(1LL, (long long)std::ceil((p->lo[b] * p->lo[b]) * sx2)));
            p->qhi.push_back((long long)std::ceil((p->hi[b] * p->hi[b]) * sx2));
            p->ilo2.push_back(0);
            p->ihi2.push_back(0);
        } else {
            p->ilo2.push_back(std::max(1, ceil_int(p->lo[b] * p->lo[b])));
            p->ihi2.push_back(ceil_int(p->hi[b] * p->hi[b]));
            p->qlo.push_back(p->ilo2.back());    // q = |m|^2 (the mixed-radix passes' test)
            p->qhi.push_back(p->ihi2.back());
        }
    }
    struct Owner {
        bispec_plan_s *p;
        bool keep = false;
        ~Owner() { if (!keep) delete p; }
    } own{p};

    // modes per shell
    if (general) {
        long long *thr = nullptr;
        unsigned long long *cnt = nullptr;
        hipError_t e = hipMalloc((void **)&thr, sizeof(long long) * 2 * nb);
        if (e == hipSuccess) e = hipMalloc((void **)&cnt, sizeof(unsigned long long) * nb);
        if (e != hipSuccess) {
            (void)hipFree(thr);
            (void)hipGetLastError();
            return record(BISPEC_E_OOM, "hipMalloc of the shell tables", e);
        }
        std::vector<long long> th(p->qlo);
        th.insert(th.end(), p->qhi.begin(), p->qhi.end());
        std::vector<unsigned long long> hc(nb, 0);
        bool ok = hipMemcpyAsync(thr, th.data(), sizeof(long long) * 2 * nb, hipMemcpyHostToDevice, p->stream) ==
                      hipSuccess &&
                  hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * nb, p->stream) == hipSuccess &&
                  gen_shell_hist(gg, nb, thr, thr + nb, cnt, p->stream) == hipSuccess &&
                  hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost,
                                 p->stream) == hipSuccess &&
                  hipStreamSynchronize(p->stream) == hipSuccess;
        (void)hipFree(thr);
        (void)hipFree(cnt);
        if (!ok) return record(BISPEC_E_HIP, "modes-per-shell pass", hipGetLastError());
        for (int b = 0; b < nb; ++b) {
            p->modes.push_back((int64_t)hc[b]);
            if (hc[b] == 0) return BISPEC_E_EMPTY_BIN;
        }
    } else {
        int *thr = nullptr;
        unsigned long long *cnt = nullptr;
        hipError_t e = hipMalloc((void **)&thr, sizeof(int) * 2 * nb);
        if (e == hipSuccess) e = hipMalloc((void **)&cnt, sizeof(unsigned long long) * nb);
        if (e != hipSuccess) {
            (void)hipFree(thr);
            (void)hipGetLastError();
            return record(BISPEC_E_OOM, "hipMalloc of the shell tables", e);
        }
        std::vector<int> th(p->ilo2);
        th.insert(th.end(), p->ihi2.begin(), p->ihi2.end());
        std::vector<unsigned long long> hc(nb, 0);
        bool ok = hipMemcpyAsync(thr, th.data(), sizeof(int) * 2 * nb, hipMemcpyHostToDevice, p->stream) == hipSuccess &&
                  hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * nb, p->stream) == hipSuccess &&
                  launch_shell_hist(n, nb, thr, thr + nb, cnt, p->stream) == hipSuccess &&
                  hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost,
                                 p->stream) == hipSuccess &&
                  hipStreamSynchronize(p->stream) == hipSuccess;
        (void)hipFree(thr);
        (void)hipFree(cnt);
        if (!ok) return record(BISPEC_E_HIP, "modes-per-shell pass", hipGetLastError());
        for (int b = 0; b < nb; ++b) {
            p->modes.push_back((int64_t)hc[b]);
            if (hc[b] == 0) return BISPEC_E_EMPTY_BIN;
        }
    }

    // configuration lists
    std::vector<int> cand;
    const bool auto_tri = d->n_tri == 0;
    if (auto_tri) {
        for (int i = 0; i < nb; ++i)
            for (int j = i; j < nb; ++j)
                for (int k = j; k < nb; ++k)
                    if (admits_triangle(*p, i, j, k)) {
                        cand.push_back(i);
                        cand.push_back(j);
                        cand.push_back(k);
                    }
    } else {
        cand.assign(d->tri, d->tri + 3 * d->n_tri);
    }
    if (d->n_quad == 0) {
        for (int a = 0; a < nb; ++a)
            for (int b = a; b < nb; ++b) {
                p->quad.push_back(a);
                p->quad.push_back(a);
                p->quad.push_back(b);
                p->quad.push_back(b);
            }
    } else {
        p->quad.assign(d->quad, d->quad + 4 * d->n_quad);
    }

    if (!general) build_pairs(*p);
    std::vector<double> tri_cnt, quad_cnt;
    bispec_status s = general ? compute_counts_general(*p, cand, tri_cnt, quad_cnt)
                              : compute_counts(*p, cand, tri_cnt, quad_cnt);
    if (s != BISPEC_OK) return s;
    if (auto_tri) {
        for (size_t t = 0; t < tri_cnt.size(); ++t)
            if (tri_cnt[t] > 0) {
                p->tri.insert(p->tri.end(), cand.begin() + 3 * t, cand.begin() + 3 * t + 3);
                p->tri_count.push_back(tri_cnt[t]);
            }
    } else {
        p->tri = cand;
        p->tri_count = tri_cnt;
    }
    p->quad_count = quad_cnt;
    p->nblk = contract_blocks(field_len(*p));
    if (!general) {
        // Tail blocks: every block contracts at most PG_CHUNK_TILES tiles
        // (its FP32 accumulation span), and there are at least 256 blocks
        // (one per CU) when the map has that many tiles.  The tuner may take
        // up to four times the default, within 2048 blocks.
        const int64_t tiles = tail_units(n);
        const int64_t need = (tiles + PG_CHUNK_TILES - 1) / PG_CHUNK_TILES;
        const int64_t lo = std::max<int64_t>(need, std::min<int64_t>(tiles, 256));
        p->nblk_pg_min = (int)need;
        p->nblk_pg = (int)lo;
        p->nblk_pg_max = (int)std::min<int64_t>(tiles, std::max<int64_t>(lo, std::min<int64_t>(4 * lo, 2048)));
    }
    build_terms(*p);
    s = build_dquads(*p, d);
    if (s != BISPEC_OK) return s;
    s = compute_dquad_counts(*p);
    if (s != BISPEC_OK) return s;
    own.keep = true;
    *out = p;
    return BISPEC_OK;
}

bispec_status upload_tables(bispec_plan_s &p) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    std::vector<float2> tw;
    if (p.general) {
        tw = gen_twiddles<float2, float>(p.gg);
    } else {
        tw.resize(p.n);
        for (int i = 0; i < p.n; ++i) {
            const double a = 2.0 * M_PI * (double)i / (double)p.n;
            tw[i] = float2{(float)std::cos(a), (float)-std::sin(a)};
        }
    }
    CK(hipMemcpyAsync(ws + L.tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice, p.stream));
    CK(hipMemcpyAsync(ws + L.terms, p.terms.data(), sizeof(uchar4) * p.terms.size(), hipMemcpyHostToDevice,
                      p.stream));
    CK(hipMemcpyAsync(ws + L.scale, p.scale.data(), sizeof(double) * p.scale.size(), hipMemcpyHostToDevice,
                      p.stream));
    if (!p.tri_count.empty())
        CK(hipMemcpyAsync(ws + L.tcount, p.tri_count.data(), sizeof(double) * p.tri_count.size(),
                          hipMemcpyHostToDevice, p.stream));
    std::vector<int> thr(p.ilo2);
    thr.insert(thr.end(), p.ihi2.begin(), p.ihi2.end());
    CK(hipMemcpyAsync(ws + L.thr, thr.data(), sizeof(int) * thr.size(), hipMemcpyHostToDevice, p.stream));
    CK(hipMemcpyAsync(ws + L.cols, p.cols.data(), sizeof(int) * p.cols.size(), hipMemcpyHostToDevice, p.stream));
    const std::vector<PairDev> pd = pair_devs(p);
    CK(hipMemcpyAsync(ws + L.pd, pd.data(), sizeof(PairDev) * pd.size(), hipMemcpyHostToDevice, p.stream));
    CK(hipMemcpyAsync(ws + L.ztab, p.ztab.data(), sizeof(int2) * p.ztab.size(), hipMemcpyHostToDevice, p.stream));
    CK(hipMemcpyAsync(ws + L.ytab, p.ytab.data(), sizeof(int2) * p.ytab.size(), hipMemcpyHostToDevice, p.stream));
    if (p.mfma_ok || p.pg_wide) {
        CK(hipMemcpyAsync(ws + L.pg_pairs, p.pg_pairs.data(), sizeof(uchar2) * p.pg_pairs.size(),
                          hipMemcpyHostToDevice, p.stream));
        CK(hipMemcpyAsync(ws + L.pg_idx, p.pg_idx.data(), sizeof(int) * p.pg_idx.size(), hipMemcpyHostToDevice,
                          p.stream));
        if (p.n_mtile_r > 0) {
            CK(hipMemcpyAsync(ws + L.pg_pairs_r, p.pg_pairs_r.data(), sizeof(uchar2) * p.pg_pairs_r.size(),
                              hipMemcpyHostToDevice, p.stream));
            CK(hipMemcpyAsync(ws + L.refine_t, p.refine_t.data(), sizeof(int) * p.refine_t.size(),
                              hipMemcpyHostToDevice, p.stream));
        }
        if (p.refine_valu) {
            CK(hipMemcpyAsync(ws + L.ref_terms, p.refine_terms.data(), sizeof(uchar4) * p.refine_terms.size(),
                              hipMemcpyHostToDevice, p.stream));
            CK(hipMemcpyAsync(ws + L.ref_scale, p.refine_scale.data(), sizeof(double) * p.refine_scale.size(),
                              hipMemcpyHostToDevice, p.stream));
            CK(hipMemcpyAsync(ws + L.ref_list, p.refine_list.data(), sizeof(int) * p.refine_list.size(),
                              hipMemcpyHostToDevice, p.stream));
            CK(hipMemcpyAsync(ws + L.ref_bins, p.refine_bins.data(), sizeof(int) * p.refine_bins.size(),
                              hipMemcpyHostToDevice, p.stream));
        }
    }
    const int ndq = (int)p.dquad.size() / 5;
    if (ndq > 0) {
        if (!p.general) {
            const std::vector<float2> dtw = gen_twiddles<float2, float>(p.gd);
            CK(hipMemcpyAsync(ws + L.dtw, dtw.data(), sizeof(float2) * dtw.size(), hipMemcpyHostToDevice,
                              p.stream));
        }
        const std::vector<DtTask> tk = dquad_tasks(p);
        CK(hipMemcpyAsync(ws + L.dtask, tk.data(), sizeof(DtTask) * tk.size(), hipMemcpyHostToDevice, p.stream));
        if (!p.didx.empty())
            CK(hipMemcpyAsync(ws + L.didx, p.didx.data(), sizeof(int) * p.didx.size(), hipMemcpyHostToDevice,
                              p.stream));
        CK(hipMemcpyAsync(ws + L.dcoef, p.dq_coef.data(), sizeof(double) * p.dq_coef.size(), hipMemcpyHostToDevice,
                          p.stream));
    }
    CK(hipStreamSynchronize(p.stream));
    return BISPEC_OK;
}

// The diagonal-binned trispectrum of batch maps, one map at a time: full
// spectrum (mean removed, scaled by 2^-spec_shift), the fields of the slots,
// each pair product's spectrum, the dot products over the diagonal shells;
// for Tdc also the |D|^4 sums and the |D|^2 pair products.
bispec_status run_trispec_diag(bispec_plan_s &p, const float *delta, int batch, double *Td, double *Tdc) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    hipStream_t st = p.stream;
    const int ndq = (int)p.dquad.size() / 5;
    const int64_t np = p.npix;
    const GenGrid &g = p.gd;
    const float2 *tw = (const float2 *)(ws + (p.general ? L.tw : L.dtw));
    float2 *spec = (float2 *)(ws + L.dspec);
    float2 *work = (float2 *)(ws + L.dwork);
    float *f = (float *)(ws + L.dfields);
    float *tmp = (float *)(ws + L.dtmp);
    float2 *ps = (float2 *)(ws + L.dpspec);
    const int *idx = (const int *)(ws + L.didx);
    const DtTask *tk = (const DtTask *)(ws + L.dtask);
    double *part = (double *)(ws + L.dpart);
    double *sums = (double *)(ws + L.dsums);
    double *mean = (double *)(ws + L.mean);
    const int nbd = (int)p.dbins.size();
    // fields of the slots from a spectrum, pair products to their spectra
    auto pair_spectra = [&](const float2 *src, const std::vector<int2> &pairs) -> hipError_t {
        for (int i = 0; i < nbd; i += 2) {
            hipError_t e = gen_inverse_pair(src, work, g, dquad_genpair(p, i), 1, tw, f + (int64_t)i * np,
                                            i + 1 < nbd ? f + (int64_t)(i + 1) * np : nullptr, 0, st);
            if (e != hipSuccess) return e;
        }
        for (size_t i = 0; i < pairs.size(); ++i) {
            hipError_t e = dt_mul_f32(f + (int64_t)pairs[i].x * np, f + (int64_t)pairs[i].y * np, tmp, np, st);
            if (e == hipSuccess) e = gen_forward(tmp, nullptr, g, 1, tw, ps + (int64_t)i * np, st, 1.0);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    for (int m = 0; m < batch; ++m) {
        const float *dm = delta + (int64_t)m * np;
        CK(gen_mean(dm, g, 1, (double *)(ws + L.mean_partial), kMeanParts, mean, st));
        CK(gen_forward(dm, mean, g, 1, tw, spec, st, spec_scale(p)));
        CK(pair_spectra(spec, p.dpairs));
        CK(dt_shell_sums(0, ps, np, idx, tk, ndq, kDtBlocks, part, sums, st));
        if (Tdc) {
            CK(dt_pow4_sums(spec, g, idx, tk + 2 * ndq, ndq, kDtBlocks, part, sums + 2 * ndq, st));
            if (!p.dupairs.empty()) {
                CK(dt_power(spec, spec, np, st));
                CK(pair_spectra(spec, p.dupairs));
                CK(dt_shell_sums(2, ps, np, idx, tk + ndq, ndq, kDtBlocks, part, sums + ndq, st));
            }
        }
        CK(dt_finalize(sums, (const double *)(ws + L.dcoef), ndq, (double)np, Td + (int64_t)m * ndq,
                       Tdc ? Tdc + (int64_t)m * ndq : nullptr, st));
    }
    return BISPEC_OK;
}

bispec_status check_call(bispec_plan_s *p, const float *delta, int batch) {
    if (!p || !delta) return BISPEC_E_INVALID;
    if (batch < 1 || batch > p->max_batch) return BISPEC_E_INVALID;
    if (!p->ws) return BISPEC_E_NO_WORKSPACE;
    return BISPEC_OK;
}

// Passes Z and Y of every shell pair, leaving the compact rows of all pairs
// in the workspace ([pair][map][N][N][W]).
hipError_t run_inverse_zy(bispec_plan_s &p, int batch) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const int n = p.n;
    return launch_inverse_zy((const float2 *)(ws + L.spec), spec_elems(n), n, batch, (const float2 *)(ws + L.tw),
                             (const PairDev *)(ws + L.pd), (const int2 *)(ws + L.ztab), (int)p.ztab.size(),
                             (const int2 *)(ws + L.ytab), (int)p.ytab.size(), (const int *)(ws + L.cols),
                             (float2 *)(ws + L.abox), (float2 *)(ws + L.bc), p.stream);
}

// mean, forward transform, and all bin fields into `fields` ([batch][nb][stride];
// on a general grid stride is the field length given, and entries from the
// end of the grid to it are zeroed when pad is set).
bispec_status run_fields(bispec_plan_s &p, const float *delta, int batch, float *fields, int64_t stride,
                         bool pad, double scale) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    if (p.general) {
        const float2 *tw = (const float2 *)(ws + L.tw);
        double *mean = (double *)(ws + L.mean);
        float2 *spec = (float2 *)(ws + L.spec);
        stamp(p, 0);
        CK(gen_mean(delta, p.gg, batch, (double *)(ws + L.mean_partial), kMeanParts, mean, p.stream));
        CK(gen_forward(delta, mean, p.gg, batch, tw, spec, p.stream, scale));
        stamp(p, 1);
        for (int b = 0; b < p.nb; b += 2)
            CK(gen_inverse_pair(spec, (float2 *)(ws + L.abox), p.gg, gen_pair(p, b), batch, tw,
                                fields + (int64_t)b * stride, b + 1 < p.nb ? fields + (int64_t)(b + 1) * stride : nullptr,
                                (int64_t)p.nb * stride, p.stream));
        if (pad) CK(gen_zero_pads_f32(fields, p.npix, stride, batch * p.nb, p.stream));
        stamp(p, 2);
        return BISPEC_OK;
    }
    const int n = p.n;
    const float2 *tw = (const float2 *)(ws + L.tw);
    double *mean = (double *)(ws + L.mean);
    float2 *spec = (float2 *)(ws + L.spec);
    stamp(p, 0);
    CK(launch_mean(delta, n, batch, (double *)(ws + L.mean_partial), kMeanParts, mean, p.stream));
    CK(launch_forward(delta, mean, n, batch, tw, spec, p.stream, scale));
    stamp(p, 1);
    CK(run_inverse_zy(p, batch));
    CK(launch_inverse_x_pairs((const float2 *)(ws + L.bc), n, batch, tw, (const PairDev *)(ws + L.pd),
                              (int)p.pairs.size(), p.nb, fields, p.stream));
    stamp(p, 2);
    return BISPEC_OK;
}

// The product-Gram over bin fields in HBM, one launch per group of 64
// columns: rows pairs[32 gtile[g] ..] against fields 64 g .. 64 g + 63,
// partial tiles gtile[g] .. gtile[g+1] - 1 of every block's set.
hipError_t pgram_groups(const bispec_plan_s &p, const float *fields, int64_t fl, int batch, const uchar2 *pairs,
                        const std::vector<int> &gtile, bool f64, int nblk, double *partial) {
    const int tiles = gtile.back();
    for (size_t g = 0; g + 1 < gtile.size(); ++g) {
        const int nt = gtile[g + 1] - gtile[g];
        if (nt == 0) continue;
        const uchar2 *pg = pairs + 32 * (int64_t)gtile[g];
        const hipError_t e =
            f64 ? launch_pgram_fields_f64(fields, fl, p.nb, batch, pg, nt, 64 * (int)g, gtile[g], tiles, nblk,
                                          partial, p.stream)
                : launch_pgram_fields(fields, fl, p.nb, batch, pg, nt, 64 * (int)g, gtile[g], tiles, nblk, partial,
                                      p.stream, false);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The product-Gram of the squares, one launch per column group.
hipError_t pgram_squares(const bispec_plan_s &p, const float *fields, int64_t fl, int batch, double *partial) {
    const int S = p.pg_sq_tiles;
    for (int g = 0; g < p.n_cgroup; ++g) {
        const hipError_t e = launch_pgram_fields(fields, fl, p.nb, batch, nullptr, S, 64 * g, g * S,
                                                 p.n_cgroup * S, p.nblk_wide, partial, p.stream, true);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Final FP64 reduction of terms [first, last) into B ([0,ntri)), P
// ([ntri, ntri+nb)) and T (the rest); gather != 0 reads the dense
// product-Gram partials at pg_idx.
bispec_status finalize_range(bispec_plan_s &p, bool gather, const double *partial, int nblk, int64_t blk_stride,
                             int first, int last, int batch, double *P, double *B, double *T) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const int ntri = (int)p.tri.size() / 3;
    const int nterm = last - first;
    if (nterm <= 0) return BISPEC_OK;
    const int n0 = std::max(0, std::min(ntri, last) - first);
    const int n1 = std::max(0, std::min(ntri + p.nb, last) - std::max(first, ntri));
    const int n2 = std::max(0, last - std::max(first, ntri + p.nb));
    double *o[3] = {B, P, T};
    int ns[3] = {n0, n1, n2};
    double *oo[3] = {nullptr, nullptr, nullptr};
    int nn[3] = {0, 0, 0};
    int k = 0;
    for (int s = 0; s < 3; ++s)
        if (ns[s] > 0) {
            oo[k] = o[s];
            nn[k] = ns[s];
            ++k;
        }
    const double *scale = (const double *)(ws + L.scale) + first;
    if (p.timing && !p.ev_cur[3]) stamp(p, 3);
    if (gather) {
        const int *idx = (const int *)(ws + L.pg_idx) + first;
        CK(launch_finalize_gather(partial, nblk, blk_stride, (const double *)(ws + L.pg_dense_r),
                                  (int64_t)refine_dense_doubles(p), idx, nterm, batch, scale, oo[0], nn[0], oo[1],
                                  nn[1], oo[2], nn[2], p.stream));
    } else {
        CK(launch_finalize(partial, nblk, nterm, batch, scale, oo[0], nn[0], oo[1], nn[1], oo[2], nn[2], p.stream));
    }
    return BISPEC_OK;
}

// The ill-conditioned triplets as terms on the vector ALUs over the bin
// fields (k_refine_terms, one launch per slot batch; FP32 products in
// split-BF16 mode, FP64 otherwise, FP64 sums), written over their entries
// of B (after B's own finalisation).
bispec_status refine_valu_run(bispec_plan_s &p, const float *fields, int64_t fl, int batch, double *B) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const int nslot = (int)p.refine_terms.size();
    const int ntri = (int)p.tri.size() / 3;
    const int spl = refine_slots_per_launch(p.refine_nbs);
    double *partial = (double *)(ws + L.ref_partial);
    const int nl = (int)p.refine_bins_off.size() - 1;
    if (nslot != nl * spl) return BISPEC_E_INVALID;
    for (int l = 0; l < nl; ++l) {
        const int b0 = p.refine_bins_off[l], nbs = p.refine_bins_off[l + 1] - b0;
        CK(launch_refine_terms(fields, fl, (int64_t)p.nb * fl, batch, (const int *)(ws + L.ref_bins) + b0, nbs,
                               p.refine_nbs, (const uchar4 *)(ws + L.ref_terms), l * spl, nslot, p.refine_nblk,
                               partial, p.stream, p.precision != BISPEC_SPLIT_BF16));
    }
    // fixed-order segmented sums over the blocks, then scale and scatter
    CK(launch_reduce_dense(partial, p.refine_nblk, nslot, batch, (double *)(ws + L.ref_out),
                           (double *)(ws + L.ref_tmp), p.stream));
    CK(launch_scatter_list((const double *)(ws + L.ref_out), nslot, (const int *)(ws + L.ref_list),
                           (const double *)(ws + L.ref_scale), batch, B, ntri, p.stream));
    return BISPEC_OK;
}

// VALU contraction of terms [first, last) followed by their reduction.
bispec_status valu_terms(bispec_plan_s &p, const float *fields, int first, int last, int batch, double *P, double *B,
                         double *T) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const int64_t vol = field_len(p);
    const int nterm = last - first;
    if (nterm <= 0) return BISPEC_OK;
    double *partial = (double *)(ws + L.partial);
    CK(launch_contract_terms_f32(fields, vol, p.nb, (int64_t)p.nb * vol, batch, (const uchar4 *)(ws + L.terms) + first,
                                 nterm, p.nblk, partial, p.stream));
    return finalize_range(p, false, partial, p.nblk, nterm, first, last, batch, P, B, T);
}

bispec_status run_estimate_body(bispec_plan_s &p, const float *delta, int batch, double *P, double *B,
                                double *T) {
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const int n = p.n;
    const int ntri = (int)p.tri.size() / 3, nq = (int)p.quad.size() / 4;
    const int t_first = ntri + p.nb, t_last = ntri + p.nb + nq;
    // B and P share the lower term range
    int first = B ? 0 : ntri, last = P ? ntri + p.nb : ntri;
    if (!B && !P) first = last = 0;
    const bool mfma = p.mfma_ok && p.precision != BISPEC_FP32_VALU;
    if ((!mfma || (T && !p.quads_collapsed) || (B && p.n_mtile_r > 0)) && !p.ws_fields) return BISPEC_E_NO_WORKSPACE;
    if (!mfma) {
        float *fields = (float *)(ws + L.fields);
        const int64_t fl = field_len(p);
        bispec_status s = BISPEC_OK;
        if (delta) {
            p.resident = 0;
            s = run_fields(p, delta, batch, fields, fl, true, spec_scale(p));
            if (s != BISPEC_OK) return s;
            p.resident = batch;          // these maps' fields stay in the workspace
        } else if (p.resident != batch) {
            return BISPEC_E_INVALID;
        }
        // split mode over the fields in HBM (33..128 bins, general grids):
        // the triplets on MFMA; then P and collapsed quads from the
        // product-Gram of the squares (nb not a multiple of 64); what is left
        // runs on the vector ALUs below
        const bool wide = p.pg_wide && p.precision == BISPEC_SPLIT_BF16;
        // (the partial and dense regions hold the larger of the two passes;
        // each pass strides its blocks by its own tile count)
        double *pg = (double *)(ws + L.pg_partial);
        double *dense = (double *)(ws + L.pg_dense);
        if (wide && B && ntri > 0) {
            const int64_t n_dense = (int64_t)p.n_mtile * 2048;
            CK(pgram_groups(p, fields, fl, batch, (const uchar2 *)(ws + L.pg_pairs), p.pg_gtile, false, p.nblk_wide,
                            pg));
            CK(launch_reduce_dense(pg, p.nblk_wide, n_dense, batch, dense, (double *)(ws + L.pg_tmp), p.stream));
            if (p.n_mtile_r > 0 && !p.refine_valu) {
                // ill-conditioned triplets: FP64 product-Gram rows of their own
                double *pr = (double *)(ws + L.pg_partial_r);
                CK(pgram_groups(p, fields, fl, batch, (const uchar2 *)(ws + L.pg_pairs_r), p.pg_gtile_r, true,
                                p.nblk_r, pr));
                CK(launch_reduce_dense(pr, p.nblk_r, (int64_t)refine_dense_doubles(p), batch,
                                       (double *)(ws + L.pg_dense_r), (double *)(ws + L.pg_tmp_r), p.stream));
            }
            s = finalize_range(p, true, dense, 1, n_dense, 0, ntri, batch, P, B, T);
            if (s != BISPEC_OK) return s;
            if (p.refine_valu) {
                s = refine_valu_run(p, fields, fl, batch, B);
                if (s != BISPEC_OK) return s;
            }
            first = ntri;
            if (first == last && !T) return BISPEC_OK;
        }
        if (wide && p.pg_sq_ok && (first < last || (T && p.quads_collapsed))) {
            const int64_t n_dense = (int64_t)p.n_cgroup * p.pg_sq_tiles * 2048;
            const int sets = p.nblk_wide * pgram_fields_kparts(p.pg_sq_tiles, true);
            CK(pgram_squares(p, fields, fl, batch, pg));
            CK(launch_reduce_dense(pg, sets, n_dense, batch, dense, (double *)(ws + L.pg_tmp), p.stream));
            if (first < last) {
                s = finalize_range(p, true, dense, 1, n_dense, first, last, batch, P, B, T);
                if (s != BISPEC_OK) return s;
                first = last;
            }
            if (T && p.quads_collapsed) return finalize_range(p, true, dense, 1, n_dense, t_first, t_last, batch, P, B, T);
            if (!T) return BISPEC_OK;
            return valu_terms(p, fields, t_first, t_last, batch, P, B, T);
        }
        if (!T) s = valu_terms(p, fields, first, last, batch, P, B, T);
        else if (first == last) s = valu_terms(p, fields, t_first, t_last, batch, P, B, T);
        else if (last == t_first) s = valu_terms(p, fields, first, t_last, batch, P, B, T);
        else {
            s = valu_terms(p, fields, first, last, batch, P, B, T);
            if (s == BISPEC_OK) s = valu_terms(p, fields, t_first, t_last, batch, P, B, T);
        }
        if (s != BISPEC_OK) return s;
        // ill-conditioned triplets of the vector-ALU route (FP32 mode): the
        // FP64 refinement rows, written over the vector-ALU values
        if (B && first == 0 && ntri > 0 && p.n_mtile_r > 0 && p.precision != BISPEC_FP32_VALU && p.refine_valu)
            return refine_valu_run(p, fields, fl, batch, B);
        if (B && first == 0 && ntri > 0 && p.n_mtile_r > 0 && p.precision != BISPEC_FP32_VALU) {
            double *pr = (double *)(ws + L.pg_partial_r);
            CK(pgram_groups(p, fields, fl, batch, (const uchar2 *)(ws + L.pg_pairs_r), p.pg_gtile_r, true, p.nblk_r,
                            pr));
            CK(launch_reduce_dense(pr, p.nblk_r, (int64_t)refine_dense_doubles(p), batch,
                                   (double *)(ws + L.pg_dense_r), (double *)(ws + L.pg_tmp_r), p.stream));
            CK(launch_scatter_alt((const double *)(ws + L.pg_dense_r), (int64_t)refine_dense_doubles(p),
                                  (const int *)(ws + L.pg_idx), (const double *)(ws + L.scale),
                                  (const int *)(ws + L.refine_t), (int)p.refine_t.size(), batch, B, ntri, p.stream));
        }
        return BISPEC_OK;
    }
    // FFT-domain part, then the fused last pass + product-Gram
    const float2 *tw = (const float2 *)(ws + L.tw);
    double *mean = (double *)(ws + L.mean);
    stamp(p, 0);
    CK(launch_mean(delta, n, batch, (double *)(ws + L.mean_partial), kMeanParts, mean, p.stream));
    CK(launch_forward(delta, mean, n, batch, tw, (float2 *)(ws + L.spec), p.stream, spec_scale(p)));
    stamp(p, 1);
    CK(run_inverse_zy(p, batch));
    stamp(p, 2);
    const bool t_mfma = T && p.quads_collapsed;
    bispec_status s = BISPEC_OK;
    if (first < last || t_mfma) {
        const int mode = p.precision == BISPEC_SPLIT_BF16 ? PG_MODE_SPLIT : PG_MODE_F32;
        TailPairs tp{};
        tp.npairs = (int)p.pairs.size();
        for (int q = 0; q < tp.npairs; ++q) {
            tp.R[q] = p.pairs[q].R;
            tp.W[q] = p.pairs[q].Wp;       // row stride of the compact rows
            tp.off[q] = p.bc_off[q] * (long long)n * n * p.max_batch;
        }
        double *pg = (double *)(ws + L.pg_partial);
        double *dense = (double *)(ws + L.pg_dense);
        CK(launch_tail(mode, t_mfma, (const float2 *)(ws + L.bc), tp, n, p.nb, batch,
                       (const uchar2 *)(ws + L.pg_pairs), p.n_mtile, tw, p.nblk_pg, pg, p.stream, p.tail_shape));
        const int64_t n_dense = (int64_t)pgram_partial_doubles(p.n_mtile, t_mfma);
        const bool refine = first < ntri && p.n_mtile_r > 0;
        float *rfields = (float *)(ws + L.fields);
        if (refine) {
            // ill-conditioned triplets: the bin fields from the compact rows
            // (still in place), then FP64 product-Gram rows of their own (or
            // FP64-product terms on the vector ALUs, after the finalisation)
            CK(launch_inverse_x_pairs((const float2 *)(ws + L.bc), n, batch, tw, (const PairDev *)(ws + L.pd),
                                      (int)p.pairs.size(), p.nb, rfields, p.stream));
            if (!p.refine_valu)
                CK(pgram_groups(p, rfields, (int64_t)n * n * n, batch, (const uchar2 *)(ws + L.pg_pairs_r),
                                p.pg_gtile_r, true, p.nblk_r, (double *)(ws + L.pg_partial_r)));
        }
        stamp(p, 3);
        CK(launch_reduce_dense(pg, p.nblk_pg, n_dense, batch, dense, (double *)(ws + L.pg_tmp), p.stream));
        if (refine && !p.refine_valu)
            CK(launch_reduce_dense((const double *)(ws + L.pg_partial_r), p.nblk_r,
                                   (int64_t)refine_dense_doubles(p), batch, (double *)(ws + L.pg_dense_r),
                                   (double *)(ws + L.pg_tmp_r), p.stream));
        if (first < last) {
            s = finalize_range(p, true, dense, 1, n_dense, first, last, batch, P, B, T);
            if (s != BISPEC_OK) return s;
        }
        if (refine && p.refine_valu && B) {
            s = refine_valu_run(p, rfields, (int64_t)n * n * n, batch, B);
            if (s != BISPEC_OK) return s;
        }
        if (t_mfma) {
            s = finalize_range(p, true, dense, 1, n_dense, t_first, t_last, batch, P, B, T);
            if (s != BISPEC_OK) return s;
        }
    }
    if (T && !p.quads_collapsed) {
        // general quads: bin fields in HBM and the VALU contraction
        float *fields = (float *)(ws + L.fields);
        const int64_t vol = (int64_t)n * n * n;
        for (size_t q = 0; q < p.pairs.size(); ++q) {
            const int b = 2 * (int)q;
            const PairGeom &g = p.pairs[q];
            float2 *bc = (float2 *)(ws + L.bc) + p.bc_off[q] * (int64_t)n * n * p.max_batch;
            CK(launch_inverse_x(bc, (int64_t)n * n * g.Wp, n, batch, tw, g, fields + (int64_t)b * vol,
                                b + 1 < p.nb ? fields + (int64_t)(b + 1) * vol : nullptr, (int64_t)p.nb * vol,
                                p.stream));
        }
        return valu_terms(p, fields, t_first, t_last, batch, P, B, T);
    }
    return BISPEC_OK;
}

bispec_status run_estimate(bispec_plan_s &p, const float *delta, int batch, double *P, double *B, double *T) {
    bispec_status s = run_estimate_body(p, delta, batch, P, B, T);
    stamp_rest(p, 3);
    return s;
}

}  // namespace

extern "C" {

bispec_status bispec_plan(const bispec_plan_desc *desc, bispec_plan_t *out) {
    try {
        return plan_impl(desc, out);
    } catch (const std::bad_alloc &) {
        return BISPEC_E_OOM;
    } catch (...) {
        return BISPEC_E_INVALID;
    }
}

bispec_status bispec_plan_footprint(bispec_plan_t plan, int32_t batch, size_t *bytes) {
    if (!plan || !bytes || batch < 1) return BISPEC_E_INVALID;
    *bytes = make_layout(*plan, batch).total;
    return BISPEC_OK;
}

bispec_status bispec_set_workspace(bispec_plan_t plan, void *dev_ptr, size_t bytes) {
    if (!plan || !dev_ptr) return BISPEC_E_INVALID;
    if (((uintptr_t)dev_ptr) % kAlign) return BISPEC_E_INVALID;
    if (bytes < make_layout(*plan, plan->max_batch).total) return BISPEC_E_NO_WORKSPACE;
    plan->drop_graphs();
    plan->ws = dev_ptr;
    plan->ws_bytes = bytes;
    plan->resident = 0;
    plan->ws_fields = needs_fields(*plan);
    try {
        bispec_status s = upload_tables(*plan);
        if (s != BISPEC_OK) plan->ws = nullptr;
        return s;
    } catch (...) {
        plan->ws = nullptr;
        return BISPEC_E_OOM;
    }
}

bispec_status bispec_set_precision(bispec_plan_t plan, int32_t precision) {
    if (!plan || precision < BISPEC_FP32 || precision > BISPEC_FP32_VALU) return BISPEC_E_INVALID;
    plan->precision = precision;
    plan->drop_graphs();
    return BISPEC_OK;
}

bispec_status bispec_set_stream(bispec_plan_t plan, void *stream) {
    if (!plan) return BISPEC_E_INVALID;
    plan->stream = (hipStream_t)stream;
    plan->drop_graphs();
    return BISPEC_OK;
}

bispec_status bispec_plan_query(bispec_plan_t plan, int32_t *n_tri, int32_t *tri_out, double *counts_out,
                                double *quad_counts_out) {
    if (!plan) return BISPEC_E_INVALID;
    const int nt = (int)plan->tri.size() / 3;
    if (n_tri) *n_tri = nt;
    if (tri_out) std::memcpy(tri_out, plan->tri.data(), sizeof(int32_t) * 3 * nt);
    if (counts_out) std::memcpy(counts_out, plan->tri_count.data(), sizeof(double) * nt);
    if (quad_counts_out)
        std::memcpy(quad_counts_out, plan->quad_count.data(), sizeof(double) * plan->quad_count.size());
    return BISPEC_OK;
}

bispec_status bispec_plan_query_quads(bispec_plan_t plan, int32_t *n_quad, int32_t *quad_out) {
    if (!plan) return BISPEC_E_INVALID;
    const int nq = (int)plan->quad.size() / 4;
    if (n_quad) *n_quad = nq;
    if (quad_out) std::memcpy(quad_out, plan->quad.data(), sizeof(int32_t) * 4 * nq);
    return BISPEC_OK;
}

bispec_status bispec_plan_mode_counts(bispec_plan_t plan, int64_t *modes_out) {
    if (!plan || !modes_out) return BISPEC_E_INVALID;
    std::memcpy(modes_out, plan->modes.data(), sizeof(int64_t) * plan->nb);
    return BISPEC_OK;
}

bispec_status bispec_bin_fields(bispec_plan_t plan, const float *delta, int32_t batch, float *fields) {
    bispec_status s = check_call(plan, delta, batch);
    if (s != BISPEC_OK) return s;
    if (!fields) {
        // keep the fields resident in the workspace for polyspec_estimate(delta = NULL)
        if (!plan->ws_fields) return BISPEC_E_NO_WORKSPACE;
        try {
            const Layout L = make_layout(*plan, plan->max_batch);
            plan->resident = 0;
            bispec_status st = run_fields(*plan, delta, batch, (float *)((char *)plan->ws + L.fields),
                                          field_len(*plan), true, spec_scale(*plan));
            stamp_rest(*plan, 3);
            if (st == BISPEC_OK) plan->resident = batch;
            return st;
        } catch (...) {
            return BISPEC_E_HIP;
        }
    }
    try {
        const int64_t len = plan->general ? plan->npix : (int64_t)plan->n * plan->n * plan->n;
        bispec_status st = run_fields(*plan, delta, batch, fields, len, false, 1.0);   // the fields as defined
        stamp_rest(*plan, 3);
        return st;
    } catch (...) {
        return BISPEC_E_HIP;
    }
}

bispec_status polyspec_estimate(bispec_plan_t plan, const float *delta, int32_t batch, double *P, double *B,
                                double *T) {
    // delta = NULL: contract the bin fields resident in the workspace
    bispec_status s = check_call(plan, delta ? delta : (const float *)plan, batch);
    if (s != BISPEC_OK) return s;
    if (!delta && (plan->resident != batch || (plan->mfma_ok && plan->precision != BISPEC_FP32_VALU)))
        return BISPEC_E_INVALID;
    try {
        bispec_plan_s &p = *plan;
        if (!p.use_graph || p.timing || p.stream == nullptr) return run_estimate(p, delta, batch, P, B, T);
        for (auto &g : p.graphs)
            if (g.delta == delta && g.P == P && g.B == B && g.T == T && g.batch == batch && g.precision == p.precision) {
                CK(hipGraphLaunch(g.exec, p.stream));
                return BISPEC_OK;
            }
        // capture the launch sequence once for these arguments
        hipGraph_t graph = nullptr;
        CK(hipStreamBeginCapture(p.stream, hipStreamCaptureModeThreadLocal));
        s = run_estimate(p, delta, batch, P, B, T);
        const hipError_t e = hipStreamEndCapture(p.stream, &graph);
        if (s != BISPEC_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return s != BISPEC_OK ? s : record(BISPEC_E_HIP, "hipStreamEndCapture", e);
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return record(BISPEC_E_HIP, "hipGraphInstantiate", ei);
        if (p.graphs.size() >= 8) {
            (void)hipGraphExecDestroy(p.graphs.front().exec);
            p.graphs.erase(p.graphs.begin());
        }
        p.graphs.push_back({delta, P, B, T, batch, p.precision, exec});
        CK(hipGraphLaunch(exec, p.stream));
        return BISPEC_OK;
    } catch (...) {
        return BISPEC_E_HIP;
    }
}

bispec_status polyspec_estimate_noalloc(bispec_plan_t plan, const float *delta, int32_t batch, double *P, double *B,
                                        double *T) {
    if (!plan || !delta) return BISPEC_E_INVALID;
    if (batch < 1 || batch > plan->max_batch) return BISPEC_E_INVALID;
    bispec_plan_s &p = *plan;
    int dev = 0;
    CK(hipGetDevice(&dev));
    void *scr = nullptr;
    CK(scratch_address(dev, &scr));
    const size_t need = make_layout(p, p.max_batch).total;
    if (need > kScratchBytes) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "the plan's workspace of %zu bytes exceeds the static scratch of %zu bytes", need,
                      kScratchBytes);
        return BISPEC_E_NO_WORKSPACE;
    }
    // The plan's own workspace is set aside for the call and restored after.
    struct Swap {
        bispec_plan_s &p;
        void *ws;
        size_t bytes;
        bool fields;
        ~Swap() {
            p.ws = ws;
            p.ws_bytes = bytes;
            p.ws_fields = fields;
        }
    } swap{p, p.ws, p.ws_bytes, p.ws_fields};
    p.ws = scr;
    p.ws_bytes = kScratchBytes;
    p.ws_fields = needs_fields(p);
    try {
        if (!scratch_claim(dev, p.uid)) {
            // another plan (or none) used the scratch last: this plan's tables
            bispec_status s = upload_tables(p);
            if (s != BISPEC_OK) {
                scratch_release(dev);
                return s;
            }
        }
        return run_estimate(p, delta, batch, P, B, T);
    } catch (...) {
        scratch_release(dev);
        return BISPEC_E_HIP;
    }
}

bispec_status bispec_autotune(bispec_plan_t plan, const float *delta, int32_t *nblk_out, int32_t *shape_out) {
    if (!plan) return BISPEC_E_INVALID;
    bispec_plan_s &p = *plan;
    if (!p.ws) return BISPEC_E_NO_WORKSPACE;
    if (p.mfma_ok) {
        try {
            const Layout L = make_layout(p, p.max_batch);
            char *ws = (char *)p.ws;
            const int n = p.n;
            // operands: the compact rows of the given map, else zeros
            CK(hipMemsetAsync(ws + L.bc, 0, sizeof(float2) * (size_t)n * n * p.wsum * p.max_batch, p.stream));
            if (delta) {
                double *mean = (double *)(ws + L.mean);
                CK(launch_mean(delta, n, 1, (double *)(ws + L.mean_partial), kMeanParts, mean, p.stream));
                CK(launch_forward(delta, mean, n, 1, (const float2 *)(ws + L.tw), (float2 *)(ws + L.spec),
                                  p.stream, spec_scale(p)));
                CK(run_inverse_zy(p, 1));
            }
            TailPairs tp{};
            tp.npairs = (int)p.pairs.size();
            for (int q = 0; q < tp.npairs; ++q) {
                tp.R[q] = p.pairs[q].R;
                tp.W[q] = p.pairs[q].Wp;
                tp.off[q] = p.bc_off[q] * (long long)n * n * p.max_batch;
            }
            const int mode = p.precision == BISPEC_SPLIT_BF16 ? PG_MODE_SPLIT : PG_MODE_F32;
            const bool t = p.quads_collapsed;
            hipEvent_t e0, e1;
            CK(hipEventCreate(&e0));
            CK(hipEventCreate(&e1));
            // candidates: the wide, twin and deep shapes (those that fit the
            // tile count) at the default block count and two and four times
            // it, each timed (tail kernel plus the reduction of its partials)
            // as the median of five runs after one warm-up; a later candidate
            // must win by 3 % to be kept (the first ones write and reduce
            // fewer partial tiles)
            float best = 1e30f;
            int best_nblk = p.nblk_pg;
            int best_shape = p.tail_shape;
            const int base = p.nblk_pg;
            // bring the clocks up before the first candidate is timed
            for (int rep = 0; rep < 8; ++rep)
                CK(launch_tail(mode, t, (const float2 *)(ws + L.bc), tp, n, p.nb, 1, (const uchar2 *)(ws + L.pg_pairs),
                               p.n_mtile, (const float2 *)(ws + L.tw), base, (double *)(ws + L.pg_partial), p.stream,
                               PG_SHAPE_DEEP));
            for (int sh : {PG_SHAPE_WIDE, PG_SHAPE_TWIN, PG_SHAPE_DEEP}) {
                if (!tail_shape_fits(n, p.n_mtile, t, sh)) continue;
                for (int nb : {base, 2 * base, 4 * base}) {
                    if (nb > p.nblk_pg_max) continue;
                    float ms[6];
                    for (int rep = 0; rep < 6; ++rep) {
                        CK(hipEventRecord(e0, p.stream));
                        CK(launch_tail(mode, t, (const float2 *)(ws + L.bc), tp, n, p.nb, 1,
                                       (const uchar2 *)(ws + L.pg_pairs), p.n_mtile, (const float2 *)(ws + L.tw),
                                       nb, (double *)(ws + L.pg_partial), p.stream, sh));
                        CK(launch_reduce_dense((const double *)(ws + L.pg_partial), nb,
                                               (int64_t)pgram_partial_doubles(p.n_mtile, t), 1,
                                               (double *)(ws + L.pg_dense), (double *)(ws + L.pg_tmp), p.stream));
                        CK(hipEventRecord(e1, p.stream));
                        CK(hipEventSynchronize(e1));
                        CK(hipEventElapsedTime(&ms[rep], e0, e1));
                    }
                    std::sort(ms + 1, ms + 6);     // ms[0] warms up
                    const float tot = ms[3];
                    if (tot < best * 0.97f || best >= 1e30f) {
                        best = tot;
                        best_nblk = nb;
                        best_shape = sh;
                    }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            p.nblk_pg = best_nblk;
            p.tail_shape = best_shape;
            p.drop_graphs();
        } catch (...) {
            return BISPEC_E_HIP;
        }
    }
    if (nblk_out) *nblk_out = p.nblk_pg;
    if (shape_out) *shape_out = p.tail_shape;
    return BISPEC_OK;
}

static_assert(BISPEC_TAIL_DEEP == PG_SHAPE_DEEP && BISPEC_TAIL_WIDE == PG_SHAPE_WIDE &&
                  BISPEC_TAIL_TWIN == PG_SHAPE_TWIN,
              "public and internal tail shapes agree");

bispec_status bispec_set_tuning(bispec_plan_t plan, int32_t nblk, int32_t shape) {
    if (!plan || nblk < plan->nblk_pg_min || nblk > plan->nblk_pg_max) return BISPEC_E_INVALID;
    if (shape != BISPEC_TAIL_DEEP && shape != BISPEC_TAIL_WIDE && shape != BISPEC_TAIL_TWIN) return BISPEC_E_INVALID;
    plan->nblk_pg = nblk;
    plan->tail_shape = shape;
    plan->drop_graphs();
    return BISPEC_OK;
}

bispec_status bispec_plan_condition(bispec_plan_t plan, double *kappa_out) {
    if (!plan || !kappa_out) return BISPEC_E_INVALID;
    const double npix = (double)plan->npix;
    const int nt = (int)plan->tri.size() / 3;
    for (int t = 0; t < nt; ++t) {
        const double m = (double)plan->modes[plan->tri[3 * t]] * (double)plan->modes[plan->tri[3 * t + 1]] *
                         (double)plan->modes[plan->tri[3 * t + 2]];
        const double c = plan->tri_count[t];
        kappa_out[t] = c > 0 ? std::sqrt(m / (npix * c)) : std::numeric_limits<double>::infinity();
    }
    return BISPEC_OK;
}

bispec_status bispec_theta_groups(bispec_plan_t plan, int32_t b1, int32_t b2, int32_t n_cos, int32_t *group_out,
                                  double *cos_out) {
    if (!plan || !group_out || n_cos < 1) return BISPEC_E_INVALID;
    if (b1 < 0 || b1 >= plan->nb || b2 < 0 || b2 >= plan->nb) return BISPEC_E_BIN_RANGE;
    const int nt = (int)plan->tri.size() / 3;
    auto centre = [&](int b) { return 0.5 * (plan->lo[b] + plan->hi[b]); };
    const double c1 = centre(b1), c2 = centre(b2);
    for (int t = 0; t < nt; ++t) {
        // take one b1 and one b2 out of the triplet's bins; what is left is k3
        int rest[3] = {plan->tri[3 * t], plan->tri[3 * t + 1], plan->tri[3 * t + 2]};
        int left = 3;
        for (int want : {b1, b2}) {
            int at = -1;
            for (int i = 0; i < left; ++i)
                if (rest[i] == want) at = i;
            if (at < 0) {
                left = -1;
                break;
            }
            rest[at] = rest[--left];
        }
        group_out[t] = -1;
        if (cos_out) cos_out[t] = std::numeric_limits<double>::quiet_NaN();
        if (left != 1) continue;
        const double c3 = centre(rest[0]);
        // cos theta = num / den; both are exact for half-integer centres
        const double num = c1 * c1 + c2 * c2 - c3 * c3, den = 2.0 * c1 * c2;
        if (cos_out) cos_out[t] = num / den;
        if (!(num >= -den && num <= den)) continue;
        int g = (int)std::floor((num / den + 1.0) * 0.5 * n_cos);
        g = std::min(std::max(g, 0), n_cos - 1);
        // the rounded quotient can land one group off at an exact edge; group
        // g holds num / den >= -1 + 2 g / n_cos, i.e. n_cos num >= (2 g - n_cos) den
        while (g + 1 < n_cos && n_cos * num >= (2.0 * (g + 1) - n_cos) * den) ++g;
        while (g > 0 && n_cos * num < (2.0 * g - n_cos) * den) --g;
        group_out[t] = g;
    }
    return BISPEC_OK;
}

bispec_status bispec_rebin(bispec_plan_t plan, const double *B, int32_t batch, const int32_t *group,
                           int32_t n_group, double *out) {
    if (!plan || !B || !group || !out || n_group < 1) return BISPEC_E_INVALID;
    if (batch < 1 || batch > plan->max_batch) return BISPEC_E_INVALID;
    if (!plan->ws) return BISPEC_E_NO_WORKSPACE;
    const int nt = (int)plan->tri.size() / 3;
    const Layout L = make_layout(*plan, plan->max_batch);
    CK(launch_rebin(B, nt, (const double *)((const char *)plan->ws + L.tcount), group, n_group, batch, out,
                    plan->stream));
    return BISPEC_OK;
}

bispec_status bispec_graph_enable(bispec_plan_t plan, int32_t on) {
    if (!plan) return BISPEC_E_INVALID;
    plan->use_graph = on != 0;
    if (!plan->use_graph) plan->drop_graphs();
    return BISPEC_OK;
}

bispec_status bispec_estimate(bispec_plan_t plan, const float *delta, int32_t batch, double *B, double *P) {
    if (!B) return BISPEC_E_INVALID;
    return polyspec_estimate(plan, delta, batch, P, B, nullptr);
}

bispec_status trispec_estimate(bispec_plan_t plan, const float *delta, int32_t batch, double *T) {
    if (!T) return BISPEC_E_INVALID;
    return polyspec_estimate(plan, delta, batch, nullptr, nullptr, T);
}

bispec_status trispec_connected_estimate(bispec_plan_t plan, const float *delta, int32_t batch, double *T,
                                        double *Tc) {
    if (!T || !Tc) return BISPEC_E_INVALID;
    bispec_status s = check_call(plan, delta, batch);
    if (s != BISPEC_OK) return s;
    bispec_plan_s &p = *plan;
    if (p.general) return BISPEC_E_UNSUPPORTED_N;   // the spectral moments run on the half spectrum of a cube
    const int nq = (int)p.quad.size() / 4, ntri = (int)p.tri.size() / 3;
    // shells of a quad identical or disjoint: then only (a, a, b, b) has
    // pairings, and the connected T of any other quad is its raw T
    for (int q = 0; q < nq; ++q)
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                const int x = p.quad[4 * q + i], y = p.quad[4 * q + j];
                if (x != y && p.ilo2[x] < p.ihi2[y] && p.ilo2[y] < p.ihi2[x]) return BISPEC_E_INVALID;
            }
    s = polyspec_estimate(plan, delta, batch, nullptr, nullptr, T);
    if (s != BISPEC_OK) return s;
    const Layout L = make_layout(p, p.max_batch);
    char *ws = (char *)p.ws;
    const double npix = (double)p.n * p.n * p.n;
    CK(launch_shell_moments((const float2 *)(ws + L.spec), spec_elems(p.n), p.n, p.nb, batch,
                            (const int *)(ws + L.thr), kMomBlocks, (double *)(ws + L.mom_partial), p.stream));
    CK(launch_reduce_dense((const double *)(ws + L.mom_partial), kMomBlocks, 2 * p.nb, batch,
                           (double *)(ws + L.mom), (double *)(ws + L.mom_tmp), p.stream));
    CK(launch_trispec_connected(T, (const double *)(ws + L.mom), (const uchar4 *)(ws + L.terms) + ntri + p.nb,
                                (const double *)(ws + L.scale) + ntri + p.nb, npix, nq, p.nb, batch, Tc, p.stream));
    return BISPEC_OK;
}

bispec_status trispec_diag_estimate(bispec_plan_t plan, const float *delta, int32_t batch, double *Td,
                                    double *Tdc) {
    if (!Td) return BISPEC_E_INVALID;
    bispec_status s = check_call(plan, delta, batch);
    if (s != BISPEC_OK) return s;
    if (plan->dquad.empty()) return BISPEC_E_INVALID;
    if (Tdc && !plan->dconn_ok) return BISPEC_E_INVALID;
    try {
        return run_trispec_diag(*plan, delta, batch, Td, Tdc);
    } catch (...) {
        return BISPEC_E_HIP;
    }
}

bispec_status bispec_set_count_memory(size_t bytes) {
    g_count_memory.store(bytes);
    return BISPEC_OK;
}

bispec_status bispec_plan_query_dquads(bispec_plan_t plan, int32_t *n_dquad, double *counts_out) {
    if (!plan) return BISPEC_E_INVALID;
    const int ndq = (int)plan->dquad.size() / 5;
    if (n_dquad) *n_dquad = ndq;
    if (counts_out)
        for (int t = 0; t < ndq; ++t) counts_out[t] = plan->dq_count[t];
    return BISPEC_OK;
}

bispec_status bispec_timing_enable(bispec_plan_t plan, int32_t on) {
    if (!plan) return BISPEC_E_INVALID;
    plan->timing = on != 0;
    return BISPEC_OK;
}

bispec_status bispec_timing_read(bispec_plan_t plan, double *stage_ms, int32_t *calls) {
    if (!plan) return BISPEC_E_INVALID;
    double acc[BISPEC_N_STAGES] = {0, 0, 0, 0};
    const size_t nrec = plan->ev_rec.size() / 5;
    bispec_status st = BISPEC_OK;
    for (size_t r = 0; r < nrec; ++r) {
        hipEvent_t *e = &plan->ev_rec[5 * r];
        if (hipEventSynchronize(e[4]) != hipSuccess) st = BISPEC_E_HIP;
        for (int k = 0; k < BISPEC_N_STAGES; ++k) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e[k], e[k + 1]) != hipSuccess) st = BISPEC_E_HIP;
            acc[k] += ms;
        }
    }
    plan->ev_pool.insert(plan->ev_pool.end(), plan->ev_rec.begin(), plan->ev_rec.end());
    plan->ev_rec.clear();
    if (stage_ms)
        for (int k = 0; k < BISPEC_N_STAGES; ++k) stage_ms[k] = acc[k];
    if (calls) *calls = (int32_t)nrec;
    return st;
}

bispec_status bispec_destroy(bispec_plan_t plan) {
    delete plan;
    return BISPEC_OK;
}

const char *bispec_last_error(void) { return g_last_error; }

const char *bispec_status_string(bispec_status s) {
    switch (s) {
        case BISPEC_OK: return "ok";
        case BISPEC_E_INVALID: return "invalid argument";
        case BISPEC_E_UNSUPPORTED_N: return "n_side must be a power of two in [8, 512]";
        case BISPEC_E_BIN_RANGE: return "bin edges must satisfy 0 <= k_lo < k_hi <= N/2";
        case BISPEC_E_EMPTY_BIN: return "a shell contains no mode";
        case BISPEC_E_NO_WORKSPACE: return "workspace missing or smaller than the footprint";
        case BISPEC_E_OOM: return "device allocation failed";
        case BISPEC_E_HIP: return "HIP runtime error";
        case BISPEC_E_NUMERIC: return "an FFT count was not close to an integer";
    }
    return "unknown status";
}

}  // extern "C"
