// hepk_pipeline and the plan API: host side of the fused analysis pass
// (tables, work chunks, query slots, launches, graph replay, launch-shape
// search).  The kernel itself is in pipeline_kernel.hpp.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.hpp"

namespace hepk {
// the multi-scale kernels are instantiated in pipeline_ms.hip, the kernels
// that write per-event records in pipeline_dbg.hip and pipeline_ms_dbg.hip,
// the kernels with lookup corrections in pipeline_lk*.hip
extern template KernelFn pick_kernel<true, false, false>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<false, true, false>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<true, true, false>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<false, false, true>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<true, false, true>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<false, true, true>(int, bool, int, int, bool);
extern template KernelFn pick_kernel<true, true, true>(int, bool, int, int, bool);
template KernelFn pick_kernel<false, false, false>(int, bool, int, int, bool);
}  // namespace hepk

namespace hepk {

constexpr int kStageRing = 32;

// LDS layout of the active queries (compact) and whether it fits in LDS.
static void relayout(hepk_plan p) {
    int32_t acc = 0;
    for (auto &o : p->qd) {
        o.lslot0 = acc;
        int32_t per = 0;
        for (int h = 0; h < 3; ++h) {
            o.lhoff[h] = per;
            per += o.nbins[h] + 2;
        }
        o.lper_scale = per;
        if (o.active) acc += per * o.n_scale;
    }
    p->lds_slots = acc;
}

// LDS bytes of the edge and scale tables (when they are copied there).
static size_t table_lds_bytes(hepk_plan p) {
    return (p->edges_lds ? static_cast<size_t>(p->n_edges) * sizeof(float) : 0) +
           (p->scales_lds ? static_cast<size_t>(p->n_scales) * sizeof(float) : 0);
}

// LDS histograms: float64 sums (and, in lookup plans, float64 sums of squared
// weights) and uint32 counts per slot.
static size_t hist_lds_bytes(hepk_plan p) {
    return static_cast<size_t>(p->lds_slots) * ((p->lk ? 2 : 1) * sizeof(double) + sizeof(uint32_t));
}

// LDS histograms when asked for, within their budget, and when the kernel's
// own LDS, the histograms and the tables fit in one workgroup's LDS.
static bool use_lds_hist(hepk_plan p) {
    return p->tune.hist_mode == 0 && hist_lds_bytes(p) <= static_cast<size_t>(kMaxLdsHistBytes) &&
           p->lds_static_lds + hist_lds_bytes(p) + table_lds_bytes(p) <= p->lds_max;
}

// Where the kernels' bin guess can be wrong.  The guess for x is
// floor(g(x)) + 1 with g(x) = (x - lo) * inv_w in float32 (each operation
// rounded, as on the device), capped at nb; g is monotone in x.  For x in bin
// i (E[i-1] <= x < E[i]), g(x) lies between A = g(E[i-1]) and B = g(the float
// below E[i]), so the guess is too high only if B >= i, and then only where
// f = frac(g) <= B - i, and too low only if A < i - 1, and then only where
// f >= 1 - (i - 1 - A); the last bin is never too high (the cap).  Returned:
// t with every such f satisfying |f - 0.5| >= t in the kernel's float32
// (0.5 - f and f - 0.5 round monotonically in f); t > 0.5 flags none of them
// and t <= 0 all.
static float guess_bound(const float *e, int nb, float lo, float iw) {
    auto g = [&](float x) {
        const float d = x - lo;
        const float r = d * iw;
        return static_cast<double>(r);
    };
    double dhi = -1.0, dlo = 0.0;
    bool finite = true;
    for (int i = 1; i <= nb; ++i) {
        const double a = g(e[i - 1]);
        finite &= std::isfinite(a);
        dlo = std::max(dlo, (i - 1) - a);
        if (i < nb) {
            const double b = g(std::nextafter(e[i], -INFINITY));
            finite &= std::isfinite(b);
            dhi = std::max(dhi, b - i);
        }
    }
    if (!finite || dhi >= 0.5 || dlo >= 0.5) return -1.0f;
    float t = 1.5f;  // neither side can be wrong
    if (dhi >= 0.0) {
        // too high possible for f <= dhi: flagged by 0.5 - f >= 0.5 - fh
        // with fh = dhi rounded up to float32
        float fh = static_cast<float>(dhi);
        if (static_cast<double>(fh) < dhi) fh = std::nextafter(fh, INFINITY);
        t = std::min(t, 0.5f - fh);
    }
    if (dlo > 0.0) {
        // too low possible for f >= 1 - dlo: flagged by f - 0.5 >= fl - 0.5
        // with fl = 1 - dlo rounded down to float32
        float fl = static_cast<float>(1.0 - dlo);
        if (static_cast<double>(fl) > 1.0 - dlo) fl = std::nextafter(fl, -INFINITY);
        t = std::min(t, fl - 0.5f);
    }
    return t;
}

// Fills the query-dependent fields of a table entry; the caller has checked q.
static void set_qdev(QDev &o, const hepk_query &Q, const float *const edges[3]) {
    o.mu_pt = Q.mu_pt;
    o.mu_abseta = Q.mu_abseta;
    o.mu_iso = Q.mu_iso;
    o.el_pt = Q.el_pt;
    o.el_abseta = Q.el_abseta;
    o.jet_pt = Q.jet_pt;
    o.jet_abseta = Q.jet_abseta;
    o.thr2 = Q.dr * Q.dr;  // rounded once to float32
    o.btag = Q.btag;
    o.min_mu = Q.min_mu;
    o.min_jet = Q.min_jet;
    o.min_b = Q.min_b;
    o.n_scale = Q.n_scale;
    o.smax = Q.scales[0];
    o.smin = Q.scales[0];
    for (int v = 1; v < Q.n_scale; ++v) {
        o.smax = std::max(o.smax, Q.scales[v]);
        o.smin = std::min(o.smin, Q.scales[v]);
    }
    o.active = 1;
    // lookup tables: placed by the plan (lk_place); absent until then
    o.pu_nb = o.sf_nb = o.jr_nb = o.jc_nb = 0;
    o.jes_mode = Q.jes_mode;
    for (int h = 0; h < 3; ++h) {
        const int nb = Q.nbins[h];
        const float *e = edges[h];
        o.nbins[h] = nb;
        const float span = e[nb] - e[0];
        o.lo[h] = e[0];
        o.hi[h] = e[nb];
        o.inv_w[h] = (span > 0.0f && std::isfinite(span)) ? static_cast<float>(nb) / span : 0.0f;
        o.chk[h] = guess_bound(e, nb, o.lo[h], o.inv_w[h]);
    }
}

// A lookup table's edges (nb + 1, strictly increasing, neighbour sums finite).
static int check_table(const float *e, int32_t nb, const void *c, int i, const char *what) {
    HEPK_REQUIRE(e && c && nb >= 1 && nb <= (1 << 16), "query %d %s table invalid", i, what);
    for (int k = 0; k <= nb; ++k) HEPK_REQUIRE(std::isfinite(e[k]), "query %d %s edge %d not finite", i, what, k);
    for (int k = 0; k < nb; ++k) {
        HEPK_REQUIRE(e[k] < e[k + 1], "query %d %s edges not strictly increasing at %d", i, what, k);
        HEPK_REQUIRE(std::isfinite(e[k] + e[k + 1]), "query %d %s edges %d, %d: sum not finite", i, what, k, k + 1);
    }
    return HEPK_OK;
}

static bool has_lookups(const hepk_query &Q) { return Q.pu_edges || Q.sf_edges || Q.jes_mode != 0; }

static int check_query(const hepk_query &Q, int i) {
    HEPK_REQUIRE(Q.n_scale >= 1 && Q.scales, "query %d needs >= 1 scale", i);
    HEPK_REQUIRE(Q.jes_mode == 0 || Q.jes_mode == 1, "query %d jes_mode %d not 0 or 1", i, Q.jes_mode);
    for (int v = 0; v < Q.n_scale; ++v) {
        if (Q.jes_mode == 1)
            HEPK_REQUIRE(std::isfinite(Q.scales[v]), "query %d shift %d is not finite", i, v);
        else
            HEPK_REQUIRE(Q.scales[v] > 0.0f && std::isfinite(Q.scales[v]),
                         "query %d scale %d is not positive and finite", i, v);
    }
    if (Q.pu_edges)
        if (int rc = check_table(Q.pu_edges, Q.pu_nbins, Q.pu_contents, i, "pileup")) return rc;
    if (Q.sf_edges)
        if (int rc = check_table(Q.sf_edges, Q.sf_nbins, Q.sf_contents, i, "muon scale-factor")) return rc;
    if (Q.jes_mode == 1) {
        if (int rc = check_table(Q.jes_eta_edges, Q.jes_n_eta, Q.jes_delta, i, "jet-energy-scale |eta|")) return rc;
        if (int rc = check_table(Q.jes_pt_edges, Q.jes_n_pt, Q.jes_delta, i, "jet-energy-scale pt")) return rc;
        HEPK_REQUIRE(static_cast<int64_t>(Q.jes_n_eta) * Q.jes_n_pt <= (1 << 16),
                     "query %d jet-energy-scale table has more than 65536 values", i);
    }
    for (int h = 0; h < 3; ++h) {
        HEPK_REQUIRE(Q.nbins[h] >= 1 && Q.edges[h], "query %d histogram %d invalid", i, h);
        for (int k = 0; k < Q.nbins[h]; ++k)
            HEPK_REQUIRE(Q.edges[h][k] < Q.edges[h][k + 1], "query %d edges %d not strictly increasing at %d", i,
                         h, k);
    }
    return HEPK_OK;
}

static int64_t hist_base(hepk_plan p, int d) { return p->shared ? 0 : d * p->ds_block; }

// Appends the query's lookup tables to the plan's edge table and points the
// table entry at them.
static void lk_place(QDev &o, const hepk_query &Q, std::vector<float> &tab) {
    auto put = [&](const float *a, size_t n) {
        const int32_t at = static_cast<int32_t>(tab.size());
        tab.insert(tab.end(), a, a + n);
        return at;
    };
    auto axis = [](const float *e, int nb, float &lo, float &hi, float &iw) {
        lo = e[0];
        hi = e[nb];
        iw = bin_inv_width(lo, hi, nb);
    };
    if (Q.pu_edges) {
        o.pu_nb = Q.pu_nbins;
        o.pu_e = put(Q.pu_edges, Q.pu_nbins + 1);
        o.pu_c = put(Q.pu_contents, Q.pu_nbins + 2);
        axis(Q.pu_edges, Q.pu_nbins, o.pu_lo, o.pu_hi, o.pu_iw);
    }
    if (Q.sf_edges) {
        o.sf_nb = Q.sf_nbins;
        o.sf_e = put(Q.sf_edges, Q.sf_nbins + 1);
        o.sf_c = put(Q.sf_contents, Q.sf_nbins + 2);
        axis(Q.sf_edges, Q.sf_nbins, o.sf_lo, o.sf_hi, o.sf_iw);
    }
    if (Q.jes_mode == 1) {
        o.jr_nb = Q.jes_n_eta;
        o.jr_e = put(Q.jes_eta_edges, Q.jes_n_eta + 1);
        o.jc_nb = Q.jes_n_pt;
        o.jc_e = put(Q.jes_pt_edges, Q.jes_n_pt + 1);
        o.jd = put(Q.jes_delta, static_cast<size_t>(Q.jes_n_eta) * Q.jes_n_pt);
        axis(Q.jes_eta_edges, Q.jes_n_eta, o.jr_lo, o.jr_hi, o.jr_iw);
        axis(Q.jes_pt_edges, Q.jes_n_pt, o.jc_lo, o.jc_hi, o.jc_iw);
    }
}

Launch make_launch(hepk_plan p, int32_t c0, int32_t c1, double *sumw, uint64_t *counts, hepk_event_record *rec,
                   double *sumw2) {
    Launch L{};
    const bool ldsh = use_lds_hist(p);
    L.fn = rec ? (ldsh ? p->fn_lds_dbg : p->fn_glob_dbg) : (ldsh ? p->fn_lds : p->fn_glob);
    L.block = p->tune.block;
    // workgroups: as many as fit, but at least one tile per wavefront each
    const int64_t n_tiles = p->tile_pre[c1] - p->tile_pre[c0];
    L.grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(p->grid, ceil_div(n_tiles, p->tune.block / 64))));
    L.lds = (ldsh ? hist_lds_bytes(p) : 0) + table_lds_bytes(p);
    L.lds_static = ldsh ? p->lds_static_lds : p->lds_static_glob;
    L.lds_max = p->lds_max;
    L.a = p->args;
    L.a.chunk_begin = c0;
    L.a.chunk_end = c1;
    L.a.ds_slots = ldsh ? p->lds_slots : 0;
    L.a.sumw = sumw;
    L.a.counts = counts;
    L.a.sumw2 = sumw2;
    L.a.rec = rec;
    L.a.rec_events = p->ev_pre.back();
    return L;
}

// A launch whose LDS exceeds the device's is refused here (the runtime would
// abort the queue).
static int check_lds(const Launch &L) {
    HEPK_REQUIRE(L.lds_static + L.lds <= L.lds_max, "hepk_pipeline: %zu bytes of LDS per workgroup, device has %zu",
                 L.lds_static + L.lds, L.lds_max);
    return HEPK_OK;
}

int run_launch(const Launch &L, hipStream_t stream) {
    if (int rc = check_lds(L)) return rc;
    void *kargs[] = {const_cast<PipeArgs *>(&L.a)};
    HEPK_HIP(hipLaunchKernel(reinterpret_cast<const void *>(L.fn), dim3(L.grid), dim3(L.block), kargs, L.lds,
                             stream));
    return check_launch("hepk_pipeline");
}

static bool any_active(hepk_plan p) {
    for (const auto &o : p->qd)
        if (o.active) return true;
    return false;
}

bool has_work(hepk_plan p, int32_t c0, int32_t c1) {
    return c1 > c0 && p->tile_pre[c1] != p->tile_pre[c0] && any_active(p);
}

void free_plan(hepk_plan p) {
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto e : p->ring_ev) (void)hipEventDestroy(e);
    if (p->pinned) (void)hipHostFree(p->pinned);
    if (p->dev_mem) (void)hipFree(p->dev_mem);
    delete p;
}

}  // namespace hepk

static int plan_fail(hepk_plan p, int rc) {
    hepk::free_plan(p);
    return rc;
}

namespace hepk {

int plan_build(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                      const hepk_plan_opts *opts, hepk_plan *out, std::vector<char> &img, TableLayout &lay) {
    HEPK_REQUIRE(out, "hepk_plan_create: out is NULL");
    *out = nullptr;
    HEPK_REQUIRE(n_ds >= 1 && ds, "hepk_plan_create: need at least one dataset");
    HEPK_REQUIRE(n_query >= 1 && q, "hepk_plan_create: need at least one query");
    const int dtype = ds[0].dtype;
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16, "hepk_plan_create: content dtype %d unsupported", dtype);
    bool ext = false;
    for (int d = 0; d < n_ds; ++d) {
        const hepk_dataset &D = ds[d];
        HEPK_REQUIRE(D.dtype == dtype, "hepk_plan_create: dataset %d dtype differs from dataset 0", d);
        HEPK_REQUIRE(D.n_events >= 0 && D.n_events < (int64_t(1) << 31),
                     "hepk_plan_create: dataset %d n_events %lld out of [0, 2^31)", d, (long long)D.n_events);
        HEPK_REQUIRE(D.jets.offsets && D.muons.offsets, "hepk_plan_create: dataset %d lacks jet/muon offsets", d);
        // an empty dataset never touches its content columns
        const bool any = D.n_events > 0;
        HEPK_REQUIRE(!any || (D.jets.pt && D.jets.eta && D.jets.phi), "hepk_plan_create: dataset %d jet column NULL",
                     d);
        HEPK_REQUIRE(!any || (D.muons.pt && D.muons.eta && D.muons.phi),
                     "hepk_plan_create: dataset %d muon column NULL", d);
        if (D.electrons.offsets) {
            HEPK_REQUIRE(!any || (D.electrons.pt && D.electrons.eta && D.electrons.phi),
                         "hepk_plan_create: dataset %d electron column NULL", d);
            ext = true;
        }
        if (D.jets.extra) ext = true;
    }
    for (int i = 0; i < n_query; ++i) {
        int rc = check_query(q[i], i);
        if (rc) return rc;
    }
    hepk_plan_opts o{};
    if (opts) o = *opts;
    HEPK_REQUIRE(o.sumw2 == 0 || o.sumw2 == 1, "hepk_plan_create: sumw2 %d not 0 or 1", o.sumw2);
    bool lk = o.sumw2 != 0;
    for (int i = 0; i < n_query; ++i) lk |= has_lookups(q[i]);
    // default launch shape: 512 threads; 1024 when a query has several
    // jet-energy scales (one LDS copy of their many histograms shared by 16
    // wavefronts instead of 8)
    int32_t q_scales = 1;
    for (int i = 0; i < n_query; ++i) q_scales = std::max(q_scales, q[i].n_scale);
    hepk_tune t = o.tune;
    if (t.block == 0) t = hepk_tune{q_scales > 1 ? 1024 : 512, 1, 0, 0};
    HEPK_REQUIRE(t.block == 256 || t.block == 512 || t.block == 1024,
                 "hepk_plan_create: block %d not 256, 512 or 1024", t.block);
    HEPK_REQUIRE(t.ev_per_thread == 1 || t.ev_per_thread == 2, "hepk_plan_create: ev_per_thread %d not 1 or 2",
                 t.ev_per_thread);
    HEPK_REQUIRE(t.block < 1024 || t.ev_per_thread == 1, "hepk_plan_create: block 1024 takes ev_per_thread 1");
    if (lk) t.ev_per_thread = 1;  // the lookup kernels take one event per thread
    HEPK_REQUIRE(t.hist_mode == 0 || t.hist_mode == 1, "hepk_plan_create: hist_mode %d not 0 or 1", t.hist_mode);
    HEPK_REQUIRE(t.grid >= 0, "hepk_plan_create: grid < 0");
    HEPK_REQUIRE(o.reserve_bins >= 0 && o.reserve_bins < (1 << 20), "hepk_plan_create: reserve_bins out of range");

    hepk_plan p = new hepk_plan_s();
    if (hipGetDevice(&p->device) != hipSuccess) {
        set_error("hepk_plan_create: no current HIP device");
        return plan_fail(p, HEPK_EHIP);
    }
    p->n_ds = n_ds;
    p->n_q = n_query;
    p->dtype = dtype;
    p->ext = ext;
    p->shared = o.shared_hist != 0;
    p->lk = lk;

    // query slots: reserved bins/scales, global histogram blocks, edge and scale regions
    p->qd.assign(n_query, QDev{});
    p->cap_bins.assign(3 * n_query, 0);
    p->cap_scales.assign(n_query, 0);
    std::vector<float> edge_table, scales;
    int64_t gacc = 0;
    int32_t max_cap = 0, max_sc = 0;
    for (int i = 0; i < n_query; ++i) {
        QDev &e = p->qd[i];
        set_qdev(e, q[i], q[i].edges);
        p->cap_scales[i] = q[i].n_scale;
        max_sc = std::max(max_sc, q[i].n_scale);
        e.scale0 = static_cast<int32_t>(scales.size());
        for (int v = 0; v < q[i].n_scale; ++v) scales.push_back(q[i].scales[v]);
        int32_t per = 0;
        for (int h = 0; h < 3; ++h) {
            const int cap = std::max(q[i].nbins[h], o.reserve_bins);
            p->cap_bins[3 * i + h] = cap;
            max_cap = std::max(max_cap, cap);
            e.ghoff[h] = per;
            per += cap + 2;
            e.ebase[h] = static_cast<int32_t>(edge_table.size());
            edge_table.insert(edge_table.end(), q[i].edges[h], q[i].edges[h] + q[i].nbins[h] + 1);
            edge_table.resize(e.ebase[h] + cap + 1, 0.0f);
        }
        lk_place(e, q[i], edge_table);
        e.gper_scale = per;
        e.gslot0 = static_cast<int32_t>(gacc);
        gacc += static_cast<int64_t>(per) * q[i].n_scale;
    }
    if (o.hist_arena_slots < 0 || o.hist_arena_slots >= (int64_t(1) << 31)) {
        set_error("hepk_plan_create: hist_arena_slots %lld out of [0, 2^31)", (long long)o.hist_arena_slots);
        return plan_fail(p, HEPK_EINVAL);
    }
    gacc = std::max<int64_t>(gacc, o.hist_arena_slots);
    if (gacc >= (int64_t(1) << 31) || edge_table.size() >= (size_t(1) << 30)) {
        set_error("hepk_plan_create: %lld histogram slots per dataset is too many", (long long)gacc);
        return plan_fail(p, HEPK_EINVAL);
    }
    p->ds_block = gacc;
    p->n_slots = p->shared ? gacc : gacc * n_ds;
    p->n_edges = static_cast<int32_t>(edge_table.size());
    p->edges_lds = static_cast<size_t>(p->n_edges) * sizeof(float) <= static_cast<size_t>(kMaxLdsEdgeBytes);
    p->n_scales = static_cast<int32_t>(scales.size());
    p->scales_lds = scales.size() * sizeof(float) <= static_cast<size_t>(kMaxLdsScaleBytes);
    p->tune = t;
    relayout(p);

    const int tw = 64 * t.ev_per_thread;
    std::vector<DsDev> dd(n_ds);
    std::vector<int64_t> tiles(n_ds);
    p->ev_pre.assign(n_ds + 1, 0);
    for (int d = 0; d < n_ds; ++d) {
        const hepk_dataset &D = ds[d];
        DsDev &e = dd[d];
        e.n_events = D.n_events;
        e.joff = D.jets.offsets;
        e.moff = D.muons.offsets;
        e.eoff = D.electrons.offsets;
        e.jpt = D.jets.pt;
        e.jeta = D.jets.eta;
        e.jphi = D.jets.phi;
        e.jbt = D.jets.extra;
        e.mpt = D.muons.pt;
        e.meta = D.muons.eta;
        e.mphi = D.muons.phi;
        e.miso = D.muons.extra;
        e.ept = D.electrons.pt;
        e.eeta = D.electrons.eta;
        e.ephi = D.electrons.phi;
        e.w = D.weights;
        e.npu = D.npu;
        e.hist0 = hist_base(p, d);
        e.ev0 = p->ev_pre[d];
        p->ev_pre[d + 1] = p->ev_pre[d] + D.n_events;
        tiles[d] = ceil_div(D.n_events, tw);
    }

    p->ms = max_sc > 1;
    auto pick = p->lk ? (p->ms ? pick_kernel<true, false, true> : pick_kernel<false, false, true>)
                      : (p->ms ? pick_kernel<true, false, false> : pick_kernel<false, false, false>);
    auto pick_dbg = p->lk ? (p->ms ? pick_kernel<true, true, true> : pick_kernel<false, true, true>)
                          : (p->ms ? pick_kernel<true, true, false> : pick_kernel<false, true, false>);
    // With the default launch shape, a smaller workgroup is taken when the
    // histograms do not fit in LDS beside a larger one's per-wavefront
    // staging (many histograms with squared weights): LDS histograms at lower
    // occupancy beat global atomics on a few hot bins by far.
    const bool default_block = o.tune.block == 0;
    for (;;) {
        p->fn_lds = pick(dtype, ext, t.block, t.ev_per_thread, true);
        p->fn_glob = pick(dtype, ext, t.block, t.ev_per_thread, false);
        p->fn_lds_dbg = pick_dbg(dtype, ext, t.block, t.ev_per_thread, true);
        p->fn_glob_dbg = pick_dbg(dtype, ext, t.block, t.ev_per_thread, false);
        hipFuncAttributes fa{}, fg{}, fad{}, fgd{};
        int mx = 0;
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(p->fn_lds)) != hipSuccess ||
            hipFuncGetAttributes(&fg, reinterpret_cast<const void *>(p->fn_glob)) != hipSuccess ||
            hipFuncGetAttributes(&fad, reinterpret_cast<const void *>(p->fn_lds_dbg)) != hipSuccess ||
            hipFuncGetAttributes(&fgd, reinterpret_cast<const void *>(p->fn_glob_dbg)) != hipSuccess ||
            hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess) {
            set_error("hepk_plan_create: kernel or device attribute query failed");
            return plan_fail(p, HEPK_EHIP);
        }
        p->lds_static_lds = fa.sharedSizeBytes;
        p->lds_static_glob = fg.sharedSizeBytes;
        // the record kernels take the same launch only with the same LDS
        p->dbg_ok = fad.sharedSizeBytes == fa.sharedSizeBytes && fgd.sharedSizeBytes == fg.sharedSizeBytes;
        p->lds_max = static_cast<size_t>(mx);
        // the tables go to LDS only if they fit beside the kernel's own LDS
        p->edges_lds = static_cast<size_t>(p->n_edges) * sizeof(float) <= static_cast<size_t>(kMaxLdsEdgeBytes);
        p->scales_lds = static_cast<size_t>(p->n_scales) * sizeof(float) <= static_cast<size_t>(kMaxLdsScaleBytes);
        if (p->lds_static_glob + table_lds_bytes(p) > p->lds_max) p->edges_lds = p->scales_lds = false;
        if (p->lds_static_glob + table_lds_bytes(p) > p->lds_max) {
            set_error("hepk_plan_create: kernel needs %zu bytes of LDS, device has %zu", p->lds_static_glob,
                      p->lds_max);
            return plan_fail(p, HEPK_EUNSUPPORTED);
        }
        if (!default_block || t.hist_mode != 0 || use_lds_hist(p) || t.block == 256) break;
        t.block = t.block == 1024 ? 512 : 256;
        p->tune = t;
    }
    const size_t lds_hist = use_lds_hist(p) ? hist_lds_bytes(p) : 0;
    const size_t lds_bytes = lds_hist + table_lds_bytes(p);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(use_lds_hist(p) ? p->fn_lds : p->fn_glob), t.block,
            lds_bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t grid = t.grid > 0 ? t.grid : static_cast<int64_t>(per_cu) * device_cus();

    // Work: one chunk per dataset (its tiles), with the tiles of the datasets
    // before it; a launch over chunks [c0, c1) gives each workgroup an equal
    // slice of their concatenated tiles (the kernel finds its slice).
    std::vector<Chunk> chunks(n_ds);
    p->tile_pre.assign(n_ds + 1, 0);
    for (int d = 0; d < n_ds; ++d) {
        chunks[d] = Chunk{d, 0, 0, tiles[d], p->tile_pre[d]};
        p->tile_pre[d + 1] = p->tile_pre[d] + tiles[d];
    }
    p->grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(grid, 1 << 20)));
    p->tune.grid = p->grid;

    // the table image: one block for all tables
    const size_t sz_ds = sizeof(DsDev) * n_ds, sz_ch = sizeof(Chunk) * std::max<size_t>(1, chunks.size());
    const size_t sz_q = sizeof(QDev) * n_query, sz_sc = sizeof(float) * scales.size();
    const size_t sz_e = sizeof(float) * edge_table.size();
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    lay.o_ds = 0;
    lay.o_ch = al(sz_ds);
    lay.o_q = lay.o_ch + al(sz_ch);
    lay.o_sc = lay.o_q + al(sz_q);
    lay.o_e = lay.o_sc + al(sz_sc);
    lay.total = lay.o_e + al(sz_e);
    lay.max_cap = max_cap;
    lay.max_sc = max_sc;
    img.assign(lay.total, 0);
    std::memcpy(img.data() + lay.o_ds, dd.data(), sz_ds);
    if (!chunks.empty()) std::memcpy(img.data() + lay.o_ch, chunks.data(), sizeof(Chunk) * chunks.size());
    std::memcpy(img.data() + lay.o_q, p->qd.data(), sz_q);
    if (sz_sc) std::memcpy(img.data() + lay.o_sc, scales.data(), sz_sc);
    if (sz_e) std::memcpy(img.data() + lay.o_e, edge_table.data(), sz_e);
    *out = p;
    return HEPK_OK;
}

void plan_bind(hepk_plan p, char *base, const TableLayout &lay) {
    p->d_q = reinterpret_cast<QDev *>(base + lay.o_q);
    p->d_scales = reinterpret_cast<float *>(base + lay.o_sc);
    p->d_edges = reinterpret_cast<float *>(base + lay.o_e);
    PipeArgs &A = p->args;
    A.ds = reinterpret_cast<const DsDev *>(base + lay.o_ds);
    A.qs = p->d_q;
    A.scales = p->d_scales;
    A.chunks = reinterpret_cast<const Chunk *>(base + lay.o_ch);
    A.edges = p->d_edges;
    A.n_q = p->n_q;
    A.n_edges = p->n_edges;
    A.edges_in_lds = p->edges_lds ? 1 : 0;
    A.n_scales = p->n_scales;
    A.scales_in_lds = p->scales_lds ? 1 : 0;
}

}  // namespace hepk

extern "C" int hepk_plan_create_ex(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                                   const hepk_plan_opts *opts, hepk_plan *out) {
    using namespace hepk;
    clear_error();
    std::vector<char> img;
    TableLayout lay{};
    hepk_plan p = nullptr;
    if (int rc = plan_build(ds, n_ds, q, n_query, opts, &p, img, lay)) return rc;
    if (hipMalloc(&p->dev_mem, lay.total) != hipSuccess) {
        set_error("hepk_plan_create: hipMalloc of %zu bytes failed", lay.total);
        return plan_fail(p, HEPK_ENOMEM);
    }
    if (hipMemcpy(p->dev_mem, img.data(), lay.total, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hepk_plan_create: table upload failed");
        return plan_fail(p, HEPK_EHIP);
    }
    plan_bind(p, static_cast<char *>(p->dev_mem), lay);

    // staging ring: a full query table plus one slot's edges and scales per entry
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    p->stage_bytes = al(sizeof(QDev) * n_query) + al(sizeof(float) * 3 * (lay.max_cap + 1)) +
                     al(sizeof(float) * lay.max_sc);
    if (hipHostMalloc(reinterpret_cast<void **>(&p->pinned), p->stage_bytes * kStageRing, hipHostMallocDefault) !=
        hipSuccess) {
        set_error("hepk_plan_create: pinned staging allocation failed");
        return plan_fail(p, HEPK_ENOMEM);
    }
    p->ring_ev.assign(kStageRing, nullptr);
    p->ring_used.assign(kStageRing, false);
    for (int r = 0; r < kStageRing; ++r)
        if (hipEventCreateWithFlags(&p->ring_ev[r], hipEventDisableTiming) != hipSuccess) {
            set_error("hepk_plan_create: event creation failed");
            return plan_fail(p, HEPK_EHIP);
        }
    *out = p;
    return HEPK_OK;
}

extern "C" int hepk_plan_create(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                                const hepk_tune *tune, hepk_plan *out) {
    hepk_plan_opts o{};
    if (tune) o.tune = *tune;
    if (tune && tune->block == 0) {
        hepk::set_error("hepk_plan_create: block 0 not 256 or 512");
        return HEPK_EINVAL;
    }
    return hepk_plan_create_ex(ds, n_ds, q, n_query, &o, out);
}

// Installs q (NULL: idle) in a slot; at >= 0 also places the slot's
// histograms at that slot of the histogram buffers, laid out compactly.
static int set_query(hepk_plan p, int32_t slot, const hepk_query *q, int64_t at, hipStream_t stream) {
    using namespace hepk;
    HEPK_REQUIRE(p, "hepk_plan_set_query: plan is NULL");
    HEPK_REQUIRE(slot >= 0 && slot < p->n_q, "hepk_plan_set_query: slot %d out of [0, %d)", slot, p->n_q);
    if (q) {
        int rc = check_query(*q, slot);
        if (rc) return rc;
        if (has_lookups(*q)) {
            set_error("hepk_plan_set_query: lookup corrections are installed by plan creation only");
            return HEPK_EUNSUPPORTED;
        }
        HEPK_REQUIRE(q->n_scale <= p->cap_scales[slot], "hepk_plan_set_query: %d scales, slot holds %d", q->n_scale,
                     p->cap_scales[slot]);
        for (int h = 0; h < 3; ++h)
            HEPK_REQUIRE(q->nbins[h] <= p->cap_bins[3 * slot + h], "hepk_plan_set_query: %d bins, slot holds %d",
                         q->nbins[h], p->cap_bins[3 * slot + h]);
    }
    const int r = p->ring_pos;
    p->ring_pos = (p->ring_pos + 1) % kStageRing;
    if (p->ring_used[r]) HEPK_HIP(hipEventSynchronize(p->ring_ev[r]));
    char *st = p->pinned + r * p->stage_bytes;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t sz_q = sizeof(QDev) * p->n_q;
    QDev &e = p->qd[slot];
    const int max_cap = *std::max_element(p->cap_bins.begin(), p->cap_bins.end());
    float *st_e = reinterpret_cast<float *>(st + al(sz_q));
    float *st_s = reinterpret_cast<float *>(st + al(sz_q) + al(sizeof(float) * 3 * (max_cap + 1)));
    if (q && at >= 0) {
        // the compact layout of this query from `at`, inside the buffers
        int32_t per = 0;
        for (int h = 0; h < 3; ++h) per += q->nbins[h] + 2;
        const int64_t need = static_cast<int64_t>(per) * q->n_scale;
        HEPK_REQUIRE(at + need <= p->ds_block, "hepk_plan_set_query_at: slots [%lld, %lld) beyond the %lld of the plan",
                     (long long)at, (long long)(at + need), (long long)p->ds_block);
    }
    if (q) {
        set_qdev(e, *q, q->edges);
        if (at >= 0) {
            int32_t per = 0;
            for (int h = 0; h < 3; ++h) {
                e.ghoff[h] = per;
                per += q->nbins[h] + 2;
            }
            e.gper_scale = per;
            e.gslot0 = static_cast<int32_t>(at);
        }
        for (int h = 0; h < 3; ++h) std::memcpy(st_e + h * (max_cap + 1), q->edges[h], sizeof(float) * (q->nbins[h] + 1));
        std::memcpy(st_s, q->scales, sizeof(float) * q->n_scale);
    } else {
        e.active = 0;
    }
    relayout(p);
    std::memcpy(st, p->qd.data(), sz_q);
    if (q) {
        for (int h = 0; h < 3; ++h)
            HEPK_HIP(hipMemcpyAsync(p->d_edges + e.ebase[h], st_e + h * (max_cap + 1), sizeof(float) * (q->nbins[h] + 1),
                                    hipMemcpyHostToDevice, stream));
        HEPK_HIP(hipMemcpyAsync(p->d_scales + e.scale0, st_s, sizeof(float) * q->n_scale, hipMemcpyHostToDevice,
                                stream));
    }
    HEPK_HIP(hipMemcpyAsync(p->d_q, st, sz_q, hipMemcpyHostToDevice, stream));
    HEPK_HIP(hipEventRecord(p->ring_ev[r], stream));
    p->ring_used[r] = true;
    return HEPK_OK;
}

extern "C" int hepk_plan_set_query(hepk_plan p, int32_t slot, const hepk_query *q, hipStream_t stream) {
    hepk::clear_error();
    return set_query(p, slot, q, -1, stream);
}

extern "C" int hepk_plan_set_query_at(hepk_plan p, int32_t slot, const hepk_query *q, int64_t hist_slot0,
                                      hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(q, "hepk_plan_set_query_at: query is NULL (use hepk_plan_set_query to idle a slot)");
    HEPK_REQUIRE(hist_slot0 >= 0, "hepk_plan_set_query_at: hist_slot0 < 0");
    return set_query(p, slot, q, hist_slot0, stream);
}

extern "C" int hepk_plan_hist_slots(hepk_plan p, int64_t *n_slots) {
    hepk::clear_error();
    HEPK_REQUIRE(p && n_slots, "hepk_plan_hist_slots: NULL argument");
    *n_slots = p->n_slots;
    return HEPK_OK;
}

extern "C" int hepk_plan_hist_offset(hepk_plan p, int32_t d, int32_t iq, int32_t v, int32_t h, int64_t *offset,
                                     int32_t *nbins) {
    hepk::clear_error();
    HEPK_REQUIRE(p && offset && nbins, "hepk_plan_hist_offset: NULL argument");
    HEPK_REQUIRE(d >= 0 && d < p->n_ds && iq >= 0 && iq < p->n_q && h >= 0 && h < 3,
                 "hepk_plan_hist_offset: index out of range");
    const hepk::QDev &e = p->qd[iq];
    HEPK_REQUIRE(v >= 0 && v < p->cap_scales[iq], "hepk_plan_hist_offset: scale index out of range");
    *offset = hepk::hist_base(p, d) + e.gslot0 + static_cast<int64_t>(v) * e.gper_scale + e.ghoff[h];
    *nbins = e.nbins[h];
    return HEPK_OK;
}

extern "C" int hepk_plan_get_tune(hepk_plan p, hepk_tune *tune) {
    hepk::clear_error();
    HEPK_REQUIRE(p && tune, "hepk_plan_get_tune: NULL argument");
    *tune = p->tune;
    tune->hist_mode = hepk::use_lds_hist(p) ? 0 : 1;
    return HEPK_OK;
}

static int pipeline_chunks(hepk_plan p, int32_t c0, int32_t c1, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    if (!has_work(p, c0, c1)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline: plan made on device %d, current device %d", p->device, dev);
    return run_launch(make_launch(p, c0, c1, sumw, counts), stream);
}

extern "C" int hepk_pipeline(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline: histogram buffers are NULL");
    return pipeline_chunks(p, 0, p->n_ds, sumw, counts, stream);
}

extern "C" int hepk_pipeline_w2(hepk_plan p, double *sumw, double *sumw2, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_w2: plan is NULL");
    HEPK_REQUIRE(sumw && sumw2 && counts, "hepk_pipeline_w2: histogram buffers are NULL");
    HEPK_REQUIRE(p->lk, "hepk_pipeline_w2: plan made without lookup corrections or opts.sumw2");
    if (!has_work(p, 0, p->n_ds)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline_w2: plan made on device %d, current device %d", p->device, dev);
    return run_launch(make_launch(p, 0, p->n_ds, sumw, counts, nullptr, sumw2), stream);
}

extern "C" int hepk_plan_debug_layout(hepk_plan p, int32_t d, int32_t q, int64_t *base, int64_t *stride,
                                      int64_t *n_records) {
    hepk::clear_error();
    HEPK_REQUIRE(p, "hepk_plan_debug_layout: plan is NULL");
    HEPK_REQUIRE(d >= 0 && d < p->n_ds && q >= 0 && q < p->n_q, "hepk_plan_debug_layout: index out of range");
    const int64_t ne = p->ev_pre.back();
    if (base) *base = static_cast<int64_t>(p->qd[q].scale0) * ne + p->ev_pre[d];
    if (stride) *stride = ne;
    if (n_records) *n_records = static_cast<int64_t>(p->n_scales) * ne;
    return HEPK_OK;
}

extern "C" int hepk_pipeline_debug(hepk_plan p, double *sumw, uint64_t *counts, hepk_event_record *rec,
                                   hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_debug: plan is NULL");
    HEPK_REQUIRE(sumw && counts && rec, "hepk_pipeline_debug: NULL buffer");
    if (!p->dbg_ok) {
        set_error("hepk_pipeline_debug: record kernels differ in LDS from the product kernels");
        return HEPK_EUNSUPPORTED;
    }
    if (p->tile_pre[p->n_ds] == 0 || !any_active(p)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline_debug: plan made on device %d, current device %d", p->device, dev);
    return run_launch(make_launch(p, 0, p->n_ds, sumw, counts, rec), stream);
}

extern "C" int hepk_pipeline_range(hepk_plan p, int32_t d0, int32_t nd, double *sumw, uint64_t *counts,
                                   hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_range: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline_range: histogram buffers are NULL");
    HEPK_REQUIRE(d0 >= 0 && nd >= 0 && d0 + nd <= p->n_ds, "hepk_pipeline_range: datasets [%d, %d) out of [0, %d)",
                 d0, d0 + nd, p->n_ds);
    return pipeline_chunks(p, d0, d0 + nd, sumw, counts, stream);
}

extern "C" int hepk_pipeline_graph(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_graph: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline_graph: histogram buffers are NULL");
    if (p->tile_pre[p->n_ds] == 0 || !any_active(p)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline_graph: plan made on device %d, current device %d", p->device, dev);
    const Launch L = make_launch(p, 0, p->n_ds, sumw, counts);
    if (int rc = check_lds(L)) return rc;
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(L.fn);
    kp.gridDim = dim3(L.grid);
    kp.blockDim = dim3(L.block);
    kp.sharedMemBytes = static_cast<unsigned int>(L.lds);
    PipeArgs a = L.a;
    void *kargs[] = {&a};
    kp.kernelParams = kargs;
    if (!p->gexec || p->gfn != L.fn || p->ggrid != L.grid) {
        if (p->gexec) HEPK_HIP(hipGraphExecDestroy(p->gexec));
        if (p->graph) HEPK_HIP(hipGraphDestroy(p->graph));
        p->gexec = nullptr;
        p->graph = nullptr;
        HEPK_HIP(hipGraphCreate(&p->graph, 0));
        HEPK_HIP(hipGraphAddKernelNode(&p->gnode, p->graph, nullptr, 0, &kp));
        HEPK_HIP(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    } else if (std::memcmp(&p->gargs, &a, sizeof(a)) != 0 || p->glds != L.lds) {
        HEPK_HIP(hipGraphExecKernelNodeSetParams(p->gexec, p->gnode, &kp));
    }
    p->gfn = L.fn;
    p->ggrid = L.grid;
    p->gargs = a;
    p->glds = L.lds;
    HEPK_HIP(hipGraphLaunch(p->gexec, stream));
    return HEPK_OK;
}

extern "C" int hepk_plan_destroy(hepk_plan p) {
    hepk::clear_error();
    if (!p) return HEPK_OK;
    if (!p->ring_ev.empty())
        for (size_t r = 0; r < p->ring_ev.size(); ++r)
            if (p->ring_used[r]) (void)hipEventSynchronize(p->ring_ev[r]);
    hepk::free_plan(p);
    return HEPK_OK;
}

extern "C" int hepk_autotune(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                             double *sumw, uint64_t *counts, int32_t reps, hepk_tune *best, float *best_ms,
                             hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(best && sumw && counts, "hepk_autotune: NULL argument");
    HEPK_REQUIRE(reps >= 1 && reps <= 1000, "hepk_autotune: reps %d out of [1, 1000]", reps);
    const hepk_tune cands[] = {{256, 1, 0, 0}, {512, 1, 0, 0}, {1024, 1, 0, 0}, {256, 2, 0, 0}, {512, 2, 0, 0},
                               {256, 1, 1, 0}, {512, 1, 1, 0}, {1024, 1, 1, 0}, {256, 2, 1, 0}, {512, 2, 1, 0}};
    hipEvent_t e0, e1;
    HEPK_HIP(hipEventCreate(&e0));
    HEPK_HIP(hipEventCreate(&e1));
    float best_t = INFINITY;
    hepk_tune best_c{};
    std::vector<hepk_tune> seen;
    int rc = HEPK_OK;
    for (const hepk_tune &c : cands) {
        hepk_plan p = nullptr;
        rc = hepk_plan_create(ds, n_ds, q, n_query, &c, &p);
        if (rc) break;
        hepk_tune eff{};
        hepk_plan_get_tune(p, &eff);
        bool dup = false;
        for (const auto &s : seen)
            dup |= s.block == eff.block && s.ev_per_thread == eff.ev_per_thread && s.hist_mode == eff.hist_mode;
        if (dup) {
            hepk_plan_destroy(p);
            continue;
        }
        seen.push_back(eff);
        std::vector<float> ts;
        rc = hepk_pipeline(p, sumw, counts, stream);  // warm-up
        for (int r = 0; rc == HEPK_OK && r < reps; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) rc = HEPK_EHIP;
            if (rc == HEPK_OK) rc = hepk_pipeline(p, sumw, counts, stream);
            if (rc == HEPK_OK && hipEventRecord(e1, stream) != hipSuccess) rc = HEPK_EHIP;
            float ms = 0.0f;
            if (rc == HEPK_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = HEPK_EHIP;
            ts.push_back(ms);
        }
        hepk_plan_destroy(p);
        if (rc) break;
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        if (med < best_t) {
            best_t = med;
            best_c = eff;
            best_c.grid = 0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = best_c;
    if (best_ms) *best_ms = best_t;
    return HEPK_OK;
}
