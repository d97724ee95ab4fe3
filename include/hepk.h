/*
 * hepk -- columnar jagged-array analysis kernels for AMD MI355X (gfx950).
 *
 * A C ABI over hand-written HIP kernels for the method of "Processing
 * Columnar Collider Data with GPU-Accelerated Kernels" (Pata & Spiropulu,
 * arXiv:1906.06242): collider events stored as jagged columns are reduced to
 * weighted histograms by object selection, lepton-jet Delta-R cleaning,
 * per-event reductions, event selection and histogram filling.
 *
 * Data model (Sec. II).  A collection of N events holding M objects in total
 * is an int64 offsets array of N+1 entries plus one contiguous content array
 * of M entries per feature; the objects of event e are
 * offsets[e] .. offsets[e+1]-1.  Preconditions the caller guarantees (checked
 * only by hepk_validate_offsets): offsets[0] == 0, offsets non-decreasing,
 * offsets[N] == M.  Object masks (M bytes) and event masks (N bytes) chain
 * between calls without copying the data (Sec. III); a mask byte is "true"
 * when non-zero, and masks written by this library hold exactly 0 or 1.
 *
 * Arithmetic.  Cuts, Delta-R and sums of per-object data are float32, each
 * operation rounded on its own (no fused multiply-add contraction); float16
 * content is widened exactly to float32 first.  Histogram weights are summed
 * in float64, counts in uint64.
 *
 * Memory and ownership.  Every array argument is a device pointer into memory
 * the caller allocated and owns, unless marked (host); host structs are read
 * before the call returns.  Per-object and per-event outputs are overwritten
 * for every row; histograms accumulate into the caller's contents.  The only
 * allocations the library makes are inside a hepk_plan (released by
 * hepk_plan_destroy).
 *
 * Execution.  Every call enqueues its kernels on `stream` (NULL: the null
 * stream of the current device) and returns without synchronising.
 *
 * Errors.  Calls return HEPK_OK or a negative hepk_status; invalid
 * arguments are rejected before anything is enqueued.  hepk_last_error()
 * gives a message for the calling thread's last failure.
 */
#ifndef HEPK_H
#define HEPK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HEPK_ABI_VERSION 4
#define HEPK_MAX_CUTS 8

typedef enum hepk_status {
    HEPK_OK = 0,
    HEPK_EINVAL = -1,        /* bad argument: null pointer, negative size, bad enum */
    HEPK_EHIP = -2,          /* a HIP runtime call or kernel launch failed */
    HEPK_EUNSUPPORTED = -3,  /* valid but unsupported combination (e.g. int32 sum) */
    HEPK_ENOMEM = -4         /* device allocation failed */
} hepk_status;

typedef enum hepk_dtype { HEPK_F32 = 0, HEPK_F16 = 1, HEPK_I32 = 2, HEPK_U8 = 3 } hepk_dtype;

/* v > t, v >= t, v < t, v <= t, |v| < t, |v| <= t */
typedef enum hepk_cmp {
    HEPK_GT = 0, HEPK_GE = 1, HEPK_LT = 2, HEPK_LE = 3, HEPK_ABS_LT = 4, HEPK_ABS_LE = 5
} hepk_cmp;

/* One cut on one column: float columns (F32, F16) compare against `thr`,
 * int32 columns against `ithr`.  (host struct; `col` is a device pointer) */
typedef struct hepk_cut {
    const void *col;
    int32_t dtype;
    int32_t op;
    float thr;
    int32_t ithr;
} hepk_cut;

/* Object or event selection mask (Sec. III object/event masks; Sec. IV
 * object selection on pt and eta, event selection on event variables):
 *   mask_out[i] = (mask_in == NULL || mask_in[i]) && cut_0(i) && ... && cut_{n_cuts-1}(i)
 * for i in [0, n).  0 <= n_cuts <= HEPK_MAX_CUTS; every column has n entries.
 * NaN fails every float comparison. */
int hepk_select(const hepk_cut *cuts /* host, n_cuts */, int32_t n_cuts, int64_t n,
                const uint8_t *mask_in /* nullable, n */, uint8_t *mask_out /* n */,
                hipStream_t stream);

typedef enum hepk_reduce_op {
    HEPK_COUNT = 0, HEPK_SUM = 1, HEPK_MAX = 2, HEPK_MIN = 3, HEPK_ARGMAX = 4, HEPK_ARGMIN = 5,
    HEPK_PROD = 6
} hepk_reduce_op;

/* Per-event reduction over the objects of each event (Sec. III: the H_T kernel
 * of Listing 1 and the sum/max/min-within-offsets kernels).  An object counts
 * when obj_mask is NULL or obj_mask[i] != 0; an event with evt_mask[e] == 0
 * gets the empty result.
 *   COUNT  out int32[N]: number of counted objects; offsets_out (nullable,
 *          int64[N+1]): 0 followed by the running sum of out (the offsets of
 *          the selected sub-collection; the scan stages its partial sums in
 *          offsets_out itself, so no temporary is allocated).  content may
 *          be NULL.
 *   SUM    out float32[N]: left-to-right float32 sum from 0.0f, in object
 *          order -- the order of Listing 1's inner loop, kept exactly.
 *   MAX/MIN out float32[N]: extremum (-inf/+inf when empty); out_arg
 *          (nullable, int32[N]): local index of the first extremum, -1 if empty.
 *   ARGMAX/ARGMIN out int32[N]: that local index only.
 *   PROD   out float32[N]: left-to-right float32 product from 1.0f (the
 *          generic pairwise operator of Sec. III taken as the product; e.g. the
 *          product of per-lepton scale factors that weights an event, Sec. IV).
 * content dtype F32 or F16 for SUM/PROD/MAX/MIN/ARG*.  Reduced content must be
 * NaN-free for MAX/MIN results to be meaningful. */
int hepk_reduce(int32_t op, const int64_t *offsets /* N+1 */, int64_t n_events,
                const void *content /* M, nullable for COUNT */, int32_t dtype,
                const uint8_t *obj_mask /* nullable, M */, const uint8_t *evt_mask /* nullable, N */,
                void *out /* N */, int32_t *out_arg /* nullable, N */,
                int64_t *offsets_out /* nullable, N+1, COUNT only */, hipStream_t stream);

/* Delta-R matching of collection a against collection b of the same event
 * (Sec. III: masking objects of a first collection within a Delta-R cone of an
 * object of a second collection; Sec. IV: jet-lepton matching).  For every
 * object of a, over the objects of b with mask_b (NULL: all):
 *   dR^2 = deta^2 + dphi^2, dphi = phi_a - phi_b brought into [-pi, pi] by
 *   one subtraction or addition of 2*pi (inputs are angles in [-pi, pi]);
 *   min_dr2 = smallest dR^2 (+inf if none), idx_b = local index of that b
 *   (lowest on ties, -1 if none), clean = (mask_a == NULL || mask_a[a]) &&
 *   !(min_dr2 <= dr*dr), dr*dr rounded to float32.
 * eta/phi of both collections share `dtype` (F32 or F16).  Any output may be
 * NULL. */
int hepk_match_dr(const int64_t *off_a, const void *eta_a, const void *phi_a,
                  const uint8_t *mask_a,
                  const int64_t *off_b, const void *eta_b, const void *phi_b,
                  const uint8_t *mask_b, int32_t dtype, int64_t n_events, float dr,
                  float *min_dr2 /* nullable, Ma */, int32_t *idx_b /* nullable, Ma */,
                  uint8_t *clean_out /* nullable, Ma */, hipStream_t stream);

/* A 1-D histogram: nbins half-open bins [edges[i], edges[i+1]) with strictly
 * increasing float32 edges; slot 0 holds x < edges[0] (underflow), slots
 * 1..nbins the bins, slot nbins+1 x >= edges[nbins] (overflow).  (host struct;
 * arrays are device pointers: edges nbins+1, sumw and counts nbins+2) */
typedef struct hepk_hist {
    const float *edges;
    int32_t nbins;
    double *sumw;
    uint64_t *counts;
} hepk_hist;

/* Weighted histogram fill (Sec. III fill-histogram kernel): for each row i
 * with evt_mask[i] (NULL: all) and x[i] not NaN, counts[slot] += 1 and
 * sumw[slot] += (double)w[i] (w NULL: 1).  x dtype F32, F16 or I32 (converted
 * to float32).  Accumulates. */
int hepk_hist_fill(const void *x, int32_t dtype, const float *w /* nullable, n */,
                   const uint8_t *evt_mask /* nullable, n */, int64_t n,
                   const hepk_hist *h /* host */, hipStream_t stream);

/* The same fill that also accumulates the sum of squared weights,
 * sumw2[slot] += (double)w[i] * (double)w[i] (sumw2: device, nbins+2 float64,
 * required), the per-bin variance estimate of a weighted histogram. */
int hepk_hist_fill_w2(const void *x, int32_t dtype, const float *w /* nullable, n */,
                      const uint8_t *evt_mask /* nullable, n */, int64_t n,
                      const hepk_hist *h /* host */, double *sumw2 /* nbins+2 */, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Lookup histograms (Sec. III get_bin_contents: histogram-based reweighting;
 * Sec. IV: event weights and jet energy corrections from histogram lookups,
 * systematic corrections by linear interpolation).
 *
 * A lookup histogram has the slot layout of a filled one: strictly increasing
 * float32 edges E[0..nbins] and nbins+2 float32 contents, contents[0] for
 * x < E[0], contents[s] for E[s-1] <= x < E[s], contents[nbins+1] for
 * x >= E[nbins].  Neighbouring edges must have a finite float32 sum.
 * ------------------------------------------------------------------------- */

/* out[i] = the content of the slot holding x[i]; NaN x gives the quiet NaN
 * 0x7fc00000.  x dtype F32, F16 or I32 (converted to float32). */
int hepk_get_bin_contents(const void *x, int32_t dtype, int64_t n, const float *edges /* nbins+1 */,
                          int32_t nbins, const float *contents /* nbins+2 */, float *out /* n */,
                          hipStream_t stream);

/* Linear interpolation between bin centres.  With m_s = (E[s-1] + E[s]) * 0.5
 * the centre of bin s and c_s = contents[s] (s = 1..nbins; the under- and
 * overflow contents are not used): out = c_1 for x <= m_1, c_nbins for
 * x >= m_nbins, else, for m_i <= x < m_{i+1},
 * c_i + (x - m_i) * ((c_{i+1} - c_i) / (m_{i+1} - m_i)), each operation one
 * float32 rounding.  NaN x gives 0x7fc00000.  x dtype F32, F16 or I32. */
int hepk_interp(const void *x, int32_t dtype, int64_t n, const float *edges /* nbins+1 */, int32_t nbins,
                const float *contents /* nbins+2 */, float *out /* n */, hipStream_t stream);

/* Jet-energy-scale shift from a two-dimensional table (Sec. IV: jet energy
 * corrections from histogram lookups): the row of |eta[i]| among n_eta bins
 * (eta_edges; |eta| below the first edge or NaN takes the first row, at or
 * beyond the last edge the last row), then hepk_interp in pt[i] over that
 * row's n_pt values (pt_edges).  delta: n_eta * n_pt float32, row-major, bin
 * values only.  pt/eta dtype F32 or F16. */
int hepk_jes_delta(const void *pt, const void *eta, int32_t dtype, int64_t n,
                   const float *eta_edges /* n_eta+1 */, int32_t n_eta,
                   const float *pt_edges /* n_pt+1 */, int32_t n_pt, const float *delta /* n_eta*n_pt */,
                   float *out /* n */, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Positional kernels (Sec. III: get_in_offsets / set_in_offsets address the
 * n-th element of every row; select_opposite_sign_muons is one of the
 * specialised kernels) and compaction of a selected sub-collection.
 * ------------------------------------------------------------------------- */

/* For every event e with evt_mask[e] (NULL: all), the n-th (from 0) object of
 * the event among those with obj_mask (NULL: all), n = idx[e] (idx NULL: the
 * constant n; negative: none): out[e] = its content (F32 or F16, widened),
 * out_index[e] (nullable) = its local index; events without such an object
 * (or masked out) get out[e] = fill and out_index[e] = -1.  E.g. the leading
 * jet's pt of pT-ordered jets is n = 0 over the selected jets. */
int hepk_get_in_offsets(const int64_t *offsets /* N+1 */, int64_t n_events, const void *content /* M */,
                        int32_t dtype, const uint8_t *obj_mask /* nullable, M */,
                        const uint8_t *evt_mask /* nullable, N */, const int32_t *idx /* nullable, N */,
                        int32_t n, float fill, float *out /* N */, int32_t *out_index /* nullable, N */,
                        hipStream_t stream);

/* The same object of every event is set to value in place: content F32
 * (value) or U8 (1 when value != 0, else 0; e.g. building a mask of the
 * first two selected jets with n = 0 then n = 1).  Other objects are left as
 * they are. */
int hepk_set_in_offsets(const int64_t *offsets /* N+1 */, int64_t n_events, void *content /* M */,
                        int32_t dtype, const uint8_t *obj_mask /* nullable, M */,
                        const uint8_t *evt_mask /* nullable, N */, const int32_t *idx /* nullable, N */,
                        int32_t n, float value, hipStream_t stream);

/* Per event, among the objects with obj_mask (NULL: all) taken in pT order
 * (larger pt first; NaN pt after every number; equal pt by lower index): the
 * first object that has a later object of opposite charge sign (a > 0 > b or
 * a < 0 < b) and its first such partner get mask_out = 1, every other object
 * of the event 0 (all 0 when no such pair).  pt F32 or F16, charge int32. */
int hepk_select_opposite_sign(const int64_t *offsets /* N+1 */, int64_t n_events, const void *pt /* M */,
                              int32_t dtype, const int32_t *charge /* M */, const uint8_t *obj_mask /* nullable, M */,
                              uint8_t *mask_out /* M */, hipStream_t stream);

/* Compaction: the objects with obj_mask (NULL: all), in order, written
 * contiguously to out: the content of a collection whose offsets are
 * offsets_out, the exclusive prefix counts of the kept objects per event
 * (hepk_reduce COUNT with the same obj_mask and its offsets_out; N+1
 * entries).  n_out (= offsets_out[N]) bounds the writes.  Elements of dtype
 * F32/I32 (4 bytes), F16 (2) or U8 (1) are moved bit for bit. */
int hepk_compact(const int64_t *offsets /* N+1 */, int64_t n_events, const void *content /* M */, int32_t dtype,
                 const uint8_t *obj_mask /* nullable, M */, const int64_t *offsets_out /* N+1 */, int64_t n_out,
                 void *out /* n_out */, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Top-quark candidate (Sec. IV high-level variable reconstruction: the jet
 * triplet with invariant mass closest to M = 172 GeV).
 * ------------------------------------------------------------------------- */

/* Four-momenta from (pt, eta, phi, mass), float32:
 * px = pt cos phi, py = pt sin phi, pz = pt sinh eta,
 * E = sqrt(px^2 + py^2 + pz^2 + mass^2), with the device's float32 cos, sin
 * and sinh (a few ulp; not bit-reproducible across machines). */
int hepk_p4(const float *pt, const float *eta, const float *phi, const float *mass, int64_t n,
            float *px, float *py, float *pz, float *en, hipStream_t stream);

/* Per event, over the triplets i < j < k of objects with obj_mask (NULL:
 * all): M = sqrt(E^2 - px^2 - py^2 - pz^2) of the summed four-momenta (sums
 * (i + j) + k per component; products and differences each one float32
 * rounding, left to right; a negative square gives 0; correctly rounded
 * square root), the triplet with the smallest |M - target| (first in
 * (i, j, k) order on ties; NaN distances never chosen).  out_mass[e] = its
 * M (NaN if none), out_idx[3e .. 3e+2] = its local indices (-1 if none).
 * Bit-reproducible: only +, -, *, sqrt. */
int hepk_best_triplet(const int64_t *offsets /* N+1 */, int64_t n_events, const float *px, const float *py,
                      const float *pz, const float *en, const uint8_t *obj_mask /* nullable, M */, float target,
                      float *out_mass /* N */, int32_t *out_idx /* 3N */, hipStream_t stream);

/* Checks offsets[0] == 0, offsets non-decreasing and offsets[n_events] ==
 * n_objects; writes the number of violations to *bad (device int64). */
int hepk_validate_offsets(const int64_t *offsets, int64_t n_events, int64_t n_objects,
                          int64_t *bad /* device, 1 */, hipStream_t stream);

/* Measurement helper, not a step of the method: reads nbytes (a multiple of
 * 16, p 16-byte aligned) with nontemporal 16-byte loads, eight in flight per
 * thread, one 256-thread workgroup per compute unit, and nothing else -- the streaming rate the HBM-bound kernels above are
 * compared with.  *sink (device, 1) may receive a value derived from the
 * data (a data-dependent store keeps the loads); its content is meaningless. */
int hepk_stream_read(const void *p, int64_t nbytes, uint32_t *sink /* device, 1 */, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The fused analysis pass.
 *
 * One launch of one persistent kernel runs the whole pass of Sec. IV's
 * analysis for every (dataset, query, jet-energy scale):
 *   muons      sel = pt > mu_pt && |eta| < mu_abseta && iso < mu_iso
 *   electrons  sel = pt > el_pt && |eta| < el_abseta            (if present)
 *   jets       clean = no selected muon or electron with dR^2 <= dr*dr
 *              (dR^2 as in hepk_match_dr); for scale s: ptv = pt * s
 *              (float32), sel = ptv > jet_pt && |eta| < jet_abseta && clean,
 *              b-tagged = sel && btag > btag_thr                (if present)
 *   event      nMu = #sel muons, nJet = #sel jets, nB = #b-tagged jets,
 *              H_T = left-to-right float32 sum of ptv over selected jets,
 *              lead = max ptv over selected jets,
 *              pass = nMu >= min_mu && nJet >= min_jet && nB >= min_b
 *   histograms for passing events, weight w: H_T, lead and (float)nJet
 * exactly as the chain hepk_select -> hepk_match_dr -> hepk_reduce ->
 * hepk_select -> hepk_hist_fill computes them.  Per-object and per-event
 * intermediates stay on chip; only the input columns are read from HBM.
 * Scheduling and fusion (Sec. IV: hundreds of kernel calls left the GPU half
 * idle) are what this entry point is for.
 * ------------------------------------------------------------------------- */

typedef struct hepk_collection {
    const int64_t *offsets;          /* n_events+1; NULL: collection absent */
    const void *pt, *eta, *phi;      /* content, dataset dtype */
    const void *extra;               /* muons: isolation (required);
                                        jets: b-tag score (optional); electrons: unused */
} hepk_collection;

typedef struct hepk_dataset {
    int64_t n_events;                /* 0 <= n_events < 2^31 */
    int32_t dtype;                   /* content dtype: HEPK_F32 or HEPK_F16 */
    hepk_collection jets, muons, electrons;
    const float *weights;            /* float32[n_events]; NULL: weight 1 */
    const float *npu;                /* float32[n_events] pileup (number of simultaneous
                                        interactions) per event; NULL: absent, then a
                                        query's pileup weight factor is not applied */
} hepk_dataset;

typedef struct hepk_query {
    float mu_pt, mu_abseta, mu_iso;
    float el_pt, el_abseta;
    float jet_pt, jet_abseta;
    float dr, btag;
    int32_t min_mu, min_jet, min_b;
    int32_t n_scale;                 /* >= 1 */
    const float *scales;             /* (host) n_scale jet-energy-scale factors, each
                                        positive and finite (else HEPK_EINVAL) */
    const float *edges[3];           /* (host) H_T, lead, nJet bin edges, nbins+1 each,
                                        strictly increasing; copied into the plan */
    int32_t nbins[3];
    /* Lookup corrections (Sec. IV: event weights and jet energy corrections
     * from histogram lookups), all (host) tables copied into the plan;
     * NULL edges: that correction is absent.  Lookup histograms have the
     * layout of hepk_get_bin_contents (contents nbins+2).
     *   event weight = (w * pu(npu)) * (product, left to right from 1, of
     *   sf(pt) over the event's selected muons), each product one float32
     *   rounding; pu applies only to datasets with an npu column.
     *   jes_mode 0: the scales are factors, ptv = pt * s (positive, finite);
     *   jes_mode 1: the scales are shifts s (finite, any sign) and
     *   ptv = pt * (1 + s * delta), delta = hepk_jes_delta(pt, eta) of the
     *   table (jes_eta_edges, jes_pt_edges, jes_delta). */
    const float *pu_edges, *pu_contents;   /* pu_nbins+1, pu_nbins+2 */
    int32_t pu_nbins;
    const float *sf_edges, *sf_contents;   /* sf_nbins+1, sf_nbins+2 */
    int32_t sf_nbins;
    int32_t jes_mode;
    const float *jes_eta_edges, *jes_pt_edges, *jes_delta;  /* n_eta+1, n_pt+1, n_eta*n_pt */
    int32_t jes_n_eta, jes_n_pt;
} hepk_query;

/* Launch configuration of the fused kernel.  block: threads per workgroup
 * (256, 512 or 1024; 1024 with ev_per_thread 1 only: the workgroups that
 * share one LDS copy of many histograms); ev_per_thread: events per thread in
 * a tile (1 or 2); hist_mode:
 * 0 = per-workgroup LDS histograms merged with global atomics, 1 = global
 * atomics only; grid: workgroups (0: enough to fill the device). */
typedef struct hepk_tune {
    int32_t block;
    int32_t ev_per_thread;
    int32_t hist_mode;
    int32_t grid;
} hepk_tune;

typedef struct hepk_plan_s *hepk_plan;

/* Builds a plan for datasets ds[0..n_ds) and queries q[0..n_query): uploads
 * the dataset and query tables (with a copy of every query's bin edges) to
 * device memory and fixes the launch configuration (tune NULL: a default for
 * the device).  Histogram layout in the sumw/counts buffers given to
 * hepk_pipeline: one block of nbins+2 slots per (dataset, query, scale,
 * observable), blocks ordered dataset-major, then query, then scale, then
 * observable (H_T, lead, nJet); hepk_plan_hist_offset gives each block. */
int hepk_plan_create(const hepk_dataset *ds /* host, n_ds */, int32_t n_ds,
                     const hepk_query *q /* host, n_query */, int32_t n_query,
                     const hepk_tune *tune /* host, nullable */, hepk_plan *out /* host */);

/* Options of hepk_plan_create_ex (zero-initialised: hepk_plan_create). */
typedef struct hepk_plan_opts {
    hepk_tune tune;          /* block == 0: the default launch configuration
                                (block 512, or 1024 when a query has several
                                scales; one event per thread; LDS histograms) */
    int32_t shared_hist;     /* 1: all datasets accumulate into one set of histograms
                                (the layout of dataset 0), e.g. the chunks of one sample */
    int32_t reserve_bins;    /* > 0: every query slot reserves reserve_bins bins per
                                histogram so hepk_plan_set_query can later install any query
                                with nbins <= reserve_bins (and n_scale <= the slot's) */
    int32_t sumw2;           /* 1: the plan can also keep sums of squared weights
                                (hepk_pipeline_w2); implied by lookup corrections */
    int64_t hist_arena_slots;/* > 0: the histogram buffers have at least this many slots
                                (hepk_plan_hist_slots), an arena in which
                                hepk_plan_set_query_at places each query's histograms */
} hepk_plan_opts;

int hepk_plan_create_ex(const hepk_dataset *ds /* host, n_ds */, int32_t n_ds,
                        const hepk_query *q /* host, n_query */, int32_t n_query,
                        const hepk_plan_opts *opts /* host, nullable */, hepk_plan *out /* host */);

/* Replaces the query in slot `slot` (q NULL: the slot goes idle and is
 * skipped).  The new thresholds and edges are staged in the plan's pinned
 * host memory (a ring of 32 staging areas, each reused only after its
 * previous copy has executed) and copied on `stream`, so launches enqueued on
 * that stream afterwards see the new query and earlier ones the old.  The
 * slot's histogram blocks stay where they are; with reserve_bins > 0 the
 * blocks have reserve_bins + 2 slots of which the first nbins + 2 are used.
 * Updates and launches of one plan must go to one stream.  A query with
 * lookup corrections is installed only by plan creation (HEPK_EUNSUPPORTED
 * here). */
int hepk_plan_set_query(hepk_plan p, int32_t slot, const hepk_query *q /* host, nullable */,
                        hipStream_t stream);

/* hepk_plan_set_query that also places the slot's histograms: the query's
 * blocks are laid out compactly (nbins+2 per observable, observables then
 * scales) from slot hist_slot0 of the histogram buffers, which must hold
 * them (HEPK_EINVAL otherwise).  The caller owns the placement, e.g. an
 * allocator over an arena made with opts.hist_arena_slots, so histogram memory
 * is what gates which queries a server can hold at once; queries with up to
 * reserve_bins bins per histogram fit a slot's edge table.  Later
 * hepk_plan_set_query calls on the slot keep this placement. */
int hepk_plan_set_query_at(hepk_plan p, int32_t slot, const hepk_query *q /* host */, int64_t hist_slot0,
                           hipStream_t stream);

/* Total histogram slots of the plan (length of sumw and counts). */
int hepk_plan_hist_slots(hepk_plan p, int64_t *n_slots /* host */);

/* Slot offset and bin count of histogram (dataset d, query iq, scale v, observable h). */
int hepk_plan_hist_offset(hepk_plan p, int32_t d, int32_t iq, int32_t v, int32_t h,
                          int64_t *offset /* host */, int32_t *nbins /* host */);

/* The launch configuration the plan uses. */
int hepk_plan_get_tune(hepk_plan p, hepk_tune *tune /* host */);

/* Runs the fused pass, accumulating into sumw/counts (hepk_plan_hist_slots
 * entries each). */
int hepk_pipeline(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream);

/* Per-event record of the fused pass for one (event, query, scale): the
 * intermediate values of Sec. IV's selection -- the number of selected muons,
 * of selected and of b-tagged jets, H_T (Listing 1's left-to-right float32
 * sum of the selected jets' scaled pt) and the leading selected jet's scaled
 * pt (-inf when none), as the chain of primitives would compute them.
 *   state 3: the event passes (it was filled into the histograms);
 *   state 2: its jets were walked and it fails;
 *   state 1: it was shown unable to pass before the walk (fewer selected
 *            muons than min_mu, fewer jets before any cut than min_jet, or --
 *            several scales and jet_pt >= 0 -- fewer selected or b-tagged jets
 *            at the largest scale than required); only n_mu is meaningful,
 *            the other fields hold 0, 0, 0.0f and -inf. */
typedef struct hepk_event_record {
    int32_t n_mu, n_jet, n_b, state;
    float ht, lead;
    float w;            /* the event's weight for this query (with lookup factors) */
    int32_t reserved;   /* 0 */
} hepk_event_record;

/* Where the records of hepk_pipeline_debug go: the record of event e of
 * dataset d for scale v of query slot q is rec[base + v * stride + e]
 * (stride = total events of the plan's datasets); *n_records (host) is the
 * length rec must have.  Any output pointer may be NULL. */
int hepk_plan_debug_layout(hepk_plan p, int32_t d, int32_t q, int64_t *base /* host */,
                           int64_t *stride /* host */, int64_t *n_records /* host */);

/* hepk_pipeline that also writes every event's record for every active query
 * and scale into rec (device, hepk_plan_debug_layout's n_records entries;
 * records of idle slots are left as they are).  Same kernels as
 * hepk_pipeline, instantiated with the record stores; the histograms it adds
 * are the same.  For checking the pass event by event; not for production
 * passes. */
int hepk_pipeline_debug(hepk_plan p, double *sumw, uint64_t *counts, hepk_event_record *rec /* device */,
                        hipStream_t stream);

/* hepk_pipeline that also accumulates the sums of squared weights,
 * sumw2[slot] += (double)w * (double)w per fill (hepk_plan_hist_slots
 * float64 entries), the per-bin variance of weighted histograms.  The plan
 * must have lookup corrections or opts.sumw2 (else HEPK_EINVAL). */
int hepk_pipeline_w2(hepk_plan p, double *sumw, double *sumw2, uint64_t *counts, hipStream_t stream);

/* Same as hepk_pipeline, over datasets [d0, d0 + nd) only. */
int hepk_pipeline_range(hepk_plan p, int32_t d0, int32_t nd, double *sumw, uint64_t *counts,
                        hipStream_t stream);

/* Same as hepk_pipeline, launched as a HIP graph owned by the plan: the
 * graph (one kernel node) is built on the first call and its arguments are
 * updated in place when sumw/counts change, so repeated passes cost one
 * graph launch each. */
int hepk_pipeline_graph(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * pass of hepk_plan_create + hepk_pipeline in one call that allocates
 * nothing.  The tables a plan would upload (datasets, work chunks, queries,
 * scales, bin edges) are copied, stream-ordered on `stream`, into a fixed
 * device array of 1 MiB that the library holds per device until the process
 * ends; tables larger than that are rejected with HEPK_EINVAL before anything
 * is enqueued.  Same kernels, launch configuration (tune NULL: the default)
 * and histogram layout as hepk_plan_create; accumulates into sumw/counts
 * (hepk_plan_hist_slots entries of that plan).  Every call on a device
 * shares its array: calls that overlap on one device (other streams or host
 * threads) race; calls on one stream follow each other safely. */
int hepk_pipeline_noalloc(const hepk_dataset *ds /* host, n_ds */, int32_t n_ds,
                          const hepk_query *q /* host, n_query */, int32_t n_query,
                          const hepk_tune *tune /* host, nullable */, double *sumw, uint64_t *counts,
                          hipStream_t stream);

/* Launch-configuration search (Sec. IV: kernel scheduling was the bottleneck
 * of the paper's GPU runs).  Times the fused pass over ds/q for every
 * candidate -- block 256/512 with 1 or 2 events per thread, block 1024 with
 * one, LDS or global-atomic
 * histograms -- with `reps` timed runs each (after one warm-up) and returns
 * the fastest in *best and its median time in *best_ms (host).  sumw/counts
 * are scratch histogram buffers of hepk_plan_hist_slots entries for this
 * ds/q (their contents are garbage afterwards).  Synchronises `stream`. */
int hepk_autotune(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                  double *sumw, uint64_t *counts, int32_t reps, hepk_tune *best /* host */,
                  float *best_ms /* host, nullable */, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Out-of-core passes (Sec. II: a cache of uncompressed columns in host memory
 * or memory-mapped files; Fig. 1: loaded in batches of a few GB of contiguous
 * arrays, the kernels running on device memory).  A streamer cuts a dataset
 * held in host memory into batches of consecutive events and runs the fused
 * pass batch by batch: the columns of the next batches are gathered
 * (pageable sources: by host threads into pinned memory) and copied to
 * device staging slots on a copy stream of the streamer while the pass over
 * the current batch runs on the caller's stream.  Results equal a pass over
 * the whole dataset resident in device memory.
 * ------------------------------------------------------------------------- */

typedef struct hepk_stream_opts {
    int64_t batch_events;    /* events per batch (0: 2^22) */
    int32_t n_buffers;       /* device staging slots, 1..8 (0: 2, double buffering) */
    int32_t host_threads;    /* threads gathering pageable sources (0: 8) */
    hepk_tune tune;          /* launch configuration (block 0: the default) */
} hepk_stream_opts;

typedef struct hepk_streamer_s *hepk_streamer;

/* host_ds: a dataset whose offsets and columns are HOST pointers (pageable,
 * memory-mapped or pinned); they and the queries' host arrays must stay valid
 * and unchanged until hepk_streamer_destroy.  Allocates the staging slots
 * (n_buffers x the largest batch's bytes on the device, and as much pinned
 * host memory for pageable sources). */
int hepk_streamer_create(const hepk_dataset *host_ds /* host */, const hepk_query *q /* host, n_query */,
                         int32_t n_query, const hepk_stream_opts *opts /* host, nullable */,
                         hepk_streamer *out /* host */);

/* Histogram slots a pass fills (the layout of hepk_plan_create over one
 * dataset with these queries). */
int hepk_streamer_hist_slots(hepk_streamer s, int64_t *n_slots /* host */);

/* One pass over every batch, accumulating into sumw/counts (device).  Returns
 * once every batch is enqueued (the host waits only for staging slots to come
 * free); synchronise `stream` before reading the histograms. */
int hepk_stream_pass(hepk_streamer s, double *sumw, uint64_t *counts, hipStream_t stream);

int hepk_streamer_destroy(hepk_streamer s);

int hepk_plan_destroy(hepk_plan p);

/* Message for the calling thread's last non-OK return ("" if none). */
const char *hepk_last_error(void);

/* HEPK_ABI_VERSION of the built library. */
int hepk_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
