/*
 * hepkref -- CPU oracle for the columnar jagged-array analysis kernels of
 * "Processing Columnar Collider Data with GPU-Accelerated Kernels"
 * (Pata & Spiropulu, arXiv:1906.06242).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Data model (Sec. II): a collection of N events and M objects is an int64
 * offsets array of N+1 entries plus one content array of M entries per
 * feature; objects of event e are offsets[e] .. offsets[e+1]-1.  Object masks
 * (M bytes) and event masks (N bytes) are chained between calls (Sec. III).
 *
 * Arithmetic: every cut, difference, square and sum of per-object data is
 * float32, each operation rounded on its own (built with -ffp-contract=off,
 * no fast-math); histogram weights are summed in float64.  float16 content is
 * widened to float32 exactly before any arithmetic.
 *
 * All pointers are host pointers.  Functions return 0 on success and a
 * negative value on invalid arguments (see HEPKREF_E*).
 */
#ifndef HEPKREF_H
#define HEPKREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HEPKREF_OK = 0, HEPKREF_EINVAL = -1, HEPKREF_EUNSUPPORTED = -3 };

/* content element types */
enum { HEPKREF_F32 = 0, HEPKREF_F16 = 1, HEPKREF_I32 = 2, HEPKREF_U8 = 3 };

/* comparisons of a column against a threshold: v > t, v >= t, v < t, v <= t,
 * |v| < t, |v| <= t.  Float columns compare against `thr`, int32 columns
 * against `ithr`. */
enum { HEPKREF_GT = 0, HEPKREF_GE, HEPKREF_LT, HEPKREF_LE, HEPKREF_ABS_LT, HEPKREF_ABS_LE };

typedef struct {
    const void *col;
    int32_t dtype;
    int32_t op;
    float thr;
    int32_t ithr;
} hepkref_cut;

/* per-event reductions over the objects of each event (Sec. III) */
enum { HEPKREF_COUNT = 0, HEPKREF_SUM, HEPKREF_MAX, HEPKREF_MIN, HEPKREF_ARGMAX, HEPKREF_ARGMIN,
       HEPKREF_PROD };

/* exact float16 -> float32 widening (IEEE 754 binary16) */
float hepkref_half_to_float(uint16_t h);

/* mask_out[i] = mask_in[i] && cut_0(i) && ... && cut_{k-1}(i), as 0/1 bytes */
int hepkref_select(const hepkref_cut *cuts, int32_t n_cuts, int64_t n,
                   const uint8_t *mask_in, uint8_t *mask_out);

/* Per-event reduction.  COUNT -> int32 out (number of masked-in objects) and
 * optional offsets_out (int64, N+1, exclusive prefix sum of the counts);
 * SUM -> float32 left-to-right sum starting at 0; PROD -> float32
 * left-to-right product starting at 1; MAX/MIN -> float32 value
 * (-inf/+inf when empty) and optional int32 out_arg (local index of the first
 * extremum, -1 when empty); ARGMAX/ARGMIN -> int32 local index into out.
 * Events with evt_mask == 0 get the empty result. */
int hepkref_reduce(int32_t op, const int64_t *offsets, int64_t n_events,
                   const void *content, int32_t dtype,
                   const uint8_t *obj_mask, const uint8_t *evt_mask,
                   void *out, int32_t *out_arg, int64_t *offsets_out);

/* Delta-R matching of collection a against collection b in the same event:
 * for every object of a, the minimum over masked-in b of
 * dR^2 = deta^2 + dphi^2 (dphi wrapped once into [-pi, pi]), the local index
 * of that b (-1 if none, lowest index on ties) and
 * clean = mask_a && !(min dR^2 <= dr*dr).  Any output may be NULL. */
int hepkref_match_dr(const int64_t *off_a, const void *eta_a, const void *phi_a,
                     const uint8_t *mask_a,
                     const int64_t *off_b, const void *eta_b, const void *phi_b,
                     const uint8_t *mask_b, int32_t dtype, int64_t n_events,
                     float dr, float *min_dr2, int32_t *idx_b, uint8_t *clean);

/* Weighted fill into a histogram of nbins half-open bins [e_i, e_{i+1}) with
 * slot 0 = underflow (x < e_0) and slot nbins+1 = overflow (x >= e_nbins).
 * Accumulates counts (uint64) and sum of weights (float64); NaN x is skipped;
 * w NULL means weight 1; evt_mask NULL means every row. */
int hepkref_hist_fill(const void *x, int32_t dtype, const float *w,
                      const uint8_t *evt_mask, int64_t n,
                      const float *edges, int32_t nbins,
                      double *sumw, uint64_t *counts);

/* The same fill that also accumulates the sum of squared weights,
 * sumw2[b] += (double)w * (double)w (sumw2 may be NULL). */
int hepkref_hist_fill_w2(const void *x, int32_t dtype, const float *w,
                         const uint8_t *evt_mask, int64_t n,
                         const float *edges, int32_t nbins,
                         double *sumw, double *sumw2, uint64_t *counts);

/* ---- lookup histograms ----------------------------------------------------
 * A lookup histogram is bin edges e_0 < ... < e_nbins plus a float32 content
 * per slot, laid out like a filled histogram: contents[0] for x < e_0,
 * contents[i] for e_{i-1} <= x < e_i, contents[nbins+1] for x >= e_nbins. */

/* out[i] = the content of the slot holding x[i] (NaN x -> NaN). */
int hepkref_get_bin_contents(const void *x, int32_t dtype, int64_t n,
                             const float *edges, int32_t nbins, const float *contents,
                             float *out);

/* Linear interpolation between bin centres: with m_i = (e_{i-1} + e_i) * 0.5
 * (float32) the centre of bin i and c_i = contents[i] (i = 1..nbins):
 * out = c_1 for x <= m_1, c_nbins for x >= m_nbins, else for
 * m_i <= x < m_{i+1}: c_i + (x - m_i) * s_i with the slope
 * s_i = (c_{i+1} - c_i) / (m_{i+1} - m_i), every operation rounded to
 * float32.  NaN x -> NaN. */
int hepkref_interp(const void *x, int32_t dtype, int64_t n,
                   const float *edges, int32_t nbins, const float *contents, float *out);

/* Jet-energy-scale shift from a two-dimensional table: the row of |eta|
 * among n_eta bins (eta_edges, n_eta+1 entries; |eta| below the first edge,
 * beyond the last or NaN take the nearest row: first for NaN), then the
 * linear interpolation of hepkref_interp in pt over that row's n_pt values
 * (pt_edges, n_pt+1 entries).  delta is n_eta * n_pt float32, row-major (bin
 * values only, no under/overflow entries). */
int hepkref_jes_delta(const void *pt, const void *eta, int32_t dtype, int64_t n,
                      const float *eta_edges, int32_t n_eta,
                      const float *pt_edges, int32_t n_pt, const float *delta, float *out);

/* ---- positional kernels (Sec. III get_in_offsets / set_in_offsets,
 * select_opposite_sign_muons) and compaction ------------------------------ */

/* For every event e with evt_mask[e] (NULL: all): the n-th (from 0) object
 * of the event among those with obj_mask (NULL: all), n = idx[e] (idx NULL:
 * the constant n; negative: none); out[e] = its content (F32/F16),
 * out_index[e] (may be NULL) = its local index; otherwise fill and -1. */
int hepkref_get_in_offsets(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                           const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                           float fill, float *out, int32_t *out_index);

/* The same object of every event set to value: content F32 (value) or U8
 * (1 when value != 0, else 0). */
int hepkref_set_in_offsets(const int64_t *offsets, int64_t n_events, void *content, int32_t dtype,
                           const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                           float value);

/* Per event, the objects with obj_mask in pT order (larger pt first, NaN
 * after every number, equal pt by lower index); the first pair of positions
 * (p, r), p < r, whose charges have opposite signs gets mask_out 1, every
 * other object of the event 0. */
int hepkref_select_opposite_sign(const int64_t *offsets, int64_t n_events, const void *pt, int32_t dtype,
                                 const int32_t *charge, const uint8_t *obj_mask, uint8_t *mask_out);

/* The objects with obj_mask (NULL: all), in order, copied contiguously to
 * out (elements of 4, 2 or 1 bytes by dtype F32/I32, F16, U8); *n_out = how
 * many. */
int hepkref_compact(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                    const uint8_t *obj_mask, void *out, int64_t *n_out);

/* ---- top-quark candidate (Sec. IV: jet triplet with invariant mass closest
 * to 172 GeV) -------------------------------------------------------------- */

/* Four-momenta from (pt, eta, phi, mass), computed in float64 and rounded
 * once: px = pt cos phi, py = pt sin phi, pz = pt sinh eta,
 * E = sqrt(px^2 + py^2 + pz^2 + m^2). */
int hepkref_p4(const void *pt, const void *eta, const void *phi, const void *mass, int32_t dtype, int64_t n,
               float *px, float *py, float *pz, float *en);

/* Per event, over the triplets i < j < k of objects with obj_mask (NULL:
 * all), in float32: component sums (i + j) + k, m2 = E^2 - px^2 - py^2 - pz^2
 * left to right, M = 0 if m2 < 0 else sqrt(m2); the first triplet with the
 * smallest |M - target| (a NaN distance is never the smallest);
 * out_mass[e] = M (NaN if none), out_idx[3e..3e+2] = local indices (-1). */
int hepkref_best_triplet(const int64_t *offsets, int64_t n_events, const float *px, const float *py,
                         const float *pz, const float *en, const uint8_t *obj_mask, float target,
                         float *out_mass, int32_t *out_idx);

/* ---- the end-to-end analysis pass --------------------------------------- */

typedef struct {
    const int64_t *off;      /* N+1 */
    const void *pt, *eta, *phi;
    const void *extra;       /* muons: isolation; jets: b-tag score; else NULL */
} hepkref_coll;

typedef struct {
    int64_t n_events;
    int32_t dtype;           /* content dtype, F32 or F16 */
    hepkref_coll jets, muons, electrons;  /* electrons.off == NULL: absent */
    const float *weights;    /* float32[N] */
    const float *npu;        /* float32[N] pileup per event; NULL: absent */
} hepkref_dataset;

typedef struct {
    float mu_pt, mu_abseta, mu_iso;
    float el_pt, el_abseta;
    float jet_pt, jet_abseta;
    float dr, btag;
    int32_t min_mu, min_jet, min_b;
    int32_t n_scale;
    const float *scales;     /* n_scale jet-energy-scale factors */
    const float *edges[3];   /* HT, leading-jet pt, jet multiplicity */
    int32_t nbins[3];
    /* event weight from lookups (NULL edges: that factor is absent):
     * w * pileup(npu) * product over selected muons of sf(muon pt) */
    const float *pu_edges, *pu_contents;
    int32_t pu_nbins;
    const float *sf_edges, *sf_contents;
    int32_t sf_nbins;
    /* jet energy scale: jes_mode 0: ptv = pt * s_v (scales are factors);
     * 1: ptv = pt * (1 + s_v * delta(pt, |eta|)) (scales are shifts; delta
     * from hepkref_jes_delta's table) */
    int32_t jes_mode;
    const float *jes_eta_edges, *jes_pt_edges, *jes_delta;
    int32_t jes_n_eta, jes_n_pt;
} hepkref_query;

/* For each query q and scale v, fills histograms (HT, leading pt, nJet) of the
 * events passing the selection.  sumw[k], counts[k] (and sumw2[k] when
 * sumw2 is not NULL) point at the k-th histogram (nbins+2 slots), k running
 * over q, then v, then the three observables.  Accumulates. */
int hepkref_pipeline(const hepkref_dataset *ds, const hepkref_query *q, int32_t n_query,
                     double *const *sumw, double *const *sumw2, uint64_t *const *counts);

#ifdef __cplusplus
}
#endif
#endif
