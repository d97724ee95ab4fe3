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
enum { HEPKREF_F32 = 0, HEPKREF_F16 = 1, HEPKREF_I32 = 2 };

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
enum { HEPKREF_COUNT = 0, HEPKREF_SUM, HEPKREF_MAX, HEPKREF_MIN, HEPKREF_ARGMAX, HEPKREF_ARGMIN };

/* exact float16 -> float32 widening (IEEE 754 binary16) */
float hepkref_half_to_float(uint16_t h);

/* mask_out[i] = mask_in[i] && cut_0(i) && ... && cut_{k-1}(i), as 0/1 bytes */
int hepkref_select(const hepkref_cut *cuts, int32_t n_cuts, int64_t n,
                   const uint8_t *mask_in, uint8_t *mask_out);

/* Per-event reduction.  COUNT -> int32 out (number of masked-in objects) and
 * optional offsets_out (int64, N+1, exclusive prefix sum of the counts);
 * SUM -> float32 left-to-right sum starting at 0; MAX/MIN -> float32 value
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
} hepkref_query;

/* For each query q and scale v, fills histograms (HT, leading pt, nJet) of the
 * events passing the selection.  sumw[k], counts[k] point at the k-th
 * histogram (nbins+2 slots), k running over q, then v, then the three
 * observables.  Accumulates. */
int hepkref_pipeline(const hepkref_dataset *ds, const hepkref_query *q, int32_t n_query,
                     double *const *sumw, uint64_t *const *counts);

#ifdef __cplusplus
}
#endif
#endif
