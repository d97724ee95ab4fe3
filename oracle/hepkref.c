/*
 * hepkref -- CPU oracle of the jagged-array analysis kernels (arXiv:1906.06242).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.
 *
 * Plain and single-threaded on purpose: events in ascending order, objects of
 * an event in ascending content index, one operation at a time, so that each
 * function can be checked against the paper by eye.  Build with
 * -O2 -ffp-contract=off and without -ffast-math so float32 expressions are
 * rounded operation by operation.
 */
#include "hepkref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* float32 pi and 2*pi, rounded to nearest (0x40490FDB, 0x40C90FDB) */
static const float REF_PI = 0x1.921fb6p+1f;
static const float REF_TWO_PI = 0x1.921fb6p+2f;

/* IEEE 754 binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits. */
float hepkref_half_to_float(uint16_t h)
{
    uint32_t sign = (uint32_t)(h >> 15) & 1u;
    uint32_t ex = (uint32_t)(h >> 10) & 0x1fu;
    uint32_t fr = (uint32_t)h & 0x3ffu;
    float mag;
    if (ex == 0) {
        /* zero or subnormal: fr * 2^-24, exact in float32 */
        mag = ldexpf((float)fr, -24);
    } else if (ex == 31) {
        if (fr == 0) {
            mag = INFINITY;
        } else {
            /* NaN: keep the payload in the top fraction bits, as a widening does */
            uint32_t bits = (sign << 31) | 0x7f800000u | (fr << 13);
            float f;
            memcpy(&f, &bits, 4);
            return f;
        }
    } else {
        /* normal: (1 + fr/1024) * 2^(ex-15), exact in float32 */
        mag = ldexpf((float)(1024u + fr), (int)ex - 25);
    }
    return sign ? -mag : mag;
}

static float load_f(const void *col, int32_t dtype, int64_t i)
{
    if (dtype == HEPKREF_F16)
        return hepkref_half_to_float(((const uint16_t *)col)[i]);
    return ((const float *)col)[i];
}

static int valid_float_dtype(int32_t dtype)
{
    return dtype == HEPKREF_F32 || dtype == HEPKREF_F16;
}

/* ---- object and event masks (Sec. III: masks chained between kernels) ---- */

static int cmp_float(float v, int32_t op, float t)
{
    switch (op) {
    case HEPKREF_GT: return v > t;
    case HEPKREF_GE: return v >= t;
    case HEPKREF_LT: return v < t;
    case HEPKREF_LE: return v <= t;
    case HEPKREF_ABS_LT: return fabsf(v) < t;
    case HEPKREF_ABS_LE: return fabsf(v) <= t;
    }
    return 0;
}

static int cmp_int(int32_t v, int32_t op, int32_t t)
{
    switch (op) {
    case HEPKREF_GT: return v > t;
    case HEPKREF_GE: return v >= t;
    case HEPKREF_LT: return v < t;
    case HEPKREF_LE: return v <= t;
    case HEPKREF_ABS_LT: return abs(v) < t;
    case HEPKREF_ABS_LE: return abs(v) <= t;
    }
    return 0;
}

int hepkref_select(const hepkref_cut *cuts, int32_t n_cuts, int64_t n,
                   const uint8_t *mask_in, uint8_t *mask_out)
{
    if (n < 0 || n_cuts < 0 || (n > 0 && !mask_out) || (n_cuts > 0 && !cuts))
        return HEPKREF_EINVAL;
    for (int32_t k = 0; k < n_cuts; k++) {
        if (!cuts[k].col && n > 0) return HEPKREF_EINVAL;
        if (cuts[k].op < HEPKREF_GT || cuts[k].op > HEPKREF_ABS_LE) return HEPKREF_EINVAL;
        if (cuts[k].dtype != HEPKREF_F32 && cuts[k].dtype != HEPKREF_F16 &&
            cuts[k].dtype != HEPKREF_I32)
            return HEPKREF_EINVAL;
    }
    for (int64_t i = 0; i < n; i++) {
        int pass = mask_in ? (mask_in[i] != 0) : 1;
        for (int32_t k = 0; k < n_cuts; k++) {
            const hepkref_cut *c = &cuts[k];
            int ok;
            if (c->dtype == HEPKREF_I32)
                ok = cmp_int(((const int32_t *)c->col)[i], c->op, c->ithr);
            else
                ok = cmp_float(load_f(c->col, c->dtype, i), c->op, c->thr);
            pass = pass && ok;
        }
        mask_out[i] = (uint8_t)(pass ? 1 : 0);
    }
    return HEPKREF_OK;
}

/* ---- per-event reductions (Sec. III: the H_T kernel of Listing 1 and the
 * sum/max/min-within-offsets kernels).  Listing 1 visits events one by one and
 * the objects of an event in order, adding selected objects into the event's
 * output; here every event's output is written, with the empty result when
 * the event is masked out or has no selected object. ---- */

int hepkref_reduce(int32_t op, const int64_t *offsets, int64_t n_events,
                   const void *content, int32_t dtype,
                   const uint8_t *obj_mask, const uint8_t *evt_mask,
                   void *out, int32_t *out_arg, int64_t *offsets_out)
{
    if (n_events < 0 || !offsets || (n_events > 0 && !out)) return HEPKREF_EINVAL;
    if (op < HEPKREF_COUNT || op > HEPKREF_PROD) return HEPKREF_EINVAL;
    if (op != HEPKREF_COUNT) {
        if (!valid_float_dtype(dtype)) return HEPKREF_EUNSUPPORTED;
        if (!content && n_events > 0 && offsets[n_events] > 0) return HEPKREF_EINVAL;
    }
    int64_t running = 0;
    if (offsets_out) offsets_out[0] = 0;
    for (int64_t e = 0; e < n_events; e++) {
        int take_event = evt_mask ? (evt_mask[e] != 0) : 1;
        int64_t i0 = offsets[e], i1 = offsets[e + 1];
        if (op == HEPKREF_COUNT) {
            int32_t cnt = 0;
            if (take_event)
                for (int64_t i = i0; i < i1; i++)
                    if (!obj_mask || obj_mask[i]) cnt++;
            ((int32_t *)out)[e] = cnt;
            running += cnt;
            if (offsets_out) offsets_out[e + 1] = running;
        } else if (op == HEPKREF_SUM) {
            float acc = 0.0f;
            if (take_event)
                for (int64_t i = i0; i < i1; i++)
                    if (!obj_mask || obj_mask[i]) acc = acc + load_f(content, dtype, i);
            ((float *)out)[e] = acc;
        } else if (op == HEPKREF_PROD) {
            /* the pairwise operator of the generic reduction taken as the
             * float32 product, left to right from 1 */
            float prod = 1.0f;
            if (take_event)
                for (int64_t i = i0; i < i1; i++)
                    if (!obj_mask || obj_mask[i]) prod = prod * load_f(content, dtype, i);
            ((float *)out)[e] = prod;
        } else {
            int want_max = (op == HEPKREF_MAX || op == HEPKREF_ARGMAX);
            float best = want_max ? -INFINITY : INFINITY;
            int32_t bi = -1;
            if (take_event)
                for (int64_t i = i0; i < i1; i++) {
                    if (obj_mask && !obj_mask[i]) continue;
                    float v = load_f(content, dtype, i);
                    int better = want_max ? (v > best) : (v < best);
                    if (bi < 0 || better) {
                        best = v;
                        bi = (int32_t)(i - i0);
                    }
                }
            if (op == HEPKREF_MAX || op == HEPKREF_MIN) {
                ((float *)out)[e] = best;
                if (out_arg) out_arg[e] = bi;
            } else {
                ((int32_t *)out)[e] = bi;
            }
        }
    }
    return HEPKREF_OK;
}

/* ---- Delta-R matching between two collections (Sec. III: the kernel that
 * masks objects of a first collection lying within a given Delta-R of an object
 * of a second collection; Sec. IV: jet-lepton matching).
 * dR^2 = deta^2 + dphi^2, dphi brought back into [-pi, pi] once. ---- */

int hepkref_match_dr(const int64_t *off_a, const void *eta_a, const void *phi_a,
                     const uint8_t *mask_a,
                     const int64_t *off_b, const void *eta_b, const void *phi_b,
                     const uint8_t *mask_b, int32_t dtype, int64_t n_events,
                     float dr, float *min_dr2, int32_t *idx_b, uint8_t *clean)
{
    if (n_events < 0 || !off_a || !off_b) return HEPKREF_EINVAL;
    if (!valid_float_dtype(dtype)) return HEPKREF_EUNSUPPORTED;
    float thr2 = dr * dr;
    for (int64_t e = 0; e < n_events; e++) {
        for (int64_t a = off_a[e]; a < off_a[e + 1]; a++) {
            float ea = load_f(eta_a, dtype, a);
            float pa = load_f(phi_a, dtype, a);
            float best = INFINITY;
            int32_t bi = -1;
            for (int64_t b = off_b[e]; b < off_b[e + 1]; b++) {
                if (mask_b && !mask_b[b]) continue;
                float deta = ea - load_f(eta_b, dtype, b);
                float dphi = pa - load_f(phi_b, dtype, b);
                if (dphi > REF_PI)
                    dphi = dphi - REF_TWO_PI;
                else if (dphi < -REF_PI)
                    dphi = dphi + REF_TWO_PI;
                float dr2 = deta * deta + dphi * dphi;
                if (dr2 < best) {
                    best = dr2;
                    bi = (int32_t)(b - off_b[e]);
                }
            }
            if (min_dr2) min_dr2[a] = best;
            if (idx_b) idx_b[a] = bi;
            if (clean) {
                int keep = mask_a ? (mask_a[a] != 0) : 1;
                clean[a] = (uint8_t)((keep && !(best <= thr2)) ? 1 : 0);
            }
        }
    }
    return HEPKREF_OK;
}

/* ---- weighted histogram fill (Sec. III: the fill-histogram kernel) ---- */

int hepkref_hist_fill(const void *x, int32_t dtype, const float *w,
                      const uint8_t *evt_mask, int64_t n,
                      const float *edges, int32_t nbins,
                      double *sumw, uint64_t *counts)
{
    return hepkref_hist_fill_w2(x, dtype, w, evt_mask, n, edges, nbins, sumw, NULL, counts);
}

int hepkref_hist_fill_w2(const void *x, int32_t dtype, const float *w,
                         const uint8_t *evt_mask, int64_t n,
                         const float *edges, int32_t nbins,
                         double *sumw, double *sumw2, uint64_t *counts)
{
    if (n < 0 || nbins < 1 || !edges || !sumw || !counts || (n > 0 && !x))
        return HEPKREF_EINVAL;
    if (dtype != HEPKREF_F32 && dtype != HEPKREF_F16 && dtype != HEPKREF_I32)
        return HEPKREF_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        if (evt_mask && !evt_mask[i]) continue;
        float v = (dtype == HEPKREF_I32) ? (float)((const int32_t *)x)[i] : load_f(x, dtype, i);
        if (v != v) continue; /* NaN */
        int32_t b;
        if (v < edges[0]) {
            b = 0;
        } else {
            b = nbins + 1;
            for (int32_t k = 0; k < nbins; k++) {
                if (v < edges[k + 1]) {
                    b = k + 1;
                    break;
                }
            }
        }
        counts[b] += 1u;
        sumw[b] += (double)(w ? w[i] : 1.0f);
        if (sumw2) {
            double wi = (double)(w ? w[i] : 1.0f);
            sumw2[b] += wi * wi;
        }
    }
    return HEPKREF_OK;
}

/* ---- lookup histograms (Sec. III: the kernel that returns, for each element
 * of a data array, the content of the lookup-histogram bin holding it, used
 * for histogram-based reweighting; Sec. IV: event weights and jet energy
 * corrections from histogram lookups, systematic corrections by linear
 * interpolation) ---- */

static float load_any(const void *x, int32_t dtype, int64_t i)
{
    if (dtype == HEPKREF_I32) return (float)((const int32_t *)x)[i];
    return load_f(x, dtype, i);
}

/* The slot of v (not NaN) in edges[0..nbins]: the number of edges at or below v
 * (0 below the first edge, nbins+1 at or above the last). */
static int32_t edges_at_or_below(float v, const float *edges, int32_t nbins)
{
    int32_t s = 0;
    for (int32_t k = 0; k <= nbins; k++)
        if (edges[k] <= v) s++;
    return s;
}

int hepkref_get_bin_contents(const void *x, int32_t dtype, int64_t n,
                             const float *edges, int32_t nbins, const float *contents,
                             float *out)
{
    if (n < 0 || nbins < 1 || !edges || !contents || (n > 0 && (!x || !out))) return HEPKREF_EINVAL;
    if (dtype != HEPKREF_F32 && dtype != HEPKREF_F16 && dtype != HEPKREF_I32) return HEPKREF_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        float v = load_any(x, dtype, i);
        out[i] = (v != v) ? NAN : contents[edges_at_or_below(v, edges, nbins)];
    }
    return HEPKREF_OK;
}

/* centre of bin i (1..nbins), float32 */
static float bin_centre(const float *edges, int32_t i)
{
    return (edges[i - 1] + edges[i]) * 0.5f;
}

/* interpolation of one value in bins 1..nbins of c (c[i] is bin i's value) */
static float interp_one(float v, const float *edges, int32_t nbins, const float *c)
{
    if (v != v) return NAN;
    if (v <= bin_centre(edges, 1)) return c[1];
    if (v >= bin_centre(edges, nbins)) return c[nbins];
    int32_t i = 1;
    while (!(v < bin_centre(edges, i + 1))) i++;
    float m_i = bin_centre(edges, i);
    float slope = (c[i + 1] - c[i]) / (bin_centre(edges, i + 1) - m_i);
    return c[i] + (v - m_i) * slope;
}

int hepkref_interp(const void *x, int32_t dtype, int64_t n,
                   const float *edges, int32_t nbins, const float *contents, float *out)
{
    if (n < 0 || nbins < 1 || !edges || !contents || (n > 0 && (!x || !out))) return HEPKREF_EINVAL;
    if (dtype != HEPKREF_F32 && dtype != HEPKREF_F16 && dtype != HEPKREF_I32) return HEPKREF_EINVAL;
    for (int64_t i = 0; i < n; i++) out[i] = interp_one(load_any(x, dtype, i), edges, nbins, contents);
    return HEPKREF_OK;
}

int hepkref_jes_delta(const void *pt, const void *eta, int32_t dtype, int64_t n,
                      const float *eta_edges, int32_t n_eta,
                      const float *pt_edges, int32_t n_pt, const float *delta, float *out)
{
    if (n < 0 || n_eta < 1 || n_pt < 1 || !eta_edges || !pt_edges || !delta ||
        (n > 0 && (!pt || !eta || !out)))
        return HEPKREF_EINVAL;
    if (!valid_float_dtype(dtype)) return HEPKREF_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        float ae = fabsf(load_f(eta, dtype, i));
        int32_t row = (ae != ae) ? 1 : edges_at_or_below(ae, eta_edges, n_eta);
        if (row < 1) row = 1;
        if (row > n_eta) row = n_eta;
        /* the row's values as bins 1..n_pt of interp_one */
        const float *c = delta + (int64_t)(row - 1) * n_pt - 1;
        out[i] = interp_one(load_f(pt, dtype, i), pt_edges, n_pt, c);
    }
    return HEPKREF_OK;
}

/* ---- the analysis pass: object selection, lepton-jet cleaning, per-event
 * reductions, event selection and histograms (Sec. IV feature list), built from
 * the kernels above as the steering code of Sec. III would chain them. ---- */

static void *xmalloc(size_t n)
{
    return malloc(n ? n : 1);
}

/* ---- positional kernels (Sec. III: get_in_offsets and set_in_offsets
 * retrieve or set the n-th element of every row; the specialised kernel
 * select_opposite_sign_muons keeps, per event, the first two objects in pT
 * order that have opposite charges; compaction gathers the selected objects
 * into a contiguous collection laid out by the offsets of their counts) ---- */

/* Content index of the n-th (from 0) object of event e with obj_mask set
 * (every object when obj_mask is NULL); -1 when the event has fewer. */
static int64_t nth_selected(const int64_t *offsets, int64_t e, const uint8_t *obj_mask, int32_t n)
{
    if (n < 0) return -1;
    int32_t seen = 0;
    for (int64_t i = offsets[e]; i < offsets[e + 1]; i++) {
        if (obj_mask && !obj_mask[i]) continue;
        if (seen == n) return i;
        seen++;
    }
    return -1;
}

int hepkref_get_in_offsets(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                           const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                           float fill, float *out, int32_t *out_index)
{
    if (n_events < 0 || !offsets || (n_events > 0 && !out)) return HEPKREF_EINVAL;
    if (!valid_float_dtype(dtype)) return HEPKREF_EINVAL;
    if (!content && n_events > 0 && offsets[n_events] > 0) return HEPKREF_EINVAL;
    for (int64_t e = 0; e < n_events; e++) {
        int64_t i = -1;
        if (!evt_mask || evt_mask[e]) i = nth_selected(offsets, e, obj_mask, idx ? idx[e] : n);
        out[e] = (i >= 0) ? load_f(content, dtype, i) : fill;
        if (out_index) out_index[e] = (i >= 0) ? (int32_t)(i - offsets[e]) : -1;
    }
    return HEPKREF_OK;
}

int hepkref_set_in_offsets(const int64_t *offsets, int64_t n_events, void *content, int32_t dtype,
                           const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                           float value)
{
    if (n_events < 0 || !offsets) return HEPKREF_EINVAL;
    if (dtype != HEPKREF_F32 && dtype != HEPKREF_U8) return HEPKREF_EINVAL;
    if (!content && n_events > 0 && offsets[n_events] > 0) return HEPKREF_EINVAL;
    for (int64_t e = 0; e < n_events; e++) {
        if (evt_mask && !evt_mask[e]) continue;
        int64_t i = nth_selected(offsets, e, obj_mask, idx ? idx[e] : n);
        if (i < 0) continue;
        if (dtype == HEPKREF_F32)
            ((float *)content)[i] = value;
        else
            ((uint8_t *)content)[i] = (value != 0.0f) ? 1 : 0;
    }
    return HEPKREF_OK;
}

/* i comes before j in pT order: larger pt first, NaN pt after every number,
 * equal (or both NaN) pt by lower index */
static int pt_before(float pi, int64_t i, float pj, int64_t j)
{
    int ni = pi != pi, nj = pj != pj;
    if (ni != nj) return nj;
    if (!ni && pi != pj) return pi > pj;
    return i < j;
}

static int opposite(int32_t a, int32_t b)
{
    return (a > 0 && b < 0) || (a < 0 && b > 0);
}

int hepkref_select_opposite_sign(const int64_t *offsets, int64_t n_events, const void *pt, int32_t dtype,
                                 const int32_t *charge, const uint8_t *obj_mask, uint8_t *mask_out)
{
    if (n_events < 0 || !offsets) return HEPKREF_EINVAL;
    if (!valid_float_dtype(dtype)) return HEPKREF_EINVAL;
    int64_t m = n_events > 0 ? offsets[n_events] : 0;
    if (m > 0 && (!pt || !charge || !mask_out)) return HEPKREF_EINVAL;
    for (int64_t e = 0; e < n_events; e++) {
        int64_t i0 = offsets[e], i1 = offsets[e + 1];
        for (int64_t i = i0; i < i1; i++) mask_out[i] = 0;
        /* the selected objects in pT order (selection sort on the definition) */
        int64_t cnt = 0;
        for (int64_t i = i0; i < i1; i++)
            if (!obj_mask || obj_mask[i]) cnt++;
        int64_t *order = xmalloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
        uint8_t *taken = xmalloc((size_t)(i1 - i0 > 0 ? i1 - i0 : 1));
        memset(taken, 0, (size_t)(i1 - i0 > 0 ? i1 - i0 : 1));
        for (int64_t p = 0; p < cnt; p++) {
            int64_t best = -1;
            for (int64_t i = i0; i < i1; i++) {
                if ((obj_mask && !obj_mask[i]) || taken[i - i0]) continue;
                if (best < 0 || pt_before(load_f(pt, dtype, i), i, load_f(pt, dtype, best), best)) best = i;
            }
            order[p] = best;
            taken[best - i0] = 1;
        }
        /* the first pair of positions (p, r), p < r, with opposite charges */
        int found = 0;
        for (int64_t p = 0; p < cnt && !found; p++)
            for (int64_t r = p + 1; r < cnt && !found; r++)
                if (opposite(charge[order[p]], charge[order[r]])) {
                    mask_out[order[p]] = 1;
                    mask_out[order[r]] = 1;
                    found = 1;
                }
        free(order);
        free(taken);
    }
    return HEPKREF_OK;
}

static size_t dtype_size(int32_t dtype)
{
    return dtype == HEPKREF_F16 ? 2 : (dtype == HEPKREF_U8 ? 1 : 4);
}

int hepkref_compact(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                    const uint8_t *obj_mask, void *out, int64_t *n_out)
{
    if (n_events < 0 || !offsets || !n_out) return HEPKREF_EINVAL;
    if (dtype < HEPKREF_F32 || dtype > HEPKREF_U8) return HEPKREF_EINVAL;
    size_t es = dtype_size(dtype);
    int64_t k = 0;
    for (int64_t e = 0; e < n_events; e++) {
        for (int64_t i = offsets[e]; i < offsets[e + 1]; i++) {
            if (obj_mask && !obj_mask[i]) continue;
            memcpy((char *)out + (size_t)k * es, (const char *)content + (size_t)i * es, es);
            k++;
        }
    }
    *n_out = k;
    return HEPKREF_OK;
}

/* ---- top-quark candidate (Sec. IV high-level variable reconstruction: the
 * jet triplet whose invariant mass is closest to M = 172 GeV) ---- */

int hepkref_p4(const void *pt, const void *eta, const void *phi, const void *mass, int32_t dtype, int64_t n,
               float *px, float *py, float *pz, float *en)
{
    if (n < 0 || (n > 0 && (!pt || !eta || !phi || !mass || !px || !py || !pz || !en))) return HEPKREF_EINVAL;
    if (!valid_float_dtype(dtype)) return HEPKREF_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        double p = load_f(pt, dtype, i), h = load_f(eta, dtype, i);
        double f = load_f(phi, dtype, i), m = load_f(mass, dtype, i);
        double x = p * cos(f), y = p * sin(f), z = p * sinh(h);
        px[i] = (float)x;
        py[i] = (float)y;
        pz[i] = (float)z;
        en[i] = (float)sqrt(x * x + y * y + z * z + m * m);
    }
    return HEPKREF_OK;
}

int hepkref_best_triplet(const int64_t *offsets, int64_t n_events, const float *px, const float *py,
                         const float *pz, const float *en, const uint8_t *obj_mask, float target,
                         float *out_mass, int32_t *out_idx)
{
    if (n_events < 0 || !offsets || (n_events > 0 && (!out_mass || !out_idx))) return HEPKREF_EINVAL;
    int64_t m = n_events > 0 ? offsets[n_events] : 0;
    if (m > 0 && (!px || !py || !pz || !en)) return HEPKREF_EINVAL;
    for (int64_t e = 0; e < n_events; e++) {
        int64_t i0 = offsets[e], i1 = offsets[e + 1];
        float best_d = INFINITY, best_m = NAN;
        int32_t bi = -1, bj = -1, bk = -1;
        for (int64_t i = i0; i < i1; i++) {
            if (obj_mask && !obj_mask[i]) continue;
            for (int64_t j = i + 1; j < i1; j++) {
                if (obj_mask && !obj_mask[j]) continue;
                for (int64_t k = j + 1; k < i1; k++) {
                    if (obj_mask && !obj_mask[k]) continue;
                    /* summed four-momentum, i + j first, then k */
                    float sx = (px[i] + px[j]) + px[k];
                    float sy = (py[i] + py[j]) + py[k];
                    float sz = (pz[i] + pz[j]) + pz[k];
                    float se = (en[i] + en[j]) + en[k];
                    float m2 = se * se;
                    m2 = m2 - sx * sx;
                    m2 = m2 - sy * sy;
                    m2 = m2 - sz * sz;
                    /* a negative square (rounding of a light system) is mass 0; NaN stays NaN */
                    float mm = (m2 < 0.0f) ? 0.0f : sqrtf(m2);
                    float d = fabsf(mm - target);
                    if (d < best_d) {
                        best_d = d;
                        best_m = mm;
                        bi = (int32_t)(i - i0);
                        bj = (int32_t)(j - i0);
                        bk = (int32_t)(k - i0);
                    }
                }
            }
        }
        out_mass[e] = best_m;
        out_idx[3 * e] = bi;
        out_idx[3 * e + 1] = bj;
        out_idx[3 * e + 2] = bk;
    }
    return HEPKREF_OK;
}

static hepkref_cut mkcut(const void *col, int32_t dtype, int32_t op, float thr)
{
    hepkref_cut c;
    c.col = col;
    c.dtype = dtype;
    c.op = op;
    c.thr = thr;
    c.ithr = 0;
    return c;
}

static hepkref_cut mkicut(const void *col, int32_t op, int32_t ithr)
{
    hepkref_cut c;
    c.col = col;
    c.dtype = HEPKREF_I32;
    c.op = op;
    c.thr = 0.0f;
    c.ithr = ithr;
    return c;
}

int hepkref_pipeline(const hepkref_dataset *ds, const hepkref_query *qs, int32_t n_query,
                     double *const *sumw, double *const *sumw2, uint64_t *const *counts)
{
    if (!ds || !qs || n_query < 0 || !sumw || !counts) return HEPKREF_EINVAL;
    if (!valid_float_dtype(ds->dtype) || ds->n_events < 0) return HEPKREF_EINVAL;
    const int64_t N = ds->n_events;
    const int32_t dt = ds->dtype;
    const int has_el = ds->electrons.off != NULL;
    const int has_btag = ds->jets.extra != NULL;
    const int64_t Mj = ds->jets.off[N], Mm = ds->muons.off[N];
    const int64_t Me = has_el ? ds->electrons.off[N] : 0;

    uint8_t *msel = xmalloc((size_t)Mm), *esel = xmalloc((size_t)Me);
    uint8_t *clean = xmalloc((size_t)Mj), *clean_e = xmalloc((size_t)Mj);
    uint8_t *jsel = xmalloc((size_t)Mj), *bsel = xmalloc((size_t)Mj);
    float *ptv = xmalloc(sizeof(float) * (size_t)Mj);
    float *delta = xmalloc(sizeof(float) * (size_t)Mj);
    float *mu_sf = xmalloc(sizeof(float) * (size_t)Mm);
    float *wev = xmalloc(sizeof(float) * (size_t)N), *evf = xmalloc(sizeof(float) * (size_t)N);
    int32_t *n_mu = xmalloc(sizeof(int32_t) * (size_t)N);
    int32_t *n_jet = xmalloc(sizeof(int32_t) * (size_t)N);
    int32_t *n_b = xmalloc(sizeof(int32_t) * (size_t)N);
    float *ht = xmalloc(sizeof(float) * (size_t)N);
    float *lead = xmalloc(sizeof(float) * (size_t)N);
    uint8_t *pass = xmalloc((size_t)N);

    int32_t k = 0;
    for (int32_t iq = 0; iq < n_query; iq++) {
        const hepkref_query *q = &qs[iq];
        /* muon selection: pt, |eta|, isolation */
        hepkref_cut mc[3];
        int nmc = 0;
        mc[nmc++] = mkcut(ds->muons.pt, dt, HEPKREF_GT, q->mu_pt);
        mc[nmc++] = mkcut(ds->muons.eta, dt, HEPKREF_ABS_LT, q->mu_abseta);
        if (ds->muons.extra) mc[nmc++] = mkcut(ds->muons.extra, dt, HEPKREF_LT, q->mu_iso);
        hepkref_select(mc, nmc, Mm, NULL, msel);
        hepkref_reduce(HEPKREF_COUNT, ds->muons.off, N, NULL, dt, msel, NULL, n_mu, NULL, NULL);

        /* jets cleaned against selected muons (and selected electrons) */
        hepkref_match_dr(ds->jets.off, ds->jets.eta, ds->jets.phi, NULL,
                         ds->muons.off, ds->muons.eta, ds->muons.phi, msel,
                         dt, N, q->dr, NULL, NULL, clean);
        if (has_el) {
            hepkref_cut ec[2];
            ec[0] = mkcut(ds->electrons.pt, dt, HEPKREF_GT, q->el_pt);
            ec[1] = mkcut(ds->electrons.eta, dt, HEPKREF_ABS_LT, q->el_abseta);
            hepkref_select(ec, 2, Me, NULL, esel);
            hepkref_match_dr(ds->jets.off, ds->jets.eta, ds->jets.phi, clean,
                             ds->electrons.off, ds->electrons.eta, ds->electrons.phi, esel,
                             dt, N, q->dr, NULL, NULL, clean_e);
            memcpy(clean, clean_e, (size_t)Mj);
        }

        /* event weights: w, times the pileup lookup, times the product of
         * the selected muons' scale factors (Sec. IV: event weights from
         * histogram lookups), each product rounded to float32 */
        for (int64_t e = 0; e < N; e++) wev[e] = ds->weights[e];
        if (q->pu_edges && ds->npu) {
            hepkref_get_bin_contents(ds->npu, HEPKREF_F32, N, q->pu_edges, q->pu_nbins, q->pu_contents, evf);
            for (int64_t e = 0; e < N; e++) wev[e] = wev[e] * evf[e];
        }
        if (q->sf_edges) {
            hepkref_get_bin_contents(ds->muons.pt, dt, Mm, q->sf_edges, q->sf_nbins, q->sf_contents, mu_sf);
            hepkref_reduce(HEPKREF_PROD, ds->muons.off, N, mu_sf, HEPKREF_F32, msel, NULL, evf, NULL, NULL);
            for (int64_t e = 0; e < N; e++) wev[e] = wev[e] * evf[e];
        }
        /* jet energy scale from a lookup: the shift per jet, once per query */
        if (q->jes_mode == 1)
            hepkref_jes_delta(ds->jets.pt, ds->jets.eta, dt, Mj, q->jes_eta_edges, q->jes_n_eta,
                              q->jes_pt_edges, q->jes_n_pt, q->jes_delta, delta);

        for (int32_t v = 0; v < q->n_scale; v++) {
            /* jet energy scale applied to pt (one float32 product; with a
             * lookup, the factor 1 + s * delta rounded first) */
            const float s = q->scales[v];
            if (q->jes_mode == 1)
                for (int64_t j = 0; j < Mj; j++) ptv[j] = load_f(ds->jets.pt, dt, j) * (1.0f + s * delta[j]);
            else
                for (int64_t j = 0; j < Mj; j++) ptv[j] = load_f(ds->jets.pt, dt, j) * s;
            hepkref_cut jc[2];
            jc[0] = mkcut(ptv, HEPKREF_F32, HEPKREF_GT, q->jet_pt);
            jc[1] = mkcut(ds->jets.eta, dt, HEPKREF_ABS_LT, q->jet_abseta);
            hepkref_select(jc, 2, Mj, clean, jsel);

            hepkref_reduce(HEPKREF_COUNT, ds->jets.off, N, NULL, dt, jsel, NULL, n_jet, NULL, NULL);
            hepkref_reduce(HEPKREF_SUM, ds->jets.off, N, ptv, HEPKREF_F32, jsel, NULL, ht, NULL, NULL);
            hepkref_reduce(HEPKREF_MAX, ds->jets.off, N, ptv, HEPKREF_F32, jsel, NULL, lead, NULL, NULL);

            hepkref_cut ev[3];
            int nev = 0;
            ev[nev++] = mkicut(n_mu, HEPKREF_GE, q->min_mu);
            ev[nev++] = mkicut(n_jet, HEPKREF_GE, q->min_jet);
            if (has_btag) {
                hepkref_cut bc = mkcut(ds->jets.extra, dt, HEPKREF_GT, q->btag);
                hepkref_select(&bc, 1, Mj, jsel, bsel);
                hepkref_reduce(HEPKREF_COUNT, ds->jets.off, N, NULL, dt, bsel, NULL, n_b, NULL, NULL);
                ev[nev++] = mkicut(n_b, HEPKREF_GE, q->min_b);
            }
            hepkref_select(ev, nev, N, NULL, pass);

            hepkref_hist_fill_w2(ht, HEPKREF_F32, wev, pass, N, q->edges[0], q->nbins[0],
                                 sumw[k], sumw2 ? sumw2[k] : NULL, counts[k]);
            k++;
            hepkref_hist_fill_w2(lead, HEPKREF_F32, wev, pass, N, q->edges[1], q->nbins[1],
                                 sumw[k], sumw2 ? sumw2[k] : NULL, counts[k]);
            k++;
            hepkref_hist_fill_w2(n_jet, HEPKREF_I32, wev, pass, N, q->edges[2], q->nbins[2],
                                 sumw[k], sumw2 ? sumw2[k] : NULL, counts[k]);
            k++;
        }
    }
    free(msel); free(esel); free(clean); free(clean_e); free(jsel); free(bsel); free(ptv);
    free(delta); free(mu_sf); free(wev); free(evf);
    free(n_mu); free(n_jet); free(n_b); free(ht); free(lead); free(pass);
    return HEPKREF_OK;
}
