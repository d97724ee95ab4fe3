// Lookup histograms (Sec. III get_bin_contents: the content of the bin of a
// lookup histogram that holds each element, used for histogram-based
// reweighting; Sec. IV: event weights and jet energy corrections from
// histogram lookups, systematic corrections by linear interpolation).
//
// A lookup histogram has the slot layout of a filled one: edges
// E[0] < ... < E[nbins], content c[0] for x < E[0], c[s] for
// E[s-1] <= x < E[s], c[nbins+1] for x >= E[nbins].
//
// Interpolation runs between bin centres m_s = (E[s-1] + E[s]) * 0.5 (float32,
// s = 1..nbins): x <= m_1 gives c[1], x >= m_nbins gives c[nbins], otherwise,
// with i the number of centres at or below x (m_i <= x < m_{i+1}),
// c[i] + (x - m_i) * slope_i, slope_i = (c[i+1] - c[i]) / (m_{i+1} - m_i),
// every operation one float32 rounding (division correctly rounded).
//
// The interval of x among the centres follows from its bin: a centre lies
// between its bin's edges (the rounded midpoint of two float32 values stays
// between them), so with x in bin s, every centre below s is <= E[s-1] <= x
// and every centre above s is >= E[s] > x; the count is s - 1 plus one when
// m_s <= x.  (Edges whose neighbour sums overflow float32 are outside this
// and are not supported.)
#pragma once

#include "common.hpp"

namespace hepk {

__host__ __device__ inline float bin_centre(float lo_edge, float hi_edge) { return (lo_edge + hi_edge) * 0.5f; }

// Start value of the bin search (nbins / (hi - lo), 0 when not finite).
__host__ __device__ inline float bin_inv_width(float lo, float hi, int nbins) {
    const float span = hi - lo;
    return (span > 0.0f && span < INFINITY) ? static_cast<float>(nbins) / span : 0.0f;
}

// One lookup table as the kernels read it: nb bins with edges E[0..nb] and
// lo = E[0], hi = E[nb], iw = bin_inv_width(lo, hi, nb).
struct Axis {
    const float *E;
    int nb;
    float lo, hi, iw;
};

// Content of the slot holding x (C: nb + 2 slot contents); NaN x gives the
// quiet NaN 0x7fc00000.
__device__ __forceinline__ float lookup_bin(const Axis &a, const float *C, float x) {
    if (x != x) return __builtin_nanf("");
    return C[hist_slot_lohi(x, a.E, a.nb, a.lo, a.hi, a.iw)];
}

// Interpolation between bin centres of the values V[0..nb) (V[k] is bin
// k+1's value); NaN x gives the quiet NaN 0x7fc00000.
__device__ __forceinline__ float lookup_interp(const Axis &a, const float *V, float x) {
    if (x != x) return __builtin_nanf("");
    const int nb = a.nb;
    if (x <= bin_centre(a.E[0], a.E[1])) return V[0];
    if (x >= bin_centre(a.E[nb - 1], a.E[nb])) return V[nb - 1];
    // m_1 < x < m_nb, so E[0] <= m_1 < x < m_nb <= E[nb]: x lies in bin s
    const int s = hist_slot_lohi(x, a.E, nb, a.lo, a.hi, a.iw);  // 1..nb
    const int i = (bin_centre(a.E[s - 1], a.E[s]) <= x) ? s : s - 1;  // centre interval, 1..nb-1
    const float m0 = bin_centre(a.E[i - 1], a.E[i]);
    const float m1 = bin_centre(a.E[i], a.E[i + 1]);
    const float v0 = V[i - 1], v1 = V[i];
    const float slope = (v1 - v0) / (m1 - m0);
    const float d = x - m0;
    const float p = d * slope;
    return v0 + p;
}

// Row of a two-dimensional table for |eta|: the bin of ae among the rows'
// edges, the nearest row outside them, the first row for NaN (1-based).
__device__ __forceinline__ int lookup_row(const Axis &rows, float ae) {
    if (ae != ae) return 1;
    const int s = hist_slot_lohi(ae, rows.E, rows.nb, rows.lo, rows.hi, rows.iw);
    return s < 1 ? 1 : (s > rows.nb ? rows.nb : s);
}

// Slots of N values at once: pos[n] becomes the number of edges at or below
// x[n] (0 for NaN), the slot hist_slot_lohi finds.  With guess (a table
// whose edges are close to uniform), first the uniform-bin guess of every
// value, checked against its two edges (one round of reads); without it, or
// if some value of the wavefront missed, a branch-free binary search in
// which every value takes the same fixed steps (the largest power of two not
// above nb + 1, halving), so the N reads of a step go out together -- one
// memory round trip per step instead of one dependent chain per value.
template <int N>
__device__ __forceinline__ void edge_count_n(const Axis &a, const float (&x)[N], int (&pos)[N], bool guess) {
    const int nb = a.nb;
    if (guess) {
    float el[N], eh[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const float g = (x[n] - a.lo) * a.iw;
        const int gi = g >= 0.0f ? (g < static_cast<float>(nb) ? static_cast<int>(g) + 1 : nb) : 1;
        pos[n] = !(x[n] >= a.lo) ? 0 : (x[n] >= a.hi ? nb + 1 : gi);
        const int k = min(max(pos[n], 1), nb);
        el[n] = a.E[k - 1];
        eh[n] = a.E[k];
    }
    bool miss = false;
#pragma unroll
    for (int n = 0; n < N; ++n) miss |= (pos[n] >= 1) & (pos[n] <= nb) & ((x[n] < el[n]) | (x[n] >= eh[n]));
    if (__ballot(miss) == 0) return;
    }
#pragma unroll
    for (int n = 0; n < N; ++n) pos[n] = 0;
    int top = 1;
    while (top * 2 <= nb + 1) top *= 2;
    for (int step = top; step > 0; step >>= 1) {
        float e[N];
#pragma unroll
        for (int n = 0; n < N; ++n) e[n] = a.E[min(pos[n] + step, nb + 1) - 1];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int t = pos[n] + step;
            pos[n] = (t <= nb + 1 && e[n] <= x[n]) ? t : pos[n];
        }
    }
}

// Whether the uniform-bin guess suits edges E[0..nb] (every edge within a
// quarter bin width of its uniform position), decided by the whole
// workgroup (every thread must call it; E readable by all).
__device__ __forceinline__ bool near_uniform(const float *E, int nb) {
    const float lo = E[0], hi = E[nb];
    const float w = (hi - lo) / static_cast<float>(nb);
    bool bad = !(w > 0.0f) || !(w < INFINITY);
    for (int i = threadIdx.x; i <= nb; i += blockDim.x)
        bad |= !(fabsf(E[i] - (lo + w * static_cast<float>(i))) <= 0.25f * w);
    return __syncthreads_or(bad) == 0;
}

// lookup_bin of N values at once (values with use[n] unset give 1).
template <int N>
__device__ __forceinline__ void lookup_bin_n(const Axis &a, const float *C, const float (&x)[N],
                                             const bool (&use)[N], float (&out)[N], bool guess) {
    int pos[N];
    edge_count_n<N>(a, x, pos, guess);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const float c = C[pos[n]];
        out[n] = use[n] ? ((x[n] != x[n]) ? __builtin_nanf("") : c) : 1.0f;
    }
}

// lookup_interp of N values at once given their slots pos[n] (edge counts)
// and value rows V[n]; every value the interpolation may need is read in
// one round (indices clamped into the table; outside m_1 < x < m_nb the
// result is replaced), the arithmetic exactly lookup_interp's.
template <int N>
__device__ __forceinline__ void interp_at_n(const Axis &c, const float *const (&V)[N], const float (&x)[N],
                                            const int (&pos)[N], float (&out)[N]) {
    const int nb = c.nb;
    const float mfirst = bin_centre(c.E[0], c.E[1]), mlast = bin_centre(c.E[nb - 1], c.E[nb]);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        // the interval is s - 1 or s
        const int s = min(max(pos[n], 1), nb);
        const float ea = c.E[max(s - 2, 0)], eb = c.E[s - 1], ec = c.E[s], ed = c.E[min(s + 1, nb)];
        const float va = V[n][max(s - 2, 0)], vb = V[n][s - 1], vc = V[n][min(s, nb - 1)];
        const float v_first = V[n][0], v_last = V[n][nb - 1];
        const float ms = bin_centre(eb, ec);
        const bool at_s = ms <= x[n];
        const float m0 = at_s ? ms : bin_centre(ea, eb);
        const float m1 = at_s ? bin_centre(ec, ed) : ms;
        const float v0 = at_s ? vb : va, v1 = at_s ? vc : vb;
        const float slope = (v1 - v0) / (m1 - m0);
        const float d = x[n] - m0;
        const float p = d * slope;
        const float r = v0 + p;
        out[n] = (x[n] != x[n]) ? __builtin_nanf("")
                                : (x[n] <= mfirst ? v_first : (x[n] >= mlast ? v_last : r));
    }
}

// lookup_interp of N values at once (values V[0..nb)).
template <int N>
__device__ __forceinline__ void lookup_interp_n(const Axis &c, const float *V, const float (&x)[N], float (&out)[N],
                                                bool guess) {
    int pos[N];
    edge_count_n<N>(c, x, pos, guess);
    const float *Vs[N];
#pragma unroll
    for (int n = 0; n < N; ++n) Vs[n] = V;
    interp_at_n<N>(c, Vs, x, pos, out);
}

// Interpolation in x over the row of a two-dimensional table (rows of cols.nb
// values from D, one per bin of |y| among the row edges; the row as in
// lookup_row: the count clamped to the rows, the first for NaN) for N values
// at once, the row and column searches interleaved.
template <int N>
__device__ __forceinline__ void lookup2_n(const Axis &rows, const Axis &cols, const float *D, const float (&x)[N],
                                          const float (&y)[N], float (&out)[N]) {
    const int nb = cols.nb, nr = rows.nb;
    int rpos[N], pos[N];
    float ay[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        ay[n] = fabsf(y[n]);
        rpos[n] = 0;
        pos[n] = 0;
    }
    int top = 1, rtop = 1;
    while (top * 2 <= nb + 1) top *= 2;
    while (rtop * 2 <= nr + 1) rtop *= 2;
    for (int step = top, rstep = rtop; step > 0 || rstep > 0; step >>= 1, rstep >>= 1) {
        float e[N], re[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            if (step > 0) e[n] = cols.E[min(pos[n] + step, nb + 1) - 1];
            if (rstep > 0) re[n] = rows.E[min(rpos[n] + rstep, nr + 1) - 1];
        }
#pragma unroll
        for (int n = 0; n < N; ++n) {
            if (step > 0) {
                const int t = pos[n] + step;
                pos[n] = (t <= nb + 1 && e[n] <= x[n]) ? t : pos[n];
            }
            if (rstep > 0) {
                const int t = rpos[n] + rstep;
                rpos[n] = (t <= nr + 1 && re[n] <= ay[n]) ? t : rpos[n];
            }
        }
    }
    const float *V[N];
#pragma unroll
    for (int n = 0; n < N; ++n) V[n] = D + static_cast<int64_t>(min(max(rpos[n], 1), nr) - 1) * nb;
    interp_at_n<N>(cols, V, x, pos, out);
}

}  // namespace hepk
