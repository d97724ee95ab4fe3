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

}  // namespace hepk
