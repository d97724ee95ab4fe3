// hepk_hist_fill: weighted 1-D histogram fill (Sec. III fill-histogram
// kernel), accumulating into the caller's histogram.
//
// Each workgroup (1024 threads, one per CU) keeps a private copy of the
// histogram in LDS (float64 sums via ds_add_f64, uint32 counts via
// ds_add_u32) together with the bin edges, walks a grid-stride range of rows
// eight at a time per thread (loads of the eight rows in flight together,
// then their eight bins found together),
// and merges its non-empty slots into HBM with global atomics at the end
// (few workgroups: few atomics on each slot); with hepk_hist_fill_w2 also the
// float64 sums of squared weights.  Histograms too large for LDS
// go straight to global atomics with the edges read from HBM.  Sums of float64 weights are exact in
// any order while every partial sum is a multiple of the smallest weight's ulp
// below 2^53 of it, which holds for the float32 weights of this analysis;
// otherwise the order changes only the last bits.
#include "common.hpp"

namespace hepk {

constexpr int HB = 1024;
constexpr int HR = 8;  // rows per thread in flight
// One workgroup per CU: a sweep of 1-4 per CU and 4-16 rows per thread in
// flight put the best at one and 8 (two workgroups: 5% slower).
constexpr int kHistWgPerCu = 1;
constexpr int kMaxLdsSlots = 3000;    // 36 KiB of histogram + 12 KiB of edges
constexpr int kMaxLdsSlotsW2 = 2400;  // with the squared weights: 48 KiB + 9.6 KiB

// hist_slot_lohi for N values at once: every guess first, then every edge
// pair read (all reads in flight together), then the checks, with a binary
// search only where a guess was off.  NaN x gets slot 0 (callers skip it).
template <int N>
__device__ __forceinline__ void hist_slots_lohi(const float (&x)[N], const float *E, int nbins, float lo, float hi,
                                                float inv_w, int (&s)[N]) {
    int k[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const float g = (x[n] - lo) * inv_w;
        const int gi = (g >= 0.0f) ? ((g < static_cast<float>(nbins)) ? static_cast<int>(g) + 1 : nbins) : 1;
        s[n] = !(x[n] >= lo) ? 0 : (x[n] >= hi ? nbins + 1 : gi);
        k[n] = (s[n] >= 1 && s[n] <= nbins) ? s[n] : 1;
    }
    float a[N], b[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        a[n] = E[k[n] - 1];
        b[n] = E[k[n]];
    }
#pragma unroll
    for (int n = 0; n < N; ++n)
        if (s[n] >= 1 && s[n] <= nbins && (x[n] < a[n] || x[n] >= b[n])) s[n] = bin_search(E, nbins, x[n]);
}

template <typename X, bool LDS, bool W2>
__global__ __launch_bounds__(HB) void hist_kernel(const X *__restrict__ x, const float *__restrict__ w,
                                                  const uint8_t *__restrict__ m, int64_t n,
                                                  const float *__restrict__ edges, int nbins,
                                                  double *__restrict__ sumw, double *__restrict__ sumw2,
                                                  uint64_t *__restrict__ counts) {
    extern __shared__ double hist_lds[];
    const int nslots = nbins + 2;
    double *sw_s = hist_lds;
    double *sw2_s = hist_lds + (LDS ? nslots : 0);
    uint32_t *c_s = reinterpret_cast<uint32_t *>(sw2_s + ((LDS && W2) ? nslots : 0));
    float *e_s = reinterpret_cast<float *>(c_s + (LDS ? nslots : 0));
    // end edges and the bin-guess start values (the guess is verified against the edges)
    const float lo = as_const(edges)[0];
    const float hi = as_const(edges)[nbins];
    const float span = hi - lo;
    const float inv_w = (span > 0.0f && span < INFINITY) ? static_cast<float>(nbins) / span : 0.0f;
    if (LDS) {
        for (int i = threadIdx.x; i < nslots; i += HB) {
            sw_s[i] = 0.0;
            if (W2) sw2_s[i] = 0.0;
            c_s[i] = 0u;
        }
        for (int i = threadIdx.x; i <= nbins; i += HB) e_s[i] = edges[i];
        __syncthreads();
    }
    auto add = [&](int s, double wt) {
        if (LDS) {
            atomic_add_f64(&sw_s[s], wt);
            if (W2) atomic_add_f64(&sw2_s[s], wt * wt);
            atomicAdd(&c_s[s], 1u);
        } else {
            atomic_add_f64(&sumw[s], wt);
            if (W2) atomic_add_f64(&sumw2[s], wt * wt);
            atomic_add_u64(&counts[s], 1u);
        }
    };
    const int64_t stride = static_cast<int64_t>(gridDim.x) * HB;
    int64_t i = static_cast<int64_t>(blockIdx.x) * HB + threadIdx.x;
    // HR rows per step (the last step predicated), loads first
    for (; i < n; i += HR * stride) {
        float v[HR];
        float wt[HR];
        bool keep[HR];
#pragma unroll
        for (int u = 0; u < HR; ++u) {
            const int64_t r = i + u * stride;
            keep[u] = false;
            v[u] = 0.0f;
            wt[u] = 1.0f;
            if (r < n) {
                keep[u] = !m || m[r] != 0;
                v[u] = static_cast<float>(x[r]);
                if (w) wt[u] = w[r];
            }
        }
        // all HR bins found together (one round of edge reads)
        int sl[HR];
        hist_slots_lohi<HR>(v, LDS ? e_s : edges, nbins, lo, hi, inv_w, sl);
#pragma unroll
        for (int u = 0; u < HR; ++u)
            if (keep[u] && v[u] == v[u]) add(sl[u], static_cast<double>(wt[u]));
    }
    if (LDS) {
        __syncthreads();
        for (int k = threadIdx.x; k < nslots; k += HB) {
            const uint32_t c = c_s[k];
            if (c) {
                atomic_add_u64(&counts[k], c);
                atomic_add_f64(&sumw[k], sw_s[k]);
                if (W2) atomic_add_f64(&sumw2[k], sw2_s[k]);
            }
        }
    }
}

// Four consecutive values of x as float (one 16- or 8-byte load).
typedef float hf32x4 __attribute__((ext_vector_type(4)));
typedef int hi32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int hu32x2 __attribute__((ext_vector_type(2)));
// Nontemporal loads: every row is read once (3-5% faster than plain loads).
template <typename V>
__device__ __forceinline__ V ldv(const V *p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ void load4(const float *p, float (&o)[4]) {
    const hf32x4 v = ldv(reinterpret_cast<const hf32x4 *>(p));
    o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
__device__ __forceinline__ void load4(const int32_t *p, float (&o)[4]) {
    const hi32x4 v = ldv(reinterpret_cast<const hi32x4 *>(p));
    o[0] = static_cast<float>(v.x), o[1] = static_cast<float>(v.y);
    o[2] = static_cast<float>(v.z), o[3] = static_cast<float>(v.w);
}
__device__ __forceinline__ void load4(const _Float16 *p, float (&o)[4]) {
    const hu32x2 v = ldv(reinterpret_cast<const hu32x2 *>(p));
    const uint32_t u[2] = {v.x, v.y};
#pragma unroll
    for (int j = 0; j < 4; ++j)
        o[j] = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(u[j >> 1] >> (16 * (j & 1)))));
}

// The same fill with rows taken four at a time (rows 4q..4q+3 of quad q):
// x, w and the mask read with one 16-, 16- and 4-byte load per quad, two
// quads per thread per step.  Needs x, w aligned to their 4-row size and the
// mask to 4 bytes.  The last quad may run past n: its loads stay inside the
// aligned 4-row block that holds row 4q (so inside the buffer's pages), and
// rows >= n are not filled.
template <typename X, bool LDS, bool W2>
__global__ __launch_bounds__(HB) void hist_vec_kernel(const X *__restrict__ x, const float *__restrict__ w,
                                                      const uint8_t *__restrict__ m, int64_t n,
                                                      const float *__restrict__ edges, int nbins,
                                                      double *__restrict__ sumw, double *__restrict__ sumw2,
                                                      uint64_t *__restrict__ counts) {
    extern __shared__ double hist_lds[];
    const int nslots = nbins + 2;
    double *sw_s = hist_lds;
    double *sw2_s = hist_lds + (LDS ? nslots : 0);
    uint32_t *c_s = reinterpret_cast<uint32_t *>(sw2_s + ((LDS && W2) ? nslots : 0));
    float *e_s = reinterpret_cast<float *>(c_s + (LDS ? nslots : 0));
    const float lo = as_const(edges)[0];
    const float hi = as_const(edges)[nbins];
    const float span = hi - lo;
    const float inv_w = (span > 0.0f && span < INFINITY) ? static_cast<float>(nbins) / span : 0.0f;
    if (LDS) {
        for (int i = threadIdx.x; i < nslots; i += HB) {
            sw_s[i] = 0.0;
            if (W2) sw2_s[i] = 0.0;
            c_s[i] = 0u;
        }
        for (int i = threadIdx.x; i <= nbins; i += HB) e_s[i] = edges[i];
        __syncthreads();
    }
    auto add = [&](int s, double wt) {
        if (LDS) {
            atomic_add_f64(&sw_s[s], wt);
            if (W2) atomic_add_f64(&sw2_s[s], wt * wt);
            atomicAdd(&c_s[s], 1u);
        } else {
            atomic_add_f64(&sumw[s], wt);
            if (W2) atomic_add_f64(&sumw2[s], wt * wt);
            atomic_add_u64(&counts[s], 1u);
        }
    };
    constexpr int HQ = HR / 4;  // quads per thread per step
    const int64_t nq = (n + 3) >> 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * HB;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * HB + threadIdx.x; q < nq; q += HQ * stride) {
        float v[HR], wt[HR];
        bool keep[HR];
#pragma unroll
        for (int h = 0; h < HQ; ++h) {
            const int64_t qq = q + h * stride;
            float xv[4] = {0.0f, 0.0f, 0.0f, 0.0f}, wv[4] = {1.0f, 1.0f, 1.0f, 1.0f};
            uint32_t mv = 0xffffffffu;
            const bool in = qq < nq;
            // quads past the end load the last quad again (kept out by
            // `in`), so no load sits under a per-lane branch
            const int64_t qc = in ? qq : nq - 1;
            load4(x + 4 * qc, xv);
            if (w) load4(w + 4 * qc, wv);
            if (m) mv = ldv(reinterpret_cast<const uint32_t *>(m + 4 * qc));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[4 * h + j] = xv[j];
                wt[4 * h + j] = wv[j];
                keep[4 * h + j] = in && 4 * qq + j < n && ((mv >> (8 * j)) & 0xffu) != 0;
            }
        }
        int sl[HR];
        hist_slots_lohi<HR>(v, LDS ? e_s : edges, nbins, lo, hi, inv_w, sl);
#pragma unroll
        for (int u = 0; u < HR; ++u)
            if (keep[u] && v[u] == v[u]) add(sl[u], static_cast<double>(wt[u]));
    }
    if (LDS) {
        __syncthreads();
        for (int k = threadIdx.x; k < nslots; k += HB) {
            const uint32_t c = c_s[k];
            if (c) {
                atomic_add_u64(&counts[k], c);
                atomic_add_f64(&sumw[k], sw_s[k]);
                if (W2) atomic_add_f64(&sumw2[k], sw2_s[k]);
            }
        }
    }
}

template <typename X, bool W2>
static int launch_hist(const void *x, const float *w, const uint8_t *m, int64_t n, const hepk_hist *h,
                       double *sumw2, hipStream_t stream) {
    const int nslots = h->nbins + 2;
    const bool lds = nslots <= (W2 ? kMaxLdsSlotsW2 : kMaxLdsSlots);
    const int grid = static_cast<int>(std::min<int64_t>(ceil_div(n, HB * HR), kHistWgPerCu * device_cus()));
    const size_t lds_bytes = static_cast<size_t>(nslots) * ((W2 ? 2 : 1) * sizeof(double) + sizeof(uint32_t)) +
                             static_cast<size_t>(h->nbins + 1) * sizeof(float);
    auto aligned = [](const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
    const X *xp = static_cast<const X *>(x);
    if (aligned(x, 4 * sizeof(X)) && (!w || aligned(w, 16)) && (!m || aligned(m, 4))) {
        if (lds)
            hist_vec_kernel<X, true, W2><<<grid, HB, lds_bytes, stream>>>(xp, w, m, n, h->edges, h->nbins, h->sumw,
                                                                          sumw2, h->counts);
        else
            hist_vec_kernel<X, false, W2><<<grid, HB, 0, stream>>>(xp, w, m, n, h->edges, h->nbins, h->sumw, sumw2,
                                                                   h->counts);
        return check_launch("hepk_hist_fill");
    }
    if (lds)
        hist_kernel<X, true, W2><<<grid, HB, lds_bytes, stream>>>(xp, w, m, n, h->edges, h->nbins, h->sumw, sumw2,
                                                                  h->counts);
    else
        hist_kernel<X, false, W2><<<grid, HB, 0, stream>>>(xp, w, m, n, h->edges, h->nbins, h->sumw, sumw2,
                                                           h->counts);
    return check_launch("hepk_hist_fill");
}

static int hist_fill(const void *x, int32_t dtype, const float *w, const uint8_t *evt_mask, int64_t n,
                     const hepk_hist *h, double *sumw2, hipStream_t stream) {
    HEPK_REQUIRE(h, "hepk_hist_fill: hist is NULL");
    HEPK_REQUIRE(n >= 0, "hepk_hist_fill: n < 0");
    HEPK_REQUIRE(h->nbins >= 1, "hepk_hist_fill: nbins %d < 1", h->nbins);
    HEPK_REQUIRE(h->edges && h->sumw && h->counts, "hepk_hist_fill: histogram array is NULL");
    HEPK_REQUIRE(n == 0 || x, "hepk_hist_fill: x is NULL");
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16 || dtype == HEPK_I32, "hepk_hist_fill: bad dtype %d",
                 dtype);
    if (n == 0) return HEPK_OK;
    if (sumw2) {
        if (dtype == HEPK_F16) return launch_hist<_Float16, true>(x, w, evt_mask, n, h, sumw2, stream);
        if (dtype == HEPK_I32) return launch_hist<int32_t, true>(x, w, evt_mask, n, h, sumw2, stream);
        return launch_hist<float, true>(x, w, evt_mask, n, h, sumw2, stream);
    }
    if (dtype == HEPK_F16) return launch_hist<_Float16, false>(x, w, evt_mask, n, h, nullptr, stream);
    if (dtype == HEPK_I32) return launch_hist<int32_t, false>(x, w, evt_mask, n, h, nullptr, stream);
    return launch_hist<float, false>(x, w, evt_mask, n, h, nullptr, stream);
}

}  // namespace hepk

extern "C" int hepk_hist_fill(const void *x, int32_t dtype, const float *w, const uint8_t *evt_mask, int64_t n,
                              const hepk_hist *h, hipStream_t stream) {
    hepk::clear_error();
    return hepk::hist_fill(x, dtype, w, evt_mask, n, h, nullptr, stream);
}

extern "C" int hepk_hist_fill_w2(const void *x, int32_t dtype, const float *w, const uint8_t *evt_mask, int64_t n,
                                 const hepk_hist *h, double *sumw2, hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(sumw2, "hepk_hist_fill_w2: sumw2 is NULL");
    return hepk::hist_fill(x, dtype, w, evt_mask, n, h, sumw2, stream);
}
