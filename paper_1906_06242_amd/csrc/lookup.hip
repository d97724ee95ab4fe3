// hepk_get_bin_contents, hepk_interp, hepk_jes_delta: per-element lookups
// in lookup histograms (Sec. III get_bin_contents; Sec. IV event weights and
// jet energy corrections from histogram lookups, corrections by linear
// interpolation).  The lookup arithmetic is in lookup.hpp.
//
// Elementwise and HBM-bound (4 or 2 bytes read per input column and 4
// written per element): each thread takes four consecutive elements, read
// with one 16-byte (float32, int32) or 8-byte (float16) load per column when
// the arrays are aligned to that, and written with one 16-byte store.  Each
// workgroup first copies the tables into LDS when they fit (the bin search
// reads a few edges per element), else reads them from HBM through the cache.
// A thread's four lookups search in lockstep (the *_n forms in lookup.hpp):
// their reads of each search step go out together.
#include "lookup.hpp"

namespace hepk {

constexpr int LB = 256;
constexpr int kMaxLookupLdsFloats = 12 * 1024;  // 48 KiB

// Element columns are read and written once: nontemporal loads and stores
// (bin contents 76 -> 70 us, interpolation 157 -> 142 us on 5e7 rows).
typedef unsigned int lu32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int lu32x2 __attribute__((ext_vector_type(2)));
typedef float lf32x4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V ldnt(const V *p) {
    return __builtin_nontemporal_load(p);
}

template <typename X>
__device__ __forceinline__ float ld1(const X *p, int64_t i) {
    return static_cast<float>(p[i]);
}

// Elements 4g .. 4g+3 of p as float (those at or beyond n as 0): one vector
// load when all four are inside (VEC: p aligned to four elements).
template <typename X, bool VEC>
__device__ __forceinline__ void load_quad(const X *p, int64_t g, int64_t n, float (&o)[4]) {
    const int64_t i0 = 4 * g;
    if (VEC && i0 + 4 <= n) {
        if constexpr (sizeof(X) == 4) {
            const lu32x4 v = ldnt(reinterpret_cast<const lu32x4 *>(p + i0));
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = static_cast<float>(__builtin_bit_cast(X, w[j]));
        } else {
            const lu32x2 v = ldnt(reinterpret_cast<const lu32x2 *>(p + i0));
            const uint32_t w[2] = {v.x, v.y};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                o[j] = static_cast<float>(__builtin_bit_cast(X, static_cast<uint16_t>(w[j >> 1] >> (16 * (j & 1)))));
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (i0 + j < n) ? ld1(p, i0 + j) : 0.0f;
}

template <bool VEC>
__device__ __forceinline__ void store_quad(float *out, int64_t g, int64_t n, const float (&v)[4]) {
    const int64_t i0 = 4 * g;
    if (VEC && i0 + 4 <= n) {
        const lf32x4 o = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(o, reinterpret_cast<lf32x4 *>(out + i0));
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (i0 + j < n) out[i0 + j] = v[j];
}

// Copies n floats of src to LDS at dst (whole workgroup).
__device__ __forceinline__ void stage(float *dst, const float *src, int n) {
    for (int i = threadIdx.x; i < n; i += LB) dst[i] = src[i];
}

// MODE 0: out = slot content (get_bin_contents); MODE 1: interpolation
// between bin centres.  LDS: the edges and contents are copied to LDS first.
template <typename X, int MODE, bool LDS, bool VEC>
__global__ __launch_bounds__(LB) void lookup1_kernel(const X *__restrict__ x, int64_t n, const float *__restrict__ E,
                                                     int nb, const float *__restrict__ C, float *__restrict__ out) {
    extern __shared__ float lk_lds[];
    const float lo = as_const(E)[0], hi = as_const(E)[nb];
    const float *e = E, *c = C;
    if (LDS) {
        stage(lk_lds, E, nb + 1);
        stage(lk_lds + nb + 1, C, nb + 2);
        __syncthreads();
        e = lk_lds;
        c = lk_lds + nb + 1;
    }
    const Axis a{e, nb, lo, hi, bin_inv_width(lo, hi, nb)};
    // guess first for near-uniform edges (tested once per workgroup on the
    // LDS copy; tables left in HBM always guess first)
    const bool guess = LDS ? near_uniform(e, nb) : true;
    const int64_t ng = (n + 3) >> 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * LB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * LB + threadIdx.x; g < ng; g += stride) {
        float v[4], r[4];
        load_quad<X, VEC>(x, g, n, v);
        if (MODE == 0) {
            const bool use[4] = {true, true, true, true};
            lookup_bin_n<4>(a, c, v, use, r, guess);
        } else {
            lookup_interp_n<4>(a, c + 1, v, r, guess);
        }
        store_quad<VEC>(out, g, n, r);
    }
}

// out = interpolation in pt over the |eta| row of the table D (n_eta rows of
// n_pt values).
template <typename X, bool LDS, bool VEC>
__global__ __launch_bounds__(LB) void jes_delta_kernel(const X *__restrict__ pt, const X *__restrict__ eta, int64_t n,
                                                       const float *__restrict__ EE, int ne,
                                                       const float *__restrict__ PE, int np,
                                                       const float *__restrict__ D, float *__restrict__ out) {
    extern __shared__ float lk_lds[];
    const float elo = as_const(EE)[0], ehi = as_const(EE)[ne];
    const float plo = as_const(PE)[0], phi = as_const(PE)[np];
    const float *ee = EE, *pe = PE, *d = D;
    if (LDS) {
        stage(lk_lds, EE, ne + 1);
        stage(lk_lds + ne + 1, PE, np + 1);
        stage(lk_lds + ne + np + 2, D, ne * np);
        __syncthreads();
        ee = lk_lds;
        pe = lk_lds + ne + 1;
        d = lk_lds + ne + np + 2;
    }
    const Axis rows{ee, ne, elo, ehi, bin_inv_width(elo, ehi, ne)};
    const Axis cols{pe, np, plo, phi, bin_inv_width(plo, phi, np)};
    const int64_t ng = (n + 3) >> 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * LB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * LB + threadIdx.x; g < ng; g += stride) {
        float p[4], h[4], r[4];
        load_quad<X, VEC>(pt, g, n, p);
        load_quad<X, VEC>(eta, g, n, h);
        lookup2_n<4>(rows, cols, d, p, h, r);
        store_quad<VEC>(out, g, n, r);
    }
}

static bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Workgroups per CU, at most (a sweep of 8-64 on 5e7 rows): 16 for the
// one-dimensional lookups, 64 for the two-dimensional shift, whose per-row
// searches are latency-bound (911 -> 747 us against 8).
constexpr int kLookup1WgPerCu = 16, kJesWgPerCu = 64;

static int lookup_grid(int64_t n, int per_cu) {
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(ceil_div(n, 4), LB), per_cu * device_cus())));
}

template <typename X, int MODE>
static int launch_lookup1(const void *x, int64_t n, const float *E, int nb, const float *C, float *out,
                          hipStream_t s) {
    const size_t floats = static_cast<size_t>(2 * nb + 3);
    const bool lds = floats <= static_cast<size_t>(kMaxLookupLdsFloats);
    const bool vec = aligned(x, 4 * sizeof(X)) && aligned(out, 16);
    const X *xp = static_cast<const X *>(x);
    const int grid = lookup_grid(n, kLookup1WgPerCu);
    const size_t lb = lds ? floats * sizeof(float) : 0;
    if (lds && vec) lookup1_kernel<X, MODE, true, true><<<grid, LB, lb, s>>>(xp, n, E, nb, C, out);
    else if (lds) lookup1_kernel<X, MODE, true, false><<<grid, LB, lb, s>>>(xp, n, E, nb, C, out);
    else if (vec) lookup1_kernel<X, MODE, false, true><<<grid, LB, 0, s>>>(xp, n, E, nb, C, out);
    else lookup1_kernel<X, MODE, false, false><<<grid, LB, 0, s>>>(xp, n, E, nb, C, out);
    return check_launch(MODE == 0 ? "hepk_get_bin_contents" : "hepk_interp");
}

template <typename X>
static int launch_jes(const void *pt, const void *eta, int64_t n, const float *EE, int ne, const float *PE, int np,
                      const float *D, float *out, hipStream_t s) {
    const size_t floats = static_cast<size_t>(ne + 1) + static_cast<size_t>(np + 1) +
                          static_cast<size_t>(ne) * static_cast<size_t>(np);
    const bool lds = floats <= static_cast<size_t>(kMaxLookupLdsFloats);
    const bool vec = aligned(pt, 4 * sizeof(X)) && aligned(eta, 4 * sizeof(X)) && aligned(out, 16);
    const X *p = static_cast<const X *>(pt), *h = static_cast<const X *>(eta);
    const int grid = lookup_grid(n, kJesWgPerCu);
    const size_t lb = lds ? floats * sizeof(float) : 0;
    if (lds && vec) jes_delta_kernel<X, true, true><<<grid, LB, lb, s>>>(p, h, n, EE, ne, PE, np, D, out);
    else if (lds) jes_delta_kernel<X, true, false><<<grid, LB, lb, s>>>(p, h, n, EE, ne, PE, np, D, out);
    else if (vec) jes_delta_kernel<X, false, true><<<grid, LB, 0, s>>>(p, h, n, EE, ne, PE, np, D, out);
    else jes_delta_kernel<X, false, false><<<grid, LB, 0, s>>>(p, h, n, EE, ne, PE, np, D, out);
    return check_launch("hepk_jes_delta");
}

template <int MODE>
static int lookup1(const char *fn, const void *x, int32_t dtype, int64_t n, const float *edges, int32_t nbins,
                   const float *contents, float *out, hipStream_t stream) {
    HEPK_REQUIRE(n >= 0, "%s: n < 0", fn);
    HEPK_REQUIRE(nbins >= 1 && nbins <= (1 << 24), "%s: nbins %d outside [1, 2^24]", fn, nbins);
    HEPK_REQUIRE(edges && contents, "%s: table is NULL", fn);
    HEPK_REQUIRE(n == 0 || (x && out), "%s: x or out is NULL", fn);
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16 || dtype == HEPK_I32, "%s: bad dtype %d", fn, dtype);
    if (n == 0) return HEPK_OK;
    if (dtype == HEPK_F16) return launch_lookup1<_Float16, MODE>(x, n, edges, nbins, contents, out, stream);
    if (dtype == HEPK_I32) return launch_lookup1<int32_t, MODE>(x, n, edges, nbins, contents, out, stream);
    return launch_lookup1<float, MODE>(x, n, edges, nbins, contents, out, stream);
}

}  // namespace hepk

extern "C" int hepk_get_bin_contents(const void *x, int32_t dtype, int64_t n, const float *edges, int32_t nbins,
                                     const float *contents, float *out, hipStream_t stream) {
    hepk::clear_error();
    return hepk::lookup1<0>("hepk_get_bin_contents", x, dtype, n, edges, nbins, contents, out, stream);
}

extern "C" int hepk_interp(const void *x, int32_t dtype, int64_t n, const float *edges, int32_t nbins,
                           const float *contents, float *out, hipStream_t stream) {
    hepk::clear_error();
    return hepk::lookup1<1>("hepk_interp", x, dtype, n, edges, nbins, contents, out, stream);
}

extern "C" int hepk_jes_delta(const void *pt, const void *eta, int32_t dtype, int64_t n, const float *eta_edges,
                              int32_t n_eta, const float *pt_edges, int32_t n_pt, const float *delta, float *out,
                              hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n >= 0, "hepk_jes_delta: n < 0");
    HEPK_REQUIRE(n_eta >= 1 && n_pt >= 1 && n_eta <= (1 << 20) && n_pt <= (1 << 20) &&
                     static_cast<int64_t>(n_eta) * n_pt <= (1 << 26),
                 "hepk_jes_delta: table shape %d x %d unsupported", n_eta, n_pt);
    HEPK_REQUIRE(eta_edges && pt_edges && delta, "hepk_jes_delta: table is NULL");
    HEPK_REQUIRE(n == 0 || (pt && eta && out), "hepk_jes_delta: pt, eta or out is NULL");
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16, "hepk_jes_delta: bad dtype %d", dtype);
    if (n == 0) return HEPK_OK;
    if (dtype == HEPK_F16)
        return launch_jes<_Float16>(pt, eta, n, eta_edges, n_eta, pt_edges, n_pt, delta, out, stream);
    return launch_jes<float>(pt, eta, n, eta_edges, n_eta, pt_edges, n_pt, delta, out, stream);
}
