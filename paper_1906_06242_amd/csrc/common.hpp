// Internal helpers of libhepk: error reporting, launch bookkeeping and the
// float32 device primitives every kernel shares (column loads with exact
// float16 widening, cut comparisons, the Delta-phi wrap, histogram slots).
//
// Build flags matter for exactness: -ffp-contract=off keeps a*b+c as a
// rounded multiply followed by a rounded add (no v_fma_f32), and denormals
// are kept (no flush-to-zero), so every float32 operation is the IEEE one.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "hepk.h"

namespace hepk {

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);
void clear_error();

#define HEPK_REQUIRE(cond, ...)                                   \
    do {                                                          \
        if (!(cond)) {                                            \
            ::hepk::set_error(__VA_ARGS__);                       \
            return HEPK_EINVAL;                                   \
        }                                                         \
    } while (0)

#define HEPK_HIP(call)                                                            \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::hepk::set_error("%s failed: %s", #call, hipGetErrorString(e_));     \
            return HEPK_EHIP;                                                     \
        }                                                                         \
    } while (0)

// Checks the launch that was just enqueued.
int check_launch(const char *what);

// Compute units of the current device (cached per device).
int device_cus();

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- device

// float32 pi and 2*pi rounded to nearest (bit patterns 0x40490FDB, 0x40C90FDB).
constexpr float kPi = 0x1.921fb6p+1f;
constexpr float kTwoPi = 0x1.921fb6p+2f;

template <typename T, typename I>
__device__ __forceinline__ float ldf(const T *p, I i) {
    return static_cast<float>(p[i]);  // _Float16 -> float is v_cvt_f32_f16: exact
}

// A raw buffer resource over the nbytes bytes at p (gfx9 format word: 32-bit
// data, no swizzle, stride 0).  The hardware range check turns every load at
// a byte offset at or beyond nbytes into 0, so a load of slot i of a tile
// needs no per-lane bounds test and no zero default.
using buf_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ buf_t buf_span(const void *p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, static_cast<int>(nbytes), 0x00020000);
}

// Element i of a float32 or float16 buffer as float (0 beyond the range).
template <typename T>
__device__ __forceinline__ float buf_ldf(buf_t r, int i) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
    } else {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, i * 2, 0, 0);
        return static_cast<float>(__builtin_bit_cast(_Float16, h));
    }
}

// The 32-bit word at byte offset `byte` of a buffer (0 beyond the range).
// Element i of a float32 or float16 buffer as its raw bits (0 beyond the
// range), converted by raw_f only where the value is used: a load whose
// conversion sits right behind it would be waited for there.
// AUX is the load's cache policy: 0, or kBufNt for the nontemporal hint
// (data read once; it measured faster in some kernels and slower in others).
constexpr int kBufNt = 2;

template <typename T, int AUX = 0>
__device__ __forceinline__ uint32_t buf_raw(buf_t r, int i) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, AUX);
    else
        return __builtin_amdgcn_raw_buffer_load_b16(r, i * 2, 0, AUX);
}

template <typename T>
__device__ __forceinline__ float raw_f(uint32_t b) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(float, b);
    else
        return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(b)));
}

template <int AUX = 0>
__device__ __forceinline__ uint32_t buf_u32(buf_t r, int byte) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, byte, 0, AUX);
}

__device__ __forceinline__ float ld_any(const void *p, int32_t dtype, int64_t i) {
    if (dtype == HEPK_F16) return static_cast<float>(static_cast<const _Float16 *>(p)[i]);
    if (dtype == HEPK_I32) return static_cast<float>(static_cast<const int32_t *>(p)[i]);
    return static_cast<const float *>(p)[i];
}

__device__ __forceinline__ bool cmp_f(float v, int32_t op, float t) {
    switch (op) {
    case HEPK_GT: return v > t;
    case HEPK_GE: return v >= t;
    case HEPK_LT: return v < t;
    case HEPK_LE: return v <= t;
    case HEPK_ABS_LT: return fabsf(v) < t;
    default: return fabsf(v) <= t;
    }
}

__device__ __forceinline__ bool cmp_i(int32_t v, int32_t op, int32_t t) {
    switch (op) {
    case HEPK_GT: return v > t;
    case HEPK_GE: return v >= t;
    case HEPK_LT: return v < t;
    case HEPK_LE: return v <= t;
    case HEPK_ABS_LT: return abs(v) < t;
    default: return abs(v) <= t;
    }
}

// dR^2 = deta^2 + dphi^2 with dphi brought into [-pi, pi] by one step of 2*pi.
// Written as separate rounded float32 operations; -ffp-contract=off keeps
// the compiler from fusing the square and the sum.
//
// Only |dphi| enters the square, and the wrapped magnitude is |dphi| - 2*pi
// whenever |dphi| > pi: for dphi > pi that is dphi - 2*pi itself, for
// dphi < -pi it is -(dphi + 2*pi), and negation is exact (round-to-nearest
// is symmetric in sign).  So the square equals that of the two-sided wrap
// bit for bit.  It is taken as min(x, 2*pi - x), x = |dphi| (two
// instructions, both with the |.| modifier): 2*pi - x = -(x - 2*pi) exactly,
// and with 2*pi = 2 * pi exact and rounding monotone, x <= pi gives
// 2*pi - x >= pi >= x while x > pi gives 2*pi - x <= pi < x, so the minimum
// is the wrapped magnitude exactly when |dphi| > pi (x = inf gives -inf,
// whose square is inf as before; a NaN x stays NaN).
__device__ __forceinline__ float delta_r2(float eta_a, float phi_a, float eta_b, float phi_b) {
    const float deta = eta_a - eta_b;
    const float adphi = fabsf(phi_a - phi_b);
    const float dphi = fminf(adphi, kTwoPi - adphi);
    const float a = deta * deta;
    const float b = dphi * dphi;
    return a + b;
}

// Read-only data seen through the constant address space: the compiler may then
// fetch it with scalar loads into SGPRs when the address is uniform (a kernel
// that also does global atomics otherwise has to assume the data may change
// and keeps every field of a table entry in VGPRs).  Only for memory the
// kernel never writes.
// (The host pass of this single-source file only type-checks device code; it
// sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;
#else
template <typename T>
using const_ptr = const T *;
#endif

template <typename T>
__device__ __forceinline__ const_ptr<T> as_const(const T *p) {
    return reinterpret_cast<const_ptr<T>>(reinterpret_cast<uintptr_t>(p));
}

// Edges E[0..nbins] strictly increasing and E[0] <= x < E[nbins]: the slot
// s of x, E[s-1] <= x < E[s] (binary search).
__device__ __forceinline__ int bin_search(const float *E, int nbins, float x) {
    int a = 0, b = nbins;  // E[a] <= x < E[b]
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (E[m] <= x)
            a = m;
        else
            b = m;
    }
    return a + 1;
}

// Histogram slot of x (not NaN) for strictly increasing edges E[0..nbins],
// lo == E[0], hi == E[nbins]: 0 if x < lo, nbins+1 if x >= hi, else s with
// E[s-1] <= x < E[s].  A guess from the uniform-bin formula (inv_w = nbins /
// (hi - lo)) is verified against the edges and replaced by a binary search
// when wrong, so any increasing edges give the exact slot.
__device__ __forceinline__ int hist_slot_lohi(float x, const float *E, int nbins, float lo, float hi, float inv_w) {
    if (!(x >= lo)) return 0;
    if (x >= hi) return nbins + 1;
    const float g = (x - lo) * inv_w;
    const int s = (g >= 0.0f) ? ((g < static_cast<float>(nbins)) ? static_cast<int>(g) + 1 : nbins) : 1;
    return (x < E[s - 1] || x >= E[s]) ? bin_search(E, nbins, x) : s;
}

__device__ __forceinline__ void atomic_add_f64(double *p, double v) {
    unsafeAtomicAdd(p, v);  // global_atomic_add_f64 / ds_add_f64 on gfx950
}

__device__ __forceinline__ void atomic_add_u64(uint64_t *p, uint64_t v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}

}  // namespace hepk
